// Multigrid Fourier transfer and Poisson solve on the device (Sec. II: the
// Hartree potential of Eqs. (vH), (vHG) and the multigrid Fourier
// interpolation that moves densities and potentials between the levels).
//
// For level l (mesh N_l, weight w_l = Omega / N_l, cutoff E_l in Ry or none):
//   rho~(G)  = sum_l mask_l(G) w_l FFT(rho_l)(G)
//   v~(G)    = 4 pi rho~(G) / |G|^2 (G != 0), v~(0) = 0
//   v_l(r)   = (1 / Omega) sum_G mask_l(G) v~(G) exp(i G.r)
//   E_J      = (1 / (2 Omega)) sum_{G != 0} 4 pi |rho~(G)|^2 / |G|^2
// with mask_l(G): |m_d| < N_{l,d} / 2 on every axis (no Nyquist plane) and
// |G|^2 < E_l, G = sum_d m_d b_d with the reciprocal vectors
// b_d = 2 pi (A^-1)[:, d] of the lattice vectors A (rows); G = 2 pi m / L for
// an orthorhombic cell.  The densities are real, so each level works on
// its half spectrum (m_z >= 0, hipFFT D2Z / Z2D); the coefficients of all
// levels meet on the half spectrum of the finest mesh, where a level's
// plane wave m sits at (m_x mod N_0x, m_y mod N_0y, m_z).  The energy sums the
// half spectrum with weight 2 off the m_z = 0 plane (no masked plane wave
// reaches the finest mesh's Nyquist plane).
#include "gpw_internal.h"

#include <hipfft/hipfft.h>

#include <mutex>
#include <new>

namespace gpw {

struct PoissonState {
    std::mutex mu;                       // creation, and set-stream + execute of the shared FFT plans
    bool ready = false;
    hipfftHandle fwd[kMaxLevels] = {};   // D2Z of each level
    hipfftHandle inv[kMaxLevels] = {};   // Z2D of each level
    size_t work = 0;                     // largest FFT work area
};

__host__ __device__ inline long long half_count(const LevelGeom &G) { return (long long)G.N[0] * G.N[1] * (G.N[2] / 2 + 1); }
static inline size_t align256p(size_t b) { return (b + 255) & ~size_t(255); }
constexpr int kEnergyBlocks = 1024;

// Integer frequency of FFT index i of an n-point transform (negative half
// above n / 2; the Nyquist index of an even n maps to -n / 2).
__device__ __forceinline__ int freq_of(int i, int n) { return 2 * i < n ? i : i - n; }

// Cartesian G = sum_d m_d b_d; B[d] holds b_d
__device__ __forceinline__ void gvec(int mx, int my, int mz, const double (*B)[3], double *g)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) g[c] = mx * B[0][c] + my * B[1][c] + mz * B[2][c];
}

// The level's masked plane wave at half-spectrum index i, as a fine-grid
// half-spectrum index, or -1.
__device__ __forceinline__ long long level_to_fine(long long i, const LevelGeom &G, const int *Nf, double cut,
                                                   const double (*B)[3])
{
    const int nzh = G.N[2] / 2 + 1;
    const int iz = (int)(i % nzh);
    const long long r = i / nzh;
    const int iy = (int)(r % G.N[1]), ix = (int)(r / G.N[1]);
    const int mx = freq_of(ix, G.N[0]), my = freq_of(iy, G.N[1]), mz = iz;
    if (2 * abs(mx) >= G.N[0] || 2 * abs(my) >= G.N[1] || 2 * mz >= G.N[2]) return -1;
    if (cut > 0.0) {
        double g[3];
        gvec(mx, my, mz, B, g);
        if (!(g[0] * g[0] + g[1] * g[1] + g[2] * g[2] < cut)) return -1;
    }
    const int fx = mx < 0 ? mx + Nf[0] : mx, fy = my < 0 ? my + Nf[1] : my;
    return ((long long)fx * Nf[1] + fy) * (Nf[2] / 2 + 1) + mz;
}

struct PoissonGeom {
    LevelGeom G;          // this level
    int Nf[3];            // the finest mesh
    double B[3][3];       // reciprocal vectors b_d (rows), 2 pi (A^-1)^T
    double cut;           // Ry, or 0 for every plane wave of the mesh
    double scale;         // w_l (scatter) or 1 / Omega (gather)
};

__global__ void __launch_bounds__(256) k_cfill(double2 *p, long long n)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = make_double2(0.0, 0.0);
}

// fine += w_l mask_l FFT(rho_l): the map is one-to-one within a level, and the
// levels' scatters are ordered on the stream, so no atomics are needed.
__global__ void __launch_bounds__(256) k_scatter(const double2 *__restrict__ c, double2 *__restrict__ fine, PoissonGeom pg)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= half_count(pg.G)) return;
    const long long f = level_to_fine(i, pg.G, pg.Nf, pg.cut, pg.B);
    if (f < 0) return;
    const double2 a = c[i];
    double2 b = fine[f];
    b.x += pg.scale * a.x;
    b.y += pg.scale * a.y;
    fine[f] = b;
}

// level half spectrum = mask_l v~ / Omega (zero elsewhere)
__global__ void __launch_bounds__(256) k_gather(const double2 *__restrict__ fine, double2 *__restrict__ c, PoissonGeom pg)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= half_count(pg.G)) return;
    const long long f = level_to_fine(i, pg.G, pg.Nf, pg.cut, pg.B);
    double2 v = make_double2(0.0, 0.0);
    if (f >= 0) {
        const double2 a = fine[f];
        v = make_double2(pg.scale * a.x, pg.scale * a.y);
    }
    c[i] = v;
}

// v~ = 4 pi rho~ / |G|^2 in place, and per-block partial sums of the energy
// terms 4 pi |rho~|^2 / |G|^2 (weight 2 off the m_z = 0 plane); a grid-stride
// loop over the fine half spectrum with kEnergyBlocks blocks.
__global__ void __launch_bounds__(256) k_coulomb(double2 *__restrict__ fine, double *__restrict__ partial, PoissonGeom pg)
{
    __shared__ double red[256];
    const int *N = pg.Nf;
    const int nzh = N[2] / 2 + 1;
    const long long n = (long long)N[0] * N[1] * nzh;
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const int iz = (int)(i % nzh);
        const long long r = i / nzh;
        const int iy = (int)(r % N[1]), ix = (int)(r / N[1]);
        double g[3];
        gvec(freq_of(ix, N[0]), freq_of(iy, N[1]), iz, pg.B, g);
        const double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
        const double coul = g2 > 0.0 ? 4.0 * M_PI / g2 : 0.0;
        const double2 a = fine[i];
        acc += (iz == 0 ? 1.0 : 2.0) * coul * (a.x * a.x + a.y * a.y);
        fine[i] = make_double2(coul * a.x, coul * a.y);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// E_J = sum of the partials / (2 Omega), in a fixed order (one block)
__global__ void __launch_bounds__(256) k_energy(const double *__restrict__ partial, int n, double inv2vol, double *ej)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += partial[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *ej = red[0] * inv2vol;
}

// Cartesian component d of G at fine half-spectrum index i
__device__ __forceinline__ double fine_g(long long i, const int *N, const double (*B)[3], int d)
{
    const int nzh = N[2] / 2 + 1;
    const int iz = (int)(i % nzh);
    const long long r = i / nzh;
    const int iy = (int)(r % N[1]), ix = (int)(r / N[1]);
    return freq_of(ix, N[0]) * B[0][d] + freq_of(iy, N[1]) * B[1][d] + iz * B[2][d];
}

// out = scale * (i G_d)^k * fine on the fine half spectrum (k = 0 or 1, d < 0
// for k = 0): the coefficients of the fine-grid density or of one gradient
// component, ready for Z2D.
__global__ void __launch_bounds__(256) k_fine_out(const double2 *__restrict__ fine, double2 *__restrict__ out,
                                                 PoissonGeom pg, int d)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= half_count(pg.G)) return;
    const double2 a = fine[i];
    if (d < 0) {
        out[i] = make_double2(pg.scale * a.x, pg.scale * a.y);
    } else {
        const double g = pg.scale * fine_g(i, pg.Nf, pg.B, d);   // i g (a.x + i a.y) = -g a.y + i g a.x
        out[i] = make_double2(-g * a.y, g * a.x);
    }
}

// fine += mask_0 scale (-i G_d)^k c (c: D2Z of a fine-grid function): the
// exchange-correlation potential (k = 0) or the GGA term, minus the divergence
// of the vector potential (k = 1, component d).
__global__ void __launch_bounds__(256) k_add_xc(const double2 *__restrict__ c, double2 *__restrict__ fine, PoissonGeom pg,
                                               int d)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= half_count(pg.G)) return;
    if (level_to_fine(i, pg.G, pg.Nf, pg.cut, pg.B) < 0) return;   // level 0's own mask: f == i
    const double2 a = c[i];
    double2 b = fine[i];
    if (d < 0) {
        b.x += pg.scale * a.x;
        b.y += pg.scale * a.y;
    } else {
        const double g = pg.scale * fine_g(i, pg.Nf, pg.B, d);   // -i g (a.x + i a.y) = g a.y - i g a.x
        b.x += g * a.y;
        b.y -= g * a.x;
    }
    fine[i] = b;
}

static hipError_t fft_error(hipfftResult r)
{
    return r == HIPFFT_SUCCESS ? hipSuccess : r == HIPFFT_ALLOC_FAILED ? hipErrorOutOfMemory : hipErrorUnknown;
}

// FFT plans of every level, created on the first call (the FFT library may
// build its kernels then); the work areas come from the caller's scratch.
static hipError_t poisson_ready(gpw_plan_s *pl, PoissonState *&ps)
{
    {
        std::lock_guard<std::mutex> g(pl->poisson_mu);
        if (!pl->poisson) pl->poisson = new (std::nothrow) PoissonState();
        ps = pl->poisson;
    }
    if (!ps) return hipErrorOutOfMemory;
    std::lock_guard<std::mutex> g(ps->mu);
    if (ps->ready) return hipSuccess;
    for (int l = 0; l < pl->nlevels; ++l) {
        const LevelGeom &G = pl->geom[l];
        for (int dir = 0; dir < 2; ++dir) {
            hipfftHandle &h = dir == 0 ? ps->fwd[l] : ps->inv[l];
            size_t ws = 0;
            hipfftResult r = hipfftCreate(&h);
            if (r == HIPFFT_SUCCESS) r = hipfftSetAutoAllocation(h, 0);
            if (r == HIPFFT_SUCCESS)
                r = hipfftMakePlan3d(h, G.N[0], G.N[1], G.N[2], dir == 0 ? HIPFFT_D2Z : HIPFFT_Z2D, &ws);
            if (r != HIPFFT_SUCCESS) return fft_error(r);
            ps->work = std::max(ps->work, ws);
        }
    }
    ps->ready = true;
    return hipSuccess;
}

void poisson_free(gpw_plan_s *pl)
{
    if (!pl->poisson) return;
    for (int l = 0; l < kMaxLevels; ++l) {
        if (pl->poisson->fwd[l]) (void)hipfftDestroy(pl->poisson->fwd[l]);
        if (pl->poisson->inv[l]) (void)hipfftDestroy(pl->poisson->inv[l]);
    }
    delete pl->poisson;
    pl->poisson = nullptr;
}

size_t poisson_spectra_bytes(const gpw_plan_s *pl)
{
    long long mx = 0;
    for (int l = 0; l < pl->nlevels; ++l) mx = std::max(mx, half_count(pl->geom[l]));
    return align256p(16 * (size_t)half_count(pl->geom[0])) + align256p(16 * (size_t)mx) +
           align256p(8 * (size_t)kEnergyBlocks);
}

// Scratch of one call: the fine half spectrum, one level-sized half spectrum,
// the energy partials, the FFT work area.
struct PoissonScratch {
    unsigned char *base = nullptr;
    double2 *fine = nullptr, *lvl = nullptr;
    double *partial = nullptr;
    void *work = nullptr;
};

static hipError_t scratch_alloc(const gpw_plan_s *pl, const PoissonState *ps, PoissonScratch &x, hipStream_t st)
{
    const size_t fine_b = align256p(16 * (size_t)half_count(pl->geom[0]));
    long long mx = 0;
    for (int l = 0; l < pl->nlevels; ++l) mx = std::max(mx, half_count(pl->geom[l]));
    const size_t lvl_b = align256p(16 * (size_t)mx), part_b = align256p(8 * (size_t)kEnergyBlocks);
    hipError_t e =
        hipMallocAsync((void **)&x.base, fine_b + lvl_b + part_b + align256p(std::max<size_t>(ps->work, 256)), st);
    if (e != hipSuccess) return e;
    x.fine = (double2 *)x.base;
    x.lvl = (double2 *)(x.base + fine_b);
    x.partial = (double *)(x.base + fine_b + lvl_b);
    x.work = x.base + fine_b + lvl_b + part_b;
    return hipSuccess;
}

static PoissonGeom base_geom(const gpw_plan_s *pl)
{
    PoissonGeom pg{};
    for (int d = 0; d < 3; ++d) {
        pg.Nf[d] = pl->geom[0].N[d];
        for (int c = 0; c < 3; ++c) pg.B[d][c] = pl->recip[d][c];
    }
    return pg;
}
static dim3 grid256(long long n) { return dim3((unsigned)((n + 255) / 256)); }

// fine = rho~ = sum_l mask_l w_l D2Z(rho_l); the caller holds ps->mu
static hipfftResult accumulate_density(const gpw_plan_s *pl, PoissonState *ps, const double *const *rho,
                                       PoissonScratch &x, hipStream_t st)
{
    PoissonGeom pg = base_geom(pl);
    hipLaunchKernelGGL(k_cfill, grid256(half_count(pl->geom[0])), dim3(256), 0, st, x.fine, half_count(pl->geom[0]));
    hipfftResult r = HIPFFT_SUCCESS;
    for (int l = 0; l < pl->nlevels && r == HIPFFT_SUCCESS; ++l) {
        r = hipfftSetStream(ps->fwd[l], st);
        if (r == HIPFFT_SUCCESS) r = hipfftSetWorkArea(ps->fwd[l], x.work);
        if (r == HIPFFT_SUCCESS) r = hipfftExecD2Z(ps->fwd[l], (hipfftDoubleReal *)rho[l], (hipfftDoubleComplex *)x.lvl);
        if (r != HIPFFT_SUCCESS) break;
        pg.G = pl->geom[l];
        pg.cut = pl->cut_ry[l];
        pg.scale = pl->geom[l].w;
        hipLaunchKernelGGL(k_scatter, grid256(half_count(pl->geom[l])), dim3(256), 0, st, x.lvl, x.fine, pg);
    }
    return r;
}

hipError_t poisson_run(gpw_plan_s *pl, const double *const *rho, const double *vxc, const double *const *vxc_grad,
                       double *const *v, double *ej, hipStream_t st)
{
    PoissonState *ps = nullptr;
    hipError_t e = poisson_ready(pl, ps);
    if (e != hipSuccess) return e;
    PoissonScratch x;
    e = scratch_alloc(pl, ps, x, st);
    if (e != hipSuccess) return e;
    const double vol = pl->volume;
    PoissonGeom pg = base_geom(pl);
    {
        // the FFT plans are shared by every caller of this plan: set their
        // stream and work area and enqueue under the lock
        std::lock_guard<std::mutex> g(ps->mu);
        hipfftResult r = accumulate_density(pl, ps, rho, x, st);
        if (r == HIPFFT_SUCCESS) {
            pg.G = pl->geom[0];
            hipLaunchKernelGGL(k_coulomb, dim3(kEnergyBlocks), dim3(256), 0, st, x.fine, x.partial, pg);
            if (ej) hipLaunchKernelGGL(k_energy, dim3(1), dim3(256), 0, st, x.partial, kEnergyBlocks, 0.5 / vol, ej);
        }
        // exchange-correlation inputs on the finest mesh: w_0 F(vxc) and
        // -i G . w_0 F(vxc_grad), on level 0's plane waves
        for (int d = -1; d < 3 && r == HIPFFT_SUCCESS; ++d) {
            const double *src = d < 0 ? vxc : (vxc_grad ? vxc_grad[d] : nullptr);
            if (!src) continue;
            r = hipfftSetStream(ps->fwd[0], st);
            if (r == HIPFFT_SUCCESS) r = hipfftSetWorkArea(ps->fwd[0], x.work);
            if (r == HIPFFT_SUCCESS) r = hipfftExecD2Z(ps->fwd[0], (hipfftDoubleReal *)src, (hipfftDoubleComplex *)x.lvl);
            pg.G = pl->geom[0];
            pg.cut = pl->cut_ry[0];
            pg.scale = pl->geom[0].w;
            if (r == HIPFFT_SUCCESS)
                hipLaunchKernelGGL(k_add_xc, grid256(half_count(pl->geom[0])), dim3(256), 0, st, x.lvl, x.fine, pg, d);
        }
        for (int l = 0; l < pl->nlevels && r == HIPFFT_SUCCESS; ++l) {
            pg.G = pl->geom[l];
            pg.cut = pl->cut_ry[l];
            pg.scale = 1.0 / vol;
            hipLaunchKernelGGL(k_gather, grid256(half_count(pl->geom[l])), dim3(256), 0, st, x.fine, x.lvl, pg);
            r = hipfftSetStream(ps->inv[l], st);
            if (r == HIPFFT_SUCCESS) r = hipfftSetWorkArea(ps->inv[l], x.work);
            if (r == HIPFFT_SUCCESS) r = hipfftExecZ2D(ps->inv[l], (hipfftDoubleComplex *)x.lvl, (hipfftDoubleReal *)v[l]);
        }
        e = r == HIPFFT_SUCCESS ? hipGetLastError() : fft_error(r);
    }
    (void)hipFreeAsync(x.base, st);
    return e;
}

hipError_t fine_density_run(gpw_plan_s *pl, const double *const *rho, double *rho_fine, double *const *grad,
                            hipStream_t st)
{
    PoissonState *ps = nullptr;
    hipError_t e = poisson_ready(pl, ps);
    if (e != hipSuccess) return e;
    PoissonScratch x;
    e = scratch_alloc(pl, ps, x, st);
    if (e != hipSuccess) return e;
    const double vol = pl->volume;
    PoissonGeom pg = base_geom(pl);
    pg.G = pl->geom[0];
    pg.scale = 1.0 / vol;
    {
        std::lock_guard<std::mutex> g(ps->mu);
        hipfftResult r = accumulate_density(pl, ps, rho, x, st);
        for (int d = -1; d < 3 && r == HIPFFT_SUCCESS; ++d) {
            double *dst = d < 0 ? rho_fine : (grad ? grad[d] : nullptr);
            if (!dst) continue;
            hipLaunchKernelGGL(k_fine_out, grid256(half_count(pl->geom[0])), dim3(256), 0, st, x.fine, x.lvl, pg, d);
            r = hipfftSetStream(ps->inv[0], st);
            if (r == HIPFFT_SUCCESS) r = hipfftSetWorkArea(ps->inv[0], x.work);
            if (r == HIPFFT_SUCCESS) r = hipfftExecZ2D(ps->inv[0], (hipfftDoubleComplex *)x.lvl, (hipfftDoubleReal *)dst);
        }
        e = r == HIPFFT_SUCCESS ? hipGetLastError() : fft_error(r);
    }
    (void)hipFreeAsync(x.base, st);
    return e;
}

}  // namespace gpw
