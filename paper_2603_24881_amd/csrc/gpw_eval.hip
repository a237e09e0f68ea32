// Collocation (rho), integration (mat) and gradient kernels for gfx950.
//
// rho  - grid-block major, after Alg. 1 of the paper, mapped to CDNA: one
//        wave64 owns one 4x4x4 block of one level, lane = grid point, and
//        keeps the block's density in a register (no cross-lane reduction, one
//        write per point).  The pair images of the block are taken in batches
//        of 64: first lane = pair image, each lane evaluating its image's 1-D
//        Gaussian envelopes and offsets on the 4 points of every axis into LDS
//        (the separable factorisation of Sec. III.A, Eqs. (gx), (gab)); then
//        lane = point, walking the batch with the pair record and the D
//        sub-block held in scalar registers, the polynomial prefactor of
//        Eq. (gab) evaluated directly per point as in the paper's GPU kernel.
// mat  - pair major: one wave per pair image walks the 4x4x4 blocks its
//        truncation sphere meets (the same block set as rho), lane = point,
//        accumulating the n_a x n_b local integrals (Alg. 2's F^local) in
//        registers over all blocks, then one wave reduction and one atomic add
//        per matrix element per pair image instead of one per (pair, block).
// grad - same traversal as mat with the six derivative accumulators of
//        Alg. 3 (d/dA and d/dB contracted with D and v on the fly).
// Every kernel is templated on (l_a, l_b) and on the per-point arithmetic
// type (double, or float for the FP32 variant; exponents, centres and the
// cross-level/matrix accumulation stay in double).
#include "gpw_internal.h"

namespace gpw {

// ------------------------------------------------------- Cartesian helpers

// Index of (lx, ly, lz) inside its shell, lexicographic order lx desc, ly desc.
__host__ __device__ constexpr int cart_index(int ly, int lz) { return (ly + lz) * (ly + lz + 1) / 2 + lz; }

template <int L, typename T>
__device__ __forceinline__ void monomials(T x, T y, T z, T *m)
{
    T px[L + 1], py[L + 1], pz[L + 1];
    px[0] = py[0] = pz[0] = T(1);
#pragma unroll
    for (int i = 1; i <= L; ++i) { px[i] = px[i - 1] * x; py[i] = py[i - 1] * y; pz[i] = pz[i - 1] * z; }
    int n = 0;
#pragma unroll
    for (int lx = L; lx >= 0; --lx)
#pragma unroll
        for (int ly = L - lx; ly >= 0; --ly) {
            const int lz = L - lx - ly;
            T v = px[lx];
            if (ly) v = v * py[ly];
            if (lz) v = v * pz[lz];
            m[n++] = v;
        }
}

// g[d] = sum_mu t_mu d(monomial_mu)/d(offset_d) for a shell of degree L.
template <int L, typename T>
__device__ __forceinline__ void poly_grad(T x, T y, T z, const T *t, T *g)
{
    g[0] = g[1] = g[2] = T(0);
    if (L == 0) return;
    T lower[(L + 1) * L / 2 > 0 ? (L + 1) * L / 2 : 1];   // monomials of degree L-1
    monomials<(L > 0 ? L - 1 : 0), T>(x, y, z, lower);
    int n = 0;
#pragma unroll
    for (int lx = L; lx >= 0; --lx)
#pragma unroll
        for (int ly = L - lx; ly >= 0; --ly) {
            const int lz = L - lx - ly;
            if (lx) g[0] += T(lx) * t[n] * lower[cart_index(ly, lz)];
            if (ly) g[1] += T(ly) * t[n] * lower[cart_index(ly - 1, lz)];
            if (lz) g[2] += T(lz) * t[n] * lower[cart_index(ly, lz - 1)];
            ++n;
        }
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// --------------------------------------------------------- small kernels

template <typename T>
__global__ void k_symmetrize(const double *__restrict__ D, T *__restrict__ out, int n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * n) return;
    const long long r = i / n, c = i % n;
    out[i] = (T)(0.5 * (D[i] + D[c * n + r]));
}

__global__ void k_fill(double *__restrict__ p, long long n, double v)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ rho

template <int LA, int LB, typename T>
__global__ void __launch_bounds__(64)
k_rho(const PairRec *__restrict__ pairs, const int2 *__restrict__ inc,
      const long long *__restrict__ inc_off, long long cbase, const int *__restrict__ blk,
      LevelGeom G, const T *__restrict__ Dm, int n_ao, double *__restrict__ rho)
{
    constexpr int NA = ncart_c(LA), NB = ncart_c(LB);
    __shared__ T tab_e[64][3][4];
    __shared__ T tab_d[64][3][4];
    const int lane = threadIdx.x;
    const int b = blk[blockIdx.x];
    const int kz = b % G.nb[2];
    const int ky = (b / G.nb[2]) % G.nb[1];
    const int kx = b / (G.nb[2] * G.nb[1]);
    const int kk[3] = {kx, ky, kz};
    const long long s0 = inc_off[cbase + b], s1 = inc_off[cbase + b + 1];
    const int tx = lane >> 4, ty = (lane >> 2) & 3, tz = lane & 3;
    T acc = T(0);
    for (long long s = s0; s < s1; s += 64) {
        const int n = (int)(s1 - s < 64 ? s1 - s : 64);
        if (lane < n) {
            const int2 en = inc[s + lane];
            const PairRec &r = pairs[en.x];
            const double ap = r.aa + r.ab;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const long long u0 = 4LL * kk[d] + (long long)shift_of(en.y, d) * G.N[d];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const double x = (double)(u0 + t) * G.h[d];
                    const double dx = x - r.P[d];
                    tab_e[lane][d][t] = (T)exp(-ap * dx * dx);
                    tab_d[lane][d][t] = (T)(x - r.A[d]);
                }
            }
        }
        __syncthreads();
        for (int q = 0; q < n; ++q) {
            const int2 en = inc[s + q];
            const PairRec &r = pairs[en.x];
            T E = tab_e[q][0][tx] * tab_e[q][1][ty] * tab_e[q][2][tz];
            E = (E >= (T)r.ER) ? E : T(0);
            const T xa = tab_d[q][0][tx], ya = tab_d[q][1][ty], za = tab_d[q][2][tz];
            T a[NA], bb[NB];
            monomials<LA, T>(xa, ya, za, a);
            monomials<LB, T>(xa + (T)r.AB[0], ya + (T)r.AB[1], za + (T)r.AB[2], bb);
            const T *Dp = Dm + (long long)r.ao_a * n_ao + r.ao_b;
            T sum = T(0);
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                T t = T(0);
#pragma unroll
                for (int j = 0; j < NB; ++j) t += Dp[(long long)i * n_ao + j] * bb[j];
                sum += a[i] * t;
            }
            acc += (T)r.Kw * E * sum;
        }
        __syncthreads();
    }
    const int wx = 4 * kx + tx, wy = 4 * ky + ty, wz = 4 * kz + tz;
    if (wx < G.N[0] && wy < G.N[1] && wz < G.N[2]) {
        const long long o = ((long long)wx * G.N[1] + wy) * G.N[2] + wz;
        rho[o] += (double)acc;
    }
}

// ----------------------------------------------- pair-major traversal (mat, grad)

// 1-D tables of a pair image over u in [lo-3, hi+3] per axis, in LDS:
// envelope exp(-alpha_p (x_u - P)^2) and offset x_u - A.
template <typename T>
__device__ __forceinline__ void pair_tables(const PairRec &r, const LevelGeom &G, T *te, T *td, int wmax)
{
    const double ap = r.aa + r.ab;
    for (int d = 0; d < 3; ++d) {
        const int W = r.hi[d] - r.lo[d] + 7;
        for (int i = threadIdx.x; i < W; i += 64) {
            const double x = (double)(r.lo[d] - 3 + i) * G.h[d];
            const double dx = x - r.P[d];
            te[d * wmax + i] = (T)exp(-ap * dx * dx);
            td[d * wmax + i] = (T)(x - r.A[d]);
        }
    }
}

// Visit every (block, shift) incidence of the pair image whose block meets
// the truncation sphere; body(valid, e, xa, ya, za, widx) per lane.
template <typename T, typename Body>
__device__ __forceinline__ void for_each_point(const PairRec &r, const LevelGeom &G, const T *te,
                                               const T *td, int wmax, Body &&body)
{
    const int lane = threadIdx.x;
    const int tx = lane >> 4, ty = (lane >> 2) & 3, tz = lane & 3;
    const double R2c = r.R2 * kCullSlack;
    const T ER = (T)r.ER;
    AxisIter ix, iy, iz;
    for (ix.start(r.lo[0], r.hi[0], G.N[0], G.nb[0]); ix.valid(); ix.next()) {
        double x0, x1;
        ix.range(G.h[0], x0, x1);
        const double gx = axis_gap2(r.P[0], x0, x1);
        if (gx > R2c) continue;
        const int wx = 4 * (int)ix.k + tx;
        const int jx = (int)(4 * ix.k + ix.S * G.N[0]) + tx - (r.lo[0] - 3);
        const T ex = te[jx], xa = td[jx];
        for (iy.start(r.lo[1], r.hi[1], G.N[1], G.nb[1]); iy.valid(); iy.next()) {
            double y0, y1;
            iy.range(G.h[1], y0, y1);
            const double gy = gx + axis_gap2(r.P[1], y0, y1);
            if (gy > R2c) continue;
            const int wy = 4 * (int)iy.k + ty;
            const int jy = (int)(4 * iy.k + iy.S * G.N[1]) + ty - (r.lo[1] - 3);
            const T exy = ex * te[wmax + jy], ya = td[wmax + jy];
            for (iz.start(r.lo[2], r.hi[2], G.N[2], G.nb[2]); iz.valid(); iz.next()) {
                double z0, z1;
                iz.range(G.h[2], z0, z1);
                if (gy + axis_gap2(r.P[2], z0, z1) > R2c) continue;
                const int wz = 4 * (int)iz.k + tz;
                const int jz = (int)(4 * iz.k + iz.S * G.N[2]) + tz - (r.lo[2] - 3);
                T E = exy * te[2 * wmax + jz];
                const bool valid = (wx < G.N[0]) && (wy < G.N[1]) && (wz < G.N[2]) && (E >= ER);
                const long long widx = valid ? ((long long)wx * G.N[1] + wy) * G.N[2] + wz : 0;
                body(valid, E, xa, ya, td[2 * wmax + jz], widx);
            }
        }
    }
}

template <int LA, int LB, typename T>
__global__ void __launch_bounds__(64)
k_mat(const PairRec *__restrict__ pairs, long long p0, LevelGeom G, const double *__restrict__ V,
      double *__restrict__ M, int n_ao, int wmax)
{
    constexpr int NA = ncart_c(LA), NB = ncart_c(LB);
    extern __shared__ unsigned char smem_raw[];
    T *te = reinterpret_cast<T *>(smem_raw);
    T *td = te + 3 * wmax;
    const PairRec &r = pairs[p0 + blockIdx.x];
    pair_tables<T>(r, G, te, td, wmax);
    __syncthreads();
    T acc[NA * NB];
#pragma unroll
    for (int i = 0; i < NA * NB; ++i) acc[i] = T(0);
    const T abx = (T)r.AB[0], aby = (T)r.AB[1], abz = (T)r.AB[2];
    for_each_point<T>(r, G, te, td, wmax, [&](bool valid, T E, T xa, T ya, T za, long long widx) {
        const T f = valid ? (T)V[widx] * E : T(0);
        T a[NA], bb[NB];
        monomials<LA, T>(xa, ya, za, a);
        monomials<LB, T>(xa + abx, ya + aby, za + abz, bb);
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const T fa = f * a[i];
#pragma unroll
            for (int j = 0; j < NB; ++j) acc[i * NB + j] += fa * bb[j];
        }
    });
    const double scale = 0.5 * G.w * r.Kw;
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const double v = wave_sum((double)acc[i * NB + j]);
            if (threadIdx.x == 0) {
                atomicAdd(&M[(long long)(r.ao_a + i) * n_ao + r.ao_b + j], scale * v);
                atomicAdd(&M[(long long)(r.ao_b + j) * n_ao + r.ao_a + i], scale * v);
            }
        }
}

template <int LA, int LB, typename T>
__global__ void __launch_bounds__(64)
k_grad(const PairRec *__restrict__ pairs, long long p0, LevelGeom G, const T *__restrict__ Dm, int n_ao,
       const double *__restrict__ V, double *__restrict__ grad, int wmax)
{
    constexpr int NA = ncart_c(LA), NB = ncart_c(LB);
    extern __shared__ unsigned char smem_raw[];
    T *te = reinterpret_cast<T *>(smem_raw);
    T *td = te + 3 * wmax;
    const PairRec &r = pairs[p0 + blockIdx.x];
    pair_tables<T>(r, G, te, td, wmax);
    __syncthreads();
    T gA[3] = {0, 0, 0}, gB[3] = {0, 0, 0};
    const T abx = (T)r.AB[0], aby = (T)r.AB[1], abz = (T)r.AB[2];
    const T two_aa = (T)(2.0 * r.aa), two_ab = (T)(2.0 * r.ab);
    const T *Dp = Dm + (long long)r.ao_a * n_ao + r.ao_b;
    for_each_point<T>(r, G, te, td, wmax, [&](bool valid, T E, T xa, T ya, T za, long long widx) {
        const T f = valid ? (T)V[widx] * E : T(0);
        const T xb = xa + abx, yb = ya + aby, zb = za + abz;
        T a[NA], bb[NB], t[NA], sv[NB];
        monomials<LA, T>(xa, ya, za, a);
        monomials<LB, T>(xb, yb, zb, bb);
#pragma unroll
        for (int j = 0; j < NB; ++j) sv[j] = T(0);
        T S0 = T(0);
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            T ti = T(0);
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const T dij = Dp[(long long)i * n_ao + j];
                ti += dij * bb[j];
                sv[j] += dij * a[i];
            }
            t[i] = ti;
            S0 += a[i] * ti;
        }
        T pa[3], pb[3];
        poly_grad<LA, T>(xa, ya, za, t, pa);
        poly_grad<LB, T>(xb, yb, zb, sv, pb);
        const T fS = f * S0;
        gA[0] += two_aa * fS * xa - f * pa[0];
        gA[1] += two_aa * fS * ya - f * pa[1];
        gA[2] += two_aa * fS * za - f * pa[2];
        gB[0] += two_ab * fS * xb - f * pb[0];
        gB[1] += two_ab * fS * yb - f * pb[1];
        gB[2] += two_ab * fS * zb - f * pb[2];
    });
    const double scale = G.w * r.Kw;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double va = wave_sum((double)gA[d]);
        const double vb = wave_sum((double)gB[d]);
        if (threadIdx.x == 0) {
            atomicAdd(&grad[3 * r.atom_a + d], scale * va);
            atomicAdd(&grad[3 * r.atom_b + d], scale * vb);
        }
    }
}

// ------------------------------------------------------------ launchers

template <typename F>
static void dispatch_cls(int c, F &&f)
{
    switch (c) {
    case 0: f(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{}); break;
    case 1: f(std::integral_constant<int, 1>{}, std::integral_constant<int, 0>{}); break;
    case 2: f(std::integral_constant<int, 1>{}, std::integral_constant<int, 1>{}); break;
    case 3: f(std::integral_constant<int, 2>{}, std::integral_constant<int, 0>{}); break;
    case 4: f(std::integral_constant<int, 2>{}, std::integral_constant<int, 1>{}); break;
    case 5: f(std::integral_constant<int, 2>{}, std::integral_constant<int, 2>{}); break;
    case 6: f(std::integral_constant<int, 3>{}, std::integral_constant<int, 0>{}); break;
    case 7: f(std::integral_constant<int, 3>{}, std::integral_constant<int, 1>{}); break;
    case 8: f(std::integral_constant<int, 3>{}, std::integral_constant<int, 2>{}); break;
    default: f(std::integral_constant<int, 3>{}, std::integral_constant<int, 3>{}); break;
    }
}

static inline unsigned nb256(long long n) { return (unsigned)((n + 255) / 256); }

template <typename T>
static hipError_t sym_density(const gpw_plan_s *pl, const double *D, T **out, hipStream_t st)
{
    const long long nn = (long long)pl->n_ao * pl->n_ao;
    hipError_t e = hipMallocAsync((void **)out, sizeof(T) * (size_t)(nn > 0 ? nn : 1), st);
    if (e != hipSuccess) return e;
    if (nn > 0) hipLaunchKernelGGL(k_symmetrize<T>, dim3(nb256(nn)), dim3(256), 0, st, D, *out, pl->n_ao);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_rho(const gpw_plan_s *pl, const double *D, double *const *rho, hipStream_t st)
{
    T *Ds = nullptr;
    hipError_t e = sym_density<T>(pl, D, &Ds, st);
    if (e != hipSuccess) return e;
    for (int l = 0; l < pl->nlevels; ++l) {
        hipLaunchKernelGGL(k_fill, dim3(nb256(pl->ngrid[l])), dim3(256), 0, st, rho[l], pl->ngrid[l], 0.0);
        for (int c = 0; c < kNCls; ++c) {
            const int g = l * kNCls + c;
            const long long nb = pl->blk_off[g + 1] - pl->blk_off[g];
            if (nb <= 0) continue;
            dispatch_cls(c, [&](auto la, auto lb) {
                hipLaunchKernelGGL((k_rho<decltype(la)::value, decltype(lb)::value, T>), dim3((unsigned)nb), dim3(64), 0, st,
                                   (const PairRec *)pl->d_pairs, (const int2 *)pl->d_inc,
                                   (const long long *)pl->d_inc_off, pl->cnt_base[g],
                                   (const int *)(pl->d_blk + pl->blk_off[g]), pl->geom[l], (const T *)Ds,
                                   pl->n_ao, rho[l]);
            });
        }
    }
    e = hipGetLastError();
    (void)hipFreeAsync(Ds, st);
    return e;
}

template <typename T>
static size_t pair_smem(const gpw_plan_s *pl) { return sizeof(T) * 6 * (size_t)(pl->info.max_box_width + 8); }

template <typename T>
static hipError_t launch_mat(const gpw_plan_s *pl, const double *const *v, double *M, hipStream_t st)
{
    const long long nn = (long long)pl->n_ao * pl->n_ao;
    hipLaunchKernelGGL(k_fill, dim3(nb256(nn)), dim3(256), 0, st, M, nn, 0.0);
    const int wmax = pl->info.max_box_width + 8;
    for (int l = 0; l < pl->nlevels; ++l)
        for (int c = 0; c < kNCls; ++c) {
            const int g = l * kNCls + c;
            const long long np = pl->group_off[g + 1] - pl->group_off[g];
            if (np <= 0) continue;
            dispatch_cls(c, [&](auto la, auto lb) {
                hipLaunchKernelGGL((k_mat<decltype(la)::value, decltype(lb)::value, T>), dim3((unsigned)np), dim3(64),
                                   pair_smem<T>(pl), st, (const PairRec *)pl->d_pairs, pl->group_off[g], pl->geom[l],
                                   v[l], M, pl->n_ao, wmax);
            });
        }
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_grad(const gpw_plan_s *pl, const double *D, const double *const *v, double *grad,
                              hipStream_t st)
{
    T *Ds = nullptr;
    hipError_t e = sym_density<T>(pl, D, &Ds, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fill, dim3(nb256(3LL * pl->natm)), dim3(256), 0, st, grad, 3LL * pl->natm, 0.0);
    const int wmax = pl->info.max_box_width + 8;
    for (int l = 0; l < pl->nlevels; ++l)
        for (int c = 0; c < kNCls; ++c) {
            const int g = l * kNCls + c;
            const long long np = pl->group_off[g + 1] - pl->group_off[g];
            if (np <= 0) continue;
            dispatch_cls(c, [&](auto la, auto lb) {
                hipLaunchKernelGGL((k_grad<decltype(la)::value, decltype(lb)::value, T>), dim3((unsigned)np), dim3(64),
                                   pair_smem<T>(pl), st, (const PairRec *)pl->d_pairs, pl->group_off[g], pl->geom[l],
                                   (const T *)Ds, pl->n_ao, v[l], grad, wmax);
            });
        }
    e = hipGetLastError();
    (void)hipFreeAsync(Ds, st);
    return e;
}

hipError_t eval_rho(const gpw_plan_s *pl, const double *D, double *const *rho, hipStream_t st)
{
    return pl->precision == GPW_FP32 ? launch_rho<float>(pl, D, rho, st) : launch_rho<double>(pl, D, rho, st);
}

hipError_t eval_mat(const gpw_plan_s *pl, const double *const *v, double *M, hipStream_t st)
{
    return pl->precision == GPW_FP32 ? launch_mat<float>(pl, v, M, st) : launch_mat<double>(pl, v, M, st);
}

hipError_t eval_grad(const gpw_plan_s *pl, const double *D, const double *const *v, double *grad, hipStream_t st)
{
    return pl->precision == GPW_FP32 ? launch_grad<float>(pl, D, v, grad, st)
                                     : launch_grad<double>(pl, D, v, grad, st);
}

}  // namespace gpw
