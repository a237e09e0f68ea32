// Internal declarations shared by the host code and the HIP kernels of libgpw.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/gpw.h"

namespace gpw {

constexpr int kMaxLevels = GPW_MAX_LEVELS;
constexpr int kNCls = GPW_NCLASS;
constexpr int kMaxGroups = kMaxLevels * kNCls;   // (level, class) groups

__host__ __device__ inline int ncart(int l) { return (l + 1) * (l + 2) / 2; }
__host__ __device__ constexpr int ncart_c(int l) { return (l + 1) * (l + 2) / 2; }
// class index of (la, lb), la >= lb: ss ps pp ds dp dd fs fp fd ff gs gp gd gf gg
__host__ __device__ inline int cls_of(int la, int lb) { return la * (la + 1) / 2 + lb; }
__host__ __device__ constexpr int cls_la_c(int c)
{
    int la = 0;
    while ((la + 1) * (la + 2) / 2 <= c) ++la;
    return la;
}
__host__ __device__ constexpr int cls_lb_c(int c) { return c - cls_la_c(c) * (cls_la_c(c) + 1) / 2; }
__host__ __device__ inline int cls_la(int c) { return cls_la_c(c); }
__host__ __device__ inline int cls_lb(int c) { return cls_lb_c(c); }

// Monomials (x-A_x)^lx (y-A_y)^ly (z-A_z)^lz of total degree <= L.
__host__ __device__ constexpr int ntab(int L) { return (L + 1) * (L + 2) * (L + 3) / 6; }

// Whether the rho kernel of class (la, lb) evaluates a pair image's density
// through its coefficient tensor (Sec. III.A, Eq. (rho1): ntab(la + lb)
// values per pair image) or directly as sum_ij D_ij a_i b_j (n_a n_b
// values): the tensor needs fewer operations per point, the direct form
// offers more independent operations; chosen per class by measurement on
// the 256-water system.
__host__ __device__ constexpr bool rho_tensor(int la, int lb)
{
    return la == 2 || la == 3 || (la == 4 && lb >= 1);
}
// Whether the mat kernel of class (la, lb) accumulates the potential moments
// of the monomials of r - A one axis at a time and forms the matrix elements
// from them once per pair image (the integration analogue of Eq. (rho1)), or
// accumulates the n_a n_b products a_i b_j per point directly.
__host__ __device__ constexpr bool mat_tensor(int la, int lb) { return la + lb >= 2; }
__host__ __device__ constexpr int rho_ncoef(int la, int lb)
{
    return rho_tensor(la, lb) ? ntab(la + lb) : ncart_c(la) * ncart_c(lb);
}

// One canonical pair image (unordered pair of primitive shells plus the
// lattice translation of the second one).  The first factor carries the
// higher angular momentum.  256 bytes.
struct alignas(64) PairRec {
    double A[3];      // centre of the first primitive
    double AB[3];     // A - B', B' = centre of the second primitive incl. image
    double P[3];      // product centre
    double aa, ab;    // exponents of the first and second primitive
    double Kw;        // w_c * c_a c_b exp(-a b / (a+b) |A - B'|^2), w_c = 1 or 2
    double R2;        // squared truncation radius
    double ER;        // exp(-(a+b) R^2): point kept iff envelope >= ER
    double c[3];      // exp(-(a+b) h_d^2) on the pair's level (grid-step factor)
    // the 4x4x4 blocks the bounding box meets, per axis: the first one's
    // wrapped index k0 and period shift s0 (unwrapped = k0 + s0 nb), their
    // count n, and the first z entry whose upper end reaches P (em)
    int bk0[3], bs0[3], bn[3], bem;
    int bpad[2];
    int ao_a, ao_b;   // first AO of each shell
    int atom_a, atom_b;
    int lo[3], hi[3]; // unwrapped bounding box of the sphere on the pair's level
    int la, lb, level, cls;
    int pad2, pad3;
};
static_assert(sizeof(PairRec) == 256, "PairRec layout");

// Compact per-pair geometry read by the rho kernel (one 128-byte line).
struct alignas(128) RhoRec {
    double A[3];      // centre of the first primitive
    double AB[3];     // A - B'
    double P[3];      // product centre
    double ap;        // alpha_p
    double Kw;        // w_c c_a c_b exp(-a b / (a+b) |A - B'|^2)
    double ER;        // exp(-alpha_p R^2)
    double c[3];      // exp(-alpha_p h_d^2)
    double pad;
};
static_assert(sizeof(RhoRec) == 128, "RhoRec layout");

// Highest degree of the monomial transforms of a general cell (the moments of
// the meta-GGA gradient of a (g|g) pair).
constexpr int kMaxTDeg = 11;

// Geometry of one level of a general (non-orthogonal) cell, in device memory.
// Grid point i sits at r = sum_d i_d h_d with the step vectors h_d = a_d / N_d;
// the kernels then work in grid-index coordinates s (r = s H, H the rows h_d):
// positions, products and offsets in index units, the envelope
// exp(-alpha |r - P|^2) = exp(-alpha (s - s_P)^T g (s - s_P)) with the metric
// g = H H^T, whose off-diagonal terms give the cross factors of the
// non-orthogonal recursion.  Cartesian monomials of r - A and monomials of
// the index offset s - s_A of the same degree n are related by T_n:
// (r - A)^m = sum_k T_n[m][k] (s - s_A)^k (m, k Cartesian exponents in shell
// order).
struct TriGeom {
    double H[3][3];        // step vectors as rows (bohr)
    double Hinv[3][3];     // s = r Hinv
    double g[3][3];        // metric h_d . h_e
    double lmin;           // smallest eigenvalue of g: |r|^2 >= lmin |s|^2
    double rf[3];          // |Hinv[:, d]|: index-box half width per unit radius
    int toff[kMaxTDeg + 1];   // offset of T_n in T
    const double *T;       // T_n, n = 0..kMaxTDeg, row-major ncart(n) x ncart(n)
};

// Per-level geometry passed by value to kernels.
struct LevelGeom {
    int N[3];         // mesh
    int nb[3];        // 4^3 blocks per axis (ceil(N/4))
    double h[3];      // grid spacing (index units, 1, for a general cell)
    double w;         // quadrature weight Omega / N_l
    const TriGeom *tri;   // general cell: device geometry of the level; nullptr: orthorhombic
};

// Slot of a 4x4x4 block in the per-group incidence lists: tiles of 8x8x8
// blocks in row-major order, Morton (z-order) inside a tile, so that a run
// of consecutive slots is a compact region of space (neighbouring blocks
// share most of their pair images).  Slots of padding blocks of partial
// tiles stay empty.
__host__ __device__ inline int spread3(int v)   // 3 bits -> bits 0, 3, 6
{
    return (v & 1) | ((v & 2) << 2) | ((v & 4) << 4);
}
__host__ __device__ inline int gather3(int v) { return (v & 1) | ((v >> 2) & 2) | ((v >> 4) & 4); }
__host__ __device__ inline long long block_slot(const LevelGeom &G, int kx, int ky, int kz)
{
    const int ty = (G.nb[1] + 7) >> 3, tz = (G.nb[2] + 7) >> 3;
    const long long tile = ((long long)(kx >> 3) * ty + (ky >> 3)) * tz + (kz >> 3);
    return tile * 512 + ((spread3(kx & 7) << 2) | (spread3(ky & 7) << 1) | spread3(kz & 7));
}
__host__ __device__ inline void slot_block(const LevelGeom &G, long long slot, int &kx, int &ky, int &kz)
{
    const int ty = (G.nb[1] + 7) >> 3, tz = (G.nb[2] + 7) >> 3;
    const long long tile = slot >> 9;
    const int m = (int)(slot & 511);
    const int tkz = (int)(tile % tz), tky = (int)((tile / tz) % ty), tkx = (int)(tile / ((long long)tz * ty));
    kx = tkx * 8 + gather3(m >> 2);
    ky = tky * 8 + gather3(m >> 1);
    kz = tkz * 8 + gather3(m);
}
inline long long block_slots(const LevelGeom &G)
{
    return (long long)((G.nb[0] + 7) >> 3) * ((G.nb[1] + 7) >> 3) * ((G.nb[2] + 7) >> 3) * 512;
}

// Incidence entry: pair index and the fold shifts (unwrapped = wrapped + S*N).
__host__ __device__ inline int pack_shift(int sx, int sy, int sz)
{
    return (sx + 128) | ((sy + 128) << 8) | ((sz + 128) << 16);
}
__host__ __device__ inline int shift_of(int packed, int d) { return ((packed >> (8 * d)) & 0xff) - 128; }

// Squared distance from P to the axis-aligned box [x0, x1] per axis.
__host__ __device__ inline double axis_gap2(double p, double x0, double x1)
{
    double g = p < x0 ? x0 - p : (p > x1 ? p - x1 : 0.0);
    return g * g;
}

// Conservative factor for block culling: a block is visited when its closest
// point lies within R (1 + 1e-12); the per-point test decides exactly.
constexpr double kCullSlack = 1.0 + 1e-12;

// Widest bounding box (points per axis) of one pair image: the pair-major
// kernels keep its 1-D tables in LDS.
constexpr int kMaxBoxWidth = 1024;

__device__ inline long long floordiv(long long a, long long b)
{
    long long q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}
__device__ inline int floordiv(int a, int b)
{
    int q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}

// Per-axis enumeration of the (block, fold shift) pairs whose unwrapped
// points [4k + S N, min(4k+3, N-1) + S N] meet [lo, hi]: k runs over the
// wrapped 4-point blocks of a mesh of N points (the last one may be partial),
// S over the lattice images.  Unwrapped point u = w + S N, wrapped w = 4k + t.
struct AxisIter {
    int S, Send, k, kend;
    int N, nb, lo, hi;
    __device__ void start(int lo_, int hi_, int N_, int nb_)
    {
        lo = lo_; hi = hi_; N = N_; nb = nb_;
        S = (int)floordiv(lo, N);
        Send = (int)floordiv(hi, N);
        if (hi < lo) { S = Send + 1; return; }
        set_k();
        skip_empty();
    }
    __device__ void set_k()
    {
        const int base = S * N;
        k = (int)floordiv(lo - base, 4);
        if (k < 0) k = 0;
        kend = (int)floordiv(hi - base, 4);
        if (kend > nb - 1) kend = nb - 1;
    }
    __device__ void skip_empty()
    {
        while (S <= Send && k > kend) { ++S; if (S <= Send) set_k(); }
    }
    __device__ bool valid() const { return S <= Send; }
    __device__ void next()
    {
        if (++k > kend) { ++S; if (S <= Send) { set_k(); skip_empty(); } }
    }
    // unwrapped coordinate range of the current block
    __device__ void range(double h, double &x0, double &x1) const
    {
        const int u0 = 4 * k + S * N;
        const int u1 = (4 * k + 3 < N - 1 ? 4 * k + 3 : N - 1) + S * N;
        x0 = (double)u0 * h;
        x1 = (double)u1 * h;
    }
};

// The 4-point blocks (with their fold shifts) that an unwrapped index range
// [lo, hi] of one axis meets, in increasing order of the unwrapped index: the
// unwrapped index u lies in block k = (u - S N) / 4 of period S = floor(u / N);
// numbered g(u) = S nb + k these blocks form the contiguous range
// [g(lo), g(hi)] (g grows by at most one per index), so entry e of the list
// is g(lo) + e.  The same list as AxisIter, in closed form.
__device__ inline int axis_block_id(int u, int N, int nb)
{
    const int S = floordiv(u, N);
    return S * nb + (u - S * N) / 4;
}
__device__ inline int axis_block_count(int lo, int hi, int N, int nb)
{
    return hi < lo ? 0 : axis_block_id(hi, N, nb) - axis_block_id(lo, N, nb) + 1;
}

// Workgroups are dealt to the eight XCDs round robin (workgroup b runs on XCD
// b % 8); a segment's workgroup range is padded to a multiple of 8.
inline unsigned xcd_grid(long long n) { return (unsigned)(8 * ((n + 7) / 8)); }
// Workgroup b of a segment whose items are dealt to the eight XCDs in
// contiguous ranges [xs[x], xs[x + 1]) of about equal work (each XCD, with its
// own L2, walks one spatially compact part of the group): its item, or -1 past
// its XCD's range.  The segment has 8 max_x (xs[x + 1] - xs[x]) workgroups.
__device__ inline long long xcd_ranged(long long b, const int *xs)
{
    const int x = (int)(b & 7);
    const long long it = xs[x] + (b >> 3);
    return it < xs[x + 1] ? it : -1;
}

struct PsTable {
    const int *atom, *l, *ao;
    const double *alpha, *coef, *coords;
    int n;
};

struct PlanConst {
    double L[3];          // |a_d|
    int tri;              // general cell
    double A[3][3];       // lattice vectors as rows
    double Ainv[3][3];    // r = u A, u = r Ainv (fractional coordinates)
    double logtau;
    double rel_cut;
    int nlevels;
    double cut[kMaxLevels];
    LevelGeom geom[kMaxLevels];
};

struct PartitionInput {
    PsTable ps;
    PlanConst pc;
};

struct PoissonState;   // FFT plans of the multigrid transfer (gpw_poisson.hip)

}  // namespace gpw

struct gpw_plan_s {
    int device = 0;
    int precision = GPW_FP64;
    double L[3] = {0, 0, 0};          // |a_d|
    int tri = 0;                      // general (non-orthogonal) cell
    double A[3][3] = {};              // lattice vectors as rows
    double recip[3][3] = {};          // reciprocal vectors b_d = 2 pi (A^-1)[:, d] as rows
    double volume = 0.0;
    gpw::TriGeom tri_host[gpw::kMaxLevels] = {};   // host copies (device pointers inside)
    gpw::TriGeom *d_tri = nullptr;                 // per level, device
    int nlevels = 0;
    gpw::LevelGeom geom[gpw::kMaxLevels];
    long long ngrid[gpw::kMaxLevels] = {};
    long long nblocks[gpw::kMaxLevels] = {};
    int natm = 0, nshell = 0, n_ao = 0, n_ps = 0;
    double tau = 1e-6, rel_cut = 60.0;
    double cut_ry[gpw::kMaxLevels] = {};

    // primitive shells
    int *d_ps_atom = nullptr, *d_ps_l = nullptr, *d_ps_ao = nullptr;
    double *d_ps_alpha = nullptr, *d_ps_coef = nullptr, *d_coords = nullptr;

    // canonical pair images grouped by (level, class)
    gpw::PairRec *d_pairs = nullptr;
    gpw::RhoRec *d_rrec = nullptr;   // compact copy for the rho kernel
    long long n_pairs = 0;
    long long group_off[gpw::kMaxGroups + 1] = {};

    // block incidences: counters per (group, block), CSR offsets, entries
    long long cnt_base[gpw::kMaxGroups + 1] = {};   // counter index base per group
    long long *d_inc_off = nullptr;                  // cnt_base[last] + 1 offsets
    int2 *d_inc = nullptr;
    long long n_inc = 0;
    // compacted nonempty blocks per group
    int *d_blk = nullptr;
    long long blk_off[gpw::kMaxGroups + 1] = {};
    // per group, the nonempty blocks (collocation) and the pair images
    // (pair-major kernels) dealt to the eight XCDs: contiguous item ranges
    // [xsplit[g][x], xsplit[g][x + 1]) of about equal work
    int xsplit[gpw::kMaxGroups][9] = {};
    int xsplit_pair[gpw::kMaxGroups][9] = {};

    gpw_plan_info info{};
    int max_axis_blocks = 0;   // longest per-axis block list of a pair image
    std::vector<void *> allocations;

    // multigrid transfer + Poisson: FFT plans, created on first use
    gpw::PoissonState *poisson = nullptr;
    std::mutex poisson_mu;
};

namespace gpw {
// One evaluation of a batch (the fields of gpw_task after validation).
struct TaskRef {
    const gpw_plan_s *pl;
    int op;                   // gpw_op
    const double *D;
    const double *const *v;
    double *const *rho;
    double *out;
};
hipError_t eval_batch(const TaskRef *tasks, int n, hipStream_t st);
// The allocation-free evaluation: scratch comes from a fixed per-device array
// of kNoAllocScratchBytes (its size is checked by the caller beforehand).
constexpr size_t kNoAllocScratchBytes = GPW_NOALLOC_SCRATCH_BYTES;
hipError_t eval_noalloc(const TaskRef &t, hipStream_t st);
// Address of that array on device dev, looked up on the first call for dev
// (which must be the current device then) and cached.
hipError_t noalloc_scratch(int dev, unsigned char **ptr);
// Device scratch one evaluation of op (gpw_op) takes from the stream-ordered pool.
size_t eval_scratch_bytes(const gpw_plan_s *pl, int op);
// Multigrid transfer + Poisson solve (gpw_poisson.hip): enqueue on st; free
// the FFT plans; device bytes of the spectra one call takes from the pool
// (the FFT library's work area comes on top).
hipError_t poisson_run(gpw_plan_s *pl, const double *const *rho, const double *vxc, const double *const *vxc_grad,
                       double *const *v, double *ej, hipStream_t st);
// density (and optionally its gradient) on the finest mesh from the level densities
hipError_t fine_density_run(gpw_plan_s *pl, const double *const *rho, double *rho_fine, double *const *grad,
                            hipStream_t st);
void poisson_free(gpw_plan_s *pl);
size_t poisson_spectra_bytes(const gpw_plan_s *pl);
// LDS bytes a workgroup of the pair-major kernels (mat, grad) needs for a plan
// whose longest per-axis block list of a pair image has emax entries.
size_t pair_kernel_lds_bytes(int emax, int precision, bool tri);
}  // namespace gpw
