// Kernel templates of libgpw for gfx950: collocation (rho, tau), integration
// (mat, mat_tau) and gradient (grad, grad_tau) per (l_a, l_b) class, their
// device helpers, the segment tables the launches pass by value, and the host
// containers that collect segments.  Included by the host batching code
// (gpw_eval.hip) and by the per-class launch source (gpw_class.hip, compiled
// once per class), so that each class's kernels compile in their own
// translation unit.
//
// rho  - grid-block major, after Alg. 1 of the paper, mapped to CDNA: one
//        wave64 owns one 4x4x4 block of one level and walks the block's list
//        of pair images in batches of 64, lane = pair image.  Each lane holds
//        its image's geometry and coefficients in registers, evaluates the
//        separable envelope of Sec. III.A (Eqs. (gx), (gab), (exp_rr)) on the
//        block's 64 points and the polynomial prefactor per point, either
//        through the coefficient tensor of Eq. (rho1) by Horner's rule one
//        axis at a time (d and f classes) or directly from the Kw-scaled D
//        sub-block (s and p classes), and accumulates the 64 point values in
//        registers; one LDS transpose-reduction per block sums the lanes and
//        each point is written once.
// mat  - pair major: one wave per pair image walks the 4x4x4 blocks its
//        truncation sphere meets (the same block set as rho), lane = point,
//        accumulating over all blocks either the potential moments of the
//        monomials of r - A one axis at a time (the integration analogue of
//        Eq. (rho1), l_a + l_b >= 2) or the n_a x n_b local integrals (Alg. 2's
//        F^local), then one wave reduction and one atomic add per matrix
//        element per pair image instead of one per (pair, block).
// grad - same traversal as mat, moments one degree higher, from which the
//        d/dA and d/dB contributions of Alg. 3 are formed and contracted
//        with D once per pair image.
// Every kernel is templated on (l_a, l_b) and on the per-point arithmetic
// type (double, or float for the FP32 variant; exponents, centres and the
// cross-level/matrix accumulation stay in double).
//
// Launches: a kernel launch covers one (operation, class) for any number of
// (task, level) segments, described by a table passed by value; a work item
// (grid block or pair image) finds its segment from the table.  A single
// evaluation is a batch of one task, so batched and single calls run the
// same kernels in the same order.

#pragma once

#include "gpw_internal.h"

#include <utility>

namespace gpw {

// ------------------------------------------------------- segment tables

constexpr int kMaxSeg = 16;

// Segments of one launch: segment k owns the workgroups [s[k].item0,
// s[k+1].item0) (the last one up to total).
template <typename S>
struct SegTable {
    S s[kMaxSeg];
    long long total;
    int n;
};

template <typename S>
__device__ __forceinline__ int seg_of(const SegTable<S> &t, long long item)
{
    int k = 0;
    for (int j = 1; j < t.n; ++j) k = item >= t.s[j].item0 ? j : k;
    return k;
}

// element-wise segments, one 256-thread block per item
struct FillSeg { long long item0; double *p; long long count; };
struct GridSeg { long long item0; const double *v; double *vb; long long count; int vz; LevelGeom G; };
struct SymSeg { long long item0; const double *D; void *out; int n, nt; };
// tri (a general cell): the coefficients are formed on the Cartesian
// monomials and written in FP64 to tmp, for k_to_index
struct PackSeg {
    long long item0; const PairRec *pairs; const double *D; void *out; long long count; int n;
    const TriGeom *tri; double *tmp;
};
// Cartesian coefficient tensors of degree L (K = ntab(L) per pair image, in
// src) rewritten on the monomials of the index offset into dst (stride cs)
struct IdxSeg { long long item0; const double *src; void *dst; long long count; int L, K, cs; const TriGeom *tri; };
// one wave per grid block (rho) or per pair image (mat, grad)
// Their items are mapped with xcd_ranged inside the segment, so that every
// segment (a level of a task) is spread over all eight XCDs in contiguous
// ranges of about equal work, as a launch of its own would be.
struct RhoSeg {
    long long item0;
    long long count;             // nonempty blocks
    const RhoRec *rr;            // records of the (level, class) group
    const int2 *inc;             // (pair image, shift) entries
    const long long *inc_off;    // CSR offsets of the group's blocks
    const int *blk;              // slots of the group's nonempty blocks
    const void *Dpk;             // packed D sub-blocks of the group
    double *rho;                 // level grid
    int p0;                      // plan index of the group's first pair image
    int xs[9];                   // items of the eight XCDs (xcd_ranged), balanced by work
    LevelGeom G;
};
// Blocks of slack past the end of a block copy: the pair-major traversal
// always loads four whole blocks from a run's start.
constexpr int kBlockCopyTail = 4;
struct PairSeg {
    long long item0;
    long long count;             // pair images
    const PairRec *pairs;        // records of the (level, class) group
    const void *Dm;              // grad: symmetrised D
    const double *Vb;            // block-ordered level potential, vz blocks per (x, y) column
    double *out;                 // mat: M; grad: natm x 3
    int n_ao, emax, vz;
    int row_cap;                 // block rows the LDS holds (row_capacity(emax))
    int xs[9];                   // items of the eight XCDs (xcd_ranged), balanced by work
    LevelGeom G;
};

// ------------------------------------------------------- Cartesian helpers

// Index of (lx, ly, lz) inside its shell, lexicographic order lx desc, ly desc.
__host__ __device__ constexpr int cart_index(int ly, int lz) { return (ly + lz) * (ly + lz + 1) / 2 + lz; }
// Components of the n-th Cartesian function of a shell of degree L.
__host__ __device__ constexpr int cart_ly(int L, int n)
{
    int lx = L;
    while (n > L - lx) {
        n -= L - lx + 1;
        --lx;
    }
    return L - lx - n;
}
__host__ __device__ constexpr int cart_lx(int L, int n)
{
    int lx = L;
    while (n > L - lx) {
        n -= L - lx + 1;
        --lx;
    }
    return lx;
}
__host__ __device__ constexpr int binom(int n, int k)
{
    int b = 1;
    for (int i = 0; i < k; ++i) b = b * (n - i) / (i + 1);
    return b;
}

// Coefficient tensor of a pair image (Sec. III.A, Eqs. (binomial), (rho1)):
// with every product of a Cartesian function on A and one on B written as a
// polynomial in r - A (the factor (x - B_x)^b expanded binomially around A),
// a pair image's density or potential moments live on the monomials
// (x-A_x)^lx (y-A_y)^ly (z-A_z)^lz of total degree <= L = l_a + l_b.  They are
// packed lx-major, then ly, then lz: ntab(L) entries.
__host__ __device__ constexpr int tidx(int L, int lx, int ly, int lz)
{
    int n = 0;
    for (int a = 0; a < lx; ++a) n += (L - a + 1) * (L - a + 2) / 2;
    for (int b = 0; b < ly; ++b) n += L - lx - b + 1;
    return n + lz;
}
// (ly, lz) pairs of total degree <= L, ly-major
__host__ __device__ constexpr int ntab2(int L) { return (L + 1) * (L + 2) / 2; }
__host__ __device__ constexpr int t2idx(int L, int ly, int lz)
{
    int n = 0;
    for (int b = 0; b < ly; ++b) n += L - b + 1;
    return n + lz;
}

// (ly, lz) of entry k of the ly-major (ly, lz) list (inverse of t2idx)
__host__ __device__ constexpr int t2_ly(int L, int k)
{
    int ly = 0;
    while (k >= L - ly + 1) {
        k -= L - ly + 1;
        ++ly;
    }
    return ly;
}
__host__ __device__ constexpr int t2_lz(int L, int k)
{
    int ly = 0;
    while (k >= L - ly + 1) {
        k -= L - ly + 1;
        ++ly;
    }
    return k;
}

// The Cartesian monomials of degree L in shell order, each one product of
// powers (expanded by a fold over the components, so every index is a
// compile-time constant).
template <int LX, int LY, int LZ, typename T>
__device__ __forceinline__ T mono_term(const T *px, const T *py, const T *pz)
{
    T v = px[LX];
    if constexpr (LY > 0) v = v * py[LY];
    if constexpr (LZ > 0) v = v * pz[LZ];
    return v;
}
template <int L, typename T, int... N>
__device__ __forceinline__ void mono_all(const T *px, const T *py, const T *pz, T *m, std::integer_sequence<int, N...>)
{
    ((m[N] = mono_term<cart_lx(L, N), cart_ly(L, N), L - cart_lx(L, N) - cart_ly(L, N), T>(px, py, pz)), ...);
}
template <int L, typename T>
__device__ __forceinline__ void monomials(T x, T y, T z, T *m)
{
    T px[L + 1], py[L + 1], pz[L + 1];
    px[0] = py[0] = pz[0] = T(1);
#pragma unroll
    for (int i = 1; i <= L; ++i) { px[i] = px[i - 1] * x; py[i] = py[i - 1] * y; pz[i] = pz[i - 1] * z; }
    mono_all<L, T>(px, py, pz, m, std::make_integer_sequence<int, ncart_c(L)>{});
}

// --------------------------------------------------------- small kernels



// ------------------------------------------------------------------ rho

// Separable Gaussian envelope of a pair image on the 4x4x4 points of a block,
// exp(-alpha |r - P|^2) = fx[tx] fy[ty] fz[tz], from four exps: the value at
// the block's first point and one ratio g_d = exp(-2 alpha h_d d_d) per axis;
// along each axis the factors then follow the grid recursion
// f_{t+1} = f_t g c^(2t+1), c = exp(-alpha h^2) (Sec. III.A, Eqs. (exp_rr),
// (exp_rr1)).  Direct exps per point factor when a ratio would overflow.
__device__ __forceinline__ void block_envelope(double alpha, const double *d, const LevelGeom &G,
                                               const double *c, double *fx, double *fy, double *fz)
{
    double *f[3] = {fx, fy, fz};
    const double a0 = 2.0 * alpha * G.h[0] * d[0], a1 = 2.0 * alpha * G.h[1] * d[1],
                 a2 = 2.0 * alpha * G.h[2] * d[2];
    if (fabs(a0) < 600.0 && fabs(a1) < 600.0 && fabs(a2) < 600.0) {
        const double an[3] = {a0, a1, a2};
        f[0][0] = exp(-alpha * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]));
        f[1][0] = 1.0;
        f[2][0] = 1.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double c2 = c[k] * c[k];
            double q = exp(-an[k]) * c[k];
            f[k][1] = f[k][0] * q;
            q *= c2;
            f[k][2] = f[k][1] * q;
            q *= c2;
            f[k][3] = f[k][2] * q;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const double x = d[k] + t * G.h[k];
                f[k][t] = exp(-alpha * x * x);
            }
    }
}

// General cell (index coordinates s, metric g; the non-orthogonal recursion
// of the appendix applied block-wise): with d = s0 - s_P at the block's first
// point and t the offset in the block,
//   exp(-alpha (d + t)^T g (d + t)) = fx[tx] fy[ty] fz[tz] Qxy^(tx ty) Qxz^(tx tz) Qyz^(ty tz),
// fx[0] = exp(-alpha d^T g d), fy[0] = fz[0] = 1, per axis the recursion
// f_{t+1} = f_t exp(-2 alpha (g d)_k) c_k^(2t+1) with c_k = exp(-alpha g_kk),
// and the cross factors Q_de = exp(-2 alpha g_de).  Single factors can be
// large where the Gaussian is sharp on the level's grid far from the block;
// when one could leave the FP64 range the lane takes one exp per point
// instead (direct).
struct TriEnv {
    double q[3];     // Qxy, Qxz, Qyz
    double ap, qd;   // alpha_p and d^T g d (direct form)
    double gd[3];    // g d (direct form)
    bool direct;
};
__device__ __forceinline__ void block_envelope_tri(double alpha, const double *d, const TriGeom *tg, const double *c,
                                                   double *fx, double *fy, double *fz, TriEnv &te)
{
    double *f[3] = {fx, fy, fz};
    const double(*g)[3] = tg->g;
#pragma unroll
    for (int k = 0; k < 3; ++k) te.gd[k] = g[k][0] * d[0] + g[k][1] * d[1] + g[k][2] * d[2];
    te.qd = d[0] * te.gd[0] + d[1] * te.gd[1] + d[2] * te.gd[2];
    te.ap = alpha;
    // largest exponent a factor or partial product reaches
    double big = alpha * te.qd;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double off = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j)
            if (j != k) off += fabs(g[k][j]);
        big = fmax(big, alpha * (6.0 * fabs(te.gd[k]) + 9.0 * g[k][k] + 18.0 * off));
    }
    te.direct = big > 600.0;
    te.q[0] = exp(-2.0 * alpha * g[0][1]);
    te.q[1] = exp(-2.0 * alpha * g[0][2]);
    te.q[2] = exp(-2.0 * alpha * g[1][2]);
    f[0][0] = te.direct ? 0.0 : exp(-alpha * te.qd);
    f[1][0] = 1.0;
    f[2][0] = 1.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double c2 = c[k] * c[k];
        double r = te.direct ? 0.0 : exp(-2.0 * alpha * te.gd[k]) * c[k];
        f[k][1] = f[k][0] * r;
        r *= c2;
        f[k][2] = f[k][1] * r;
        r *= c2;
        f[k][3] = f[k][2] * r;
    }
}

// q^n for n = 0..3
template <typename T>
__device__ __forceinline__ T pow03(T q, int n)
{
    const T q2 = q * q;
    return n == 0 ? T(1) : n == 1 ? q : n == 2 ? q2 : q2 * q;
}

// Transpose-reduction through LDS: lane l holds acc[j], its pair images'
// partial density at point p0 + j (j < NP); afterwards the lane that owns
// point p0 + j (lane index = point index) holds the sum over all lanes.
template <int NP, typename T>
__device__ __forceinline__ void reduce_points(const T *acc, double (*red)[65], int p0, double &out)
{
    constexpr int CH = NP < 32 ? NP : 32;   // points per LDS chunk
    const int lane = threadIdx.x & 63;
    const int j = lane % CH, part = lane / CH;
#pragma unroll
    for (int c0 = 0; c0 < NP; c0 += CH) {
#pragma unroll
        for (int jj = 0; jj < CH; ++jj) red[jj][lane] = (double)acc[c0 + jj];
        __syncthreads();
        double s = 0.0;
#pragma unroll 8
        for (int m = 0; m < CH; ++m) s += red[j][part * CH + m];
#pragma unroll
        for (int o = CH; o < 64; o <<= 1) s += __shfl_xor(s, o, 64);
        if (lane == p0 + c0 + j) out = s;
        __syncthreads();
    }
}

// A - B' of a pair image in Cartesian units: a general cell's records hold it
// in index units (s = r Hinv), so r = s H.
__device__ __forceinline__ void cart_ab(const PairRec &r, const TriGeom *tg, double *AB)
{
    if (tg) {
#pragma unroll
        for (int c = 0; c < 3; ++c) AB[c] = r.AB[0] * tg->H[0][c] + r.AB[1] * tg->H[1][c] + r.AB[2] * tg->H[2][c];
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) AB[c] = r.AB[c];
    }
}

// Elements per packed per-pair coefficient set of nc values, padded to a
// multiple of 16 bytes (the rho kernel copies them in 16-byte pieces).
template <typename T>
__host__ __device__ constexpr int cstride(int nc)
{
    return (nc * (int)sizeof(T) + 15) / 16 * 16 / (int)sizeof(T);
}


// Kw-scaled, symmetrised D sub-blocks of every pair image of one (level,
// class) group, packed per pair image (n_a n_b values each, padded to 16
// bytes), for the classes evaluated directly.
template <typename T, int NA, int NB>
__global__ void __launch_bounds__(256)
k_pack_direct(SegTable<PackSeg> tab)
{
    const PackSeg &sg = tab.s[seg_of(tab, blockIdx.x)];
    const long long e = (long long)(blockIdx.x - sg.item0) * 256 + threadIdx.x;
    if (e >= sg.count) return;
    const double *__restrict__ D = sg.D;
    const int n = sg.n;
    T *__restrict__ out = (T *)sg.out;
    const long long lp = e / (NA * NB);
    const int ij = (int)(e % (NA * NB));
    const int i = ij / NB, j = ij % NB;
    const PairRec &r = sg.pairs[lp];
    const long long a = r.ao_a + i, b = r.ao_b + j;
    out[lp * cstride<T>(NA * NB) + ij] = (T)(r.Kw * 0.5 * (D[a * n + b] + D[b * n + a]));
}

// One (i, j) element's share of a pair image's density coefficient tensor:
// d_ij (x-A)^a (x-B)^b with (x - B_x)^b_x = sum_k binom(b_x, k) (x - A_x)^k
// (A_x - B_x)^(b_x - k) per axis (Eq. (binomial)).
template <int LA, int LB, int I, int J>
__device__ __forceinline__ void pack_term(double *C, double dij, const double (*ab)[LB + 1])
{
    constexpr int L = LA + LB;
    constexpr int ax = cart_lx(LA, I), ay = cart_ly(LA, I), az = LA - ax - ay;
    constexpr int bx = cart_lx(LB, J), by = cart_ly(LB, J), bz = LB - bx - by;
#pragma unroll
    for (int kx = 0; kx <= bx; ++kx)
#pragma unroll
        for (int ky = 0; ky <= by; ++ky)
#pragma unroll
            for (int kz = 0; kz <= bz; ++kz) {
                const double w = (double)(binom(bx, kx) * binom(by, ky) * binom(bz, kz)) * ab[0][bx - kx] *
                                 ab[1][by - ky] * ab[2][bz - kz];
                C[tidx(L, ax + kx, ay + ky, az + kz)] += w * dij;
            }
}
template <int LA, int LB, int... E>
__device__ __forceinline__ void pack_terms(std::integer_sequence<int, E...>, double *C, const double *D, long long n,
                                           long long a0, long long b0, double h, const double (*ab)[LB + 1])
{
    constexpr int NB = ncart_c(LB);
    ((pack_term<LA, LB, E / NB, E % NB>(
         C, h * (D[(a0 + E / NB) * n + b0 + E % NB] + D[(b0 + E % NB) * n + a0 + E / NB]), ab)),
     ...);
}

// Density coefficient tensors of every pair image of one (level, class)
// group, one thread per pair image (Eqs. (binomial), (rho1)): the Kw-scaled
// symmetrised D sub-block contracted with the binomial expansion of the B
// factors around A, in FP64, packed per pair image.
template <typename T, int LA, int LB>
__global__ void __launch_bounds__(256)
k_pack_density(SegTable<PackSeg> tab)
{
    constexpr int NA = ncart_c(LA), NB = ncart_c(LB), L = LA + LB, K = ntab(L);
    const PackSeg &sg = tab.s[seg_of(tab, blockIdx.x)];
    const long long lp = (long long)(blockIdx.x - sg.item0) * 256 + threadIdx.x;
    if (lp >= sg.count) return;
    const PairRec &r = sg.pairs[lp];
    double AB[3];
    cart_ab(r, sg.tri, AB);
    double ab[3][LB + 1];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ab[d][0] = 1.0;
#pragma unroll
        for (int k = 1; k <= LB; ++k) ab[d][k] = ab[d][k - 1] * AB[d];
    }
    double C[K];
#pragma unroll
    for (int k = 0; k < K; ++k) C[k] = 0.0;
    pack_terms<LA, LB>(std::make_integer_sequence<int, NA * NB>{}, C, sg.D, sg.n, r.ao_a, r.ao_b, 0.5 * r.Kw, ab);
    if (sg.tri) {
        double *__restrict__ o = sg.tmp + lp * K;
#pragma unroll
        for (int k = 0; k < K; ++k) o[k] = C[k];
    } else {
        T *__restrict__ out = (T *)sg.out + lp * cstride<T>(K);
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] = (T)C[k];
    }
}

// ------------------------------------------------- kinetic energy density terms
//
// With a_i = (r-A)^a e^{-alpha |r-A|^2} and b_j likewise on B' = B + T, the
// gradient of a factor along axis d is d_d a_i = a_d (r-A)^(a - e_d) e -
// 2 alpha (r-A)^(a + e_d) e, so grad a_i . grad b_j is a polynomial of degree
// l_a + l_b + 2 times the pair envelope: the same separable structure as the
// density, two degrees higher (Sec. II, the meta-GGA terms; Sec. III.B).

// Adds s (r-A)^(AX,AY,AZ) (r-B)^(BX,BY,BZ), with (x - B_x)^b expanded around A
// (Eq. (binomial)), to the coefficient tensor C of degree LT; ab[d][p] =
// (A_d - B_d)^p.
template <int LT, int NP, int AX, int AY, int AZ, int BX, int BY, int BZ>
__device__ __forceinline__ void add_product(double *C, double s, const double (*ab)[NP])
{
#pragma unroll
    for (int kx = 0; kx <= BX; ++kx)
#pragma unroll
        for (int ky = 0; ky <= BY; ++ky)
#pragma unroll
            for (int kz = 0; kz <= BZ; ++kz)
                C[tidx(LT, AX + kx, AY + ky, AZ + kz)] += s * (double)(binom(BX, kx) * binom(BY, ky) * binom(BZ, kz)) *
                                                          ab[0][BX - kx] * ab[1][BY - ky] * ab[2][BZ - kz];
}

// d_D a_i d_D b_j of element (I, J) as four products of shifted monomials.
template <int LA, int LB, int I, int J, int D>
__device__ __forceinline__ void tau_dir(double *C, double dij, double two_a, double two_b, const double (*ab)[LB + 2])
{
    constexpr int LT = LA + LB + 2;
    constexpr int ax = cart_lx(LA, I), ay = cart_ly(LA, I), az = LA - ax - ay;
    constexpr int bx = cart_lx(LB, J), by = cart_ly(LB, J), bz = LB - bx - by;
    constexpr int ex = D == 0, ey = D == 1, ez = D == 2;
    constexpr int ad = D == 0 ? ax : D == 1 ? ay : az;
    constexpr int bd = D == 0 ? bx : D == 1 ? by : bz;
    if constexpr (ad > 0 && bd > 0)
        add_product<LT, LB + 2, ax - ex, ay - ey, az - ez, bx - ex, by - ey, bz - ez>(C, dij * (ad * bd), ab);
    if constexpr (ad > 0)
        add_product<LT, LB + 2, ax - ex, ay - ey, az - ez, bx + ex, by + ey, bz + ez>(C, -dij * ad * two_b, ab);
    if constexpr (bd > 0)
        add_product<LT, LB + 2, ax + ex, ay + ey, az + ez, bx - ex, by - ey, bz - ez>(C, -dij * bd * two_a, ab);
    add_product<LT, LB + 2, ax + ex, ay + ey, az + ez, bx + ex, by + ey, bz + ez>(C, dij * two_a * two_b, ab);
}
template <int LA, int LB, int I, int J>
__device__ __forceinline__ void tau_elem(double *C, double dij, double two_a, double two_b, const double (*ab)[LB + 2])
{
    tau_dir<LA, LB, I, J, 0>(C, dij, two_a, two_b, ab);
    tau_dir<LA, LB, I, J, 1>(C, dij, two_a, two_b, ab);
    tau_dir<LA, LB, I, J, 2>(C, dij, two_a, two_b, ab);
}
template <int LA, int LB, int... E>
__device__ __forceinline__ void tau_terms(std::integer_sequence<int, E...>, double *C, const double *D, long long n,
                                          long long a0, long long b0, double h, double two_a, double two_b,
                                          const double (*ab)[LB + 2])
{
    constexpr int NB = ncart_c(LB);
    ((tau_elem<LA, LB, E / NB, E % NB>(
         C, h * (D[(a0 + E / NB) * n + b0 + E % NB] + D[(b0 + E % NB) * n + a0 + E / NB]), two_a, two_b, ab)),
     ...);
}

// Kinetic-energy-density coefficient tensors of every pair image of one
// (level, class) group, one thread per pair image: 1/2 Kw times the
// symmetrised D sub-block contracted with grad a_i . grad b_j written as a
// polynomial in r - A of degree l_a + l_b + 2 (FP64), packed per pair image.
template <typename T, int LA, int LB>
__global__ void __launch_bounds__(256)
k_pack_tau(SegTable<PackSeg> tab)
{
    constexpr int NA = ncart_c(LA), NB = ncart_c(LB), LT = LA + LB + 2, K = ntab(LT);
    const PackSeg &sg = tab.s[seg_of(tab, blockIdx.x)];
    const long long lp = (long long)(blockIdx.x - sg.item0) * 256 + threadIdx.x;
    if (lp >= sg.count) return;
    const PairRec &r = sg.pairs[lp];
    double AB[3];
    cart_ab(r, sg.tri, AB);
    double ab[3][LB + 2];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ab[d][0] = 1.0;
#pragma unroll
        for (int k = 1; k <= LB + 1; ++k) ab[d][k] = ab[d][k - 1] * AB[d];
    }
    double C[K];
#pragma unroll
    for (int k = 0; k < K; ++k) C[k] = 0.0;
    // 1/2 of tau times the 1/2 of the symmetrisation
    tau_terms<LA, LB>(std::make_integer_sequence<int, NA * NB>{}, C, sg.D, sg.n, r.ao_a, r.ao_b, 0.25 * r.Kw,
                      2.0 * r.aa, 2.0 * r.ab, ab);
    if (sg.tri) {
        double *__restrict__ o = sg.tmp + lp * K;
#pragma unroll
        for (int k = 0; k < K; ++k) o[k] = C[k];
    } else {
        T *__restrict__ out = (T *)sg.out + lp * cstride<T>(K);
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] = (T)C[k];
    }
}

// (lx, ly, lz) of entry k of the lx-major tensor layout of degree <= L
// (inverse of tidx)
__device__ __forceinline__ void tidx_decode(int L, int k, int &lx, int &ly, int &lz)
{
    lx = 0;
    while (k >= ntab2(L - lx)) {
        k -= ntab2(L - lx);
        ++lx;
    }
    ly = t2_ly(L - lx, k);
    lz = t2_lz(L - lx, k);
}

// A general cell's coefficient tensors on the monomials of the index offset:
// with (r - A)^m = sum_k T_n[m][k] (s - s_A)^k over the monomials of one
// degree n, a polynomial sum_m C_m (r - A)^m has the coefficients
// C'_k = sum_m C_m T_n[m][k].  One thread per (pair image, coefficient).
template <typename T>
__global__ void __launch_bounds__(256)
k_to_index(SegTable<IdxSeg> tab)
{
    const IdxSeg &sg = tab.s[seg_of(tab, blockIdx.x)];
    const long long e = (long long)(blockIdx.x - sg.item0) * 256 + threadIdx.x;
    if (e >= sg.count) return;
    const int K = sg.K, L = sg.L;
    const long long lp = e / K;
    const int k = (int)(e - lp * K);
    int kx, ky, kz;
    tidx_decode(L, k, kx, ky, kz);
    const int n = kx + ky + kz, nc = ncart(n), ks = cart_index(ky, kz);
    const double *__restrict__ Tn = sg.tri->T + sg.tri->toff[n];
    const double *__restrict__ src = sg.src + lp * K;
    double v = 0.0;
    for (int m = 0; m < nc; ++m) {
        const int mx = cart_lx(n, m), my = cart_ly(n, m);
        v += src[tidx(L, mx, my, n - mx - my)] * Tn[m * nc + ks];
    }
    ((T *)sg.dst)[lp * sg.cs + k] = (T)v;
}

// Per-lane state of one pair image in the rho kernel.  The record and the D
// sub-block of the next batch are copied from global memory straight into
// LDS (16-byte direct-to-LDS loads, one instruction per 16-byte piece for
// the whole wave, piece c of lane l at c * 1024 + l * 16), so the copy needs
// no registers while the current batch is computed.
template <typename T, int K>
struct RhoLane {
    static constexpr int DB = cstride<T>(K) * (int)sizeof(T);         // bytes of a coefficient set
    static constexpr int NCH = 8 + DB / 16;                          // 16-byte pieces per lane
    static constexpr int STAGE = NCH * 1024;                         // LDS bytes of a batch
    double A[3], AB[3], P[3], c[3];
    double ap, ER;
    T Ct[K];
    static __device__ __forceinline__ void stage(const RhoRec *__restrict__ rr, const T *__restrict__ Dpk, int lp,
                                                 unsigned char *lds)
    {
        const unsigned char *gr = reinterpret_cast<const unsigned char *>(rr + lp);
        const unsigned char *gd = reinterpret_cast<const unsigned char *>(Dpk + (long long)lp * cstride<T>(K));
#pragma unroll
        for (int k = 0; k < 8; ++k)
            __builtin_amdgcn_global_load_lds((const void *)(gr + 16 * k),
                                             (__attribute__((address_space(3))) void *)(lds + k * 1024), 16, 0, 0);
#pragma unroll
        for (int k = 0; k < DB / 16; ++k)
            __builtin_amdgcn_global_load_lds((const void *)(gd + 16 * k),
                                             (__attribute__((address_space(3))) void *)(lds + (8 + k) * 1024), 16, 0,
                                             0);
    }
    // pieces [k0, k1) only (two waves that share a batch each copy a part)
    static __device__ __forceinline__ void stage_part(const RhoRec *__restrict__ rr, const T *__restrict__ Dpk,
                                                      int lp, unsigned char *lds, int k0, int k1)
    {
        const unsigned char *gr = reinterpret_cast<const unsigned char *>(rr + lp);
        const unsigned char *gd = reinterpret_cast<const unsigned char *>(Dpk + (long long)lp * cstride<T>(K));
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            if (k < k0 || k >= k1) continue;
            const unsigned char *g = k < 8 ? gr + 16 * k : gd + 16 * (k - 8);
            __builtin_amdgcn_global_load_lds((const void *)g, (__attribute__((address_space(3))) void *)(lds + k * 1024),
                                             16, 0, 0);
        }
    }
    // the same state straight from global memory (classes that do not stage)
    __device__ __forceinline__ void load_global(const RhoRec *__restrict__ rr, const T *__restrict__ Dpk, int lp)
    {
        const RhoRec &r = rr[lp];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            A[d] = r.A[d];
            AB[d] = r.AB[d];
            P[d] = r.P[d];
            c[d] = r.c[d];
        }
        ap = r.ap;
        ER = r.ER;
        const T *src = Dpk + (long long)lp * cstride<T>(K);
#pragma unroll
        for (int k = 0; k < K; ++k) Ct[k] = src[k];
    }
    __device__ __forceinline__ void load(const unsigned char *lds, int lane)
    {
        double r[16];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const double2 v = *reinterpret_cast<const double2 *>(lds + k * 1024 + lane * 16);
            r[2 * k] = v.x;
            r[2 * k + 1] = v.y;
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            A[d] = r[d];          // RhoRec: A[3] AB[3] P[3] ap Kw ER c[3] pad
            AB[d] = r[3 + d];
            P[d] = r[6 + d];
            c[d] = r[12 + d];
        }
        ap = r[9];
        ER = r[11];
        constexpr int PER = 16 / (int)sizeof(T);
#pragma unroll
        for (int k = 0; k < K; ++k)
            Ct[k] = *reinterpret_cast<const T *>(lds + (8 + k / PER) * 1024 + lane * 16 + (k % PER) * sizeof(T));
    }
};

// Horner's rule in x for the (y, z) coefficient (LY, LZ) of the tensor:
// sum_lx Ct[tidx(L, lx, LY, LZ)] xa^lx; over all (ly, lz) into cyz (fold
// expressions: every index is a compile-time constant at any degree).
template <int L, int LY, int LZ, typename T, int... I>
__device__ __forceinline__ T horner_x(const T *Ct, T xa, std::integer_sequence<int, I...>)
{
    constexpr int top = L - LY - LZ;
    T v = Ct[tidx(L, top, LY, LZ)];
    ((v = v * xa + Ct[tidx(L, top - 1 - I, LY, LZ)]), ...);
    return v;
}
template <int L, typename T, int... K>
__device__ __forceinline__ void horner_x_all(const T *Ct, T xa, T *cyz, std::integer_sequence<int, K...>)
{
    ((cyz[K] = horner_x<L, t2_ly(L, K), t2_lz(L, K), T>(
          Ct, xa, std::make_integer_sequence<int, L - t2_ly(L, K) - t2_lz(L, K)>{})),
     ...);
}
// Horner's rule in y for the z coefficient LZ: sum_ly cyz[t2idx(L, ly, LZ)] ya^ly.
template <int L, int LZ, typename T, int... I>
__device__ __forceinline__ T horner_y(const T *cyz, T ya, std::integer_sequence<int, I...>)
{
    constexpr int top = L - LZ;
    T v = cyz[t2idx(L, top, LZ)];
    ((v = v * ya + cyz[t2idx(L, top - 1 - I, LZ)]), ...);
    return v;
}
template <int L, typename T, int... Z>
__device__ __forceinline__ void horner_y_all(const T *cyz, T ya, T *cz, std::integer_sequence<int, Z...>)
{
    ((cz[Z] = horner_y<L, Z, T>(cyz, ya, std::make_integer_sequence<int, L - Z>{})), ...);
}

// f where keep holds, else a value of magnitude below 2^-1022 (FP64: the
// high word cleared, one select instead of two; FP32: 0).  Accumulated over
// at most the points of a pair image or a block list, such values stay below 1e-300.
__device__ __forceinline__ double keep_if(double f, bool keep)
{
    const long long b = __double_as_longlong(f);
    const int hi = keep ? (int)(b >> 32) : 0;
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)(b & 0xffffffffLL));
}
__device__ __forceinline__ float keep_if(float f, bool keep) { return keep ? f : 0.0f; }

// 1 / x from the hardware reciprocal and Newton steps r' = r + r (1 - x r)
// (two in FP64, one in FP32): a few ulps, in place of a full division.  x = 0
// gives NaN, which compares false.
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    return fma(fma(-x, r, 1.0), r, r);
}
__device__ __forceinline__ float recip(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(fmaf(-x, r, 1.0f), r, r);
}

// Density contributions of one lane's pair image to NX x-slices (x points
// tx0 .. tx0 + NX - 1) of a block: rho(r) += E(r) sum_k Ct_k (r-A)^k with
// the envelope E = fx fy fz cut at ER.  The polynomial is evaluated by
// Horner's rule one axis at a time: per x point its coefficients in (y, z),
// per (x, y) column those in z, per point the z polynomial (Eq. (rho1)).
// TRI (a general cell): coordinates and monomials in index units, and the
// cross factors of block_envelope_tri enter the envelope,
// E = fx[tx] fy[ty] Qxy^(tx ty) fz[tz] (Qxz^tx Qyz^ty)^tz, formed in FP64
// (single factors may exceed the float range; the partial products from fx
// on are envelope values, at most 1), or per point from d^T g d, g d and g
// for a lane in the direct form.
template <int L, int NX, typename T, bool TRI = false>
__device__ __forceinline__ void rho_points(const T *Ct, double xa0, double ya0, double za0, const LevelGeom &G,
                                           const double *fx, const double *fy, const double *fz, T ER, T on,
                                           int tx0, T *acc, const TriEnv *te = nullptr)
{
    T zat[4], fzt[4];   // z offsets and factors, the same for every column
#pragma unroll
    for (int tz = 0; tz < 4; ++tz) {
        zat[tz] = (T)(za0 + tz * G.h[2]);
        fzt[tz] = (T)fz[tz];
    }
#pragma unroll
    for (int ix = 0; ix < NX; ++ix) {
        const T xa = (T)(xa0 + (tx0 + ix) * G.h[0]);
        const T ex = (T)fx[ix] * on;
        T cyz[ntab2(L)];
        horner_x_all<L, T>(Ct, xa, cyz, std::make_integer_sequence<int, ntab2(L)>{});
        double qxy = 1.0, qxz = 1.0;   // Qxy^tx, Qxz^tx
        if constexpr (TRI) {
            qxy = pow03<double>(te->q[0], tx0 + ix);
            qxz = pow03<double>(te->q[1], tx0 + ix);
        }
#pragma unroll
        for (int ty = 0; ty < 4; ++ty) {
            const T ya = (T)(ya0 + ty * G.h[1]);
            T cz[L + 1];
            horner_y_all<L, T>(cyz, ya, cz, std::make_integer_sequence<int, L + 1>{});
            // the four points of the column side by side: independent chains
            T E[4], q[4];
            if constexpr (TRI) {
                if (!te->direct) {
                    const double exy = fx[ix] * fy[ty] * pow03<double>(qxy, ty);
                    const double m = qxz * pow03<double>(te->q[2], ty), m2 = m * m;
                    E[0] = (T)(exy * fz[0]) * on;
                    E[1] = (T)(exy * (fz[1] * m)) * on;
                    E[2] = (T)(exy * (fz[2] * m2)) * on;
                    E[3] = (T)(exy * (fz[3] * (m2 * m))) * on;
                } else {
                    // (d + t)^T g (d + t) = d^T g d + 2 t . g d + t^T g t
                    const double(*g)[3] = G.tri->g;
                    const double tx = tx0 + ix, tyd = ty;
                    const double qxy2 = te->qd + 2.0 * (tx * te->gd[0] + tyd * te->gd[1]) + g[0][0] * tx * tx +
                                        g[1][1] * tyd * tyd + 2.0 * g[0][1] * tx * tyd;
                    const double lz = 2.0 * (te->gd[2] + g[0][2] * tx + g[1][2] * tyd);
#pragma unroll
                    for (int tz = 0; tz < 4; ++tz)
                        E[tz] = (T)exp(-te->ap * (qxy2 + tz * (lz + g[2][2] * tz))) * on;
                }
            } else {
                const T exy = ex * (T)fy[ty];
#pragma unroll
                for (int tz = 0; tz < 4; ++tz) E[tz] = exy * fzt[tz];
            }
#pragma unroll
            for (int tz = 0; tz < 4; ++tz) q[tz] = cz[L];
#pragma unroll
            for (int lz = L - 1; lz >= 0; --lz)
#pragma unroll
                for (int tz = 0; tz < 4; ++tz) q[tz] = q[tz] * zat[tz] + cz[lz];
#pragma unroll
            for (int tz = 0; tz < 4; ++tz) acc[ix * 16 + ty * 4 + tz] += keep_if(E[tz], E[tz] >= ER) * q[tz];
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// The same contributions evaluated directly: rho(r) += E(r) sum_ij D_ij
// a_i(r - A) b_j(r - B), with the Kw-scaled symmetrised D sub-block Dk.
template <int LA, int LB, int NX, typename T>
__device__ __forceinline__ void rho_points_direct(const T *Dk, double xa0, double ya0, double za0, const double *AB,
                                                  const LevelGeom &G, const double *fx, const double *fy,
                                                  const double *fz, T ER, T on, int tx0, T *acc)
{
    constexpr int NA = ncart_c(LA), NB = ncart_c(LB);
    const T abx = (T)AB[0], aby = (T)AB[1], abz = (T)AB[2];
#pragma unroll
    for (int ix = 0; ix < NX; ++ix) {
        const T xa = (T)(xa0 + (tx0 + ix) * G.h[0]);
        const T xb = xa + abx;
        const T ex = (T)fx[ix] * on;
#pragma unroll
        for (int ty = 0; ty < 4; ++ty) {
            const T ya = (T)(ya0 + ty * G.h[1]);
            const T yb = ya + aby;
            const T exy = ex * (T)fy[ty];
#pragma unroll
            for (int tz = 0; tz < 4; ++tz) {
                const T za = (T)(za0 + tz * G.h[2]);
                const T zb = za + abz;
                T E = exy * (T)fz[tz];
                E = keep_if(E, E >= ER);
                T a[NA], bb[NB];
                monomials<LA, T>(xa, ya, za, a);
                monomials<LB, T>(xb, yb, zb, bb);
                T sum = T(0);
#pragma unroll
                for (int i = 0; i < NA; ++i) {
                    T t = T(0);
#pragma unroll
                    for (int jb = 0; jb < NB; ++jb) t += Dk[i * NB + jb] * bb[jb];
                    sum += a[i] * t;
                }
                acc[ix * 16 + ty * 4 + tz] += E * sum;
            }
            // bounds the live monomials of the widest classes; the others
            // schedule better across columns
            if constexpr (LA + LB >= 5) __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// One lane's contributions, in the form the class uses.  XL = 2: the
// kinetic energy density, always through its coefficient tensor of degree
// l_a + l_b + 2.  A general cell (TRI) always takes the tensor form, whose
// monomials are those of the index offset.
template <int LA, int LB, int XL, int NX, typename T, bool TRI = false>
__device__ __forceinline__ void rho_lane_points(const T *C, double xa0, double ya0, double za0, const double *AB,
                                                const LevelGeom &G, const double *fx, const double *fy,
                                                const double *fz, T ER, T on, int tx0, T *acc,
                                                const TriEnv *te = nullptr)
{
    if constexpr (TRI || XL > 0 || rho_tensor(LA, LB))
        rho_points<LA + LB + XL, NX, T, TRI>(C, xa0, ya0, za0, G, fx, fy, fz, ER, on, tx0, acc, te);
    else
        rho_points_direct<LA, LB, NX, T>(C, xa0, ya0, za0, AB, G, fx, fy, fz, ER, on, tx0, acc);
}

// Coefficients per pair image in the packed rho / tau inputs.
__host__ __device__ constexpr int grid_ncoef(int la, int lb, int xl, bool tri = false)
{
    return (xl > 0 || tri) ? ntab(la + lb + xl) : rho_ncoef(la, lb);
}

// Density of one (level, class) group on its nonempty 4x4x4 blocks.  One wave
// per block; lane = pair image of the block's list (batches of 64), as in
// Alg. 1.  Each lane holds its image's geometry and Kw-scaled D sub-block in
// registers and accumulates its contributions to the block's points over the
// whole list; one LDS transpose-reduction per block sums the lanes (instead of
// a block reduction per point).  The loads of the next batch (list entries two
// batches ahead; geometry and D one batch ahead, straight into LDS) are issued
// before the current batch is computed, so their latency hides behind the
// arithmetic.  NPASS splits the 64 points to bound the accumulator registers.
// XL = 0: density; XL = 2: kinetic energy density (its coefficient tensor).
template <int LA, int LB, int XL, int NPASS, bool STG, bool PREF, typename T, bool TRI = false>
__device__ __forceinline__ void rho_blocks(const SegTable<RhoSeg> &tab)
{
    constexpr int NX = 4 / NPASS;
    constexpr int NP = 16 * NX;
    using Lane = RhoLane<T, grid_ncoef(LA, LB, XL, TRI)>;
    constexpr int LDSB = STG && Lane::STAGE > 32 * 65 * 8 ? Lane::STAGE : 32 * 65 * 8;
    // the batch staging area, and after the last batch the reduction buffer
    __shared__ __attribute__((aligned(16))) unsigned char lds[LDSB];
    double(*red)[65] = reinterpret_cast<double(*)[65]>(lds);
    const int lane = threadIdx.x;
    const RhoSeg &sg = tab.s[seg_of(tab, blockIdx.x)];
    const long long item = xcd_ranged(blockIdx.x - sg.item0, sg.xs);
    if (item < 0) return;
    const LevelGeom &G = sg.G;
    const int2 *__restrict__ inc = sg.inc;
    const T *__restrict__ Dpk = (const T *)sg.Dpk;
    const int p0 = sg.p0;
    const int b = sg.blk[item];   // block slot
    int kx, ky, kz;
    slot_block(G, b, kx, ky, kz);
    const int kk[3] = {kx, ky, kz};
    const long long s0 = sg.inc_off[b], s1 = sg.inc_off[b + 1];
    const RhoRec *rr = sg.rr;
    double mine = 0.0;
#pragma unroll 1
    for (int pass = 0; pass < NPASS; ++pass) {
        T acc[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) acc[i] = T(0);
        // list entries two batches ahead, record and D one batch ahead (in LDS)
        // (classes without staging: entries one batch ahead, record and D at
        // the start of each batch)
        int2 en1 = inc[s0 + lane < s1 ? s0 + lane : s1 - 1];
        int2 en2 = inc[s0 + 64 + lane < s1 ? s0 + 64 + lane : s1 - 1];
        Lane nxt;   // PREF: the next batch's state, loaded while this one is computed
        if constexpr (STG) {
            asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
            Lane::stage(rr, Dpk, en1.x - p0, lds);
        } else if constexpr (PREF) {
            nxt.load_global(rr, Dpk, en1.x - p0);
        }
        for (long long s = s0; s < s1; s += 64) {
            const bool act = s + lane < s1;
            const int2 en = en1;
            Lane cur;
            if constexpr (STG) {
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this batch's pieces are in LDS
                cur.load(lds, lane);
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); // read before the area is refilled
                if (s + 64 < s1) Lane::stage(rr, Dpk, en2.x - p0, lds);
            } else if constexpr (PREF) {
                cur = nxt;
                if (s + 64 < s1) nxt.load_global(rr, Dpk, en2.x - p0);
            } else {
                cur.load_global(rr, Dpk, en.x - p0);
            }
            en1 = en2;
            {
                const long long q2 = s + 128 + lane;
                en2 = inc[q2 < s1 ? q2 : s1 - 1];
            }
            double fx[4], fy[4], fz[4];
            const double x0 = (double)(4 * kk[0] + shift_of(en.y, 0) * G.N[0]) * G.h[0];
            const double y0 = (double)(4 * kk[1] + shift_of(en.y, 1) * G.N[1]) * G.h[1];
            const double z0 = (double)(4 * kk[2] + shift_of(en.y, 2) * G.N[2]) * G.h[2];
            const double dP[3] = {x0 - cur.P[0], y0 - cur.P[1], z0 - cur.P[2]};
            TriEnv te;
            if constexpr (TRI)
                block_envelope_tri(cur.ap, dP, G.tri, cur.c, fx, fy, fz, te);
            else
                block_envelope(cur.ap, dP, G, cur.c, fx, fy, fz);
            const T ER = (T)cur.ER;
            const T on = act ? T(1) : T(0);
            const double xa0 = x0 - cur.A[0], ya0 = y0 - cur.A[1], za0 = z0 - cur.A[2];
            double fxp[NX];   // this pass's x factors
#pragma unroll
            for (int ix = 0; ix < NX; ++ix) {
                fxp[ix] = fx[ix];
#pragma unroll
                for (int q = 1; q < NPASS; ++q)
                    if (pass == q) fxp[ix] = fx[q * NX + ix];
            }
            rho_lane_points<LA, LB, XL, NX, T, TRI>(cur.Ct, xa0, ya0, za0, cur.AB, G, fxp, fy, fz, ER, on,
                                                    pass * NX, acc, &te);
        }
        reduce_points<NP, T>(acc, red, pass * NP, mine);
    }
    const int tx = lane >> 4, ty = (lane >> 2) & 3, tz = lane & 3;
    const int wx = 4 * kx + tx, wy = 4 * ky + ty, wz = 4 * kz + tz;
    if (wx < G.N[0] && wy < G.N[1] && wz < G.N[2]) {
        const long long o = ((long long)wx * G.N[1] + wy) * G.N[2] + wz;
        sg.rho[o] += mine;
    }
}

template <int LA, int LB, int NPASS, int WPE, bool STG, bool PREF, typename T>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
k_rho(SegTable<RhoSeg> tab)
{
    rho_blocks<LA, LB, 0, NPASS, STG, PREF, T>(tab);
}

// The density and the kinetic energy density of a general cell: index
// coordinates, the cross factors of block_envelope_tri, coefficients in the
// monomials of the index offset (k_to_index).  No staging; NPASS bounds the
// accumulators next to the cross factors.
template <int LA, int LB, int NPASS, typename T>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_rho_tri(SegTable<RhoSeg> tab)
{
    rho_blocks<LA, LB, 0, NPASS, false, false, T, true>(tab);
}
template <int LA, int LB, int NPASS, typename T>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_tau_tri(SegTable<RhoSeg> tab)
{
    rho_blocks<LA, LB, 2, NPASS, false, false, T, true>(tab);
}

// Kinetic energy density tau(r) = 1/2 sum D grad a . grad b (Sec. II, the
// meta-GGA term; Sec. III.B, Alg. 1 with the pair function replaced by the
// product of gradients): the density kernel with each pair image's
// coefficient tensor of degree l_a + l_b + 2 (k_pack_tau), loaded per batch.
template <int LA, int LB, int NPASS, int WPE, typename T>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
k_tau(SegTable<RhoSeg> tab)
{
    rho_blocks<LA, LB, 2, NPASS, false, false, T>(tab);
}

// The same density for the heavy classes with two waves per block: both
// waves walk the block's list with the same lane = pair image mapping and
// share one copy of every batch in LDS (double-buffered, each wave copying
// half of the pieces), and each wave accumulates 32 of the 64 points, which
// halves the accumulator registers so that two such workgroups fit a SIMD.
template <int LA, int LB, int WPE, typename T>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
k_rho2(SegTable<RhoSeg> tab)
{
    using Lane = RhoLane<T, grid_ncoef(LA, LB, 0)>;
    constexpr int SB = Lane::STAGE;
    constexpr int REDB = 2 * 32 * 65 * 8;
    constexpr int LDSB = 2 * SB > REDB ? 2 * SB : REDB;
    // two staging buffers, and after the last batch one reduction buffer per wave
    __shared__ __attribute__((aligned(16))) unsigned char lds[LDSB];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const RhoSeg &sg = tab.s[seg_of(tab, blockIdx.x)];
    const long long item = xcd_ranged(blockIdx.x - sg.item0, sg.xs);
    if (item < 0) return;
    const LevelGeom &G = sg.G;
    const int2 *__restrict__ inc = sg.inc;
    const T *__restrict__ Dpk = (const T *)sg.Dpk;
    const int p0 = sg.p0;
    const int b = sg.blk[item];   // block slot
    int kx, ky, kz;
    slot_block(G, b, kx, ky, kz);
    const int kk[3] = {kx, ky, kz};
    const long long s0 = sg.inc_off[b], s1 = sg.inc_off[b + 1];
    const RhoRec *rr = sg.rr;
    const int kh = (Lane::NCH + 1) / 2;                 // pieces copied by wave 0
    const int k0 = w ? kh : 0, k1 = w ? Lane::NCH : kh;
    T acc[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) acc[i] = T(0);
    int2 en1 = inc[s0 + lane < s1 ? s0 + lane : s1 - 1];
    int2 en2 = inc[s0 + 64 + lane < s1 ? s0 + 64 + lane : s1 - 1];
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    Lane::stage_part(rr, Dpk, en1.x - p0, lds, k0, k1);
    int buf = 0;
    for (long long s = s0; s < s1; s += 64) {
        const bool act = s + lane < s1;
        const int2 en = en1;
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wave's pieces of the batch
        __syncthreads();                                    // and the other wave's; old buffer free
        Lane cur;
        cur.load(lds + buf * SB, lane);
        if (s + 64 < s1) Lane::stage_part(rr, Dpk, en2.x - p0, lds + (buf ^ 1) * SB, k0, k1);
        buf ^= 1;
        en1 = en2;
        {
            const long long q2 = s + 128 + lane;
            en2 = inc[q2 < s1 ? q2 : s1 - 1];
        }
        double fx[4], fy[4], fz[4];
        const double x0 = (double)(4 * kk[0] + shift_of(en.y, 0) * G.N[0]) * G.h[0];
        const double y0 = (double)(4 * kk[1] + shift_of(en.y, 1) * G.N[1]) * G.h[1];
        const double z0 = (double)(4 * kk[2] + shift_of(en.y, 2) * G.N[2]) * G.h[2];
        const double dP[3] = {x0 - cur.P[0], y0 - cur.P[1], z0 - cur.P[2]};
        block_envelope(cur.ap, dP, G, cur.c, fx, fy, fz);
        const T ER = (T)cur.ER;
        const T on = act ? T(1) : T(0);
        const double xa0 = x0 - cur.A[0], ya0 = y0 - cur.A[1], za0 = z0 - cur.A[2];
        const double fxp[2] = {w ? fx[2] : fx[0], w ? fx[3] : fx[1]};
        rho_lane_points<LA, LB, 0, 2, T>(cur.Ct, xa0, ya0, za0, cur.AB, G, fxp, fy, fz, ER, on, 2 * w, acc);
    }
    __syncthreads();   // every read of the staging buffers is done
    double mine = 0.0;
    reduce_points<32, T>(acc, reinterpret_cast<double(*)[65]>(lds + w * (32 * 65 * 8)), 0, mine);
    if (lane < 32) {
        const int p = 32 * w + lane;
        const int tx = p >> 4, ty = (p >> 2) & 3, tz = p & 3;
        const int wx = 4 * kx + tx, wy = 4 * ky + ty, wz = 4 * kz + tz;
        if (wx < G.N[0] && wy < G.N[1] && wz < G.N[2]) {
            const long long o = ((long long)wx * G.N[1] + wy) * G.N[2] + wz;
            sg.rho[o] += mine;
        }
    }
}

// per class: points per pass (NPASS), waves per SIMD, whether the next batch
// is staged in LDS or else (pref) loaded into registers one batch ahead, and
// whether two waves share a block (k_rho2, at WPE2 workgroups per SIMD)
// (chosen by measurement on the 256-water system)
template <int LA, int LB> struct RhoSplit {
    static constexpr int npass = 1, wpe = 2, wpe2 = 1;
    static constexpr bool stage = false, two = false, pref = true;
};
template <> struct RhoSplit<1, 1> {
    static constexpr int npass = 1, wpe = 2, wpe2 = 2;
    static constexpr bool stage = true, two = false, pref = false;
};
template <> struct RhoSplit<2, 0> {
    static constexpr int npass = 1, wpe = 1, wpe2 = 2;
    static constexpr bool stage = true, two = true, pref = false;
};
template <> struct RhoSplit<2, 1> {
    static constexpr int npass = 1, wpe = 1, wpe2 = 2;
    static constexpr bool stage = true, two = false, pref = false;
};
template <> struct RhoSplit<2, 2> {
    static constexpr int npass = 1, wpe = 1, wpe2 = 2;
    static constexpr bool stage = true, two = false, pref = false;
};
template <> struct RhoSplit<3, 0> {
    static constexpr int npass = 1, wpe = 1, wpe2 = 1;
    static constexpr bool stage = false, two = false, pref = false;
};
template <> struct RhoSplit<3, 1> {
    static constexpr int npass = 1, wpe = 1, wpe2 = 1;
    static constexpr bool stage = false, two = false, pref = false;
};
template <> struct RhoSplit<3, 2> {
    static constexpr int npass = 1, wpe = 1, wpe2 = 1;
    static constexpr bool stage = false, two = false, pref = false;
};
template <> struct RhoSplit<3, 3> {
    static constexpr int npass = 4, wpe = 1, wpe2 = 1;
    static constexpr bool stage = false, two = false, pref = false;
};
// g classes: the accumulators share the registers with 15 D values (g|s) or a
// tensor of 56 to 165 values
template <> struct RhoSplit<4, 0> {
    static constexpr int npass = 1, wpe = 1, wpe2 = 1;
    static constexpr bool stage = false, two = false, pref = false;
};
template <> struct RhoSplit<4, 1> {
    static constexpr int npass = 2, wpe = 1, wpe2 = 1;
    static constexpr bool stage = false, two = false, pref = false;
};
template <int LB> struct RhoSplit<4, LB> {
    static constexpr int npass = 4, wpe = 1, wpe2 = 1;
    static constexpr bool stage = false, two = false, pref = false;
};

// Kinetic energy density: points per pass and waves per SIMD by the degree
// LT of the coefficient tensor (its ntab(LT) values and the accumulators
// share the lane's registers).
template <int LT> struct TauSplit {
    static constexpr int npass = LT <= 4 ? 1 : LT == 5 ? 2 : 4;
    static constexpr int wpe = LT <= 3 ? 2 : 1;
};

// ----------------------------------------------- pair-major traversal (mat, grad)

// Per-axis list entry of the blocks a pair image's bounding box meets:
// wrapped block index k and the squared distance from P to the block's
// extent along the axis.
struct AxisBlock {
    int k, pad;
    double gap2;
};

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uni(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// 1-D point tables of a pair image, at point 4 e + t of an axis (point t of
// block list entry e): the envelope factor exp(-alpha_p (x - P)^2) and the
// offset x - A.
template <typename T> struct alignas(2 * sizeof(T)) PtXY { T e, a; };
template <typename T> struct alignas(2 * sizeof(T)) PtZ { T e, a; };
constexpr int kZSlots = 5;   // z table slots per block entry (4 points, 1 unused)

// LDS set-up of one pair image: per axis, the list of the blocks (with fold
// shifts) its bounding box meets, one entry per lane, and the point tables of
// the entries, so that the points of a run of consecutive entries sit at
// consecutive table positions.  emax bounds every list (the plan's longest).
// The z table holds 8 emax points: past the box's 4 nz points, points that no
// sphere contains (envelope factor 0; TRI: an offset of 1e18, whose squared
// metric length exceeds any R^2 and stays finite in FP32), so that a
// traversal may step past the end of a run without a bounds test.  Point i
// sits in slot i + i / 4 (kZSlots slots per block entry, one unused): the
// rows that a traversal reads together start at different entries, and the
// odd stride puts their points in different LDS banks.
// TRI (a general cell, index units): the tables hold the offset from P in
// place of the envelope factor (the envelope does not separate; the visitor
// forms it per point), and the gaps are scaled by the metric's smallest
// eigenvalue so that their sum stays below the squared distance.
template <bool MOM, typename T, bool TRI = false>
__device__ __forceinline__ void pair_setup(const PairRec &r, const LevelGeom &G, PtXY<T> *txy, PtZ<T> *tz,
                                           AxisBlock *bl, int emax, int *cnt)
{
    const double ap = r.aa + r.ab;
    double gs = 1.0;
    if constexpr (TRI) gs = G.tri->lmin;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int N = G.N[d], nb = G.nb[d];
        const int k0 = r.bk0[d], s0 = r.bs0[d], n = r.bn[d];
        // entry e: wrapped block k0 + e folded into [0, nb), shift s0 + folds
        for (int e = threadIdx.x; e < n; e += 64) {
            int k = k0 + e, S = s0;
            while (k >= nb) {
                k -= nb;
                ++S;
            }
            const int u0 = 4 * k + S * N;
            const int u1 = (4 * k + 3 < N - 1 ? 4 * k + 3 : N - 1) + S * N;
            AxisBlock eb;
            eb.k = k;
            eb.pad = 0;
            eb.gap2 = gs * axis_gap2(r.P[d], (double)u0 * G.h[d], (double)u1 * G.h[d]);
            bl[d * emax + e] = eb;
        }
        // points of the entries; a partial block's padding points get the
        // coordinates past the period's end (their potential is zero)
        for (int i = threadIdx.x; i < 4 * n; i += 64) {
            int k = k0 + (i >> 2), S = s0;
            while (k >= nb) {
                k -= nb;
                ++S;
            }
            const int u = 4 * k + (i & 3) + S * N;
            const double x = (double)u * G.h[d];
            const double dx = x - r.P[d];
            const double e = TRI ? dx : exp(-ap * dx * dx), a = x - r.A[d];
            if (d < 2) {
                txy[d * 4 * emax + i] = PtXY<T>{(T)e, (T)a};
            } else {
                tz[i + (i >> 2)] = PtZ<T>{(T)e, (T)a};
            }
        }
    }
    for (int i = 4 * r.bn[2] + threadIdx.x; i < 8 * emax; i += 64)
        tz[i + (i >> 2)] = PtZ<T>{TRI ? T(1e18) : T(0), T(0)};
    if (threadIdx.x == 0) {
        cnt[0] = r.bn[0];
        cnt[1] = r.bn[1];
        cnt[2] = r.bn[2];
        cnt[3] = r.bem;
    }
}


// One (x, y) row of blocks of a pair image whose z run meets the sphere:
// the block-copy index of the run's first block (the run is contiguous
// there), the x and y entries, and the run's first z entry and length.
struct BlockRow {
    int vb;    // block index in the level's block copy
    int ex;    // x entry
    int ey;    // y entry
    int zn;    // zlo | n << 16
};

// Rows of the pair image's blocks with x entries in [ex0, ex1), longest run
// first: built by the wave with one candidate row per lane and a ballot
// compaction into tmp, then placed by a counting sort on the run length
// (hist: emax + 1 counters), so that the rows a traversal takes four at a
// time have runs of about the same length.
__device__ __forceinline__ int build_rows(const double R2c, const LevelGeom &G, int vz, const AxisBlock *bl,
                                          int emax, const int *cnt, BlockRow *rows, BlockRow *tmp, int *hist,
                                          int ex0, int ex1)
{
    const int lane = threadIdx.x;
    const int ny = uni(cnt[1]), nz = uni(cnt[2]), em = uni(cnt[3]);
    const int ncand = (ex1 - ex0) * ny;
    const AxisBlock *blx = bl, *bly = bl + emax, *blz = bl + 2 * emax;
    const float rny = 1.0f / (float)ny;
    int nrows = 0;
    for (int base = 0; base < ncand; base += 64) {
        const int i = base + lane;
        bool ok = false;
        BlockRow row;
        if (i < ncand) {
            // i / ny in single precision: exact while i and ny stay far below 2^20
            const int exr = (int)(((float)i + 0.5f) * rny), ey = i - exr * ny, ex = ex0 + exr;
            const double g = blx[ex].gap2 + bly[ey].gap2;
            if (g <= R2c) {
                const double rem = R2c - g;
                // the z gaps fall on [0, em) and rise on [em, nz): the run of
                // entries with gap <= rem from two binary searches
                int zlo, zhi;
                {
                    int a = 0, b = em;   // first e < em with gap <= rem, else em
                    while (a < b) {
                        const int c = (a + b) >> 1;
                        if (blz[c].gap2 <= rem) b = c; else a = c + 1;
                    }
                    zlo = a;
                }
                {
                    int a = em - 1, b = nz - 1;   // last e >= em with gap <= rem, else em - 1
                    while (a < b) {
                        const int c = (a + b + 1) >> 1;
                        if (blz[c].gap2 <= rem) a = c; else b = c - 1;
                    }
                    zhi = a;
                }
                if (zlo == em && (em >= nz || blz[em].gap2 > rem)) zlo = nz;   // nothing on [em, nz)
                ok = zlo <= zhi;
                if (ok) {
                    row.vb = (blx[ex].k * G.nb[1] + bly[ey].k) * vz + blz[zlo].k;
                    row.ex = ex;
                    row.ey = ey;
                    row.zn = zlo | ((zhi - zlo + 1) << 16);
                }
            }
        }
        const unsigned long long m = __ballot(ok);
        if (ok) tmp[nrows + __popcll(m & ((1ull << lane) - 1))] = row;
        nrows += __popcll(m);
    }
    for (int k = lane; k <= emax; k += 64) hist[k] = 0;
    __syncthreads();
    for (int i = lane; i < nrows; i += 64) atomicAdd(&hist[tmp[i].zn >> 16], 1);
    __syncthreads();
    // first position of each length: the rows of greater length before it
    // (a wave scan over the lengths from emax down, 64 at a time)
    int carry = 0;
    for (int top = emax; top >= 1; top -= 64) {
        const int n = top - lane;
        const int h = n >= 1 ? hist[n] : 0;
        int sc = h;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int t = __shfl_up(sc, d, 64);
            if (lane >= d) sc += t;
        }
        if (n >= 1) hist[n] = carry + sc - h;
        carry += __shfl(sc, 63, 64);
    }
    __syncthreads();
    for (int i = lane; i < nrows; i += 64) {
        const BlockRow w = tmp[i];
        rows[atomicAdd(&hist[w.zn >> 16], 1)] = w;
    }
    return nrows;
}

// Visit every (block, shift) incidence of the pair image whose block meets
// the truncation sphere (the incidences the partitioner lists), four block
// rows at a time: lane = (row slot g of the group, point (tx, ty) of the
// 4x4 cross-section of the row's blocks).  The wave steps along z one point
// plane at a time, through the runs of all four rows together; a row shorter
// than the group's longest (the first, rows being sorted longest first) and
// an empty slot of the last group step on past their end over points that no
// sphere contains (the z table's padding, or points of blocks beyond the run,
// which the sphere cut removes), and an empty slot's lanes are cut by the
// visitor.  The block copy holds each block's points as four z planes of
// 16 (x, y) points, so that a plane of a run is one 128-byte line per row and
// the run is contiguous; reads past a run's end stay inside its column
// (at most emax blocks from a start inside the cell).  The potential of the
// next block's four planes is loaded before the current one is used.
// The visitor sees vis.row(X, Y, ok) at the start of every group (X, Y: the
// lane's x and y table entries; ok: the lane's slot holds a row) and
// vis.point(v, Z) for every point (v the potential, Z the z table entry),
// then vis.done().
template <typename T, typename Vis>
__device__ __forceinline__ void for_each_point(const PtXY<T> *txy, const PtZ<T> *tzt, int emax, const BlockRow *rows,
                                               int nrows, const double *__restrict__ Vb, Vis &vis)
{
    const int lane = threadIdx.x;
    const int g = lane >> 4, col = lane & 15;
    const PtXY<T> *px = txy + (col >> 2), *py = txy + 4 * emax + (col & 3);
    if (nrows <= 0) return;
    // cursor: group (first row q), block b of the runs, the group's longest
    // run; per lane: its row's potential column, z table position and x, y
    // entries
    struct Cur {
        int q, b, nmax;
        const double *vp;
        int zi, ex, ey;
        bool ok;
    };
    auto fetch_group = [&](Cur &c, int q) {
        const int slot = q + g;
        c.q = q;
        c.b = 0;
        c.ok = slot < nrows;
        const BlockRow w = rows[c.ok ? slot : q];
        c.nmax = uni(w.zn >> 16);   // lane 0 holds row q, the group's longest
        c.vp = Vb + (long long)w.vb * 64 + col;
        c.zi = kZSlots * (w.zn & 0xffff);
        c.ex = w.ex;
        c.ey = w.ey;
    };
    auto load4 = [&](const Cur &c, double *v) {
        const double *p = c.vp + (long long)c.b * 64;
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = p[u * 16];
    };
    // advance c to the next block; false at the end (c then stays put)
    auto advance = [&](Cur &c) {
        if (c.b + 1 < c.nmax) {
            c.b += 1;
            return true;
        }
        if (c.q + 4 >= nrows) return false;
        fetch_group(c, c.q + 4);
        return true;
    };
    auto run = [&](const Cur &c, const double *v) {
        if (c.b == 0) vis.row(px[4 * c.ex], py[4 * c.ey], c.ok);
        const PtZ<T> *z = tzt + c.zi + kZSlots * c.b;
#pragma unroll
        for (int u = 0; u < 4; ++u) vis.point((T)v[u], z[u]);
    };
    Cur a;
    fetch_group(a, 0);
    double va[4], vb4[4];
    load4(a, va);
    // two blocks per trip, alternating the two potential buffers
    for (;;) {
        Cur b = a;
        const bool mb = advance(b);
        load4(b, vb4);
        run(a, va);
        if (!mb) break;
        a = b;
        const bool ma = advance(a);
        load4(a, va);
        run(b, vb4);
        if (!ma) break;
    }
    vis.done();
}

// Visitor of the direct form: body(f, xa, ya, za, xb, yb, zb) per point with
// f = v(r) exp(-alpha_p |r-P|^2) inside the sphere, else 0, (xa, ya, za) =
// r - A and (xb, yb, zb) = r - B.
template <typename T, typename Body>
struct DirectVisit {
    Body &body;
    T ER, abx, aby, abz;
    T xa = 0, ya = 0, xb = 0, yb = 0, exy = 0, er = 0;
    __device__ DirectVisit(Body &b, const PairRec &r)
        : body(b), ER((T)r.ER), abx((T)r.AB[0]), aby((T)r.AB[1]), abz((T)r.AB[2])
    {
    }
    // ok = false: a lane without a row, every point cut
    __device__ __forceinline__ void row(const PtXY<T> &X, const PtXY<T> &Y, bool ok)
    {
        xa = X.a;
        ya = Y.a;
        xb = xa + abx;
        yb = ya + aby;
        exy = X.e * Y.e;
        er = ok ? ER : T(__builtin_huge_val());
    }
    __device__ __forceinline__ void point(T v, const PtZ<T> &Z)
    {
        const T E = exy * Z.e;
        body(keep_if(v * E, E >= er), xa, ya, Z.a, xb, yb, Z.a + abz);
    }
    __device__ __forceinline__ void done() {}
};

// Visitor of the separable form (the potential analogue of Eq. (rho1)): the
// moments sum_r v(r) E(r) (x-A_x)^lx (y-A_y)^ly (z-A_z)^lz of total degree
// <= L, accumulated one axis at a time: per point the z moments of the
// lane's current (x, y) column (W), at the end of a group of rows the full
// moments (Vm += W_lz ex ey (x-A_x)^lx (y-A_y)^ly).  E(r) = ex ey ez is
// split the same way; the sphere cut uses the full product.
template <int L, typename T>
struct TensorVisit {
    static constexpr int K = ntab(L);
    T Vm[K], W[L + 1];
    T ER;
    T xa = 0, ya = 0, exy = 0, thr = 0;
    __device__ TensorVisit(const PairRec &r, const LevelGeom &) : TensorVisit(r) {}
    __device__ explicit TensorVisit(const PairRec &r) : ER((T)r.ER)
    {
#pragma unroll
        for (int k = 0; k < K; ++k) Vm[k] = T(0);
#pragma unroll
        for (int k = 0; k <= L; ++k) W[k] = T(0);
    }
    __device__ __forceinline__ void flush()
    {
        T gx = exy;   // ex ey (x-A_x)^lx
#pragma unroll
        for (int lx = 0; lx <= L; ++lx) {
            T g = gx;
#pragma unroll
            for (int ly = 0; lx + ly <= L; ++ly) {
#pragma unroll
                for (int lz = 0; lx + ly + lz <= L; ++lz) Vm[tidx(L, lx, ly, lz)] += W[lz] * g;
                g *= ya;
            }
            gx *= xa;
        }
#pragma unroll
        for (int k = 0; k <= L; ++k) W[k] = T(0);
    }
    // ok = false: a lane without a row, every point cut.  The cut
    // ex ey ez >= E_R is taken as ez >= E_R / (ex ey) (+inf or NaN: none
    // kept).
    __device__ __forceinline__ void row(const PtXY<T> &X, const PtXY<T> &Y, bool ok)
    {
        flush();
        xa = X.a;
        ya = Y.a;
        exy = X.e * Y.e;
        thr = ok ? ER * recip(exy) : T(__builtin_huge_val());
    }
    __device__ __forceinline__ void point(T v, const PtZ<T> &Z)
    {
        const T f = keep_if(v * Z.e, Z.e >= thr);
        W[0] += f;
        if constexpr (L >= 1) {
            T p = f * Z.a;   // f (z - A_z)^(lz - 1) for the next lz
            W[1] += p;
#pragma unroll
            for (int lz = 2; lz <= L; ++lz) {
                W[lz] += p * Z.a;
                if (lz < L) p *= Z.a;
            }
        }
    }
    __device__ __forceinline__ void done() { flush(); }
};

template <typename T> __device__ __forceinline__ T texp(T x);
template <> __device__ __forceinline__ double texp<double>(double x) { return exp(x); }
template <> __device__ __forceinline__ float texp<float>(float x) { return expf(x); }

// The moments of a general cell (index units): sum_r v(r) E(r) (s - s_A)^k
// over the monomials of the index offset, with the envelope
// E = exp(-alpha_p q), q = (s - s_P)^T g (s - s_P) = |r - P|^2, formed per point
// from the row's part (x and y offsets) and the z offset in the table, and
// the point kept iff q <= R^2.  Accumulated one axis at a time as in
// TensorVisit, with the envelope applied per point.
template <int L, typename T>
struct TensorVisitTri {
    static constexpr int K = ntab(L);
    T Vm[K], W[L + 1];
    T R2, nap;
    T gxx, gyy, gzz, gxy2, gxz2, gyz2;   // metric, off-diagonal terms doubled
    T xa = 0, ya = 0, qrow = 0, crow = 0, r2 = 0;
    __device__ TensorVisitTri(const PairRec &r, const LevelGeom &G) : R2((T)r.R2), nap((T)(-(r.aa + r.ab)))
    {
        const double(*g)[3] = G.tri->g;
        gxx = (T)g[0][0];
        gyy = (T)g[1][1];
        gzz = (T)g[2][2];
        gxy2 = (T)(2.0 * g[0][1]);
        gxz2 = (T)(2.0 * g[0][2]);
        gyz2 = (T)(2.0 * g[1][2]);
#pragma unroll
        for (int k = 0; k < K; ++k) Vm[k] = T(0);
#pragma unroll
        for (int k = 0; k <= L; ++k) W[k] = T(0);
    }
    __device__ __forceinline__ void flush()
    {
        T gx = T(1);   // (x-A_x)^lx
#pragma unroll
        for (int lx = 0; lx <= L; ++lx) {
            T g = gx;
#pragma unroll
            for (int ly = 0; lx + ly <= L; ++ly) {
#pragma unroll
                for (int lz = 0; lx + ly + lz <= L; ++lz) Vm[tidx(L, lx, ly, lz)] += W[lz] * g;
                g *= ya;
            }
            gx *= xa;
        }
#pragma unroll
        for (int k = 0; k <= L; ++k) W[k] = T(0);
    }
    // X.e, Y.e: offsets from P; X.a, Y.a: offsets from A; ok = false: a lane
    // without a row, every point cut (q >= 0 > -1)
    __device__ __forceinline__ void row(const PtXY<T> &X, const PtXY<T> &Y, bool ok)
    {
        flush();
        xa = X.a;
        ya = Y.a;
        const T dx = X.e, dy = Y.e;
        qrow = gxx * dx * dx + gxy2 * dx * dy + gyy * dy * dy;
        crow = gxz2 * dx + gyz2 * dy;
        r2 = ok ? R2 : T(-1);
    }
    // Z.e: z offset from P; Z.a: z - A_z
    __device__ __forceinline__ void point(T v, const PtZ<T> &Z)
    {
        const T q = qrow + Z.e * (gzz * Z.e + crow);
        const T f = keep_if(v * texp<T>(nap * q), q <= r2);
        W[0] += f;
        if constexpr (L >= 1) {
            T p = f * Z.a;   // f (z - A_z)^(lz - 1) for the next lz
            W[1] += p;
#pragma unroll
            for (int lz = 2; lz <= L; ++lz) {
                W[lz] += p * Z.a;
                if (lz < L) p *= Z.a;
            }
        }
    }
    __device__ __forceinline__ void done() { flush(); }
};

// Cartesian moments of a general cell's pair image from those of the index
// offset (degree <= L, tensor layout): with (r - A)^m = sum_k T_n[m][k]
// (s - s_A)^k, M_m = sum_k T_n[m][k] M'_k.  The wave splits the entries.
__device__ __forceinline__ void moments_to_cart(int L, const TriGeom *tg, const double *ms, double *mc)
{
    for (int e = threadIdx.x; e < ntab(L); e += 64) {
        int mx, my, mz;
        tidx_decode(L, e, mx, my, mz);
        const int n = mx + my + mz, nc = ncart(n);
        const double *__restrict__ Tn = tg->T + tg->toff[n] + cart_index(my, mz) * nc;
        double v = 0.0;
        for (int k = 0; k < nc; ++k) {
            const int kx = cart_lx(n, k), ky = cart_ly(n, k);
            v += Tn[k] * ms[tidx(L, kx, ky, n - kx - ky)];
        }
        mc[e] = v;
    }
}

// Wave sums of the K per-lane accumulators of a pair-major kernel, eight at
// a time through LDS (red[8][65], the kernel's LDS area once the traversal is
// done): lane 8q + s adds eight values of accumulator q, three shuffles
// finish the sum, and lane 8q applies emit(k, sum) for k = chunk + q.  The
// eight results of a chunk leave in parallel instead of one lane issuing
// every atomic.
constexpr size_t kRedBytes = (8 * 65 + 364) * sizeof(double);   // red[8][65] and up to ntab(11) moments
// a general cell: both sets of moments (index offset and Cartesian)
constexpr size_t kRedBytesTri = (8 * 65 + 2 * 364) * sizeof(double);
template <int K, typename T, typename Emit>
__device__ __forceinline__ void wave_reduce_emit(const T *acc, double *red, Emit &&emit)
{
    const int lane = threadIdx.x;
    const int q = lane >> 3, seg = lane & 7;
#pragma unroll
    for (int c0 = 0; c0 < K; c0 += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (c0 + u < K) red[u * 65 + lane] = (double)acc[c0 + u];
        __syncthreads();
        double v = 0.0;
#pragma unroll
        for (int m = 0; m < 8; ++m) v += red[q * 65 + seg * 8 + m];
        v += __shfl_xor(v, 1, 64);
        v += __shfl_xor(v, 2, 64);
        v += __shfl_xor(v, 4, 64);
        if (seg == 0 && c0 + q < K) emit(c0 + q, v);
        __syncthreads();
    }
}

// Block rows held in LDS at once: all emax^2 of the widest box up to
// kRowCap; wider boxes are traversed in slices of whole x entries (at least
// one: ny <= emax rows).
constexpr int kRowCap = 1024;
__host__ __device__ constexpr int row_capacity(int emax)
{
    return emax * emax <= kRowCap ? emax * emax : (kRowCap > emax ? kRowCap : emax);
}

// LDS layout of the pair-major kernels: the z point table tz[2 kZSlots emax]
// (its second half padding), the x and y point tables txy[2][4 emax], the block
// lists bl[3][emax], their counts, the run-length counters hist[emax + 1],
// and the block rows and their unsorted copy (row_capacity(emax) each).
template <typename T>
struct PairLds {
    PtXY<T> *txy;
    PtZ<T> *tz;
    AxisBlock *bl;
    int *cnt, *hist;
    BlockRow *rows, *tmp;
};
template <typename T>
struct PairSmem {
    static __host__ __device__ size_t table_bytes(int emax)
    {
        const size_t b = (8 * sizeof(PtXY<T>) + 2 * kZSlots * sizeof(PtZ<T>)) * (size_t)emax;
        return (b + 15) & ~size_t(15);
    }
    static __host__ __device__ size_t hist_ints(int emax) { return ((size_t)emax + 1 + 3) & ~size_t(3); }
    static __device__ __forceinline__ PairLds<T> carve(unsigned char *raw, int emax)
    {
        PairLds<T> l;
        l.tz = reinterpret_cast<PtZ<T> *>(raw);
        l.txy = reinterpret_cast<PtXY<T> *>(l.tz + 2 * kZSlots * emax);
        l.bl = reinterpret_cast<AxisBlock *>(raw + table_bytes(emax));
        l.cnt = reinterpret_cast<int *>(l.bl + 3 * emax);
        l.hist = l.cnt + 4;
        l.rows = reinterpret_cast<BlockRow *>(l.hist + hist_ints(emax));
        l.tmp = l.rows + row_capacity(emax);
        return l;
    }
    static size_t bytes(int emax, bool tri = false)
    {
        const size_t off = table_bytes(emax);
        const size_t b = off + sizeof(AxisBlock) * 3 * (size_t)emax + 16 + sizeof(int) * hist_ints(emax) +
                         2 * sizeof(BlockRow) * (size_t)row_capacity(emax);
        const size_t red = tri ? kRedBytesTri : kRedBytes;
        return b > red ? b : red;   // the area is reused for the final reduction
    }
};

// The pair image's blocks, row by row, in slices of whole x entries that fit
// the LDS rows (one slice unless the box is wider than kRowCap rows); the
// visitor's state carries over from slice to slice.  Ends with a barrier.
template <typename T, typename Vis>
__device__ __forceinline__ void traverse_slices(const PairRec &r, const PairSeg &sg, const PairLds<T> &l, Vis &vis)
{
    const int nx = uni(l.cnt[0]), ny = uni(l.cnt[1]);
    const int xs = ny > 0 ? (sg.row_cap / ny > 1 ? sg.row_cap / ny : 1) : nx;
    for (int ex0 = 0; ex0 < nx; ex0 += xs) {
        const int nrows = build_rows(r.R2 * kCullSlack, sg.G, sg.vz, l.bl, sg.emax, l.cnt, l.rows, l.tmp, l.hist,
                                     ex0, ex0 + xs < nx ? ex0 + xs : nx);
        __syncthreads();
        for_each_point<T>(l.txy, l.tz, sg.emax, l.rows, nrows, sg.Vb, vis);
        __syncthreads();   // the rows are rebuilt for the next slice
    }
}

// Moments of degree LT of one pair image (pair-major traversal), wave-summed
// into LDS past the reduction area; returns their address.  A general cell
// (TRI) accumulates the moments of the index offset and returns the
// Cartesian moments formed from them (after the first set).
template <int LT, typename T, bool TRI = false>
__device__ __forceinline__ const double *pair_moments(const PairSeg &sg, const PairRec &r, unsigned char *smem_raw)
{
    const LevelGeom &G = sg.G;
    const int emax = sg.emax;
    const PairLds<T> l = PairSmem<T>::carve(smem_raw, emax);
    pair_setup<true, T, TRI>(r, G, l.txy, l.tz, l.bl, emax, l.cnt);
    __syncthreads();
    using Vis = std::conditional_t<TRI, TensorVisitTri<LT, T>, TensorVisit<LT, T>>;
    Vis vis(r, G);
    traverse_slices<T>(r, sg, l, vis);
    // the traversal's LDS reads are done; the area becomes red[8][65]
    double *red = reinterpret_cast<double *>(smem_raw);
    double *mom = red + 8 * 65;
    wave_reduce_emit<ntab(LT), T>(vis.Vm, red, [&](int k, double v) { mom[k] = v; });
    __syncthreads();
    if constexpr (TRI) {
        double *mc = mom + ntab(LT);
        moments_to_cart(LT, G.tri, mom, mc);
        __syncthreads();
        return mc;
    }
    return mom;
}

// ------------------------------------ element formation from the moments
//
// Two forms.  Compile-time: element e of the pair image goes to lane e % 64
// with every exponent and expansion term resolved at compile time, each
// element under its own lane's mask (the wave steps through all of them).
// Runtime: one lane per element (i, j) with the element's Cartesian exponents
// as runtime values, every lane running the same instructions on products of
// one-axis factors (polynomials in u = x - A_x) contracted with the moments.
// Chosen per class by measurement on the 256-water system: the runtime form
// for the classes with many elements, the compile-time one where its
// specialised code is shorter.
__host__ __device__ constexpr bool mat_runtime_form(int la, int lb) { return (la == 2 && lb == 2) || (la >= 3 && lb >= 1); }
__host__ __device__ constexpr bool grad_runtime_form(int la, int lb)
{
    return (la == 1 && lb == 1) || (la == 2 && lb == 2) || (la >= 3 && lb >= 1);
}

// (d/du)^N (u^p e^{-a u^2}) / e^{-a u^2}, coefficients of u^k for k = 0..W-1
// (two_a = 2a): u^p; p u^(p-1) - 2a u^(p+1); p(p-1) u^(p-2) - 2a(2p+1) u^p +
// 4a^2 u^(p+2).
template <int W, int N>
__device__ __forceinline__ void deriv_poly(int p, double two_a, double *g)
{
#pragma unroll
    for (int k = 0; k < W; ++k) {
        double v;
        if constexpr (N == 0)
            v = k == p ? 1.0 : 0.0;
        else if constexpr (N == 1)
            v = (k == p - 1 ? (double)p : 0.0) + (k == p + 1 ? -two_a : 0.0);
        else
            v = (k == p - 2 ? (double)(p * (p - 1)) : 0.0) + (k == p ? -two_a * (2 * p + 1) : 0.0) +
                (k == p + 2 ? two_a * two_a : 0.0);
        g[k] = v;
    }
}

// One-axis factor of a term: [(d/du)^NA (u^p e^{-a u^2})] [(d/dv)^NB
// (v^q e^{-b v^2})] divided by both exponentials, with v = u + c (c = A - B),
// as a polynomial in u: f[k], k = 0..W-1 (W at least p + q + NA + NB + 1 for
// the lane's p <= PM, q <= QM; higher entries are zero).
template <int W, int PM, int QM, int NA, int NB>
__device__ __forceinline__ void axis_factor(int p, int q, double two_a, double two_b, double c, double *f)
{
    constexpr int GW = PM + NA + 1, HW = QM + NB + 1;
    static_assert(GW + HW - 1 <= W, "factor width");
    double g[GW], h[HW], hu[HW];
    deriv_poly<GW, NA>(p, two_a, g);
    deriv_poly<HW, NB>(q, two_b, h);
    // h(u + c) by Horner's rule in (u + c)
#pragma unroll
    for (int k = 0; k < HW; ++k) hu[k] = 0.0;
    hu[0] = h[HW - 1];
#pragma unroll
    for (int m = HW - 2; m >= 0; --m) {
#pragma unroll
        for (int k = HW - 1 - m; k >= 1; --k) hu[k] = hu[k - 1] + c * hu[k];
        hu[0] = c * hu[0] + h[m];
    }
#pragma unroll
    for (int k = 0; k < W; ++k) f[k] = 0.0;
#pragma unroll
    for (int i = 0; i < GW; ++i)
#pragma unroll
        for (int j = 0; j < HW; ++j) f[i + j] += g[i] * hu[j];
}

// sum over kx + ky + kz <= LT of fx[kx] fy[ky] fz[kz] mom[tidx(LT, kx, ky, kz)]
template <int LT, int W>
__device__ __forceinline__ double contract3(const double *fx, const double *fy, const double *fz, const double *mom)
{
    double sx = 0.0;
#pragma unroll
    for (int kx = 0; kx < W && kx <= LT; ++kx) {
        double sy = 0.0;
#pragma unroll
        for (int ky = 0; ky < W && kx + ky <= LT; ++ky) {
            double sz = 0.0;
#pragma unroll
            for (int kz = 0; kz < W && kx + ky + kz <= LT; ++kz) sz += fz[kz] * mom[tidx(LT, kx, ky, kz)];
            sy += fy[ky] * sz;
        }
        sx += fx[kx] * sy;
    }
    return sx;
}

__device__ __forceinline__ void cart_exps(int l, int n, int *e)
{
    e[0] = cart_lx(l, n);
    e[1] = cart_ly(l, n);
    e[2] = l - e[0] - e[1];
}

// Matrix element (i, j) from the moments of degree l_a + l_b, runtime form:
// per axis the factor u^a (u + c)^b with c = A - B (the binomial expansion of
// Eq. (binomial)), contracted with the moments.
template <int LA, int LB>
__device__ __forceinline__ double mat_element_rt(int i, int j, const double *AB, const double *mom)
{
    constexpr int L = LA + LB, W = L + 1;
    int a[3], b[3];
    cart_exps(LA, i, a);
    cart_exps(LB, j, b);
    double f[3][W];
#pragma unroll
    for (int e = 0; e < 3; ++e) axis_factor<W, LA, LB, 0, 0>(a[e], b[e], 0.0, 0.0, AB[e], f[e]);
    return contract3<L, W>(f[0], f[1], f[2], mom);
}

// d/dA_f and d/dB_f of the element (i, j) from the moments of degree
// l_a + l_b + 1, runtime form: with a_i depending on r - A, d/dA_f a_i =
// -d_f a_i (the derivative in r, the Gaussian factor included), and likewise
// for b_j; into g6[f] (A) and g6[3 + f] (B).
template <int LA, int LB>
__device__ __forceinline__ void grad_element_rt(int i, int j, double two_a, double two_b, const double *AB,
                                                const double *mom, double *g6)
{
    constexpr int L1 = LA + LB + 1, W = L1 + 1;
    int a[3], b[3];
    cart_exps(LA, i, a);
    cart_exps(LB, j, b);
    double f0[3][W], fA[3][W], fB[3][W];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        axis_factor<W, LA, LB, 0, 0>(a[e], b[e], two_a, two_b, AB[e], f0[e]);
        axis_factor<W, LA, LB, 1, 0>(a[e], b[e], two_a, two_b, AB[e], fA[e]);
        axis_factor<W, LA, LB, 0, 1>(a[e], b[e], two_a, two_b, AB[e], fB[e]);
    }
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        g6[f] = -contract3<L1, W>(f == 0 ? fA[0] : f0[0], f == 1 ? fA[1] : f0[1], f == 2 ? fA[2] : f0[2], mom);
        g6[3 + f] = -contract3<L1, W>(f == 0 ? fB[0] : f0[0], f == 1 ? fB[1] : f0[1], f == 2 ? fB[2] : f0[2], mom);
    }
}

// Matrix element (I, J) of a pair image from its potential moments:
// sum over the binomial expansion of (x-B)^b around A (Eq. (binomial)) of
// binom * (A-B)^(b-k) * moment(a + k); ab[d][p] = (A_d - B_d)^p.
template <int LA, int LB, int I, int J>
__device__ __forceinline__ double mat_element(const double *mom, const double (*ab)[LB + 1])
{
    constexpr int L = LA + LB;
    constexpr int ax = cart_lx(LA, I), ay = cart_ly(LA, I), az = LA - ax - ay;
    constexpr int bx = cart_lx(LB, J), by = cart_ly(LB, J), bz = LB - bx - by;
    double m = 0.0;
#pragma unroll
    for (int kx = 0; kx <= bx; ++kx)
#pragma unroll
        for (int ky = 0; ky <= by; ++ky)
#pragma unroll
            for (int kz = 0; kz <= bz; ++kz)
                m += (double)(binom(bx, kx) * binom(by, ky) * binom(bz, kz)) * ab[0][bx - kx] * ab[1][by - ky] *
                     ab[2][bz - kz] * mom[tidx(L, ax + kx, ay + ky, az + kz)];
    return m;
}
// Element e of the pair image goes to lane e % 64 (slot e / 64 of m[]); each
// element is computed under its own lane's mask, so the work is the sum of
// the elements' terms.
template <int LA, int LB, int... E>
__device__ __forceinline__ void mat_elements(std::integer_sequence<int, E...>, const double *mom,
                                             const double (*ab)[LB + 1], int lane, double *m)
{
    constexpr int NB = ncart_c(LB);
    ((lane == E % 64 ? (void)(m[E / 64] = mat_element<LA, LB, E / NB, E % NB>(mom, ab)) : (void)0), ...);
}

// TRI: a general cell, always through the moments (formed on the index
// offset, then made Cartesian).
template <int LA, int LB, typename T, bool TRI = false>
__global__ void __launch_bounds__(64)
k_mat(SegTable<PairSeg> tab)
{
    constexpr int NA = ncart_c(LA), NB = ncart_c(LB);
    extern __shared__ unsigned char smem_raw[];
    const PairSeg &sg = tab.s[seg_of(tab, blockIdx.x)];
    const long long item = xcd_ranged(blockIdx.x - sg.item0, sg.xs);
    if (item < 0) return;
    const LevelGeom &G = sg.G;
    const int n_ao = sg.n_ao;
    const PairRec &r = sg.pairs[item];
    const double scale = 0.5 * G.w * r.Kw;
    if constexpr (!TRI && !mat_tensor(LA, LB)) {
        const int emax = sg.emax;
        const PairLds<T> l = PairSmem<T>::carve(smem_raw, emax);
        pair_setup<false, T>(r, G, l.txy, l.tz, l.bl, emax, l.cnt);
        __syncthreads();
        T acc[NA * NB];
#pragma unroll
        for (int i = 0; i < NA * NB; ++i) acc[i] = T(0);
        auto body = [&](T f, T xa, T ya, T za, T xb, T yb, T zb) {
            T a[NA], bb[NB];
            monomials<LA, T>(xa, ya, za, a);
            monomials<LB, T>(xb, yb, zb, bb);
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                const T fa = f * a[i];
#pragma unroll
                for (int j = 0; j < NB; ++j) acc[i * NB + j] += fa * bb[j];
            }
        };
        DirectVisit<T, decltype(body)> vis(body, r);
        traverse_slices<T>(r, sg, l, vis);
        // the traversal's LDS reads are done; the area becomes red[8][65]
        wave_reduce_emit<NA * NB, T>(acc, reinterpret_cast<double *>(smem_raw), [&](int k, double v) {
            const int i = k / NB, j = k - (k / NB) * NB;
            atomicAdd(&sg.out[(long long)(r.ao_a + i) * n_ao + r.ao_b + j], scale * v);
            atomicAdd(&sg.out[(long long)(r.ao_b + j) * n_ao + r.ao_a + i], scale * v);
        });
    } else {
        // the moments of the monomials of r - A up to degree l_a + l_b, then
        // element (i, j) from the moments of (x-A)^a (x-B)^b with every
        // (x - B_x)^b_x expanded binomially around A (Eq. (binomial))
        const double *mom = pair_moments<LA + LB, T, TRI>(sg, r, smem_raw);
        double AB[3];
        cart_ab(r, TRI ? G.tri : nullptr, AB);
        double ab[3][LB + 1];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            ab[d][0] = 1.0;
#pragma unroll
            for (int k = 1; k <= LB; ++k) ab[d][k] = ab[d][k - 1] * AB[d];
        }
        constexpr int NE = NA * NB, NS = (NE + 63) / 64;
        double m[NS];
        if constexpr (mat_runtime_form(LA, LB)) {
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const int ij = q * 64 + (int)threadIdx.x;
                m[q] = ij < NE ? mat_element_rt<LA, LB>(ij / NB, ij % NB, AB, mom) : 0.0;
            }
        } else {
            mat_elements<LA, LB>(std::make_integer_sequence<int, NE>{}, mom, ab, (int)threadIdx.x, m);
        }
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int ij = q * 64 + (int)threadIdx.x;
            if (ij < NE) {
                const int i = ij / NB, j = ij - (ij / NB) * NB;
                atomicAdd(&sg.out[(long long)(r.ao_a + i) * n_ao + r.ao_b + j], scale * m[q]);
                atomicAdd(&sg.out[(long long)(r.ao_b + j) * n_ao + r.ao_a + i], scale * m[q]);
            }
        }
    }
}

// Gradient contributions of element (I, J) of a pair image from its potential
// moments up to degree l_a + l_b + 1: with E = exp(-a |r-A|^2 - b |r-B|^2),
//   d/dA_d [a_i b_j E] = (2 a (r-A)_d a_i - d_d a_i) b_j E,
//   d/dB_d [a_i b_j E] = (2 b (r-B)_d b_j - d_d b_j) a_i E,
// both polynomials in r - A once (r - B) = (r - A) + (A - B) is expanded
// binomially (Eq. (binomial)); weighted by the symmetrised D_ij into g6.
template <int LA, int LB, int I, int J>
__device__ __forceinline__ void grad_element(const double *mom, const double (*ab)[LB + 1], double two_a,
                                             double two_b, const double *AB, double dij, double *g6)
{
    constexpr int L1 = LA + LB + 1;
    constexpr int a[3] = {cart_lx(LA, I), cart_ly(LA, I), LA - cart_lx(LA, I) - cart_ly(LA, I)};
    constexpr int b[3] = {cart_lx(LB, J), cart_ly(LB, J), LB - cart_lx(LB, J) - cart_ly(LB, J)};
    double ga[3] = {0.0, 0.0, 0.0}, gb[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int kx = 0; kx <= b[0]; ++kx)
#pragma unroll
        for (int ky = 0; ky <= b[1]; ++ky)
#pragma unroll
            for (int kz = 0; kz <= b[2]; ++kz) {
                const double c = (double)(binom(b[0], kx) * binom(b[1], ky) * binom(b[2], kz)) * ab[0][b[0] - kx] *
                                 ab[1][b[1] - ky] * ab[2][b[2] - kz];
                const int m0 = a[0] + kx, m1 = a[1] + ky, m2 = a[2] + kz;
                const double M0 = mom[tidx(L1, m0, m1, m2)];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double Md = mom[tidx(L1, m0 + (d == 0), m1 + (d == 1), m2 + (d == 2))];
                    double da = 0.0;   // d_d (r-A)^a_d
                    if (a[d] > 0) da = a[d] * mom[tidx(L1, m0 - (d == 0), m1 - (d == 1), m2 - (d == 2))];
                    ga[d] += c * (two_a * Md - da);
                    gb[d] += c * two_b * (Md + AB[d] * M0);
                }
            }
    // - a_i d_d b_j(r - B) = - b_d a_i (r - B)^(b - e_d), expanded the same way
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (b[d] == 0) continue;
        const int c0 = b[0] - (d == 0), c1 = b[1] - (d == 1), c2 = b[2] - (d == 2);
#pragma unroll
        for (int kx = 0; kx <= c0; ++kx)
#pragma unroll
            for (int ky = 0; ky <= c1; ++ky)
#pragma unroll
                for (int kz = 0; kz <= c2; ++kz) {
                    const double c = (double)(binom(c0, kx) * binom(c1, ky) * binom(c2, kz)) * ab[0][c0 - kx] *
                                     ab[1][c1 - ky] * ab[2][c2 - kz];
                    gb[d] -= b[d] * c * mom[tidx(L1, a[0] + kx, a[1] + ky, a[2] + kz)];
                }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        g6[d] += dij * ga[d];
        g6[3 + d] += dij * gb[d];
    }
}
template <int LA, int LB, typename T, int... E>
__device__ __forceinline__ void grad_elements(std::integer_sequence<int, E...>, const double *mom,
                                              const double (*ab)[LB + 1], double two_a, double two_b,
                                              const double *AB, const T *Dp, long long n_ao, int lane, double *g6)
{
    constexpr int NB = ncart_c(LB);
    ((lane == E % 64 ? grad_element<LA, LB, E / NB, E % NB>(mom, ab, two_a, two_b, AB,
                                                            (double)Dp[(E / NB) * n_ao + E % NB], g6)
                     : (void)0),
     ...);
}

template <int LA, int LB, typename T, bool TRI = false>
__global__ void __launch_bounds__(64)
k_grad(SegTable<PairSeg> tab)
{
    constexpr int NA = ncart_c(LA), NB = ncart_c(LB);
    extern __shared__ unsigned char smem_raw[];
    const PairSeg &sg = tab.s[seg_of(tab, blockIdx.x)];
    const long long item = xcd_ranged(blockIdx.x - sg.item0, sg.xs);
    if (item < 0) return;
    const LevelGeom &G = sg.G;
    const int n_ao = sg.n_ao;
    const PairRec &r = sg.pairs[item];
    // potential moments of the monomials of r - A up to degree l_a + l_b + 1
    const double *mom = pair_moments<LA + LB + 1, T, TRI>(sg, r, smem_raw);
    const T *Dp = (const T *)sg.Dm + (long long)r.ao_a * n_ao + r.ao_b;
    double AB[3];
    cart_ab(r, TRI ? G.tri : nullptr, AB);
    double ab[3][LB + 1];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ab[d][0] = 1.0;
#pragma unroll
        for (int k = 1; k <= LB; ++k) ab[d][k] = ab[d][k - 1] * AB[d];
    }
    double g6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if constexpr (grad_runtime_form(LA, LB)) {
#pragma unroll 1
        for (int e0 = 0; e0 < NA * NB; e0 += 64) {
            const int e = e0 + (int)threadIdx.x;
            if (e < NA * NB) {
                double t6[6];
                grad_element_rt<LA, LB>(e / NB, e % NB, 2.0 * r.aa, 2.0 * r.ab, AB, mom, t6);
                const double dij = (double)Dp[(long long)(e / NB) * n_ao + e % NB];
#pragma unroll
                for (int k = 0; k < 6; ++k) g6[k] += dij * t6[k];
            }
        }
    } else {
        grad_elements<LA, LB, T>(std::make_integer_sequence<int, NA * NB>{}, mom, ab, 2.0 * r.aa, 2.0 * r.ab, AB,
                                 Dp, n_ao, (int)threadIdx.x, g6);
    }
    const double scale = G.w * r.Kw;
    __syncthreads();   // every read of the moments is done
    wave_reduce_emit<6, double>(g6, reinterpret_cast<double *>(smem_raw), [&](int k, double v) {
        atomicAdd(&sg.out[3 * (k < 3 ? r.atom_a : r.atom_b) + (k < 3 ? k : k - 3)], scale * v);
    });
}

// ---------------------------------- kinetic-energy-density integration and gradient
//
// Matrix elements and gradients of the meta-GGA term from potential moments of
// degree l_a + l_b + 2 (integration) and l_a + l_b + 3 (gradient), in the
// runtime form for every class.

// sum_d of the d_d a_i d_d b_j moments (moments of degree l_a + l_b + 2).
template <int LA, int LB>
__device__ __forceinline__ double mat_tau_element(int i, int j, double two_a, double two_b, const double *AB,
                                                  const double *mom)
{
    constexpr int LT = LA + LB + 2, W = LT + 1;
    int a[3], b[3];
    cart_exps(LA, i, a);
    cart_exps(LB, j, b);
    double f0[3][W], f1[3][W];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        axis_factor<W, LA, LB, 0, 0>(a[e], b[e], two_a, two_b, AB[e], f0[e]);
        axis_factor<W, LA, LB, 1, 1>(a[e], b[e], two_a, two_b, AB[e], f1[e]);
    }
    return contract3<LT, W>(f1[0], f0[1], f0[2], mom) + contract3<LT, W>(f0[0], f1[1], f0[2], mom) +
           contract3<LT, W>(f0[0], f0[1], f1[2], mom);
}

// d/dA_f and d/dB_f of sum_d d_d a_i d_d b_j (moments of degree
// l_a + l_b + 3): with a_i depending on r - A, d/dA_f d_d a_i = -d_f d_d a_i,
// and likewise for b_j; the results go to g6[f] (A) and g6[3 + f] (B).
template <int LA, int LB>
__device__ __forceinline__ void grad_tau_element(int i, int j, double two_a, double two_b, const double *AB,
                                                 const double *mom, double *g6)
{
    constexpr int LT = LA + LB + 3, W = LT + 1;
    int a[3], b[3];
    cart_exps(LA, i, a);
    cart_exps(LB, j, b);
#pragma unroll
    for (int k = 0; k < 6; ++k) g6[k] = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        // per axis: the factors of this direction d (on d: both differentiated
        // once more or not; elsewhere: plain or one side differentiated)
        double fp[3][W], fA[3][W], fB[3][W];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            if (e == d) {
                axis_factor<W, LA, LB, 1, 1>(a[e], b[e], two_a, two_b, AB[e], fp[e]);
                axis_factor<W, LA, LB, 2, 1>(a[e], b[e], two_a, two_b, AB[e], fA[e]);
                axis_factor<W, LA, LB, 1, 2>(a[e], b[e], two_a, two_b, AB[e], fB[e]);
            } else {
                axis_factor<W, LA, LB, 0, 0>(a[e], b[e], two_a, two_b, AB[e], fp[e]);
                axis_factor<W, LA, LB, 1, 0>(a[e], b[e], two_a, two_b, AB[e], fA[e]);
                axis_factor<W, LA, LB, 0, 1>(a[e], b[e], two_a, two_b, AB[e], fB[e]);
            }
        }
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            g6[f] -= contract3<LT, W>(f == 0 ? fA[0] : fp[0], f == 1 ? fA[1] : fp[1], f == 2 ? fA[2] : fp[2], mom);
            g6[3 + f] -= contract3<LT, W>(f == 0 ? fB[0] : fp[0], f == 1 ? fB[1] : fp[1], f == 2 ? fB[2] : fp[2],
                                          mom);
        }
    }
}

// Kinetic-energy-density term of the matrix (the variational derivative of
// E_tau = sum_l w_l <vtau_l, tau_l(D)>): M_ij += 1/2 w sum_r vtau grad a_i .
// grad b_j (Sec. II, Eq. (J_metaGGA); Sec. III.B with Alg. 2), one wave per
// pair image, both triangles.
template <int LA, int LB, typename T, bool TRI = false>
__global__ void __launch_bounds__(64)
k_mat_tau(SegTable<PairSeg> tab)
{
    constexpr int NA = ncart_c(LA), NB = ncart_c(LB);
    extern __shared__ unsigned char smem_raw[];
    const PairSeg &sg = tab.s[seg_of(tab, blockIdx.x)];
    const long long item = xcd_ranged(blockIdx.x - sg.item0, sg.xs);
    if (item < 0) return;
    const PairRec &r = sg.pairs[item];
    const double *mom = pair_moments<LA + LB + 2, T, TRI>(sg, r, smem_raw);
    double AB[3];
    cart_ab(r, TRI ? sg.G.tri : nullptr, AB);
    // 1/2 of the meta-GGA term times the 1/2 that splits Kw over both triangles
    const double scale = 0.25 * sg.G.w * r.Kw;
    const int n_ao = sg.n_ao;
#pragma unroll 1
    for (int e0 = 0; e0 < NA * NB; e0 += 64) {
        const int e = e0 + (int)threadIdx.x;
        if (e < NA * NB) {
            const int i = e / NB, j = e - (e / NB) * NB;
            const double m = scale * mat_tau_element<LA, LB>(i, j, 2.0 * r.aa, 2.0 * r.ab, AB, mom);
            atomicAdd(&sg.out[(long long)(r.ao_a + i) * n_ao + r.ao_b + j], m);
            atomicAdd(&sg.out[(long long)(r.ao_b + j) * n_ao + r.ao_a + i], m);
        }
    }
}

// Nuclear gradient of E_tau at fixed D and vtau (Sec. III.B, the meta-GGA
// note with Alg. 3): second derivatives of the first factor and first
// derivatives of the second, one lane per element weighted by the symmetrised
// D_ij, a wave sum of the six components, atomics into the two atoms.
template <int LA, int LB, typename T, bool TRI = false>
__global__ void __launch_bounds__(64)
k_grad_tau(SegTable<PairSeg> tab)
{
    constexpr int NA = ncart_c(LA), NB = ncart_c(LB);
    extern __shared__ unsigned char smem_raw[];
    const PairSeg &sg = tab.s[seg_of(tab, blockIdx.x)];
    const long long item = xcd_ranged(blockIdx.x - sg.item0, sg.xs);
    if (item < 0) return;
    const PairRec &r = sg.pairs[item];
    const double *mom = pair_moments<LA + LB + 3, T, TRI>(sg, r, smem_raw);
    double AB[3];
    cart_ab(r, TRI ? sg.G.tri : nullptr, AB);
    const int n_ao = sg.n_ao;
    const T *Dp = (const T *)sg.Dm + (long long)r.ao_a * n_ao + r.ao_b;
    double g6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int e0 = 0; e0 < NA * NB; e0 += 64) {
        const int e = e0 + (int)threadIdx.x;
        if (e < NA * NB) {
            const int i = e / NB, j = e - (e / NB) * NB;
            double t6[6];
            grad_tau_element<LA, LB>(i, j, 2.0 * r.aa, 2.0 * r.ab, AB, mom, t6);
            const double dij = (double)Dp[(long long)i * n_ao + j];
#pragma unroll
            for (int k = 0; k < 6; ++k) g6[k] += dij * t6[k];
        }
    }
    // 1/2 of the meta-GGA term; Kw carries the weight of the canonical pair
    const double scale = 0.5 * sg.G.w * r.Kw;
    __syncthreads();   // every read of the moments is done
    wave_reduce_emit<6, double>(g6, reinterpret_cast<double *>(smem_raw), [&](int k, double v) {
        atomicAdd(&sg.out[3 * (k < 3 ? r.atom_a : r.atom_b) + (k < 3 ? k : k - 3)], scale * v);
    });
}

// Growable array with room for N elements inline: the launch path of a
// single evaluation stays inside the inline storage and so makes no host
// allocation (the heap holds only what a large batch adds past N).
template <typename T, int N>
struct SmallVec {
    T buf[N];
    std::vector<T> more;
    size_t n = 0;
    size_t size() const { return n; }
    T &operator[](size_t i) { return i < (size_t)N ? buf[i] : more[i - N]; }
    const T &operator[](size_t i) const { return i < (size_t)N ? buf[i] : more[i - N]; }
    void push_back(const T &x)
    {
        if (n < (size_t)N) buf[n] = x;
        else more.push_back(x);
        ++n;
    }
    void resize(size_t m)
    {
        if (m > (size_t)N) more.resize(m - N);
        n = m;
    }
};

// Segments of one (operation, class) and the launches that cover them, at
// most kMaxSeg segments per launch.
template <typename S>
struct SegList {
    SmallVec<S, kMaxSeg> v;
    SmallVec<long long, kMaxSeg> items;
    void add(const S &s, long long n)
    {
        if (n <= 0) return;
        v.push_back(s);
        items.push_back(n);
    }
    // launch(table, grid) once per chunk of at most kMaxSeg segments
    template <typename L>
    void launch(L &&fn, bool xcd) const
    {
        for (size_t i0 = 0; i0 < v.size(); i0 += kMaxSeg) {
            SegTable<S> t;
            t.n = (int)std::min<size_t>(kMaxSeg, v.size() - i0);
            long long tot = 0;
            for (int k = 0; k < t.n; ++k) {
                t.s[k] = v[i0 + k];
                t.s[k].item0 = tot;
                tot += xcd ? (long long)xcd_grid(items[i0 + k]) : items[i0 + k];
            }
            t.total = tot;
            fn(t, (unsigned)tot);
        }
    }
};

// The segments of one (l_a, l_b) class for every operation of a batch, and
// how to launch them.
struct ClassLaunch {
    SegList<PackSeg> packs, tpacks;      // packed coefficients of rho / tau
    SegList<RhoSeg> rhos, taus;          // grid-block major collocation
    SegList<PairSeg> mats, grads, mtaus, gtaus;   // pair-major integration / gradient
    // general cells: the density's coefficient tensors (every class), their
    // rewrite on the index offset (rho and tau), and the kernels of index units
    SegList<PackSeg> packs_t;
    SegList<IdxSeg> idxs;
    SegList<RhoSeg> rhos_t, taus_t;
    SegList<PairSeg> mats_t, grads_t, mtaus_t, gtaus_t;
    size_t smem = 0;                     // LDS bytes of the pair-major kernels
    size_t smem_t = 0;                   // the same, general cells
    hipStream_t st = nullptr;
    bool fp32 = false;                   // per-point arithmetic in float
};
// Enqueue the launches of class c (defined in gpw_class.hip, one object per class).
void launch_class(int c, const ClassLaunch &cl);

}  // namespace gpw
