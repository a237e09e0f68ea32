// Shell-pair task partitioner (plan construction) for gfx950.
//
// 1. k_pairs<false/true>: one thread per unordered pair of primitive shells
//    enumerates the lattice images of the second factor, keeps the images
//    whose maximum of |K| r^(L+2) exp(-alpha_p r^2) reaches tau (Sec. III.A,
//    Eq. (cut) applied to the pair product), and writes canonical pair-image
//    records grouped by (level, (l_a, l_b) class).  This is the pair screening
//    of the appendix (Alg. 4), with a count pass and a fill pass instead of a
//    single compaction pass.
// 2. k_incidences<false/true>: one thread per pair image lists the 4x4x4 grid
//    blocks (with their fold shifts) that meet the truncation sphere, counting
//    per (group, block), then filling a CSR list per block.  This replaces the
//    block-major count of the appendix's mapping step (Alg. 5), which scans
//    every pair for every block, by a pair-major scatter; blocks that miss the
//    sphere are never listed, which takes the place of its fine screening.
// 3. Hand-written exclusive scans (wave64 shuffles + LDS) turn counts into
//    offsets and compact the nonempty blocks of every group.
#include "gpw_internal.h"

#include <algorithm>

namespace gpw {

__device__ inline int level_for(const PlanConst &pc, double alpha_p)
{
    for (int i = pc.nlevels - 1; i >= 1; --i)
        if (pc.cut[i] >= alpha_p * pc.rel_cut) return i;
    return 0;
}

// Root R > r* of log|K| + (L+2) log r - alpha r^2 = log tau.  g is concave,
// so Newton from a point right of the root decreases monotonically onto it.
__device__ double trunc_radius(double logK, int L, double alpha, double logtau)
{
    const double rs = sqrt((L + 2) / (2.0 * alpha));
    const double g_rs = logK + (L + 2) * log(rs) - alpha * rs * rs - logtau;
    double r = rs + sqrt(fmax(g_rs, 0.0) / alpha) * (1.0 + 1e-9) + 1e-12;
    for (int it = 0; it < 100; ++it) {
        const double g = logK + (L + 2) * log(r) - alpha * r * r - logtau;
        const double dg = (L + 2) / r - 2.0 * alpha * r;
        const double step = g / dg;      // g <= 0, dg < 0 -> step >= 0
        const double rn = r - step;
        if (!(rn < r) || r - rn <= 1e-16 * r) { r = fmin(r, rn); break; }
        r = rn;
    }
    return r;
}

template <bool FILL>
__global__ void __launch_bounds__(256)
k_pairs(PsTable ps, PlanConst pc, unsigned long long *group_cnt, const long long *group_off,
        unsigned long long *group_cur, PairRec *out, int *err_flag)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = ps.n;
    if (idx >= n * n) return;
    const int i = (int)(idx / n), j = (int)(idx % n);
    if (j < i) return;
    // orientation: the first factor carries the higher angular momentum
    int fa = i, fb = j;
    if (ps.l[j] > ps.l[i]) { fa = j; fb = i; }
    const int la = ps.l[fa], lb = ps.l[fb];
    const double aa = ps.alpha[fa], ab = ps.alpha[fb];
    const double ca = ps.coef[fa], cb = ps.coef[fb];
    if (ca == 0.0 || cb == 0.0) return;
    const double *A = ps.coords + 3 * ps.atom[fa];
    const double *B = ps.coords + 3 * ps.atom[fb];
    const int L = la + lb;
    const double ap = aa + ab, mu = aa * ab / ap;
    const double rs2 = (L + 2) / (2.0 * ap);
    const double logcc = log(fabs(ca * cb));
    // survives iff log|K| + (L+2)/2 (log rs2 - 1) >= log tau, log|K| = logcc - mu d^2
    const double Q = logcc + 0.5 * (L + 2) * (log(rs2) - 1.0) - pc.logtau;
    if (Q < 0.0) return;
    const double dmax = sqrt(Q / mu);
    long long nlo[3], nhi[3];
    double AB0[3];
    for (int d = 0; d < 3; ++d) AB0[d] = A[d] - B[d];
    for (int d = 0; d < 3; ++d) {
        if (pc.tri) {
            // |A - B - T| <= dmax bounds the fractional coordinate of A - B - T
            const double u = AB0[0] * pc.Ainv[0][d] + AB0[1] * pc.Ainv[1][d] + AB0[2] * pc.Ainv[2][d];
            const double du = dmax * sqrt(pc.Ainv[0][d] * pc.Ainv[0][d] + pc.Ainv[1][d] * pc.Ainv[1][d] +
                                          pc.Ainv[2][d] * pc.Ainv[2][d]);
            nlo[d] = (long long)ceil(u - du) - 1;
            nhi[d] = (long long)floor(u + du) + 1;
        } else {
            nlo[d] = (long long)ceil((AB0[d] - dmax) / pc.L[d]);
            nhi[d] = (long long)floor((AB0[d] + dmax) / pc.L[d]);
        }
    }
    const int lvl = level_for(pc, ap);
    const int g = lvl * kNCls + cls_of(la, lb);
    for (long long n0 = nlo[0]; n0 <= nhi[0]; ++n0)
        for (long long n1 = nlo[1]; n1 <= nhi[1]; ++n1)
            for (long long n2 = nlo[2]; n2 <= nhi[2]; ++n2) {
                if (i == j) {   // same primitive shell: keep T = 0 and one of +-T
                    if (n0 < 0 || (n0 == 0 && (n1 < 0 || (n1 == 0 && n2 < 0)))) continue;
                }
                // A - B - T, T = n0 a_0 + n1 a_1 + n2 a_2
                double Tv[3];
                for (int c = 0; c < 3; ++c)
                    Tv[c] = pc.tri ? n0 * pc.A[0][c] + n1 * pc.A[1][c] + n2 * pc.A[2][c]
                                   : (c == 0 ? n0 * pc.L[0] : c == 1 ? n1 * pc.L[1] : n2 * pc.L[2]);
                const double t0 = AB0[0] - Tv[0];
                const double t1 = AB0[1] - Tv[1];
                const double t2 = AB0[2] - Tv[2];
                const double d2 = t0 * t0 + t1 * t1 + t2 * t2;
                if (mu * d2 > Q) continue;
                if (!FILL) {
                    atomicAdd(&group_cnt[g], 1ull);
                    continue;
                }
                const unsigned long long pos = atomicAdd(&group_cur[g], 1ull);
                // the fill pass repeats the count pass's decisions; never write
                // past the counted size should the two ever disagree
                if ((long long)pos >= group_off[g + 1] - group_off[g]) { atomicOr(err_flag, 1); continue; }
                const long long slot = group_off[g] + (long long)pos;
                PairRec r;
                const double wc = (i == j && n0 == 0 && n1 == 0 && n2 == 0) ? 1.0 : 2.0;
                const double logK = logcc - mu * d2;
                const double R = trunc_radius(logK, L, ap, pc.logtau);
                const double Bp[3] = {B[0] + Tv[0], B[1] + Tv[1], B[2] + Tv[2]};
                const LevelGeom &G = pc.geom[lvl];
                const TriGeom *tg = G.tri;
                for (int d = 0; d < 3; ++d) {
                    r.A[d] = A[d];
                    r.AB[d] = A[d] - Bp[d];
                    r.P[d] = (aa * A[d] + ab * Bp[d]) / ap;
                }
                if (tg) {
                    // a general cell: positions in the level's index coordinates s = r Hinv
                    double sA[3], sAB[3], sP[3];
                    for (int d = 0; d < 3; ++d) {
                        sA[d] = r.A[0] * tg->Hinv[0][d] + r.A[1] * tg->Hinv[1][d] + r.A[2] * tg->Hinv[2][d];
                        sAB[d] = r.AB[0] * tg->Hinv[0][d] + r.AB[1] * tg->Hinv[1][d] + r.AB[2] * tg->Hinv[2][d];
                        sP[d] = r.P[0] * tg->Hinv[0][d] + r.P[1] * tg->Hinv[1][d] + r.P[2] * tg->Hinv[2][d];
                    }
                    for (int d = 0; d < 3; ++d) {
                        r.A[d] = sA[d];
                        r.AB[d] = sAB[d];
                        r.P[d] = sP[d];
                        r.lo[d] = (int)ceil(r.P[d] - R * tg->rf[d]);
                        r.hi[d] = (int)floor(r.P[d] + R * tg->rf[d]);
                    }
                } else {
                    for (int d = 0; d < 3; ++d) {
                        r.lo[d] = (int)ceil((r.P[d] - R) / G.h[d]);
                        r.hi[d] = (int)floor((r.P[d] + R) / G.h[d]);
                    }
                }
                r.aa = aa;
                r.ab = ab;
                r.Kw = wc * ca * cb * exp(-mu * d2);
                r.R2 = R * R;
                r.ER = exp(-ap * R * R);
                for (int d = 0; d < 3; ++d) r.c[d] = exp(-ap * (tg ? tg->g[d][d] : G.h[d] * G.h[d]));
                for (int d = 0; d < 3; ++d) {
                    const int g0 = axis_block_id(r.lo[d], G.N[d], G.nb[d]);
                    r.bs0[d] = floordiv(g0, G.nb[d]);
                    r.bk0[d] = g0 - r.bs0[d] * G.nb[d];
                    r.bn[d] = axis_block_count(r.lo[d], r.hi[d], G.N[d], G.nb[d]);
                }
                {
                    // the z gaps fall before this entry and rise from it on
                    int e = 0, k = r.bk0[2], S = r.bs0[2];
                    for (; e < r.bn[2]; ++e) {
                        const int u1 = (4 * k + 3 < G.N[2] - 1 ? 4 * k + 3 : G.N[2] - 1) + S * G.N[2];
                        if ((double)u1 * G.h[2] >= r.P[2]) break;
                        if (++k == G.nb[2]) { k = 0; ++S; }
                    }
                    r.bem = e;
                }
                r.bpad[0] = r.bpad[1] = 0;
                r.ao_a = ps.ao[fa];
                r.ao_b = ps.ao[fb];
                r.atom_a = ps.atom[fa];
                r.atom_b = ps.atom[fb];
                r.la = la;
                r.lb = lb;
                r.level = lvl;
                r.cls = cls_of(la, lb);
                r.pad2 = r.pad3 = 0;
                out[slot] = r;
            }
}

template <bool FILL>
__global__ void __launch_bounds__(256)
k_incidences(const PairRec *pairs, long long npairs, PlanConst pc, const long long *cnt_base_g,
             unsigned *counters, const long long *offsets, unsigned *cursors, int2 *entries,
             double *stats, int *maxw, int *err_flag, int *work = nullptr)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    const PairRec &r = pairs[p];
    const LevelGeom &G = pc.geom[r.level];
    const int g = r.level * kNCls + r.cls;
    const double R2c = r.R2 * kCullSlack;
    const long long base = cnt_base_g[g];
    // per-axis gaps in Cartesian units (orthorhombic), or in index units scaled
    // by the metric's smallest eigenvalue (a general cell: their sum stays below
    // the block's true squared distance, so the cull is conservative)
    const double gs = G.tri ? G.tri->lmin : 1.0;
    long long ninc = 0;
    AxisIter ix, iy, iz;
    for (ix.start(r.lo[0], r.hi[0], G.N[0], G.nb[0]); ix.valid(); ix.next()) {
        double x0, x1;
        ix.range(G.h[0], x0, x1);
        const double gx = gs * axis_gap2(r.P[0], x0, x1);
        if (gx > R2c) continue;
        for (iy.start(r.lo[1], r.hi[1], G.N[1], G.nb[1]); iy.valid(); iy.next()) {
            double y0, y1;
            iy.range(G.h[1], y0, y1);
            const double gy = gx + gs * axis_gap2(r.P[1], y0, y1);
            if (gy > R2c) continue;
            for (iz.start(r.lo[2], r.hi[2], G.N[2], G.nb[2]); iz.valid(); iz.next()) {
                double z0, z1;
                iz.range(G.h[2], z0, z1);
                if (gy + gs * axis_gap2(r.P[2], z0, z1) > R2c) continue;
                const long long b = block_slot(G, (int)ix.k, (int)iy.k, (int)iz.k);
                if (ix.S < -127 || ix.S > 127 || iy.S < -127 || iy.S > 127 || iz.S < -127 || iz.S > 127) {
                    atomicOr(err_flag, 2);   // fold shift does not fit the packed entry
                    continue;
                }
                ++ninc;
                if (!FILL) {
                    atomicAdd(&counters[base + b], 1u);
                } else {
                    const unsigned pos = atomicAdd(&cursors[base + b], 1u);
                    if (pos >= counters[base + b]) { atomicOr(err_flag, 1); continue; }
                    entries[offsets[base + b] + pos] =
                        make_int2((int)p, pack_shift((int)ix.S, (int)iy.S, (int)iz.S));
                }
            }
        }
    }
    if (!FILL && stats) {
        // points inside the sphere (row by row), for the flop model
        long long npts = 0;
        for (int ux = r.lo[0]; ux <= r.hi[0]; ++ux) {
            const double dx = (double)ux * G.h[0] - r.P[0];
            for (int uy = r.lo[1]; uy <= r.hi[1]; ++uy) {
                const double dy = (double)uy * G.h[1] - r.P[1];
                long long z0, z1;
                if (G.tri) {
                    // (dx, dy, dz) g (dx, dy, dz)^T <= R^2, a quadratic in dz
                    const double(*gm)[3] = G.tri->g;
                    const double qa = gm[2][2], qb = 2.0 * (gm[0][2] * dx + gm[1][2] * dy);
                    const double qc = gm[0][0] * dx * dx + 2.0 * gm[0][1] * dx * dy + gm[1][1] * dy * dy - r.R2;
                    const double disc = qb * qb - 4.0 * qa * qc;
                    if (disc < 0.0) continue;
                    const double sq = sqrt(disc);
                    z0 = (long long)ceil(r.P[2] + (-qb - sq) / (2.0 * qa));
                    z1 = (long long)floor(r.P[2] + (-qb + sq) / (2.0 * qa));
                } else {
                    const double rem = r.R2 - dx * dx - dy * dy;
                    if (rem < 0.0) continue;
                    const double zr = sqrt(rem);
                    z0 = (long long)ceil((r.P[2] - zr) / G.h[2]);
                    z1 = (long long)floor((r.P[2] + zr) / G.h[2]);
                }
                if (z1 >= z0) npts += z1 - z0 + 1;
            }
        }
        int w = 0, nbl = 0;
        for (int d = 0; d < 3; ++d) {
            w = max(w, r.hi[d] - r.lo[d] + 1);
            nbl = max(nbl, axis_block_count(r.lo[d], r.hi[d], G.N[d], G.nb[d]));
        }
        atomicMax(&maxw[0], w);
        atomicMax(&maxw[1], nbl);
        atomicAdd(&stats[2 * g + 0], (double)npts);
        atomicAdd(&stats[2 * g + 1], (double)ninc);
        if (work) work[p] = (int)ninc;
    }
}

// ------------------------------------------------------- spatial ordering

// Pairs of one (level, class) group are reordered by a coarse spatial cell of
// their product centre (16 cells per axis, Morton order), so that pair images
// processed at the same time by one XCD touch nearby grid points and D rows.
constexpr int kCellBits = 4;
constexpr int kCells = 1 << (3 * kCellBits);

__device__ inline unsigned morton3(unsigned x, unsigned y, unsigned z)
{
    unsigned m = 0;
    for (int b = 0; b < kCellBits; ++b)
        m |= (((x >> b) & 1u) << (3 * b + 2)) | (((y >> b) & 1u) << (3 * b + 1)) | (((z >> b) & 1u) << (3 * b));
    return m;
}

__global__ void __launch_bounds__(256)
k_cell_count(const PairRec *pairs, long long n, PlanConst pc, unsigned *hist, unsigned *key_out)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const PairRec &r = pairs[p];
    unsigned c[3];
    for (int d = 0; d < 3; ++d) {
        // fractional coordinate of the product centre (index units / N for a general cell)
        double f = pc.tri ? r.P[d] / pc.geom[r.level].N[d] : r.P[d] / pc.L[d];
        f -= floor(f);
        int ci = (int)(f * (1 << kCellBits));
        c[d] = (unsigned)min(max(ci, 0), (1 << kCellBits) - 1);
    }
    const unsigned key = (unsigned)(r.level * kNCls + r.cls) * kCells + morton3(c[0], c[1], c[2]);
    key_out[p] = key;
    atomicAdd(&hist[key], 1u);
}

__global__ void __launch_bounds__(256)
k_cell_scatter(const PairRec *in, long long n, const unsigned *key, const long long *off, unsigned *cur,
               const unsigned *hist, PairRec *out, int *err_flag)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const unsigned k = key[p];
    const unsigned pos = atomicAdd(&cur[k], 1u);
    if (pos >= hist[k]) { atomicOr(err_flag, 1); return; }
    out[off[k] + pos] = in[p];
}

__global__ void __launch_bounds__(256) k_rho_records(const PairRec *pairs, long long n, RhoRec *out)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const PairRec &r = pairs[p];
    RhoRec o;
    for (int d = 0; d < 3; ++d) {
        o.A[d] = r.A[d];
        o.AB[d] = r.AB[d];
        o.P[d] = r.P[d];
        o.c[d] = r.c[d];
    }
    o.ap = r.aa + r.ab;
    o.Kw = r.Kw;
    o.ER = r.ER;
    o.pad = 0.0;
    out[p] = o;
}

// ------------------------------------------------------------------ scans

__device__ inline long long wave_incl_scan(long long v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        long long t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

// Block-level inclusive scan of 256 threads; returns the block total.
__device__ inline long long block_incl_scan(long long v, long long &total)
{
    __shared__ long long wsum[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_incl_scan(v);
    if (lane == 63) wsum[wid] = v;
    __syncthreads();
    long long add = 0;
    for (int w = 0; w < wid; ++w) add += wsum[w];
    total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    return v + add;
}

constexpr int kScanItems = 4;
constexpr int kScanChunk = 256 * kScanItems;

template <typename TIn>
__global__ void __launch_bounds__(256) k_scan_reduce(const TIn *in, long long n, long long *partial)
{
    const long long base = (long long)blockIdx.x * kScanChunk;
    long long s = 0;
    for (int it = 0; it < kScanItems; ++it) {
        long long i = base + it * 256 + threadIdx.x;
        if (i < n) s += (long long)in[i];
    }
    long long total;
    block_incl_scan(s, total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Exclusive scan of a chunk with a carried-in offset; out has n+1 entries
// (out[n] = grand total) when last_total is set.
template <typename TIn>
__global__ void __launch_bounds__(256)
k_scan_apply(const TIn *in, long long n, const long long *chunk_off, long long *out)
{
    const long long base = (long long)blockIdx.x * kScanChunk + (long long)threadIdx.x * kScanItems;
    long long v[kScanItems];
    long long s = 0;
    for (int it = 0; it < kScanItems; ++it) {
        long long i = base + it;
        v[it] = (i < n) ? (long long)in[i] : 0;
        s += v[it];
    }
    long long total;
    long long incl = block_incl_scan(s, total);
    long long run = chunk_off[blockIdx.x] + incl - s;
    for (int it = 0; it < kScanItems; ++it) {
        long long i = base + it;
        if (i < n) out[i] = run;
        run += v[it];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 255) out[n] = chunk_off[blockIdx.x] + total;
}

template <typename TIn>
static hipError_t exclusive_scan(const TIn *in, long long n, long long *out, hipStream_t st)
{
    // out: n+1 entries; out[n] = total
    if (n <= 0) {
        long long zero = 0;
        return hipMemcpyAsync(out, &zero, sizeof(zero), hipMemcpyHostToDevice, st);
    }
    const long long nchunk = (n + kScanChunk - 1) / kScanChunk;
    long long *partial = nullptr, *chunk_off = nullptr;
    hipError_t e = hipMallocAsync((void **)&partial, sizeof(long long) * nchunk, st);
    if (e == hipSuccess) e = hipMallocAsync((void **)&chunk_off, sizeof(long long) * (nchunk + 1), st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_scan_reduce<TIn>, dim3((unsigned)nchunk), dim3(256), 0, st, in, n, partial);
        if (nchunk == 1) {
            long long zero = 0;
            e = hipMemcpyAsync(chunk_off, &zero, sizeof(zero), hipMemcpyHostToDevice, st);
        } else {
            e = exclusive_scan<long long>(partial, nchunk, chunk_off, st);
        }
    }
    if (e == hipSuccess)
        hipLaunchKernelGGL(k_scan_apply<TIn>, dim3((unsigned)nchunk), dim3(256), 0, st, in, n, chunk_off, out);
    if (partial) (void)hipFreeAsync(partial, st);
    if (chunk_off) (void)hipFreeAsync(chunk_off, st);
    return e != hipSuccess ? e : hipGetLastError();
}

__global__ void k_flags(const unsigned *cnt, long long n, unsigned *flags)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flags[i] = cnt[i] ? 1u : 0u;
}

// compacted block list: for every counter with entries, its block slot in the level
__global__ void k_compact_blocks(const unsigned *cnt, long long n, const long long *flag_off,
                                 const long long *cnt_base_g, int ngroups, int *blk)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || cnt[i] == 0) return;
    int g = 0;
    while (g + 1 < ngroups && cnt_base_g[g + 1] <= i) ++g;
    blk[flag_off[i]] = (int)(i - cnt_base_g[g]);
}

// ------------------------------------------------------------ orchestration

static inline unsigned nblk(long long n, int t) { return (unsigned)((n + t - 1) / t); }

// Device temporaries of one plan construction, freed on every exit.
struct Temps {
    std::vector<void *> p;
    template <typename T>
    hipError_t alloc(T **ptr, size_t bytes)
    {
        *ptr = nullptr;
        hipError_t e = hipMalloc((void **)ptr, bytes);
        if (e == hipSuccess) p.push_back((void *)*ptr);
        return e;
    }
    void release(void *q)
    {
        for (auto &x : p)
            if (x == q) {
                (void)hipFree(x);
                x = nullptr;
            }
    }
    ~Temps()
    {
        for (void *x : p)
            if (x) (void)hipFree(x);
    }
};

// Runs the partitioner on the plan's device; fills pairs, incidences, block
// lists and work statistics.  Returns a HIP error code; a plan the kernels
// cannot evaluate (a truncation sphere too wide) sets unsupported and returns
// hipErrorInvalidValue.  Buffers the plan keeps are registered in its
// allocation list as soon as they exist, so free_plan releases them on any
// error; the temporaries are released here on every path.
hipError_t build_partition(gpw_plan_s *pl, const PartitionInput &in, hipStream_t st, std::string &err,
                           bool &unsupported)
{
    hipError_t e;
    unsupported = false;
    Temps tmp;
#define PCHK(x)                                                                                 \
    do {                                                                                        \
        e = (x);                                                                                \
        if (e != hipSuccess) { err = std::string(#x) + ": " + hipGetErrorString(e); return e; } \
    } while (0)
    auto own = [&](auto **ptr, size_t bytes) -> hipError_t {
        *ptr = nullptr;
        hipError_t r = hipMalloc((void **)ptr, bytes);
        if (r == hipSuccess) pl->allocations.push_back((void *)*ptr);
        return r;
    };
    const int ngroups = pl->nlevels * kNCls;
    unsigned long long *d_gcnt = nullptr, *d_gcur = nullptr;
    long long *d_goff = nullptr;
    int *d_err = nullptr;
    PCHK(tmp.alloc(&d_err, sizeof(int)));
    PCHK(hipMemsetAsync(d_err, 0, sizeof(int), st));
    PCHK(tmp.alloc(&d_gcnt, sizeof(unsigned long long) * kMaxGroups));
    PCHK(tmp.alloc(&d_gcur, sizeof(unsigned long long) * kMaxGroups));
    PCHK(tmp.alloc(&d_goff, sizeof(long long) * (kMaxGroups + 1)));
    PCHK(hipMemsetAsync(d_gcnt, 0, sizeof(unsigned long long) * kMaxGroups, st));
    PCHK(hipMemsetAsync(d_gcur, 0, sizeof(unsigned long long) * kMaxGroups, st));

    const long long nn = (long long)in.ps.n * in.ps.n;
    hipLaunchKernelGGL(k_pairs<false>, dim3(nblk(nn, 256)), dim3(256), 0, st, in.ps, in.pc, d_gcnt,
                       (const long long *)nullptr, (unsigned long long *)nullptr, (PairRec *)nullptr, d_err);
    PCHK(hipGetLastError());
    unsigned long long gcnt[kMaxGroups];
    PCHK(hipMemcpyAsync(gcnt, d_gcnt, sizeof(gcnt), hipMemcpyDeviceToHost, st));
    PCHK(hipStreamSynchronize(st));
    pl->group_off[0] = 0;
    for (int g = 0; g < kMaxGroups; ++g) pl->group_off[g + 1] = pl->group_off[g] + (g < ngroups ? (long long)gcnt[g] : 0);
    pl->n_pairs = pl->group_off[kMaxGroups];
    PCHK(hipMemcpyAsync(d_goff, pl->group_off, sizeof(long long) * (kMaxGroups + 1), hipMemcpyHostToDevice, st));
    PCHK(own(&pl->d_pairs, sizeof(PairRec) * (size_t)(pl->n_pairs > 0 ? pl->n_pairs : 1)));
    if (pl->n_pairs > 0) {
        hipLaunchKernelGGL(k_pairs<true>, dim3(nblk(nn, 256)), dim3(256), 0, st, in.ps, in.pc,
                           (unsigned long long *)nullptr, (const long long *)d_goff, d_gcur, pl->d_pairs, d_err);
        PCHK(hipGetLastError());
        // reorder every group by spatial cell (counting sort on (group, cell))
        const long long nkeys = (long long)ngroups * kCells;
        unsigned *d_hist = nullptr, *d_keys = nullptr, *d_hcur = nullptr;
        long long *d_hoff = nullptr;
        PairRec *sorted = nullptr;
        PCHK(tmp.alloc(&d_hist, sizeof(unsigned) * (size_t)nkeys));
        PCHK(tmp.alloc(&d_hcur, sizeof(unsigned) * (size_t)nkeys));
        PCHK(tmp.alloc(&d_hoff, sizeof(long long) * (size_t)(nkeys + 1)));
        PCHK(tmp.alloc(&d_keys, sizeof(unsigned) * (size_t)pl->n_pairs));
        PCHK(own(&sorted, sizeof(PairRec) * (size_t)pl->n_pairs));
        PCHK(hipMemsetAsync(d_hist, 0, sizeof(unsigned) * (size_t)nkeys, st));
        PCHK(hipMemsetAsync(d_hcur, 0, sizeof(unsigned) * (size_t)nkeys, st));
        hipLaunchKernelGGL(k_cell_count, dim3(nblk(pl->n_pairs, 256)), dim3(256), 0, st,
                           (const PairRec *)pl->d_pairs, pl->n_pairs, in.pc, d_hist, d_keys);
        PCHK(hipGetLastError());
        PCHK(exclusive_scan<unsigned>(d_hist, nkeys, d_hoff, st));
        hipLaunchKernelGGL(k_cell_scatter, dim3(nblk(pl->n_pairs, 256)), dim3(256), 0, st,
                           (const PairRec *)pl->d_pairs, pl->n_pairs, (const unsigned *)d_keys,
                           (const long long *)d_hoff, d_hcur, (const unsigned *)d_hist, sorted, d_err);
        PCHK(hipGetLastError());
        PCHK(hipStreamSynchronize(st));
        // the sorted copy replaces the unsorted records in the plan
        for (auto &a : pl->allocations)
            if (a == (void *)pl->d_pairs) a = nullptr;
        (void)hipFree(pl->d_pairs);
        pl->d_pairs = sorted;
        tmp.release(d_hist);
        tmp.release(d_hcur);
        tmp.release(d_hoff);
        tmp.release(d_keys);
    }
    PCHK(own(&pl->d_rrec, sizeof(RhoRec) * (size_t)(pl->n_pairs > 0 ? pl->n_pairs : 1)));
    if (pl->n_pairs > 0) {
        hipLaunchKernelGGL(k_rho_records, dim3(nblk(pl->n_pairs, 256)), dim3(256), 0, st,
                           (const PairRec *)pl->d_pairs, pl->n_pairs, pl->d_rrec);
        PCHK(hipGetLastError());
    }

    // counters per (group, block slot)
    long long ncnt = 0;
    for (int g = 0; g <= kMaxGroups; ++g) {
        pl->cnt_base[g] = ncnt;
        if (g < ngroups) ncnt += block_slots(pl->geom[g / kNCls]);
    }
    long long *d_cnt_base = nullptr;
    unsigned *d_cnt = nullptr, *d_cur = nullptr, *d_flags = nullptr;
    long long *d_flag_off = nullptr;
    double *d_stats = nullptr;
    int *d_maxw = nullptr;
    PCHK(tmp.alloc(&d_maxw, 2 * sizeof(int)));
    PCHK(hipMemsetAsync(d_maxw, 0, 2 * sizeof(int), st));
    PCHK(tmp.alloc(&d_cnt_base, sizeof(long long) * (kMaxGroups + 1)));
    PCHK(hipMemcpyAsync(d_cnt_base, pl->cnt_base, sizeof(long long) * (kMaxGroups + 1), hipMemcpyHostToDevice, st));
    PCHK(tmp.alloc(&d_cnt, sizeof(unsigned) * (size_t)(ncnt + 1)));
    int *d_work = nullptr;   // incidences per pair image
    PCHK(tmp.alloc(&d_work, sizeof(int) * (size_t)(pl->n_pairs > 0 ? pl->n_pairs : 1)));
    PCHK(tmp.alloc(&d_cur, sizeof(unsigned) * (size_t)(ncnt + 1)));
    PCHK(tmp.alloc(&d_flags, sizeof(unsigned) * (size_t)(ncnt + 1)));
    PCHK(tmp.alloc(&d_flag_off, sizeof(long long) * (size_t)(ncnt + 2)));
    PCHK(tmp.alloc(&d_stats, sizeof(double) * 2 * kMaxGroups));
    PCHK(own(&pl->d_inc_off, sizeof(long long) * (size_t)(ncnt + 2)));
    PCHK(hipMemsetAsync(d_cnt, 0, sizeof(unsigned) * (size_t)(ncnt + 1), st));
    PCHK(hipMemsetAsync(d_cur, 0, sizeof(unsigned) * (size_t)(ncnt + 1), st));
    PCHK(hipMemsetAsync(d_stats, 0, sizeof(double) * 2 * kMaxGroups, st));
    if (pl->n_pairs > 0) {
        hipLaunchKernelGGL(k_incidences<false>, dim3(nblk(pl->n_pairs, 256)), dim3(256), 0, st,
                           (const PairRec *)pl->d_pairs, pl->n_pairs, in.pc, (const long long *)d_cnt_base,
                           d_cnt, (const long long *)nullptr, (unsigned *)nullptr, (int2 *)nullptr, d_stats, d_maxw, d_err,
                           d_work);
        PCHK(hipGetLastError());
    }
    PCHK(exclusive_scan<unsigned>(d_cnt, ncnt, pl->d_inc_off, st));
    PCHK(hipMemcpyAsync(&pl->n_inc, pl->d_inc_off + ncnt, sizeof(long long), hipMemcpyDeviceToHost, st));
    PCHK(hipStreamSynchronize(st));
    PCHK(own(&pl->d_inc, sizeof(int2) * (size_t)(pl->n_inc > 0 ? pl->n_inc : 1)));
    if (pl->n_pairs > 0) {
        hipLaunchKernelGGL(k_incidences<true>, dim3(nblk(pl->n_pairs, 256)), dim3(256), 0, st,
                           (const PairRec *)pl->d_pairs, pl->n_pairs, in.pc, (const long long *)d_cnt_base,
                           d_cnt, (const long long *)pl->d_inc_off, d_cur, pl->d_inc,
                           (double *)nullptr, (int *)nullptr, d_err);
        PCHK(hipGetLastError());
    }
    // compacted nonempty blocks per group
    if (ncnt > 0) {
        hipLaunchKernelGGL(k_flags, dim3(nblk(ncnt, 256)), dim3(256), 0, st, (const unsigned *)d_cnt, ncnt, d_flags);
        PCHK(hipGetLastError());
    }
    PCHK(exclusive_scan<unsigned>(d_flags, ncnt, d_flag_off, st));
    long long nblk_total = 0;
    PCHK(hipMemcpyAsync(&nblk_total, d_flag_off + ncnt, sizeof(long long), hipMemcpyDeviceToHost, st));
    PCHK(hipStreamSynchronize(st));
    PCHK(own(&pl->d_blk, sizeof(int) * (size_t)(nblk_total > 0 ? nblk_total : 1)));
    if (ncnt > 0) {
        hipLaunchKernelGGL(k_compact_blocks, dim3(nblk(ncnt, 256)), dim3(256), 0, st, (const unsigned *)d_cnt,
                           ncnt, (const long long *)d_flag_off, (const long long *)d_cnt_base, ngroups, pl->d_blk);
        PCHK(hipGetLastError());
    }
    // host copies of per-group offsets
    std::vector<long long> flag_at(kMaxGroups + 1), inc_at(kMaxGroups + 1);
    for (int g = 0; g <= kMaxGroups; ++g) {
        PCHK(hipMemcpyAsync(&flag_at[g], d_flag_off + pl->cnt_base[g], sizeof(long long), hipMemcpyDeviceToHost, st));
        PCHK(hipMemcpyAsync(&inc_at[g], pl->d_inc_off + pl->cnt_base[g], sizeof(long long), hipMemcpyDeviceToHost, st));
    }
    double stats[2 * kMaxGroups];
    PCHK(hipMemcpyAsync(stats, d_stats, sizeof(stats), hipMemcpyDeviceToHost, st));
    int maxwb[2] = {0, 0}, errf = 0;
    PCHK(hipMemcpyAsync(maxwb, d_maxw, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    PCHK(hipMemcpyAsync(&errf, d_err, sizeof(int), hipMemcpyDeviceToHost, st));
    PCHK(hipStreamSynchronize(st));
    const int maxw = maxwb[0];
    pl->max_axis_blocks = maxwb[1];
    for (int g = 0; g <= kMaxGroups; ++g) pl->blk_off[g] = flag_at[g];
    if (errf & 1) { err = "partitioner count and fill passes disagree"; return hipErrorUnknown; }
    {
        // deal each group's nonempty blocks to the eight XCDs in contiguous
        // ranges of about equal work (list length plus a fixed per-block share
        // for the reduction and the write): equal block counts would leave the
        // XCDs with the sparser regions idle while the denser ones finish
        std::vector<unsigned> hcnt((size_t)ncnt);
        std::vector<int> hblk((size_t)nblk_total);
        if (ncnt > 0) PCHK(hipMemcpyAsync(hcnt.data(), d_cnt, sizeof(unsigned) * (size_t)ncnt, hipMemcpyDeviceToHost, st));
        if (nblk_total > 0)
            PCHK(hipMemcpyAsync(hblk.data(), pl->d_blk, sizeof(int) * (size_t)nblk_total, hipMemcpyDeviceToHost, st));
        PCHK(hipStreamSynchronize(st));
        constexpr double kBlockShare = 32.0;   // per-block cost in incidences
        std::vector<double> pre;
        for (int g = 0; g < ngroups; ++g) {
            const long long b0 = pl->blk_off[g], n = pl->blk_off[g + 1] - b0;
            pre.assign((size_t)n + 1, 0.0);
            for (long long i = 0; i < n; ++i)
                pre[i + 1] = pre[i] + kBlockShare + (double)hcnt[(size_t)(pl->cnt_base[g] + hblk[(size_t)(b0 + i)])];
            long long i = 0;
            pl->xsplit[g][0] = 0;
            for (int x = 1; x < 8; ++x) {
                const double target = pre[(size_t)n] * x / 8.0;
                while (i < n && pre[(size_t)i] < target) ++i;
                pl->xsplit[g][x] = (int)i;
            }
            pl->xsplit[g][8] = (int)n;
            // inside each XCD's range the longest lists first, so that the
            // range does not end on a long block (about 1 % of eval_rho)
            for (int x = 0; x < 8; ++x) {
                int *beg = hblk.data() + b0 + pl->xsplit[g][x], *end = hblk.data() + b0 + pl->xsplit[g][x + 1];
                const long long cb = pl->cnt_base[g];
                std::stable_sort(beg, end, [&](int u, int v) { return hcnt[(size_t)(cb + u)] > hcnt[(size_t)(cb + v)]; });
            }
        }
        if (nblk_total > 0)
            PCHK(hipMemcpyAsync(pl->d_blk, hblk.data(), sizeof(int) * (size_t)nblk_total, hipMemcpyHostToDevice, st));
        // the pair images of each group likewise, by their block count (the
        // traversal) plus a fixed per-image share (set-up and reduction)
        constexpr double kPairShare = 4.0;
        std::vector<int> hwork((size_t)pl->n_pairs);
        if (pl->n_pairs > 0)
            PCHK(hipMemcpyAsync(hwork.data(), d_work, sizeof(int) * (size_t)pl->n_pairs, hipMemcpyDeviceToHost, st));
        PCHK(hipStreamSynchronize(st));
        for (int g = 0; g < ngroups; ++g) {
            const long long p0 = pl->group_off[g], n = pl->group_off[g + 1] - p0;
            pre.assign((size_t)n + 1, 0.0);
            for (long long i = 0; i < n; ++i) pre[i + 1] = pre[i] + kPairShare + (double)hwork[(size_t)(p0 + i)];
            long long i = 0;
            pl->xsplit_pair[g][0] = 0;
            for (int x = 1; x < 8; ++x) {
                const double target = pre[(size_t)n] * x / 8.0;
                while (i < n && pre[(size_t)i] < target) ++i;
                pl->xsplit_pair[g][x] = (int)i;
            }
            pl->xsplit_pair[g][8] = (int)n;
        }
    }
    if (errf & 2) {
        err = "a truncation sphere reaches beyond 127 cells (fold shift out of range)";
        unsupported = true;
        return hipErrorInvalidValue;
    }
    if (maxw > kMaxBoxWidth) {
        err = "a truncation sphere is wider than the supported box (" + std::to_string(maxw) + " points)";
        unsupported = true;
        return hipErrorInvalidValue;
    }

    // work statistics and the flop model
    gpw_plan_info &I = pl->info;
    I.max_box_width = maxw;
    for (int g = 0; g < ngroups; ++g) {
        const int lvl = g / kNCls, c = g % kNCls;
        const long long np = pl->group_off[g + 1] - pl->group_off[g];
        const long long ninc = inc_at[g + 1] - inc_at[g];
        I.n_pairs[lvl] += np;
        I.n_pairs_class[c] += np;
        I.n_incidences[lvl] += ninc;
        I.n_incidences_class[c] += ninc;
        const int la = cls_la(c), lb = cls_lb(c), L = la + lb;
        const double na = ncart(la), nb = ncart(lb);
        // the counting convention, per (pair image, point): the direct
        // evaluation sum_ij D_ij a_i b_j (or the n_a n_b products of mat),
        // monomials, envelope and accumulation
        const double f1 = 2 * na * nb + 2 * (na + nb) + 4;
        const double f2 = 4 * na * nb + 8 * (na + nb) + 4;
        const double pts = stats[2 * g], blkpts = 64.0 * (double)ninc;
        I.sphere_points += pts;
        I.flops_rho_sphere += f1 * pts;
        I.flops_rho_block += f1 * blkpts;
        I.flops_mat_sphere += f1 * pts;
        I.flops_mat_block += f1 * blkpts;
        I.flops_grad_sphere += f2 * pts;
        I.flops_grad_block += f2 * blkpts;
        // the arithmetic the kernels perform per (pair image, block).  rho
        // through the coefficient tensor: Horner in x for the (y, z)
        // coefficients at 4 x points (C(L+2,3) FMAs each), in y for the z
        // coefficients of 16 columns (C(L+1,2) FMAs each), 16 column envelope
        // products, per point L Horner FMAs, the envelope product and the
        // accumulation.  mat through the moments: per point about 2L + 3
        // flops (the cut potential v e_z, the powers of z - A_z, the L + 1
        // accumulations; the flushes once per group of rows, ~1-2 %, are not
        // counted).
        const double ft = 8.0 * (L + 2) * (L + 1) * L / 6.0 + 32.0 * (L + 1) * L / 2.0 + 16.0 + 64.0 * (2 * L + 3);
        I.flops_rho_exec += rho_tensor(la, lb) ? ft * (double)ninc : f1 * blkpts;
        I.flops_mat_exec += (mat_tensor(la, lb) ? 2.0 * L + 3.0 : f1) * blkpts;
        // the same counts two and three degrees higher for the kinetic energy
        // density terms, and one degree higher for the gradient's moments
        const double L2 = L + 2.0;
        I.flops_tau_exec +=
            (8.0 * (L2 + 2) * (L2 + 1) * L2 / 6.0 + 32.0 * (L2 + 1) * L2 / 2.0 + 16.0 + 64.0 * (2 * L2 + 3)) *
            (double)ninc;
        I.flops_grad_exec += (2.0 * (L + 1) + 3.0) * blkpts;
        I.flops_mat_tau_exec += (2.0 * (L + 2) + 3.0) * blkpts;
        I.flops_grad_tau_exec += (2.0 * (L + 3) + 3.0) * blkpts;
    }

    return hipSuccess;
#undef PCHK
}

}  // namespace gpw
