// Host side of the evaluations: per-task scratch layout, the element-wise
// helper kernels (zero fills, symmetrised D, block-ordered potential copies),
// the batching of tasks into per-(operation, class) launches, and the
// allocation-free entry point's scratch.  The class kernels themselves are in
// gpw_kernels.h and are launched from gpw_class.hip.
//
// Launches: a kernel launch covers one (operation, class) for any number of
// (task, level) segments, described by a table passed by value; a work item
// (grid block or pair image) finds its segment from the table.  A single
// evaluation is a batch of one task, so batched and single calls run the
// same kernels in the same order.
#include "gpw_kernels.h"

#include <mutex>

namespace gpw {

// --------------------------------------------------------- small kernels

// out = (D + D^T) / 2 through 32x32 LDS tiles (both reads coalesced).
template <typename T>
__global__ void __launch_bounds__(256) k_symmetrize(SegTable<SymSeg> tab)
{
    __shared__ double tile[32][33];
    const SymSeg &sg = tab.s[seg_of(tab, blockIdx.x)];
    const double *__restrict__ D = sg.D;
    T *__restrict__ out = (T *)sg.out;
    const int n = sg.n;
    const int it = (int)(blockIdx.x - sg.item0);
    const int bx = (it / sg.nt) * 32, by = (it % sg.nt) * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int j = ty; j < 32; j += 8) {
        const int r = bx + j, c = by + tx;
        tile[j][tx] = (r < n && c < n) ? D[(long long)r * n + c] : 0.0;
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int r = by + j, c = bx + tx;
        if (r < n && c < n) out[(long long)r * n + c] = (T)(0.5 * (D[(long long)r * n + c] + tile[tx][j]));
    }
}

__global__ void __launch_bounds__(256) k_fill(SegTable<FillSeg> tab)
{
    const FillSeg &sg = tab.s[seg_of(tab, blockIdx.x)];
    const long long i = (long long)(blockIdx.x - sg.item0) * 256 + threadIdx.x;
    if (i < sg.count) sg.p[i] = 0.0;
}

// Copy of a level grid in 4x4x4-block order (block b = (kx nb1 + ky) vz + kz,
// then the 64 points as four z planes of 16 points, y fastest), zero at the
// padding points of partial blocks, so that one plane of a block is one
// 128-byte line and the planes of a run of blocks along z are consecutive.
// Each (x, y) column holds vz >= nb2 blocks: past its nb2 blocks it repeats
// the column periodically, so that a run of up to vz - nb2 + 1 blocks along z
// that starts in the cell is contiguous in memory.
__global__ void __launch_bounds__(256) k_block_grid(SegTable<GridSeg> tab)
{
    const GridSeg &sg = tab.s[seg_of(tab, blockIdx.x)];
    const long long i = (long long)(blockIdx.x - sg.item0) * 256 + threadIdx.x;
    if (i >= sg.count) return;
    const LevelGeom &G = sg.G;
    const double *__restrict__ v = sg.v;
    double *__restrict__ vb = sg.vb;
    const long long b = i >> 6;
    const int t = (int)(i & 63);
    const int kz = (int)(b % sg.vz) % G.nb[2];
    const int ky = (int)((b / sg.vz) % G.nb[1]);
    const int kx = (int)(b / ((long long)sg.vz * G.nb[1]));
    const int wx = 4 * kx + ((t >> 2) & 3), wy = 4 * ky + (t & 3), wz = 4 * kz + (t >> 4);
    vb[i] = (wx < G.N[0] && wy < G.N[1] && wz < G.N[2]) ? v[((long long)wx * G.N[1] + wy) * G.N[2] + wz] : 0.0;
}


static inline long long nb256(long long n) { return (n + 255) / 256; }


static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Blocks per (x, y) column of a level's block copy: the level's nb2 plus
// enough periodic repeats that a z run of the plan's longest block list
// starting anywhere in the cell stays inside the column.
static int block_column(const gpw_plan_s *pl, int l)
{
    return pl->geom[l].nb[2] + std::max(1, pl->max_axis_blocks) - 1;
}
static long long block_copy_blocks(const gpw_plan_s *pl, int l)
{
    return (long long)pl->geom[l].nb[0] * pl->geom[l].nb[1] * block_column(pl, l);
}

// Scratch of one task inside the batch's stream-ordered allocation.
struct TaskScratch {
    size_t dpk = 0, ds = 0, vb = 0;      // byte offsets
    size_t tmp = 0;                      // general cells: Cartesian coefficient tensors (FP64)
    long long dbase[kMaxGroups + 1];     // packed-D offsets of the groups (elements)
    long long tbase[kMaxGroups + 1];     // their offsets in tmp (doubles)
    long long voff[kMaxLevels];          // block-grid offsets of the levels (doubles)
};

// Operations that collocate onto the level grids (packed coefficients per
// pair image), and those that read level potentials (block-ordered copies).
static bool grid_op(int op) { return op == GPW_OP_RHO || op == GPW_OP_TAU; }
static bool sym_op(int op) { return op == GPW_OP_GRAD || op == GPW_OP_GRAD_TAU; }
static int extra_degree(int op) { return op == GPW_OP_TAU ? 2 : 0; }

// Layout of one task's scratch (byte offsets from base) and its size.
template <typename T>
static size_t task_scratch(const gpw_plan_s *pl, int op, size_t base, TaskScratch &x)
{
    size_t bytes = base;
    if (grid_op(op)) {
        const bool tri = pl->tri != 0;
        x.dbase[0] = 0;
        x.tbase[0] = 0;
        for (int g = 0; g < kMaxGroups; ++g) {
            const int c = g % kNCls;
            const long long np = pl->group_off[g + 1] - pl->group_off[g];
            const int K = grid_ncoef(cls_la(c), cls_lb(c), extra_degree(op), tri);
            x.dbase[g + 1] = x.dbase[g] + np * cstride<T>(K);
            x.tbase[g + 1] = x.tbase[g] + (tri ? np * K : 0);
        }
        x.dpk = bytes;
        bytes += align256(sizeof(T) * (size_t)x.dbase[kMaxGroups]);
        if (tri) {
            x.tmp = bytes;
            bytes += align256(sizeof(double) * (size_t)x.tbase[kMaxGroups]);
        }
    } else {
        long long tot = 0;
        for (int l = 0; l < pl->nlevels; ++l) {
            x.voff[l] = tot;
            tot += block_copy_blocks(pl, l) * 64;
        }
        x.vb = bytes;
        bytes += align256(sizeof(double) * (size_t)(tot + 64 * kBlockCopyTail));
        if (sym_op(op)) {
            x.ds = bytes;
            bytes += align256(sizeof(T) * (size_t)pl->n_ao * pl->n_ao);
        }
    }
    return bytes - base;
}

size_t eval_scratch_bytes(const gpw_plan_s *pl, int op)
{
    TaskScratch x;
    return pl->precision == GPW_FP32 ? task_scratch<float>(pl, op, 0, x) : task_scratch<double>(pl, op, 0, x);
}

// One batch of tasks of one precision.  Scratch: a stream-ordered allocation
// of the batch's size, or, when ext is given, the caller's ext_cap bytes at
// ext (then nothing is allocated or freed).
template <typename T>
static hipError_t batch_t(const TaskRef *tasks, int n, hipStream_t st, unsigned char *ext = nullptr,
                          size_t ext_cap = 0)
{
    SmallVec<TaskScratch, 1> ts;
    ts.resize((size_t)n);
    size_t bytes = 0;
    int emax_all = 1;
    for (int i = 0; i < n; ++i) {
        bytes += task_scratch<T>(tasks[i].pl, tasks[i].op, bytes, ts[i]);
        if (!grid_op(tasks[i].op)) emax_all = std::max(emax_all, tasks[i].pl->max_axis_blocks);
    }
    unsigned char *scr = ext;
    hipError_t e = hipSuccess;
    if (ext) {
        if (bytes > ext_cap) return hipErrorInvalidValue;
    } else {
        e = hipMallocAsync((void **)&scr, bytes > 0 ? bytes : 256, st);
        if (e != hipSuccess) return e;
    }

    // outputs to zero, symmetrised D of gradient tasks, block-ordered potentials
    SegList<FillSeg> fills;
    SegList<SymSeg> syms;
    SegList<GridSeg> grids;
    for (int i = 0; i < n; ++i) {
        const TaskRef &t = tasks[i];
        const gpw_plan_s *pl = t.pl;
        if (grid_op(t.op)) {
            for (int l = 0; l < pl->nlevels; ++l) fills.add({0, t.rho[l], pl->ngrid[l]}, nb256(pl->ngrid[l]));
            continue;
        }
        const long long cnt =
            (t.op == GPW_OP_MAT || t.op == GPW_OP_MAT_TAU) ? (long long)pl->n_ao * pl->n_ao : 3LL * pl->natm;
        fills.add({0, t.out, cnt}, nb256(cnt));
        for (int l = 0; l < pl->nlevels; ++l) {
            const long long m = block_copy_blocks(pl, l) * 64;
            grids.add({0, t.v[l], (double *)(scr + ts[i].vb) + ts[i].voff[l], m, block_column(pl, l), pl->geom[l]},
                      nb256(m));
        }
        if (sym_op(t.op) && pl->n_ao > 0) {
            const int nt = (pl->n_ao + 31) / 32;
            syms.add({0, t.D, scr + ts[i].ds, pl->n_ao, nt}, (long long)nt * nt);
        }
    }
    fills.launch([&](const SegTable<FillSeg> &tb, unsigned g) {
        hipLaunchKernelGGL(k_fill, dim3(g), dim3(256), 0, st, tb);
    }, false);
    syms.launch([&](const SegTable<SymSeg> &tb, unsigned g) {
        hipLaunchKernelGGL(k_symmetrize<T>, dim3(g), dim3(256), 0, st, tb);
    }, false);
    grids.launch([&](const SegTable<GridSeg> &tb, unsigned g) {
        hipLaunchKernelGGL(k_block_grid, dim3(g), dim3(256), 0, st, tb);
    }, false);

    for (int c = 0; c < kNCls; ++c) {
        ClassLaunch cl;
        for (int i = 0; i < n; ++i) {
            const TaskRef &t = tasks[i];
            const gpw_plan_s *pl = t.pl;
            const int emax = std::max(1, pl->max_axis_blocks);
            // collocation: coarse levels first.  Their few blocks carry long pair
            // lists (diffuse pairs); started first, those long waves overlap the
            // many short ones of the fine level instead of forming the launch's
            // tail (eval_rho 6.7 % faster on the 256-water system)
            for (int li = 0; li < pl->nlevels; ++li) {
                const int l = grid_op(t.op) ? pl->nlevels - 1 - li : li;
                const int g = l * kNCls + c;
                const long long np = pl->group_off[g + 1] - pl->group_off[g];
                const PairRec *pairs = (const PairRec *)pl->d_pairs + pl->group_off[g];
                if (grid_op(t.op)) {
                    const bool tau = t.op == GPW_OP_TAU;
                    T *Dpk = (T *)(scr + ts[i].dpk) + ts[i].dbase[g];
                    if (pl->tri) {
                        // Cartesian tensors in FP64, then on the index offset
                        double *tmp = (double *)(scr + ts[i].tmp) + ts[i].tbase[g];
                        const int Lt = cls_la(c) + cls_lb(c) + extra_degree(t.op), K = ntab(Lt);
                        (tau ? cl.tpacks : cl.packs_t)
                            .add({0, pairs, t.D, Dpk, np, pl->n_ao, pl->geom[l].tri, tmp}, nb256(np));
                        cl.idxs.add({0, tmp, Dpk, np * K, Lt, K, cstride<T>(K), pl->geom[l].tri}, nb256(np * K));
                    } else {
                        const long long ne = (tau || rho_tensor(cls_la(c), cls_lb(c)))
                                                 ? np
                                                 : np * ncart(cls_la(c)) * ncart(cls_lb(c));
                        (tau ? cl.tpacks : cl.packs).add({0, pairs, t.D, Dpk, ne, pl->n_ao, nullptr, nullptr},
                                                         nb256(ne));
                    }
                    RhoSeg r;
                    r.item0 = 0;
                    r.count = pl->blk_off[g + 1] - pl->blk_off[g];
                    r.rr = (const RhoRec *)pl->d_rrec + pl->group_off[g];
                    r.inc = (const int2 *)pl->d_inc;
                    r.inc_off = (const long long *)pl->d_inc_off + pl->cnt_base[g];
                    r.blk = (const int *)pl->d_blk + pl->blk_off[g];
                    r.Dpk = Dpk;
                    r.rho = t.rho[l];
                    r.p0 = (int)pl->group_off[g];
                    r.G = pl->geom[l];
                    int chunk = 0;   // the longest XCD range sets the segment's workgroups
                    for (int x = 0; x < 9; ++x) r.xs[x] = pl->xsplit[g][x];
                    for (int x = 0; x < 8; ++x) chunk = std::max(chunk, r.xs[x + 1] - r.xs[x]);
                    if (pl->tri)
                        (tau ? cl.taus_t : cl.rhos_t).add(r, 8LL * chunk);
                    else
                        (tau ? cl.taus : cl.rhos).add(r, 8LL * chunk);
                } else {
                    PairSeg q;
                    q.item0 = 0;
                    q.count = np;
                    q.pairs = pairs;
                    q.Dm = sym_op(t.op) ? (const void *)(scr + ts[i].ds) : nullptr;
                    q.Vb = (const double *)(scr + ts[i].vb) + ts[i].voff[l];
                    q.out = t.out;
                    q.n_ao = pl->n_ao;
                    q.emax = emax;
                    q.row_cap = row_capacity(emax);
                    q.vz = block_column(pl, l);
                    q.G = pl->geom[l];
                    int chunk = 0;   // the longest XCD range sets the segment's workgroups
                    for (int x = 0; x < 9; ++x) q.xs[x] = pl->xsplit_pair[g][x];
                    for (int x = 0; x < 8; ++x) chunk = std::max(chunk, q.xs[x + 1] - q.xs[x]);
                    if (pl->tri)
                        (t.op == GPW_OP_MAT       ? cl.mats_t
                         : t.op == GPW_OP_GRAD    ? cl.grads_t
                         : t.op == GPW_OP_MAT_TAU ? cl.mtaus_t
                                                  : cl.gtaus_t)
                            .add(q, 8LL * chunk);
                    else
                        (t.op == GPW_OP_MAT       ? cl.mats
                         : t.op == GPW_OP_GRAD    ? cl.grads
                         : t.op == GPW_OP_MAT_TAU ? cl.mtaus
                                                  : cl.gtaus)
                            .add(q, 8LL * chunk);
                }
            }
        }
        cl.smem = PairSmem<T>::bytes(emax_all);
        cl.smem_t = PairSmem<T>::bytes(emax_all, true);
        cl.st = st;
        cl.fp32 = std::is_same<T, float>::value;
        launch_class(c, cl);
    }
    e = hipGetLastError();
    if (!ext) (void)hipFreeAsync(scr, st);
    return e;
}

// one launcher per class, each in its own object (gpw_class.hip)
void launch_class_0(const ClassLaunch &);
void launch_class_1(const ClassLaunch &);
void launch_class_2(const ClassLaunch &);
void launch_class_3(const ClassLaunch &);
void launch_class_4(const ClassLaunch &);
void launch_class_5(const ClassLaunch &);
void launch_class_6(const ClassLaunch &);
void launch_class_7(const ClassLaunch &);
void launch_class_8(const ClassLaunch &);
void launch_class_9(const ClassLaunch &);
void launch_class_10(const ClassLaunch &);
void launch_class_11(const ClassLaunch &);
void launch_class_12(const ClassLaunch &);
void launch_class_13(const ClassLaunch &);
void launch_class_14(const ClassLaunch &);

void launch_class(int c, const ClassLaunch &cl)
{
    static void (*const fn[kNCls])(const ClassLaunch &) = {
        launch_class_0,  launch_class_1,  launch_class_2,  launch_class_3,  launch_class_4,
        launch_class_5,  launch_class_6,  launch_class_7,  launch_class_8,  launch_class_9,
        launch_class_10, launch_class_11, launch_class_12, launch_class_13, launch_class_14};
    fn[c](cl);
}

size_t pair_kernel_lds_bytes(int emax, int precision, bool tri)
{
    return precision == GPW_FP32 ? PairSmem<float>::bytes(emax, tri) : PairSmem<double>::bytes(emax, tri);
}

// ------------------------------------------------- evaluation without allocation

// Scratch of the allocation-free entry point: one copy per device, resident
// from the library's first use of the device until the process ends.  Host
// code never names it directly (on the host the name is only a stand-in for
// the symbol): noalloc_scratch() looks up each device's address once, with
// that device current, and every use goes through that address.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(int dev, unsigned char **ptr)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev) return hipErrorInvalidDevice;   // the caller makes dev current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (unsigned char *)p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t eval_noalloc(const TaskRef &t, hipStream_t st)
{
    unsigned char *scr = nullptr;
    hipError_t e = noalloc_scratch(t.pl->device, &scr);
    if (e != hipSuccess) return e;
    return t.pl->precision == GPW_FP32 ? batch_t<float>(&t, 1, st, scr, kNoAllocScratchBytes)
                                       : batch_t<double>(&t, 1, st, scr, kNoAllocScratchBytes);
}

hipError_t eval_batch(const TaskRef *tasks, int n, hipStream_t st)
{
    std::vector<TaskRef> t64, t32;
    for (int i = 0; i < n; ++i) (tasks[i].pl->precision == GPW_FP32 ? t32 : t64).push_back(tasks[i]);
    hipError_t e = hipSuccess;
    if (!t64.empty()) e = batch_t<double>(t64.data(), (int)t64.size(), st);
    if (e == hipSuccess && !t32.empty()) e = batch_t<float>(t32.data(), (int)t32.size(), st);
    return e;
}

}  // namespace gpw
