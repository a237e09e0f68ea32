// C ABI of libgpw: argument checking, plan construction and the eval entry
// points.  See include/gpw.h for the contract of every call.
#include <cmath>
#include <cstring>
#include <new>

#include "gpw_internal.h"

namespace gpw {
hipError_t build_partition(gpw_plan_s *pl, const PartitionInput &in, hipStream_t st, std::string &err,
                           bool &unsupported);
}  // namespace gpw

using namespace gpw;

namespace {

thread_local std::string g_err;

gpw_status fail(gpw_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

gpw_status hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? GPW_ENOMEM : GPW_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

bool smooth235(long n)
{
    if (n < 1) return false;
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

// RAII guard that makes the plan's device current and restores the caller's.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev)
    {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Inverse and determinant of a 3 x 3 matrix.
double inverse3(const double a[3][3], double inv[3][3])
{
    const double det = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
                       a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
                       a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const int i1 = (j + 1) % 3, i2 = (j + 2) % 3, j1 = (i + 1) % 3, j2 = (i + 2) % 3;
            inv[i][j] = (a[i1][j1] * a[i2][j2] - a[i1][j2] * a[i2][j1]) / det;
        }
    return det;
}

// Smallest eigenvalue of a symmetric positive definite 3 x 3 matrix (cyclic
// Jacobi rotations).
double min_eigenvalue(const double m[3][3])
{
    double a[3][3];
    std::memcpy(a, m, sizeof(a));
    for (int sweep = 0; sweep < 60; ++sweep) {
        const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
        if (off < 1e-30 * (a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2])) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (a[p][q] == 0.0) continue;
                const double th = 0.5 * std::atan2(2.0 * a[p][q], a[q][q] - a[p][p]);
                const double c = std::cos(th), s = std::sin(th);
                for (int k = 0; k < 3; ++k) {   // columns
                    const double akp = a[k][p], akq = a[k][q];
                    a[k][p] = c * akp - s * akq;
                    a[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {   // rows
                    const double apk = a[p][k], aqk = a[q][k];
                    a[p][k] = c * apk - s * aqk;
                    a[q][k] = s * apk + c * aqk;
                }
            }
    }
    return std::min(a[0][0], std::min(a[1][1], a[2][2]));
}

// T_n of a level: the coefficients of (r - A)^m, r - A = s H, as a polynomial
// in the index offset s (ncart(n) x ncart(n), row m, column k, both in shell
// order), by multiplying out one linear factor (s H)_c at a time.
void monomial_transform(const double H[3][3], int n, double *T)
{
    const int nc = ncart(n);
    auto idx = [](int ly, int lz) { return (ly + lz) * (ly + lz + 1) / 2 + lz; };
    int m = 0;
    for (int mx = n; mx >= 0; --mx)
        for (int my = n - mx; my >= 0; --my, ++m) {
            const int me[3] = {mx, my, n - mx - my};
            std::vector<double> poly(1, 1.0), next;
            int deg = 0;
            for (int c = 0; c < 3; ++c)
                for (int rep = 0; rep < me[c]; ++rep) {
                    next.assign(ncart(deg + 1), 0.0);
                    int k = 0;
                    for (int kx = deg; kx >= 0; --kx)
                        for (int ky = deg - kx; ky >= 0; --ky, ++k) {
                            const int kz = deg - kx - ky;
                            next[idx(ky, kz)] += poly[k] * H[0][c];       // s_x h_x,c
                            next[idx(ky + 1, kz)] += poly[k] * H[1][c];   // s_y h_y,c
                            next[idx(ky, kz + 1)] += poly[k] * H[2][c];   // s_z h_z,c
                        }
                    poly.swap(next);
                    ++deg;
                }
            for (int k = 0; k < nc; ++k) T[(size_t)m * nc + k] = poly[k];
        }
}

void free_plan(gpw_plan_s *pl)
{
    if (!pl) return;
    gpw::poisson_free(pl);
    for (void *p : pl->allocations)
        if (p) (void)hipFree(p);
    delete pl;
}

}  // namespace

extern "C" {

const char *gpw_last_error(void) { return g_err.c_str(); }

gpw_status gpw_plan(const gpw_cell *cell, const gpw_basis *basis, const gpw_cutoffs *cut, gpw_plan_t *out)
{
    if (!out) return fail(GPW_EINVAL, "gpw_plan: out is NULL");
    *out = nullptr;
    if (!cell || !basis || !cut) return fail(GPW_EINVAL, "gpw_plan: NULL cell, basis or cutoffs");
    // ---- cell: a diagonal matrix is orthorhombic, anything else a general cell
    double L[3], Alat[3][3], Ainv[3][3];
    int tri = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double a = cell->a[i][j];
            if (!std::isfinite(a)) return fail(GPW_EINVAL, "gpw_plan: non-finite lattice vector");
            Alat[i][j] = a;
            if (i != j && a != 0.0) tri = 1;
        }
    for (int d = 0; d < 3; ++d) {
        L[d] = std::sqrt(Alat[d][0] * Alat[d][0] + Alat[d][1] * Alat[d][1] + Alat[d][2] * Alat[d][2]);
        if (!tri && !(Alat[d][d] > 0.0)) return fail(GPW_EINVAL, "gpw_plan: lattice lengths must be positive");
    }
    const double det = inverse3(Alat, Ainv);
    if (!(std::fabs(det) > 1e-6 * L[0] * L[1] * L[2]))
        return fail(GPW_EINVAL, "gpw_plan: lattice vectors are (nearly) linearly dependent");
    // ---- basis
    const gpw_basis &B = *basis;
    if (B.natm < 1 || B.nshell < 1) return fail(GPW_EINVAL, "gpw_plan: need at least one atom and one shell");
    if (!B.coords || !B.shell_atom || !B.shell_l || !B.shell_nprim || !B.shell_prim0 || !B.exps || !B.coefs)
        return fail(GPW_EINVAL, "gpw_plan: NULL basis array");
    for (int a = 0; a < B.natm; ++a)
        for (int d = 0; d < 3; ++d) {
            const double x = B.coords[3 * a + d];
            if (!std::isfinite(x) || std::fabs(x) > 100.0 * L[d])
                return fail(GPW_EINVAL, "gpw_plan: atom coordinates must be finite and within 100 cells of the origin");
        }
    int n_ao = 0, n_ps = 0;
    for (int s = 0; s < B.nshell; ++s) {
        if (B.shell_atom[s] < 0 || B.shell_atom[s] >= B.natm) return fail(GPW_EINVAL, "gpw_plan: shell_atom out of range");
        if (B.shell_l[s] < 0) return fail(GPW_EINVAL, "gpw_plan: negative angular momentum");
        if (B.shell_l[s] > 4) return fail(GPW_EUNSUPPORTED, "gpw_plan: angular momentum above 4 (g) is not supported");
        if (B.shell_nprim[s] < 1 || B.shell_prim0[s] < 0) return fail(GPW_EINVAL, "gpw_plan: bad primitive range");
        for (int k = 0; k < B.shell_nprim[s]; ++k) {
            const double e = B.exps[B.shell_prim0[s] + k], c = B.coefs[B.shell_prim0[s] + k];
            if (!(e > 0.0) || !std::isfinite(e)) return fail(GPW_EINVAL, "gpw_plan: exponents must be positive and finite");
            if (!std::isfinite(c)) return fail(GPW_EINVAL, "gpw_plan: non-finite coefficient");
        }
        n_ao += ncart(B.shell_l[s]);
        n_ps += B.shell_nprim[s];
    }
    // ---- cutoffs
    const gpw_cutoffs &C = *cut;
    if (C.nlevels < 1 || C.nlevels > kMaxLevels) return fail(GPW_EINVAL, "gpw_plan: nlevels must be in 1..8");
    if (!(C.tau > 0.0 && C.tau < 1.0)) return fail(GPW_EINVAL, "gpw_plan: tau must be in (0, 1)");
    if (C.precision != GPW_FP64 && C.precision != GPW_FP32) return fail(GPW_EINVAL, "gpw_plan: bad precision");
    if (!C.mesh && !C.ke_cutoff_ry) return fail(GPW_EINVAL, "gpw_plan: need ke_cutoff_ry or mesh");
    if (C.nlevels > 1 && !C.ke_cutoff_ry) return fail(GPW_EINVAL, "gpw_plan: multigrid needs ke_cutoff_ry");
    if (C.ke_cutoff_ry) {
        for (int i = 0; i < C.nlevels; ++i) {
            if (!(C.ke_cutoff_ry[i] > 0.0) || !std::isfinite(C.ke_cutoff_ry[i]))
                return fail(GPW_EINVAL, "gpw_plan: cutoffs must be positive");
            if (i > 0 && !(C.ke_cutoff_ry[i] < C.ke_cutoff_ry[i - 1]))
                return fail(GPW_EINVAL, "gpw_plan: cutoffs must be strictly descending");
        }
        if (C.nlevels > 1 && !(C.rel_cutoff_ry > 0.0)) return fail(GPW_EINVAL, "gpw_plan: rel_cutoff_ry must be positive");
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(GPW_EDEVICE, "gpw_plan: no HIP device");
    if (C.device < 0 || C.device >= ndev) return fail(GPW_EINVAL, "gpw_plan: device ordinal out of range");

    gpw_plan_s *pl = new (std::nothrow) gpw_plan_s();
    if (!pl) return fail(GPW_ENOMEM, "gpw_plan: host allocation failed");
    pl->device = C.device;
    pl->precision = C.precision;
    pl->nlevels = C.nlevels;
    pl->natm = B.natm;
    pl->nshell = B.nshell;
    pl->n_ao = n_ao;
    pl->n_ps = n_ps;
    pl->tau = C.tau;
    pl->rel_cut = C.rel_cutoff_ry;
    for (int d = 0; d < 3; ++d) pl->L[d] = L[d];
    pl->tri = tri;
    std::memcpy(pl->A, Alat, sizeof(Alat));
    for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 3; ++c) pl->recip[d][c] = 2.0 * M_PI * Ainv[c][d];
    const double vol = std::fabs(det);
    pl->volume = vol;
    for (int l = 0; l < C.nlevels; ++l) {
        LevelGeom &G = pl->geom[l];
        pl->cut_ry[l] = C.ke_cutoff_ry ? C.ke_cutoff_ry[l] : 0.0;
        for (int d = 0; d < 3; ++d) {
            long n;
            if (C.mesh) {
                n = C.mesh[3 * l + d];
                if (n < 1 || n > (1 << 20)) { free_plan(pl); return fail(GPW_EINVAL, "gpw_plan: mesh out of range"); }
            } else {
                // |a_d| = L[d]: a plane wave with |G|^2 < E has
                // |m_d| = |G . a_d| / (2 pi) < sqrt(E) |a_d| / (2 pi) <= N / 2
                n = (long)std::ceil(std::sqrt(C.ke_cutoff_ry[l]) * L[d] / M_PI);
                if (n < 1) n = 1;
                while (!smooth235(n)) ++n;
            }
            G.N[d] = (int)n;
            G.nb[d] = (int)((n + 3) / 4);
            G.h[d] = tri ? 1.0 : L[d] / (double)n;   // index units for a general cell
        }
        pl->ngrid[l] = (long long)G.N[0] * G.N[1] * G.N[2];
        pl->nblocks[l] = (long long)G.nb[0] * G.nb[1] * G.nb[2];
        G.w = vol / (double)pl->ngrid[l];
        G.tri = nullptr;
        if (tri) {
            TriGeom &t = pl->tri_host[l];
            for (int d = 0; d < 3; ++d)
                for (int c = 0; c < 3; ++c) t.H[d][c] = Alat[d][c] / G.N[d];
            inverse3(t.H, t.Hinv);
            for (int d = 0; d < 3; ++d)
                for (int e2 = 0; e2 < 3; ++e2)
                    t.g[d][e2] = t.H[d][0] * t.H[e2][0] + t.H[d][1] * t.H[e2][1] + t.H[d][2] * t.H[e2][2];
            t.lmin = min_eigenvalue(t.g) * (1.0 - 1e-9);   // a hair below: the bound stays conservative
            for (int d = 0; d < 3; ++d)
                t.rf[d] = std::sqrt(t.Hinv[0][d] * t.Hinv[0][d] + t.Hinv[1][d] * t.Hinv[1][d] +
                                    t.Hinv[2][d] * t.Hinv[2][d]);
        }
    }

    // primitive-shell table (host flattening of the basis arrays)
    std::vector<int> ps_atom(n_ps), ps_l(n_ps), ps_ao(n_ps);
    std::vector<double> ps_alpha(n_ps), ps_coef(n_ps);
    {
        int q = 0, ao = 0;
        for (int s = 0; s < B.nshell; ++s) {
            for (int k = 0; k < B.shell_nprim[s]; ++k, ++q) {
                ps_atom[q] = B.shell_atom[s];
                ps_l[q] = B.shell_l[s];
                ps_ao[q] = ao;
                ps_alpha[q] = B.exps[B.shell_prim0[s] + k];
                ps_coef[q] = B.coefs[B.shell_prim0[s] + k];
            }
            ao += ncart(B.shell_l[s]);
        }
    }

    DeviceGuard guard(pl->device);
    if (guard.err != hipSuccess) { free_plan(pl); return hip_fail(guard.err, "gpw_plan: hipSetDevice"); }
    {
        // The eval calls take their scratch from the device's default stream-ordered
        // pool; keep freed blocks in the pool instead of returning them to the HIP runtime
        // at every synchronisation, so that repeated evaluations do not remap memory.
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, pl->device) == hipSuccess) {
            uint64_t keep = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        }
    }
    {
        // set-up of the allocation-free entry point on this device: look up the
        // address of its fixed scratch array once, with the device current
        unsigned char *scr = nullptr;
        const hipError_t es = gpw::noalloc_scratch(pl->device, &scr);
        if (es != hipSuccess) { free_plan(pl); return hip_fail(es, "gpw_plan: scratch symbol address"); }
    }
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) { free_plan(pl); return hip_fail(e, "gpw_plan: hipStreamCreate"); }
    auto upload = [&](auto *&dst, const auto &vec) -> hipError_t {
        using V = typename std::remove_reference<decltype(vec)>::type::value_type;
        hipError_t r = hipMalloc((void **)&dst, sizeof(V) * vec.size());
        if (r != hipSuccess) return r;
        pl->allocations.push_back(dst);
        return hipMemcpy(dst, vec.data(), sizeof(V) * vec.size(), hipMemcpyHostToDevice);
    };
    std::vector<double> coords(B.coords, B.coords + 3 * B.natm);
    if ((e = upload(pl->d_ps_atom, ps_atom)) != hipSuccess || (e = upload(pl->d_ps_l, ps_l)) != hipSuccess ||
        (e = upload(pl->d_ps_ao, ps_ao)) != hipSuccess || (e = upload(pl->d_ps_alpha, ps_alpha)) != hipSuccess ||
        (e = upload(pl->d_ps_coef, ps_coef)) != hipSuccess || (e = upload(pl->d_coords, coords)) != hipSuccess) {
        (void)hipStreamDestroy(st);
        free_plan(pl);
        return hip_fail(e, "gpw_plan: upload");
    }
    PartitionInput in;
    in.ps = PsTable{pl->d_ps_atom, pl->d_ps_l, pl->d_ps_ao, pl->d_ps_alpha, pl->d_ps_coef, pl->d_coords, n_ps};
    if (tri) {
        // the levels' transforms T_n and geometry records on the device
        size_t per = 0;
        int toff[kMaxTDeg + 1];
        for (int n2 = 0; n2 <= kMaxTDeg; ++n2) {
            toff[n2] = (int)per;
            per += (size_t)ncart(n2) * ncart(n2);
        }
        std::vector<double> T(per * C.nlevels);
        for (int l = 0; l < C.nlevels; ++l)
            for (int n2 = 0; n2 <= kMaxTDeg; ++n2) monomial_transform(pl->tri_host[l].H, n2, &T[l * per + toff[n2]]);
        double *dT = nullptr;
        if ((e = upload(dT, T)) != hipSuccess) {
            (void)hipStreamDestroy(st);
            free_plan(pl);
            return hip_fail(e, "gpw_plan: upload");
        }
        std::vector<TriGeom> tg(C.nlevels);
        for (int l = 0; l < C.nlevels; ++l) {
            pl->tri_host[l].T = dT + l * per;
            std::memcpy(pl->tri_host[l].toff, toff, sizeof(toff));
            tg[l] = pl->tri_host[l];
        }
        if ((e = upload(pl->d_tri, tg)) != hipSuccess) {
            (void)hipStreamDestroy(st);
            free_plan(pl);
            return hip_fail(e, "gpw_plan: upload");
        }
        for (int l = 0; l < C.nlevels; ++l) pl->geom[l].tri = pl->d_tri + l;
    }
    for (int d = 0; d < 3; ++d) in.pc.L[d] = L[d];
    in.pc.tri = tri;
    std::memcpy(in.pc.A, Alat, sizeof(Alat));
    std::memcpy(in.pc.Ainv, Ainv, sizeof(Ainv));
    in.pc.logtau = std::log(C.tau);
    in.pc.rel_cut = C.rel_cutoff_ry;
    in.pc.nlevels = C.nlevels;
    for (int l = 0; l < kMaxLevels; ++l) {
        in.pc.cut[l] = l < C.nlevels ? pl->cut_ry[l] : 0.0;
        in.pc.geom[l] = pl->geom[l];
    }
    std::string err;
    bool unsupported = false;
    e = build_partition(pl, in, st, err, unsupported);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
    if (e != hipSuccess) {
        free_plan(pl);
        const gpw_status st_code = unsupported ? GPW_EUNSUPPORTED
                                   : e == hipErrorOutOfMemory ? GPW_ENOMEM
                                                              : GPW_EDEVICE;
        return fail(st_code, "gpw_plan: " + err);
    }
    {
        // the pair-major kernels keep a pair image's point tables, block lists
        // and block rows in LDS: the widest sphere must fit one workgroup's share
        int lds_max = 0;
        (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, pl->device);
        const size_t need = gpw::pair_kernel_lds_bytes(pl->max_axis_blocks > 0 ? pl->max_axis_blocks : 1,
                                                       pl->precision, pl->tri != 0);
        if (lds_max > 0 && need > (size_t)lds_max) {
            const std::string msg = "gpw_plan: the widest truncation sphere (" +
                                    std::to_string(pl->info.max_box_width) + " points per axis) needs " +
                                    std::to_string(need) + " bytes of LDS per workgroup, above the device's " +
                                    std::to_string(lds_max);
            free_plan(pl);
            return fail(GPW_EUNSUPPORTED, msg);
        }
    }
    gpw_plan_info &I = pl->info;
    I.nlevels = pl->nlevels;
    for (int l = 0; l < pl->nlevels; ++l) {
        for (int d = 0; d < 3; ++d) I.mesh[l][d] = pl->geom[l].N[d];
        I.weight[l] = pl->geom[l].w;
        I.n_grid[l] = pl->ngrid[l];
    }
    I.n_ao = pl->n_ao;
    I.natm = pl->natm;
    I.precision = pl->precision;
    I.device_bytes = (long long)(sizeof(PairRec) * pl->n_pairs + sizeof(int2) * pl->n_inc) +
                     (long long)sizeof(long long) * (pl->cnt_base[kMaxGroups] + 2) +
                     (long long)sizeof(int) * pl->blk_off[kMaxGroups] +
                     (long long)n_ps * (3 * sizeof(int) + 2 * sizeof(double)) + 24LL * pl->natm;
    for (int op = GPW_OP_RHO; op <= GPW_OP_GRAD_TAU; ++op)
        I.scratch_bytes[op] = (long long)gpw::eval_scratch_bytes(pl, op);
    I.poisson_scratch_bytes = (long long)gpw::poisson_spectra_bytes(pl);
    *out = pl;
    return GPW_OK;
}

gpw_status gpw_plan_destroy(gpw_plan_t plan)
{
    if (!plan) return GPW_OK;
    DeviceGuard guard(plan->device);
    free_plan(plan);
    return GPW_OK;
}

gpw_status gpw_plan_query(gpw_plan_t plan, gpw_plan_info *out)
{
    if (!plan || !out) return fail(GPW_EINVAL, "gpw_plan_query: NULL argument");
    *out = plan->info;
    return GPW_OK;
}

static gpw_status check_levels(const gpw_plan_s *pl, const void *const *arr, const char *what)
{
    if (!arr) return fail(GPW_EINVAL, std::string(what) + ": NULL level array");
    for (int l = 0; l < pl->nlevels; ++l)
        if (!arr[l]) return fail(GPW_EINVAL, std::string(what) + ": NULL level pointer");
    return GPW_OK;
}

// Validated copy of one task.
static gpw_status check_task(const gpw_task &t, TaskRef &out, const char *what)
{
    if (!t.plan) return fail(GPW_EINVAL, std::string(what) + ": NULL plan");
    gpw_status s = GPW_OK;
    switch (t.op) {
    case GPW_OP_RHO:
    case GPW_OP_TAU:
        if (!t.D) return fail(GPW_EINVAL, std::string(what) + ": NULL D");
        s = check_levels(t.plan, (const void *const *)t.rho, what);
        break;
    case GPW_OP_MAT:
    case GPW_OP_MAT_TAU:
        if (!t.out) return fail(GPW_EINVAL, std::string(what) + ": NULL M");
        s = check_levels(t.plan, (const void *const *)t.v, what);
        break;
    case GPW_OP_GRAD:
    case GPW_OP_GRAD_TAU:
        if (!t.D || !t.out) return fail(GPW_EINVAL, std::string(what) + ": NULL D or grad");
        s = check_levels(t.plan, (const void *const *)t.v, what);
        break;
    default: return fail(GPW_EINVAL, std::string(what) + ": unknown op");
    }
    if (s != GPW_OK) return s;
    out = TaskRef{t.plan, t.op, t.D, t.v, t.rho, t.out};
    return GPW_OK;
}

static gpw_status run_tasks(const gpw_task *tasks, int n, void *stream, const char *what)
{
    std::vector<TaskRef> refs((size_t)n);
    for (int i = 0; i < n; ++i) {
        gpw_status s = check_task(tasks[i], refs[(size_t)i], what);
        if (s != GPW_OK) return s;
        if (tasks[i].plan->device != tasks[0].plan->device)
            return fail(GPW_EINVAL, std::string(what) + ": plans on different devices");
    }
    if (n == 0) return GPW_OK;
    DeviceGuard guard(tasks[0].plan->device);
    if (guard.err != hipSuccess) return hip_fail(guard.err, what);
    hipError_t e = gpw::eval_batch(refs.data(), n, (hipStream_t)stream);
    return e == hipSuccess ? GPW_OK : hip_fail(e, what);
}

gpw_status gpw_eval_rho(gpw_plan_t plan, const double *D, double *const *rho, void *stream)
{
    gpw_task t{plan, GPW_OP_RHO, D, nullptr, rho, nullptr};
    return run_tasks(&t, 1, stream, "gpw_eval_rho");
}

gpw_status gpw_eval_mat(gpw_plan_t plan, const double *const *v, double *M, void *stream)
{
    gpw_task t{plan, GPW_OP_MAT, nullptr, v, nullptr, M};
    return run_tasks(&t, 1, stream, "gpw_eval_mat");
}

gpw_status gpw_eval_grad(gpw_plan_t plan, const double *D, const double *const *v, double *grad, void *stream)
{
    gpw_task t{plan, GPW_OP_GRAD, D, v, nullptr, grad};
    return run_tasks(&t, 1, stream, "gpw_eval_grad");
}

gpw_status gpw_eval_tau(gpw_plan_t plan, const double *D, double *const *tau, void *stream)
{
    gpw_task t{plan, GPW_OP_TAU, D, nullptr, tau, nullptr};
    return run_tasks(&t, 1, stream, "gpw_eval_tau");
}

gpw_status gpw_eval_mat_tau(gpw_plan_t plan, const double *const *vtau, double *M, void *stream)
{
    gpw_task t{plan, GPW_OP_MAT_TAU, nullptr, vtau, nullptr, M};
    return run_tasks(&t, 1, stream, "gpw_eval_mat_tau");
}

gpw_status gpw_eval_grad_tau(gpw_plan_t plan, const double *D, const double *const *vtau, double *grad,
                             void *stream)
{
    gpw_task t{plan, GPW_OP_GRAD_TAU, D, vtau, nullptr, grad};
    return run_tasks(&t, 1, stream, "gpw_eval_grad_tau");
}

// Preconditions of the Fourier-space calls: level 0 holds the finest mesh on
// every axis, and a multigrid plan has its level cutoffs (the masks).
static gpw_status check_fourier(const gpw_plan_s *pl, const void *const *rho, const char *what)
{
    if (!pl) return fail(GPW_EINVAL, std::string(what) + ": NULL plan");
    gpw_status s = check_levels(pl, rho, what);
    if (s != GPW_OK) return s;
    for (int l = 1; l < pl->nlevels; ++l)
        for (int d = 0; d < 3; ++d)
            if (pl->geom[l].N[d] > pl->geom[0].N[d])
                return fail(GPW_EINVAL, std::string(what) + ": level 0 must hold the finest mesh on every axis");
    if (pl->nlevels > 1)
        for (int l = 0; l < pl->nlevels; ++l)
            if (!(pl->cut_ry[l] > 0.0))
                return fail(GPW_EINVAL, std::string(what) + ": a multigrid plan needs the level cutoffs");
    return GPW_OK;
}

gpw_status gpw_hxc_potential(gpw_plan_t plan, const double *const *rho, const double *vxc,
                             const double *const *vxc_grad, double *const *v, double *e_j, void *stream)
{
    gpw_status s = check_fourier(plan, (const void *const *)rho, "gpw_hxc_potential");
    if (s != GPW_OK) return s;
    s = check_levels(plan, (const void *const *)v, "gpw_hxc_potential");
    if (s != GPW_OK) return s;
    if (vxc_grad && (!vxc_grad[0] || !vxc_grad[1] || !vxc_grad[2]))
        return fail(GPW_EINVAL, "gpw_hxc_potential: NULL component of vxc_grad");
    DeviceGuard guard(plan->device);
    if (guard.err != hipSuccess) return hip_fail(guard.err, "gpw_hxc_potential");
    const hipError_t e = gpw::poisson_run(plan, rho, vxc, vxc_grad, v, e_j, (hipStream_t)stream);
    return e == hipSuccess ? GPW_OK : hip_fail(e, "gpw_hxc_potential");
}

gpw_status gpw_poisson(gpw_plan_t plan, const double *const *rho, double *const *v, double *e_j, void *stream)
{
    gpw_status s = check_fourier(plan, (const void *const *)rho, "gpw_poisson");
    if (s != GPW_OK) return s;
    s = check_levels(plan, (const void *const *)v, "gpw_poisson");
    if (s != GPW_OK) return s;
    DeviceGuard guard(plan->device);
    if (guard.err != hipSuccess) return hip_fail(guard.err, "gpw_poisson");
    const hipError_t e = gpw::poisson_run(plan, rho, nullptr, nullptr, v, e_j, (hipStream_t)stream);
    return e == hipSuccess ? GPW_OK : hip_fail(e, "gpw_poisson");
}

gpw_status gpw_fine_density(gpw_plan_t plan, const double *const *rho, double *rho_fine, double *const *grad,
                            void *stream)
{
    gpw_status s = check_fourier(plan, (const void *const *)rho, "gpw_fine_density");
    if (s != GPW_OK) return s;
    if (grad && (!grad[0] || !grad[1] || !grad[2]))
        return fail(GPW_EINVAL, "gpw_fine_density: NULL component of grad");
    DeviceGuard guard(plan->device);
    if (guard.err != hipSuccess) return hip_fail(guard.err, "gpw_fine_density");
    const hipError_t e = gpw::fine_density_run(plan, rho, rho_fine, grad, (hipStream_t)stream);
    return e == hipSuccess ? GPW_OK : hip_fail(e, "gpw_fine_density");
}

gpw_status gpw_eval_mat_noalloc(gpw_plan_t plan, const double *const *v, double *M, void *stream)
{
    const gpw_task t{plan, GPW_OP_MAT, nullptr, v, nullptr, M};
    TaskRef ref;
    gpw_status s = check_task(t, ref, "gpw_eval_mat_noalloc");
    if (s != GPW_OK) return s;
    const size_t need = gpw::eval_scratch_bytes(plan, GPW_OP_MAT);
    if (need > gpw::kNoAllocScratchBytes)
        return fail(GPW_EBUDGET, "gpw_eval_mat_noalloc: the plan needs " + std::to_string(need) +
                                     " bytes of scratch, above the fixed " +
                                     std::to_string(gpw::kNoAllocScratchBytes) + " of this entry point");
    DeviceGuard guard(plan->device);
    if (guard.err != hipSuccess) return hip_fail(guard.err, "gpw_eval_mat_noalloc");
    const hipError_t e = gpw::eval_noalloc(ref, (hipStream_t)stream);
    return e == hipSuccess ? GPW_OK : hip_fail(e, "gpw_eval_mat_noalloc");
}

gpw_status gpw_eval_batch(const gpw_task *tasks, int ntasks, void *stream)
{
    if (ntasks < 0 || (ntasks > 0 && !tasks)) return fail(GPW_EINVAL, "gpw_eval_batch: bad task array");
    return run_tasks(tasks, ntasks, stream, "gpw_eval_batch");
}

}  // extern "C"
