/*
 * gpw.h - C ABI of the MI355X (gfx950) multigrid Gaussian-plane-wave
 * collocation / integration library.
 *
 * The library evaluates, on one GPU, the three kernels of the multigrid FFTDF
 * Fock build and nuclear gradient described in "Implementation of the
 * multigrid Gaussian-Plane-Wave algorithm with GPU acceleration in PySCF"
 * (arXiv 2603.24881):
 *
 *   gpw_eval_rho   density matrix D -> rho_l(r) on every multigrid level
 *                  (Sec. II, Eq. (rho); Sec. III.A, Eq. (rho_wrap); Alg. 1)
 *   gpw_eval_mat   level potentials v_l(r) -> matrix M_{mu nu}
 *                  (Sec. II, Eq. (J); Sec. III.A, Eq. (J_wrap); Alg. 2)
 *   gpw_eval_grad  D, v_l -> dE/dR_A of E = sum_l w_l <v_l, rho_l>
 *                  (Sec. III.B, Alg. 3)
 *
 * behind a plan (gpw_plan) that screens primitive Gaussian pairs and maps them
 * to grid blocks (Sec. III.B and the appendix on GTO screening, Algs. 4, 5).
 *
 * Conventions shared by all calls
 * -------------------------------
 * Units: bohr, bohr^-2 for exponents, Rydberg for plane-wave cutoffs.
 * Cell: lattice vectors a_d are the rows of a[3][3], right- or left-handed,
 *   linearly independent.  A diagonal a is an orthorhombic cell; any other a
 *   is a general (non-orthogonal) cell, evaluated in the grid-index
 *   coordinates of each level with the cross terms of the Gaussian envelope
 *   (appendix on non-orthogonal lattices).
 * Basis: contracted Cartesian shells, l = 0..4.  exps/coefs are the primitive
 *   exponents and raw coefficients: a contracted AO is
 *   sum_k coefs[k] (x-Ax)^i (y-Ay)^j (z-Az)^k exp(-exps[k] |r-A|^2)
 *   (un-normalised Cartesian primitives, Sec. III.A, Eq. (gx)).
 * AO order: shells in input order; inside a shell the Cartesian components in
 *   lexicographic order (lx descending, then ly descending): s; x y z;
 *   xx xy xz yy yz zz; xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz.
 * Matrices: n_ao x n_ao, row-major, FP64, device memory.
 * Grids: level l holds mesh[l][0]*mesh[l][1]*mesh[l][2] FP64 values in C
 *   order [i0][i1][i2]; point (i0,i1,i2) sits at sum_d (i_d / mesh[l][d]) a_d
 *   (origin at the cell corner; (i0 h0, i1 h1, i2 h2) with h_d = L_d / mesh[l][d]
 *   for an orthorhombic cell of side lengths L_d).
 * Quadrature weight of level l: w_l = Omega / N_l (Sec. III.A, the weight in
 *   the definition of the V tensor).  eval_mat and eval_grad apply it; rho is
 *   unweighted.
 * Truncation: a primitive pair image p (exponents a, b; centres A, B + T)
 *   with alpha_p = a + b, P = (a A + b (B+T)) / alpha_p, L = l_a + l_b and
 *   K = c_a c_b exp(-a b / alpha_p |A - B - T|^2) is dropped when the maximum
 *   of f(r) = |K| r^(L+2) exp(-alpha_p r^2) is below tau; otherwise it
 *   contributes at the grid points with |r - P| <= R, f(R) = tau, R beyond the
 *   maximum (Sec. III.A, Eq. (cut) and the sphere about P used with
 *   Eq. (exp_rr)).
 * Levels: a pair image goes to the coarsest level i with
 *   ke_cutoff_ry[i] >= alpha_p * rel_cutoff_ry, or to level 0 (finest) when
 *   none qualifies (Sec. II, multigrid).  Default mesh of a level: per axis the
 *   smallest 2,3,5-smooth N >= sqrt(E) |a_d| / pi, so that every plane wave
 *   with |G|^2 < E has |m_d| = |G . a_d| / (2 pi) < N / 2.
 *
 * Errors: every call returns a gpw_status.  Argument errors are detected
 * before anything is enqueued.  A device fault surfaces as GPW_EDEVICE on a
 * later call.  On error the outputs are unspecified and the plan stays valid.
 * gpw_last_error() returns a thread-local message for the last failure.
 *
 * Scratch: eval calls take temporary device memory from the device's default
 *   stream-ordered pool (hipMallocAsync) and return it on the same stream;
 *   gpw_plan sets that pool's release threshold to "keep everything", so the
 *   pool retains its peak size for the life of the process.
 * Streams: eval calls enqueue on the given hipStream_t (NULL = the default
 * stream) and return without synchronising.  Inputs must stay valid and
 * outputs untouched until the stream reaches the end of the call.  One plan
 * may serve several streams concurrently when their outputs differ.
 */
#ifndef GPW_H
#define GPW_H

#ifdef __cplusplus
extern "C" {
#endif

#define GPW_MAX_LEVELS 8
#define GPW_NCLASS 15   /* (l_a, l_b) with 4 >= l_a >= l_b >= 0 */

typedef enum {
    GPW_OK = 0,
    GPW_EINVAL = 1,        /* bad argument (NULL pointer, l < 0, exponent <= 0, ...) */
    GPW_EUNSUPPORTED = 2,  /* valid but not implemented (l > 4, a truncation sphere too wide) */
    GPW_ENOMEM = 3,        /* device allocation failed */
    GPW_EDEVICE = 4,       /* HIP runtime error or device fault */
    GPW_EBUDGET = 5        /* the call's scratch does not fit a fixed budget (gpw_eval_mat_noalloc) */
} gpw_status;

typedef enum { GPW_FP64 = 0, GPW_FP32 = 1 } gpw_precision;

typedef struct gpw_plan_s *gpw_plan_t;

typedef struct {
    double a[3][3];        /* lattice vectors as rows (bohr); must be diagonal */
} gpw_cell;

typedef struct {
    int natm;
    const double *coords;       /* natm*3, any position (not wrapped) */
    int nshell;
    const int *shell_atom;      /* nshell, atom index of each shell */
    const int *shell_l;         /* nshell, 0..4 */
    const int *shell_nprim;     /* nshell, >= 1 */
    const int *shell_prim0;     /* nshell, offset of the shell's primitives */
    const double *exps;         /* primitive exponents, > 0 */
    const double *coefs;        /* raw primitive coefficients */
} gpw_basis;

typedef struct {
    int nlevels;                /* 1..GPW_MAX_LEVELS */
    const double *ke_cutoff_ry; /* nlevels, strictly descending; may be NULL when nlevels == 1
                                   and mesh is given */
    const int *mesh;            /* optional nlevels*3 mesh override (NULL = mesh rule) */
    double rel_cutoff_ry;       /* E_rel of the level rule */
    double tau;                 /* screening threshold (> 0), e.g. 1e-6 */
    int precision;              /* gpw_precision of the per-point arithmetic */
    int device;                 /* HIP device ordinal */
} gpw_cutoffs;

typedef struct {
    int nlevels;
    int mesh[GPW_MAX_LEVELS][3];
    double weight[GPW_MAX_LEVELS];            /* w_l = Omega / N_l */
    long long n_grid[GPW_MAX_LEVELS];         /* points per level */
    int n_ao;
    int natm;
    int precision;
    long long n_pairs[GPW_MAX_LEVELS];        /* canonical pair images per level */
    long long n_pairs_class[GPW_NCLASS];      /* canonical pair images per (l_a, l_b) class */
    long long n_incidences[GPW_MAX_LEVELS];   /* (pair image, 4^3 block) incidences */
    long long n_incidences_class[GPW_NCLASS];
    double sphere_points;                     /* sum over pair images of points inside the sphere */
    /* flop model (FMA = 2), a fixed counting convention: per (pair image, point), with n_a,
       n_b the Cartesian counts, F_rho = F_mat = 2 n_a n_b + 2 (n_a + n_b) + 4 and
       F_grad = 4 n_a n_b + 8 (n_a + n_b) + 4 (the direct evaluation).  "block" counts 64
       points per (pair image, 4^3 block) incidence (the points the block method visits);
       "sphere" counts only points inside the sphere. */
    double flops_rho_block, flops_rho_sphere;
    double flops_mat_block, flops_mat_sphere;
    double flops_grad_block, flops_grad_sphere;
    /* the arithmetic the rho and mat kernels perform over the block points (FMA = 2): the
       direct F for the classes evaluated directly; with L = l_a + l_b, per incidence
       8 C(L+2,3) + 32 C(L+1,2) + 16 + 64 (2L + 3) for the rho classes evaluated through the
       coefficient tensor (Eq. (rho1)) and 64 (2L + 3) for the mat classes accumulating
       moments */
    double flops_rho_exec, flops_mat_exec;
    long long device_bytes;                   /* device memory held by the plan */
    int max_box_width;                        /* widest bounding box (points per axis) */
    long long scratch_bytes[6];               /* device scratch of one evaluation, indexed by the op
                                                 value GPW_OP_RHO .. GPW_OP_GRAD_TAU; taken from the
                                                 pool for the duration of the call (a batch takes the
                                                 sum over its tasks) */
    /* the arithmetic of the other kernels, by the same rules as flops_rho_exec / _mat_exec:
       grad accumulates moments of degree L + 1 (64 (2 (L+1) + 3) per incidence); the kinetic
       energy density terms work two degrees higher: tau through its coefficient tensor of
       degree L + 2 (the rho tensor count with L + 2), mat_tau and grad_tau through moments of
       degree L + 2 and L + 3.  The per-pair-image formation of matrix elements and gradient
       components from the moments is not counted. */
    double flops_grad_exec, flops_tau_exec, flops_mat_tau_exec, flops_grad_tau_exec;
    long long poisson_scratch_bytes;          /* device scratch of gpw_poisson's spectra; the FFT library's
                                                 work area (known once its plans exist) comes on top */
} gpw_plan_info;

/* Build a plan: screen primitive pair images, assign levels, compute their
 * truncation spheres, and map them to 4x4x4 grid blocks of each level
 * (Sec. III.B; appendix on GTO screening, Algs. 4 and 5).  All host inputs
 * are copied; the caller may free them on return.  The plan owns its device
 * memory on cut->device.  Synchronous.  Errors: GPW_EINVAL for NULL or invalid
 * arguments (including linearly dependent lattice vectors), GPW_EUNSUPPORTED
 * for l > 4, or a truncation
 * sphere too wide for the kernels (more than 1024 points per axis, more than
 * 127 cell periods, or per-axis point tables beyond one workgroup's LDS; the
 * block rows of a wide sphere are walked in slices and never limit it),
 * GPW_ENOMEM,
 * GPW_EDEVICE. */
gpw_status gpw_plan(const gpw_cell *cell, const gpw_basis *basis,
                    const gpw_cutoffs *cut, gpw_plan_t *out);

/* Free a plan and its device memory (NULL is accepted).  The caller must make
 * sure no enqueued call still uses it. */
gpw_status gpw_plan_destroy(gpw_plan_t plan);

/* Sizes, meshes, weights, work counts and the flop model of a plan. */
gpw_status gpw_plan_query(gpw_plan_t plan, gpw_plan_info *out);

/* Density collocation (Sec. II, Eq. (rho); Sec. III.A, Eq. (rho_wrap);
 * Alg. 1).  D: device, n_ao x n_ao row-major; only (D + D^T)/2 is used.
 * rho: host array of nlevels device pointers; rho[l] receives the level-l
 * partial density (overwritten, unweighted).  Enqueued on stream. */
gpw_status gpw_eval_rho(gpw_plan_t plan, const double *D, double *const *rho, void *stream);

/* Potential integration (Sec. II, Eq. (J); Sec. III.A, Eq. (J_wrap); Alg. 2):
 * M_{mu nu} = sum_l w_l sum_r v_l(r) sum_{pair images p of (mu, nu)}
 * Lambda_p,mu nu(r), contracted Cartesian basis, full symmetric matrix.
 * v: host array of nlevels device pointers to the level potentials.
 * M: device n_ao x n_ao, overwritten.  Enqueued on stream. */
gpw_status gpw_eval_mat(gpw_plan_t plan, const double *const *v, double *M, void *stream);

/* Nuclear gradient of the collocation (Sec. III.B, Alg. 3):
 * grad[A][x] = d/dR_{A,x} sum_l w_l <v_l, rho_l(D; R)> at fixed D and v
 * (the force is -grad).  D as in gpw_eval_rho, v as in gpw_eval_mat;
 * grad: device natm x 3, overwritten.  Enqueued on stream. */
gpw_status gpw_eval_grad(gpw_plan_t plan, const double *D, const double *const *v,
                         double *grad, void *stream);

/* Kinetic energy density of meta-GGA functionals (Sec. II, the kinetic
 * energy density and Eq. (J_metaGGA); Sec. III.B, the pair function of
 * Algs. 1-3 replaced by the product of the two factors' gradients):
 * tau_l(r) = 1/2 sum_{mu nu} D_{mu nu} grad phi_mu(r) . grad phi_nu(r) over the
 * same pair images, levels and truncation spheres as gpw_eval_rho (the plan
 * is shared).  D and tau as D and rho of gpw_eval_rho (tau[l] overwritten,
 * unweighted).  Enqueued on stream. */
gpw_status gpw_eval_tau(gpw_plan_t plan, const double *D, double *const *tau, void *stream);

/* The kinetic-energy-density term of the matrix, the derivative of
 * E_tau = sum_l w_l <vtau_l, tau_l(D)> with respect to D_{mu nu}:
 * M_{mu nu} = 1/2 sum_l w_l sum_r vtau_l(r) grad phi_mu . grad phi_nu
 * (Sec. II, Eq. (J_metaGGA); Sec. III.B with Alg. 2).  vtau, M as v, M of
 * gpw_eval_mat (M overwritten, full symmetric).  Enqueued on stream. */
gpw_status gpw_eval_mat_tau(gpw_plan_t plan, const double *const *vtau, double *M, void *stream);

/* Nuclear gradient of E_tau at fixed D and vtau (Sec. III.B, the meta-GGA
 * note with Alg. 3; second derivatives of the basis functions):
 * grad[A][x] = d/dR_{A,x} sum_l w_l <vtau_l, tau_l(D; R)>.  Arguments as
 * gpw_eval_grad (grad overwritten).  Enqueued on stream. */
gpw_status gpw_eval_grad_tau(gpw_plan_t plan, const double *D, const double *const *vtau, double *grad,
                             void *stream);

/* Multigrid Fourier transfer and Poisson solve (Sec. II: the Hartree
 * potential of Eqs. (vH), (vHG) and the multigrid Fourier interpolation
 * between the levels), the step between gpw_eval_rho and gpw_eval_mat of a
 * Fock build.  With w_l = Omega / N_l, plane waves G = sum_d m_d b_d with
 * integer m and the reciprocal vectors b_d = 2 pi (A^-1)[:, d] (G = 2 pi m / L
 * for an orthorhombic cell), and
 * mask_l(G) = {|m_d| < N_{l,d} / 2 on every axis and |G|^2 < E_l (Ry, bohr^-2)}
 * (every non-Nyquist plane wave for a single-level plan built from a mesh):
 *   rho~(G) = sum_l mask_l(G) w_l sum_r rho_l(r) exp(-i G.r)
 *   v_l(r)  = (1 / Omega) sum_G mask_l(G) 4 pi rho~(G) / |G|^2 exp(i G.r), G != 0
 *   E_J     = (1 / (2 Omega)) sum_{G != 0} 4 pi |rho~(G)|^2 / |G|^2
 * so that E_J = 1/2 sum_l w_l <v_l, rho_l> and dE_J / d rho_l = w_l v_l: v is the
 * potential gpw_eval_mat and gpw_eval_grad take for the Hartree term.
 * rho: host array of nlevels device pointers (level densities, read only);
 * v: host array of nlevels device pointers, overwritten; e_j: device pointer to
 * one double receiving E_J, or NULL.  Level 0 must hold the finest mesh; a
 * multigrid plan must have been built from cutoffs.  FP64 throughout (hipFFT
 * D2Z / Z2D), whatever the plan's precision.  The first call on a plan builds
 * the FFT plans (host work, synchronous); every call takes its spectra and the
 * FFT work area from the stream-ordered pool.  Enqueued on stream. */
gpw_status gpw_poisson(gpw_plan_t plan, const double *const *rho, double *const *v, double *e_j, void *stream);

/* The same transfer with an exchange-correlation potential given on the
 * finest mesh (level 0), for LDA and GGA functionals (Sec. II, Eqs. (vH),
 * (vHG), the GGA integration by parts and the divergence in Fourier space):
 *   v~(G) = 4 pi rho~(G) / |G|^2 + w_0 F(vxc)(G) - i G . w_0 F(vxc_grad)(G)
 * with F the discrete transform on level 0 and w_0 = Omega / N_0, restricted to
 * level 0's plane waves, then v_l(r) = (1 / Omega) sum_G mask_l(G) v~(G)
 * exp(i G.r) as in gpw_poisson.  vxc: device, N_0 doubles (dE_xc / d rho on the
 * finest mesh), or NULL; vxc_grad: host array of three device pointers (the
 * x, y, z components of dE_xc / d grad rho on the finest mesh), or NULL.
 * E_J (e_j, device, or NULL) is the Hartree energy alone.  With rho from
 * gpw_fine_density, sum_l w_l <v_l, rho_l> of the xc part equals
 * w_0 (<vxc, rho> + sum_d <vxc_grad_d, d_d rho>) on the finest mesh.  Other
 * arguments and conditions as gpw_poisson.  Enqueued on stream. */
gpw_status gpw_hxc_potential(gpw_plan_t plan, const double *const *rho, const double *vxc,
                             const double *const *vxc_grad, double *const *v, double *e_j, void *stream);

/* The total density and its gradient on the finest mesh (level 0) by Fourier
 * interpolation of the level densities (Sec. II: rho~ as in gpw_poisson; the
 * GGA density gradient as the inverse transform of i G rho~):
 *   rho(r) = (1 / Omega) sum_G rho~(G) exp(i G.r),
 *   d_d rho(r) = (1 / Omega) sum_G i G_d rho~(G) exp(i G.r).
 * rho: host array of nlevels device pointers; rho_fine: device, N_0 doubles,
 * or NULL; grad: host array of three device pointers (N_0 doubles each), or
 * NULL.  Conditions as gpw_poisson.  Enqueued on stream. */
gpw_status gpw_fine_density(gpw_plan_t plan, const double *const *rho, double *rho_fine, double *const *grad,
                            void *stream);

/* One task of a batched launch. */
typedef enum {
    GPW_OP_RHO = 0, GPW_OP_MAT = 1, GPW_OP_GRAD = 2,
    GPW_OP_TAU = 3, GPW_OP_MAT_TAU = 4, GPW_OP_GRAD_TAU = 5
} gpw_op;

typedef struct {
    gpw_plan_t plan;
    int op;                      /* gpw_op */
    const double *D;             /* RHO, GRAD, TAU, GRAD_TAU */
    const double *const *v;      /* MAT, GRAD, MAT_TAU, GRAD_TAU: host array of nlevels device pointers
                                    (vtau for the _TAU operations) */
    double *const *rho;          /* RHO, TAU: host array of nlevels device pointers (the output grids) */
    double *out;                 /* MAT, MAT_TAU: M (n_ao x n_ao); GRAD, GRAD_TAU: natm x 3 */
} gpw_task;

/* Batched evaluation for serving: the tasks, possibly of different plans and
 * operations, share launches so that the work of several requests overlaps on
 * the device.  Per (operation, (l_a, l_b) class) one launch covers the
 * (task, level) segments of every task, described by a segment table passed
 * by value (at most 16 segments per launch; more segments take more
 * launches); the hardware dispatcher deals each launch's workgroups to the
 * compute units as they free up.  FP64 and FP32 plans form two such sets of
 * launches, back to back.  A single call is a batch of one task: each task
 * computes exactly what the corresponding single call computes (rho and tau
 * bit for bit; matrices and gradients up to the order of their atomic
 * additions).  The scratch of all tasks is one stream-ordered allocation.
 * Outputs of different tasks must not overlap.  Enqueued on stream. */
gpw_status gpw_eval_batch(const gpw_task *tasks, int ntasks, void *stream);

/* gpw_eval_mat without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, result and kernels as gpw_eval_mat; the
 * per-call scratch (the block-ordered copies of the level potentials) lives
 * in a fixed array of GPW_NOALLOC_SCRATCH_BYTES (128 MiB) per device, which
 * the library holds from the first plan built on that device until the
 * process ends.  Calls make no hipMalloc, hipMallocAsync or hipFree.  A plan
 * whose scratch (gpw_plan_info.scratch_bytes[GPW_OP_MAT]) exceeds that size
 * is rejected with GPW_EBUDGET before anything is enqueued.  Every call on a
 * device shares that device's array and overwrites it: calls that may
 * overlap on one device (different streams without ordering between them)
 * race and give undefined results; calls on one stream are ordered.  Nothing
 * of a previous call's contents is read. */
#define GPW_NOALLOC_SCRATCH_BYTES (128ull << 20)
gpw_status gpw_eval_mat_noalloc(gpw_plan_t plan, const double *const *v, double *M, void *stream);

/* Thread-local message describing the last failure in this thread. */
const char *gpw_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GPW_H */
