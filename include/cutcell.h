/*
 * cutcell.h -- C ABI of the MI355X fourth-order cut-cell multigrid Poisson solver.
 *
 * Problem (paper Sec. 1 and Sec. 2.3): Delta phi = f in Omega, N phi = g on the
 * boundary, with Omega = R \ (union of ellipsoids), R = x_O + [0, n h]^3 and N the
 * Dirichlet (identity) or Neumann (outward normal derivative) operator.  The
 * unknowns are cell averages over the cut cells C_i ∩ Omega of the Cartesian grid
 * (Sec. 2.2); the discrete system is L phi = r := f - N g (Sec. 2.4), solved by
 * the modified multigrid of Sec. 5.3 (weighted Jacobi on regular cells, exact
 * LU-correction on FV-PLG cells, piecewise-constant transfers, LU bottom solve).
 *
 * Conventions
 *   - Cell arrays have n^3 entries (n of the level), linear index i + n (j + n k),
 *     x fastest, FP64.  On output exterior cells hold 0 and cells merged into a
 *     host cell hold 0 on coarse levels; on level 0 the solution of a merged cell
 *     is the host's value (cc_solve fills it).
 *   - Device pointers are caller-owned; the library never frees them.  Work runs
 *     on the stream given to cc_build (NULL: a library-created stream); calls that
 *     return host data synchronise that stream, others are asynchronous.
 *   - Every function returns CC_OK (0) or a negative status; cc_last_error() gives
 *     a thread-local message.  Inputs are validated on the host before any launch.
 *   - The problem handle owns geometry, per-level rows, factorizations and
 *     workspaces; it is not thread-safe (one caller at a time).
 */
#ifndef CUTCELL_H
#define CUTCELL_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CC_OK = 0,
  CC_EINVAL = -1,     /* bad argument */
  CC_ENOMEM = -2,     /* host or device allocation failed */
  CC_EDEVICE = -3,    /* HIP error, or no device (host-only handle) */
  CC_EGEOM = -4,      /* geometry outside the supported class (see cc_build) */
  CC_EPLG = -5,       /* no poised lattice for some cell */
  CC_ESINGULAR = -6,  /* a pivot below the threshold in a factorization */
  CC_ENOCONV = -7     /* max_iter V-cycles without reaching tol */
};

enum { CC_DIRICHLET = 0, CC_NEUMANN = 1, CC_ROBIN = 2 };
enum { CC_ELLIPSOID = 0, CC_TORUS = 1 };
enum { CC_FP64 = 0, CC_MIXED = 1 };

/* An ellipsoid { x : (x-c)^T R diag(axes^-2) R^T (x-c) <= 1 } removed from the box.
 * rot is row-major 3x3; its column j is the direction of semi-axis j. */
typedef struct cc_obstacle {
  double center[3];
  double axes[3];     /* CC_ELLIPSOID: semi-axes (> 0); ignored for CC_TORUS */
  double rot[9];      /* row-major orthonormal; column j is the direction of semi-axis j
                         (CC_TORUS: column 2 is the torus axis) */
  int bc;             /* CC_DIRICHLET, CC_NEUMANN or CC_ROBIN on this obstacle's surface */
  double robin[2];    /* (alpha, beta) of CC_ROBIN: alpha phi + beta dphi/dn = g, n outward of
                         Omega; the FV-PLG site row and its datum are scaled by
                         h / (|alpha| h + |beta|), so (1, 0) and (0, 1) are the Dirichlet and
                         Neumann rows (Sec. 2.3 boundary sites); ignored otherwise */
  int kind;           /* CC_ELLIPSOID (0): the quadric (x-c)^T A (x-c) = 1; CC_TORUS (1): the
                         solid torus of the paper's Problem 2 (Sec. 6), the points within
                         radii[1] of the circle of radius radii[0] around center in the
                         plane normal to rot's column 2, bounded by a quartic level set */
  double radii[2];    /* CC_TORUS: major R and minor r, R > r > 0; ignored otherwise */
} cc_obstacle;

/* Grid and domain (Sec. 2.2).  Walls ordered -x,+x,-y,+y,-z,+z; each CC_DIRICHLET,
 * CC_NEUMANN or CC_ROBIN. */
typedef struct cc_domain {
  int n;              /* cells per axis on the finest level */
  double origin[3];   /* x_O */
  double h;           /* cell size; must equal 1/n */
  int wall_bc[6];
  int n_obst;
  const cc_obstacle* obst;
  int inside;         /* 0: Omega = the box minus the obstacles; 1: Omega = the interior
                         of the one obstacle (n_obst must be 1; the walls then carry no
                         unknowns) */
  double wall_robin[6][2]; /* (alpha, beta) of each CC_ROBIN wall: alpha phi + beta dphi/dn = g
                         on the wall, n out of the box; the two ghost cells beyond it are
                         filled from the quartic that matches the 4 nearest cell averages
                         and the condition (Sec. 2.3 ghost formulas, with the Robin face
                         condition in place of the Dirichlet or Neumann one), so (1, 0)
                         and (0, 1) give the Dirichlet and Neumann walls; FV-PLG wall sites
                         are scaled as on obstacles; ignored for other walls */
} cc_domain;

/* Method parameters (Sec. 4.2 theta; Sec. 5.3 omega, nu1, nu2, eps, I_max). */
typedef struct cc_params {
  double theta;       /* merging threshold, default 0.1 */
  double omega;       /* Jacobi weight, default 0.8 */
  int nu1, nu2;       /* smoothing steps, default 3, 3 */
  int n_min;          /* coarsen while n/2 >= n_min, default 16 */
  int max_iter;       /* I_max, default 200 */
  double tol;         /* eps on max-norm relative residual, default 1e-10 */
  int precision;      /* CC_FP64 or CC_MIXED (FP32 V-cycles, see cc_solve) */
  int leaf_size;      /* nested-dissection leaf size, default 64 */
  int device;         /* HIP device ordinal; -1 builds a host-only handle */
  int use_graph;      /* capture the V-cycle in a hipGraph (default 1) */
  int krylov;         /* 0 (default): the plain multigrid iteration; k > 0: restarted
                         flexible GMRES(k) in FP64 preconditioned by one V-cycle per
                         iteration (an FP32 V-cycle with CC_MIXED); converges also
                         where the plain iteration does not contract */
  double pivot_tol;   /* factorizations (Sec. 5.3 LU-correction and bottom solve): a pivot
                         below pivot_tol times the largest entry of the factored matrix is
                         CC_ESINGULAR; default 1e-14, must lie in (0, 1e6] */
  int fit_on_device;  /* 1 (default): the FV-PLG weighted least-squares fits (Sec. 2.3) run on
                         the GPU in FP64 (one wavefront per row, Householder QR); 0: on the
                         host (a host-only handle always fits on the host) */
} cc_params;

/* Analytic fields (problem data).  data layout by kind:
 *   CC_FIELD_POLY    n_terms x (a0, a1, a2, coef): sum coef x^a0 y^a1 z^a2, degree <= 4
 *   CC_FIELD_SINPROD (amp, k0, k1, k2, p0, p1, p2): amp prod_d sin(k_d x_d + p_d)
 *   CC_FIELD_EXPCOS  (amp, a, b, c, p): amp exp(a x + b y) cos(c z + p)
 *   CC_FIELD_GAUSS   n_terms x (amp, mu0, mu1, mu2, sigma)
 *   CC_FIELD_XSINEXP (amp): amp x sin(y) e^z (harmonic; the function of the paper's
 *                    geometry accuracy test, Sec. 6.1, with amp = 10)
 * The library copies what it needs; data may be freed after the call. */
enum { CC_FIELD_ZERO = 0, CC_FIELD_POLY = 1, CC_FIELD_SINPROD = 2, CC_FIELD_EXPCOS = 3,
       CC_FIELD_GAUSS = 4, CC_FIELD_XSINEXP = 5 };
enum { CC_VALUE = 0, CC_LAPLACIAN = 1 };
typedef struct cc_field {
  int kind;
  int n_terms;
  const double* data;
} cc_field;

typedef struct cc_problem cc_problem;

#define CC_HISTORY_MAX 256
typedef struct cc_solve_info {
  int iterations;                       /* V-cycles applied */
  double rel_residual;                  /* final max|r - L phi| / max|r| */
  int history_len;
  double history[CC_HISTORY_MAX];       /* relative residual before each V-cycle */
  double seconds;                       /* wall time of the call */
} cc_solve_info;

typedef struct cc_level_info {
  int n;
  long long n_unknowns;   /* cells carrying an unknown (hosts included) */
  long long n_phi2;       /* FV-PLG rows (N_2) */
  long long n_cut;        /* cut cells */
  long long n_merged;     /* cells absorbed into a host */
  long long lu_vars;      /* variables of the level's factorization */
  long long lu_entries;   /* FP64 entries of the stored supernodal factors */
  int lu_nodes;           /* supernodes */
  int lu_depth;           /* levels of the supernode tree */
  double setup_seconds;   /* host set-up of the level: geometry, merging, rows, LU factorization */
  int lu_subtree_cut;     /* device sweeps: heights below this run as one launch of subtrees */
  int lu_subtrees;        /* number of those subtrees (0: one launch per height throughout) */
  int lu_entries_per_lane;/* device sweeps: factor entries per lane of a row (chosen at build) */
  double lu_tune_ms[10];  /* the build-time trials: ms of one FP64 LU solve with 2^(k+1) entries
                             per lane at [2k] (one launch per height) and [2k+1] (subtree launch
                             for the low heights); 0 where not tried; the fastest over the
                             wavefront caps */
  int lu_waves_cap;       /* device sweeps: wavefronts per height launch at most (chosen at build;
                             0: no cap) */
  int stencil_march;      /* regular-row kernels (SMO-1, residual, apply): 0 one cell per thread,
                             1 z-marching, 2 z-marching in the XCD-aware tile order (chosen at build
                             by timing, or cc_set_stencil_schedule) */
  int stencil_planes;     /* z-planes per workgroup of the marching kernels */
  double stencil_tune_us[9]; /* the build-time trials: us per FP64 SMO-1 sweep (the best of 3
                             interleaved rounds of 5 sweeps), one cell per thread at [0], marching
                             with 4, 8, 16, 32 planes at [1..4], the same in the XCD-aware order
                             at [5..8] (0: not tried); the smallest decides */
  long long n_near;       /* phi_1 cells within 3 cells of a phi_2 cell along an axis: the near
                             SMO-1 sweep (cc_set_overlap) */
  double lu_seconds;      /* the share of setup_seconds spent assembling, ordering and factoring
                             the level's LU matrix: L on the bottom level (the paper's setup of the
                             bottom solver), L22 on the others (its setup of the LU-correction),
                             Table 4 */
} cc_level_info;

/* Fill p with the defaults listed above. */
void cc_default_params(cc_params* p);

/* Build geometry, merging, rows and factorizations of every level (Secs. 2-5):
 * classification and moments (exact ellipsoids), cell merging, the phi_1/phi_2
 * split, FV-PLG stencils and least-squares rows, nested dissection and the LU of
 * L22 on levels m < M and of L on level M, then the device upload.
 * Supported geometry: every obstacle's bounding sphere keeps the wall layer free
 * and meets no cell that another obstacle's bounding sphere meets, on every
 * level (else CC_EGEOM).  8 <= n <= 1290 (cell indices are 32-bit; else
 * CC_EINVAL).  stream: hipStream_t or NULL.  *out owned by the caller until
 * cc_destroy. */
int cc_build(const cc_domain* dom, const cc_params* prm, void* stream, cc_problem** out);

int cc_num_levels(const cc_problem* p);
int cc_get_level_info(const cc_problem* p, int level, cc_level_info* info);

/* r = f - N g on level 0 (Sec. 2.4): cell averages of f (f_mode CC_VALUE) or of
 * Delta f (CC_LAPLACIAN) over each unknown's cell, minus the wall-ghost and FV-PLG
 * boundary-site terms of the data g (Dirichlet: the value of g; Neumann: the
 * outward normal derivative of g).  r_dev: device, n^3. */
int cc_assemble_rhs(cc_problem* p, const cc_field* f, int f_mode, const cc_field* g,
                    double* r_dev);
/* The same on level `level` (its cells, rows and boundary sites; r_dev has n_m^3
 * doubles): the right-hand sides of the coarse levels for cc_fmg. */
int cc_assemble_rhs_level(cc_problem* p, int level, const cc_field* f, int f_mode, const cc_field* g,
                          double* r_dev);

/* cc_assemble_rhs_level for nf problems on the same geometry at once: field k
 * is f[k] (f_mode as above) with boundary data g[k] (g_per_field = 1) or g[0]
 * for all (g_per_field = 0; g may be NULL: zero data).  Each cut cell's
 * quadrature rule is built once for all fields.  r_dev: nf arrays of n_m^3
 * doubles at stride n_m^3 (device).  Errors: CC_EINVAL. */
int cc_assemble_rhs_batched(cc_problem* p, int level, int nf, const cc_field* f, int f_mode, const cc_field* g,
                            int g_per_field, double* r_dev);

/* Multigrid (Sec. 5.3): phi <- phi + VCycle(r - L phi) until the max-norm relative
 * residual < tol or max_iter.  phi_dev is the initial guess on entry and the
 * solution on exit (merged cells hold their host's value).  info may be NULL.
 * Returns CC_ENOCONV (with phi holding the last iterate) if tol is not reached.
 *
 * precision CC_MIXED (set at cc_build) runs the same iteration as defect
 * correction: the residual s = r - L phi, its max-norm and the update of phi
 * stay FP64; each V-cycle runs in FP32 on d = s / max|s| (smoothers, FV-PLG rows,
 * LU-correction with FP32 copies of the factors, transfers), except the bottom
 * solve, which stays FP64; then phi += max|s| * e.  The stopping test is the FP64
 * one, so the result meets the same tolerance.  FP32 copies of the rows and
 * factors are made at cc_build; FP32 work arrays at the first mixed solve. */
int cc_solve(cc_problem* p, const double* r_dev, double* phi_dev, cc_solve_info* info);

/* Several problems (geometries, sizes) at once: problem i solves L phi_i = r_i as
 * cc_solve does, each on its own host thread and its own stream (every handle
 * must have been built with a distinct stream, e.g. NULL: a library stream), so
 * the problems' kernels run concurrently.  info, if not NULL, has nprob entries.
 * Returns CC_OK, else the status of a failing problem (message names it). */
int cc_solve_multi(int nprob, cc_problem* const* probs, const double* const* r_dev,
                   double* const* phi_dev, cc_solve_info* info);

/* The same as cc_solve_multi for the plain multigrid iteration (Sec. 5.3;
 * FP64 or CC_MIXED per problem, krylov 0), from the calling thread alone: after
 * each problem's prologue, every iteration launches each unconverged problem's
 * captured outer step (a hipGraph kept by the problem) on the problem's own
 * stream, then reads back all their residual norms; problems on different
 * streams overlap on the device, problems sharing a stream run one after the
 * other.  The problems live on one device and appear once each.  info[i]
 * (optional) as for cc_solve, with the whole call's time.  Errors: CC_EINVAL
 * (empty list, null or host-only problem, two devices, a repeated problem,
 * krylov > 0), CC_ENOCONV (some problem hit max_iter; all outputs filled),
 * CC_EDEVICE. */
int cc_solve_multi_graph(int nprob, cc_problem* const* probs, const double* const* r, double* const* phi,
                         cc_solve_info* info);

/* Switch the precision of later cc_solve / cc_solve_batched calls (CC_FP64 or
 * CC_MIXED); the build-time value is cc_params.precision. */
int cc_set_precision(cc_problem* p, int precision);

/* Overlap of SMO-1 with the LU-correction (Sec. 5.3 smoothing steps; default
 * off): every SMO-1 that follows an SMO-2 runs as a far sweep (the phi_1 rows
 * that read no phi_2 cell, and the cells without an unknown) on a side stream,
 * concurrently with that SMO-2, and a near sweep (cc_level_info.n_near cells)
 * after it; the next SMO-2 waits for both.  Same arithmetic, same result; on = 0
 * runs every SMO-1 as one sweep.  Waits for the problem's stream and drops
 * captured iterations.  Errors: CC_EINVAL. */
int cc_set_overlap(cc_problem* p, int on);

/* Switch between the plain multigrid iteration (0) and GMRES(k) preconditioned
 * by the V-cycle (k in 1..64) for later solves; build-time value cc_params.krylov. */
int cc_set_krylov(cc_problem* p, int krylov);

/* Replace the build-time choice of the device sweep schedule of `level`'s
 * factorization (the LU-correction of Sec. 5.3 on levels m < M, the bottom
 * solve on level M): entries_per_lane in {2, 4, 8, 16, 32} sets the lanes per
 * row of a task, subtree = 1 runs the low heights as one launch of subtrees
 * (only where cc_level_info.lu_subtrees > 0), subtree = 2 runs each sweep
 * of a single right-hand side as one launch (opt-in; slower than the
 * per-height launches on MI355X; every wait bounded in time, and a wait that
 * gave up makes the next cc_solve, cc_vcycle, cc_fmg, cc_smo2,
 * cc_bottom_solve or cc_time_kernel fail with CC_EDEVICE), waves_cap caps the
 * wavefronts of a height launch, or of the one launch (0: no cap; else at
 * least 4).  Waits for the problem's
 * stream, rebuilds the task lists (device allocation) and drops captured
 * iterations.  The solution does not depend on the schedule beyond rounding.
 * Errors: CC_EINVAL for a bad level or value. */
int cc_set_lu_schedule(cc_problem* p, int level, int entries_per_lane, int subtree, int waves_cap);

/* Replace the build-time schedule of the regular-row kernels (SMO-1, the
 * outer residual and the operator apply of Sec. 5.3, evaluated on the fly from
 * the cell types) on `level` (-1: every level): march = 1 runs the z-marching
 * kernels (a workgroup takes a 64 x 4 column tile through `planes` consecutive
 * z-planes; 0: the build's count, else 1..n), march = 2 the same with the
 * tiles handed to the 8 XCDs in contiguous ranges (z-blocks of a column on one
 * XCD, one after the other), march = 0 one cell per thread, march = -1 the
 * build's choice.  At cc_build the library times one cell per thread and both
 * marching orders with 4, 8, 16 and 32 planes on the device and keeps the
 * fastest (cc_level_info.stencil_*).  The
 * result does not depend on the schedule (same arithmetic order).  Waits for
 * the problem's stream and drops captured iterations.  Errors: CC_EINVAL. */
int cc_set_stencil_schedule(cc_problem* p, int level, int march, int planes);
/* The schedule in force on `level`: *march (0 or 1) and *planes. */
int cc_get_stencil_schedule(const cc_problem* p, int level, int* march, int* planes);

/* Several right-hand sides on one geometry (with krylov > 0 they are solved one
 * after the other): r_dev and phi_dev hold nrhs arrays of
 * n^3 at a stride of n^3 (batch-major).  Groups of up to CC_BATCH_MAX
 * right-hand sides run together: every kernel of the V-cycle processes the whole
 * group in one launch, and the LU-correction reads each factor entry once for
 * the group.  A group iterates until every member meets tol (members that meet it
 * early keep receiving V-cycles).  info, if not NULL, has nrhs entries; each
 * member's iterations count the V-cycles of its group.  Work arrays for a group
 * are allocated at the first call (3 arrays per level of min(nrhs, CC_BATCH_MAX)
 * * n_m^3 values in the working precision, plus one FP64 array of the finest
 * level), grown by a later call with more right-hand sides, and kept until
 * cc_destroy.  Returns CC_ENOCONV if some member misses tol. */
#define CC_BATCH_MAX 64
int cc_solve_batched(cc_problem* p, int nrhs, const double* r_dev, double* phi_dev, cc_solve_info* info);

/* Parity hooks, one per step of the V-cycle, on level `level` arrays (n_m^3):
 *   cc_apply:      y = L x on unknown cells, 0 elsewhere (Sec. 2.4)
 *   cc_residual:   s = r - L x on unknown cells; *maxabs = max |s| (host)
 *   cc_smo1:       one SMO-1 sweep on phi_1 cells: e <- e + omega D^-1 (s - L e)
 *   cc_smo2:       one SMO-2 LU-correction: e_2 <- L22^-1 (s_2 - L21 e_1)
 *   cc_restrict:   s_c = 2^-3 sum over children of (s - L e) on phi_1 children
 *   cc_prolong_add: e_f += e_c(parent) on phi_1 cells of level `level`
 *   cc_bottom_solve: e = L^(M)^-1 s on the coarsest level
 *   cc_vcycle:     e = VCycle(s) from level `level` down (e is overwritten)
 * Each hook synchronises the problem's stream before it returns. */
int cc_apply(cc_problem* p, int level, const double* x_dev, double* y_dev);
int cc_residual(cc_problem* p, int level, const double* r_dev, const double* x_dev,
                double* s_dev, double* maxabs);
int cc_smo1(cc_problem* p, int level, const double* s_dev, double* e_dev);
int cc_smo2(cc_problem* p, int level, const double* s_dev, double* e_dev);
int cc_restrict(cc_problem* p, int level, const double* s_dev, const double* e_dev,
                double* sc_dev);
int cc_prolong_add(cc_problem* p, int level, const double* ec_dev, double* ef_dev);
int cc_bottom_solve(cc_problem* p, const double* s_dev, double* e_dev);

/* Full multigrid (Sec. 5, algorithm FMG), FP64 whatever cc_params.precision:
 * phi_dev (n^3 doubles on the device, overwritten) receives an approximation
 * of L phi = r_dev built from the coarsest level up with `cycles` V-cycles per
 * level (1..64); pass it to cc_solve as the initial guess to continue to the
 * tolerance.  coarse_rhs (host array of M device pointers, level m's at
 * [m - 1], n_m^3 doubles each) gives each coarser level's right-hand side,
 * normally the same problem assembled there (cc_assemble_rhs_level); if NULL
 * they are restricted from r_dev by 2^-3 times the sum over the children that
 * carry an unknown, which is consistent only when the boundary data vanish
 * (the boundary terms of r scale with the fine h).  The coarser solution is
 * interpolated trilinearly in the cell centres over the coarse cells that
 * carry an unknown (weights renormalised).  Cells merged into a host hold the
 * host's value, cells without an unknown 0.  The first call allocates the
 * coarse levels' arrays.  Synchronizes the problem's stream.
 * Errors: CC_EINVAL. */
int cc_fmg(cc_problem* p, const double* r_dev, const double* const* coarse_rhs, double* phi_dev, int cycles);
/* cc_fmg without any device allocation, for callers that cannot allocate
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation and result as cc_fmg, with the coarse
 * levels' solution arrays (and, when coarse_rhs is NULL, their restricted
 * right-hand sides) carved from one fixed device array per GPU of
 * 6 Mi doubles (48 MiB), held until the process ends.  Problems whose coarse
 * levels need more (sum over levels m >= 1 of n_m^3 doubles, twice that
 * without coarse_rhs; 256^3 fits, 512^3 does not) get CC_EINVAL, and nothing
 * runs.  Every array of the scratch is written in full before it is read, so it
 * needs no clearing between calls.  All calls on one GPU share the array:
 * calls that overlap on one GPU (other streams, other host threads) race and
 * must be serialised by the caller.  The V-cycles use the handle's work
 * arrays (allocated at cc_build).  Synchronizes the problem's stream.
 * Errors: CC_EINVAL, CC_EDEVICE. */
int cc_fmg_noalloc(cc_problem* p, const double* r, const double* const* coarse_rhs, double* phi, int cycles);
/* cc_fmg for nrhs right-hand sides at a stride of n^3 (groups of up to
 * CC_BATCH_MAX share each level's V-cycles, as in cc_solve_batched);
 * coarse_rhs[m - 1] then holds nrhs arrays of n_m^3 doubles.  Start
 * cc_solve_batched from phi_dev.  Errors: CC_EINVAL. */
int cc_fmg_batched(cc_problem* p, int nrhs, const double* r_dev, const double* const* coarse_rhs, double* phi_dev,
                   int cycles);
/* The two FMG transfers between level and level + 1 (parity hooks):
 * sc = restriction of the right-hand side s; xf = interpolation of xc. */
int cc_fmg_restrict(cc_problem* p, int level, const double* s_dev, double* sc_dev);
int cc_fmg_prolong(cc_problem* p, int level, const double* xc_dev, double* xf_dev);
int cc_vcycle(cc_problem* p, int level, const double* s_dev, double* e_dev);

/* The paper's boundary fitting (Sec. 3.1) on the cut cells of `level`, as a
 * check of the exact geometry the solver uses (the geometry accuracy test of
 * Sec. 6.1, Table 1).  Per cut cell, in ascending cell index
 * (cc_level_info.n_cut cells): points of the exact boundary inside the cell
 * (the surface nodes of a 4-point-per-piece height-function rule), the height
 * axis w of the patch's mean normal (u < v the other two), the least-squares
 * quadratic W = a U^2 + b U V + c V^2 + d U + e V + g in the cell-centred
 * coordinates scaled by h (minimum-norm; singular values below 1e-12 of the
 * largest dropped), and the fitted region {s (W - p(U, V)) > 0}, s putting
 * Omega's side positive, integrated with the same 12-point height-function
 * rule as the exact one.  Outputs (host arrays, caller-owned, each may be
 * NULL): cell[n_cut], axis[n_cut] (-1 where the patch gives fewer than 6
 * points; its other outputs are NaN), coef[6 n_cut] (a, b, c, d, e, g), and
 * exact[4 n_cut], fitted[4 n_cut]: volume, patch area, the average of u over
 * the region and over the patch.  Host-only; works on host-only handles.
 * Errors: CC_EINVAL (bad level or field). */
int cc_fit_patches(const cc_problem* p, int level, const cc_field* u, int* cell, int* axis, double* coef,
                   double* exact, double* fitted);

/* Host copies of a level's integer decisions and rows (Sec. 2.2-2.4), for
 * exact comparison.  Any pointer may be NULL.
 *   type[n^3]: 0 no unknown, 1 phi_1, 2 phi_2;  host[n^3]: -1 exterior, else the
 *   cell whose unknown covers this cell;  volfrac[n^3]: |C_i ∩ Omega| / h^3.
 *   PLG rows: row_cell[N2], cols[N2*35] (cell indices), vals[N2*35]. */
int cc_export_cells(const cc_problem* p, int level, unsigned char* type, int* host,
                    double* volfrac);
int cc_export_plg(const cc_problem* p, int level, int* row_cell, int* cols, double* vals);

/* Host check of a level's factorization (L22 on levels m < M, L on the
 * coarsest level): solves with the stored supernodal factors for a random
 * right-hand side and returns max|A x - b| / max|b|.  Diagnostic only. */
int cc_selfcheck_lu(const cc_problem* p, int level, double* rel_residual);

/* Supernode structure of a level's factorization (postorder): first variable,
 * size p, number of later variables q, height in the tree (leaves 0) and parent
 * (-1 for roots).  Arrays hold lu_nodes entries (cc_level_info); NULL skips. */
int cc_export_lu_nodes(const cc_problem* p, int level, int* base, int* np, int* nq, int* height,
                       int* parent);

/* Timing hook for roofline figures: average device time in ms of `reps`
 * back-to-back launches (HIP events on the problem's stream) of
 *   CC_TIME_SMO1      the level-0 SMO-1 kernel, FP64 (25 bytes per cell: e, s,
 *                     the cell type and e')
 *   CC_TIME_SMO1_F32  the same in FP32 (13 bytes per cell)
 *   CC_TIME_LU        the level-0 LU-correction sweeps (all forward and backward
 *                     launches of one correction, FP64)
 *   CC_TIME_LU_F32    the same with the FP32 factors
 *   CC_TIME_COPY      a plain copy of n^3 doubles (16 bytes per cell), the
 *                     reference for memory-traffic counters
 * *bytes (may be NULL) receives the algorithmic bytes moved per launch (per
 * correction for the LU sweeps).  The timed kernels overwrite the library's
 * level-0 work arrays only. */
enum { CC_TIME_SMO1 = 0, CC_TIME_SMO1_F32 = 1, CC_TIME_LU = 2, CC_TIME_LU_F32 = 3, CC_TIME_COPY = 4 };
int cc_time_kernel(cc_problem* p, int which, int reps, double* ms_per_launch, double* bytes);

void cc_destroy(cc_problem* p);
const char* cc_last_error(void);

/* ---------------------------------------------------------------------------
 * Learned initial guess (an addition on top of the paper's method: the
 * multigrid solve still decides the result, the network only supplies phi_0).
 *
 * A 3D U-Net of `depth` levels (3 or 4) with base width C (16 or 32; encoder
 * channels C on the upper levels, 2C on the two coarsest): two input channels
 * (the scaled right-hand side and a geometry channel), one output channel,
 * 3x3x3 convolutions with bias, 2x2x2 average pooling, nearest upsampling and
 * skip connections (see the architecture in csrc/net.hip; depth 4 with C = 32
 * has 581k parameters).  Weights are kept in FP32 with a BF16 copy;
 * activations are BF16; convolutions accumulate in FP32 on MFMA (gfx950's
 * double-K BF16 instruction where the input channels allow).  Tensors are
 * channel-last:
 *   x:      nb x n^3 x 2 FP32 (device), voxel i + n (j + n k)
 *   y, t:   nb x n^3 FP32 (device)
 *   mask:   nb x n^3 bytes (device), nonzero where the loss counts
 * n must be a multiple of 2^(depth+1).  Work runs on `stream` (NULL: the default
 * stream); every call synchronises it.  Parameters are one flat FP32 array in
 * layer order, each layer W[27][Cout][Cin] (tap = (dz+1) 9 + (dy+1) 3 + (dx+1))
 * then bias[Cout]; the first layer has 16 input slots (2 used) and the last 16
 * outputs (1 used; the others are held at zero). */
typedef struct cc_net cc_net;
int cc_net_create(int base_channels, int depth, unsigned long long seed, void* stream, cc_net** out);
long long cc_net_num_params(const cc_net* net);
int cc_net_get_params(const cc_net* net, float* host);
int cc_net_set_params(cc_net* net, const float* host);
/* y = net(x) */
int cc_net_forward(cc_net* net, int n, int nb, const float* x_dev, float* y_dev);
/* loss = sum over mask of (net(x) - t)^2 / count(mask); gradients of the loss
 * with respect to the parameters are left in the network (for cc_net_adam_step)
 * and, if grad_host is not NULL, copied to it (cc_net_num_params floats). */
int cc_net_loss_grad(cc_net* net, int n, int nb, const float* x_dev, const float* t_dev,
                     const unsigned char* mask_dev, double* loss, float* grad_host);
/* one Adam update with the gradients of the last cc_net_loss_grad */
int cc_net_adam_step(cc_net* net, float lr, float beta1, float beta2, float eps);
void cc_net_destroy(cc_net* net);

/* Training pairs for the network from nrhs solved problems on this geometry
 * (r_dev, phi_dev: nrhs arrays of n^3 doubles at stride n^3 on the device: the
 * right-hand sides and their solutions), on level `level` (m^3 cells): per pair
 * b and level cell V,
 *   x[b][V] = (mean of r_b over V's fine cells / max|r_b|, volume fraction of V),
 *   t[b][V] = phi_scale * (mean of phi_b over V's fine cells with an unknown) / max|r_b|,
 *   mask[b][V] = 1 where V holds a fine cell with an unknown, else 0;
 * x_dev: nrhs x m^3 x 2 floats, t_dev: nrhs x m^3 floats, mask_dev: nrhs x m^3
 * bytes (device).  Synchronises the problem's stream.  Errors: CC_EINVAL. */
int cc_net_pairs(cc_problem* p, int level, int nrhs, const double* r_dev, const double* phi_dev, double phi_scale,
                 float* x_dev, float* t_dev, unsigned char* mask_dev);

/* Initial guess for cc_solve from the network, evaluated on level `level` of
 * the problem (m cells per axis, a multiple of 2^(depth+1)): the features are the mean of
 * r over each level cell scaled by 1 / max|r| and the cell's volume fraction;
 * the output y is turned into phi = y * max|r| / phi_scale at the level cells
 * and interpolated trilinearly to the level-0 unknowns (other cells get 0).
 * phi_scale is the factor the targets were scaled by in training (targets =
 * phi_scale * phi / max|r|).  r_dev, phi_dev: level-0 arrays (n^3, device).
 * Synchronises the problem's stream; the network runs on its own stream. */
int cc_learned_guess(cc_problem* p, cc_net* net, int level, double phi_scale, const double* r_dev,
                     double* phi_dev);

/* The network's output fed in at the coarse level, as the iterate the full
 * multigrid ascent (Sec. 5, algorithm FMG) starts from: the features of r on
 * `level` (as for cc_learned_guess), the network's prediction scaled by
 * max|r| / phi_scale there (0 on cells without an unknown), `cycles` V-cycles on
 * that level, then for each finer level the FMG interpolation and `cycles`
 * V-cycles, as cc_fmg does above its coarsest level.  coarse_rhs as for cc_fmg
 * (NULL: restrictions of r).  level in [1, levels - 1), cycles in [1, 16].
 * Device arrays; phi (n^3) receives the level-0 iterate.  Errors: CC_EINVAL,
 * CC_EDEVICE. */
int cc_learned_fmg(cc_problem* p, cc_net* net, int level, double phi_scale, const double* r_dev,
                   const double* const* coarse_rhs, double* phi_dev, int cycles);

#ifdef __cplusplus
}
#endif
#endif /* CUTCELL_H */
