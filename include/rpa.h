/*
 * rpa.h -- C ABI of the MI355X (gfx950) hot path of the matrix-free
 * real-space RPA correlation energy by Lanczos quadrature and interpolation
 * (Haque, Chow, Shah, Medford, Pask, Suryanarayana).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Grid: periodic orthorhombic, n = (nx, ny, nz), N_d = nx*ny*nz, flat index
 *    (ix*ny + iy)*nz + iz (z fastest), spacing h_d = L_d / n_d, volume
 *    element dV = hx*hy*hz.
 *  - Pointers marked [dev] are device pointers on the current HIP device;
 *    [host] are host pointers.  The caller owns every buffer it passes in.
 *    The library owns only the resident copies it makes in rpa_setup and its
 *    internal workspaces, which it frees in rpa_destroy.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  All
 *    device work of a call is enqueued on that stream.  A call that fills an
 *    rpa_stats or a host output synchronises the stream before returning.
 *  - No C++ exception crosses the ABI.  Every call returns an rpa_status;
 *    rpa_last_error() gives a message for the calling thread.
 *  - Argument errors (RPA_E_ARG) have no side effects.  RPA_W_* are
 *    warnings: outputs are written and the counts are in rpa_stats.
 *  - A handle is not thread safe; calls on one handle must be serialised.
 */
#ifndef RPA_MI355X_H
#define RPA_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rpa_ctx* rpa_handle;

typedef enum {
  RPA_OK = 0,
  RPA_E_ARG = 1,        /* invalid argument; nothing was done */
  RPA_E_OOM = 2,        /* device allocation failed or exceeds hbm_budget */
  RPA_E_HIP = 3,        /* a HIP runtime call failed */
  RPA_E_STATE = 4,      /* handle unusable (e.g. after an earlier HIP error) */
  RPA_W_NOCONV = 16,    /* some Sternheimer solve hit stern_maxit */
  RPA_W_BREAKDOWN = 17  /* some Lanczos run broke down (T truncated) or a COCG
                           solve met p^T A p = 0 */
} rpa_status;

typedef enum {
  RPA_FP64 = 0,         /* Sternheimer COCG in FP64 throughout */
  RPA_FP32_REFINE = 1   /* FP32 stencil/Krylov, FP64 residual refinement */
} rpa_precision;

typedef enum {
  RPA_INTERP_NONE = 0,      /* stride must be 1 */
  RPA_INTERP_TRILINEAR = 1, /* 2 points per axis, periodic */
  RPA_INTERP_TRICUBIC = 2,  /* 4-point Lagrange per axis, periodic */
  RPA_INTERP_FOURIER = 3    /* spectrum zero-padding, Nyquist split evenly */
} rpa_interp;

/* Problem definition.  The Kohn-Sham eigenpairs of the FD Hamiltonian
 * H = -1/2 Lap_h + V_loc (+ V_nl) are inputs (paper: Background, Eq. 3). */
typedef struct {
  int32_t n[3];               /* grid points per axis, each >= 7 */
  double L[3];                /* cell lengths (bohr) */
  int32_t fd_radius;          /* must be 6: 12th-order central differences */
  int32_t n_occ;              /* N_s occupied orbitals, 1 <= N_s < N_d */
  const double* v_loc;        /* [dev] [N_d] local potential (Ha) */
  const double* psi;          /* [dev] [n_occ][N_d] orbitals, dV*sum(psi^2) = 1 */
  const double* eps;          /* [host] [n_occ] orbital energies (Ha) */
  /* optional separable nonlocal projectors, CSR over grid indices:
   * V_nl = dV * sum_p gamma_p chi_p chi_p^T.  n_proj = 0 disables. */
  int32_t n_proj;
  const int64_t* proj_ptr;    /* [host] [n_proj+1] */
  const int64_t* proj_idx;    /* [host] [proj_ptr[n_proj]] grid indices */
  const double* proj_val;     /* [host] [proj_ptr[n_proj]] chi values */
  const double* proj_gamma;   /* [host] [n_proj] coefficients (Ha) */
  /* solver settings */
  int32_t precision;          /* rpa_precision */
  double stern_tol;           /* relative residual ||b - A x||_2/||b||_2 (> 0) */
  int32_t stern_maxit;        /* cap on COCG iterations per solve (> 0) */
  int32_t batch;              /* Lanczos start vectors per launch; 0 = auto */
  uint64_t hbm_budget;        /* bytes the handle may allocate; 0 = no cap */
  /* tuning knobs (0 = automatic) */
  int32_t tile_y;             /* rows of the stencil tile (must divide ny) */
  int32_t slots_per_cu;       /* resident COCG workgroups per compute unit */
  double inner_tol;           /* RPA_FP32_REFINE: the FP32 recursive residual is replaced
                                 by the FP64 residual each time it drops by this
                                 factor (reliable update); in (0, 1), 0 = 0.001 */
  int32_t use_graph;          /* != 0: lanczos_energy_density captures the per-batch
                                 launch sequence (all Lanczos steps) into a hipGraph
                                 and replays it for later batches of the same size;
                                 per-launch COCG timing is then not recorded */
  int32_t fp32_maxit;         /* RPA_FP32_REFINE: FP32 COCG iterations a solve may take
                                 before it is handed to the FP64 COCG, which continues
                                 from the last folded FP64 solution with a budget of
                                 stern_maxit iterations; 0 = stern_maxit */
  double lanczos_breakdown;   /* Lanczos breakdown threshold (Algorithm 1 recurrence):
                                 T is truncated at the first beta_k <= lanczos_breakdown *
                                 max_i |alpha_i|, k < N_l; in [0, 1), 0 = 1e-13 */
  int32_t precond;            /* Sternheimer preconditioner (Conclusions and Future Work:
                                 preconditioned solves): 0 = none (plain COCG);
                                 1 = shifted kinetic operator M_n = -1/2 Lap_h + sigma_n,
                                 sigma_n = max(mean(V_loc) - eps_n, 1/4 Ha) - i omega,
                                 inverted exactly in the per-axis eigenbasis of the FD
                                 Laplacian; COCG then runs on z = M^-1 r with
                                 rho = r^T z and the stopping rule stays on ||b - A x||.
                                 Needs every n[d] <= 64 (RPA_E_ARG otherwise). */
  double precond_omega_min;   /* with precond = 1: only solves at frequencies omega with */
  double precond_omega_max;   /* min <= omega <= max are preconditioned (max = 0: no upper
                                 bound); the others run plain COCG in the same Lanczos
                                 step.  Both 0: every solve is preconditioned. */
  int32_t progress;           /* nonzero: lanczos_energy_density waits for each Lanczos
                                 step of a batch and prints one line per step to stderr
                                 (for long runs; eager batches only: a replayed graph
                                 prints nothing) */
  int32_t n_extra;            /* extra eigenpairs of H above the occupied ones that widen
                                 the Galerkin initial guess of every Sternheimer solve
                                 (Implementation section: the guess is the exact solution
                                 inside the projection space): x0 = sum_m psi_m (dV psi_m^T b)
                                 / (eps_m - eps_n - i omega) over the occupied and the extra
                                 states, so the initial residual has no component along the
                                 low unoccupied states that slow COCG at small omega.  The
                                 solutions and chi0 are unchanged (same stopping rule).
                                 0 = occupied states only; at most 1024. */
  const double* psi_extra;    /* [dev] [n_extra][N_d] eigenvectors, dV*sum(psi^2) = 1,
                                 orthogonal to the occupied ones (copied at setup) */
  const double* eps_extra;    /* [host] [n_extra] their eigenvalues (Ha) */
} rpa_setup_params;

typedef struct {
  int64_t n_systems;          /* Sternheimer solves performed */
  int64_t cocg_iters_total;   /* sum of COCG iterations over solves */
  int64_t cocg_iters_max;     /* largest per-solve iteration count */
  int64_t refine_cycles;      /* FP64 residual replacements (RPA_FP32_REFINE) */
  int64_t n_noconv;           /* solves that hit stern_maxit */
  int64_t n_breakdown;        /* COCG breakdowns + Lanczos truncations */
  double seconds;             /* host wall time of the call */
  int64_t n_fp64_fallback;    /* RPA_FP32_REFINE solves finished by FP64 COCG after the
                                 FP32 iteration stagnated, broke down or overflowed */
} rpa_stats;

/* Create a handle: copy V, psi (FP64 and FP32), eps to resident device
 * storage, build the per-axis eigenbasis of the periodic FD second
 * derivative for nu^1/2 (Implementation section, Kronecker formalism) and
 * the FD coefficients.  Enqueues on `stream` and synchronises it. */
rpa_status rpa_setup(const rpa_setup_params* params, void* stream, rpa_handle* out);

/* Free every device allocation of the handle (synchronises the device). */
rpa_status rpa_destroy(rpa_handle h);

/* Last error message of the calling thread ("" if none).  h may be NULL. */
const char* rpa_last_error(rpa_handle h);

/* [host] Gauss-Legendre frequency rule of Eq. 9 on [0, inf): nodes x_k of
 * the n_omega-point rule mapped by omega = (1+x)/(1-x), weights
 * W_k * 2/(1-x_k)^2 (Jacobian included).  omega, weight: [host] [n_omega]. */
rpa_status rpa_frequency_rule(int32_t n_omega, double* omega, double* weight);

/* y[v] = chi0(i omega) x[v] by Sternheimer (Eq. 4, Algorithm 1 inner loop):
 * per occupied n solve (H - eps_n - i omega) dpsi = -psi_n (.) u by COCG from
 * the Galerkin-projection guess (Implementation section), then
 * y = 4 sum_n psi_n (.) Re dpsi_n.  With symmetrized != 0 the result is
 * nu^1/2 chi0 nu^1/2 x (Eq. 8).  x, y: [dev] FP64 [nvec][N_d]; omega > 0. */
rpa_status chi0_apply(rpa_handle h, double omega, int32_t nvec, const double* x, double* y,
                      int32_t symmetrized, rpa_stats* st, void* stream);

/* chi0_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation and result as chi0_apply, but every workspace comes from
 * one fixed 128 MiB device array that the library holds on each GPU it runs
 * on until the process ends; the call makes no hipMalloc, hipFree or other
 * allocating call and records no timing events.  Vectors are processed in
 * the largest batches (at most the handle's batch) whose workspaces fit the
 * array.  RPA_E_ARG (nothing launched) when even one vector does not fit:
 * about 16 B x N_d x n_occ for the solutions plus one COCG workspace per
 * resident workgroup, so cells up to roughly 24 x 24 x 48 points with 32
 * orbitals.  All calls on one GPU share the array: calls that overlap in
 * time on one GPU (other streams, other threads, other handles) race and
 * must be serialised by the caller.  The array keeps the last call's
 * contents; everything a call needs zeroed it clears itself. */
rpa_status chi0_apply_noalloc(rpa_handle h, double omega, int32_t nvec, const double* x, double* y,
                              int32_t symmetrized, rpa_stats* st, void* stream);

/* Lanczos quadrature (Eqs. 6-7, Algorithm 1): for every pair (k, p)
 * d[k][p] = [f(T_m)]_11, f(x) = log(1-x) + x, T_m from m = n_lanczos steps of
 * Lanczos on nu^1/2 chi0(i omega_k) nu^1/2 started from e_j, j = point_idx[p],
 * with full reorthogonalisation.  omega: [host] [n_omega] (> 0);
 * point_idx: [host] [n_pts] in [0, N_d); d: [dev] FP64 [n_omega][n_pts]. */
rpa_status lanczos_energy_density(rpa_handle h, int32_t n_omega, const double* omega,
                                  int32_t n_pts, const int64_t* point_idx, int32_t n_lanczos,
                                  double* d, rpa_stats* st, void* stream);

/* Block Lanczos quadrature over groups of grid points (the block operations
 * for several points proposed in the Conclusions and Future Work section):
 * for each frequency the points are taken in consecutive groups of `block`
 * (the last group of a frequency holds the remainder), each group runs
 * n_lanczos steps of block Lanczos on nu^1/2 chi0(i omega_k) nu^1/2 from
 * Q_1 = [e_j ...] with full reorthogonalisation (two classical
 * Gram-Schmidt passes) and a thin QR per step, and
 * d[k][p] = [E_1^T f(T) E_1]_ii for the group's i-th point, T the block
 * tridiagonal matrix.  A group stops early (T truncated, RPA_W_BREAKDOWN)
 * when a diagonal entry of the QR factor is at most the handle's Lanczos
 * breakdown threshold times the largest |A_k| entry.  block = 1 is the
 * estimate of lanczos_energy_density.  Each group costs n_lanczos chi0
 * applications per point, as the scalar path does.  block in [1, 8],
 * n_lanczos * block <= 64 (RPA_E_ARG otherwise); arrays as for
 * lanczos_energy_density.  Batches run eagerly (no graph replay). */
rpa_status lanczos_energy_density_block(rpa_handle h, int32_t n_omega, const double* omega,
                                        int32_t n_pts, const int64_t* point_idx, int32_t n_lanczos,
                                        int32_t block, double* d, rpa_stats* st, void* stream);

/* Coarse-to-fine interpolation I_g (section "Interpolating Diagonal
 * Entries"): coarse values live on the origin-aligned sublattice of points
 * whose three indices are multiples of `stride` (stride divides every n_d).
 * coarse: [dev] FP64 [n_fields][N_d/stride^3] (x-major coarse layout);
 * fine: [dev] FP64 [n_fields][N_d]. */
rpa_status interpolate(rpa_handle h, int32_t kind, int32_t stride, int32_t n_fields,
                       const double* coarse, double* fine, void* stream);

/* Frequency integration of given coarse diagonals: interpolate each
 * omega's field, then E_c = 1/(2 pi) sum_k w_k sum_j dhat_j(omega_k) and
 * e(r) = 1/(2 pi) sum_k w_k dhat_k(r) / dV.  d_coarse: [dev]
 * [n_omega][N_d/stride^3]; weight: [host] [n_omega]; e_c: [host] scalar;
 * e_fine: [dev] [N_d] or NULL. */
rpa_status rpa_energy_from_coarse(rpa_handle h, int32_t n_omega, const double* weight,
                                  int32_t stride, int32_t kind, const double* d_coarse,
                                  double* e_c, double* e_fine, void* stream);

/* Algorithm 1 end to end: Lanczos quadrature at every coarse point for every
 * frequency, interpolation, frequency integration (E_c^(g) of the section
 * "Interpolating Diagonal Entries").  omega, weight: [host] [n_omega];
 * e_c: [host] (Ha); e_fine: [dev] [N_d] or NULL. */
rpa_status correlation_energy(rpa_handle h, int32_t n_omega, const double* omega,
                              const double* weight, int32_t stride, int32_t kind,
                              int32_t n_lanczos, double* e_c, double* e_fine,
                              rpa_stats* st, void* stream);

/* Building blocks exposed for tests and measurement ------------------------ */

/* y[v] = (H - shift_v) x[v] for complex vectors (interleaved re, im) in the
 * compute precision: x, y: [dev] [nvec][N_d][2] of double for RPA_FP64 or of
 * float for RPA_FP32_REFINE; shift_re, shift_im: [host] [nvec].  This is the
 * FD Hamiltonian of Eq. 3 with the complex shift of Eq. 4, the operator every
 * COCG iteration applies. */
rpa_status rpa_hamiltonian_apply(rpa_handle h, int32_t nvec, const double* shift_re,
                                 const double* shift_im, const void* x, void* y,
                                 int32_t precision, void* stream);

/* The Sternheimer solutions themselves (Eq. 4; Implementation section):
 * x[v][n] solves (H - eps_n - i omega) x = -psi_n (.) u[v] by COCG from the
 * Galerkin-projection guess, to the handle's stopping rule and precision --
 * the solves chi0_apply accumulates.  u: [dev] FP64 [nvec][N_d];
 * x: [dev] FP64 complex interleaved (re, im) [nvec][n_occ][N_d][2].  For
 * checking solves against their true residuals; omega > 0. */
rpa_status rpa_sternheimer_solve(rpa_handle h, double omega, int32_t nvec, const double* u,
                                 double* x, rpa_stats* st, void* stream);

/* y[v] = nu^(power/2) x[v], power 1 (nu^1/2) or 2 (nu); Kronecker form.
 * x, y: [dev] FP64 [nvec][N_d]. */
rpa_status rpa_coulomb_apply(rpa_handle h, int32_t power, int32_t nvec, const double* x,
                             double* y, void* stream);

/* Shifted kinetic preconditioner: y[v] = (-1/2 Lap_h + sigma_v)^-1 x[v], the
 * inverse taken exactly in the per-axis eigenbasis of the same 12th-order
 * FD Laplacian as in H (Kronecker form, as for the Coulomb operator, with
 * the diagonal 1/(kin + sigma_v)).  It is the building block of
 * preconditioned Sternheimer solves, which the Conclusions and Future Work
 * section names as a way to cut the COCG iteration counts; with
 * sigma_v = max(mean V_loc - eps_n, 1/4) - i omega it approximates
 * H - eps_n - i omega.
 * A plan is independent of any rpa_handle.  create: n[3] (each in
 * [7, 4096]) and L[3] > 0 (bohr), host; it uploads the 1D bases and the
 * kinetic diagonal on `stream` and waits for them.  apply: x, y [dev] FP64
 * complex, planar per vector: [nvec][2][N_d] (the N_d real parts, then the
 * N_d imaginary parts); y may alias x; sigma_re, sigma_im [host] [nvec].
 * The plan owns its workspaces (2 x 16 B x nvec x N_d, grown on demand) and
 * serves one stream at a time.  Errors: RPA_E_ARG (nothing launched) for a
 * bad grid, a null pointer or a sigma that is not finite with a positive
 * real part; RPA_E_OOM; RPA_E_HIP.  These calls report by status only and do
 * not set rpa_last_error. */
typedef struct rpa_kinetic_precond_s* rpa_kinetic_precond;
rpa_status rpa_kinetic_precond_create(const int32_t* n, const double* L, void* stream,
                                      rpa_kinetic_precond* out);
rpa_status rpa_kinetic_precond_apply(rpa_kinetic_precond p, int32_t nvec, const double* sigma_re,
                                     const double* sigma_im, const double* x, double* y,
                                     void* stream);
rpa_status rpa_kinetic_precond_destroy(rpa_kinetic_precond p);

/* Device time of the batched Sternheimer (COCG) launches of the last
 * chi0_apply / lanczos_energy_density / correlation_energy call (sum in ms,
 * measured with HIP events on the call's stream, and the launch count), or
 * of the last rpa_hamiltonian_apply launch; plus the launch shape.  Any
 * output pointer may be NULL.  For measurement only. */
rpa_status rpa_last_cocg_timing(rpa_handle h, double* ms, int32_t* launches, int32_t* grid,
                                int32_t* block, int32_t* tile_y);

/* The Sternheimer launch time of the last call split by kernel (ms, HIP
 * events): the plain persistent COCG launches (FP32 or FP64), the
 * preconditioned ones, and the FP64 launches that continue solves the FP32
 * launch handed over.  Any output may be NULL.  For measurement only. */
rpa_status rpa_last_cocg_split(rpa_handle h, double* ms_plain, double* ms_prec, double* ms_followup);

/* Per-frequency COCG iteration statistics of the last chi0_apply or
 * lanczos_energy_density call (the quantities of the paper's iteration
 * tables in the Performance section: mean, standard deviation, minimum and
 * maximum iterations per Sternheimer solve at each frequency).  One entry
 * per frequency argument of the call (omega[k] of lanczos_energy_density,
 * the single omega of chi0_apply), in that order: omega, the number of
 * solves, and their iteration counts' mean, standard deviation
 * (population), minimum and maximum, and the total of its FP64 reliable
 * updates (RPA_FP32_REFINE).  A solve handed from FP32 to FP64 COCG counts
 * once, with the iterations of both.  Outputs are [host] arrays of at
 * least `cap` entries (any may be NULL); n_out receives the number of
 * entries (also when it exceeds cap; then only cap are filled).  The
 * statistics were read back when the call returned: this synchronises
 * nothing. */
rpa_status rpa_last_iteration_stats(rpa_handle h, int32_t cap, double* omega, int64_t* count,
                                    double* mean, double* stdev, int64_t* min_iters,
                                    int64_t* max_iters, int64_t* refine_cycles, int32_t* n_out);

/* Launch-shape tuning (the handle's tile rows, workgroups per CU and start
 * vectors per launch).  Each candidate shape -- the whole (y, z) plane if it
 * fits a workgroup, else the four tallest row counts that divide n[1], with
 * one or two workgroups per CU where occupancy allows -- runs a fixed-work
 * probe: one-hot start vectors through nu^1/2 at omega = 0.69, every
 * Sternheimer system for exactly probe_iters COCG iterations (0: 16); the
 * fastest in system-iterations per second is kept.  batch becomes the most
 * start vectors (at most 64) whose workspaces for n_lanczos steps fit the
 * hbm_budget, or 80% of the free device memory when there is none.  Later
 * results change by rounding only: each system's reductions follow the
 * workgroup shape, which the tile rows set (workgroups per CU and batch do
 * not change any result bit).  Invalidates captured graphs.  out: host. */
typedef struct {
  int32_t tile_y;
  int32_t slots_per_cu;
  int32_t batch;
  int32_t n_tried;             /* shapes timed */
  double system_iters_per_s;   /* probe rate of the chosen shape */
} rpa_tune_result;
rpa_status rpa_autotune(rpa_handle h, int32_t n_lanczos, int32_t probe_iters,
                        rpa_tune_result* out, void* stream);

/* Release every workspace of the handle (resident problem data stays). */
rpa_status rpa_release_workspace(rpa_handle h);

/* Serving -------------------------------------------------------------------
 * Energy-density jobs (cell, one frequency omega, a block of points, N_l) are
 * queued and run by worker threads, each with its own HIP stream, so jobs
 * that arrive while others run overlap on the device.  A job is admitted
 * (oldest first) when a worker is idle and its workspace estimate fits the
 * HBM budget next to the resident cell data; a job that can never fit is
 * refused at submission with RPA_E_OOM.  Start vectors are batched inside a
 * job only, so a job's result is the same alone and in any mix.  Paper:
 * Algorithm 1 point loop; the jobs play the role of the per-rank point
 * blocks of the Implementation section. */
typedef struct rpa_server_s* rpa_server;
typedef struct {
  int32_t n_workers;          /* concurrent jobs (1..16) */
  uint64_t hbm_budget;        /* bytes; 0 = no cap */
  int32_t fake_executor_us;   /* > 0: jobs sleep this long instead of computing
                                 (host-only tests of admission and timing) */
} rpa_server_params;
typedef struct {
  int32_t status;             /* rpa_status of the job, -1 while pending */
  double t_submit, t_start, t_finish;   /* host steady clock, seconds */
  int64_t footprint;          /* admitted workspace estimate, bytes */
  rpa_stats stats;
} rpa_job_info;

rpa_status rpa_server_create(const rpa_server_params* p, rpa_server* out);
/* Register a cell (device data is copied; eps host) and return its id. */
rpa_status rpa_server_add_cell(rpa_server s, const rpa_setup_params* p, int32_t* cell_id);
/* Queue a job; pts [host] are copied; d_out [dev] FP64 [n_pts] receives d_j(omega). */
rpa_status rpa_server_submit(rpa_server s, int32_t cell_id, double omega, int32_t n_pts,
                             const int64_t* pts, int32_t n_lanczos, double* d_out,
                             int64_t* job_id);
/* Block until the job has finished; info (host) receives its record. */
rpa_status rpa_server_wait(rpa_server s, int64_t job_id, rpa_job_info* info);
/* Queue and memory state: jobs waiting and running, the workspace bytes of
 * admitted jobs, and the high-water mark of resident cell data plus admitted
 * workspaces since creation (the admission model's estimate).  Outputs are
 * host pointers; any may be NULL. */
rpa_status rpa_server_status(rpa_server s, int32_t* waiting, int32_t* running, uint64_t* in_use,
                             uint64_t* high_water);
/* Finish every queued job, stop the workers and free the cells. */
rpa_status rpa_server_destroy(rpa_server s);

#ifdef __cplusplus
}
#endif

#endif /* RPA_MI355X_H */
