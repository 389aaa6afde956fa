/*
 * dsweep -- diagonal-sweeping source-transfer domain decomposition for the
 * PML-truncated Helmholtz equation, on one AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Every pointer argument ending in "_dev" is device memory owned by
 * the caller; every pointer ending in "_host" is host memory owned by the
 * caller.  The plan owns everything it allocates (factors, coefficient arrays,
 * sweep and Krylov workspaces) and frees it in dsd_destroy.
 *
 * Layouts.
 *   Global grid: the physical cells n[0] x n[1] (x n[2]) plus `pml` cells on
 *   every side, N_g = prod_a (n[a] + 2 pml) cells, x fastest.  A batch of
 *   complex vectors is [nrhs][N_g], complex values interleaved (re, im) in
 *   FP64 (complex128).  This is torch's (nrhs, ny, nx) complex128 layout.
 *   The medium is m = 1/c^2 on the physical cells only, FP64, x fastest; the
 *   library extends it into the PML by clamping.
 *   Right-hand sides are J-scaled sources on the global grid (equal to the
 *   source itself wherever the source lies inside the physical box).
 *
 * Streams.  `stream` is a hipStream_t (NULL = the default stream).  Calls are
 * ordered on that stream.  Calls that return host values (iteration counts,
 * residuals, the misfit) synchronise the stream before returning; the others
 * are asynchronous.
 *
 * Errors.  0 = success.  Negative codes are errors; outputs are then
 * unspecified.  DSD_NOT_CONVERGED (> 0) means outputs, iteration counts and
 * residuals are valid but the tolerance was not met.  dsd_strerror() gives a
 * message for any code; dsd_last_error_detail() adds context (which
 * subdomain, which check) for the last failing call of this thread.
 */
#ifndef DSWEEP_H
#define DSWEEP_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DSD_OK = 0,
  DSD_NOT_CONVERGED = 1,
  DSD_EINVAL = -1,     /* bad shape, overlap < 3, a part smaller than the overlap, an
                          interior part smaller than 2*overlap-2 ...                   */
  DSD_ENOMEM = -2,     /* device allocation failed                                    */
  DSD_EHIP = -3,       /* HIP runtime error                                           */
  DSD_EPIVOT = -4,     /* zero pivot in a subdomain factorisation                     */
  DSD_ENOTFINITE = -5  /* NaN/Inf in a residual norm                                  */
};

enum { DSD_C64 = 1, DSD_C128 = 2 };   /* precision of factors and sweeps */

typedef struct dsd_plan dsd_plan;     /* opaque */

typedef struct {
  int dim;               /* 2 or 3                                                     */
  int n[3];              /* physical cells per axis (n[2] ignored in 2D)               */
  double h;              /* cell size                                                  */
  int pml;               /* PML cells, global and around every subdomain               */
  int overlap;           /* overlap d in cells, >= 3                                   */
  int parts[3];          /* subdomains per axis (N_x, N_y[, N_z])                     */
  double sigma0_delta;   /* S in sigma(t) = (S/W) (t/W)^2, W = pml*h; 60 if <= 0       */
  int precision;         /* DSD_C64 or DSD_C128                                        */
  int max_rhs;           /* largest batch any later call will pass                     */
  int rhs_per_group;     /* RHS handled by one workgroup in the subdomain solves;
                            0 = let the library choose                                 */
  int schedule;          /* 0: launch every solve as soon as the solves it depends on
                               are done (dependency levels of Algorithms 3.1 / 4.1);
                            1: the anti-diagonal steps of each sweep in order.  Both
                               give identical results.
                            2: instead of the sweeps, the additive overlapping DDM they
                               re-order (Section 2, Algorithms 2.1 / 2.2): every
                               subdomain solves at each of the sum(N_a - 1) + 1 steps,
                               with the transfers of all its neighbours from earlier
                               steps; the same local solves, transfers and assembly. */
  int local_solver;      /* factorisation and solve of the block-tridiagonal subdomain
                            operators: 1: twisted block LDL^T (two Schur-complement
                               chains meeting in the middle block; least memory,
                               sequential in the blocks; one workgroup runs a chain);
                            2: block cyclic reduction (about three times the factor
                               memory; every reduction level is one batched launch);
                            3: the LDL^T chains of 1 with one launch per block step,
                               every chain of a launch group in it (wide blocks);
                            4: nested dissection (multifrontal, the local solver of
                               Section 5's experiments): recursive bisection of the
                               subdomain box, the Schur complements of the separators
                               stored inverted, the separators above a depth applied
                               as one dense inverse, one launch per tree level over
                               every node of a launch group (in 3D about a sixth of
                               the band factor; the only one full C4 fits in);
                            0: 4 in 3D; in 2D 2 unless its factor would exceed 45% of
                               device memory, else 3 for blocks of 512 cells or more,
                               else 1 (in 2D nested dissection first eliminates closed
                               boxes of physical medium many wavelengths wide, whose
                               separator blocks can be near singular; see
                               dsd_plan_pivots).                                          */
  int dense_top;         /* block cyclic reduction only: the reduction stops at the first
                            level that has at most this many blocks (at least 2) and
                            applies the precomputed inverse of that reduced system as one
                            dense product (fewer, wider launches for the deep levels);
                            0: the library's bound (8, lowered to fit the solve kernel's
                            LDS and an order of at most 2048); -1: reduce to one block.
                            Valid range -1..64.                                          */
  int sweep_order;       /* 3D sweep order (Section 4.1): 0 the order (Sorder3D) -- the 2D
                            order with +z, then with -z; 1 the other order given there,
                            along which the L1 distance from (+1,+1,+1) never decreases.
                            Transfers are routed by Rules 4.1/4.2 over the chosen order.
                            2D has one order (must be 0).                               */
  int nd_leaf;           /* nested dissection: boxes of at most this many cells are not
                            bisected further (0: 128)                                  */
  int nd_top_cells;      /* nested dissection: the separators of the shallowest depths
                            whose cells total at most this many form the dense top
                            (0: 1200; at most 9000)                                    */
  int nd_wide;           /* nested dissection: nodes whose front (separator plus
                            boundary) has at least this many cells apply their blocks
                            as tiled products over all right-hand sides of a group at
                            once, the vectors streamed through LDS (0: 1024); nodes
                            with more than 512 rows always do                          */
  int nd_wave_steps;     /* nested dissection: a tree level whose largest narrow node
                            needs at most this many 64-lane steps (row passes of
                            64 / rhs_per_group rows times columns, / 64) runs one node
                            per wave instead of one node per workgroup (0: 4)           */
  int nd_fuse;           /* nested dissection: from the shallowest subtree level below
                            which every node's front has at most this many cells
                            (0: 128; at most 512), each subtree runs in one workgroup,
                            level after level, in one launch per direction; 1 turns
                            this off                                                    */
} dsd_params;

/*
 * Build a plan: checkerboard partition and extended subdomains (Section 2.1),
 * assembly of every subdomain's J-scaled PML operator with the shifted profile
 * (eq. (eq:PML), (eq:PMLprofile)), and the factorisation of every subdomain
 * problem (the factorisation phase of sweeping methods, Section 1) as a
 * block-tridiagonal LDL^T whose diagonal Schur blocks are stored inverted.
 *   m_dev : [prod n] FP64, m = 1/c^2 on physical cells.  Read during the call.
 *   omega : angular frequency.
 * Returns DSD_EINVAL for an invalid partition, DSD_EPIVOT if a Schur block is
 * singular (the subdomain index is in dsd_last_error_detail()).
 */
int dsd_plan_create(const dsd_params* params, double omega, const double* m_dev,
                    void* stream, dsd_plan** out);

void dsd_destroy(dsd_plan* plan);

/* Sizes of a plan (host outputs; any pointer may be NULL). */
int dsd_plan_info(const dsd_plan* plan, long long* n_global, int* n_subdomains,
                  long long* factor_bytes, long long* workspace_bytes);

/* Pivot report of the factorisation (host outputs; either may be NULL): every
 * dense block the local solver inverts (Gauss-Jordan with partial pivoting in
 * FP64) records its largest and smallest pivot magnitude; *ratio is the largest
 * max|pivot| / min|pivot| over all of them (a lower bound on that block's
 * condition number: a large value flags a nearly singular local block, whose
 * complex64 factor loses that many digits) and *subdomain its subdomain. */
int dsd_plan_pivots(const dsd_plan* plan, double* ratio, int* subdomain);

/* Local solver in use: 1 = twisted block LDL^T chains, 2 = block cyclic reduction,
 * 3 = LDL^T chains with one launch per block step, 4 = nested dissection
 * (dsd_params.local_solver after the automatic choice); negative on a NULL plan. */
int dsd_plan_local_solver(const dsd_plan* plan);

/* Graph mode: when on, dsd_sweep_apply (and the preconditioner applications
 * inside dsd_gmres_solve and the FWI calls) run as a HIP graph captured on the
 * first call for each (input pointer, output pointer, nrhs) and replayed on
 * the caller's stream afterwards (the several hundred kernel launches of an
 * application become one graph launch).  The plan keeps the graphs until dsd_destroy; the
 * buffers a graph was captured with must stay valid while it can be replayed.
 * Off by default; results are identical either way. */
int dsd_set_graph(dsd_plan* plan, int on);

/* Autotuner: times `reps` preconditioner applications of `nrhs` right-hand
 * sides for every candidate shape of the subdomain-solve launches -- RHS per
 * workgroup (2, 4, 8, 16 as the LDS and register budgets allow) and, for the
 * cyclic reduction, a set of level-shape policies: two thresholds on the blocks
 * per subdomain left at a level split the levels into wide, middle and deep
 * ones, and each class has its own count of wave groups splitting the columns
 * of a job and of 64-row tiles per workgroup -- and keeps the fastest in the
 * plan.  Results of later calls may change at rounding level (a different
 * summation order), never more.  Outputs (host, may be NULL): the chosen RHS
 * per workgroup, the two thresholds of the chosen policy, and the time of one
 * application (ms).  Captured graphs are dropped.  Synchronises the stream. */
int dsd_autotune(dsd_plan* plan, int nrhs, int reps, int* kg_host, int* cg_wide_host,
                 int* cg_mid_host, double* ms_host, void* stream);

/* Launch shape of the subdomain solves as 13 ints: RHS per workgroup, then
 * the cyclic-reduction level policy: cg_wide, cg_mid (thresholds on the blocks
 * per subdomain left at a level that make it a wide, middle or deep level),
 * (wide_cg, wide_rt), (mid_cg, mid_rt), (deep_cg, deep_rt) (wave groups
 * splitting the columns of a job, 64-row tiles per workgroup: rt 0 = up to 4),
 * dense_cg, wide_kg (RHS per workgroup on the wide levels; 0 = the first
 * entry), and (chain_cg, chain_rt) for the chain block steps (local solver 3).
 * get writes the plan's current shape (for instance after dsd_autotune); set
 * applies a saved one without timing anything (rt 0 with cg 1..4 or rt 1 with
 * cg 1..12; RHS-per-workgroup entries must be ones the plan supports, else
 * DSD_EINVAL).  set drops captured graphs. */
int dsd_get_solve_shape(const dsd_plan* plan, int* shape13_host);
int dsd_set_solve_shape(dsd_plan* plan, const int* shape13_host);

/* Local grid of subdomain `sub` (lexicographic index, x part fastest):
 * dims[3] = local cells per axis, g0[3] = global array index of its first cell
 * per axis (local PML cells included). */
int dsd_subdomain_grid(const dsd_plan* plan, int sub, int* dims, int* g0);

/*
 * Solve one subdomain's local PML problem L_sub u = r (the local solve of
 * Algorithms 3.1 / 4.1) with the plan's factors.
 *   r_dev, u_dev : [nrhs][N_loc] complex128 on the subdomain's local grid
 *                  (x fastest).  Computed in the plan precision.
 */
int dsd_local_solve(dsd_plan* plan, int sub, const double* r_dev, double* u_dev, int nrhs,
                    void* stream);

/*
 * Allocation-free variant of dsd_local_solve, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, layouts and results as
 * dsd_local_solve (the same kernels), but its working memory -- the packed
 * right-hand sides and solutions of the call in the plan precision,
 * 2 x N_loc x nrhs values, each half rounded up to 256 bytes -- lives in a
 * static device array of DSD_NOALLOC_SCRATCH_BYTES per GPU (held by every GPU
 * the library runs on until the process ends), and the job tables were built
 * with the plan.  The call allocates, frees and uploads nothing and does not
 * synchronise: it is ordered on `stream` like the other calls.  Every call on
 * one GPU shares that GPU's array and nothing in it needs to start at zero
 * (every value is written before it is read); calls that overlap on one GPU
 * (other streams, other threads, other plans on the same device) race on it
 * and must be serialised by the caller.
 * DSD_EINVAL for a bad argument, for a current device other than the plan's,
 * or when 2 x N_loc x nrhs values exceed DSD_NOALLOC_SCRATCH_BYTES.
 */
#define DSD_NOALLOC_SCRATCH_BYTES (64LL << 20)
int dsd_local_solve_noalloc(dsd_plan* plan, int sub, const double* r_dev, double* u_dev,
                            int nrhs, void* stream);

/*
 * One application of the diagonal-sweeping DDM (Algorithm 3.1 in 2D, 4.1 in
 * 3D): 2^dim sweeps; every subdomain solve is launched, batched with all other
 * solves of its dependency level (schedule 0) or of its anti-diagonal step
 * (schedule 1), as soon as its sources exist; the source-transfer operator Psi passes the
 * cutoff-weighted sources to the neighbours (Section 2.2) routed by Rules
 * 3.1/3.2 (4.1/4.2), and u_DDM = sum beta_{0;ij} u_ij (eq. (eq:sumdiag2D),
 * (eq:sumdiag3D)) is accumulated in FP64.  With schedule 2 the same operators
 * run the additive DDM of Section 2 instead (every subdomain at every step).
 *   f_dev, u_dev : [nrhs][N_g] complex128; nrhs in 1..max_rhs (else DSD_EINVAL).
 *                  They may alias: f is read before u is first written.
 */
int dsd_sweep_apply(dsd_plan* plan, const double* f_dev, double* u_dev, int nrhs, void* stream);

/* y = M x with the FP64 J-scaled global operator (5/7-point, Section 5).
 *   x_dev, y_dev : [nrhs][N_g] complex128, must not alias. */
int dsd_apply_operator(dsd_plan* plan, const double* x_dev, double* y_dev, int nrhs,
                       void* stream);

/*
 * Solve M x = b by flexible GMRES (FP64: residual, Gram-Schmidt, solution
 * update) right-preconditioned by dsd_sweep_apply in the plan precision
 * (Remark 1 of Section 4; stopping rule of Section 5.2).  Restarting from the
 * current iterate with the true FP64 residual is the iterative refinement of
 * the complex64 path.
 *   b_dev, x_dev  : [nrhs][N_g] complex128 (x is overwritten; x0 = 0).
 *   tol           : stop when ||b - M x|| / ||b|| <= tol (true residual), per RHS.
 *   maxit         : cap on preconditioner applications per RHS.
 *   restart       : Krylov vectors kept before a restart (<= 0: library default).
 *   iters_host    : [nrhs] preconditioner applications used per RHS (may be NULL).
 *   relres_host   : [nrhs] final true relative residual per RHS (may be NULL).
 * Returns DSD_NOT_CONVERGED if some RHS missed tol within maxit.
 */
int dsd_gmres_solve(dsd_plan* plan, const double* b_dev, double* x_dev, int nrhs, double tol,
                    int maxit, int restart, int* iters_host, double* relres_host, void* stream);

/*
 * The diagonal sweeps as a stand-alone iterative solver (Section 5.2, the
 * three-layer residual-decay test): x_0 = 0, x_{k+1} = x_k + DDM(f - M x_k)
 * with DDM = dsd_sweep_apply in the plan precision and the residual in FP64.
 *   f_dev, x_dev     : [nrhs][N_g] complex128, must not alias (x overwritten).
 *   iters            : sweep applications (>= 0).
 *   relres_hist_host : [iters + 1][nrhs] ||f - M x_k|| / ||f|| for k = 0..iters
 *                      (1 at k = 0; 0 for a zero right-hand side).
 * Synchronises the stream after every iteration (the history is host data).
 * DSD_EINVAL for a bad pointer, nrhs outside 1..max_rhs or iters < 0;
 * DSD_ENOTFINITE for a non-finite right-hand side or residual.
 */
int dsd_ddm_iterate(dsd_plan* plan, const double* f_dev, double* x_dev, int nrhs, int iters,
                    double* relres_hist_host, void* stream);

/* Solve the adjoint system M^H x = b with the same factors: the discrete
 * PML operator of Section 2.1 (eq. (eq:PML) multiplied through by J, central
 * differences of Section 5) is complex symmetric, so x = conj(M^{-1} conj(b))
 * is one FGMRES solve of Remark 1 of Section 4 between two conjugations.  It
 * is the adjoint solve of the many-right-hand-side inversion setting that
 * Remark 2 of Section 4 motivates.  Arguments, outputs and error codes as
 * dsd_gmres_solve. */
int dsd_adjoint_solve(dsd_plan* plan, const double* b_dev, double* x_dev, int nrhs, double tol,
                      int maxit, int restart, int* iters_host, double* relres_host,
                      void* stream);

/*
 * Full-waveform-inversion misfit and gradient for the plan's medium (the
 * multi-RHS application motivating Remark 2 of Section 4):
 *   J(m) = 1/2 sum_s || P u_s - d_s ||^2,   M(m) u_s = f_s,
 *   dJ/dm = -omega^2 Re sum_s conj(lam_s) J u_s  (transposed through the clamp
 *   extension onto the physical cells),  M^H lam_s = P^T (P u_s - d_s).
 *   f_dev      : [nsrc][N_g] complex128 sources (J-scaled).
 *   rec_dev    : [nrec] int64 global flat indices of the receiver cells.
 *   dobs_dev   : [nsrc][nrec] complex128 observed data.
 *   grad_dev   : [prod n] FP64 gradient w.r.t. m on physical cells (output).
 *   misfit_host: J (output).
 *   u_dev      : optional [nsrc][N_g] complex128 output of the forward fields (may be NULL).
 */
int dsd_fwi_gradient(dsd_plan* plan, const double* f_dev, int nsrc, const long long* rec_dev,
                     int nrec, const double* dobs_dev, double tol, int maxit, double* grad_dev,
                     double* misfit_host, double* u_dev, void* stream);

/* Forward modelling only: d = P u_s for every source (complex128 [nsrc][nrec]). */
int dsd_fwi_forward(dsd_plan* plan, const double* f_dev, int nsrc, const long long* rec_dev,
                    int nrec, double tol, int maxit, double* d_dev, void* stream);

const char* dsd_strerror(int code);
const char* dsd_last_error_detail(void);

/* Kernel timing hooks for measurement: accumulated device time (ms) of the
 * subdomain-solve kernels and their launch count since the last reset, and the
 * algorithmic bytes those launches had to move (factor blocks once per RHS
 * group sharing them, plus the vectors).  Timing uses a pair of HIP events
 * around every solve launch on the plan's stream, recorded without waiting so
 * that launches stay back to back, and read once per preconditioner
 * application (which then waits for the stream).  Active only while enabled. */
int dsd_timing_enable(dsd_plan* plan, int on);
int dsd_timing_read(dsd_plan* plan, double* solve_ms, long long* solve_launches,
                    double* solve_bytes, double* other_ms);
/* The algorithmic flops of the same launches since the last reset: 8 real
 * flops per complex factor entry and right-hand side (each factor block applied
 * to every right-hand side of the call).  With dsd_timing_read's bytes this
 * places the solves against the matrix-core roof when the right-hand-side
 * count makes them compute bound.  DSD_EINVAL for a null argument. */
int dsd_timing_flops(dsd_plan* plan, double* solve_flops);

#ifdef __cplusplus
}
#endif
#endif /* DSWEEP_H */
