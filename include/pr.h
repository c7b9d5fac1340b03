/*
 * pr.h -- C ABI of the MOR-based adaptive parareal hot path on MI355X (gfx950).
 *
 * Method: arXiv 2601.10981, "A model order reduction based adaptive parareal
 * method for time-dependent PDEs". The library implements, for the periodic
 * 3-D advection-diffusion equation u_t = kappa Lap u - v . grad u + f (eq1 of
 * Sec. 4 with c = 0; a steady velocity with f = 0, or the time-dependent
 * velocity and forcing of the two flows of Sec. 4), the fine propagator F,
 * POD_Mode (Algorithm 1), the POD-Galerkin coarse propagator G with
 * augmentation by the interface state (eqaug, eq12, eq13) and the whole
 * adaptive parareal iteration (formula4, Algorithm 2).
 *
 * Discretisation (replaces the paper's FEM + implicit Euler, Sec. 3.1):
 *   grid      periodic cube [0, L)^3, n^3 nodes x_i = i h, h = L / n
 *   layout    one field = n^3 contiguous values indexed ((i n) + j) n + k for
 *             (x_i, y_j, z_k): z fastest
 *   operator  (L u)_p = kappa sum_d (u_{p+e_d} - 2 u_p + u_{p-e_d}) / h^2
 *                       - sum_d v_d(p) (u_{p+e_d} - u_{p-e_d}) / (2 h)
 *   fine step classical RK4 (one step = P4(dt L) for a steady flow; for the
 *             forced flows stages at t, t + dt/2, t + dt/2, t + dt of
 *             du/dt = L(t) u + f(t), L(t) the same stencil with v(., t))
 *   mass      M = h^3 I (discrete L2 inner product)
 *
 * Conventions for every entry point:
 *   - Buffers named "device" are device pointers on the context's device;
 *     the caller allocates and frees them and keeps them alive until the work
 *     queued on `stream` has completed. The library keeps no caller pointer
 *     after a call returns.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream). Unless
 *     stated otherwise a call only enqueues work on it and returns.
 *   - Field precision: PR_F64 fields are double; under PR_MIXED the stencil,
 *     the snapshots and the POD bases are float while states (u_in, u_out,
 *     U_out) and every reduction, eigen-decomposition, re-orthogonalisation
 *     and reduced system stay double.
 *   - Every entry point returns a pr_status; nothing throws or aborts across
 *     the ABI. pr_last_error() describes the last failure of the context. On
 *     an error other than PR_ENOTCONV the outputs are unspecified.
 *   - One host thread at a time per context.
 */
#ifndef PR_H
#define PR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PR_OK = 0,
  PR_EINVAL = -1,     /* bad shape or parameter                              */
  PR_ENOMEM = -2,     /* request exceeds the context's HBM budget            */
  PR_EDEVICE = -3,    /* HIP runtime error                                   */
  PR_EUNSTABLE = -4,  /* dt * rho(L) > 2.6: outside the RK4 stability region */
  PR_ENOTCONV = -5,   /* max_iter reached above tol; outputs = last iterate  */
  PR_ENUMERIC = -6,   /* NaN or Inf in a jump norm                           */
  PR_EBUSY = -7       /* context in use                                      */
} pr_status;

enum {
  PR_FLOW_UNIFORM = 0,
  PR_FLOW_ABC = 1,
  PR_FLOW_KOLMOGOROV = 2,
  PR_FLOW_KOLMOGOROV_T = 3, /* the Kolmogorov flow of Sec. 4 (eq. koleq), forced */
  PR_FLOW_ABC_T = 4         /* the ABC flow of Sec. 4 with phase sin(w t), forced */
};
enum { PR_F64 = 0, PR_MIXED = 1 };
enum { PR_MODE_ADAPTIVE = 0, PR_MODE_FIXED_POD = 1, PR_MODE_COARSE_GRID = 2 };

/* Problem of eq1 (Sec. 4) on the finite-difference grid.
 *   flow PR_FLOW_ABC:        v = (A sin z + C cos y, B sin x + A cos z,
 *                                 C sin y + B cos x),  fp = {A, B, C}
 *   flow PR_FLOW_KOLMOGOROV: v = (a sin(k_f y), 0, 0),  fp = {a, k_f, -}
 *   flow PR_FLOW_UNIFORM:    v = (c_x, c_y, c_z),        fp = {c_x, c_y, c_z}
 *   flow PR_FLOW_KOLMOGOROV_T, fp = {a_v, a_f, w} (the paper: {1, 1, 1}):
 *     v(t) = a_v [(cos y, cos z, cos x) + (sin z, sin x, sin y) cos(w t)],
 *     f(t) = a_f [-cos y - sin z cos(w t)]
 *   flow PR_FLOW_ABC_T, fp = {a_v, a_f, w}, s = sin(w t):
 *     v(t) = a_v (sin(z+s) + cos(y+s), sin(x+s) + cos(z+s), sin(y+s) + cos(x+s)),
 *     f(t) = a_f [-sin(z+s) - cos(y+s)]
 *   For these two, sum_d max|v_d| = 6 |a_v| at every t in the stability
 *   bound below, and the reduced systems use the flows' separation
 *   v = sum_j theta_j(t) v_j, f = sum_j theta_j(t) f_j (Sec. 4: B and f are
 *   separable in time and space).
 * n >= 4; L > 0; kappa >= 0. */
typedef struct {
  int n;
  double L;
  double kappa;
  int flow;
  double fp[3];
  int precision; /* PR_F64 or PR_MIXED */
} pr_grid_problem;

typedef struct pr_ctx pr_ctx;

/* Create a context on HIP device `device`. The context owns the library's
 * device scratch memory (never more than hbm_budget_bytes; 0 = 90% of the
 * device's free memory), its pinned staging memory and its events.
 * Returns PR_EINVAL for a bad device, PR_EDEVICE on a HIP failure. */
pr_status pr_ctx_create(int device, size_t hbm_budget_bytes, pr_ctx** out);
/* Synchronise the context's device and release everything it owns. */
void pr_ctx_destroy(pr_ctx* ctx);
/* Message describing the last failure on ctx (never NULL; "" if none). */
const char* pr_last_error(const pr_ctx* ctx);
/* Bytes of device scratch currently held by the context. */
size_t pr_ctx_scratch_bytes(const pr_ctx* ctx);

/* ---------------------------------------------------------------------------
 * Fine propagator F (Sec. 2; Algorithm 2, fine step; snapshot matrix W of
 * Sec. 3.2 Case I): n_steps RK4 steps of size dt from u_in, for every item of
 * the batch in the same launches (items may differ in n, flow, kappa, dt and
 * n_steps but share the precision).
 *   u_in      device, N_g doubles
 *   u_out     device, N_g doubles; may equal u_in
 *   snaps     device, N_g x n_s values in field precision, n_s =
 *             floor(n_steps / snap_every) + 1, column j (contiguous, N_g
 *             values) = state after j * snap_every steps; NULL iff
 *             snap_every == 0
 * Errors: PR_EINVAL (n < 4, n_steps < 0, dt <= 0, mixed precisions in one
 * batch, snaps missing), PR_EUNSTABLE (dt * (12 kappa / h^2 +
 * sum_d max|v_d| / h) > 2.6), PR_ENOMEM (work fields exceed the budget). */
typedef struct {
  const pr_grid_problem* prob;
  double dt;
  int n_steps;
  const double* u_in;
  double* u_out;
  int snap_every;
  void* snaps;
  double t0;      /* start time (read by the forced flows only)             */
} pr_fine_item;
pr_status pr_fine_propagate(pr_ctx* ctx, int batch, const pr_fine_item* items, void* stream);
/* Tiling of the fused RK4 stencil. Every tiling gives bitwise the same
 * values; the context picks one per (precision, largest n of the batch,
 * floor(log2(batch)), steady or forced flows -- a batch mixing the two runs
 * as two launches per step) by timing one step of the first such batch in
 * each candidate tiling and x-chunk length (that first call synchronises
 * `stream`). The chunk policies: 0 and 1 halve the chunk while a launch has
 * fewer than 2048 / 768 workgroups; 2 takes the length of least modelled
 * time, rounds of the workgroups the device holds at once times the planes
 * each marches. The environment variables PR_FUSED_CFG=<index> (steady
 * flows), PR_FORCED_CFG=<index> (forced flows) and PR_FUSED_CHUNK=<policy>
 * force one; PR_TUNE_LOG=1 prints each tuning's timings (us per launch, by
 * code = tiling + 8 x policy) to stderr.
 * The steady-flow tilings include 2 x 2 register-blocked ones (each thread
 * holds four columns; tried for batches whose grids are even and whose
 * fields are aligned to two values).
 * pr_fine_tuned reports, for a key (forced = 1: the forced-flow stencil), the
 * workgroup's output tile (tile_y x tile_z points of the (y, z) plane), its
 * thread count, the x planes it marches through (for `batch` fields of n^3)
 * and whether it is a blocked tiling; every output pointer may be NULL.
 * PR_EINVAL if no batch of that key ran yet. */
pr_status pr_fine_tuned(const pr_ctx* ctx, int precision, int forced, int n, int batch,
                        int* tile_y, int* tile_z, int* threads, int* planes, int* blocked);

/* ---------------------------------------------------------------------------
 * POD_Mode (Algorithm 1; Sec. 3.2 Case I and Case II, eq. W^k_n): modes of
 * the column concatenation W = [block_0, block_1, ...] with M = h^3 I.
 *   1. G = W^T M W (FP64 sums of per-chunk MFMA partials; FP32 MFMA products
 *      under PR_MIXED, FP64 MFMA under PR_F64)
 *   2. eigenpairs of G by cyclic Jacobi in FP64, descending; each
 *      eigenvector's largest-magnitude entry made positive
 *   3. r = #{lambda_i > tau_r lambda_1} (tau_r = 1e-13 F64, 1e-6 MIXED);
 *      m = min(cap, min{k : sum_{i<=k} sqrt(lambda_i) >= gamma
 *      sum_{i<=r} sqrt(lambda_i)}); force_m >= 0 gives min(force_m, r, cap)
 *   4. R = W Y_m Lambda_m^{-1/2}, then a CholQR pass in the M inner
 *      product (a column whose Cholesky pivot falls below 1e-8 is dropped
 *      with all later ones, lowering m)
 *   blocks[b]    device pointer to block_cols[b] columns of N_g values each
 *                (field precision); block_valid[b] is NULL (all columns
 *                valid) or a device int holding how many leading columns
 *                are valid (the rest are ignored)
 *   total columns (sum of block_cols) <= 64; 1 <= cap <= 32
 *   R_out        device, N_g x cap in field precision; columns >= m zeroed
 *   m_out        device int
 *   lambda_out   device, sum(block_cols) doubles (descending; invalid
 *                columns contribute zero eigenvalues), or NULL */
typedef struct {
  const pr_grid_problem* prob;
  int n_blocks;
  const void* const* blocks;
  const int* block_cols;
  const int* const* block_valid;
  double gamma;
  int cap;
  int force_m;
  void* R_out;
  int* m_out;
  double* lambda_out;
} pr_pod_item;
pr_status pr_pod_build(pr_ctx* ctx, int batch, const pr_pod_item* items, void* stream);

/* ---------------------------------------------------------------------------
 * Snapshot Gram (Algorithm 1, step 1): G = W^T M W = h^3 W^T W for the
 * N_g x ncols column block W (field precision, column j contiguous), on
 * MFMA (FP32 products under PR_MIXED, FP64 under PR_F64) with FP64 per-chunk
 * partials summed in a fixed order.
 *   W       device, ncols * N_g values; 1 <= ncols <= 64
 *   G_out   device, ncols x ncols doubles, row-major (symmetric)
 * Errors: PR_EINVAL for a bad problem or ncols. */
pr_status pr_gram(pr_ctx* ctx, const pr_grid_problem* prob, const void* W, int ncols,
                  double* G_out, void* stream);

/* pr_gram for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, kernels and chunking as pr_gram, so G_out is bitwise the
 * same, but the call allocates nothing and uses no context scratch. Its
 * device scratch (descriptors, the padded Gram and the per-chunk partials)
 * is one file-scope array of 10.5 MiB per device, set up by pr_ctx_create
 * and held until the process ends. That size covers every Gram pr_gram
 * accepts (1 <= ncols <= 64, any N_g): larger ncols is PR_EINVAL. Every call
 * on a device shares the array and it keeps the last call's contents: calls
 * on one stream are ordered, calls that overlap on one device (several
 * streams or host threads, or several contexts) race.
 * Errors: PR_EINVAL for a bad problem or ncols, PR_EDEVICE on a HIP failure. */
pr_status pr_gram_noalloc(pr_ctx* ctx, const pr_grid_problem* prob, const void* W, int ncols,
                          double* G_out, void* stream);

/* ---------------------------------------------------------------------------
 * Coarse propagator G_{k,n} (eq. 8 / eq00; with augmentation eqaug, eq12,
 * eq13; formula4): Galerkin projection of each input state onto span(Psi),
 * n_c RK4 steps of M_r beta' = L_r beta over dT_total, optional lift. For the
 * forced flows the system is M_r beta' = sum_j theta_j(t) (L_r,j beta +
 * f_r,j) over [t0, t0 + dT_total] (L_r,j = Psi^T M L_j Psi and f_r,j =
 * Psi^T M f_j of the flow's time-space pieces, theta_0 = 1), with stages at
 * t, t + h/2, t + h/2, t + h, and the guard below uses
 * sum_j ||M_r^{-1} L_r,j||_F in place of ||M_r^{-1} L_r||_F.
 *   R            device, N_g x cap, field precision, M-orthonormal columns
 *   m            device int: valid columns of R (<= cap <= 32)
 *   u_aug        NULL, or device N_g doubles: Psi = [R, d] with
 *                d~ = u_aug - R R^T M u_aug applied twice (CGS2) and d =
 *                d~ / ||d~||_M, unless ||d~||_M <= 1e-12 ||u_aug||_M (then
 *                Psi = R); NULL: Psi = R
 *   n_in         1 or 2 states u_in[0..n_in) (device, N_g doubles)
 *   n_c          RK4 steps (>= 1), or 0 for ceil(n_f_hint / 10) with
 *                n_f_hint = round(dT_total / dt_hint)
 *   the step count is doubled while (dT_total / n_c) ||M_r^{-1} L_r||_F > 2.5
 *   u_out[i]     NULL, or device N_g doubles: Psi beta_i(dT_total)
 *   beta_out     NULL, or device n_in x (cap + 1) doubles (row i = beta_i in
 *                the basis [R(:, 0..m), d]; unused entries zero)
 *   n_c_out      NULL, or device int: steps after the guard
 * L R is applied per column, or for launches of many columns on grids with
 * 64 <= n <= 256 through an LDS window of each plane (the same values bit for
 * bit); PR_APPLYL_WIN=0 or 1 forces the per-column or the window kernel. */
typedef struct {
  const pr_grid_problem* prob;
  const void* R;
  int cap;
  const int* m;
  const double* u_aug;
  int n_in;
  const double* u_in[2];
  double dT_total;
  int n_c;
  double dt_hint;
  double* u_out[2];
  double* beta_out;
  int* n_c_out;
  double t0;      /* start time (read by the forced flows only)             */
} pr_coarse_item;
pr_status pr_coarse_propagate(pr_ctx* ctx, int batch, const pr_coarse_item* items, void* stream);

/* ---------------------------------------------------------------------------
 * The adaptive parareal solve (formula4, Algorithm 2).
 * [0, T] is split into N subintervals of DeltaT = T / N; the first n_warm of
 * them form the warm-up window [0, T_0], T_0 = n_warm DeltaT (the paper runs
 * the adaptive method with T_0 = DeltaT and its Parareal-I comparison with
 * T_0 = 2 DeltaT, Sec. 4), whose fine solve gives G_0 (Case I): snapshots
 * every dM steps across the whole window, floor(n_warm n_f / dM) + 1 <= 64
 * of them (POD modes only). The parareal partition of [T_0, T] has
 * N' = N - n_warm subintervals; U_out rows 1 .. n_warm are fine states.
 * Subinterval i of [0, T] starts at t = i DeltaT (the time the forced flows
 * read).
 *   fine steps    n_f = ceil(DeltaT / dt - 1e-9), delta_t = DeltaT / n_f;
 *                 dt <= 0 requests min(2e-3, 1.3 / rho) with the bound
 *                 rho = 12 kappa / h^2 + sum_d max|v_d| / h (max|v_d| from
 *                 the flow's coefficients: ABC |A|+|C|, |B|+|A|, |C|+|B|;
 *                 Kolmogorov |amplitude|; uniform |c_d|)
 *   snapshots     every dM steps (0: ceil(n_f / 16))
 *   coarse steps  n_c = max(1, ceil(n_f / coarse_ratio)) (then the guard)
 *   POD           gamma1 (k = 0), gamma2 (per subinterval), gamma3 (local
 *                 collection W^k_n of m_l left neighbours and p previous
 *                 iterations; 0 <= m_l, 0 <= p <= 1), rank caps cap0 (stage
 *                 1 and k = 0 use cap) and cap
 *   stopping      e_k = max_n ||U^k_n - U^{k-1}_n||_M / ||U^k_n||_M <= tol,
 *                 or k = N' (finite termination), or k = max_iter
 *                 (max_iter <= 0: N')
 *   u0            device, N_g doubles (t = 0)
 *   U_out         device, (N + 1) x N_g doubles: U_out[j] = state at j DeltaT
 *   U_ref         NULL or device (N + 1) x N_g doubles (serial fine
 *                 solution): then err[k] = max_n ||U^k_n - U_ref||/||U_ref||
 *   mode          PR_MODE_ADAPTIVE: Algorithm 2. PR_MODE_FIXED_POD: the
 *                 comparison method "Parareal-I" of Sec. 4 -- plain parareal
 *                 (formula4 without augmentation) whose coarse propagator is
 *                 the k = 0 POD Galerkin propagator for every iteration; no
 *                 snapshots or local bases are built after k = 0, and gamma2,
 *                 gamma3, cap0, m_l and p are ignored. PR_MODE_COARSE_GRID:
 *                 "Parareal-II" of Sec. 4 -- plain parareal whose coarse
 *                 propagator solves the same equation on the n/2 grid (n even,
 *                 n >= 8): full-weighting restriction, RK4 with
 *                 n_g = n_c steps doubled while DeltaT / n_g * rho_c > 2.5
 *                 (rho_c the bound above on the coarse grid), linear
 *                 interpolation back; no POD
 *   diag          1: record the coarse-gap diagnostics of Sec. 4 (its dT =
 *                 delta t runs; set coarse_ratio = 1 for those): at iteration
 *                 k >= 1 the sweep step from U_n to U_{n+1} records
 *                 ||F(U^{k-1}_n) - G_k(P U^{k-1}_n)||_M / ||F(U^{k-1}_n)||_M
 *                 and, with U_ref, ||U_{n+1} - G_k(P U^k_n)||_M /
 *                 ||U_{n+1}||_M (report gap_fine / gap_ref). POD modes only
 *                 (PR_EINVAL with PR_MODE_COARSE_GRID); costs two extra field
 *                 passes per sweep step
 * Environment: PR_SWEEP_PARTS (default 4; 1 = no second stream) cuts each
 * sweep wave into parts whose preparation (stage-1 and stage-2 POD, L Psi)
 * overlaps the sweep of the part before; PR_SWEEP_FIRST (default wave / 8;
 * 0 = even split) sizes the first part; PR_DEFER_POD1 (default 1; 0 = off)
 * moves the stage-1 POD into those preparations; PR_DEFER_CHOLQR (default
 * 1; 0 = off) folds the stage-1 CholQR into stage 2's block whitening;
 * PR_SMALL_CHOLQR (default 1; 0 = off; PR_F64 only) takes stage 2's CholQR
 * factor from C^T G C instead of a Gram pass over the formed modes (the
 * modes then keep an M-orthogonality error of about eps lambda_1 /
 * lambda_m, at most about 1e-3; the span and the Galerkin system, which
 * keeps M_r explicitly, are unchanged);
 * PR_STAGE_UPLOAD (default 1; 0 = off, read once per process) writes small
 * descriptor blocks through kernel arguments. All keep the ranks; all but
 * the two CholQR switches keep every bit, and those the iterates up to
 * round-off.
 * The call synchronises `stream` once per iteration (8-byte jump read) and
 * before returning. Returns PR_ENOTCONV (outputs = last iterate) when
 * max_iter < N' stops it above tol, PR_ENUMERIC on a NaN/Inf jump. */
typedef struct {
  double T;
  int N;
  double dt;
  int dM;
  double gamma1, gamma2, gamma3;
  int cap0, cap;
  int ml, p;
  int coarse_ratio;
  double tol;
  int max_iter;
  int mode;        /* PR_MODE_ADAPTIVE, PR_MODE_FIXED_POD or PR_MODE_COARSE_GRID */
  int diag;        /* 1: coarse-gap diagnostics (see above)                   */
  int n_warm;      /* warm-up window (see above): T_0 = n_warm DeltaT; 0 = 1 */
  const double* U_ref;
} pr_parareal_opts;

/* Per-solve report; every pointer member is an optional host array. */
typedef struct {
  int iters;          /* parareal iterations performed (k_max)            */
  int converged;      /* 1 if e_k <= tol or finite termination            */
  int n_f, dM, n_s, n_c, n_sub; /* derived sizes (n_sub = N' = N - n_warm) */
  int m0;             /* rank of V^0_POD                                   */
  double* jump;       /* [max_iter + 1]: jump[k - 1] = e_k                 */
  double* err;        /* [max_iter + 1]: err[k] vs U_ref (k = 0..iters)    */
  double* t_iter;     /* [max_iter + 1]: seconds from start to end of k    */
  int* ranks;         /* [(max_iter + 1) * n_sub]: row k, column n: m^k_n  */
  double t_phase[5];  /* seconds in F, C (POD), U (reduced ops), A, G      */
  double fine_updates;/* grid-point RK4 updates performed                  */
  double seconds;     /* wall time of the solve                            */
  double* gap_fine;   /* [(max_iter + 1) * n_sub]: row k, column n: the
                         fine-vs-coarse gap of the step from U_n (opts.diag);
                         -1 where no such step ran                          */
  double* gap_ref;    /* the same layout: reference-vs-coarse gap (needs
                         U_ref); -1 where not recorded                      */
  double* basis_orth; /* the same layout (opts.diag): max_ij |(Psi^T M Psi
                         - I)_ij| over the valid columns of the basis Psi of
                         that coarse step (the stage-2 basis; the k = 0
                         basis in PR_MODE_FIXED_POD); -1 where not recorded */
} pr_report;

pr_status pr_parareal_solve(pr_ctx* ctx, const pr_grid_problem* prob,
                            const pr_parareal_opts* opts, const double* u0,
                            double* U_out, pr_report* report, void* stream);

/* Derived sizes of a solve (pure host function): the readings above applied
 * to (prob, opts). n_c is before the stability guard, which the device may
 * raise per coarse step. Errors as pr_parareal_solve's validation. */
typedef struct {
  int n_sub;      /* N' = N - n_warm parareal subintervals                   */
  int n_f;        /* fine steps per subinterval                              */
  double dt;      /* fine step delta_t = DeltaT / n_f                        */
  int dM;         /* snapshot stride                                         */
  int n_s;        /* snapshots per subinterval, floor(n_f / dM) + 1          */
  int n_c;        /* coarse steps per subinterval                            */
  int max_iter;   /* iteration limit after clamping to N'                    */
} pr_plan_info;
pr_status pr_plan(const pr_grid_problem* prob, const pr_parareal_opts* opts, pr_plan_info* out);

/* Device bytes pr_parareal_solve needs for (prob, opts) with every wave at
 * full width (pure host function); a solve under a smaller budget runs its
 * fine solves and local POD in narrower waves. */
pr_status pr_footprint(const pr_grid_problem* prob, const pr_parareal_opts* opts,
                       size_t* bytes);

/* ---------------------------------------------------------------------------
 * Incremental solves for serving: the iteration of formula4 / Algorithm 2
 * split at its stopping test, so that one host loop can advance many
 * independent solves (different problems, sizes and precisions) together.
 *
 * pr_solve_begin   validates (prob, opts) as pr_parareal_solve does, allocates
 *                  the solve's own device memory on the context's budget
 *                  (PR_ENOMEM when it does not fit: admission control), copies
 *                  u0 (device, N_g doubles) and runs k = 0 (Algorithm 2's
 *                  initial POD basis and coarse sweep); synchronises `stream`.
 *                  opts->U_ref, when given, must stay alive until
 *                  pr_solve_end. On success *out is a new handle.
 * pr_solve_step_batch  one parareal iteration of every handle in
 *                  solves[0..count) that has not stopped: the fine solves
 *                  and per-subinterval POD of all of them share launches,
 *                  the sweeps run one solve after another; one
 *                  synchronisation of `stream` at the end. done[i] (host,
 *                  nullable) = 1 when handle i has stopped (tol reached,
 *                  finite termination, max_iter or a NaN/Inf jump). Each
 *                  solve's iterates are bitwise those of pr_parareal_solve
 *                  whatever else is in the batch. A handle may appear once
 *                  per call.
 * pr_solve_state   enqueues a copy of the latest iterate's state at
 *                  t = j DeltaT (0 <= j <= N; j = 0 is u0) into out (device,
 *                  N_g doubles).
 * pr_solve_done    1 when the handle has stopped (or is NULL).
 * pr_solve_bytes   device bytes the handle owns.
 * pr_solve_end     writes the last iterate to U_out (device, (N + 1) x N_g
 *                  doubles, nullable) and the report (nullable, as for
 *                  pr_parareal_solve), frees the handle (also on error) and
 *                  returns PR_OK, PR_ENOTCONV or PR_ENUMERIC as
 *                  pr_parareal_solve would.
 * Handles belong to the context that made them; end every handle before
 * destroying the context. */
typedef struct pr_solve pr_solve;
pr_status pr_solve_begin(pr_ctx* ctx, const pr_grid_problem* prob,
                         const pr_parareal_opts* opts, const double* u0,
                         pr_solve** out, void* stream);
pr_status pr_solve_step_batch(pr_ctx* ctx, int count, pr_solve* const* solves,
                              int* done, void* stream);
pr_status pr_solve_state(pr_ctx* ctx, const pr_solve* solve, int j, double* out,
                         void* stream);
int pr_solve_done(const pr_solve* solve);
size_t pr_solve_bytes(const pr_solve* solve);
pr_status pr_solve_end(pr_ctx* ctx, pr_solve* solve, double* U_out,
                       pr_report* report, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PR_H */
