// The adaptive parareal solve (formula4, Algorithm 2) on one GPU, as a
// per-solve state advanced one iteration at a time, alone or batched with
// other solves (continuous batching).
//
// Numbering: [0, T] is split into N subintervals; subinterval 0 is the
// warm-up window [0, T_0] (T_0 = DeltaT) whose fine solve gives u_hat_0 and
// the snapshots for G_0 (Case I); the parareal partition of [T_0, T] has
// N' = N - 1 subintervals with states U_n at t = (n + 1) DeltaT, n = 0..N'.
//
// Per iteration k >= 1:
//   (i)   fine solves F(U^{k-1}_n) with snapshots for n = k-1..N'-1, batched
//         in waves (and across solves), and POD_Mode(gamma_2) of each
//         snapshot set (Algorithm 2, fine step and first POD)
//   (ii)  POD_Mode(gamma_3) of W^k_n = [R_{n-m_l,0} .. R_{n,0}, R^{k-1}_{n,0}]
//         batched over n, and L applied to the modes (Algorithm 2, second POD)
//   (iii) U^k_j = U^{k-1}_j (j < k) and U^k_k = F_{k-1} (the coarse terms
//         cancel there)
//   (iv)  the sequential sweep n = k..N'-1: augmentation by U^k_n (eq12),
//         Galerkin system of eq13, RK4 of both projections and the
//         correction of formula4 with jump partials (Algorithm 2, the sweep)
//   (v)   e_k = max_n ||U^k_n - U^{k-1}_n||_M / ||U^k_n||_M read back (8 B)
// The basis of subinterval j last computed at iteration min(k, j + 1) sits
// in slot min(k, j + 1) % 2 of a two-slot ring, which also holds
// R^{k-1}_{n,0} for p = 1.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "ctx.h"

namespace pr {

// per recorded sweep step: 8 coarse-gap norm partials and the basis's loss
// of M-orthonormality
constexpr int kDiagSlots = 9;

struct Plan {
  pr_grid_problem prob;
  pr_parareal_opts o;
  int N, Np, n_f, dM, n_s, n_c, max_iter;
  int nw;          // subintervals of the warm-up window [0, T_0] (T_0 = nw DeltaT)
  int n_s0;        // snapshots of the warm-up solve, floor(nw n_f / dM) + 1
  double dTs, dt;
  long long ng;
  bool f32;
  size_t sf;
  bool fixed;      // PR_MODE_FIXED_POD: the k = 0 basis for every iteration
  bool grid;       // PR_MODE_COARSE_GRID: the n/2 grid as coarse propagator
  pr_grid_problem pc;   // the coarse-grid problem (grid mode)
  int n_g;              // coarse-grid RK4 steps per subinterval (grid mode)
  double dt_c;
  int waveF, waveS;
  size_t fixed_bytes, perF, perS;
  int np;          // time-space pieces of the flow (1: steady)
  bool forced;     // forced, time-dependent flow
  bool diag;       // coarse-gap diagnostics recorded per (k, n)
  long long ld;    // column stride (elements) of the multi-column blocks:
                   // snapshots, bases, L applied to bases, forcing fields
  size_t cs;       // bytes per column of those blocks (ld x field size)
};

// Start time of parareal subinterval n (state U_n at t_hat_n = (n + nw) DeltaT;
// subintervals 0 .. nw - 1 of [0, T] form the warm-up window).
static double t_hat(const Plan& P, int n) { return (double)(n + P.nw) * P.dTs; }

static Plan make_plan(const pr_grid_problem* p, const pr_parareal_opts* o) {
  check_problem(p);
  PR_CHECK(o != nullptr, "null options");
  Plan P{};
  P.prob = *p;
  P.o = *o;
  PR_CHECK(o->N >= 1, "N must be >= 1");
  PR_CHECK(std::isfinite(o->T) && o->T > 0, "T must be positive");
  PR_CHECK(std::isfinite(o->dt), "dt must be finite");
  PR_CHECK(o->dM >= 0, "dM must be >= 0");
  PR_CHECK(o->gamma1 > 0 && o->gamma1 <= 1 && o->gamma2 > 0 && o->gamma2 <= 1 && o->gamma3 > 0 &&
               o->gamma3 <= 1,
           "gamma must be in (0, 1]");
  PR_CHECK(o->cap0 >= 1 && o->cap0 <= kMaxCap && o->cap >= 1 && o->cap <= kMaxCap,
           "caps must be in [1, 31]");
  PR_CHECK(o->mode == PR_MODE_ADAPTIVE || o->mode == PR_MODE_FIXED_POD ||
               o->mode == PR_MODE_COARSE_GRID,
           "unknown mode");
  P.fixed = o->mode == PR_MODE_FIXED_POD;
  P.grid = o->mode == PR_MODE_COARSE_GRID;
  P.diag = o->diag != 0;
  PR_CHECK(!(P.diag && P.grid), "coarse-gap diagnostics need a POD coarse propagator");
  if (P.grid) PR_CHECK(p->n % 2 == 0 && p->n / 2 >= 4, "the coarse grid needs an even n >= 8");
  if (o->mode == PR_MODE_ADAPTIVE) {
    PR_CHECK(o->ml >= 0 && o->p >= 0 && o->p <= 1, "need m_l >= 0 and p in {0, 1}");
    PR_CHECK((o->ml + 1 + o->p) * o->cap0 <= kMaxPodCols,
             "(m_l + 1 + p) * cap0 must be <= 64 (local POD input)");
  }
  PR_CHECK(o->coarse_ratio >= 1, "coarse_ratio must be >= 1");
  PR_CHECK(std::isfinite(o->tol) && o->tol >= 0, "tol must be >= 0");
  P.N = o->N;
  P.nw = o->n_warm > 0 ? o->n_warm : 1;
  PR_CHECK(P.nw <= o->N, "the warm-up window must lie inside [0, T] (n_warm <= N)");
  P.Np = o->N - P.nw;
  P.dTs = o->T / o->N;
  // dt <= 0: half the RK4 stability radius over the spectral bound, at most 2e-3
  const double dt_req = o->dt > 0 ? o->dt : std::min(2e-3, 0.5 * kStabRK4 / spectral_bound(*p));
  P.n_f = (int)std::max(1.0, std::ceil(P.dTs / dt_req - 1e-9));
  P.dt = P.dTs / P.n_f;
  P.dM = o->dM > 0 ? o->dM : (int)std::ceil(P.n_f / 16.0);
  P.dM = std::max(1, P.dM);
  P.n_s = P.n_f / P.dM + 1;
  PR_CHECK(P.n_s <= kMaxPodCols, "too many snapshots per subinterval (n_f / dM + 1 > 64)");
  P.n_s0 = (int)(((long long)P.nw * P.n_f) / P.dM + 1);
  PR_CHECK(P.n_s0 <= kMaxPodCols || o->mode == PR_MODE_COARSE_GRID,
           "too many warm-up snapshots (n_warm n_f / dM + 1 > 64)");
  P.n_c = std::max(1, (int)std::ceil(P.n_f / (double)o->coarse_ratio));
  P.max_iter = o->max_iter > 0 ? std::min(o->max_iter, P.Np) : P.Np;
  P.ng = ngrid(*p);
  P.f32 = p->precision == PR_MIXED;
  P.sf = P.f32 ? 4 : 8;
  if (P.dt * spectral_bound(*p) > kStabRK4)
    fail(PR_EUNSTABLE, "fine step exceeds the RK4 stability bound 2.6 / rho(L)");
  if (P.grid) {
    // the same problem on the n/2 grid; the coarse step rule, doubled while
    // the explicit coarse step would leave RK4's stability region
    P.pc = *p;
    P.pc.n = p->n / 2;
    const double rho_c = spectral_bound(P.pc);
    P.n_g = P.n_c;
    while (P.dTs / P.n_g * rho_c > kGuard) P.n_g *= 2;
    P.dt_c = P.dTs / P.n_g;
  }
  P.ld = P.ng + kColPad;
  P.cs = (size_t)P.ld * P.sf;
  const size_t f8 = (size_t)P.ng * 8, cs = P.cs;
  const size_t Np1 = (size_t)std::max(P.Np, 1);
  // solve-owned memory apart from the waves: two state sets, F_n, two slots
  // of stage-1 bases, u0, small matrices. The fixed-POD mode keeps only the
  // k = 0 snapshots and basis (one wave slot each) and no stage-1 bases.
  const bool plain = P.fixed || P.grid;   // no local bases after k = 0
  // A forced flow's operator has np time-space pieces: L_j is applied to
  // every basis separately, and the np forcing fields stay resident.
  P.np = flow_pieces(*p);
  P.forced = forced_flow(*p);
  // the warm-up solve's snapshots beyond one subinterval's (n_warm > 1)
  const size_t warm_snaps = (size_t)std::max(0, P.n_s0 - P.n_s) * cs;
  P.fixed_bytes = 2 * (size_t)(P.Np + 1) * f8 + Np1 * f8 +
                  (P.grid ? 0
                          : (P.fixed ? (size_t)P.n_s0 * cs + (1 + (size_t)P.np) * o->cap * cs
                                     : 2 * Np1 * o->cap0 * cs + warm_snaps)) +
                  (P.forced && !P.grid ? (size_t)P.np * cs : 0) + (size_t)P.nw * f8 +
                  ((size_t)4 << 20) +
                  (P.diag ? (size_t)(P.max_iter + 1) * Np1 * kDiagSlots * 8 : 0);
  P.perF = plain ? 0 : (size_t)P.n_s * cs;        // snapshots of one subinterval
  // stage-2 basis and the pieces of L applied to it
  P.perS = plain ? 0 : (1 + (size_t)P.np) * o->cap * cs;
  return P;
}

// Context scratch of the helpers per batched item: the fine propagator's
// work fields and the POD's Gram partials (two Grams: <= 10 and 3 tile
// pairs of 256 doubles per chunk) with its small matrices.
static size_t fine_scratch_item(long long ng, bool f32) { return (size_t)ng * (f32 ? 12 : 8); }
static size_t pod_scratch_item(long long ng) {
  const long long ch = gram_chunk_rows(ng);
  const long long nch = (ng + ch - 1) / ch;
  return (size_t)nch * 13 * 256 * 8 + ((size_t)96 << 10);
}

static size_t held_prefix(const pr_ctx* c, const std::string& prefix) {
  size_t b = 0;
  for (auto& kv : c->bufs)
    if (kv.first.compare(0, prefix.size(), prefix) == 0) b += kv.second.bytes;
  return b;
}

// Whether the helpers' scratch can grow to fine_b work-field bytes and pod_b
// POD bytes within the budget (idle pooled blocks count as free).
static bool helpers_fit(const pr_ctx* c, size_t fine_b, size_t pod_b) {
  size_t pooled = 0;
  for (auto& kv : c->pool) pooled += kv.first;
  const size_t hf = held_prefix(c, "sol_fine"), hp = held_prefix(c, "sol_pod");
  const size_t grow = (fine_b > hf ? fine_b - hf : 0) + (pod_b > hp ? pod_b - hp : 0);
  return c->used + grow <= c->budget + pooled;
}

// Context scratch shared by the helpers (fine work fields, POD partials,
// augmentation fields, L R, Gram partials of the sweep) for one solve.
static size_t shared_scratch_bytes(const Plan& P) {
  const size_t f8 = (size_t)P.ng * 8, fs = (size_t)P.ng * P.sf;
  const size_t nch = (size_t)gram_chunks_max(P.ng);
  // coarse-grid mode: two coarse fields, the coarse fine-step work fields
  const size_t grid = P.grid ? (size_t)P.pc.n * P.pc.n * P.pc.n * (16 + (P.f32 ? 12 : 8)) : 0;
  // coarse step: augmentation fields d, L_j d (co_fields) and Gram partials
  // of the widest Galerkin product (2 x (2 + 2 np + 1) tile pairs)
  const size_t gal = (size_t)2 * (2 + 2 * P.np + 1);
  return fine_scratch_item(P.ng, P.f32) * (size_t)std::max(P.waveF, 1) +
         pod_scratch_item(P.ng) * (size_t)std::max({P.waveF, P.waveS, 1}) +
         (1 + (size_t)P.np) * fs + f8 + (size_t)P.o.cap * fs +
         nch * std::max<size_t>(10, gal) * 256 * 8 + grid + (P.diag ? f8 : 0) +
         ((size_t)16 << 20);
}

static void choose_waves(Plan& P, size_t avail) {
  const int Np = std::max(P.Np, 1);
  auto need = [&](int wf, int ws) {
    Plan Q = P;
    Q.waveF = wf;
    Q.waveS = ws;
    return P.fixed_bytes + (size_t)wf * P.perF + (size_t)ws * P.perS + shared_scratch_bytes(Q);
  };
  if (need(1, 1) > avail) fail(PR_ENOMEM, "parareal solve does not fit the HBM budget");
  int wf = Np, ws = (P.fixed || P.grid) ? 1 : Np;
  while (need(wf, ws) > avail && (wf > 1 || ws > 1)) {
    // halve the larger of the two wave buffers first
    if (((size_t)wf * P.perF >= (size_t)ws * P.perS && wf > 1) || ws == 1 || P.fixed || P.grid)
      wf = (wf + 1) / 2;
    else ws = (ws + 1) / 2;
  }
  P.waveF = wf;
  P.waveS = ws;
}

// Column idx of a block whose columns are ld elements apart.
static ColDesc colp(const void* base, int idx, long long ld, bool f32, const int* mptr) {
  return ColDesc{(const char*)base + (size_t)idx * ld * (f32 ? 4 : 8), mptr, idx, f32 ? 1 : 0};
}
static ColDesc colnull() { return ColDesc{nullptr, nullptr, 0, 0}; }

}  // namespace pr

using namespace pr;

struct pr_solve {
  Plan P;
  const double* U_ref = nullptr;
  double* U[2] = {nullptr, nullptr};  // state sets (N' + 1 fields each)
  double* u0 = nullptr;               // copy of the initial field
  double* Fn = nullptr;
  char* R0 = nullptr;
  char* snaps = nullptr;
  char* Psi = nullptr;
  char* LPsi = nullptr;     // per wave slot: np blocks of cap columns (L_j Psi)
  char* forcing = nullptr;  // forced flows: f_j fields of the np pieces
  double* gaps = nullptr;   // diag: (max_iter + 1) x N' x kDiagSlots (coarse-gap norms,
                            // basis orthogonality)
  double *norms = nullptr, *betas0 = nullptr, *S0 = nullptr, *dscal = nullptr;
  int *m0slot = nullptr, *mS = nullptr, *misc = nullptr, *ranks = nullptr;
  double* host = nullptr;  // pinned: e_k, err_k
  std::vector<std::pair<void*, size_t>> owned;
  bool ext_out = false;    // U[0] lives in the caller's U_out
  // stage-1 POD items of this iteration waiting for the sweep part that first
  // needs them (subinterval, item), in increasing subinterval order
  std::vector<std::pair<int, PodWork>> pod1_pending;
  size_t pod1_next = 0;
  int k = 0;
  int prev = 0;            // U[prev] holds the latest iterate
  bool done = false;
  bool numeric_bad = false;
  pr_status fail_st = PR_OK;  // error that stopped the solve mid-iteration
  std::vector<double> jump, err, t_iter;
  int m0 = 0;
  double t_phase[5] = {0, 0, 0, 0, 0};
  double fine_updates = 0;
  std::chrono::steady_clock::time_point t0;
};

namespace pr {

static void* owned_alloc(pr_ctx* c, pr_solve* S, size_t bytes) {
  size_t got = 0;
  void* p = pool_get(c, bytes, &got);
  S->owned.push_back({p, got});
  return p;
}

// Return the solve's blocks to the context pool. `idle`: no queued work can
// still touch them (else the device is drained first).
static void release_solve(pr_ctx* c, pr_solve* S, bool idle) {
  if (!S) return;
  if (!idle) (void)hipDeviceSynchronize();
  for (auto& o : S->owned) pool_put(c, o.first, o.second);
  S->owned.clear();
  if (S->host) (void)hipHostFree(S->host);
  S->host = nullptr;
}

static double since(const pr_solve* S) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - S->t0).count();
}

// One coarse-grid coarse step over [t0, t0 + DeltaT]: out = P(F_c(R(a - b)))
// + fine (b, fine nullable), with the jump / error partials of out into
// norms4 (the comparison method with a coarser spatial discretisation,
// Sec. 4). For a forced flow F_c is affine; with b given the forcing cancels
// in F_c(R a) - F_c(R b), so the homogeneous propagator runs on R(a - b).
static void enqueue_grid_step(pr_ctx* c, pr_solve* S, const double* a, const double* b,
                              const double* fine, double* out, const double* prev,
                              const double* ref, double* norms4, double t0, hipStream_t s) {
  const Plan& P = S->P;
  const int m = P.pc.n;
  const long long mc = (long long)m * m * m;
  double* cb = (double*)scratch(c, "co_grid", (size_t)mc * 2 * 8);
  const int nwg = (int)std::min<long long>(4096, std::max<long long>(1, (P.ng + 2047) / 2048));
  double* part = (double*)scratch(c, "co_gpart", (size_t)nwg * 4 * 8);
  RestrictDesc rd{m, a, b, cb};
  RestrictDesc* rdd = stage_push1(c, rd);
  stage_flush(c, s);
  launch_restrict(rdd, mc, s);
  enqueue_fine(c, {FineWork{&S->P.pc, P.dt_c, P.n_g, cb, cb + mc, 0, nullptr, t0, b ? 1 : 0}}, s,
               "co_fine");
  const double h = spacing(P.prob);
  ProlongDesc pd{m, cb + mc, fine, out, prev, ref, part, nwg};
  ProlongDesc* pdd = stage_push1(c, pd);
  NormReduceDesc nr{part, nwg, h * h * h, norms4};
  NormReduceDesc* nrd = stage_push1(c, nr);
  stage_flush(c, s);
  launch_prolong_add(pdd, nwg, s);
  launch_norm_reduce(nrd, 1, s);
}

// Allocate the solve, enqueue k = 0 (Algorithm 2, initialisation) and synchronise.
static pr_solve* begin_solve(pr_ctx* c, const pr_grid_problem* prob, const pr_parareal_opts* opts,
                             const double* u0, double* U_out, hipStream_t s) {
  PR_CHECK(u0 != nullptr, "null initial field");
  Plan P = make_plan(prob, opts);
  {
    // the solve-owned memory comes on top of what the context already
    // holds; shared helper scratch may be regrown to fit this solve
    const size_t avail = c->budget > c->used ? c->budget - c->used : 0;
    size_t reusable = 0;
    for (auto& kv : c->bufs) reusable += kv.second.bytes;
    for (auto& kv : c->pool) reusable += kv.first;
    choose_waves(P, avail + reusable);
  }
  pr_solve* S = new pr_solve();
  S->P = P;
  S->U_ref = opts->U_ref;
  S->t0 = std::chrono::steady_clock::now();
  try {
    const long long ng = P.ng;
    const size_t f8 = (size_t)ng * 8, fs = (size_t)ng * P.sf;
    const int Np = P.Np;
    const size_t Np1 = (size_t)std::max(Np, 1);
    // S->u0: the warm-up window's states u0, F(DeltaT), ..., at t = j DeltaT,
    // j < nw (the first nw rows of U_out)
    if (U_out) {
      S->ext_out = true;
      S->U[0] = U_out + (size_t)P.nw * ng;
      S->u0 = U_out;
    } else {
      S->U[0] = (double*)owned_alloc(c, S, (size_t)(Np + 1) * f8);
      S->u0 = (double*)owned_alloc(c, S, (size_t)P.nw * f8);
    }
    S->U[1] = (double*)owned_alloc(c, S, (size_t)(Np + 1) * f8);
    S->Fn = (double*)owned_alloc(c, S, Np1 * f8);
    const size_t cs = P.cs;
    S->R0 = (P.fixed || P.grid) ? nullptr : (char*)owned_alloc(c, S, 2 * Np1 * P.o.cap0 * cs);
    if (!P.grid) {
      S->snaps = (char*)owned_alloc(
          c, S, (size_t)std::max((P.fixed ? 1 : P.waveF) * P.n_s, P.n_s0) * cs);
      S->Psi = (char*)owned_alloc(c, S, (size_t)P.waveS * P.o.cap * cs);
      S->LPsi = (char*)owned_alloc(c, S, (size_t)P.waveS * P.np * P.o.cap * cs);
      if (P.forced) S->forcing = (char*)owned_alloc(c, S, (size_t)P.np * cs);
    }
    if (P.diag) S->gaps = (double*)owned_alloc(c, S, (size_t)(P.max_iter + 1) * Np1 * kDiagSlots * 8);
    const int maxk = P.max_iter;
    const size_t n_norms = (size_t)(Np + 2) * 4, n_betas = Np1 * 32, n_S0 = 32 * 144, n_dscal = 8;
    const size_t n_dbl = n_norms + n_betas + n_S0 + n_dscal;
    const size_t n_int = 2 * Np1 + (size_t)P.waveS + 64 + (size_t)(maxk + 1) * Np1;
    char* small = (char*)owned_alloc(c, S, n_dbl * 8 + n_int * 4);
    S->norms = (double*)small;
    S->betas0 = S->norms + n_norms;
    S->S0 = S->betas0 + n_betas;
    S->dscal = S->S0 + n_S0;
    S->m0slot = (int*)((double*)small + n_dbl);
    S->mS = S->m0slot + 2 * Np1;
    S->misc = S->mS + P.waveS;
    S->ranks = S->misc + 64;
    PR_HIP(hipHostMalloc((void**)&S->host, 64));
    // shared helper scratch, pre-sized so nothing regrows mid-iteration
    const long long nch = gram_chunks_max(ng);
    scratch(c, "co_g_part", (size_t)nch * 10 * 256 * 8);
    scratch(c, "co_fields", fs * 2 + f8);
    scratch(c, "co_LR", (size_t)P.o.cap * fs);

    PR_HIP(hipMemsetAsync(small, 0, n_dbl * 8 + n_int * 4, s));
    if (S->u0 != u0) PR_HIP(hipMemcpyAsync(S->u0, u0, f8, hipMemcpyDeviceToDevice, s));
    S->err.assign(1, 0.0);

    const pr_grid_problem& p = S->P.prob;
    const double h = spacing(p), h3 = h * h * h;
    const int cap = P.o.cap;
    double* Ua = S->U[0];
    PhaseEvents ph;
    ph.c = c;
    ph.s = s;
    stage_begin(c, s);
    ph.begin(0);
    // the warm-up solve over [0, T_0] with its snapshots, and the window's
    // inner subinterval ends (the same steps from u0, so bitwise the states
    // the long solve passes through)
    std::vector<FineWork> warm{FineWork{&S->P.prob, P.dt, P.nw * P.n_f, S->u0, Ua,
                                        P.grid ? 0 : P.dM, P.grid ? nullptr : S->snaps, 0.0, 0,
                                        P.ld}};
    for (int j = 1; j < P.nw; ++j)
      warm.push_back(FineWork{&S->P.prob, P.dt, j * P.n_f, S->u0, S->u0 + (size_t)j * ng, 0,
                              nullptr, 0.0, 0, 0});
    enqueue_fine(c, warm, s, "sol_fine");
    S->fine_updates += (double)P.nw * P.n_f * ng;
    if (Np > 0 && P.grid) {
      // U^0_{n+1} = G(U^0_n) with the coarse-grid propagator
      ph.begin(4);
      for (int n = 0; n < Np; ++n)
        enqueue_grid_step(c, S, Ua + (size_t)n * ng, nullptr, nullptr, Ua + (size_t)(n + 1) * ng,
                          nullptr, S->U_ref ? S->U_ref + (size_t)(n + 1 + P.nw) * ng : nullptr,
                          S->norms + 4 * (n + 1), t_hat(P, n), s);
    } else if (Np > 0) {
      ph.begin(1);
      PodWork pw;
      pw.prob = &S->P.prob;
      for (int j = 0; j < P.n_s0; ++j) pw.cols.push_back(colp(S->snaps, j, P.ld, P.f32, nullptr));
      pw.gamma = P.o.gamma1;
      pw.cap = cap;
      pw.force_m = -1;
      pw.R_out = S->Psi;
      pw.R_ld = P.ld;
      pw.m_out = S->mS;
      pw.lambda_out = nullptr;
      enqueue_pod(c, {pw}, s, "sol_pod");
      ph.begin(2);
      // the Galerkin products of the k = 0 basis: Psi^T M [Psi, L_j Psi, U_0,
      // f_j] (one L block per time-space piece of a forced flow)
      const int np = P.np, nb = 2 + 2 * np + 1;
      enqueue_applyL_pieces(c, p, S->Psi, S->LPsi, cap, S->mS, s, P.ld);
      if (P.forced) enqueue_forcing_fields(c, p, S->forcing, s, P.ld);
      GramWork g;
      g.nrows = ng;
      std::vector<ColDesc> a;
      for (int j = 0; j < 32; ++j) a.push_back(j < cap ? colp(S->Psi, j, P.ld, P.f32, S->mS) : colnull());
      g.cols = a;
      g.cols.insert(g.cols.end(), a.begin(), a.end());
      for (int jp = 0; jp < np; ++jp)
        for (int j = 0; j < 32; ++j)
          g.cols.push_back(j < cap ? colp(S->LPsi + (size_t)jp * cap * P.cs, j, P.ld, P.f32, S->mS)
                                   : colnull());
      g.cols.push_back(ColDesc{Ua, nullptr, 0, 0});
      g.cols.push_back(colnull());
      for (int jp = 0; jp < np && P.forced; ++jp)
        g.cols.push_back(colp(S->forcing, jp, P.ld, P.f32, nullptr));
      g.cols.resize((2 + nb) * 16, colnull());
      g.out = S->S0;
      g.ld = 16 * nb;
      g.scale = h3;
      enqueue_gram(c, {g}, 2, nb, false, s, "co_g");
      ph.begin(4);
      Reduced0Desc d{};
      d.S = S->S0;
      d.ld = 16 * nb;
      d.cap = cap;
      d.m = S->mS;
      d.off_M = 0;
      d.off_L = 32;
      d.off_U = 32 + 32 * np;
      d.forced = P.forced ? geom_of(c, p).forced : 0;
      d.npieces = np;
      d.off_F = d.off_U + 2;
      d.w = P.forced ? p.fp[2] : 0.0;
      d.dT = P.dTs;
      d.n_c = P.n_c;
      d.n_warm = P.nw;
      d.count = Np;
      d.betas = S->betas0;
      d.ld_out = 32;
      d.n_c_out = S->misc + 1;
      Reduced0Desc* dd = stage_push1(c, d);
      stage_flush(c, s);
      launch_reduced0(dd, s);
      std::vector<ColDesc> psi;
      for (int j = 0; j < cap; ++j) psi.push_back(colp(S->Psi, j, P.ld, P.f32, S->mS));
      for (int n = 0; n < Np; ++n)
        enqueue_correct(c, ng, psi, S->betas0 + (size_t)n * 32, nullptr, 0,
                        Ua + (size_t)(n + 1) * ng, nullptr,
                        S->U_ref ? S->U_ref + (size_t)(n + 1 + P.nw) * ng : nullptr,
                        S->norms + 4 * (n + 1), h3, s, "sol");
    }
    enqueue_correct(c, ng, {}, nullptr, Ua, 0, Ua, nullptr,
                    S->U_ref ? S->U_ref + (size_t)P.nw * ng : nullptr, S->norms, h3, s, "sol");
    ph.end();
    PR_HIP(hipMemcpyAsync(S->U[1], Ua, f8, hipMemcpyDeviceToDevice, s));
    launch_jump_max(S->norms, Np + 1, S->dscal, s);
    PR_HIP(hipMemcpyAsync(S->host, S->dscal, 2 * 8, hipMemcpyDeviceToHost, s));
    PR_HIP(hipMemcpyAsync((char*)S->host + 16, S->mS, 4, hipMemcpyDeviceToHost, s));
    stage_end(c, s);
    PR_HIP(hipStreamSynchronize(s));
    ph.collect();
    for (int i = 0; i < 5; ++i) S->t_phase[i] += ph.t[i];
    S->m0 = Np > 0 ? *(int*)((char*)S->host + 16) : 0;
    S->err[0] = S->host[1];
    S->t_iter.push_back(since(S));
    S->prev = 0;
    S->k = 0;
    S->done = (Np == 0) || (P.max_iter == 0);
  } catch (...) {
    release_solve(c, S, false);
    delete S;
    throw;
  }
  return S;
}

// One parareal iteration of every unfinished solve in `ss`: the fine solves
// and stage-1 POD of all of them share launches (rounds of their waves),
// stage 2 and the sweep run solve by solve; one synchronisation at the end.
static void iterate_batch_impl(pr_ctx* c, const std::vector<pr_solve*>& live, hipStream_t s);

// A failure inside an iteration leaves the affected solves mid-iteration:
// they are stopped with the error, which pr_solve_end then returns.
static void iterate_batch(pr_ctx* c, const std::vector<pr_solve*>& ss, hipStream_t s) {
  std::vector<pr_solve*> live;
  for (auto* S : ss)
    if (!S->done) live.push_back(S);
  if (live.empty()) return;
  try {
    iterate_batch_impl(c, live, s);
  } catch (const Error& e) {
    (void)hipDeviceSynchronize();
    for (auto* S : live) {
      S->done = true;
      S->fail_st = e.st;
    }
    throw;
  } catch (...) {
    (void)hipDeviceSynchronize();
    for (auto* S : live) {
      S->done = true;
      S->fail_st = PR_EDEVICE;
    }
    throw;
  }
}

// Stage-1 modes left without their CholQR, which stage 2 folds into a block
// whitening of its Gram (PR_DEFER_CHOLQR, default 1; 0 keeps the stage-1 CholQR).
static bool defer_cholqr() {
  const char* e = getenv("PR_DEFER_CHOLQR");
  return !(e && *e == '0');
}

// Stage-1 POD run per sweep part, just before the part's stage-2 POD (on the
// second stream beside the sweep of the part before), rather than after the
// fine phase (PR_DEFER_POD1, default 1). Only for a solve whose fine phase is
// one wave, so its snapshots stay in place until the sweep.
static bool defer_pod1() {
  const char* e = getenv("PR_DEFER_POD1");
  return !(e && *e == '0');
}

// Enqueues the pending stage-1 items of S below subinterval `below`.
static void flush_pod1(pr_ctx* c, pr_solve* S, int below, hipStream_t st) {
  std::vector<PodWork> pw;
  while (S->pod1_next < S->pod1_pending.size() && S->pod1_pending[S->pod1_next].first < below)
    pw.push_back(S->pod1_pending[S->pod1_next++].second);
  for (int na = 1; na <= 4; ++na) {
    std::vector<PodWork> g;
    for (auto& x : pw)
      if (((int)x.cols.size() + 15) / 16 == na) g.push_back(x);
    if (!g.empty()) enqueue_pod(c, g, st, "sol_pod");
  }
}

// Parts a sweep wave is cut into (PR_SWEEP_PARTS, default 4; 1 runs the
// stage-2 POD of the whole wave before its sweep), each of at least
// kMinPartItems subintervals.
constexpr int kMinPartItems = 4;
// Subintervals in the first part of a sweep wave of wlen: PR_SWEEP_FIRST if
// set (0 splits the wave evenly), else wlen / 8. The first part's
// preparation is the only one the sweep cannot overlap.
static int sweep_first(int wlen) {
  const char* e = getenv("PR_SWEEP_FIRST");
  if (e && *e) return std::max(0, atoi(e));
  return std::max(1, wlen / 8);
}

static int sweep_parts() {
  const char* e = getenv("PR_SWEEP_PARTS");
  const int v = (e && *e) ? atoi(e) : 4;
  return std::max(1, std::min(v, 16));
}

static void iterate_batch_impl(pr_ctx* c, const std::vector<pr_solve*>& live, hipStream_t s) {
  PhaseEvents shared;  // phases shared by the batch are charged to each solve
  shared.c = c;
  shared.s = s;
  std::vector<PhaseEvents> own(live.size());
  std::vector<PhaseEvents> aux_ph(live.size());   // work on the auxiliary stream
  std::vector<hipEvent_t> used_events;
  stage_begin(c, s);
  for (auto* S : live) ++S->k;

  // (i) fine solves and stage-1 POD, in rounds of every solve's waves
  for (int round = 0;; ++round) {
    std::vector<FineWork> fw;
    std::vector<PodWork> pw;
    for (auto* S : live) {
      const Plan& P = S->P;
      const int k = S->k, Np = P.Np;
      const int n0 = (k - 1) + round * P.waveF;
      if (round == 0) {
        S->pod1_pending.clear();
        S->pod1_next = 0;
      }
      if (n0 >= Np) continue;
      const int n1 = std::min(Np, n0 + P.waveF);
      const bool defer1 = round == 0 && n1 == Np && defer_pod1();
      const size_t cs = P.cs;
      const double* Uprev = S->U[S->prev];
      for (int n = n0; n < n1; ++n) {
        if (P.fixed || P.grid) {
          // plain fine solves: no snapshots, no stage-1 basis (an empty POD
          // item is skipped below)
          fw.push_back(FineWork{&S->P.prob, P.dt, P.n_f, Uprev + (size_t)n * P.ng,
                                S->Fn + (size_t)n * P.ng, 0, nullptr, t_hat(P, n), 0});
          PodWork none;
          none.prob = &S->P.prob;
          pw.push_back(none);
          continue;
        }
        void* sn = S->snaps + (size_t)(n - n0) * P.n_s * cs;
        fw.push_back(FineWork{&S->P.prob, P.dt, P.n_f, Uprev + (size_t)n * P.ng,
                              S->Fn + (size_t)n * P.ng, P.dM, sn, t_hat(P, n), 0, P.ld});
        PodWork w;
        w.prob = &S->P.prob;
        for (int j = 0; j < P.n_s; ++j) w.cols.push_back(colp(sn, j, P.ld, P.f32, nullptr));
        w.gamma = P.o.gamma2;
        w.cap = P.o.cap0;
        w.force_m = -1;
        const int slot = k % 2;
        w.R_out = S->R0 + ((size_t)slot * Np + n) * P.o.cap0 * cs;
        w.R_ld = P.ld;
        w.skip_tail = 1;
        // the M-orthonormalisation of the stage-1 modes happens in stage 2
        w.cholqr = defer_cholqr() ? 0 : 1;
        w.m_out = S->m0slot + slot * Np + n;
        w.lambda_out = nullptr;
        if (defer1) {
          S->pod1_pending.emplace_back(n, w);
          PodWork none;
          none.prob = &S->P.prob;
          pw.push_back(none);
          continue;
        }
        pw.push_back(w);
      }
      S->fine_updates += (double)(n1 - n0) * P.n_f * P.ng;
    }
    if (fw.empty()) break;
    // one launch sequence per precision
    for (int prec = 0; prec < 2; ++prec) {
      std::vector<FineWork> f2;
      std::vector<PodWork> p2;
      for (size_t i = 0; i < fw.size(); ++i)
        if (fw[i].prob->precision == prec) {
          f2.push_back(fw[i]);
          p2.push_back(pw[i]);
        }
      // launches of as many items as the helpers' scratch can hold (the
      // waves of one solve always fit: its admission reserved them)
      size_t i0 = 0;
      while (i0 < f2.size()) {
        size_t i1 = i0 + 1, fb = 0, pb = 0;
        fb += fine_scratch_item(ngrid(*f2[i0].prob), prec == PR_MIXED);
        pb += p2[i0].cols.empty() ? 0 : pod_scratch_item(ngrid(*f2[i0].prob));
        for (; i1 < f2.size(); ++i1) {
          const long long ng1 = ngrid(*f2[i1].prob);
          const size_t fb1 = fb + fine_scratch_item(ng1, prec == PR_MIXED);
          const size_t pb1 = pb + (p2[i1].cols.empty() ? 0 : pod_scratch_item(ng1));
          if (!helpers_fit(c, fb1, pb1)) break;
          fb = fb1;
          pb = pb1;
        }
        std::vector<FineWork> fsub(f2.begin() + i0, f2.begin() + i1);
        std::vector<PodWork> psub(p2.begin() + i0, p2.begin() + i1);
        shared.begin(0);
        enqueue_fine(c, fsub, s, "sol_fine");
        shared.begin(1);
        for (int na = 1; na <= 4; ++na) {
          std::vector<PodWork> g;
          for (auto& x : psub)
            if (((int)x.cols.size() + 15) / 16 == na) g.push_back(x);
          if (!g.empty()) enqueue_pod(c, g, s, "sol_pod");
        }
        i0 = i1;
      }
    }
  }
  shared.end();

  for (size_t si = 0; si < live.size(); ++si) {
    pr_solve* S = live[si];
    PhaseEvents& ph = own[si];
    ph.c = c;
    ph.s = s;
    const Plan& P = S->P;
    const int k = S->k, Np = P.Np, cap = P.o.cap, cap0 = P.o.cap0;
    const long long ng = P.ng;
    const size_t f8 = (size_t)ng * 8;
    const double h = spacing(P.prob), h3 = h * h * h;
    double* Uprev = S->U[S->prev];
    double* Ucur = S->U[1 - S->prev];
    const double* Uref = S->U_ref;
    // (iii) converged prefix
    ph.begin(4);
    PR_HIP(hipMemcpyAsync(Ucur + (size_t)(k - 1) * ng, Uprev + (size_t)(k - 1) * ng, f8,
                          hipMemcpyDeviceToDevice, s));
    enqueue_correct(c, ng, {}, nullptr, S->Fn + (size_t)(k - 1) * ng, 0, Ucur + (size_t)k * ng,
                    Uprev + (size_t)k * ng, Uref ? Uref + (size_t)(k + P.nw) * ng : nullptr,
                    S->norms + 4 * k, h3, s, "sol");
    // (iv) for the coarse-grid mode: G(U^k_n) - G(U^{k-1}_n) = G(U^k_n -
    // U^{k-1}_n) by linearity, plus F_n
    if (P.grid) {
      ph.begin(4);
      for (int n = k; n < Np; ++n)
        enqueue_grid_step(c, S, Ucur + (size_t)n * ng, Uprev + (size_t)n * ng,
                          S->Fn + (size_t)n * ng, Ucur + (size_t)(n + 1) * ng,
                          Uprev + (size_t)(n + 1) * ng,
                          Uref ? Uref + (size_t)(n + 1 + P.nw) * ng : nullptr, S->norms + 4 * (n + 1),
                          t_hat(P, n), s);
    }
    // (iv) for the fixed-POD mode: the k = 0 basis (wave slot 0 of the stage-2
    // buffers, never overwritten in this mode) without augmentation
    if (P.fixed) {
      ph.begin(4);
      for (int n = k; n < Np; ++n) {
        CoarseWork w{};
        w.prob = &S->P.prob;
        w.R = S->Psi;
        w.LR = S->LPsi;
        w.ld = P.ld;
        w.cap = cap;
        w.m = S->mS;
        w.u_aug = nullptr;
        w.n_in = 2;
        w.u_in[0] = Ucur + (size_t)n * ng;
        w.u_in[1] = Uprev + (size_t)n * ng;
        w.dT = P.dTs;
        w.n_c = P.n_c;
        w.t0 = t_hat(P, n);
        w.forcing = S->forcing;
        if (P.diag) {
          w.diag_norms = S->gaps + ((size_t)k * Np + n) * kDiagSlots;
          w.diag_ref = Uref ? Uref + (size_t)(n + 1 + P.nw) * ng : nullptr;
        }
        w.corr_out = Ucur + (size_t)(n + 1) * ng;
        w.fine = S->Fn + (size_t)n * ng;
        w.prev = Uprev + (size_t)(n + 1) * ng;
        w.ref = Uref ? Uref + (size_t)(n + 1 + P.nw) * ng : nullptr;
        w.norms4 = S->norms + 4 * (n + 1);
        enqueue_coarse(c, w, s, &ph);
      }
    }
    // (ii) + (iv). A wave is cut into parts: the stage-2 POD and L Psi of
    // part i + 1 run on the auxiliary stream while the sweep crosses part i
    // (they read only the stage-1 bases, and each part has its own Psi,
    // L Psi and rank slots); the sweep of a part waits for its preparation.
    for (int n0 = k; n0 < Np && !P.fixed && !P.grid; n0 += P.waveS) {
      const int n1 = std::min(Np, n0 + P.waveS);
      // a stage-1 basis has rank <= min(cap0, n_s): only those slots of each
      // block enter W^k_n (the rest are masked out by the rank anyway)
      const int r0max = std::min(cap0, P.n_s);
      auto prep = [&](int a, int b, hipStream_t st, PhaseEvents& pe) {
        std::vector<PodWork> pw;
        std::vector<ApplyLWork> aw;
        for (int n = a; n < b; ++n) {
          PodWork w;
          w.prob = &S->P.prob;
          for (int j = std::max(0, n - P.o.ml); j <= n; ++j) {
            const int slot = std::min(k, j + 1) % 2;
            const char* base = S->R0 + ((size_t)slot * Np + j) * cap0 * P.cs;
            const int* mp = S->m0slot + slot * Np + j;
            for (int c0 = 0; c0 < r0max; ++c0) w.cols.push_back(colp(base, c0, P.ld, P.f32, mp));
          }
          if (P.o.p >= 1 && k - 1 >= 1) {
            const int slot = (k - 1) % 2;
            const char* base = S->R0 + ((size_t)slot * Np + n) * cap0 * P.cs;
            const int* mp = S->m0slot + slot * Np + n;
            for (int c0 = 0; c0 < r0max; ++c0) w.cols.push_back(colp(base, c0, P.ld, P.f32, mp));
          }
          w.gamma = P.o.gamma3;
          w.cap = cap;
          w.force_m = -1;
          w.R_out = S->Psi + (size_t)(n - n0) * cap * P.cs;
          w.R_ld = P.ld;
          w.m_out = S->mS + (n - n0);
          w.lambda_out = nullptr;
          w.skip_tail = 1;
          w.whiten_bs = defer_cholqr() ? r0max : 0;
          pw.push_back(w);
          for (int jp = 0; jp < P.np; ++jp)
            aw.push_back(ApplyLWork{&S->P.prob, w.R_out,
                                    S->LPsi + ((size_t)(n - n0) * P.np + jp) * cap * P.cs, cap,
                                    w.m_out, jp, P.ld, 1});
        }
        pe.begin(1);
        // stage-1 bases of subintervals up to b - 1 (W^k_n reads those of
        // n - m_l .. n)
        flush_pod1(c, S, b, st);
        for (int na = 1; na <= 4; ++na) {
          std::vector<PodWork> g;
          for (auto& x : pw)
            if (((int)x.cols.size() + 15) / 16 == na) g.push_back(x);
          if (!g.empty()) enqueue_pod(c, g, st, "sol_pod");
        }
        pe.begin(2);
        enqueue_applyL_batch(c, aw, st);
        PR_HIP(hipMemcpyAsync(S->ranks + (size_t)k * Np + a, S->mS + (a - n0), (size_t)(b - a) * 4,
                              hipMemcpyDeviceToDevice, st));
        pe.end();
      };
      const int nparts = std::max(1, std::min(sweep_parts(), (n1 - n0) / kMinPartItems));
      std::vector<int> cut;
      const int wlen = n1 - n0, first = sweep_first(wlen);
      if (nparts > 1 && first > 0 && first <= wlen - (nparts - 1)) {
        // a short first part: its preparation is the only one not overlapped
        cut.push_back(n0);
        for (int i = 0; i < nparts; ++i)
          cut.push_back(n0 + first + (int)((long long)(wlen - first) * i / (nparts - 1)));
      } else {
        for (int i = 0; i <= nparts; ++i) cut.push_back(n0 + (int)((long long)wlen * i / nparts));
      }
      std::vector<hipEvent_t> ready(nparts, nullptr);
      prep(cut[0], cut[1], s, ph);
      if (nparts > 1) {
        if (!c->aux) PR_HIP(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
        aux_ph[si].c = c;
        aux_ph[si].s = c->aux;
        // the auxiliary stream follows everything enqueued on s so far (the
        // stage-1 bases, and the first part's use of the POD scratch)
        hipEvent_t go = event_get(c);
        PR_HIP(hipEventRecord(go, s));
        PR_HIP(hipStreamWaitEvent(c->aux, go, 0));
        used_events.push_back(go);
        for (int i = 1; i < nparts; ++i) {
          prep(cut[i], cut[i + 1], c->aux, aux_ph[si]);
          ready[i] = event_get(c);
          PR_HIP(hipEventRecord(ready[i], c->aux));
          used_events.push_back(ready[i]);
        }
      }
      for (int i = 0; i < nparts; ++i) {
        if (ready[i]) PR_HIP(hipStreamWaitEvent(s, ready[i], 0));
        for (int n = cut[i]; n < cut[i + 1]; ++n) {
          CoarseWork w{};
          w.prob = &S->P.prob;
          w.R = S->Psi + (size_t)(n - n0) * cap * P.cs;
          w.LR = S->LPsi + (size_t)(n - n0) * P.np * cap * P.cs;
          w.ld = P.ld;
          w.cap = cap;
          w.m = S->mS + (n - n0);
          w.u_aug = Ucur + (size_t)n * ng;
          w.n_in = 2;
          w.u_in[0] = Ucur + (size_t)n * ng;
          w.u_in[1] = Uprev + (size_t)n * ng;
          w.dT = P.dTs;
          w.n_c = P.n_c;
          w.t0 = t_hat(P, n);
          w.forcing = S->forcing;
          if (P.diag) {
            w.diag_norms = S->gaps + ((size_t)k * Np + n) * kDiagSlots;
            w.diag_ref = Uref ? Uref + (size_t)(n + 1 + P.nw) * ng : nullptr;
          }
          w.corr_out = Ucur + (size_t)(n + 1) * ng;
          w.fine = S->Fn + (size_t)n * ng;
          w.prev = Uprev + (size_t)(n + 1) * ng;
          w.ref = Uref ? Uref + (size_t)(n + 1 + P.nw) * ng : nullptr;
          w.norms4 = S->norms + 4 * (n + 1);
          enqueue_coarse(c, w, s, &ph);
        }
      }
    }
    // stage-1 items no sweep part took (the sweep of the last iteration is
    // empty): their bases still complete the iteration
    if (S->pod1_next < S->pod1_pending.size()) {
      ph.begin(1);
      flush_pod1(c, S, Np, s);
    }
    ph.end();
    // (v) jump and error
    launch_jump_max(S->norms + 4 * k, Np - k + 1, S->dscal, s);
    launch_jump_max(S->norms, Np + 1, S->dscal + 2, s);
    PR_HIP(hipMemcpyAsync(S->host, S->dscal, 4 * 8, hipMemcpyDeviceToHost, s));
  }
  stage_end(c, s);
  PR_HIP(hipStreamSynchronize(s));   // s waited for every auxiliary part
  for (hipEvent_t e : used_events) event_put(c, e);
  shared.collect();
  for (size_t si = 0; si < live.size(); ++si) {
    pr_solve* S = live[si];
    own[si].collect();
    aux_ph[si].collect();
    for (int i = 0; i < 5; ++i) S->t_phase[i] += own[si].t[i] + aux_ph[si].t[i] + shared.t[i];
    const double e_k = S->host[0], err_k = S->host[3];
    S->jump.push_back(e_k);
    S->err.push_back(err_k);
    S->t_iter.push_back(since(S));
    S->prev = 1 - S->prev;
    if (!(e_k == e_k) || std::isinf(e_k)) {
      S->numeric_bad = true;
      S->done = true;
      continue;
    }
    const bool conv = (e_k <= S->P.o.tol) || (S->k == S->P.Np);
    S->done = conv || S->k >= S->P.max_iter;
  }
}

static bool converged(const pr_solve* S) {
  if (S->numeric_bad || S->fail_st != PR_OK) return false;
  if (S->P.Np == 0) return true;
  if (S->k == 0) return false;
  return S->jump.back() <= S->P.o.tol || S->k == S->P.Np;
}

// Copy the result into U_out ((N + 1) x N_g; may be the buffer given at
// begin) and fill the report.
static pr_status finish_solve(pr_ctx* c, pr_solve* S, double* U_out, pr_report* rep,
                              hipStream_t s) {
  (void)c;
  const Plan& P = S->P;
  const long long ng = P.ng;
  const size_t f8 = (size_t)ng * 8;
  const int Np = P.Np;
  if (U_out) {
    if (U_out != S->u0)
      PR_HIP(hipMemcpyAsync(U_out, S->u0, (size_t)P.nw * f8, hipMemcpyDeviceToDevice, s));
    if (U_out + (size_t)P.nw * ng != S->U[S->prev])
      PR_HIP(hipMemcpyAsync(U_out + (size_t)P.nw * ng, S->U[S->prev], (size_t)(Np + 1) * f8,
                            hipMemcpyDeviceToDevice, s));
  }
  if (rep) {
    rep->iters = S->k;
    rep->converged = converged(S) ? 1 : 0;
    rep->n_f = P.n_f;
    rep->dM = P.dM;
    rep->n_s = P.n_s;
    rep->n_c = P.n_c;
    rep->n_sub = Np;
    rep->m0 = S->m0;
    for (int i = 0; i < S->k; ++i)
      if (rep->jump) rep->jump[i] = S->jump[i];
    for (int i = 0; i <= S->k; ++i) {
      if (rep->err) rep->err[i] = S->err[i];
      if (rep->t_iter) rep->t_iter[i] = S->t_iter[i];
    }
    if (rep->ranks && S->k > 0 && Np > 0)
      PR_HIP(hipMemcpyAsync(rep->ranks, S->ranks, (size_t)(S->k + 1) * Np * 4,
                            hipMemcpyDeviceToHost, s));
    for (int i = 0; i < 5; ++i) rep->t_phase[i] = S->t_phase[i];
    rep->fine_updates = S->fine_updates;
    if (rep->gap_fine || rep->gap_ref || rep->basis_orth) {
      // coarse-gap diagnostics: sqrt(|F - G|^2 / |F|^2) and sqrt(|U_ref - G|^2 /
      // |U_ref|^2) per recorded sweep step, and the loss of M-orthonormality
      // of that step's basis; -1 elsewhere
      std::vector<double> g;
      if (P.diag && S->k > 0 && Np > 0) {
        g.resize((size_t)(S->k + 1) * Np * kDiagSlots);
        PR_HIP(hipMemcpyAsync(g.data(), S->gaps, g.size() * 8, hipMemcpyDeviceToHost, s));
        PR_HIP(hipStreamSynchronize(s));
      }
      for (int kk = 0; kk <= P.max_iter; ++kk)
        for (int n = 0; n < Np; ++n) {
          double gf = -1.0, gr = -1.0, bo = -1.0;
          if (!g.empty() && kk >= 1 && kk <= S->k && n >= kk) {
            const double* a = &g[((size_t)kk * Np + n) * kDiagSlots];
            if (a[3] > 0) gf = std::sqrt(a[1] / a[3]);
            if (S->U_ref && a[7] > 0) gr = std::sqrt(a[5] / a[7]);
            bo = a[8];
          }
          if (rep->gap_fine) rep->gap_fine[(size_t)kk * Np + n] = gf;
          if (rep->gap_ref) rep->gap_ref[(size_t)kk * Np + n] = gr;
          if (rep->basis_orth) rep->basis_orth[(size_t)kk * Np + n] = bo;
        }
    }
  }
  PR_HIP(hipStreamSynchronize(s));
  if (rep) rep->seconds = since(S);
  if (S->fail_st != PR_OK) return S->fail_st;
  if (S->numeric_bad) return PR_ENUMERIC;
  return converged(S) ? PR_OK : PR_ENOTCONV;
}

static size_t footprint(const pr_grid_problem* p, const pr_parareal_opts* o) {
  Plan P = make_plan(p, o);
  P.waveF = std::max(P.Np, 1);
  P.waveS = (P.fixed || P.grid) ? 1 : std::max(P.Np, 1);
  return P.fixed_bytes + P.perF * P.waveF + P.perS * P.waveS + shared_scratch_bytes(P);
}

}  // namespace pr

#define PR_TRY(ctx, body)                        \
  if (!(ctx)) return PR_EINVAL;                  \
  try {                                          \
    body                                         \
  } catch (const pr::Error& e) {                 \
    (ctx)->err = e.msg;                          \
    return e.st;                                 \
  } catch (const std::exception& e) {            \
    (ctx)->err = e.what();                       \
    return PR_EDEVICE;                           \
  }

extern "C" {

pr_status pr_parareal_solve(pr_ctx* c, const pr_grid_problem* prob, const pr_parareal_opts* opts,
                            const double* u0, double* U_out, pr_report* report, void* stream) {
  PR_TRY(c, {
    PR_CHECK(U_out != nullptr, "null output");
    PR_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    pr_solve* S = begin_solve(c, prob, opts, u0, U_out, s);
    pr_status st = PR_OK;
    try {
      while (!S->done) iterate_batch(c, {S}, s);
      st = finish_solve(c, S, U_out, report, s);
    } catch (...) {
      release_solve(c, S, false);
      delete S;
      throw;
    }
    release_solve(c, S, true);
    delete S;
    if (st != PR_OK)
      c->err = st == PR_ENOTCONV ? "max_iter reached above tol" : "NaN or Inf in a parareal jump";
    return st;
  })
}

pr_status pr_solve_begin(pr_ctx* c, const pr_grid_problem* prob, const pr_parareal_opts* opts,
                         const double* u0, pr_solve** out, void* stream) {
  PR_TRY(c, {
    PR_CHECK(out != nullptr, "null handle");
    *out = nullptr;
    PR_HIP(hipSetDevice(c->device));
    *out = begin_solve(c, prob, opts, u0, nullptr, (hipStream_t)stream);
    return PR_OK;
  })
}

pr_status pr_solve_step_batch(pr_ctx* c, int count, pr_solve* const* solves, int* done,
                              void* stream) {
  PR_TRY(c, {
    PR_CHECK(count >= 0 && (count == 0 || solves), "bad solve list");
    PR_HIP(hipSetDevice(c->device));
    std::vector<pr_solve*> ss(solves, solves + count);
    for (auto* S : ss) PR_CHECK(S != nullptr, "null solve handle");
    iterate_batch(c, ss, (hipStream_t)stream);
    if (done)
      for (int i = 0; i < count; ++i) done[i] = ss[i]->done ? 1 : 0;
    return PR_OK;
  })
}

pr_status pr_solve_state(pr_ctx* c, const pr_solve* S, int j, double* out, void* stream) {
  PR_TRY(c, {
    PR_CHECK(S != nullptr && out != nullptr, "null handle or output");
    PR_CHECK(j >= 0 && j <= S->P.N, "state index out of range");
    PR_HIP(hipSetDevice(c->device));
    const int nw = S->P.nw;
    const double* src = j < nw ? S->u0 + (size_t)j * S->P.ng
                               : S->U[S->prev] + (size_t)(j - nw) * S->P.ng;
    PR_HIP(hipMemcpyAsync(out, src, (size_t)S->P.ng * 8, hipMemcpyDeviceToDevice,
                          (hipStream_t)stream));
    return PR_OK;
  })
}

int pr_solve_done(const pr_solve* S) { return S ? (S->done ? 1 : 0) : 1; }

size_t pr_solve_bytes(const pr_solve* S) {
  size_t b = 0;
  if (S)
    for (auto& o : S->owned) b += o.second;
  return b;
}

pr_status pr_solve_end(pr_ctx* c, pr_solve* S, double* U_out, pr_report* report, void* stream) {
  PR_TRY(c, {
    PR_CHECK(S != nullptr, "null solve handle");
    PR_HIP(hipSetDevice(c->device));
    pr_status st = PR_OK;
    try {
      st = finish_solve(c, S, U_out, report, (hipStream_t)stream);
    } catch (...) {
      release_solve(c, S, false);
      delete S;
      throw;
    }
    release_solve(c, S, true);
    delete S;
    return st;
  })
}

pr_status pr_plan(const pr_grid_problem* prob, const pr_parareal_opts* opts, pr_plan_info* out) {
  if (!out) return PR_EINVAL;
  try {
    const Plan P = make_plan(prob, opts);
    out->n_sub = P.Np;
    out->n_f = P.n_f;
    out->dt = P.dt;
    out->dM = P.dM;
    out->n_s = P.n_s;
    out->n_c = P.n_c;
    out->max_iter = P.max_iter;
    return PR_OK;
  } catch (const pr::Error& e) {
    return e.st;
  }
}

pr_status pr_footprint(const pr_grid_problem* prob, const pr_parareal_opts* opts, size_t* bytes) {
  if (!bytes) return PR_EINVAL;
  try {
    *bytes = pr::footprint(prob, opts);
    return PR_OK;
  } catch (const pr::Error& e) {
    return e.st;
  }
}

}  // extern "C"
