// The adaptive parareal solve (formula4, Algorithm 2) on one GPU.
//
// Numbering: [0, T] is split into N subintervals; subinterval 0 is the
// warm-up window [0, T_0] (T_0 = DeltaT) whose fine solve gives u_hat_0 and
// the snapshots for G_0 (Case I); the parareal partition of [T_0, T] has
// N' = N - 1 subintervals with states U_n at t = (n + 1) DeltaT, n = 0..N'.
//
// Per iteration k >= 1:
//   (i)   fine solves F(U^{k-1}_n) with snapshots for n = k-1..N'-1, batched
//         in waves, and POD_Mode(gamma_2) of each snapshot set (Alg. 2 l. 8-9)
//   (ii)  POD_Mode(gamma_3) of W^k_n = [R_{n-m_l,0} .. R_{n,0}, R^{k-1}_{n,0}]
//         batched over n, and L applied to the modes (Alg. 2 l. 9-10)
//   (iii) U^k_j = U^{k-1}_j (j < k) and U^k_k = F_{k-1} (the coarse terms
//         cancel there)
//   (iv)  the sequential sweep n = k..N'-1: augmentation by U^k_n (eq12),
//         Galerkin system of eq13, RK4 of both projections and the
//         correction of formula4 with jump partials (Alg. 2 l. 12-17)
//   (v)   e_k = max_n ||U^k_n - U^{k-1}_n||_M / ||U^k_n||_M read back (8 B)
// The basis of subinterval j last computed at iteration min(k, j + 1) sits
// in slot min(k, j + 1) % 2 of a two-slot ring, which also holds
// R^{k-1}_{n,0} for p = 1.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "ctx.h"

namespace pr {

struct Plan {
  pr_grid_problem prob;
  pr_parareal_opts o;
  int N, Np, n_f, dM, n_s, n_c, max_iter;
  double dTs, dt;
  long long ng;
  bool f32;
  size_t sf;
  int waveF, waveS;
  size_t fixed_bytes, perF, perS;
};

static Plan make_plan(const pr_grid_problem* p, const pr_parareal_opts* o) {
  check_problem(p);
  PR_CHECK(o != nullptr, "null options");
  Plan P{};
  P.prob = *p;
  P.o = *o;
  PR_CHECK(o->N >= 1, "N must be >= 1");
  PR_CHECK(std::isfinite(o->T) && o->T > 0, "T must be positive");
  PR_CHECK(std::isfinite(o->dt) && o->dt > 0, "dt must be positive");
  PR_CHECK(o->dM >= 0, "dM must be >= 0");
  PR_CHECK(o->gamma1 > 0 && o->gamma1 <= 1 && o->gamma2 > 0 && o->gamma2 <= 1 && o->gamma3 > 0 &&
               o->gamma3 <= 1,
           "gamma must be in (0, 1]");
  PR_CHECK(o->cap0 >= 1 && o->cap0 <= kMaxCap && o->cap >= 1 && o->cap <= kMaxCap,
           "caps must be in [1, 31]");
  PR_CHECK(o->ml >= 0 && o->p >= 0 && o->p <= 1, "need m_l >= 0 and p in {0, 1}");
  PR_CHECK((o->ml + 1 + o->p) * o->cap0 <= kMaxPodCols,
           "(m_l + 1 + p) * cap0 must be <= 64 (local POD input)");
  PR_CHECK(o->coarse_ratio >= 1, "coarse_ratio must be >= 1");
  PR_CHECK(std::isfinite(o->tol) && o->tol >= 0, "tol must be >= 0");
  P.N = o->N;
  P.Np = o->N - 1;
  P.dTs = o->T / o->N;
  P.n_f = (int)std::max(1.0, std::ceil(P.dTs / o->dt - 1e-9));
  P.dt = P.dTs / P.n_f;
  P.dM = o->dM > 0 ? o->dM : (int)std::ceil(P.n_f / 16.0);
  P.dM = std::max(1, P.dM);
  P.n_s = P.n_f / P.dM + 1;
  PR_CHECK(P.n_s <= kMaxPodCols, "too many snapshots per subinterval (n_f / dM + 1 > 64)");
  P.n_c = std::max(1, (int)std::ceil(P.n_f / (double)o->coarse_ratio));
  P.max_iter = o->max_iter > 0 ? std::min(o->max_iter, P.Np) : P.Np;
  P.ng = ngrid(*p);
  P.f32 = p->precision == PR_MIXED;
  P.sf = P.f32 ? 4 : 8;
  if (P.dt * spectral_bound(*p) > kStabRK4)
    fail(PR_EUNSTABLE, "fine step exceeds the RK4 stability bound 2.6 / rho(L)");
  const size_t f8 = (size_t)P.ng * 8, fs = (size_t)P.ng * P.sf;
  const size_t Np = (size_t)std::max(P.Np, 1);
  P.fixed_bytes = (size_t)(P.Np + 1) * f8          // second state buffer
                  + (size_t)P.Np * f8                // F_n
                  + 2 * Np * o->cap0 * fs            // stage-1 bases, two slots
                  + 2 * fs + f8                      // augmentation fields
                  + (size_t)o->cap * fs              // L R scratch of the coarse step
                  + ((size_t)96 << 20);              // partials, small matrices
  P.perF = (size_t)P.n_s * fs + (P.f32 ? 3 * fs : 2 * f8);
  P.perS = 2 * (size_t)o->cap * fs;
  return P;
}

static void choose_waves(Plan& P, size_t budget) {
  const size_t need_min = P.fixed_bytes + P.perF + P.perS;
  if (need_min > budget) fail(PR_ENOMEM, "parareal solve does not fit the HBM budget");
  const size_t rest = budget - P.fixed_bytes;
  const int Np = std::max(P.Np, 1);
  // fine waves first (they carry the batched stencil), then the POD waves
  size_t wf = std::min<size_t>(Np, std::max<size_t>(1, (rest / 2) / P.perF));
  size_t ws = std::min<size_t>(Np, std::max<size_t>(1, (rest - wf * P.perF) / P.perS));
  if (ws < (size_t)Np && wf > 1) {
    // rebalance when the POD wave would be starved
    wf = std::min<size_t>(Np, std::max<size_t>(1, (rest - std::min<size_t>(Np, 8) * P.perS) / P.perF));
    ws = std::min<size_t>(Np, std::max<size_t>(1, (rest - wf * P.perF) / P.perS));
  }
  P.waveF = (int)wf;
  P.waveS = (int)ws;
}

static ColDesc colp(const void* base, int idx, long long ng, bool f32, const int* mptr) {
  return ColDesc{(const char*)base + (size_t)idx * ng * (f32 ? 4 : 8), mptr, idx, f32 ? 1 : 0};
}

static void solve(pr_ctx* c, const pr_grid_problem* prob, const pr_parareal_opts* opts,
                  const double* u0, double* U_out, pr_report* rep, hipStream_t s) {
  auto t_start = std::chrono::steady_clock::now();
  PR_CHECK(u0 && U_out, "null state pointer");
  Plan P = make_plan(prob, opts);
  {
    // buffers held under other names stay allocated; the solver's own
    // (sol_*, co_*) are reused or regrown
    size_t other = 0;
    for (auto& kv : c->bufs)
      if (kv.first.rfind("sol_", 0) != 0 && kv.first.rfind("co_", 0) != 0) other += kv.second.bytes;
    choose_waves(P, c->budget > other ? c->budget - other : 0);
  }
  const pr_grid_problem& p = P.prob;
  const long long ng = P.ng;
  const size_t f8 = (size_t)ng * 8, fs = (size_t)ng * P.sf;
  const int Np = P.Np;
  const double h = spacing(p), h3 = h * h * h;
  const int cap = P.o.cap, cap0 = P.o.cap0;

  // buffers: U_out holds u0 and one of the two state sets
  double* Ua = U_out + ng;  // U_n at t = (n + 1) DeltaT, n = 0..Np
  double* Ub = (double*)scratch(c, "sol_Ub", (size_t)(Np + 1) * f8);
  double* Fn = (double*)scratch(c, "sol_F", (size_t)std::max(Np, 1) * f8);
  char* R0 = (char*)scratch(c, "sol_R0", 2 * (size_t)std::max(Np, 1) * cap0 * fs);
  char* snaps = (char*)scratch(c, "sol_snaps", (size_t)P.waveF * P.n_s * fs);
  char* Psi = (char*)scratch(c, "sol_Psi", (size_t)P.waveS * cap * fs);
  char* LPsi = (char*)scratch(c, "sol_LPsi", (size_t)P.waveS * cap * fs);
  const int maxk = P.max_iter;
  const size_t Np1 = (size_t)std::max(Np, 1);
  // small device buffers: doubles first, then ints
  const size_t o_norms = 0, n_norms = (size_t)(Np + 2) * 4;
  const size_t o_betas = o_norms + n_norms, n_betas = Np1 * 32;
  const size_t o_S0 = o_betas + n_betas, n_S0 = 32 * 80;
  const size_t o_dscal = o_S0 + n_S0, n_dscal = 8;
  const size_t n_dbl = o_dscal + n_dscal;
  const size_t n_int = 2 * Np1 + (size_t)P.waveS + 64 + (size_t)(maxk + 1) * Np1;
  char* small = (char*)scratch(c, "sol_small", n_dbl * 8 + n_int * 4);
  double* norms = (double*)small + o_norms;                // (Np + 2) x 4
  double* betas0 = (double*)small + o_betas;               // Np x 32
  double* S0 = (double*)small + o_S0;                      // 32 x 80
  double* dscal = (double*)small + o_dscal;                // 8
  int* m0slot = (int*)((double*)small + n_dbl);            // 2 x Np
  int* mS = m0slot + 2 * Np1;                              // waveS
  int* misc = mS + P.waveS;                                // 64
  int* ranks = misc + 64;                                  // (maxk + 1) x Np
  PR_HIP(hipMemsetAsync(small, 0, n_dbl * 8 + n_int * 4, s));
  // pre-size the helpers' partial buffers (no reallocation mid-solve)
  {
    const int items_max = std::max(P.waveF, P.waveS);
    const long long chunk = gram_chunk_rows(ng, 1);
    const long long nch = (ng + chunk - 1) / chunk;
    scratch(c, "co_g_part", (size_t)nch * 10 * 256 * 8);
    scratch(c, "co_fields", fs * 2 + f8);
    (void)items_max;
  }

  pr_report local{};
  pr_report& R = rep ? *rep : local;
  R.iters = 0;
  R.converged = 0;
  R.n_f = P.n_f;
  R.dM = P.dM;
  R.n_s = P.n_s;
  R.n_c = P.n_c;
  R.n_sub = Np;
  for (int i = 0; i < 5; ++i) R.t_phase[i] = 0;
  R.fine_updates = 0;

  PhaseEvents ph;
  ph.c = c;
  ph.s = s;
  double* hs = c->host_scalars;
  auto elapsed = [&]() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  };

  // ---- k = 0 (Algorithm 2, lines 3-5) -----------------------------------
  stage_begin(c);
  PR_HIP(hipMemcpyAsync(U_out, u0, f8, hipMemcpyDeviceToDevice, s));
  ph.begin(0);
  enqueue_fine(c, {FineWork{&p, P.dt, P.n_f, u0, Ua, P.dM, snaps}}, s, "sol_fine");
  R.fine_updates += (double)P.n_f * ng;
  if (Np == 0) {
    ph.end();
    stage_end(c, s);
    PR_HIP(hipStreamSynchronize(s));
    ph.collect();
    for (int i = 0; i < 5; ++i) R.t_phase[i] = ph.t[i];
    R.converged = 1;
    R.seconds = elapsed();
    if (R.t_iter) R.t_iter[0] = R.seconds;
    return;
  }
  ph.begin(1);
  {
    PodWork pw;
    pw.prob = &p;
    for (int j = 0; j < P.n_s; ++j) pw.cols.push_back(colp(snaps, j, ng, P.f32, nullptr));
    pw.gamma = P.o.gamma1;
    pw.cap = cap;
    pw.force_m = -1;
    pw.R_out = Psi;
    pw.m_out = mS;
    pw.lambda_out = nullptr;
    enqueue_pod(c, {pw}, s, "sol_pod0");
  }
  ph.begin(2);
  enqueue_applyL(c, p, Psi, LPsi, cap, mS, s);
  {
    GramWork g;
    g.nrows = ng;
    std::vector<ColDesc> a;
    for (int j = 0; j < 32; ++j)
      a.push_back(j < cap ? colp(Psi, j, ng, P.f32, mS) : ColDesc{nullptr, nullptr, 0, 0});
    g.cols = a;
    g.cols.insert(g.cols.end(), a.begin(), a.end());
    for (int j = 0; j < 32; ++j)
      g.cols.push_back(j < cap ? colp(LPsi, j, ng, P.f32, mS) : ColDesc{nullptr, nullptr, 0, 0});
    g.cols.push_back(ColDesc{Ua, nullptr, 0, 0});
    g.cols.resize((2 + 5) * 16, ColDesc{nullptr, nullptr, 0, 0});
    g.out = S0;
    g.ld = 80;
    g.scale = h3;
    enqueue_gram(c, {g}, 2, 5, false, s, "co_g");
  }
  ph.begin(4);
  {
    Reduced0Desc d{};
    d.S = S0;
    d.ld = 80;
    d.cap = cap;
    d.m = mS;
    d.off_M = 0;
    d.off_L = 32;
    d.off_U = 64;
    d.dT = P.dTs;
    d.n_c = P.n_c;
    d.count = Np;
    d.betas = betas0;
    d.ld_out = 32;
    d.n_c_out = misc + 1;
    Reduced0Desc* dd = stage_push1(c, d);
    stage_flush(c, s);
    launch_reduced0(dd, s);
    std::vector<ColDesc> psi;
    for (int j = 0; j < cap; ++j) psi.push_back(colp(Psi, j, ng, P.f32, mS));
    const double* Uref = opts->U_ref;
    for (int n = 0; n < Np; ++n)
      enqueue_correct(c, ng, psi, betas0 + (size_t)n * 32, nullptr, 0, Ua + (size_t)(n + 1) * ng,
                      nullptr, Uref ? Uref + (size_t)(n + 2) * ng : nullptr,
                      norms + 4 * (n + 1), h3, s, "sol");
    enqueue_correct(c, ng, {}, nullptr, Ua, 0, Ua, nullptr, Uref ? Uref + (size_t)1 * ng : nullptr,
                    norms, h3, s, "sol");
  }
  ph.end();
  PR_HIP(hipMemcpyAsync(Ub, Ua, f8, hipMemcpyDeviceToDevice, s));
  launch_jump_max(norms, Np + 1, dscal, s);
  PR_HIP(hipMemcpyAsync(hs, dscal, 2 * 8, hipMemcpyDeviceToHost, s));
  PR_HIP(hipMemcpyAsync(hs + 2, mS, 4, hipMemcpyDeviceToHost, s));
  stage_end(c, s);
  PR_HIP(hipStreamSynchronize(s));
  ph.collect();
  R.m0 = *(int*)(hs + 2);
  if (R.err) R.err[0] = hs[1];
  if (R.t_iter) R.t_iter[0] = elapsed();

  double* Uprev = Ua;
  double* Ucur = Ub;
  const double* Uref = opts->U_ref;
  bool converged = false;
  bool numeric_bad = false;
  int k = 0;
  while (!converged && k < P.max_iter) {
    ++k;
    stage_begin(c);
    // (i) fine solves and stage-1 POD, in waves
    for (int n0 = k - 1; n0 < Np; n0 += P.waveF) {
      const int n1 = std::min(Np, n0 + P.waveF);
      std::vector<FineWork> fw;
      std::vector<PodWork> pw;
      for (int n = n0; n < n1; ++n) {
        void* sn = snaps + (size_t)(n - n0) * P.n_s * fs;
        fw.push_back(FineWork{&p, P.dt, P.n_f, Uprev + (size_t)n * ng, Fn + (size_t)n * ng, P.dM, sn});
        PodWork w;
        w.prob = &p;
        for (int j = 0; j < P.n_s; ++j) w.cols.push_back(colp(sn, j, ng, P.f32, nullptr));
        w.gamma = P.o.gamma2;
        w.cap = cap0;
        w.force_m = -1;
        const int slot = k % 2;
        w.R_out = R0 + ((size_t)slot * Np + n) * cap0 * fs;
        w.m_out = m0slot + slot * Np + n;
        w.lambda_out = nullptr;
        pw.push_back(w);
      }
      ph.begin(0);
      enqueue_fine(c, fw, s, "sol_fine");
      R.fine_updates += (double)(n1 - n0) * P.n_f * ng;
      ph.begin(1);
      enqueue_pod(c, pw, s, "sol_pod1");
    }
    // (iii) converged prefix
    ph.begin(4);
    PR_HIP(hipMemcpyAsync(Ucur + (size_t)(k - 1) * ng, Uprev + (size_t)(k - 1) * ng, f8,
                          hipMemcpyDeviceToDevice, s));
    enqueue_correct(c, ng, {}, nullptr, Fn + (size_t)(k - 1) * ng, 0, Ucur + (size_t)k * ng,
                    Uprev + (size_t)k * ng, Uref ? Uref + (size_t)(k + 1) * ng : nullptr,
                    norms + 4 * k, h3, s, "sol");
    // (ii) + (iv)
    for (int n0 = k; n0 < Np; n0 += P.waveS) {
      const int n1 = std::min(Np, n0 + P.waveS);
      std::vector<PodWork> pw;
      std::vector<ApplyLWork> aw;
      for (int n = n0; n < n1; ++n) {
        PodWork w;
        w.prob = &p;
        for (int j = std::max(0, n - P.o.ml); j <= n; ++j) {
          const int slot = std::min(k, j + 1) % 2;
          const char* base = R0 + ((size_t)slot * Np + j) * cap0 * fs;
          const int* mp = m0slot + slot * Np + j;
          for (int c0 = 0; c0 < cap0; ++c0) w.cols.push_back(colp(base, c0, ng, P.f32, mp));
        }
        if (P.o.p >= 1 && k - 1 >= 1) {
          const int slot = (k - 1) % 2;
          const char* base = R0 + ((size_t)slot * Np + n) * cap0 * fs;
          const int* mp = m0slot + slot * Np + n;
          for (int c0 = 0; c0 < cap0; ++c0) w.cols.push_back(colp(base, c0, ng, P.f32, mp));
        }
        w.gamma = P.o.gamma3;
        w.cap = cap;
        w.force_m = -1;
        w.R_out = Psi + (size_t)(n - n0) * cap * fs;
        w.m_out = mS + (n - n0);
        w.lambda_out = nullptr;
        pw.push_back(w);
        aw.push_back(ApplyLWork{&p, w.R_out, LPsi + (size_t)(n - n0) * cap * fs, cap, w.m_out});
      }
      ph.begin(1);
      // items with equal column counts share one launch
      for (int na = 1; na <= 4; ++na) {
        std::vector<PodWork> g;
        for (auto& x : pw)
          if (((int)x.cols.size() + 15) / 16 == na) g.push_back(x);
        if (!g.empty()) enqueue_pod(c, g, s, "sol_pod2");
      }
      ph.begin(2);
      enqueue_applyL_batch(c, aw, s);
      for (int n = n0; n < n1; ++n) {
        PR_HIP(hipMemcpyAsync(ranks + (size_t)k * Np + n, mS + (n - n0), 4, hipMemcpyDeviceToDevice, s));
        CoarseWork w{};
        w.prob = &p;
        w.R = Psi + (size_t)(n - n0) * cap * fs;
        w.LR = LPsi + (size_t)(n - n0) * cap * fs;
        w.cap = cap;
        w.m = mS + (n - n0);
        w.u_aug = Ucur + (size_t)n * ng;
        w.n_in = 2;
        w.u_in[0] = Ucur + (size_t)n * ng;
        w.u_in[1] = Uprev + (size_t)n * ng;
        w.dT = P.dTs;
        w.n_c = P.n_c;
        w.corr_out = Ucur + (size_t)(n + 1) * ng;
        w.fine = Fn + (size_t)n * ng;
        w.prev = Uprev + (size_t)(n + 1) * ng;
        w.ref = Uref ? Uref + (size_t)(n + 2) * ng : nullptr;
        w.norms4 = norms + 4 * (n + 1);
        enqueue_coarse(c, w, s, &ph);
      }
    }
    ph.end();
    // (v) jump and error
    launch_jump_max(norms + 4 * k, Np - k + 1, dscal, s);
    launch_jump_max(norms, Np + 1, dscal + 2, s);
    PR_HIP(hipMemcpyAsync(hs, dscal, 4 * 8, hipMemcpyDeviceToHost, s));
    stage_end(c, s);
    PR_HIP(hipStreamSynchronize(s));
    ph.collect();
    const double e_k = hs[0], err_k = hs[3];
    if (R.jump) R.jump[k - 1] = e_k;
    if (R.err) R.err[k] = err_k;
    if (R.t_iter) R.t_iter[k] = elapsed();
    std::swap(Uprev, Ucur);
    R.iters = k;
    if (!(e_k == e_k) || std::isinf(e_k)) {
      numeric_bad = true;
      break;
    }
    converged = (e_k <= P.o.tol) || (k == Np);
  }
  if (Np > 0 && Uprev != Ua)
    PR_HIP(hipMemcpyAsync(Ua, Uprev, (size_t)(Np + 1) * f8, hipMemcpyDeviceToDevice, s));
  if (R.ranks && k > 0)
    PR_HIP(hipMemcpyAsync(R.ranks, ranks, (size_t)(k + 1) * Np * 4, hipMemcpyDeviceToHost, s));
  PR_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < 5; ++i) R.t_phase[i] = ph.t[i];
  R.converged = converged ? 1 : 0;
  R.seconds = elapsed();
  if (numeric_bad) fail(PR_ENUMERIC, "NaN or Inf in a parareal jump");
  if (!converged) fail(PR_ENOTCONV, "max_iter reached above tol");
}

static size_t footprint(const pr_grid_problem* p, const pr_parareal_opts* o) {
  Plan P = make_plan(p, o);
  return P.fixed_bytes + P.perF * std::max(P.Np, 1) + P.perS * std::max(P.Np, 1);
}

}  // namespace pr

using namespace pr;

extern "C" {

pr_status pr_parareal_solve(pr_ctx* c, const pr_grid_problem* prob, const pr_parareal_opts* opts,
                            const double* u0, double* U_out, pr_report* report, void* stream) {
  if (!c) return PR_EINVAL;
  try {
    PR_HIP(hipSetDevice(c->device));
    pr::solve(c, prob, opts, u0, U_out, report, (hipStream_t)stream);
    return PR_OK;
  } catch (const pr::Error& e) {
    c->err = e.msg;
    return e.st;
  } catch (const std::exception& e) {
    c->err = e.what();
    return PR_EDEVICE;
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
