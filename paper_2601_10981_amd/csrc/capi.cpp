// libpr: context, staging and the fine / POD / coarse entry points.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <set>

#include "ctx.h"

namespace pr {

[[noreturn]] void fail(pr_status st, const std::string& msg) { throw Error{st, msg}; }

// ---------------------------------------------------------------------------
// scratch memory

// Free idle pooled blocks, largest first, until `bytes` more fit the budget.
static void make_room(pr_ctx* c, size_t bytes) {
  while (c->used + bytes > c->budget && !c->pool.empty()) {
    auto it = std::prev(c->pool.end());
    PR_HIP(hipFree(it->second));
    c->used -= it->first;
    c->pool.erase(it);
  }
}

void* pool_get(pr_ctx* c, size_t bytes, size_t* got) {
  bytes = std::max<size_t>(256, (bytes + 4095) & ~size_t(4095));
  auto it = c->pool.lower_bound(bytes);
  if (it != c->pool.end() && it->first <= bytes + bytes / 8) {
    void* p = it->second;
    *got = it->first;
    c->pool.erase(it);
    return p;
  }
  make_room(c, bytes);
  if (c->used + bytes > c->budget) fail(PR_ENOMEM, "solve memory exceeds the HBM budget");
  void* p = nullptr;
  PR_HIP(hipMalloc(&p, bytes));
  c->used += bytes;
  *got = bytes;
  return p;
}

void pool_put(pr_ctx* c, void* p, size_t bytes) { c->pool.insert({bytes, p}); }

void* scratch(pr_ctx* c, const std::string& name, size_t bytes) {
  bytes = std::max<size_t>(bytes, 256);
  bytes = (bytes + 4095) & ~size_t(4095);
  auto& b = c->bufs[name];
  if (b.bytes >= bytes) return b.p;
  if (b.p) {
    PR_HIP(hipDeviceSynchronize());
    PR_HIP(hipFree(b.p));
    c->used -= b.bytes;
    b = pr_ctx::Buf{};
  }
  make_room(c, bytes);
  if (c->used + bytes > c->budget) {
    char msg[256];
    snprintf(msg, sizeof msg, "scratch '%s' of %zu bytes exceeds the budget (%zu of %zu used)",
             name.c_str(), bytes, c->used, c->budget);
    fail(PR_ENOMEM, msg);
  }
  PR_HIP(hipMalloc(&b.p, bytes));
  b.bytes = bytes;
  c->used += bytes;
  return b.p;
}

void release_all(pr_ctx* c) {
  for (auto& kv : c->bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  c->bufs.clear();
  for (auto& kv : c->pool) (void)hipFree(kv.second);
  c->pool.clear();
  c->used = 0;
}

// ---------------------------------------------------------------------------
// descriptor staging
void stage_begin(pr_ctx* c, hipStream_t s) {
  c->stream = s;
  stage_begin(c);
}

void stage_begin(pr_ctx* c) {
  c->slot = (c->slot + 1) % pr_ctx::kSlots;
  PR_HIP(hipEventSynchronize(c->slot_ev[c->slot]));
  c->off = 0;
  c->flushed = 0;
}

void* stage_push_bytes(pr_ctx* c, const void* src, size_t bytes) {
  if (bytes > pr_ctx::kSlotBytes) fail(PR_ENOMEM, "descriptor block larger than a staging slot");
  size_t o = (c->off + 255) & ~size_t(255);
  if (o + bytes > pr_ctx::kSlotBytes) {
    // rotate to a fresh slot; what was pushed so far is copied first
    const hipStream_t s = c->stream;
    stage_end(c, s);
    stage_begin(c, s);
    o = 0;
  }
  if (bytes) memcpy(c->host_slot[c->slot] + o, src, bytes);
  c->off = o + bytes;
  return c->dev_slot[c->slot] + o;
}

// Flushes of up to kUploadMax bytes travel in the arguments of k_upload
// launches (PR_STAGE_UPLOAD=0: always a copy). The range is widened to whole
// 4-byte words inside the slot; bytes below `flushed` are rewritten with the
// values they already hold.
constexpr size_t kUploadMax = 4 * sizeof(UploadBlob);
static bool stage_upload() {
  static const bool on = [] {
    const char* e = getenv("PR_STAGE_UPLOAD");
    return !(e && *e == '0');
  }();
  return on;
}

void stage_flush(pr_ctx* c, hipStream_t s) {
  c->stream = s;
  if (c->off > c->flushed) {
    const size_t b0 = c->flushed & ~size_t(3);
    const size_t b1 = (c->off + 3) & ~size_t(3);
    static_assert(pr_ctx::kSlotBytes % 4 == 0, "slots hold whole words");
    if (stage_upload() && b1 - b0 <= kUploadMax) {
      UploadBlob blob;
      for (size_t b = b0; b < b1; b += sizeof(UploadBlob)) {
        const size_t nb = std::min(sizeof(UploadBlob), b1 - b);
        memcpy(blob.w, c->host_slot[c->slot] + b, nb);
        launch_upload(blob, (unsigned int*)(c->dev_slot[c->slot] + b), (int)(nb / 4), s);
      }
    } else {
      PR_HIP(hipMemcpyAsync(c->dev_slot[c->slot] + c->flushed, c->host_slot[c->slot] + c->flushed,
                            c->off - c->flushed, hipMemcpyHostToDevice, s));
    }
    c->flushed = c->off;
  }
}

// The slot's event is recorded at its end and again at the end of the next
// slot: a helper that rotated mid-way may launch, in the next slot, a kernel
// still reading descriptors of this one.
void stage_end(pr_ctx* c, hipStream_t s) {
  stage_flush(c, s);
  PR_HIP(hipEventRecord(c->slot_ev[c->slot], s));
  const int prev = (c->slot + pr_ctx::kSlots - 1) % pr_ctx::kSlots;
  PR_HIP(hipEventRecord(c->slot_ev[prev], s));
}

hipEvent_t event_get(pr_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  PR_HIP(hipEventCreate(&e));
  return e;
}
void event_put(pr_ctx* c, hipEvent_t e) { c->ev_pool.push_back(e); }

hipEvent_t timing_event_get(pr_ctx* c) {
  if (!c->ev_pool_timing.empty()) {
    hipEvent_t e = c->ev_pool_timing.back();
    c->ev_pool_timing.pop_back();
    return e;
  }
  hipEvent_t e;
  PR_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  return e;
}
void timing_event_put(pr_ctx* c, hipEvent_t e) { c->ev_pool_timing.push_back(e); }

PhaseEvents::~PhaseEvents() {
  if (c)
    for (hipEvent_t e : marks) timing_event_put(c, e);
}
hipEvent_t PhaseEvents::mark() {
  hipEvent_t e = timing_event_get(c);
  marks.push_back(e);
  PR_HIP(hipEventRecord(e, s));
  return e;
}
void PhaseEvents::begin(int phase) {
  if (!c || phase == cur) return;
  hipEvent_t e = mark();
  if (cur >= 0) open.push_back({cur, {cur_start, e}});
  cur = phase;
  cur_start = e;
}
void PhaseEvents::end() {
  if (!c || cur < 0) return;
  open.push_back({cur, {cur_start, mark()}});
  cur = -1;
  cur_start = nullptr;
}
void PhaseEvents::collect() {
  if (!c) return;
  for (auto& o : open) {
    float ms = 0.f;
    PR_HIP(hipEventElapsedTime(&ms, o.second.first, o.second.second));
    t[o.first] += ms * 1e-3;
  }
  open.clear();
  // events of the running phase stay out of the pool until it ends
  size_t keep = 0;
  for (hipEvent_t e : marks) {
    if (e == cur_start) marks[keep++] = e;
    else timing_event_put(c, e);
  }
  marks.resize(keep);
}

// ---------------------------------------------------------------------------
// problems
double spacing(const pr_grid_problem& p) { return p.L / p.n; }

void check_problem(const pr_grid_problem* p) {
  PR_CHECK(p != nullptr, "null problem");
  PR_CHECK(p->n >= 4 && p->n <= 2048, "grid size n must be in [4, 2048]");
  PR_CHECK(std::isfinite(p->L) && p->L > 0, "domain length L must be positive");
  PR_CHECK(std::isfinite(p->kappa) && p->kappa >= 0, "kappa must be >= 0");
  PR_CHECK(p->flow == PR_FLOW_UNIFORM || p->flow == PR_FLOW_ABC || p->flow == PR_FLOW_KOLMOGOROV ||
               p->flow == PR_FLOW_KOLMOGOROV_T || p->flow == PR_FLOW_ABC_T,
           "unknown flow");
  PR_CHECK(p->precision == PR_F64 || p->precision == PR_MIXED, "unknown precision");
  for (int i = 0; i < 3; ++i) PR_CHECK(std::isfinite(p->fp[i]), "flow parameters must be finite");
}

// Upper bound of |lambda(L)|: 12 kappa / h^2 + sum_d sup|v_d| / h.
double spectral_bound(const pr_grid_problem& p) {
  const double h = spacing(p);
  double vs = 0;
  if (p.flow == PR_FLOW_ABC) {
    const double A = fabs(p.fp[0]), B = fabs(p.fp[1]), C = fabs(p.fp[2]);
    vs = (A + C) + (B + A) + (C + B);
  } else if (p.flow == PR_FLOW_KOLMOGOROV) {
    vs = fabs(p.fp[0]);
  } else if (forced_flow(p)) {
    vs = 6.0 * fabs(p.fp[0]);   // each component: two terms of magnitude <= |a_v|
  } else {
    vs = fabs(p.fp[0]) + fabs(p.fp[1]) + fabs(p.fp[2]);
  }
  return 12.0 * p.kappa / (h * h) + vs / h;
}

bool forced_flow(const pr_grid_problem& p) {
  return p.flow == PR_FLOW_KOLMOGOROV_T || p.flow == PR_FLOW_ABC_T;
}
int flow_pieces(const pr_grid_problem& p) {
  return p.flow == PR_FLOW_ABC_T ? 3 : (p.flow == PR_FLOW_KOLMOGOROV_T ? 2 : 1);
}

// Tables of the forced flows' pieces (layout in pr_internal.h), velocities
// pre-multiplied by s = 1 / (2 h):
//   Kolmogorov (a_v, a_f, w), theta = (1, cos(w t)):
//     piece 0: v = a_v (cos y, cos z, cos x), f = -a_f cos y
//     piece 1: v = a_v (sin z, sin x, sin y), f = -a_f sin z
//   ABC with phase s(t) = sin(w t), theta = (1, cos s, sin s):
//     piece 0: v = 0, f = 0
//     piece 1: v = a_v (sin z + cos y, sin x + cos z, sin y + cos x),
//              f = -a_f (sin z + cos y)
//     piece 2: v = a_v (cos z - sin y, cos x - sin z, cos y - sin x),
//              f = -a_f (cos z - sin y)
static std::vector<double> forced_tables(const pr_grid_problem& p) {
  const int n = p.n, np = flow_pieces(p);
  const double h = spacing(p), s = 1.0 / (2.0 * h);
  const double av = p.fp[0] * s, af = p.fp[1];
  std::vector<double> t((size_t)np * 9 * n, 0.0);
  auto T = [&](int j, int tab, int i) -> double& { return t[((size_t)j * 9 + tab) * n + i]; };
  for (int i = 0; i < n; ++i) {
    const double x = i * h, sx = sin(x), cx = cos(x);
    if (p.flow == PR_FLOW_KOLMOGOROV_T) {
      T(0, 0, i) = av * cx;    // v_x: cos y
      T(0, 3, i) = av * cx;    // v_y: cos z
      T(0, 4, i) = av * cx;    // v_z: cos x
      T(0, 7, i) = -af * cx;   // f: -cos y
      T(1, 1, i) = av * sx;    // v_x: sin z
      T(1, 2, i) = av * sx;    // v_y: sin x
      T(1, 5, i) = av * sx;    // v_z: sin y
      T(1, 8, i) = -af * sx;   // f: -sin z
    } else {
      T(1, 0, i) = av * cx;    // v_x: cos y + sin z
      T(1, 1, i) = av * sx;
      T(1, 2, i) = av * sx;    // v_y: sin x + cos z
      T(1, 3, i) = av * cx;
      T(1, 4, i) = av * cx;    // v_z: cos x + sin y
      T(1, 5, i) = av * sx;
      T(1, 7, i) = -af * cx;   // f: -(cos y + sin z)
      T(1, 8, i) = -af * sx;
      T(2, 0, i) = -av * sx;   // v_x: -sin y + cos z
      T(2, 1, i) = av * cx;
      T(2, 2, i) = av * cx;    // v_y: cos x - sin z
      T(2, 3, i) = -av * sx;
      T(2, 4, i) = -av * sx;   // v_z: -sin x + cos y
      T(2, 5, i) = av * cx;
      T(2, 7, i) = af * sx;    // f: -(cos z - sin y)
      T(2, 8, i) = -af * cx;
    }
  }
  return t;
}

Geom geom_of(pr_ctx* c, const pr_grid_problem& p) {
  char key[256];
  snprintf(key, sizeof key, "%d|%a|%d|%a|%a|%a", p.n, p.L, p.flow, p.fp[0], p.fp[1], p.fp[2]);
  const int n = p.n;
  auto it = c->tables.find(key);
  void* dev = nullptr;
  if (it == c->tables.end()) {
    const double h = spacing(p), s = 1.0 / (2.0 * h);
    std::vector<double> t(6 * (size_t)n, 0.0);
    if (forced_flow(p)) t = forced_tables(p);
    for (int i = 0; i < n && !forced_flow(p); ++i) {
      const double x = i * h;
      if (p.flow == PR_FLOW_ABC) {
        const double A = p.fp[0], B = p.fp[1], C = p.fp[2];
        t[0 * n + i] = C * cos(x) * s;   // v_x: C cos y
        t[1 * n + i] = A * sin(x) * s;   // v_x: A sin z
        t[2 * n + i] = B * sin(x) * s;   // v_y: B sin x
        t[3 * n + i] = A * cos(x) * s;   // v_y: A cos z
        t[4 * n + i] = B * cos(x) * s;   // v_z: B cos x
        t[5 * n + i] = C * sin(x) * s;   // v_z: C sin y
      } else if (p.flow == PR_FLOW_KOLMOGOROV) {
        t[0 * n + i] = p.fp[0] * sin(p.fp[1] * x) * s;
      } else {
        t[0 * n + i] = p.fp[0] * s;
        t[2 * n + i] = p.fp[1] * s;
        t[4 * n + i] = p.fp[2] * s;
      }
    }
    std::vector<float> tf(t.size());
    for (size_t i = 0; i < t.size(); ++i) tf[i] = (float)t[i];
    const size_t bytes = t.size() * 8 + tf.size() * 4;
    PR_HIP(hipMalloc(&dev, bytes));
    PR_HIP(hipMemcpy(dev, t.data(), t.size() * 8, hipMemcpyHostToDevice));
    PR_HIP(hipMemcpy((char*)dev + t.size() * 8, tf.data(), tf.size() * 4, hipMemcpyHostToDevice));
    c->tables[key] = dev;
  } else {
    dev = it->second;
  }
  const double h = spacing(p);
  Geom g;
  g.n = n;
  g.xonly = (p.flow == PR_FLOW_KOLMOGOROV) ||
            (p.flow == PR_FLOW_UNIFORM && p.fp[1] == 0.0 && p.fp[2] == 0.0);
  g.c_lap = p.kappa / (h * h);
  const size_t nt = forced_flow(p) ? (size_t)flow_pieces(p) * 9 * n : 6 * (size_t)n;
  g.tab64 = (const double*)dev;
  g.tab32 = (const float*)((char*)dev + nt * 8);
  g.forced = p.flow == PR_FLOW_KOLMOGOROV_T ? kForcedKolmogorov
                                            : (p.flow == PR_FLOW_ABC_T ? kForcedABC : kForcedNone);
  g.npieces = flow_pieces(p);
  g.w = forced_flow(p) ? p.fp[2] : 0.0;
  g.ptab64 = g.forced ? g.tab64 : nullptr;
  g.ptab32 = g.forced ? g.tab32 : nullptr;
  if (g.forced) g.xonly = 0;
  return g;
}

// Piece j of a forced flow's operator as a steady operator: kappa Lap -
// v_0 . grad for j = 0, -v_j . grad for j > 0 (tables of piece j).
Geom geom_piece(const Geom& g, int j) {
  Geom q = g;
  if (!g.forced) return q;
  q.tab64 = g.ptab64 + (size_t)9 * g.n * j;
  q.tab32 = g.ptab32 + (size_t)9 * g.n * j;
  if (j > 0) q.c_lap = 0.0;
  q.forced = kForcedNone;
  q.npieces = 1;
  q.ptab64 = nullptr;
  q.ptab32 = nullptr;
  return q;
}

// Rows per Gram chunk: a function of the row count only (about 512 chunks,
// at least 1024 rows, a multiple of 64), never of the batch composition, so
// a result is bitwise the same whatever else shares the launch.
int gram_chunk_rows(long long nrows) {
  long long ch = (nrows + 511) / 512;
  ch = std::max<long long>(ch, 1024);
  ch = (ch + 63) / 64 * 64;
  const long long cap = (nrows + 63) / 64 * 64;
  return (int)std::min(ch, std::max<long long>(cap, 64));
}

// One item alone: about three workgroups per CU (its kernel holds three
// waves per SIMD), so that enough row loads are in flight.
constexpr long long kGalerkinChunks = 768;
int galerkin_chunk_rows(long long nrows) {
  long long ch = (nrows + kGalerkinChunks - 1) / kGalerkinChunks;
  ch = std::max<long long>(ch, 1024);
  ch = (ch + 63) / 64 * 64;
  const long long cap = (nrows + 63) / 64 * 64;
  return (int)std::min(ch, std::max<long long>(cap, 64));
}

long long gram_chunks_max(long long nrows) {
  const long long a = gram_chunk_rows(nrows), b = galerkin_chunk_rows(nrows);
  return std::max((nrows + a - 1) / a, (nrows + b - 1) / b);
}

// ---------------------------------------------------------------------------
// fine propagator
// Chunk-length policies of the fused stencil (fine_chunk). Policies 0 and 1
// halve chunks while a launch has fewer than 2048 / 768 workgroups. Policy 2
// takes the length of least modelled time, ceil(workgroups / resident
// workgroups) x (planes + warm-up planes): a launch runs in rounds of the
// workgroups the chip holds at once, each marching its whole chunk, so a
// partly filled last round costs about a full one.
constexpr int kChunkPolicies = 3;
constexpr long long kChunkMinWgs[kChunkPolicies] = {2048, 768, -1};
constexpr int kWarmPlanes = 6;   // planes a chunk marches before its first output

// Tile configuration of the fused stencil: PR_FUSED_CFG=<index> forces one;
// otherwise each (precision, largest grid, batch size class) is tuned once
// per context (see tune_fine).
static int forced_cfg() {
  const char* e = getenv("PR_FUSED_CFG");
  if (!e || !*e) return -1;
  const int v = atoi(e);
  if (v < 0 || v >= kNumFusedCfgs) return -1;
  const char* p = getenv("PR_FUSED_CHUNK");
  const int pol = (p && *p) ? atoi(p) : 0;
  return v + kNumFusedCfgs * ((pol >= 0 && pol < kChunkPolicies) ? pol : 0);
}
// The same for the forced-flow stencil: PR_FORCED_CFG=<index into
// kForcedCfgs> (with PR_FUSED_CHUNK).
static int forced_cfg_forced() {
  const char* e = getenv("PR_FORCED_CFG");
  if (!e || !*e) return -1;
  const int v = atoi(e);
  if (v < 0 || v >= kNumForcedCfgs) return -1;
  const char* p = getenv("PR_FUSED_CHUNK");
  const int pol = (p && *p) ? atoi(p) : 0;
  return kForcedCfgs[v] + kNumFusedCfgs * ((pol >= 0 && pol < kChunkPolicies) ? pol : 0);
}

// x-chunk length of the fused stencil: chunks of up to kMaxChunk planes,
// halved while the batch would give fewer than min_wgs workgroups (small
// batches, e.g. the serial fine solve of one field, still fill the chip).
// Longer chunks re-read fewer warm-up planes (6 per chunk); shorter ones give
// more workgroups. The tuner tries both policies.
static int fine_chunk(const std::vector<FineWork>& items, int cfg, long long min_wgs,
                      bool forced, long long slots) {
  int xc = forced ? kForcedChunk : (kFusedCfgs[cfg].blocked ? kBlockedChunk : kMaxChunk);
  int nmax = 1;
  auto total = [&](int x) {
    long long t = 0;
    for (auto& w : items) {
      const long long ty = (w.prob->n + fused_ty(cfg) - 1) / fused_ty(cfg);
      const long long tz = (w.prob->n + fused_tz(cfg) - 1) / fused_tz(cfg);
      t += ty * tz * ((w.prob->n + x - 1) / x);
      nmax = std::max(nmax, w.prob->n);
    }
    return t;
  };
  if (min_wgs >= 0) {
    while (xc > 8 && total(xc) < min_wgs) xc /= 2;
    return xc;
  }
  int best = xc;
  double best_cost = 0.0;
  for (int x = xc; x >= 8; x /= 2) {
    const long long rounds = (total(x) + slots - 1) / slots;
    const double cost = (double)rounds * (std::min(x, nmax) + kWarmPlanes);
    if (x == xc || cost < best_cost) {   // ties keep the longer chunk
      best_cost = cost;
      best = x;
    }
  }
  return best;
}

// Workgroups of tiling cfg the device holds at once (cached per context).
static long long resident_slots(const pr_ctx* c, int cfg, bool f32, bool forced, bool xonly) {
  const int key = cfg * 8 + (f32 ? 1 : 0) + (forced ? 2 : 0) + (xonly ? 4 : 0);
  auto it = c->fused_slots.find(key);
  if (it != c->fused_slots.end()) return it->second;
  if (c->n_cu <= 0)
    PR_HIP(hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device));
  const int per_cu =
      forced ? forced_blocks_per_cu(cfg, f32) : fused_blocks_per_cu(cfg, f32, xonly);
  const long long v = std::max<long long>(1, (long long)per_cu * std::max(1, c->n_cu));
  c->fused_slots[key] = v;
  return v;
}

// Descriptors of one launch shape: per-item buffers fixed in `base`, tiles
// of configuration cfg filled in. Returns the number of workgroup tiles.
// A launch shape: tiling kFusedCfgs[code % kNumFusedCfgs], chunk policy
// code / kNumFusedCfgs.
template <typename T>
static bool all_xonly(const std::vector<FineDesc<T>>& d) {
  for (auto& x : d)
    if (!x.g.xonly) return false;
  return true;
}

template <typename T>
static long long shape_descs(pr_ctx* c, const std::vector<FineWork>& items,
                             std::vector<FineDesc<T>>& d, int code, bool forced) {
  const int cfg = code % kNumFusedCfgs;
  const long long min_wgs = kChunkMinWgs[code / kNumFusedCfgs];
  const long long slots =
      min_wgs < 0 ? resident_slots(c, cfg, std::is_same<T, float>::value, forced, all_xonly(d))
                  : 0;
  const int xc = fine_chunk(items, cfg, min_wgs, forced, slots);
  long long tiles = 0;
  for (size_t i = 0; i < items.size(); ++i) {
    const int n = items[i].prob->n;
    d[i].tiles_y = (n + fused_ty(cfg) - 1) / fused_ty(cfg);
    d[i].tiles_z = (n + fused_tz(cfg) - 1) / fused_tz(cfg);
    d[i].xc = std::min(xc, n);
    d[i].chunks_x = (n + d[i].xc - 1) / d[i].xc;
    d[i].tile_begin = tiles;
    tiles += (long long)d[i].tiles_y * d[i].tiles_z * d[i].chunks_x;
  }
  return tiles;
}

template <typename T>
static void launch_step(const FineDesc<T>* d, int nd, long long tiles, int step, int cfg,
                        bool forced, bool xonly, hipStream_t s) {
  if (forced) {
    if (std::is_same<T, float>::value)
      launch_forced_step_f32((const FineDesc<float>*)d, nd, tiles, step, cfg, s);
    else
      launch_forced_step_f64((const FineDesc<double>*)d, nd, tiles, step, cfg, s);
    return;
  }
  if (std::is_same<T, float>::value)
    launch_fine_step_f32((const FineDesc<float>*)d, nd, tiles, step, cfg, xonly, s);
  else
    launch_fine_step_f64((const FineDesc<double>*)d, nd, tiles, step, cfg, xonly, s);
}

constexpr int kTuneReps = 3;

// Tuning key: value size, largest grid, batch size class floor(log2(batch)),
// and F for the forced-flow stencil.
static std::string tune_key(int value_bytes, int nmax, int batch, bool forced, bool blocked) {
  int cls = 0;
  while ((1LL << (cls + 1)) <= batch) ++cls;
  char key[64];
  snprintf(key, sizeof key, "%d|%d|%d%s%s", value_bytes, nmax, cls, forced ? "|F" : "",
           blocked ? "|B" : "");
  return key;
}

// Whether the blocked tilings (2 x 2 columns per thread, pair loads and
// stores) apply to a batch: every grid even and every field and snapshot
// column aligned to two values.
template <typename T>
static bool blocked_ok(const std::vector<FineWork>& items, const std::vector<FineDesc<T>>& d) {
  auto al = [](const void* p) { return ((uintptr_t)p % (2 * sizeof(T))) == 0; };
  for (size_t i = 0; i < items.size(); ++i) {
    if (items[i].prob->n % 2 != 0) return false;
    if (!al(d[i].first_src) || !al(d[i].buf[0]) || !al(d[i].buf[1])) return false;
    if (d[i].snaps && (!al(d[i].snaps) || d[i].snap_ld % 2 != 0)) return false;
  }
  return true;
}

// Launch shapes the tuner tries: every tiling (the forced stencil: those of
// kForcedCfgs; in FP64 not a 1024-thread one with two columns per thread,
// whose four waves per SIMD leave too few registers) under every chunk
// policy, the modelled one first.
static std::vector<int> shape_codes(bool forced, int value_bytes, bool blocked) {
  std::vector<int> v;
  for (int pol = kChunkPolicies - 1; pol >= 0; --pol) {
    if (forced) {
      for (int i = 0; i < kNumForcedCfgs; ++i)
        if (!(value_bytes == 8 && kFusedCfgs[kForcedCfgs[i]].nt > 512 &&
              fused_slots(kForcedCfgs[i]) > 1))
          v.push_back(kForcedCfgs[i] + kNumFusedCfgs * pol);
    } else {
      for (int cfg = 0; cfg < kNumFusedCfgs; ++cfg)
        if (blocked || !kFusedCfgs[cfg].blocked) v.push_back(cfg + kNumFusedCfgs * pol);
    }
  }
  return v;
}

// Autotuner: time step 0 of the actual batch in every launch shape (one
// warm-up and kTuneReps timed launches each), then time the kTuneFinal
// fastest again in kTuneRounds interleaved rounds (so a clock change during
// tuning hits every finalist alike), each keeping its fastest launch, and keep
// the fastest finalist for this key.
// Step 0 reads the inputs and writes buffers no other step 0 reads, so
// repeating it is harmless; every configuration gives bitwise the same
// values. Synchronises `s` at the first batch of a key.
constexpr int kTuneFinal = 4;
constexpr int kTuneRounds = 6;
template <typename T>
static int tune_fine(pr_ctx* c, const std::vector<FineWork>& items, std::vector<FineDesc<T>>& d,
                     bool forced, bool blocked, hipStream_t s) {
  int nmax = 0;
  for (auto& w : items) nmax = std::max(nmax, w.prob->n);
  const std::string key = tune_key((int)sizeof(T), nmax, (int)items.size(), forced, blocked);
  auto it = c->tuned.find(key);
  if (it != c->tuned.end()) return it->second;
  hipEvent_t e0 = event_get(c), e1 = event_get(c);
  const std::vector<int> codes = shape_codes(forced, (int)sizeof(T), blocked);
  auto time_code = [&](int code, int reps) {
    const int cfg = code % kNumFusedCfgs;
    const long long tiles = shape_descs<T>(c, items, d, code, forced);
    FineDesc<T>* dd = stage_push(c, d);
    stage_flush(c, s);
    const bool xo = all_xonly(d);
    launch_step<T>(dd, (int)d.size(), tiles, 0, cfg, forced, xo, s);
    PR_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) launch_step<T>(dd, (int)d.size(), tiles, 0, cfg, forced, xo, s);
    PR_HIP(hipEventRecord(e1, s));
    PR_HIP(hipEventSynchronize(e1));
    float ms = 0;
    PR_HIP(hipEventElapsedTime(&ms, e0, e1));
    return ms / reps;
  };
  // a policy giving a launch already timed (same tiling and workgroup count,
  // hence the same chunk length) is not timed again: the earlier code keeps it
  std::set<std::pair<int, long long>> seen;
  std::vector<std::pair<float, int>> timed;   // (ms per launch, code), in code order
  for (const int code : codes) {
    const long long tiles = shape_descs<T>(c, items, d, code, forced);
    if (!seen.insert({code % kNumFusedCfgs, tiles}).second) continue;
    timed.push_back({time_code(code, kTuneReps), code});
  }
  std::stable_sort(timed.begin(), timed.end(),
                   [](const std::pair<float, int>& a, const std::pair<float, int>& b) {
                     return a.first < b.first;
                   });
  const int nf = std::min<int>(kTuneFinal, (int)timed.size());
  std::vector<float> fin(nf, 0.0f);
  for (int r = 0; r < kTuneRounds; ++r)
    for (int i = 0; i < nf; ++i) {
      const float ms = time_code(timed[i].second, 1);
      if (r == 0 || ms < fin[i]) fin[i] = ms;
    }
  int bi = 0;
  for (int i = 1; i < nf; ++i)
    if (fin[i] < fin[bi]) bi = i;
  const int best = timed[bi].second;
  const char* lg = getenv("PR_TUNE_LOG");
  if (lg && *lg && *lg != '0') {
    // diagnostics: every shape's first-pass time, then the finalists'
    std::fprintf(stderr, "tune %s:", key.c_str());
    for (auto& t : timed) std::fprintf(stderr, " %d=%.1f", t.second, 1000.0f * t.first);
    std::fprintf(stderr, " | final:");
    for (int i = 0; i < nf; ++i) std::fprintf(stderr, " %d=%.1f", timed[i].second, 1000.0f * fin[i]);
    std::fprintf(stderr, " -> %d\n", best);
  }
  event_put(c, e0);
  event_put(c, e1);
  c->tuned[key] = best;
  return best;
}

template <typename T>
static void fine_typed(pr_ctx* c, const std::vector<FineWork>& items, bool forced, hipStream_t s,
                       const std::string& tag) {
  const bool f32 = std::is_same<T, float>::value;
  const int nwork = f32 ? 3 : 1;
  size_t total = 0;
  for (auto& w : items) total += (size_t)ngrid(*w.prob) * nwork * sizeof(T);
  char* base = (char*)scratch(c, tag + (forced ? "_fw" : "_w"), total);
  std::vector<FineDesc<T>> descs;
  int max_steps = 0;
  size_t off = 0;
  for (auto& w : items) {
    const long long ng = ngrid(*w.prob);
    FineDesc<T> d{};
    d.g = geom_of(c, *w.prob);
    T* work = (T*)(base + off);
    off += (size_t)ng * nwork * sizeof(T);
    if (f32) {
      d.buf[0] = work;
      d.buf[1] = work + ng;
      T* first = work + 2 * ng;
      launch_convert_f64_to_f32(w.u_in, (float*)first, ng, s);
      d.first_src = first;
    } else {
      d.buf[0] = (T*)w.u_out;
      d.buf[1] = work;
      d.first_src = (const T*)w.u_in;
      if (w.n_steps == 0) {
        if (w.u_in != w.u_out)
          PR_HIP(hipMemcpyAsync(w.u_out, w.u_in, ng * 8, hipMemcpyDeviceToDevice, s));
      } else if (w.u_in == w.u_out && (w.n_steps - 1) % 2 == 0) {
        // the first step writes buf[0] = u_out: read the input from a copy
        PR_HIP(hipMemcpyAsync(work, w.u_in, ng * 8, hipMemcpyDeviceToDevice, s));
        d.first_src = work;
      }
    }
    d.snaps = (T*)w.snaps;
    d.snap_every = w.snap_every;
    if (w.snaps)
      PR_HIP(hipMemcpyAsync(w.snaps, d.first_src, ng * sizeof(T), hipMemcpyDeviceToDevice, s));
    d.n_steps = w.n_steps;
    d.dt = w.dt;
    d.t0 = w.t0;
    d.with_forcing = w.unforced ? 0 : 1;
    d.snap_ld = w.snap_ld > 0 ? w.snap_ld : ng;
    max_steps = std::max(max_steps, w.n_steps);
    descs.push_back(d);
  }
  if (max_steps > 0) {
    const bool blocked = !forced && blocked_ok<T>(items, descs);
    int code = forced ? forced_cfg_forced() : forced_cfg();
    if (code >= 0 && kFusedCfgs[code % kNumFusedCfgs].blocked && !blocked) code = -1;
    if (code < 0) code = tune_fine<T>(c, items, descs, forced, blocked, s);
    const int cfg = code % kNumFusedCfgs;
    const long long tiles = shape_descs<T>(c, items, descs, code, forced);
    FineDesc<T>* dd = stage_push(c, descs);
    stage_flush(c, s);
    const bool xo = all_xonly(descs);
    {
      int nmax = 0;
      for (auto& w : items) nmax = std::max(nmax, w.prob->n);
      c->fine_planes[tune_key((int)sizeof(T), nmax, (int)items.size(), forced, blocked)] =
          descs[0].xc;
    }
    if (forced) {
      for (int step = 0; step < max_steps; ++step)
        launch_step<T>(dd, (int)descs.size(), tiles, step, cfg, true, false, s);
    } else if (f32) {
      launch_fine_f32((const FineDesc<float>*)dd, (int)descs.size(), tiles, max_steps, cfg, xo, s);
    } else {
      launch_fine_f64((const FineDesc<double>*)dd, (int)descs.size(), tiles, max_steps, cfg, xo,
                      s);
    }
  }
  if (f32)
    for (size_t i = 0; i < items.size(); ++i)
      launch_convert_f32_to_f64(items[i].n_steps > 0 ? (const float*)descs[i].buf[0]
                                                     : (const float*)descs[i].first_src,
                                items[i].u_out, ngrid(*items[i].prob), s);
}

void enqueue_fine(pr_ctx* c, const std::vector<FineWork>& items, hipStream_t s,
                  const std::string& tag) {
  if (items.empty()) return;
  const int prec = items[0].prob->precision;
  for (auto& w : items) {
    check_problem(w.prob);
    PR_CHECK(w.prob->precision == prec, "all items of a batch must share the precision");
    PR_CHECK(w.n_steps >= 0, "n_steps must be >= 0");
    PR_CHECK(std::isfinite(w.dt) && w.dt > 0, "dt must be positive");
    PR_CHECK(w.u_in && w.u_out, "null state pointer");
    PR_CHECK(w.snap_every >= 0, "snap_every must be >= 0");
    PR_CHECK((w.snap_every == 0) == (w.snaps == nullptr), "snaps must be given iff snap_every > 0");
    if (w.dt * spectral_bound(*w.prob) > kStabRK4)
      fail(PR_EUNSTABLE, "dt exceeds the RK4 stability bound 2.6 / rho(L)");
  }
  std::vector<FineWork> steady, forced;
  for (auto& w : items) (forced_flow(*w.prob) ? forced : steady).push_back(w);
  for (int g = 0; g < 2; ++g) {
    const std::vector<FineWork>& v = g ? forced : steady;
    if (v.empty()) continue;
    if (prec == PR_MIXED) fine_typed<float>(c, v, g == 1, s, tag);
    else fine_typed<double>(c, v, g == 1, s, tag);
  }
}

// ---------------------------------------------------------------------------
// Gram products
StagedGram stage_gram(pr_ctx* c, const std::vector<GramWork>& items, int na, int nb, bool f32,
                      const std::string& tag) {
  StagedGram g;
  if (items.empty()) return g;
  const int P = (nb == 0) ? na * (na + 1) / 2 : na * nb;
  const size_t ncol = (size_t)(na + nb) * 16;
  std::vector<GemmDesc> descs;
  std::vector<long long> part_off;
  long long wg = 0;
  size_t part_total = 0;
  for (auto& it : items) {
    PR_CHECK(it.cols.size() == ncol, "Gram column list size mismatch");
    // the FP32-MFMA kernel reads every column as float
    if (f32)
      for (const ColDesc& cd : it.cols)
        PR_CHECK(cd.ptr == nullptr || cd.f32, "FP32 Gram over a column that is not FP32");
    GemmDesc d{};
    d.nrows = it.nrows;
    d.chunk_rows = it.chunk_rows > 0 ? it.chunk_rows : gram_chunk_rows(it.nrows);
    PR_CHECK(d.chunk_rows % 64 == 0, "Gram chunks must hold whole 64-row steps");
    d.nchunks = (int)((it.nrows + d.chunk_rows - 1) / d.chunk_rows);
    d.wg_begin = wg;
    wg += d.nchunks;
    d.out = it.out;
    d.ld = it.ld;
    d.scale = it.scale;
    if (it.a_in_b) {
      PR_CHECK(nb >= na, "A inside B needs at least as many B tiles");
      bool tail = false;
      for (int i = 0; i < na * 16; ++i) {
        const ColDesc& a = it.cols[i];
        const ColDesc& b = it.cols[(size_t)na * 16 + i];
        if (a.ptr == nullptr) {
          tail = true;
          continue;
        }
        PR_CHECK(!tail && a.ptr == b.ptr && a.mptr == b.mptr && a.idx == b.idx && a.f32 == b.f32,
                 "A columns must be a prefix of the B columns");
      }
      d.a_in_b = 1;
    }
    part_off.push_back((long long)part_total);
    part_total += (size_t)d.nchunks * P * 256;
    descs.push_back(d);
  }
  double* part = (double*)scratch(c, tag + "_part", part_total * 8);
  for (size_t i = 0; i < items.size(); ++i) {
    descs[i].partial = part + part_off[i];
    descs[i].cols = stage_push(c, items[i].cols);
  }
  g.dd = stage_push(c, descs);
  g.nd = (int)descs.size();
  g.wg = wg;
  g.na = na;
  g.nb = nb;
  g.f32 = f32;
  return g;
}

void launch_gram_staged(const StagedGram& g, hipStream_t s) {
  if (g.nd <= 0) return;
  launch_gemm_tn(g.dd, g.nd, g.wg, g.na, g.nb, g.f32, s);
  launch_gemm_reduce(g.dd, g.nd, g.na, g.nb, s);
}

void enqueue_gram(pr_ctx* c, const std::vector<GramWork>& items, int na, int nb, bool f32,
                  hipStream_t s, const std::string& tag) {
  const StagedGram g = stage_gram(c, items, na, nb, f32, tag);
  stage_flush(c, s);
  launch_gram_staged(g, s);
}

// ---------------------------------------------------------------------------
// L applied to columns
// Descriptors of one L launch of element type T: tiles of tq points of the
// (y, z) plane (tq_of(n) tiles per plane) by cx planes.
template <typename T, typename TQ>
static long long applyL_descs(pr_ctx* c, const std::vector<ApplyLWork>& items, int cx, TQ tq_of,
                              std::vector<ApplyLDesc<T>>& d) {
  long long tiles = 0;
  for (auto& w : items) {
    ApplyLDesc<T> a{};
    a.g = geom_piece(geom_of(c, *w.prob), w.piece);
    a.in = (const T*)w.in;
    a.out = (T*)w.out;
    a.ld = w.ld > 0 ? w.ld : ngrid(*w.prob);
    a.ncols = w.ncols;
    a.mptr = w.mptr;
    a.skip_tail = w.skip_tail;
    a.tiles_q = tq_of(w.prob->n);
    a.chunk_x = cx;
    a.tiles_x = (w.prob->n + cx - 1) / cx;
    a.tile_begin = tiles;
    tiles += (long long)a.tiles_q * a.tiles_x * w.ncols;
    d.push_back(a);
  }
  return tiles;
}

StagedApplyL stage_applyL_batch(pr_ctx* c, const std::vector<ApplyLWork>& items) {
  StagedApplyL st;
  if (items.empty()) return st;
  const bool f32 = items[0].prob->precision == PR_MIXED;
  st.f32 = f32;
  // The LDS-window kernel (kWinQ points per workgroup) for launches whose
  // grids all allow it and that give 2048 workgroups at an x chunk of 4 to 32
  // planes (the bases of a wave); otherwise kTileQ points per workgroup with
  // x chunks of kChunkX planes, or of 4 when that leaves a launch (one column
  // of L d in the sweep) under 2048 workgroups.
  auto win_tq = [](int n) { return (n * n + kWinQ - 1) / kWinQ; };
  bool win = true;
  long long wide = 0;
  for (auto& w : items) {
    const int n = w.prob->n;
    win = win && n >= kWinMinN && n <= kWinMaxN;
    wide += (long long)tiles_q(n) * tiles_x(n) * w.ncols;
  }
  // PR_APPLYL_WIN=0 never takes the window kernel, =1 whenever the grids
  // allow it (tests compare the two)
  const char* ew = getenv("PR_APPLYL_WIN");
  // the window kernel's x chunk: the longest of 32, 16, 8, 4 planes that
  // gives 2048 workgroups (each chunk also loads two planes ahead)
  auto win_wgs = [&](int x) {
    long long t = 0;
    for (auto& w : items) t += (long long)win_tq(w.prob->n) * ((w.prob->n + x - 1) / x) * w.ncols;
    return t;
  };
  int cxw = kChunkX;
  while (cxw > 4 && win_wgs(cxw) < 2048) cxw /= 2;
  if (ew && *ew == '0') win = false;
  else if (!(ew && *ew == '1')) win = win && win_wgs(cxw) >= 2048;
  const int cx = win ? cxw : (wide >= 2048 ? kChunkX : 4);
  auto tq = [&](int n) { return win ? win_tq(n) : tiles_q(n); };
  if (f32) {
    std::vector<ApplyLDesc<float>> d;
    st.tiles = applyL_descs<float>(c, items, cx, tq, d);
    st.dd = stage_push(c, d);
    st.nd = (int)d.size();
  } else {
    std::vector<ApplyLDesc<double>> d;
    st.tiles = applyL_descs<double>(c, items, cx, tq, d);
    st.dd = stage_push(c, d);
    st.nd = (int)d.size();
  }
  st.win = win;
  return st;
}

void launch_applyL_staged(const StagedApplyL& st, hipStream_t s) {
  if (st.nd <= 0) return;
  if (st.f32) launch_applyL_f32((const ApplyLDesc<float>*)st.dd, st.nd, st.tiles, st.win, s);
  else launch_applyL_f64((const ApplyLDesc<double>*)st.dd, st.nd, st.tiles, st.win, s);
}

void enqueue_applyL_batch(pr_ctx* c, const std::vector<ApplyLWork>& items, hipStream_t s) {
  const StagedApplyL st = stage_applyL_batch(c, items);
  stage_flush(c, s);
  launch_applyL_staged(st, s);
}

void enqueue_applyL(pr_ctx* c, const pr_grid_problem& p, const void* in, void* out, int ncols,
                    const int* mptr, hipStream_t s) {
  enqueue_applyL_batch(c, {ApplyLWork{&p, in, out, ncols, mptr}}, s);
}

// L_j applied to ncols columns (ld elements apart; 0: N_g) for every piece j
// of the problem's flow: piece j's columns at out + j * ncols columns (one
// piece, L itself, for a steady flow).
static std::vector<ApplyLWork> applyL_piece_work(const pr_grid_problem& p, const void* in,
                                                 void* out, int ncols, const int* mptr,
                                                 long long ld) {
  if (ld <= 0) ld = ngrid(p);
  const size_t col = (size_t)ld * (p.precision == PR_MIXED ? 4 : 8);
  std::vector<ApplyLWork> v;
  for (int j = 0; j < flow_pieces(p); ++j)
    v.push_back(ApplyLWork{&p, in, (char*)out + (size_t)j * ncols * col, ncols, mptr, j, ld});
  return v;
}

void enqueue_applyL_pieces(pr_ctx* c, const pr_grid_problem& p, const void* in, void* out,
                           int ncols, const int* mptr, hipStream_t s, long long ld) {
  enqueue_applyL_batch(c, applyL_piece_work(p, in, out, ncols, mptr, ld), s);
}

// The forcing fields f_j of a forced flow's pieces (field precision), one
// column each, ld elements apart (0: N_g).
void enqueue_forcing_fields(pr_ctx* c, const pr_grid_problem& p, void* out, hipStream_t s,
                            long long ld) {
  if (ld <= 0) ld = ngrid(p);
  const Geom g = geom_of(c, p);
  const bool f32 = p.precision == PR_MIXED;
  const size_t col = (size_t)ld * (f32 ? 4 : 8);
  for (int j = 0; j < g.npieces; ++j)
    launch_forcing_field(g, j, (char*)out + (size_t)j * col, f32 ? 1 : 0, s);
}

// ---------------------------------------------------------------------------
// POD_Mode
// Column idx of a block whose columns are ld elements apart.
static ColDesc col_of(const void* base, int idx, long long ld, bool f32, const int* mptr) {
  ColDesc d;
  d.ptr = (const char*)base + (size_t)idx * ld * (f32 ? 4 : 8);
  d.mptr = mptr;
  d.idx = idx;
  d.f32 = f32 ? 1 : 0;
  return d;
}
static ColDesc col_null() { return ColDesc{nullptr, nullptr, 0, 0}; }

static long long tsmm_wgs(long long nrows) { return (nrows + 511) / 512; }

// Whitened (stage-2) POD items take their CholQR factor from the coefficient
// Gram C^T G C instead of a Gram pass over the formed modes
// (PR_SMALL_CHOLQR, default 1; 0 = a pass over the modes).
static bool small_cholqr() {
  const char* e = getenv("PR_SMALL_CHOLQR");
  return !(e && *e == '0');
}

void enqueue_pod(pr_ctx* c, const std::vector<PodWork>& items, hipStream_t s,
                 const std::string& tag) {
  if (items.empty()) return;
  const int prec = items[0].prob->precision;
  const bool f32 = prec == PR_MIXED;
  int maxcols = 0;
  for (auto& w : items) {
    check_problem(w.prob);
    PR_CHECK(w.prob->precision == prec, "all items of a batch must share the precision");
    PR_CHECK(!w.cols.empty() && (int)w.cols.size() <= kMaxPodCols, "POD input needs 1..64 columns");
    PR_CHECK(w.cap >= 1 && w.cap <= kMaxCap, "cap must be in [1, 31]");
    PR_CHECK(w.gamma > 0 && w.gamma <= 1, "gamma must be in (0, 1]");
    PR_CHECK(w.R_out && w.m_out, "null POD output");
    maxcols = std::max(maxcols, (int)w.cols.size());
  }
  const int na = (maxcols + 15) / 16;
  const int ldg = na * 16;
  const int nitems = (int)items.size();
  double* G = (double*)scratch(c, tag + "_G", (size_t)nitems * ldg * ldg * 8);
  double* lam = (double*)scratch(c, tag + "_lam", (size_t)nitems * 64 * 8);
  double* coef = (double*)scratch(c, tag + "_coef", (size_t)nitems * 64 * 32 * 8);
  double* G2 = (double*)scratch(c, tag + "_G2", (size_t)nitems * 32 * 32 * 8);
  double* coef2 = (double*)scratch(c, tag + "_coef2", (size_t)nitems * 32 * 32 * 8);

  // 1. Gram of the snapshots (FP32 MFMA for float data)
  std::vector<GramWork> gw;
  for (int i = 0; i < nitems; ++i) {
    GramWork g;
    g.nrows = ngrid(*items[i].prob);
    g.cols = items[i].cols;
    g.cols.resize((size_t)na * 16, col_null());
    g.out = G + (size_t)i * ldg * ldg;
    g.ld = ldg;
    const double h = spacing(*items[i].prob);
    g.scale = h * h * h;
    gw.push_back(g);
  }
  enqueue_gram(c, gw, na, 0, f32, s, tag + "_g1");

  // 1b. inputs made of blocks whose own M-orthonormalisation was deferred:
  // whiten the Gram by the blocks' Cholesky factors
  const int wbs = items[0].whiten_bs;
  const int cq = items[0].cholqr;
  for (auto& w : items)
    PR_CHECK(w.whiten_bs == wbs && w.cholqr == cq, "POD batch items must share their options");
  WhitenDesc* wdd = nullptr;
  if (wbs > 0) {
    PR_CHECK(wbs <= 32, "whitening blocks of at most 32 columns");
    double* wT = (double*)scratch(c, tag + "_wT", (size_t)nitems * kWhitenMaxCols * 32 * 8);
    int* wm = (int*)scratch(c, tag + "_wm", (size_t)nitems * kWhitenMaxCols * 4);
    std::vector<WhitenDesc> wd;
    for (int i = 0; i < nitems; ++i) {
      const int nc = (int)items[i].cols.size();
      PR_CHECK(nc % wbs == 0 && nc <= kWhitenMaxCols, "whitening needs whole blocks");
      WhitenDesc x{};
      x.G = G + (size_t)i * ldg * ldg;
      x.ldg = ldg;
      x.nb = nc / wbs;
      x.bs = wbs;
      for (int b = 0; b < x.nb; ++b) x.m[b] = items[i].cols[(size_t)b * wbs].mptr;
      x.T = wT + (size_t)i * kWhitenMaxCols * 32;
      x.meff = wm + (size_t)i * kWhitenMaxCols;
      x.coef = coef + (size_t)i * 64 * 32;
      x.ld_coef = items[i].cap;
      x.ncoef = items[i].cap;
      wd.push_back(x);
    }
    wdd = stage_push(c, wd);
    stage_flush(c, s);
    launch_block_whiten(wdd, nitems, s);
  }

  // 2-3. eigen-decomposition, rank and mode coefficients
  std::vector<EigDesc> ed;
  for (int i = 0; i < nitems; ++i) {
    EigDesc e{};
    e.G = G + (size_t)i * ldg * ldg;
    e.ldg = ldg;
    e.nc = (int)items[i].cols.size();
    e.gamma = items[i].gamma;
    e.cap = items[i].cap;
    e.force_m = items[i].force_m;
    e.tau_r = f32 ? kTauRankF32 : kTauRankF64;
    e.lambda = items[i].lambda_out ? items[i].lambda_out : lam + (size_t)i * 64;
    e.coef = coef + (size_t)i * 64 * 32;
    e.ld_coef = items[i].cap;
    e.m_out = items[i].m_out;
    ed.push_back(e);
  }
  EigDesc* edd = stage_push(c, ed);
  stage_flush(c, s);
  launch_eig_select(edd, nitems, s);
  // whitened items: the CholQR factor from C^T G C (the modes' Gram in exact
  // arithmetic) applied to the coefficients, so the modes are formed once.
  // That factor cannot remove the rounding of G itself (about eps lambda_1
  // absolute), so the modes keep an M-orthogonality error of about
  // eps lambda_1 / lambda_m: at most about 1e-3 in FP64 with tau_r = 1e-13
  // (harmless: the Galerkin system keeps M_r explicitly and the span is
  // unchanged), but up to 1e-1 for the FP32 Gram of PR_MIXED, which
  // therefore takes the Gram pass over the formed modes.
  const bool small_cq = wdd && cq && small_cholqr() && !f32;
  if (small_cq) {
    std::vector<CoefGramDesc> gd;
    std::vector<CholDesc> cd;
    for (int i = 0; i < nitems; ++i) {
      CoefGramDesc x{};
      x.G = G + (size_t)i * ldg * ldg;
      x.ldg = ldg;
      x.nc = (int)items[i].cols.size();
      x.C = ed[i].coef;
      x.ldc = items[i].cap;
      x.cap = items[i].cap;
      x.G2 = G2 + (size_t)i * 32 * 32;
      x.U = coef2 + (size_t)i * 32 * 32;
      PR_CHECK(x.nc <= 64 && x.cap <= 32, "coefficient Gram of at most 64 x 32");
      gd.push_back(x);
      cd.push_back(CholDesc{x.G2, 32, items[i].cap, items[i].m_out, coef2 + (size_t)i * 32 * 32});
    }
    CoefGramDesc* gdd = stage_push(c, gd);
    CholDesc* cdd = stage_push(c, cd);
    stage_flush(c, s);
    launch_coef_gram(gdd, nitems, s);
    launch_cholqr_coef(cdd, nitems, s);
    launch_coef_apply(gdd, nitems, s);
  }
  if (wdd) launch_block_unwhiten(wdd, nitems, s);   // coefficients of the raw blocks

  // 4. modes R = W Y_m Lambda_m^{-1/2}
  std::vector<TsmmDesc> td;
  long long wg = 0;
  for (int i = 0; i < nitems; ++i) {
    TsmmDesc t{};
    t.nrows = ngrid(*items[i].prob);
    t.in = stage_push(c, items[i].cols);
    t.nin = (int)items[i].cols.size();
    t.C = ed[i].coef;
    t.ldc = items[i].cap;
    t.out = items[i].R_out;
    t.out_ld = items[i].R_ld > 0 ? items[i].R_ld : t.nrows;
    t.out_f32 = f32;
    t.nout = items[i].cap;
    t.out_mptr = items[i].m_out;
    t.add = nullptr;
    t.alpha = 1.0;
    t.wg_begin = wg;
    t.skip_tail = items[i].skip_tail;
    wg += tsmm_wgs(t.nrows);
    td.push_back(t);
  }
  TsmmDesc* tdd = stage_push(c, td);
  stage_flush(c, s);
  // accumulator class: every column written, or, when the columns beyond
  // the rank are left alone, the rank bound min(cap, input columns)
  int max_cap = 1;
  for (auto& it : items)
    max_cap = std::max(max_cap, it.skip_tail ? std::min(it.cap, (int)it.cols.size()) : it.cap);
  launch_tsmm(tdd, nitems, wg, max_cap, s);

  // 5. CholQR in the M inner product (FP64 MFMA Gram, FP64 Cholesky). The
  // modes enter with kappa(R) ~ 1 + eps lambda_1 / lambda_m <= 1 + 1e-3, so
  // one pass already leaves eps kappa^2 ~ eps loss of orthogonality.
  for (int pass = 0; pass < (cq && !small_cq ? kCholQRPasses : 0); ++pass) {
    std::vector<GramWork> g2;
    std::vector<std::vector<ColDesc>> rcols(nitems);
    for (int i = 0; i < nitems; ++i) {
      const long long ng = ngrid(*items[i].prob);
      const long long rld = items[i].R_ld > 0 ? items[i].R_ld : ng;
      for (int j = 0; j < 32; ++j)
        rcols[i].push_back(j < items[i].cap ? col_of(items[i].R_out, j, rld, f32, items[i].m_out)
                                            : col_null());
      GramWork g;
      g.nrows = ng;
      g.cols = rcols[i];
      g.out = G2 + (size_t)i * 32 * 32;
      g.ld = 32;
      const double h = spacing(*items[i].prob);
      g.scale = h * h * h;
      g2.push_back(g);
    }
    enqueue_gram(c, g2, 2, 0, false, s, tag + "_g2");
    std::vector<CholDesc> cd;
    for (int i = 0; i < nitems; ++i)
      cd.push_back(CholDesc{G2 + (size_t)i * 32 * 32, 32, items[i].cap, items[i].m_out,
                            coef2 + (size_t)i * 32 * 32});
    CholDesc* cdd = stage_push(c, cd);
    stage_flush(c, s);
    launch_cholqr_coef(cdd, nitems, s);
    std::vector<TsmmDesc> t2;
    wg = 0;
    for (int i = 0; i < nitems; ++i) {
      TsmmDesc t{};
      t.nrows = ngrid(*items[i].prob);
      std::vector<ColDesc> in(rcols[i].begin(), rcols[i].begin() + items[i].cap);
      t.in = stage_push(c, in);
      t.nin = items[i].cap;
      t.C = coef2 + (size_t)i * 32 * 32;
      t.ldc = items[i].cap;
      t.out = items[i].R_out;
      t.out_ld = items[i].R_ld > 0 ? items[i].R_ld : t.nrows;
      t.out_f32 = f32;
      t.nout = items[i].cap;
      t.out_mptr = items[i].m_out;
      t.alpha = 1.0;
      t.wg_begin = wg;
      t.skip_tail = items[i].skip_tail;
      wg += tsmm_wgs(t.nrows);
      t2.push_back(t);
    }
    TsmmDesc* t2d = stage_push(c, t2);
    stage_flush(c, s);
    launch_tsmm(t2d, nitems, wg, max_cap, s);
  }
}

// ---------------------------------------------------------------------------
// correction / lift
StagedCorrect stage_correct(pr_ctx* c, long long nrows, const ColDesc* psi_dev, int npsi,
                            const double* coef, const void* fine, int fine_f32, double* out,
                            const double* prev, const double* ref, double* norms4, double h3,
                            const std::string& tag) {
  // about one row per thread (at most 4096 workgroups): the correction reads
  // its columns one after another, so a small grid needs many workgroups in
  // flight to hide the load latency
  const int nwg = (int)std::min<long long>(4096, std::max<long long>(1, (nrows + 255) / 256));
  double* part = (double*)scratch(c, tag + "_cpart", (size_t)nwg * 4 * 8);
  CorrectDesc d{};
  d.nrows = nrows;
  d.psi = npsi > 0 ? psi_dev : nullptr;
  d.npsi = npsi;
  d.coef = coef;
  d.fine = fine;
  d.fine_f32 = fine_f32;
  d.out = out;
  d.prev = prev;
  d.ref = ref;
  d.partial = part;
  d.wg_begin = 0;
  d.nwg = nwg;
  StagedCorrect k;
  k.dd = stage_push1(c, d);
  NormReduceDesc nr{part, nwg, h3, norms4};
  k.nrd = stage_push1(c, nr);
  k.nwg = nwg;
  return k;
}

void launch_correct_staged(const StagedCorrect& k, hipStream_t s) {
  if (!k.dd) return;
  launch_correct(k.dd, 1, k.nwg, s);
  launch_norm_reduce(k.nrd, 1, s);
}

void enqueue_correct(pr_ctx* c, long long nrows, const std::vector<ColDesc>& psi,
                     const double* coef, const void* fine, int fine_f32, double* out,
                     const double* prev, const double* ref, double* norms4, double h3,
                     hipStream_t s, const std::string& tag) {
  const ColDesc* pd = psi.empty() ? nullptr : stage_push(c, psi);
  const StagedCorrect k = stage_correct(c, nrows, pd, (int)psi.size(), coef, fine, fine_f32, out,
                                        prev, ref, norms4, h3, tag);
  stage_flush(c, s);
  launch_correct_staged(k, s);
}

// ---------------------------------------------------------------------------
// coarse step
void enqueue_coarse(pr_ctx* c, const CoarseWork& w, hipStream_t s, PhaseEvents* ph) {
  const pr_grid_problem& p = *w.prob;
  const bool f32 = p.precision == PR_MIXED;
  const long long ng = ngrid(p);
  const size_t sf = f32 ? 4 : 8;
  const double h = spacing(p), h3 = h * h * h;
  const int cap = w.cap;
  PR_CHECK(cap >= 1 && cap <= kMaxCap, "cap must be in [1, 31]");
  PR_CHECK(w.n_in == 1 || w.n_in == 2, "n_in must be 1 or 2");

  const int np = flow_pieces(p);
  const bool forced = forced_flow(p);
  char* sm = (char*)scratch(c, "co_small", 64 * 1024);
  double* S1 = (double*)(sm);              // CGS2 pass 1: R^T M u (cap), |u|^2 at [32]
  double* S2 = (double*)(sm + 4096);       // pass 2: R^T M d~ (cap), |d~|^2 at [32]
  double* S3 = (double*)(sm + 8192);       // pass 3: |d~|^2 after the second projection
  int* flag = (int*)(sm + 12288);
  double* dscale = (double*)(sm + 12288 + 128);
  double* coef = (double*)(sm + 16384);    // cap + 1
  double* betas = (double*)(sm + 16384 + 512);  // 2 x (cap + 1)
  double* nrm = (double*)(sm + 16384 + 1024);   // scratch norms
  double* Sbig = (double*)(sm + 20480);    // Galerkin products: 32 rows x 16 nb (nb <= 9)

  PhaseEvents dummy;
  PhaseEvents& P = ph ? *ph : dummy;

  const void* LR = w.LR;
  const long long cld = w.ld > 0 ? w.ld : ng;   // column stride of R, LR, forcing
  char* ld = (char*)scratch(c, "co_fields", (size_t)ng * sf * (1 + np) + (size_t)ng * 8);
  void* dcol = ld;                          // augmented column d (field precision)
  void* Ld = ld + (size_t)ng * sf;          // L_j d, j < np
  double* dtil = (double*)(ld + (size_t)ng * sf * (1 + np));
  if (!LR) {
    P.begin(2);
    void* lr = scratch(c, "co_LR", (size_t)cld * sf * cap * np);
    enqueue_applyL_pieces(c, p, w.R, lr, cap, w.m, s, cld);
    LR = lr;
  }
  const void* forcing = w.forcing;
  if (forced && !forcing) {
    void* fb = scratch(c, "co_force", (size_t)cld * sf * np);
    enqueue_forcing_fields(c, p, fb, s, cld);
    forcing = fb;
  }

  auto Rcol = [&](int j) { return col_of(w.R, j, cld, f32, w.m); };
  // piece jp of L applied to column j
  auto LRcol = [&](int jp, int j) {
    return col_of((const char*)LR + (size_t)jp * cap * cld * sf, j, cld, f32, w.m);
  };
  auto f64col = [&](const double* x) { return ColDesc{x, nullptr, 0, 0}; };
  const int* aug = w.u_aug ? flag : nullptr;

  // Every descriptor of the launches after the Gram-Schmidt passes is staged
  // first and uploaded by one flush, so the step's launches are not
  // interleaved with descriptor uploads.
  StagedApplyL st_Ld;
  if (w.u_aug) st_Ld = stage_applyL_batch(c, applyL_piece_work(p, dcol, Ld, 1, flag, 0));
  // Galerkin products of Psi = [R, d] against [Psi, L_j Psi per piece,
  // u_in, f_j per piece], the B columns packed (cap + 1 per block) so the
  // launch shape follows the columns that can be valid
  GramWork gb;
  gb.nrows = ng;
  const int npsi = cap + 1;
  std::vector<ColDesc> psi;
  for (int j = 0; j < npsi; ++j)
    psi.push_back(j < cap ? Rcol(j)
                          : (aug ? ColDesc{dcol, aug, 0, f32 ? 1 : 0} : col_null()));
  const int na = (npsi + 15) / 16;
  gb.cols = psi;                                   // A tiles
  gb.cols.resize((size_t)na * 16, col_null());
  std::vector<ColDesc> bc(psi);                    // B: Psi
  for (int jp = 0; jp < np; ++jp)                  // B: L_j Psi per piece
    for (int j = 0; j < npsi; ++j)
      bc.push_back(j < cap ? LRcol(jp, j)
                           : (aug ? ColDesc{(const char*)Ld + (size_t)jp * ng * sf, aug, 0,
                                            f32 ? 1 : 0}
                                  : col_null()));
  const int off_U = (int)bc.size();
  for (int i = 0; i < w.n_in; ++i) bc.push_back(f64col(w.u_in[i]));   // B: states
  const int off_F = (int)bc.size();
  for (int jp = 0; forced && jp < np; ++jp)                            // B: forcing
    bc.push_back(col_of(forcing, jp, cld, f32, nullptr));
  const int nb = ((int)bc.size() + 15) / 16;
  bc.resize((size_t)nb * 16, col_null());
  gb.cols.insert(gb.cols.end(), bc.begin(), bc.end());
  gb.out = Sbig;
  gb.ld = 16 * nb;
  gb.scale = h3;
  gb.a_in_b = 1;                                   // A = B's leading Psi block
  gb.chunk_rows = galerkin_chunk_rows(ng);
  PR_CHECK(32 * gb.ld * 8 <= 57344 - 20480, "Galerkin block exceeds its scratch");
  const StagedGram st_g = stage_gram(c, {gb}, na, nb, false, "co_g");

  double* beta = w.beta_out ? w.beta_out : betas;
  const std::vector<ColDesc> psi_cols(psi.begin(), psi.begin() + cap + 1);
  const ColDesc* psi_dev = stage_push(c, psi_cols);
  // coarse-gap diagnostics: F(U_old) - G(U_old) and U_ref - G(U_new) with
  // their norms (Sec. 4, dT = delta t runs)
  const bool gaps = w.diag_norms && w.n_in == 2 && w.fine;
  double* nbeta = (double*)(sm + 57344);   // 2 x (cap + 1)
  StagedCorrect st_gap_f, st_gap_r, st_corr;
  std::vector<StagedCorrect> st_lift;
  if (gaps) {
    double* dout = (double*)scratch(c, "co_diag", (size_t)ng * 8);
    st_gap_f = stage_correct(c, ng, psi_dev, npsi, nbeta + (cap + 1), w.fine, 0, dout, nullptr,
                             w.fine, w.diag_norms, h3, "co");
    if (w.diag_ref)
      st_gap_r = stage_correct(c, ng, psi_dev, npsi, nbeta, w.diag_ref, 0, dout, nullptr,
                               w.diag_ref, w.diag_norms + 4, h3, "co");
  }
  if (w.corr_out)
    st_corr = stage_correct(c, ng, psi_dev, npsi, coef, w.fine, 0, w.corr_out, w.prev, w.ref,
                            w.norms4 ? w.norms4 : nrm, h3, "co");
  for (int i = 0; i < w.n_in; ++i)
    if (w.lift[i])
      st_lift.push_back(stage_correct(c, ng, psi_dev, npsi, beta + (size_t)i * (cap + 1), nullptr,
                                      0, w.lift[i], nullptr, nullptr, nrm, h3, "co"));
  stage_flush(c, s);

  if (w.u_aug) {
    P.begin(3);
    // CGS2 of eqaug, one fused pass each: (1) c1 = R^T M u and |u|_M^2;
    // (2) d~ = u - R c1 with c2 = R^T M d~; (3) d~ -= R c2 with |d~|_M^2
    CgsArgs ga{};
    for (int j = 0; j < cap; ++j) ga.col[j] = (const char*)w.R + (size_t)j * cld * sf;
    ga.f32 = f32 ? 1 : 0;
    ga.mptr = w.m;
    ga.n = cap;
    ga.nrows = ng;
    ga.chunk_rows = cgs_chunk_rows(ng);
    ga.nchunks = (int)((ng + ga.chunk_rows - 1) / ga.chunk_rows);
    ga.partial = (double*)scratch(c, "co_cgs_part", (size_t)ga.nchunks * (kCgsMaxCols + 1) * 8);
    ga.scale = h3;
    CgsArgs a1 = ga;
    a1.y = w.u_aug;
    a1.dots = S1;
    a1.norm = S1 + 32;
    launch_cgs(a1, s);
    CgsArgs a2 = ga;
    a2.y = w.u_aug;
    a2.c = S1;
    a2.z = dtil;
    a2.dots = S2;
    a2.norm = S2 + 32;
    launch_cgs(a2, s);
    CgsArgs a3 = ga;
    a3.y = dtil;
    a3.c = S2;
    a3.z = dtil;
    a3.norm = S3;
    a3.nu2 = S1 + 32;     // with the decision on d~ (eqaug's degenerate case)
    a3.flag = flag;
    a3.dscale = dscale;
    launch_cgs(a3, s);
    launch_scale_into(dtil, dcol, f32, ng, dscale, s);
    P.begin(2);
    launch_applyL_staged(st_Ld, s);
  }
  P.begin(2);
  launch_gram_staged(st_g, s);

  P.begin(4);
  ReducedDesc rd{};
  rd.S = Sbig;
  rd.ld = 16 * nb;
  rd.ld_piece = npsi;
  rd.cap = cap;
  rd.m = w.m;
  rd.aug = aug;
  rd.off_M = 0;
  rd.off_L = npsi;
  rd.off_U = off_U;
  rd.n_in = w.n_in;
  rd.dT = w.dT;
  rd.n_c = w.n_c;
  rd.forced = forced ? geom_of(c, p).forced : 0;
  rd.npieces = np;
  rd.off_F = off_F;
  rd.w = forced ? p.fp[2] : 0.0;
  rd.t0 = w.t0;
  rd.beta = beta;
  rd.coef = coef;
  rd.n_c_out = w.n_c_out;
  launch_reduced_one(rd, s);
  if (w.diag_norms)   // the basis block of the Galerkin Gram: R^T M R
    launch_orth_defect(Sbig, 16 * nb, w.m, cap, w.diag_norms + 8, s);
  if (gaps) {
    launch_negate(beta, nbeta, 2 * (cap + 1), s);
    launch_correct_staged(st_gap_f, s);
    launch_correct_staged(st_gap_r, s);
  }
  launch_correct_staged(st_corr, s);
  for (const StagedCorrect& k : st_lift) launch_correct_staged(k, s);
  P.end();
}

}  // namespace pr

using namespace pr;

// ---------------------------------------------------------------------------
// C ABI
#define PR_API_BEGIN(ctx) \
  if (!(ctx)) return PR_EINVAL; \
  try {
#define PR_API_END(ctx)                      \
  }                                          \
  catch (const pr::Error& e) {               \
    (ctx)->err = e.msg;                      \
    return e.st;                             \
  }                                          \
  catch (const std::exception& e) {          \
    (ctx)->err = e.what();                   \
    return PR_EDEVICE;                       \
  }                                          \
  catch (...) {                              \
    (ctx)->err = "unknown error";            \
    return PR_EDEVICE;                       \
  }

extern "C" {

pr_status pr_ctx_create(int device, size_t hbm_budget_bytes, pr_ctx** out) {
  if (!out) return PR_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return PR_EDEVICE;
  if (device < 0 || device >= ndev) return PR_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return PR_EDEVICE;
  try {
    noalloc_scratch_init(device);   // pr_gram_noalloc's scratch on this device
  } catch (const pr::Error&) {
    return PR_EDEVICE;
  }
  pr_ctx* c = new pr_ctx();
  c->device = device;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    delete c;
    return PR_EDEVICE;
  }
  c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)fr);
  for (int i = 0; i < pr_ctx::kSlots; ++i) {
    if (hipHostMalloc((void**)&c->host_slot[i], pr_ctx::kSlotBytes) != hipSuccess ||
        hipMalloc((void**)&c->dev_slot[i], pr_ctx::kSlotBytes) != hipSuccess ||
        hipEventCreateWithFlags(&c->slot_ev[i], hipEventDisableTiming) != hipSuccess) {
      pr_ctx_destroy(c);
      return PR_EDEVICE;
    }
  }
  if (hipHostMalloc((void**)&c->host_scalars, 4096) != hipSuccess) {
    pr_ctx_destroy(c);
    return PR_EDEVICE;
  }
  *out = c;
  return PR_OK;
}

void pr_ctx_destroy(pr_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  release_all(c);
  for (auto& kv : c->tables) (void)hipFree(kv.second);
  for (int i = 0; i < pr_ctx::kSlots; ++i) {
    if (c->host_slot[i]) (void)hipHostFree(c->host_slot[i]);
    if (c->dev_slot[i]) (void)hipFree(c->dev_slot[i]);
    if (c->slot_ev[i]) (void)hipEventDestroy(c->slot_ev[i]);
  }
  if (c->host_scalars) (void)hipHostFree(c->host_scalars);
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  for (auto e : c->ev_pool_timing) (void)hipEventDestroy(e);
  if (c->aux) (void)hipStreamDestroy(c->aux);
  delete c;
}

pr_status pr_fine_tuned(const pr_ctx* c, int precision, int forced, int n, int batch,
                        int* tile_y, int* tile_z, int* threads, int* planes, int* blocked) {
  if (!c || batch < 1 || (precision != PR_F64 && precision != PR_MIXED)) return PR_EINVAL;
  int code = forced ? forced_cfg_forced() : forced_cfg();
  const int vb = precision == PR_MIXED ? 4 : 8;
  std::string key = tune_key(vb, n, batch, forced != 0, forced == 0);
  if (!c->tuned.count(key) && !c->fine_planes.count(key))
    key = tune_key(vb, n, batch, forced != 0, false);
  if (code < 0) {
    auto it = c->tuned.find(key);
    if (it == c->tuned.end()) return PR_EINVAL;
    code = it->second;
  }
  const int cfg = code % kNumFusedCfgs;
  if (tile_y) *tile_y = kFusedCfgs[cfg].ty;
  if (tile_z) *tile_z = kFusedCfgs[cfg].tz;
  if (threads) *threads = kFusedCfgs[cfg].nt;
  if (blocked) *blocked = kFusedCfgs[cfg].blocked;
  if (planes) {
    // chunk length of the key's last launch, else the policy's for `batch`
    // fields of n^3 (general flows)
    auto pit = c->fine_planes.find(key);
    if (pit != c->fine_planes.end()) {
      *planes = pit->second;
    } else {
      pr_grid_problem p{};
      p.n = n;
      const std::vector<FineWork> items(batch,
                                        FineWork{&p, 0.0, 0, nullptr, nullptr, 0, nullptr});
      const long long min_wgs = kChunkMinWgs[code / kNumFusedCfgs];
      const long long slots =
          min_wgs < 0 ? resident_slots(c, cfg, precision == PR_MIXED, forced != 0, false) : 0;
      *planes = std::min(n, fine_chunk(items, cfg, min_wgs, forced != 0, slots));
    }
  }
  return PR_OK;
}

const char* pr_last_error(const pr_ctx* c) { return c ? c->err.c_str() : "null context"; }

size_t pr_ctx_scratch_bytes(const pr_ctx* c) { return c ? c->used : 0; }

pr_status pr_fine_propagate(pr_ctx* c, int batch, const pr_fine_item* items, void* stream) {
  PR_API_BEGIN(c)
  PR_CHECK(batch >= 0 && (batch == 0 || items), "bad batch");
  if (batch == 0) return PR_OK;
  PR_HIP(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  std::vector<FineWork> w;
  for (int i = 0; i < batch; ++i) {
    const pr_fine_item& it = items[i];
    w.push_back(FineWork{it.prob, it.dt, it.n_steps, it.u_in, it.u_out, it.snap_every, it.snaps,
                         it.t0, 0});
  }
  stage_begin(c, s);
  enqueue_fine(c, w, s, "api_fine");
  stage_end(c, s);
  return PR_OK;
  PR_API_END(c)
}

pr_status pr_pod_build(pr_ctx* c, int batch, const pr_pod_item* items, void* stream) {
  PR_API_BEGIN(c)
  PR_CHECK(batch >= 0 && (batch == 0 || items), "bad batch");
  if (batch == 0) return PR_OK;
  PR_HIP(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  std::vector<PodWork> w;
  for (int i = 0; i < batch; ++i) {
    const pr_pod_item& it = items[i];
    check_problem(it.prob);
    PR_CHECK(it.n_blocks >= 1 && it.blocks && it.block_cols, "POD item needs blocks");
    const bool f32 = it.prob->precision == PR_MIXED;
    const long long ng = ngrid(*it.prob);
    PodWork pw;
    pw.prob = it.prob;
    for (int b = 0; b < it.n_blocks; ++b) {
      PR_CHECK(it.blocks[b] && it.block_cols[b] >= 0, "bad POD block");
      const int* v = it.block_valid ? it.block_valid[b] : nullptr;
      for (int j = 0; j < it.block_cols[b]; ++j) pw.cols.push_back(col_of(it.blocks[b], j, ng, f32, v));
    }
    pw.gamma = it.gamma;
    pw.cap = it.cap;
    pw.force_m = it.force_m;
    pw.R_out = it.R_out;
    pw.m_out = it.m_out;
    pw.lambda_out = it.lambda_out;
    w.push_back(pw);
  }
  for (auto& x : w)
    PR_CHECK((int)x.cols.size() <= kMaxPodCols && !x.cols.empty(), "POD input needs 1..64 columns");
  // items of different column-tile counts go in separate launches
  stage_begin(c, s);
  for (int na = 1; na <= 4; ++na) {
    std::vector<PodWork> g;
    for (auto& x : w)
      if (((int)x.cols.size() + 15) / 16 == na) g.push_back(x);
    if (!g.empty()) enqueue_pod(c, g, s, "api_pod");
  }
  stage_end(c, s);
  return PR_OK;
  PR_API_END(c)
}

pr_status pr_gram(pr_ctx* c, const pr_grid_problem* prob, const void* W, int ncols,
                  double* G_out, void* stream) {
  PR_API_BEGIN(c)
  check_problem(prob);
  PR_CHECK(W && G_out, "null Gram buffer");
  PR_CHECK(ncols >= 1 && ncols <= kMaxPodCols, "ncols must be in [1, 64]");
  PR_HIP(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  const bool f32 = prob->precision == PR_MIXED;
  const long long ng = ngrid(*prob);
  const int na = (ncols + 15) / 16, ldg = na * 16;
  double* G = (double*)scratch(c, "api_gram_G", (size_t)ldg * ldg * 8);
  GramWork g;
  g.nrows = ng;
  for (int j = 0; j < ldg; ++j) g.cols.push_back(j < ncols ? col_of(W, j, ng, f32, nullptr) : col_null());
  g.out = G;
  g.ld = ldg;
  const double h = spacing(*prob);
  g.scale = h * h * h;
  stage_begin(c, s);
  enqueue_gram(c, {g}, na, 0, f32, s, "api_gram");
  PR_HIP(hipMemcpy2DAsync(G_out, (size_t)ncols * 8, G, (size_t)ldg * 8, (size_t)ncols * 8, ncols,
                          hipMemcpyDeviceToDevice, s));
  stage_end(c, s);
  return PR_OK;
  PR_API_END(c)
}

pr_status pr_gram_noalloc(pr_ctx* c, const pr_grid_problem* prob, const void* W, int ncols,
                          double* G_out, void* stream) {
  PR_API_BEGIN(c)
  check_problem(prob);
  PR_CHECK(W && G_out, "null Gram buffer");
  PR_CHECK(ncols >= 1 && ncols <= kMaxPodCols, "ncols must be in [1, 64] (the no-alloc maximum)");
  PR_HIP(hipSetDevice(c->device));
  char* area = (char*)noalloc_scratch(c->device);
  if (!area) fail(PR_EDEVICE, "no-alloc scratch not set up on this device");
  hipStream_t s = (hipStream_t)stream;
  const bool f32 = prob->precision == PR_MIXED;
  const long long ng = ngrid(*prob);
  const int na = (ncols + 15) / 16, ldg = na * 16;
  GemmDesc d{};
  d.nrows = ng;
  d.chunk_rows = gram_chunk_rows(ng);
  d.nchunks = (int)((ng + d.chunk_rows - 1) / d.chunk_rows);
  const size_t part = (size_t)d.nchunks * (na * (na + 1) / 2) * 256;
  if (d.nchunks > kGramMaxChunks || part > kNoAllocPartialDoubles)
    fail(PR_EINVAL, "Gram partials exceed the no-alloc scratch");
  // layout of the area: GemmDesc at 0, column descriptors at 256, the
  // padded Gram at kNoAllocDescBytes, the partials after it
  static_assert(sizeof(GemmDesc) <= 256, "descriptor slot");
  static_assert(256 + kMaxPodCols * sizeof(ColDesc) <= sizeof(UploadBlob), "upload blob");
  static_assert(256 + kMaxPodCols * sizeof(ColDesc) <= kNoAllocDescBytes, "descriptor area");
  ColDesc* cols_dev = (ColDesc*)(area + 256);
  double* G = (double*)(area + kNoAllocDescBytes);
  d.wg_begin = 0;
  d.cols = cols_dev;
  d.partial = G + kNoAllocGramDoubles;
  d.out = G;
  d.ld = ldg;
  const double h = spacing(*prob);
  d.scale = h * h * h;
  d.a_in_b = 0;
  // the descriptors travel in the arguments of an upload kernel
  UploadBlob b;
  memset(&b, 0, sizeof b);
  memcpy(b.w, &d, sizeof d);
  for (int j = 0; j < ldg; ++j) {
    const ColDesc cd = j < ncols ? col_of(W, j, ng, f32, nullptr) : col_null();
    memcpy((char*)b.w + 256 + (size_t)j * sizeof(ColDesc), &cd, sizeof cd);
  }
  const int nw = (int)((256 + (size_t)ldg * sizeof(ColDesc) + 3) / 4);
  launch_upload(b, (unsigned int*)area, nw, s);
  launch_gemm_tn((const GemmDesc*)area, 1, d.nchunks, na, 0, f32, s);
  launch_gemm_reduce((const GemmDesc*)area, 1, na, 0, s);
  PR_HIP(hipMemcpy2DAsync(G_out, (size_t)ncols * 8, G, (size_t)ldg * 8, (size_t)ncols * 8, ncols,
                          hipMemcpyDeviceToDevice, s));
  return PR_OK;
  PR_API_END(c)
}

pr_status pr_coarse_propagate(pr_ctx* c, int batch, const pr_coarse_item* items, void* stream) {
  PR_API_BEGIN(c)
  PR_CHECK(batch >= 0 && (batch == 0 || items), "bad batch");
  if (batch == 0) return PR_OK;
  PR_HIP(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  for (int i = 0; i < batch; ++i) {
    const pr_coarse_item& it = items[i];
    check_problem(it.prob);
    PR_CHECK(it.R && it.m, "coarse item needs R and m");
    PR_CHECK(it.cap >= 1 && it.cap <= kMaxCap, "cap must be in [1, 31]");
    PR_CHECK(it.n_in == 1 || it.n_in == 2, "n_in must be 1 or 2");
    for (int j = 0; j < it.n_in; ++j) PR_CHECK(it.u_in[j], "null input state");
    PR_CHECK(std::isfinite(it.dT_total) && it.dT_total > 0, "dT_total must be positive");
    int n_c = it.n_c;
    if (n_c <= 0) {
      PR_CHECK(it.dt_hint > 0, "n_c = 0 needs dt_hint > 0");
      const long long nf = std::max<long long>(1, llround(it.dT_total / it.dt_hint));
      n_c = (int)std::max<long long>(1, (nf + 9) / 10);
    }
    CoarseWork w{};
    w.prob = it.prob;
    w.R = it.R;
    w.LR = nullptr;
    w.cap = it.cap;
    w.m = it.m;
    w.u_aug = it.u_aug;
    w.n_in = it.n_in;
    w.u_in[0] = it.u_in[0];
    w.u_in[1] = it.n_in > 1 ? it.u_in[1] : nullptr;
    w.dT = it.dT_total;
    w.n_c = n_c;
    w.t0 = it.t0;
    w.forcing = nullptr;
    w.lift[0] = it.u_out[0];
    w.lift[1] = it.n_in > 1 ? it.u_out[1] : nullptr;
    w.beta_out = it.beta_out;
    w.n_c_out = it.n_c_out;
    stage_begin(c, s);
    enqueue_coarse(c, w, s, nullptr);
    stage_end(c, s);
  }
  return PR_OK;
  PR_API_END(c)
}

}  // extern "C"
