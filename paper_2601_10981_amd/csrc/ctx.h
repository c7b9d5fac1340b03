// Context of libpr: scratch memory under a budget, descriptor staging and
// cached velocity tables. Internal.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "pr_internal.h"

struct pr_ctx {
  int device = 0;
  size_t budget = 0;
  size_t used = 0;
  std::string err;

  struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
  };
  std::map<std::string, Buf> bufs;
  // Idle device blocks of finished solves, by size, kept for the next solve
  // (counted in `used`; given back when the budget needs the room).
  std::multimap<size_t, void*> pool;
  std::map<std::string, void*> tables;   // velocity tables by problem key
  std::map<std::string, int> tuned;      // fused-stencil configuration by batch key
  std::map<std::string, int> fine_planes;  // x chunk of the last launch of each batch key
  // resident stencil workgroups by tiling and the device's compute units
  // (caches filled on first use, also through const queries)
  mutable std::map<int, long long> fused_slots;
  mutable int n_cu = 0;

  // Descriptor staging: a ring of pinned host slots mirrored by device slots.
  static constexpr int kSlots = 8;
  static constexpr size_t kSlotBytes = size_t(16) << 20;
  char* host_slot[kSlots] = {};
  char* dev_slot[kSlots] = {};
  hipEvent_t slot_ev[kSlots] = {};
  int slot = -1;
  size_t off = 0, flushed = 0;
  hipStream_t stream = nullptr;   // stream of the current staging session
  hipStream_t aux = nullptr;      // second stream of the solver (created on first use)

  // Small pinned host buffer for scalars read back by the solver.
  double* host_scalars = nullptr;

  std::vector<hipEvent_t> ev_pool;
  // Events used only to time phases: recorded without the system-scope
  // fence, whose cache writeback otherwise stalls the stream at every mark.
  std::vector<hipEvent_t> ev_pool_timing;
};

namespace pr {

// Device scratch buffer `name` of at least `bytes` (grows; budget-checked).
void* scratch(pr_ctx* c, const std::string& name, size_t bytes);
void release_all(pr_ctx* c);
// Solve-owned blocks: pool_get reuses an idle block of the same size class
// (within 1/8) or allocates one on the budget; pool_put returns an idle one.
void* pool_get(pr_ctx* c, size_t bytes, size_t* got);
void pool_put(pr_ctx* c, void* p, size_t bytes);

// Descriptor staging. begin() takes a fresh slot (waiting for its previous
// use to complete), push() copies items into it and returns their device
// address, flush() enqueues the host-to-device copy of what was pushed since
// the last flush, end() marks the slot's use as finished on `s`.
void stage_begin(pr_ctx* c);
void stage_begin(pr_ctx* c, hipStream_t s);
void* stage_push_bytes(pr_ctx* c, const void* src, size_t bytes);
template <typename T>
T* stage_push(pr_ctx* c, const std::vector<T>& v) {
  return (T*)stage_push_bytes(c, v.data(), v.size() * sizeof(T));
}
template <typename T>
T* stage_push1(pr_ctx* c, const T& v) {
  return (T*)stage_push_bytes(c, &v, sizeof(T));
}
void stage_flush(pr_ctx* c, hipStream_t s);
void stage_end(pr_ctx* c, hipStream_t s);

// Problem geometry with device velocity tables.
Geom geom_of(pr_ctx* c, const pr_grid_problem& p);
Geom geom_piece(const Geom& g, int j);
bool forced_flow(const pr_grid_problem& p);
int flow_pieces(const pr_grid_problem& p);
double spacing(const pr_grid_problem& p);
double spectral_bound(const pr_grid_problem& p);
void check_problem(const pr_grid_problem* p);
inline long long ngrid(const pr_grid_problem& p) { return (long long)p.n * p.n * p.n; }
inline size_t field_bytes(const pr_grid_problem& p) {
  return (size_t)ngrid(p) * (p.precision == PR_MIXED ? 4 : 8);
}

// Tile counts of the stencil launches.
inline int tiles_q(int n) { return (n * n + kTileQ - 1) / kTileQ; }
inline int tiles_x(int n) { return (n + kChunkX - 1) / kChunkX; }

// Chunking of the MFMA Gram: rows per chunk (multiple of 64) for an item of
// `nrows` rows; independent of the batch.
int gram_chunk_rows(long long nrows);
// Rows per workgroup of the sweep's one-item Galerkin product, and the most
// chunks either chunking gives for nrows (partial buffers are sized by it).
int galerkin_chunk_rows(long long nrows);
long long gram_chunks_max(long long nrows);

// Enqueue helpers shared by the entry points and the solver.
struct FineWork {
  const pr_grid_problem* prob;
  double dt;
  int n_steps;
  const double* u_in;
  double* u_out;
  int snap_every;
  void* snaps;
  double t0 = 0.0;      // forced flows: start time
  int unforced = 0;     // forced flows: 1 = homogeneous propagator (no f)
  long long snap_ld = 0;  // snapshot column stride in elements (0: N_g)
};
void enqueue_fine(pr_ctx* c, const std::vector<FineWork>& items, hipStream_t s,
                  const std::string& tag);

struct PodWork {
  const pr_grid_problem* prob;
  std::vector<ColDesc> cols;   // input columns (<= 64)
  double gamma;
  int cap;
  int force_m;
  void* R_out;                 // cap columns (field precision), R_ld apart
  int* m_out;
  double* lambda_out;          // nullable, >= cols.size()
  long long R_ld = 0;          // column stride of R_out in elements (0: N_g)
  int skip_tail = 0;           // 1: R_out columns >= *m_out are left unwritten
                               // (for consumers that mask by the rank)
  int cholqr = 1;              // 0: the modes are left as W y_i / sqrt(lambda_i)
  int whiten_bs = 0;           // > 0: the input is blocks of whiten_bs columns
                               // (block b's rank in cols[b whiten_bs].mptr),
                               // each taken as M-orthonormalised (WhitenDesc)
};
void enqueue_pod(pr_ctx* c, const std::vector<PodWork>& items, hipStream_t s,
                 const std::string& tag);

// One Gram product: A columns (na tiles of 16) against B columns (nb tiles,
// 0 = symmetric Gram of A), out = scale * A^T B with leading dimension ld.
struct GramWork {
  long long nrows;
  std::vector<ColDesc> cols;   // (na + nb) * 16
  double* out;
  int ld;
  double scale;
  int a_in_b = 0;              // 1: the A columns are a prefix of the B columns
                               // (then null slots); A is taken from B's loads
  int chunk_rows = 0;          // rows per workgroup (0: gram_chunk_rows)
};
void enqueue_gram(pr_ctx* c, const std::vector<GramWork>& items, int na, int nb, bool f32,
                  hipStream_t s, const std::string& tag);
// The enqueue helpers in two halves: stage_* pushes the descriptors (no
// flush, no launch), launch_*_staged launches once a flush has uploaded them.
// A caller staging several launches flushes once for all of them.
struct StagedGram {
  GemmDesc* dd = nullptr;
  int nd = 0;
  long long wg = 0;
  int na = 0, nb = 0;
  bool f32 = false;
};
StagedGram stage_gram(pr_ctx* c, const std::vector<GramWork>& items, int na, int nb, bool f32,
                      const std::string& tag);
void launch_gram_staged(const StagedGram& g, hipStream_t s);

void enqueue_applyL(pr_ctx* c, const pr_grid_problem& p, const void* in, void* out, int ncols,
                    const int* mptr, hipStream_t s);
struct ApplyLWork {
  const pr_grid_problem* prob;
  const void* in;
  void* out;
  int ncols;
  const int* mptr;
  int piece = 0;          // forced flows: apply piece `piece` of L(t)
  long long ld = 0;       // column stride of in and out in elements (0: N_g)
  int skip_tail = 0;      // 1: columns >= *mptr left unwritten (else zeroed)
};
void enqueue_applyL_batch(pr_ctx* c, const std::vector<ApplyLWork>& items, hipStream_t s);
struct StagedApplyL {
  bool f32 = false;
  bool win = false;           // the LDS-window kernel
  const void* dd = nullptr;   // ApplyLDesc<float> or <double>
  int nd = 0;
  long long tiles = 0;
};
StagedApplyL stage_applyL_batch(pr_ctx* c, const std::vector<ApplyLWork>& items);
void launch_applyL_staged(const StagedApplyL& st, hipStream_t s);
void enqueue_applyL_pieces(pr_ctx* c, const pr_grid_problem& p, const void* in, void* out,
                           int ncols, const int* mptr, hipStream_t s, long long ld = 0);
void enqueue_forcing_fields(pr_ctx* c, const pr_grid_problem& p, void* out, hipStream_t s,
                            long long ld = 0);

// The coarse step of the sweep (eqaug, eq12, eq13, formula4): augment span(R)
// with u_aug, form the Galerkin matrices of Psi = [R, d] against [Psi, L Psi,
// u_in[0], u_in[1]], propagate the projections with RK4 over dT and either
// lift each (lift) or write the correction Psi (beta_0 - beta_1) + fine into
// corr_out with jump partials.
struct CoarseWork {
  const pr_grid_problem* prob;
  const void* R;          // N_g x cap (field precision)
  const void* LR;         // L_j R (N_g x cap per piece j), may be nullptr (then computed)
  int cap;
  const int* m;
  const double* u_aug;    // nullable
  int n_in;
  const double* u_in[2];
  double dT;
  int n_c;
  double t0;              // start time (forced flows)
  const void* forcing;    // forced flows: the pieces' f_j (field precision), nullable
  long long ld;           // column stride of R, LR and forcing in elements (0: N_g)
  // outputs
  double* lift[2];        // nullable
  double* beta_out;       // nullable, n_in x (cap + 1)
  int* n_c_out;           // nullable
  // correction (sweep): out = Psi coef + fine, partial norms
  double* corr_out;       // nullable
  const double* fine;
  const double* prev;
  const double* ref;
  double* norms4;         // 4 doubles (|U-prev|^2, |U|^2, |U-ref|^2, |ref|^2)
  // coarse-gap diagnostics (nullable): diag_norms[0..3] = the norms4 of
  // fine - Psi beta_1 against fine, [4..7] those of diag_ref - Psi beta_0
  // against diag_ref (diag_ref nullable), [8] = max |R^T M R - I| of the
  // basis R (its valid columns)
  double* diag_norms;
  const double* diag_ref;
};
struct PhaseEvents;
void enqueue_coarse(pr_ctx* c, const CoarseWork& w, hipStream_t s, PhaseEvents* ph);

// Correction / lift: out = sum_c psi_c coef_c + fine with norm partials.
void enqueue_correct(pr_ctx* c, long long nrows, const std::vector<ColDesc>& psi,
                     const double* coef, const void* fine, int fine_f32, double* out,
                     const double* prev, const double* ref, double* norms4, double h3,
                     hipStream_t s, const std::string& tag);
struct StagedCorrect {
  CorrectDesc* dd = nullptr;
  NormReduceDesc* nrd = nullptr;
  int nwg = 0;
};
// psi_dev: npsi column descriptors already staged (shared by several calls).
StagedCorrect stage_correct(pr_ctx* c, long long nrows, const ColDesc* psi_dev, int npsi,
                            const double* coef, const void* fine, int fine_f32, double* out,
                            const double* prev, const double* ref, double* norms4, double h3,
                            const std::string& tag);
void launch_correct_staged(const StagedCorrect& k, hipStream_t s);

// Phase timing with events (F, C, U, A, G). One event marks each phase
// change: it ends the interval of the phase before and starts the next one.
struct PhaseEvents {
  pr_ctx* c = nullptr;
  hipStream_t s = nullptr;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> open;
  std::vector<hipEvent_t> marks;   // every event recorded, released by collect()
  double t[5] = {0, 0, 0, 0, 0};
  int cur = -1;
  hipEvent_t cur_start = nullptr;
  PhaseEvents() = default;
  PhaseEvents(const PhaseEvents&) = delete;
  PhaseEvents& operator=(const PhaseEvents&) = delete;
  ~PhaseEvents();
  void begin(int phase);
  void end();
  void collect();   // after a synchronisation point
 private:
  hipEvent_t mark();
};

hipEvent_t event_get(pr_ctx* c);
void event_put(pr_ctx* c, hipEvent_t e);
// Timing-only events (no system-scope fence at record; not for host waits).
hipEvent_t timing_event_get(pr_ctx* c);
void timing_event_put(pr_ctx* c, hipEvent_t e);

}  // namespace pr
