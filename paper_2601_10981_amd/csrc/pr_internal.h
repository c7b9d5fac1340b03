// Internal declarations of libpr: device descriptors, launchers, context.
// Not part of the public ABI (include/pr.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "pr.h"

namespace pr {

struct Error {
  pr_status st;
  std::string msg;
};

[[noreturn]] void fail(pr_status st, const std::string& msg);

#define PR_HIP(x)                                                                  \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess)                                                          \
      ::pr::fail(PR_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));      \
  } while (0)

#define PR_CHECK(cond, msg)                                                        \
  do {                                                                             \
    if (!(cond)) ::pr::fail(PR_EINVAL, msg);                                       \
  } while (0)

constexpr int kTileQ = 256;     // stencil: (y, z) points per workgroup
constexpr int kChunkX = 32;     // L applied to columns: x planes per workgroup
constexpr int kMaxPodCols = 64;  // columns of one POD input (4 MFMA tiles)
constexpr int kMaxCap = 31;      // basis columns; cap + 1 fits two MFMA tiles
constexpr double kTauRankF64 = 1e-13;
constexpr double kTauRankF32 = 1e-6;
constexpr double kTauAug = 1e-12;
constexpr double kDropPivot = 1e-8;
constexpr int kCholQRPasses = 1;
constexpr double kGuard = 2.5;
constexpr double kStabRK4 = 2.6;
// Column stride of the solver's own multi-column blocks (snapshots, bases, L
// applied to bases): N_g + kColPad elements. With N_g a power of two (128^3,
// 256^3) unpadded columns start 2^k bytes apart, and the tall-skinny MFMA
// Grams -- which read 16 columns at one row per instruction -- then hit the
// same HBM channels (measured: a 64-column 128^3 Gram 385 -> 290 us with the
// pad). Caller buffers at the C ABI stay contiguous.
constexpr long long kColPad = 32;

// ----------------------------------------------------------------------------
// Device pointers read from descriptors are generic; casting them to the
// global address space lets the compiler emit global_load/store (counted by
// vmcnt only) instead of flat accesses, which also count against lgkmcnt and
// would make every LDS wait drain the outstanding global loads.
#define PR_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const PR_GLOBAL T* gptr(const T* p) {
  return (const PR_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ PR_GLOBAL T* gptr(T* p) {
  return (PR_GLOBAL T*)p;
}

// ----------------------------------------------------------------------------
// Grid geometry on the device. The velocity of every flow here is a sum of
// one-dimensional functions of the two other coordinates, so it is stored as
// six tables of n values, pre-multiplied by 1 / (2h):
//   v_x(y, z) = t[0][y] + t[1][z],  v_y(x, z) = t[2][x] + t[3][z],
//   v_z(x, y) = t[4][x] + t[5][y].
// tab64 holds them in double, tab32 in float (for the FP32 stencil).
//
// The forced flows of Sec. 4 separate in time and space:
// v(x, t) = sum_j theta_j(t) v_j(x) and f(x, t) = sum_j theta_j(t) f_j(x),
// theta_0 = 1 (Kolmogorov flow: theta_1 = cos(w t); ABC flow with phase
// s = sin(w t): theta_1 = cos s, theta_2 = sin s). Piece j has nine tables of
// n values at ptab + 9 n j: the six velocity tables above and
// f_j(x, y, z) = t[6][x] + t[7][y] + t[8][z]. tab64/tab32 then point at
// piece 0, so the steady kernels apply piece 0's operator.
enum { kForcedNone = 0, kForcedKolmogorov = 1, kForcedABC = 2 };
constexpr int kMaxPieces = 3;
struct Geom {
  int n;
  int xonly;             // velocity has only an x component (v_y = v_z = 0)
  double c_lap;          // kappa / h^2
  const double* tab64;   // 6 n doubles
  const float* tab32;    // 6 n floats
  int forced;            // kForced*: which theta functions
  int npieces;           // pieces of the forced flow (1 for steady flows)
  double w;              // frequency of the time dependence
  const double* ptab64;  // npieces x 9 n doubles (forced flows)
  const float* ptab32;
};

// theta_j(t) of a forced flow's piece j.
__host__ __device__ inline double theta_of(int kind, double w, int j, double t) {
  if (j == 0) return 1.0;
  if (kind == kForcedKolmogorov) return cos(w * t);
  const double s = sin(w * t);
  return j == 1 ? cos(s) : sin(s);
}

// Column of a tall-skinny operand: N_g values at ptr (float if f32), valid iff
// mptr == nullptr || idx < *mptr (invalid columns read as zero).
struct ColDesc {
  const void* ptr;
  const int* mptr;
  int idx;
  int f32;
};

// ---- fine propagator -------------------------------------------------------
// One launch advances every field of the batch by one RK4 step (all four
// stages fused). Step j reads src(j) and writes buf[ob(j)], with
// ob(j) = (n_steps - 1 - j) % 2, so the last step lands in buf[0];
// src(0) = first_src and src(j) = buf[ob(j - 1)].
template <typename T>
struct FineDesc {
  Geom g;
  const T* first_src;
  T* buf[2];
  T* snaps;        // nullptr or n_s columns: column j = state after j * snap_every steps
  long long snap_ld;  // elements from one snapshot column to the next (>= N_g)
  int snap_every;
  int n_steps;
  double dt;
  int tiles_y, tiles_z, chunks_x, xc;  // (y, z) tiles of the launch's shape, x chunks
  long long tile_begin;
  // forced flows: step j runs from t0 + j dt; with_forcing = 0 drops f (the
  // homogeneous propagator, used for differences of two solutions)
  double t0;
  int with_forcing;
};
constexpr int kFusedHalo = 4;      // one halo layer per RK4 stage
constexpr int kMaxChunk = 256;     // x planes per fused-stencil workgroup (at most)
constexpr int kForcedChunk = 128;  // the same for the forced-flow stencil
// Tile configurations of the fused stencil: output tile TY x TZ of the
// (y, z) plane per workgroup of NT threads. Every configuration computes
// bitwise the same values (each point's arithmetic does not depend on the
// tiling), so the choice is a pure performance knob.
// blocked = 1: the 2 x 2 register-blocked kernel (k_rk4_b22, stencil22.hip),
// one block of four columns per thread; it needs an even n and 2-value
// aligned fields.
struct FusedCfg {
  int ty, tz, nt, blocked;
};
constexpr int kNumFusedCfgs = 11;
constexpr int kNumColumnCfgs = 8;   // the one-column-per-thread tilings come first
constexpr FusedCfg kFusedCfgs[kNumFusedCfgs] = {
    {32, 32, 512, 0}, {16, 32, 256, 0}, {16, 32, 512, 0}, {32, 32, 1024, 0},
    {8, 32, 256, 0},  {16, 64, 512, 0}, {8, 64, 512, 0},  {16, 32, 1024, 0},
    {32, 32, 448, 1}, {16, 64, 512, 1}, {16, 32, 256, 1}};
constexpr int kBlockedChunk = 128;   // x planes per workgroup of the blocked tilings (at most)
inline int fused_ty(int cfg) { return kFusedCfgs[cfg].ty; }
inline int fused_tz(int cfg) { return kFusedCfgs[cfg].tz; }
// Tilings of the forced-flow stencil (at most three columns per thread: it
// keeps per-stage coefficients and an accumulator in registers).
constexpr int kNumForcedCfgs = 5;
constexpr int kForcedCfgs[kNumForcedCfgs] = {2, 3, 4, 6, 7};
// Columns per thread of a tiling (the region with its 4-layer halo over the
// thread count).
inline int fused_slots(int cfg) {
  const FusedCfg& f = kFusedCfgs[cfg];
  if (f.blocked) return 4;
  return ((f.ty + 8) * (f.tz + 8) + f.nt - 1) / f.nt;
}

// ---- L applied to basis columns -------------------------------------------
template <typename T>
struct ApplyLDesc {
  Geom g;
  const T* in;     // ncols columns of N_g values, ld apart
  T* out;
  long long ld;    // column stride in elements (>= N_g)
  int ncols;
  const int* mptr;  // valid columns (nullptr = all); the others are written as zero
  int tiles_q, tiles_x;
  int chunk_x;      // x planes per workgroup (tiles_x = ceil(n / chunk_x))
  long long tile_begin;  // tiles per column = tiles_q * tiles_x
  int skip_tail;    // 1: columns >= *mptr are left unwritten instead
};

// ---- tall-skinny Gram / A^T B on MFMA --------------------------------------
struct GemmDesc {
  long long nrows;
  int chunk_rows;     // multiple of 64
  int nchunks;
  long long wg_begin;
  const ColDesc* cols;   // (NA + NB) * 16 descriptors (A tiles then B tiles;
                         //  for the symmetric form only NA tiles)
  double* partial;       // nchunks x npairs x 256
  double* out;           // reduced output (ld x ...), row = A column
  int ld;
  double scale;
  int a_in_b;            // 1: A's slots are a prefix of B's slots followed by
                         //  null ones, so A's packed tiles are B's leading
                         //  packed tiles; A is not loaded separately
};

// ---- tall-skinny times small (out = sum_c in_c C[c][j] (+ add)) ------------
struct TsmmDesc {
  long long nrows;
  const ColDesc* in;     // nin descriptors
  int nin;
  const double* C;       // nin x ldc, FP64, device
  int ldc;
  void* out;             // nout columns of N_g values, out_ld apart
  long long out_ld;      // output column stride in elements (>= N_g)
  int out_f32;
  int nout;
  const int* out_mptr;   // columns >= *out_mptr written as zero (nullptr: none)
  const double* add;     // nullptr or N_g doubles added to column 0
  double alpha;
  long long wg_begin;
  int skip_tail;         // 1: columns >= *out_mptr are left unwritten instead
};

// ---- correction with jump partials ----------------------------------------
struct CorrectDesc {
  long long nrows;
  const ColDesc* psi;    // npsi basis columns
  int npsi;
  const double* coef;    // npsi doubles (device): beta_new - beta_old
  const void* fine;      // F_n (double or float if fine_f32); nullptr = 0
  int fine_f32;
  double* out;           // U^k_{n+1}
  const double* prev;    // U^{k-1}_{n+1} (nullable)
  const double* ref;     // reference (nullable)
  double* partial;       // nwg x 4: |U-prev|^2, |U|^2, |U-ref|^2, |ref|^2
  long long wg_begin;
  int nwg;
};

// ---- launchers -------------------------------------------------------------
// Fused RK4 steps; cfg selects the tile shape (0: 32 x 32 tile, 512 threads;
// 1: 16 x 32 tile, 256 threads). Every field of a launch uses one cfg.
// xonly: every field of the launch has a velocity along x only (the blocked
// tilings then use a kernel without the per-plane velocity table).
void launch_fine_f64(const FineDesc<double>* d_descs, int nfields, long long total_tiles,
                     int max_steps, int cfg, bool xonly, hipStream_t s);
void launch_fine_f32(const FineDesc<float>* d_descs, int nfields, long long total_tiles,
                     int max_steps, int cfg, bool xonly, hipStream_t s);
// One RK4 step (step index `step`) of every field with step < n_steps.
void launch_fine_step_f64(const FineDesc<double>* d_descs, int nfields, long long total_tiles,
                          int step, int cfg, bool xonly, hipStream_t s);
void launch_fine_step_f32(const FineDesc<float>* d_descs, int nfields, long long total_tiles,
                          int step, int cfg, bool xonly, hipStream_t s);
// The same for the forced flows (classical RK4 with stage times and forcing);
// cfg must be one of kForcedCfgs.
void launch_forced_step_f64(const FineDesc<double>* d_descs, int nfields, long long total_tiles,
                            int step, int cfg, hipStream_t s);
void launch_forced_step_f32(const FineDesc<float>* d_descs, int nfields, long long total_tiles,
                            int step, int cfg, hipStream_t s);
// The blocked tilings (kFusedCfgs[cfg].blocked).
void launch_b22_step_f64(const FineDesc<double>* d_descs, int nfields, long long total_tiles,
                         int step, int cfg, bool xonly, hipStream_t s);
void launch_b22_step_f32(const FineDesc<float>* d_descs, int nfields, long long total_tiles,
                         int step, int cfg, bool xonly, hipStream_t s);
int b22_blocks_per_cu(int cfg, bool f32, bool xonly);
// Workgroups of a tiling resident per CU at once (registers, LDS, threads),
// from the runtime's occupancy calculator.
int fused_blocks_per_cu(int cfg, bool f32, bool xonly);
int forced_blocks_per_cu(int cfg, bool f32);
// f_j of piece j of a forced flow written as an N_g field (double or float).
void launch_forcing_field(const Geom& g, int piece, void* out, int out_f32, hipStream_t s);
void launch_convert_f64_to_f32(const double* in, float* out, long long n, hipStream_t s);

// Small host-to-device uploads carried in the kernel arguments: words[0, nw)
// of the blob are written to dst (4-byte aligned). Cheaper than a copy whose
// engine reads pinned host memory across the bus.
constexpr int kUploadWords = 512;
struct UploadBlob {
  unsigned int w[kUploadWords];
};
void launch_upload(const UploadBlob& b, unsigned int* dst, int nw, hipStream_t s);
void launch_convert_f32_to_f64(const float* in, double* out, long long n, hipStream_t s);
// win: the LDS-window kernel (every item's n in [kWinMinN, kWinMaxN]; tiles of kWinQ
// points of the (y, z) plane); else tiles of kTileQ points.
void launch_applyL_f64(const ApplyLDesc<double>* d, int nitems, long long total_tiles, bool win,
                       hipStream_t s);
void launch_applyL_f32(const ApplyLDesc<float>* d, int nitems, long long total_tiles, bool win,
                       hipStream_t s);
constexpr int kWinQ = 1024;     // points of the (y, z) plane per workgroup of the window kernel
constexpr int kWinMaxN = 256;   // largest n of the window kernel (window kWinQ + 2 n values)
constexpr int kWinMinN = 64;    // smallest (n^2 > kWinQ + n, so a window wraps at most once)

// Gram / A^T B: shape = number of A tiles (na) and B tiles (nb, 0 = symmetric
// Gram of the A tiles). f32 selects the FP32 MFMA (products of float data).
void launch_gemm_tn(const GemmDesc* d, int nitems, long long total_wg, int na, int nb,
                    bool f32, hipStream_t s);
void launch_gemm_reduce(const GemmDesc* d, int nitems, int na, int nb, hipStream_t s);

// ---- the Gram without device allocation (pr_gram_noalloc) -------------------
// A file-scope device array (gemm.hip), one per device, holds the
// descriptors, the padded Gram and the per-chunk partials of one Gram of up
// to 64 columns of any row count (gram_chunk_rows gives at most
// kGramMaxChunks chunks, and four column tiles have 10 tile pairs).
constexpr int kGramMaxChunks = 512;
constexpr size_t kNoAllocDescBytes = 4096;
constexpr size_t kNoAllocGramDoubles = 64 * 64;
constexpr size_t kNoAllocPartialDoubles = (size_t)kGramMaxChunks * 10 * 256;
constexpr size_t kNoAllocBytes =
    kNoAllocDescBytes + 8 * (kNoAllocGramDoubles + kNoAllocPartialDoubles);
// Look up the array's device address on `device` (which must be current);
// does the lookup once per device. Throws PR_EDEVICE on failure.
void noalloc_scratch_init(int device);
// The address looked up for `device`, or nullptr before noalloc_scratch_init.
void* noalloc_scratch(int device);

// ---- one Gram-Schmidt pass of the augmentation (eqaug) ----------------------
// Over the rows of one field: z = y - sum_{j < m} c[j] X_j (or z = y without
// coefficients), then dots[j] = scale * X_j^T z (j < n, zero for j >= m) and
// norm = scale * z^T z. Every column X_j (j < m) is read once, with the lanes
// of a wave on consecutive rows; partial sums per row chunk are added in a
// fixed order, so a result depends on the row count only.
constexpr int kCgsMaxCols = 32;
struct CgsArgs {
  const void* col[kCgsMaxCols];  // X_j, j < n: N_g values each (all FP64 or all FP32)
  int f32;
  const int* mptr;     // device rank: columns j >= *mptr count as zero (nullptr: m = n)
  int n;               // 0..32
  long long nrows;
  int chunk_rows;      // multiple of 256
  int nchunks;
  const double* y;     // N_g doubles
  const double* c;     // nullptr, or n coefficients (device)
  double* z;           // nullptr, or N_g doubles written (may alias y)
  double* partial;     // nchunks x (n + 1)
  double* dots;        // nullptr, or n doubles
  double* norm;        // one double
  double scale;
  // nullptr, or the augmentation decision taken from norm (||d~||_M^2) and
  // *nu2 (||u||_M^2): *flag = 1 and *dscale = 1 / ||d~||_M if d~ is kept
  const double* nu2;
  int* flag;
  double* dscale;
};
int cgs_chunk_rows(long long nrows);
void launch_cgs(const CgsArgs& a, hipStream_t s);

// max_nout: the largest nout of the items (selects the accumulator count).
void launch_tsmm(const TsmmDesc* d, int nitems, long long total_wg, int max_nout, hipStream_t s);
void launch_correct(const CorrectDesc* d, int nitems, long long total_wg, hipStream_t s);

// Small dense FP64 kernels (one workgroup per item).
struct EigDesc {
  const double* G;   // nc x nc (leading dimension ldg)
  int ldg;
  int nc;
  double gamma;
  int cap;
  int force_m;
  double tau_r;
  double* lambda;    // nc (sorted descending)
  double* coef;      // nc x ld_coef: Y_m Lambda_m^{-1/2} (columns >= m zero)
  int ld_coef;
  int* m_out;
};
void launch_eig_select(const EigDesc* d, int nitems, hipStream_t s);

struct CholDesc {
  const double* G;   // cap x cap (leading dimension ldg): Gram of the modes
  int ldg;
  int cap;
  int* m;            // in/out: valid columns (lowered if a pivot is dropped)
  double* coef;      // cap x cap: L^{-T} (upper triangular), zero beyond m
};
void launch_cholqr_coef(const CholDesc* d, int nitems, hipStream_t s);

// CholQR of modes W C taken from the Gram G of W instead of a pass over the
// modes: G2 = C^T G C (rows i of C with G_ii = 0 are skipped: zero columns of
// W), then, after launch_cholqr_coef on G2, C <- C U with U its upper
// triangular factor (zero beyond the rank).
struct CoefGramDesc {
  const double* G;   // nc x nc, leading dimension ldg
  int ldg;
  int nc;            // <= 64
  double* C;         // nc x cap, leading dimension ldc (in place)
  int ldc;
  int cap;           // <= 32
  double* G2;        // cap x cap, leading dimension 32
  const double* U;   // cap x cap, leading dimension cap (launch_cholqr_coef's)
};
void launch_coef_gram(const CoefGramDesc* d, int nitems, hipStream_t s);
void launch_coef_apply(const CoefGramDesc* d, int nitems, hipStream_t s);

// Block whitening of a Gram over nb blocks of bs columns (block b's first
// *m[b] columns valid, the rest zero rows and columns): with the Cholesky
// factors T_b^T T_b = G_bb of the diagonal blocks (a pivot <= kDropPivot
// ends block b's valid columns there), G <- D^{-T} G D^{-1}, D = blockdiag(T_b):
// the Gram the blocks would have after an M-orthonormalisation of each. Then,
// after the eigenproblem, coefficients C (rows = the same columns) become
// D^{-1} C, so W D^{-1} C = W (D^{-1} C) forms the modes from the raw blocks.
constexpr int kWhitenMaxCols = 64;
struct WhitenDesc {
  double* G;         // nb bs x nb bs, leading dimension ldg (in place)
  int ldg;
  int nb, bs;        // nb * bs <= 64, bs <= 32
  const int* m[kWhitenMaxCols];  // per block: device rank (nullptr: bs)
  double* T;         // nb x bs x bs: the factors (written by whiten)
  int* meff;         // nb: valid columns kept per block (written by whiten)
  double* coef;      // nb bs x ld_coef (unwhiten, in place)
  int ld_coef;
  int ncoef;         // coefficient columns
};
void launch_block_whiten(const WhitenDesc* d, int nitems, hipStream_t s);
void launch_block_unwhiten(const WhitenDesc* d, int nitems, hipStream_t s);

// Reduced propagation (one item per coarse solve). The reduced matrices are
// read from the Gram output: S (q x ld) with Psi^T M Psi in columns
// [0, q) and Psi^T M L Psi in columns [q_off_L, q_off_L + q) and the
// projections Psi^T M u_i in column q_off_U + i.
// Forced flows: S holds Psi^T M L_j Psi in columns [off_L + ld_piece j, ...)
// for piece j < npieces and Psi^T M f_j in column off_F + j; the system is
// M_r beta' = sum_j theta_j(t) (L_r,j beta + f_r,j) from t0.
struct ReducedDesc {
  const double* S;
  int ld;            // leading dimension of S (row = basis index)
  int ld_piece;      // column distance of the L pieces in S (0: 32)
  int cap;           // R columns (rows 0..cap-1); the augmented column is row cap
  const int* m;      // valid R columns
  const int* aug;    // device flag: 1 if column `cap` (d) is present
  int off_M, off_L, off_U;
  int n_in;
  double dT;
  int n_c;
  int forced, npieces, off_F;
  double w, t0;
  double* beta;      // n_in x (cap + 1): beta_i(dT)
  double* coef;      // nullable: (cap+1): beta_0 - beta_1 (correction coefficients)
  int* n_c_out;      // nullable
};
void launch_reduced(const ReducedDesc* d, int nitems, hipStream_t s);
void launch_reduced_one(const ReducedDesc& d, hipStream_t s);

// k = 0 recurrence: beta_{n+1} = S^{n_c} beta_n for n = 0..count-1 written
// into coef rows (count x ld_out) for the lift.
struct Reduced0Desc {
  const double* S;
  int ld, cap;
  int ld_piece;      // column distance of the L pieces in S (0: 32)
  const int* m;
  int off_M, off_L, off_U;
  double dT;
  int n_c;
  int forced, npieces, off_F;
  double w;          // subinterval n starts at (n + n_warm) dT
  int n_warm;        // subintervals of the warm-up window
  int count;
  double* betas;     // count x ld_out
  int ld_out;
  int* n_c_out;
};
void launch_reduced0(const Reduced0Desc* d, hipStream_t s);

// out[i] = -in[i], i < n (one small vector, n <= 256).
void launch_negate(const double* in, double* out, int n, hipStream_t s);

// out[0] = max_{i, j < min(*m, cap)} |G[i ld + j] - delta_ij| (device m).
void launch_orth_defect(const double* G, int ld, const int* m, int cap, double* out,
                        hipStream_t s);

// Partial-sum reduction of jump norms: per item sums partial (nwg x 4) in
// fixed order into out (4 doubles, times h^3).
// ---- grid transfers of the coarse-grid coarse propagator ---------------------
struct RestrictDesc {
  int m;               // coarse points per axis (fine n = 2 m)
  const double* a;     // fine field
  const double* b;     // fine field subtracted first (nullable)
  double* out;         // m^3 coarse values
};
struct ProlongDesc {
  int m;               // coarse points per axis
  const double* c;     // m^3 coarse values
  const double* fine;  // added after interpolation (nullable)
  double* out;         // (2 m)^3 fine values
  const double* prev;  // nullable: jump partials against it
  const double* ref;   // nullable: error partials against it
  double* partial;     // nwg x 4 (layout of CorrectDesc::partial)
  int nwg;
};
void launch_restrict(const RestrictDesc* d, long long coarse_points, hipStream_t s);
void launch_prolong_add(const ProlongDesc* d, int nwg, hipStream_t s);

struct NormReduceDesc {
  const double* partial;
  int nwg;
  double scale;
  double* out;
};
void launch_norm_reduce(const NormReduceDesc* d, int nitems, hipStream_t s);

// e_k = max_n sqrt(j_n) / sqrt(u_n) over the items' 4-vectors; err likewise
// from entries 2 and 3. Writes {e_k, err_k} to out.
void launch_jump_max(const double* norms4, int count, double* out, hipStream_t s);

// out = (*scale) * in, with out double or float (out_f32).
void launch_scale_into(const double* in, void* out, int out_f32, long long n,
                       const double* scale, hipStream_t s);

}  // namespace pr
