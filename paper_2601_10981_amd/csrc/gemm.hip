// Tall-skinny contractions of the POD and reduced-system path:
//   * Gram / A^T B on MFMA (the snapshot Gram W^T M W of Algorithm 1 and the
//     Galerkin products Psi^T M (L Psi), Psi^T M Psi, Psi^T M U of eq. 8 /
//     eq13), split over row chunks with per-chunk FP64 partials summed in a
//     fixed order (deterministic);
//   * out = alpha * In C (+ add): modes r_i = W y_i / sqrt(lambda_i),
//     re-orthonormalisation, projection residual and lift;
//   * the parareal correction U^k_{n+1} = Psi (beta_new - beta_old) + F_n
//     (formula4) with wave-shuffle partial sums of the jump norms.
#include <mutex>

#include "pr_internal.h"

namespace pr {

// ---------------------------------------------------------------------------
// Device scratch of pr_gram_noalloc, for callers that cannot allocate device
// memory: kNoAllocDescBytes of descriptors, the padded 64 x 64 Gram, then the
// per-chunk partials. In host code the array's name only stands in for the
// symbol; its device address on each device is looked up once (at context
// creation) and only that address is passed to kernels and copies.
static __device__ __align__(256) double noalloc_area[kNoAllocBytes / 8];

constexpr int kMaxDevices = 64;
static std::mutex noalloc_mu;
static void* noalloc_ptr[kMaxDevices];

void noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) fail(PR_EDEVICE, "device index beyond 64");
  std::lock_guard<std::mutex> lock(noalloc_mu);
  if (noalloc_ptr[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_area));
  if (e != hipSuccess || p == nullptr)
    fail(PR_EDEVICE, std::string("hipGetSymbolAddress(noalloc_area): ") + hipGetErrorString(e));
  noalloc_ptr[device] = p;
}

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(noalloc_mu);
  return noalloc_ptr[device];
}

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename D>
__device__ __forceinline__ int find_wg(const D* d, int nd, long long w) {
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].wg_begin <= w) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ bool col_valid(const ColDesc& c) {
  return c.ptr != nullptr && (c.mptr == nullptr || c.idx < *c.mptr);
}

template <typename In>
__device__ __forceinline__ In load_col(const void* p, int f32, long long row) {
  return f32 ? (In)gptr((const float*)p)[row] : (In)gptr((const double*)p)[row];
}

typedef double v2d_t __attribute__((ext_vector_type(2)));
typedef float v4f_t __attribute__((ext_vector_type(4)));

// Rows row .. row + 3 of a column in vector loads: row a multiple of 4 and
// the column base 16-byte aligned (checked by the caller).
template <typename In>
__device__ __forceinline__ void load_col4(const void* p, int f32, long long row, In* v) {
  if (f32) {
    const v4f_t a = *(const PR_GLOBAL v4f_t*)(gptr((const float*)p) + row);
    v[0] = (In)a.x;
    v[1] = (In)a.y;
    v[2] = (In)a.z;
    v[3] = (In)a.w;
  } else {
    const v2d_t a = *(const PR_GLOBAL v2d_t*)(gptr((const double*)p) + row);
    const v2d_t b = *(const PR_GLOBAL v2d_t*)(gptr((const double*)p) + row + 2);
    v[0] = (In)a.x;
    v[1] = (In)a.y;
    v[2] = (In)b.x;
    v[3] = (In)b.y;
  }
}

// ---------------------------------------------------------------------------
// MFMA 16x16x4 operand layout (wave64): lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; the 16x16 result has lane l holding, in its
// register v = 0..3, column l % 16 and row
//   4 (l / 16) + v   for v_mfma_f32_16x16x4_f32,
//   l / 16 + 4 v     for v_mfma_f64_16x16x4_f64.
// For a Gram over rows r, A[i][k] = X[r_k][i] and B[k][j] = Y[r_k][j] with
// the same row r_k for lane group k: lane (i, kq) loads rows
// r0 + 4 kq + u (u = 0..3) of its column, i.e. 16 lanes x 4 rows of one
// column are 16 consecutive values (128 B for FP64), and the four u give
// four MFMA steps over 16 rows.
template <bool F32>
struct Mfma;
template <>
struct Mfma<false> {
  using In = double;
  using Acc = v4d;
  __device__ static Acc op(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<true> {
  using In = float;
  using Acc = v4f;
  __device__ static Acc op(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

template <int NA, int NB>
struct PairList {
  static constexpr int P = (NB == 0) ? NA * (NA + 1) / 2 : NA * NB;
  static constexpr int NT = NA + NB;
  __host__ __device__ static constexpr int a(int p) {
    if (NB != 0) return p / NB;
    int i = 0, c = NA;
    while (p >= c) { p -= c; ++i; --c; }
    return i;
  }
  __host__ __device__ static constexpr int b(int p) {
    if (NB != 0) return NA + p % NB;
    int i = 0, c = NA;
    while (p >= c) { p -= c; ++i; --c; }
    return i + p;
  }
};

constexpr int kFlushSteps = 4;  // FP32 MFMA: fold into FP64 every 4 x 64 rows

// Runtime compaction of a column group (one wave): the valid columns among
// cols[base, base + count) in their order. src[base + i] receives the
// descriptor index of the i-th valid column and pos[base + c] the compact
// position of column c (-1 if invalid); either may be null. Returns the
// number of valid columns. Columns whose validity hangs on a device rank
// (POD modes beyond m, an absent augmentation column) thus take no MFMA
// tile of their own.
__device__ int compact_group(const ColDesc* __restrict__ cols, int base, int count, short* src,
                             short* pos, int lane) {
  int off = 0;
  for (int c0 = 0; c0 < count; c0 += 64) {
    const int c = c0 + lane;
    const bool v = c < count && col_valid(cols[base + c]);
    const unsigned long long mask = __ballot(v);
    const int p = off + __popcll(mask & ((1ull << lane) - 1ull));
    if (v && src) src[base + p] = (short)(base + c);
    if (c < count && pos) pos[base + c] = (short)(v ? p : -1);
    off += __popcll(mask);
  }
  return off;
}

template <int NA, int NB, bool F32>
__global__ __launch_bounds__(256) void k_gemm_tn(const GemmDesc* __restrict__ descs, int nd) {
  using M = Mfma<F32>;
  using In = typename M::In;
  using PL = PairList<NA, NB>;
  constexpr int P = PL::P;
  constexpr int NT = PL::NT;
  __shared__ double red[4][256];

  const long long w = blockIdx.x;
  const int f = find_wg(descs, nd, w);
  const GemmDesc& d = descs[f];
  const int chunk = (int)(w - d.wg_begin);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ci = lane & 15, kq = lane >> 4;

  // valid columns packed into the leading tiles of each group (A, then B);
  // only tile pairs holding some of them are computed
  __shared__ short s_src[NT * 16];
  __shared__ int s_cnt[2];
  if (wave == 0) {
    const int na = compact_group(d.cols, 0, NA * 16, s_src, nullptr, lane);
    const int nb = NB == 0 ? 0 : compact_group(d.cols, NA * 16, NB * 16, s_src, nullptr, lane);
    if (lane == 0) {
      s_cnt[0] = na;
      s_cnt[1] = nb;
    }
  }
  __syncthreads();
  const int tA = (s_cnt[0] + 15) >> 4;
  const int tB = NB == 0 ? tA : (s_cnt[1] + 15) >> 4;
  // A's packed tiles are B's leading packed tiles: only B is loaded, and B's
  // registers serve as the A operand (the 16x16x4 operand layouts of A^T and
  // B coincide). Entries at packed A positions past A's count then hold B
  // columns; the reduction never reads them.
  constexpr bool kCanAinB = NB >= NA;
  const bool a_in_b = kCanAinB && d.a_in_b != 0;
  const void* cp[NT];
  int cf[NT];
  bool cv[NT], c16[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int slot = (t < NA) ? t * 16 + ci : (t - NA) * 16 + ci;
    const int n_grp = (t < NA) ? s_cnt[0] : s_cnt[1];
    cv[t] = slot < n_grp;
    const ColDesc c = d.cols[cv[t] ? s_src[t * 16 + ci] : 0];
    cp[t] = c.ptr;
    cf[t] = c.f32;
    c16[t] = ((unsigned long long)c.ptr & 15ull) == 0;
  }

  v4d acc[P];
#pragma unroll
  for (int p = 0; p < P; ++p) acc[p] = v4d{0.0, 0.0, 0.0, 0.0};
  typename M::Acc acc32[P];
  if constexpr (F32) {
#pragma unroll
    for (int p = 0; p < P; ++p) acc32[p] = typename M::Acc{0, 0, 0, 0};
  }

  const long long r_begin = (long long)chunk * d.chunk_rows;
  const long long r_end = min(d.nrows, r_begin + (long long)d.chunk_rows);
  int since_flush = 0;
  for (long long r0 = r_begin + wave * 16; r0 < r_end; r0 += 64) {
    // wide tile sets hold one row per column at a time (register pressure);
    // narrow ones load the lane's four consecutive rows at once
    constexpr int UL = (NT > 5) ? 1 : 4;
#pragma unroll
    for (int u0 = 0; u0 < 4; u0 += UL) {
      In v[NT][UL];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const bool act = (t < NA) ? (t < tA && !a_in_b) : t - NA < tB;
        const long long rb = r0 + 4 * kq + u0;
        // vector loads pay in the symmetric (POD) Grams; the sweep's one-item
        // Galerkin products measured slower with them
        if (UL == 4 && NB == 0 && act && cv[t] && c16[t] && rb + 3 < r_end) {
          load_col4<In>(cp[t], F32 ? 1 : cf[t], rb, v[t]);
        } else {
#pragma unroll
          for (int u = 0; u < UL; ++u) {
            const long long row = rb + u;
            v[t][u] = (act && cv[t] && row < r_end) ? load_col<In>(cp[t], F32 ? 1 : cf[t], row)
                                                    : (In)0;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < UL; ++u) {
        // pairs in PairList order, as nested compile-time loops so every
        // register index is a constant after unrolling
#pragma unroll
        for (int ia = 0; ia < NA; ++ia) {
#pragma unroll
          for (int jb = 0; jb < (NB == 0 ? NA : NB); ++jb) {
            if (NB == 0 && jb < ia) continue;
            const int p = (NB == 0) ? ia * NA - ia * (ia - 1) / 2 + (jb - ia) : ia * NB + jb;
            const int ib = (NB == 0) ? jb : NA + jb;
            // FP32 multiplies every tile pair (padding tiles hold zeros):
            // a per-pair branch there splits the FP32 accumulators' live
            // ranges and the compiler copies them around every MFMA
            if (!F32 && (ia >= tA || jb >= tB)) continue;
            const In va = (kCanAinB && a_in_b) ? v[kCanAinB ? NA + ia : ia][u] : v[ia][u];
            if constexpr (F32)
              acc32[p] = M::op(va, v[ib][u], acc32[p]);
            else
              acc[p] = M::op(va, v[ib][u], acc[p]);
          }
        }
      }
    }
    if constexpr (F32) {
      if (++since_flush < kFlushSteps) continue;
      since_flush = 0;
#pragma unroll
      for (int p = 0; p < P; ++p) {
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[p][e] += (double)acc32[p][e];
        acc32[p] = typename M::Acc{0, 0, 0, 0};
      }
    }
  }
  if constexpr (F32) {
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[p][e] += (double)acc32[p][e];
  }

  // Sum the four waves' tiles through LDS, one pair at a time; thread
  // t = v * 64 + lane handles the element register v of `lane` holds.
  const int tv = threadIdx.x >> 6, tl = threadIdx.x & 63;
  const int e_row = F32 ? 4 * (tl >> 4) + tv : (tl >> 4) + 4 * tv;
  const int e_out = e_row * 16 + (tl & 15);
  PR_GLOBAL double* part = gptr(d.partial) + (long long)chunk * P * 256;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    if (PL::a(p) >= tA || PL::b(p) - (NB == 0 ? 0 : NA) >= tB) continue;  // uniform
#pragma unroll
    for (int e = 0; e < 4; ++e) red[wave][e * 64 + lane] = acc[p][e];
    __syncthreads();
    const double s = (red[0][threadIdx.x] + red[1][threadIdx.x]) +
                     (red[2][threadIdx.x] + red[3][threadIdx.x]);
    part[p * 256 + e_out] = s;
    __syncthreads();
  }
}

// Sum of the per-chunk partials of one tile pair, scaled, written to the
// output (and its mirror for the symmetric form). Workgroup (x, item) owns 16
// of the pair's 256 entries (x = pair * 16 + sixteenth) in the original
// column order; each entry is looked up at its compact position (the
// compaction of k_gemm_tn, redone here), and entries of invalid columns are
// zero. Its 256 threads form 16 chunk groups q = 0..15 of 16 threads (one per
// entry). Group q sums the chunks q, q + 16, q + 32, ... into eight
// accumulators, accumulator u taking the chunks congruent to q + 16 u modulo
// 128 in increasing order; the eight combine as ((0+1)+(2+3))+((4+5)+(6+7)),
// and the 16 groups' sums as the same tree over the pairs (2g, 2g + 1). The
// order depends only on the chunk count, so the result does not depend on
// the batch. Small workgroups start in the gaps that concurrent kernels leave
// (a 1024-thread one waits for a nearly free CU).
template <int NA, int NB>
__global__ __launch_bounds__(256) void k_gemm_reduce(const GemmDesc* __restrict__ descs) {
  using PL = PairList<NA, NB>;
  constexpr int P = PL::P;
  __shared__ double red[16][16];
  __shared__ short s_pos[(NA + NB) * 16];
  const GemmDesc& d = descs[blockIdx.y];
  const int p = blockIdx.x >> 4;
  const int e = ((blockIdx.x & 15) << 4) | (threadIdx.x & 15);
  const int q = threadIdx.x >> 4;
  if (threadIdx.x < 64) {   // wave 0
    compact_group(d.cols, 0, NA * 16, nullptr, s_pos, threadIdx.x);
    if (NB != 0) compact_group(d.cols, NA * 16, NB * 16, nullptr, s_pos, threadIdx.x);
  }
  __syncthreads();
  const int ta = PL::a(p), tb = PL::b(p);
  int pa = s_pos[ta * 16 + (e >> 4)], pb = s_pos[tb * 16 + (e & 15)];
  const bool valid = pa >= 0 && pb >= 0;
  int pc = 0;
  if (valid) {
    if (NB == 0 && (pa >> 4) > (pb >> 4)) {
      const int t = pa;
      pa = pb;
      pb = t;
    }
    const int ia = pa >> 4, jb = pb >> 4;
    pc = (NB == 0) ? ia * NA - ia * (ia - 1) / 2 + (jb - ia) : ia * NB + jb;
    pc = pc * 256 + (pa & 15) * 16 + (pb & 15);
  }
  const PR_GLOBAL double* src = gptr(d.partial) + pc;
  const long long stride = (long long)P * 256;
  const int nch = valid ? d.nchunks : 0;
  // eight chunk loads in flight per round (the sum is latency-bound: a few
  // MB spread over few workgroups)
  double a[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) a[u] = 0.0;
  int c = q;
  for (; c + 7 * 16 < nch; c += 8 * 16) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = src[(long long)(c + 16 * u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += t[u];
  }
#pragma unroll
  for (int u = 0; u < 7; ++u)
    if (c + 16 * u < nch) a[u] += src[(long long)(c + 16 * u) * stride];
  red[q][threadIdx.x & 15] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  __syncthreads();
  if (q != 0) return;
  const int l = threadIdx.x & 15;
  double t[8];
#pragma unroll
  for (int g = 0; g < 8; ++g) t[g] = red[2 * g][l] + red[2 * g + 1][l];
  const double sum =
      d.scale * (((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7])));
  const int row = e >> 4, col = e & 15;
  PR_GLOBAL double* out = gptr(d.out);
  if (NB == 0) {
    out[(long long)(ta * 16 + row) * d.ld + tb * 16 + col] = sum;
    if (ta != tb) out[(long long)(tb * 16 + col) * d.ld + ta * 16 + row] = sum;
  } else {
    out[(long long)(ta * 16 + row) * d.ld + (tb - NA) * 16 + col] = sum;
  }
}

template <int NA, int NB>
static void launch_gemm_shape(const GemmDesc* d, int nd, long long total_wg, bool f32,
                              hipStream_t s) {
  if (f32)
    hipLaunchKernelGGL((k_gemm_tn<NA, NB, true>), dim3((unsigned)total_wg), dim3(256), 0, s, d, nd);
  else
    hipLaunchKernelGGL((k_gemm_tn<NA, NB, false>), dim3((unsigned)total_wg), dim3(256), 0, s, d,
                       nd);
}

template <int NA, int NB>
static void launch_reduce_shape(const GemmDesc* d, int nd, hipStream_t s) {
  hipLaunchKernelGGL((k_gemm_reduce<NA, NB>), dim3(PairList<NA, NB>::P * 16, nd), dim3(256), 0, s,
                     d);
}

// Symmetric Grams of 1..4 tiles; A^T B for the Galerkin products (A: the
// basis, 1 or 2 tiles; B: the packed blocks, at most 5 tiles beside one A
// tile and 3..9 beside two)
#define PR_GEMM_SHAPES(X) \
  X(1, 0) X(2, 0) X(3, 0) X(4, 0) X(1, 1) X(1, 2) X(1, 3) X(1, 4) X(1, 5) \
  X(2, 3) X(2, 4) X(2, 5) X(2, 6) X(2, 7) X(2, 8) X(2, 9)

void launch_gemm_tn(const GemmDesc* d, int nd, long long total_wg, int na, int nb, bool f32,
                    hipStream_t s) {
  if (total_wg <= 0) return;
#define X(A, B)                                             \
  if (na == A && nb == B) {                                 \
    launch_gemm_shape<A, B>(d, nd, total_wg, f32, s);       \
    PR_HIP(hipGetLastError());                              \
    return;                                                 \
  }
  PR_GEMM_SHAPES(X)
#undef X
  fail(PR_EINVAL, "unsupported Gram shape");
}

void launch_gemm_reduce(const GemmDesc* d, int nd, int na, int nb, hipStream_t s) {
  if (nd <= 0) return;
#define X(A, B)                                  \
  if (na == A && nb == B) {                      \
    launch_reduce_shape<A, B>(d, nd, s);         \
    PR_HIP(hipGetLastError());                   \
    return;                                      \
  }
  PR_GEMM_SHAPES(X)
#undef X
  fail(PR_EINVAL, "unsupported Gram shape");
}

// ---------------------------------------------------------------------------
// out[:, j] = alpha * sum_c in_c * C[c][j] (+ add for j = 0); j < nout, and
// columns j >= *out_mptr are zero (with skip_tail: not written). Rows are
// private to a thread, so the output may alias the input columns (all reads
// of a row precede its writes).
// The valid input columns (validity may depend on a device rank) are
// compacted into LDS with their rows of C, once per workgroup, so the
// products run over valid inputs and outputs j < *out_mptr only; each thread
// owns two rows.
constexpr int kTsmmMaxOut = 32;
constexpr int kTsmmMaxIn = 64;
constexpr int kTsmmRowsPerWg = 512;

// MAXOUT bounds the outputs formed (the accumulators held per thread): a
// narrow product (a low-rank basis) then runs at far higher occupancy, which
// is what hides this kernel's memory latency.
template <int MAXOUT>
__global__ __launch_bounds__(256) void k_tsmm(const TsmmDesc* __restrict__ descs, int nd) {
  __shared__ const void* sp[kTsmmMaxIn];
  __shared__ int sf[kTsmmMaxIn];
  __shared__ int so[kTsmmMaxIn];
  __shared__ double sC[kTsmmMaxIn * MAXOUT];
  __shared__ int s_mo, s_nv;
  const long long w = blockIdx.x;
  const int f = find_wg(descs, nd, w);
  const TsmmDesc& d = descs[f];
  const int nin = d.nin, nout = d.nout;
  if (threadIdx.x < 64) {
    // compact the valid inputs (nin <= 64: one wave)
    const int c = threadIdx.x;
    ColDesc cd{};
    const bool v = c < nin && col_valid(cd = d.in[c]);
    const unsigned long long mask = __ballot(v);
    const int p = __popcll(mask & ((1ull << c) - 1ull));
    if (v) {
      sp[p] = cd.ptr;
      sf[p] = cd.f32;
      so[p] = c;
    }
    if (c == 0) {
      s_nv = __popcll(mask);
      s_mo = min(d.out_mptr ? min(*d.out_mptr, nout) : nout, MAXOUT);
    }
  }
  __syncthreads();
  const int nv = s_nv;
  // outputs j >= mo are zero (or left alone): no products for them
  const int mo = s_mo;
  for (int e = threadIdx.x; e < nv * mo; e += 256) {
    const int k = e / mo, j = e - k * mo;
    sC[k * MAXOUT + j] = gptr(d.C)[(long long)so[k] * d.ldc + j];
  }
  __syncthreads();
  const long long r0 = (w - d.wg_begin) * kTsmmRowsPerWg + threadIdx.x;
  const long long r1 = r0 + 256;
  const bool v0 = r0 < d.nrows, v1 = r1 < d.nrows;
  if (!v0) return;
  const long long q1 = v1 ? r1 : r0;
  double a0[MAXOUT], a1[MAXOUT];
#pragma unroll
  for (int j = 0; j < MAXOUT; ++j) a0[j] = a1[j] = 0.0;
  // wide outputs (few waves resident): four input columns per round, their
  // loads issued together before the multiply-adds, so a wave waits for
  // memory once per round; narrow ones already hide the latency with
  // occupancy
  auto ld = [&](int c, long long r) -> double {
    if (sf[c]) return (double)gptr((const float*)sp[c])[r];
    return gptr((const double*)sp[c])[r];
  };
  int c = 0;
  for (; MAXOUT > 8 && c + 4 <= nv; c += 4) {
    double x0[4], x1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x0[u] = ld(c + u, r0);
      x1[u] = ld(c + u, q1);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double* Cr = sC + (c + u) * MAXOUT;
#pragma unroll
      for (int j = 0; j < MAXOUT; ++j)
        if (j < mo) {
          a0[j] += x0[u] * Cr[j];
          a1[j] += x1[u] * Cr[j];
        }
    }
  }
  for (; c < nv; ++c) {
    const double x0 = ld(c, r0), x1 = ld(c, q1);
    const double* Cr = sC + c * MAXOUT;
#pragma unroll
    for (int j = 0; j < MAXOUT; ++j)
      if (j < mo) {
        a0[j] += x0 * Cr[j];
        a1[j] += x1 * Cr[j];
      }
  }
  const int nw = d.skip_tail ? mo : nout;
  const PR_GLOBAL double* add = d.add ? gptr(d.add) : nullptr;
  const double ad0 = add ? add[r0] : 0.0, ad1 = add ? add[q1] : 0.0;
#pragma unroll
  for (int j = 0; j < MAXOUT; ++j) {
    if (j < nw) {
      double y0 = (j < mo) ? d.alpha * a0[j] : 0.0;
      double y1 = (j < mo) ? d.alpha * a1[j] : 0.0;
      if (j == 0) {
        y0 += ad0;
        y1 += ad1;
      }
      if (d.out_f32) {
        PR_GLOBAL float* o = gptr((float*)d.out) + (long long)j * d.out_ld;
        o[r0] = (float)y0;
        if (v1) o[r1] = (float)y1;
      } else {
        PR_GLOBAL double* o = gptr((double*)d.out) + (long long)j * d.out_ld;
        o[r0] = y0;
        if (v1) o[r1] = y1;
      }
    }
  }
}

void launch_tsmm(const TsmmDesc* d, int nd, long long total_wg, int max_nout, hipStream_t s) {
  if (total_wg <= 0) return;
  PR_CHECK(max_nout >= 1 && max_nout <= kTsmmMaxOut, "tsmm: 1..32 outputs");
  const dim3 g((unsigned)total_wg), b(256);
  if (max_nout <= 1) hipLaunchKernelGGL(k_tsmm<1>, g, b, 0, s, d, nd);
  else if (max_nout <= 8) hipLaunchKernelGGL(k_tsmm<8>, g, b, 0, s, d, nd);
  else if (max_nout <= 16) hipLaunchKernelGGL(k_tsmm<16>, g, b, 0, s, d, nd);
  else if (max_nout <= 24) hipLaunchKernelGGL(k_tsmm<24>, g, b, 0, s, d, nd);
  else hipLaunchKernelGGL(k_tsmm<32>, g, b, 0, s, d, nd);
  PR_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Parareal correction with jump partials.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(256) void k_correct(const CorrectDesc* __restrict__ descs, int nd) {
  __shared__ double red[4][4];
  __shared__ const void* sp[kTsmmMaxOut + 1];
  __shared__ int sf[kTsmmMaxOut + 1];
  __shared__ double sc[kTsmmMaxOut + 1];
  __shared__ int s_np;
  const long long w = blockIdx.x;
  const int f = find_wg(descs, nd, w);
  const CorrectDesc& d = descs[f];
  if (threadIdx.x == 0) {
    // compact the valid basis columns (their coefficients are read once)
    int k = 0;
    for (int c = 0; c < d.npsi; ++c) {
      const ColDesc cd = d.psi[c];
      if (!col_valid(cd)) continue;
      sp[k] = cd.ptr;
      sf[k] = cd.f32;
      sc[k] = d.coef[c];
      ++k;
    }
    s_np = k;
  }
  __syncthreads();
  const int np = s_np;
  const long long wl = w - d.wg_begin;
  const long long rows_per_wg = (d.nrows + d.nwg - 1) / d.nwg;
  const long long r0 = wl * rows_per_wg;
  const long long r1 = min(d.nrows, r0 + rows_per_wg);
  const PR_GLOBAL double* prev = d.prev ? gptr(d.prev) : nullptr;
  const PR_GLOBAL double* ref = d.ref ? gptr(d.ref) : nullptr;
  PR_GLOBAL double* out = gptr(d.out);
  double s_jump = 0, s_u = 0, s_err = 0, s_ref = 0;
  auto col = [&](int c, long long row) {
    return sf[c] ? (double)gptr((const float*)sp[c])[row] : gptr((const double*)sp[c])[row];
  };
  for (long long row = r0 + threadIdx.x; row < r1; row += 256) {
    // every load of the row is issued before the sums that use it (out,
    // prev and ref are distinct buffers); the sums keep their order
    double v = 0.0;
    if (d.fine) v = d.fine_f32 ? (double)gptr((const float*)d.fine)[row] : gptr((const double*)d.fine)[row];
    const double pv = prev ? prev[row] : 0.0;
    const double r = ref ? ref[row] : 0.0;
    double g = 0.0;
    int c = 0;
    for (; c + 4 <= np; c += 4) {
      double x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = col(c + u, row);
#pragma unroll
      for (int u = 0; u < 4; ++u) g += sc[c + u] * x[u];
    }
    for (; c < np; ++c) g += sc[c] * col(c, row);
    v += g;
    out[row] = v;
    s_u += v * v;
    if (prev) {
      const double dj = v - pv;
      s_jump += dj * dj;
    }
    if (ref) {
      const double de = v - r;
      s_err += de * de;
      s_ref += r * r;
    }
  }
  s_jump = wave_sum(s_jump);
  s_u = wave_sum(s_u);
  s_err = wave_sum(s_err);
  s_ref = wave_sum(s_ref);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[wave][0] = s_jump;
    red[wave][1] = s_u;
    red[wave][2] = s_err;
    red[wave][3] = s_ref;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int i = threadIdx.x;
    gptr(d.partial)[wl * 4 + i] = (red[0][i] + red[1][i]) + (red[2][i] + red[3][i]);
  }
}

void launch_correct(const CorrectDesc* d, int nd, long long total_wg, hipStream_t s) {
  if (total_wg <= 0) return;
  hipLaunchKernelGGL(k_correct, dim3((unsigned)total_wg), dim3(256), 0, s, d, nd);
  PR_HIP(hipGetLastError());
}

// Per item (one workgroup each): out[0..4) = scale * fixed-order sums of
// partial[nwg][4] (strided per thread, each wave's butterfly, then the four
// waves in order). The partials are 32-byte aligned rows of four.
__global__ __launch_bounds__(256) void k_norm_reduce(const NormReduceDesc* __restrict__ descs) {
  __shared__ double red[4][4];
  const NormReduceDesc& d = descs[blockIdx.x];
  const PR_GLOBAL v2d_t* part = (const PR_GLOBAL v2d_t*)gptr(d.partial);
  double s[4] = {0, 0, 0, 0};
#pragma unroll 4
  for (int w = threadIdx.x; w < d.nwg; w += 256) {
    const v2d_t a = part[2 * w], b = part[2 * w + 1];
    s[0] += a.x;
    s[1] += a.y;
    s[2] += b.x;
    s[3] += b.y;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) s[i] = wave_sum(s[i]);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < 4; ++i) red[wave][i] = s[i];
  __syncthreads();
  if (threadIdx.x < 4) {
    const int i = threadIdx.x;
    d.out[i] = d.scale * ((red[0][i] + red[1][i]) + (red[2][i] + red[3][i]));
  }
}

void launch_norm_reduce(const NormReduceDesc* d, int nd, hipStream_t s) {
  if (nd <= 0) return;
  hipLaunchKernelGGL(k_norm_reduce, dim3(nd), dim3(256), 0, s, d);
  PR_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Gram-Schmidt pass of the augmentation (CgsArgs). Thread t of workgroup b
// owns rows b * chunk_rows + t + 256 i; its column loads are coalesced across
// the wave. Columns j >= m are read from column 0 (a finite value, in
// bounds) and replaced by zero, so the loads of a row are branch-free and
// issued together.
template <int MAXC, bool DOTS, bool SUB, typename In>
__global__ __launch_bounds__(256) void k_cgs(const CgsArgs a) {
  __shared__ double red[4][MAXC + 1];
  const int n = a.n;
  const int m = a.mptr ? min(*a.mptr, n) : n;
  const long long r_begin = (long long)blockIdx.x * a.chunk_rows;
  const long long r_end = min(a.nrows, r_begin + (long long)a.chunk_rows);
  const PR_GLOBAL In* p[MAXC];
  double cj[MAXC];
#pragma unroll
  for (int j = 0; j < MAXC; ++j) {
    p[j] = gptr((const In*)a.col[j < m ? j : 0]);
    cj[j] = (SUB && j < m) ? a.c[j] : 0.0;
  }
  double acc[MAXC + 1];
#pragma unroll
  for (int j = 0; j <= MAXC; ++j) acc[j] = 0.0;
  const PR_GLOBAL double* y = gptr(a.y);
  PR_GLOBAL double* z = a.z ? gptr(a.z) : nullptr;
  for (long long r = r_begin + threadIdx.x; r < r_end; r += 256) {
    double x[MAXC];
    if (m > 0) {
      if constexpr (!SUB) {
        // the dots pass loads no column j >= m (m is uniform: whole-wave
        // branches); 63 -> 56 us per call at 128^3. The update passes lost
        // 1-2 us that way and load all MAXC columns in one block.
#pragma unroll
        for (int j = 0; j < MAXC; ++j) x[j] = j < m ? (double)p[j][r] : 0.0;
      } else {
#pragma unroll
        for (int j = 0; j < MAXC; ++j) {
          const double v = (double)p[j][r];
          x[j] = j < m ? v : 0.0;
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < MAXC; ++j) x[j] = 0.0;
    }
    double v = y[r];
    if constexpr (SUB) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < MAXC; ++j) s += cj[j] * x[j];
      v -= s;
    }
    if (z) z[r] = v;
    if constexpr (DOTS) {
#pragma unroll
      for (int j = 0; j < MAXC; ++j) acc[j] += x[j] * v;
    }
    acc[MAXC] += v * v;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j <= MAXC; ++j) {
    if (!DOTS && j < MAXC) continue;
    const double s = wave_sum(acc[j]);
    if (lane == 0) red[wave][j] = s;
  }
  __syncthreads();
  PR_GLOBAL double* part = gptr(a.partial) + (long long)blockIdx.x * (n + 1);
  const int t = threadIdx.x;
  if (t <= n) {
    const int k = (t == n) ? MAXC : t;
    double s = 0.0;
    if (t == n || (DOTS && t < m)) s = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
    part[t] = s;
  }
}

// Per output j <= n (one workgroup each): scale * the chunk partials summed
// in a fixed order (strided per thread, each wave's butterfly, then the four
// waves in order).
__global__ __launch_bounds__(256) void k_cgs_reduce(const CgsArgs a) {
  __shared__ double red[4];
  const int j = blockIdx.x == 0 ? a.n : (int)blockIdx.x - 1;
  const PR_GLOBAL double* part = gptr(a.partial);
  double s = 0.0;
#pragma unroll 4
  for (int q = threadIdx.x; q < a.nchunks; q += 256) s += part[(long long)q * (a.n + 1) + j];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    s = (red[0] + red[1]) + (red[2] + red[3]);
    if (j == a.n) {
      const double nd2 = a.scale * s;
      *gptr(a.norm) = nd2;
      if (a.flag) {
        // the degenerate-augmentation test (||d~|| <= tau ||u||), squared
        const double nu2 = *gptr(a.nu2);
        const int flag = (nd2 > 0.0 && nd2 > kTauAug * kTauAug * nu2) ? 1 : 0;
        *gptr(a.flag) = flag;
        *gptr(a.dscale) = flag ? 1.0 / sqrt(nd2) : 0.0;
      }
    } else {
      gptr(a.dots)[j] = a.scale * s;
    }
  }
}

int cgs_chunk_rows(long long nrows) {
  long long ch = (nrows + 1023) / 1024;
  ch = std::max<long long>(ch, 1024);
  return (int)((ch + 255) / 256 * 256);
}

template <int MAXC, bool DOTS, bool SUB>
static void cgs_launch(const CgsArgs& a, hipStream_t s) {
  const dim3 g((unsigned)a.nchunks), b(256);
  if (a.f32) hipLaunchKernelGGL((k_cgs<MAXC, DOTS, SUB, float>), g, b, 0, s, a);
  else hipLaunchKernelGGL((k_cgs<MAXC, DOTS, SUB, double>), g, b, 0, s, a);
}

template <bool DOTS, bool SUB>
static void cgs_width(const CgsArgs& a, hipStream_t s) {
  // the column count rounded up to a multiple of 4 (few padding loads)
  switch ((a.n + 3) / 4) {
    case 0:
    case 1: cgs_launch<4, DOTS, SUB>(a, s); break;
    case 2: cgs_launch<8, DOTS, SUB>(a, s); break;
    case 3: cgs_launch<12, DOTS, SUB>(a, s); break;
    case 4: cgs_launch<16, DOTS, SUB>(a, s); break;
    case 5: cgs_launch<20, DOTS, SUB>(a, s); break;
    case 6: cgs_launch<24, DOTS, SUB>(a, s); break;
    case 7: cgs_launch<28, DOTS, SUB>(a, s); break;
    default: cgs_launch<32, DOTS, SUB>(a, s); break;
  }
}

void launch_cgs(const CgsArgs& a, hipStream_t s) {
  PR_CHECK(a.n >= 0 && a.n <= kCgsMaxCols, "cgs: 0..32 columns");
  PR_CHECK(a.y && a.partial && a.norm, "cgs: null vector");
  PR_CHECK(a.chunk_rows % 256 == 0 && a.chunk_rows > 0, "cgs: chunk rows");
  PR_CHECK(a.nchunks == (int)((a.nrows + a.chunk_rows - 1) / a.chunk_rows), "cgs: chunk count");
  for (int j = 0; j < a.n; ++j) PR_CHECK(a.col[j] != nullptr, "cgs: null column");
  if (a.nchunks <= 0) return;
  const bool dots = a.dots != nullptr, sub = a.c != nullptr;
  PR_CHECK(dots || sub, "cgs: a pass without coefficients returns the dots");
  PR_CHECK(!a.flag || (a.nu2 && a.dscale), "cgs: the augmentation decision needs nu2 and dscale");
  if (dots && sub) cgs_width<true, true>(a, s);
  else if (dots) cgs_width<true, false>(a, s);
  else cgs_width<false, true>(a, s);
  PR_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_cgs_reduce, dim3(dots ? a.n + 1 : 1), dim3(256), 0, s, a);
  PR_HIP(hipGetLastError());
}

// out[0] = max_i sqrt(n[i][0] / n[i][1]) (jump), out[1] = max_i
// sqrt(n[i][2] / n[i][3]) (error). A NaN in any of an item's norms (a NaN
// or Inf in the iterate, the previous iterate or the reference) makes the
// corresponding output NaN; fmax alone would drop it.
__global__ void k_jump_max(const double* __restrict__ n4, int count, double* out) {
  if (threadIdx.x != 0) return;
  double e = 0.0, r = 0.0;
  bool bad = false, bad_r = false;
  for (int i = 0; i < count; ++i) {
    const double j = n4[4 * i + 0], u = n4[4 * i + 1];
    const double ee = n4[4 * i + 2], rr = n4[4 * i + 3];
    if (j != j || u != u) bad = true;
    if (ee != ee || rr != rr) bad_r = true;
    const double q = (u > 0) ? sqrt(j / u) : (j > 0 ? INFINITY : 0.0);
    if (q != q) bad = true;
    e = fmax(e, q);
    const double qe = (rr > 0) ? sqrt(ee / rr) : 0.0;
    if (qe != qe) bad_r = true;
    r = fmax(r, qe);
  }
  out[0] = bad ? NAN : e;
  out[1] = bad_r ? NAN : r;
}

void launch_jump_max(const double* norms4, int count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_jump_max, dim3(1), dim3(64), 0, s, norms4, count, out);
  PR_HIP(hipGetLastError());
}

}  // namespace pr
