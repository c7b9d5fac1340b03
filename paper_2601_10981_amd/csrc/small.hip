// Small dense FP64 kernels, one workgroup per matrix:
//   * eigen-decomposition of the POD Gram (Algorithm 1, step 1) by cyclic
//     two-sided Jacobi in round-robin pair order (all N/2 disjoint rotations of
//     a round applied together), descending sort, sign normalisation, the
//     numerical rank and the sqrt(lambda) criterion (Algorithm 1, step 2) and
//     the mode coefficients Y_m Lambda_m^{-1/2} (r_i = W y_i / sqrt(lambda_i));
//   * Cholesky of the modes' Gram for CholQR re-orthonormalisation;
//   * the reduced Galerkin system M_r beta' = L_r beta (eq. 8 / eq13) solved
//     by RK4 with the step-doubling stability guard.
#include "pr_internal.h"

namespace pr {

constexpr int kMaxN = 64;
constexpr int kMaxSweeps = 40;
constexpr double kJacobiRel = 1e-15;
// A rotation is also skipped when |a_pq| is at the rounding level of the whole
// matrix (unit roundoff times its trace, the sum of the eigenvalues of the
// PSD Gram). With the relative test alone, pairs of eigenvalues near the
// bottom of a fast-decaying spectrum keep rotating on rounding noise until
// the sweep limit; their eigenvectors are no better resolved by it.
constexpr double kJacobiAbs = 0x1p-53;

__global__ __launch_bounds__(256) void k_eig_select(const EigDesc* __restrict__ descs) {
  const EigDesc d = descs[blockIdx.x];
  __shared__ double A[kMaxN][kMaxN + 1];
  __shared__ double V[kMaxN][kMaxN + 1];
  __shared__ double cs[kMaxN / 2], sn[kMaxN / 2];
  __shared__ int pp[kMaxN / 2], qq[kMaxN / 2];
  __shared__ int rotated;
  __shared__ double lam[kMaxN];
  __shared__ int order[kMaxN];
  __shared__ double sgn[kMaxN];
  __shared__ int m_sh;
  // rows with an exactly zero diagonal (masked columns: a PSD Gram's zero
  // diagonal means a zero row) hold eigenvalue 0 with eigenvector e_i; the
  // rotations run on the other rows only, compacted (kid: compact ->
  // original, kpos: original -> compact or -1)
  __shared__ int kid[kMaxN], kpos[kMaxN];
  __shared__ int nk_sh;
  __shared__ double trace_sh;
  const int tid = threadIdx.x;
  const int nc = d.nc;
  if (tid < 64) {
    const bool v = tid < nc && d.G[(long long)tid * d.ldg + tid] != 0.0;
    const unsigned long long mask = __ballot(v);
    const int p = __popcll(mask & ((1ull << tid) - 1ull));
    if (v) kid[p] = tid;
    if (tid < nc) kpos[tid] = v ? p : -1;
    if (tid == 0) nk_sh = __popcll(mask);
  }
  __syncthreads();
  const int nk = nk_sh;
  const int N = nk + (nk & 1);
  for (int e = tid; e < N * N; e += 256) {
    const int i = e / N, j = e % N;
    A[i][j] = (i < nk && j < nk) ? d.G[(long long)kid[i] * d.ldg + kid[j]] : 0.0;
    V[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    double tr = 0.0;
    for (int i = 0; i < nk; ++i) tr += A[i][i];
    trace_sh = tr;
  }
  __syncthreads();
  const double floor_abs = kJacobiAbs * trace_sh;
  const int half = N / 2;
  // this thread's (pair, column) slots of a round's updates: the same in every
  // round, so their index arithmetic stays out of the rotation loop
  constexpr int kSlots = (kMaxN / 2 * kMaxN + 255) / 256;
  int slot_i[kSlots], slot_k[kSlots];
#pragma unroll
  for (int r = 0; r < kSlots; ++r) {
    const int e = tid + 256 * r;
    slot_i[r] = e < half * N ? e / N : -1;
    slot_k[r] = e < half * N ? e % N : 0;
  }
  for (int sweep = 0; sweep < kMaxSweeps && N >= 2; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < N - 1; ++r) {
      if (tid < half) {
        // round-robin tournament: position 0 fixed, the others rotate
        const int a = (tid == 0) ? 0 : 1 + (tid - 1 + r) % (N - 1);
        const int b = 1 + (N - 2 - tid + r) % (N - 1);
        const int p = min(a, b), q = max(a, b);
        const double apq = A[p][q], app = A[p][p], aqq = A[q][q];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > 1e-300 && fabs(apq) > kJacobiRel * sqrt(fabs(app * aqq)) &&
            fabs(apq) > floor_abs) {
          const double tau = (aqq - app) / (2.0 * apq);
          double t;
          if (fabs(tau) > 1e150) t = 0.5 / tau;
          else t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
          rotated = 1;
        }
        cs[tid] = c;
        sn[tid] = s;
        pp[tid] = p;
        qq[tid] = q;
      }
      __syncthreads();
#pragma unroll
      for (int r2 = 0; r2 < kSlots; ++r2) {
        const int i = slot_i[r2], k = slot_k[r2];
        if (i < 0) break;
        const double s = sn[i];
        if (s == 0.0) continue;
        const double c = cs[i];
        const int p = pp[i], q = qq[i];
        const double apk = A[p][k], aqk = A[q][k];
        A[p][k] = c * apk - s * aqk;
        A[q][k] = s * apk + c * aqk;
      }
      __syncthreads();
#pragma unroll
      for (int r2 = 0; r2 < kSlots; ++r2) {
        const int i = slot_i[r2], k = slot_k[r2];
        if (i < 0) break;
        const double s = sn[i];
        if (s == 0.0) continue;
        const double c = cs[i];
        const int p = pp[i], q = qq[i];
        const double akp = A[k][p], akq = A[k][q];
        A[k][p] = c * akp - s * akq;
        A[k][q] = s * akp + c * akq;
        const double vkp = V[k][p], vkq = V[k][q];
        V[k][p] = c * vkp - s * vkq;
        V[k][q] = s * vkp + c * vkq;
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  // descending order over all nc (original) indices, ties by index. The sort
  // key orders a NaN below everything, so the ranks stay a permutation (and
  // every index read through `order` stays in range) whatever the data.
  auto val = [&](int i) -> double { const int p = kpos[i]; return p >= 0 ? A[p][p] : 0.0; };
  auto key = [&](int i) -> double { const double v = val(i); return v == v ? v : -INFINITY; };
  if (tid < nc) {
    const double li = key(tid);
    int rank = 0;
    for (int j = 0; j < nc; ++j) {
      const double lj = key(j);
      if (lj > li || (lj == li && j < tid)) ++rank;
    }
    order[rank] = tid;
  }
  __syncthreads();
  if (tid < nc) {
    const int col = order[tid];
    const int pc = kpos[col];
    lam[tid] = val(col);
    double sg = 1.0;
    if (pc >= 0) {
      // kid is increasing: the lowest compact index is the lowest original one
      int kmax = 0;
      double vmax = -1.0;
      for (int k = 0; k < nk; ++k) {
        const double v = fabs(V[k][pc]);
        if (v > vmax) { vmax = v; kmax = k; }
      }
      sg = (V[kmax][pc] < 0.0) ? -1.0 : 1.0;
    }
    sgn[tid] = sg;
  }
  __syncthreads();
  if (tid == 0) {
    int m = 0;
    const double l0 = (nc > 0) ? lam[0] : 0.0;
    if (l0 > 0.0) {
      int r = 0;
      while (r < nc && lam[r] > d.tau_r * l0) ++r;
      if (d.force_m >= 0) {
        m = min(d.force_m, r);
      } else {
        double total = 0.0;
        for (int i = 0; i < r; ++i) total += sqrt(lam[i]);
        double acc = 0.0;
        m = r;
        for (int i = 0; i < r; ++i) {
          acc += sqrt(lam[i]);
          if (acc >= d.gamma * total) { m = i + 1; break; }
        }
      }
      m = min(m, d.cap);
    }
    m_sh = m;
    *d.m_out = m;
  }
  __syncthreads();
  const int m = m_sh;
  if (d.lambda)
    for (int i = tid; i < nc; i += 256) d.lambda[i] = lam[i];
  // columns j < m have lam > 0, hence a kept (compact) eigenvector
  for (int e = tid; e < nc * d.ld_coef; e += 256) {
    const int c = e / d.ld_coef, j = e % d.ld_coef;
    double v = 0.0;
    if (j < m && kpos[c] >= 0) v = sgn[j] * V[kpos[c]][kpos[order[j]]] / sqrt(lam[j]);
    d.coef[e] = v;
  }
}

void launch_eig_select(const EigDesc* d, int nd, hipStream_t s) {
  if (nd <= 0) return;
  hipLaunchKernelGGL(k_eig_select, dim3(nd), dim3(256), 0, s, d);
  PR_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Cholesky G = L L^T of the leading m x m block of the modes' Gram; a pivot
// <= kDropPivot drops that column and all later ones (m lowered). Writes
// coef = L^{-T} (upper triangular, zero beyond the new m), so that
// R <- R coef has M-orthonormal columns.
constexpr int kMaxQ = 32;

__global__ __launch_bounds__(256) void k_cholqr_coef(const CholDesc* __restrict__ descs) {
  const CholDesc d = descs[blockIdx.x];
  __shared__ double Lm[kMaxQ][kMaxQ + 1];
  __shared__ double Li[kMaxQ][kMaxQ + 1];
  __shared__ int m_sh;
  const int tid = threadIdx.x;
  const int cap = d.cap;
  if (tid == 0) m_sh = *d.m;
  for (int e = tid; e < kMaxQ * kMaxQ; e += 256) {
    const int i = e / kMaxQ, j = e % kMaxQ;
    Lm[i][j] = (i < cap && j < cap) ? d.G[(long long)i * d.ldg + j] : 0.0;
    Li[i][j] = 0.0;
  }
  __syncthreads();
  const int m0 = m_sh;
  for (int j = 0; j < m0; ++j) {
    // column j of the right-looking factorisation; Lm's lower triangle is
    // overwritten with L, the trailing block with the Schur complement
    if (tid == 0) {
      const double dj = Lm[j][j];
      if (!(dj > kDropPivot) && m_sh > j) m_sh = j;
      if (m_sh > j) Lm[j][j] = sqrt(dj);
    }
    __syncthreads();
    if (m_sh <= j) break;
    const double ljj = Lm[j][j];
    for (int i = j + 1 + tid; i < m0; i += 256) Lm[i][j] /= ljj;
    __syncthreads();
    const int t = m0 - j - 1;
    for (int e = tid; e < t * t; e += 256) {
      const int i = j + 1 + e / t, k = j + 1 + e % t;
      if (k <= i) Lm[i][k] -= Lm[i][j] * Lm[k][j];
    }
    __syncthreads();
  }
  const int m = m_sh;
  // columns of L^{-1} by forward substitution (one column per thread)
  if (tid < m) {
    const int c = tid;
    for (int i = c; i < m; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) s -= Lm[i][k] * Li[k][c];
      Li[i][c] = s / Lm[i][i];
    }
  }
  __syncthreads();
  for (int e = tid; e < cap * cap; e += 256) {
    const int c = e / cap, j = e % cap;
    d.coef[e] = (c < m && j < m && c <= j) ? Li[j][c] : 0.0;
  }
  if (tid == 0) *d.m = m;
}

void launch_cholqr_coef(const CholDesc* d, int nd, hipStream_t s) {
  if (nd <= 0) return;
  hipLaunchKernelGGL(k_cholqr_coef, dim3(nd), dim3(256), 0, s, d);
  PR_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// CholQR factors from the coefficient Gram (CoefGramDesc). One workgroup of
// 256 threads per item.
__global__ __launch_bounds__(256) void k_coef_gram(const CoefGramDesc* __restrict__ descs) {
  const CoefGramDesc& d = descs[blockIdx.x];
  __shared__ double Cs[64][33];
  __shared__ double H[64][33];
  __shared__ int live[64];
  const int nc = d.nc, cap = d.cap, tid = threadIdx.x;
  if (tid < 64) live[tid] = tid < nc && d.G[(long long)tid * d.ldg + tid] != 0.0;
  __syncthreads();
  for (int e = tid; e < nc * cap; e += 256) {
    const int i = e / cap, a = e % cap;
    Cs[i][a] = live[i] ? d.C[(long long)i * d.ldc + a] : 0.0;
  }
  __syncthreads();
  // H = G C (G read from memory: at most 64 x 64, cached)
  for (int e = tid; e < nc * cap; e += 256) {
    const int i = e / cap, a = e % cap;
    double v = 0.0;
    if (live[i]) {
      const double* gi = d.G + (long long)i * d.ldg;
      for (int j = 0; j < nc; ++j)
        if (live[j]) v += gi[j] * Cs[j][a];
    }
    H[i][a] = v;
  }
  __syncthreads();
  // G2 = C^T H
  for (int e = tid; e < cap * cap; e += 256) {
    const int a = e / cap, b = e % cap;
    double v = 0.0;
    for (int i = 0; i < nc; ++i) v += Cs[i][a] * H[i][b];
    d.G2[a * 32 + b] = v;
  }
}

// C <- C U, U upper triangular (cap x cap, leading dimension 32)
__global__ __launch_bounds__(256) void k_coef_apply(const CoefGramDesc* __restrict__ descs) {
  const CoefGramDesc& d = descs[blockIdx.x];
  __shared__ double Cs[64][33];
  const int nc = d.nc, cap = d.cap, tid = threadIdx.x;
  for (int e = tid; e < nc * cap; e += 256) Cs[e / cap][e % cap] = d.C[(long long)(e / cap) * d.ldc + e % cap];
  __syncthreads();
  for (int e = tid; e < nc * cap; e += 256) {
    const int i = e / cap, a = e % cap;
    double v = 0.0;
    for (int b = 0; b <= a; ++b) v += Cs[i][b] * d.U[b * cap + a];
    d.C[(long long)i * d.ldc + a] = v;
  }
}

void launch_coef_gram(const CoefGramDesc* d, int nd, hipStream_t s) {
  if (nd <= 0) return;
  hipLaunchKernelGGL(k_coef_gram, dim3(nd), dim3(256), 0, s, d);
  PR_HIP(hipGetLastError());
}

void launch_coef_apply(const CoefGramDesc* d, int nd, hipStream_t s) {
  if (nd <= 0) return;
  hipLaunchKernelGGL(k_coef_apply, dim3(nd), dim3(256), 0, s, d);
  PR_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Descriptor upload through the kernel arguments.
__global__ __launch_bounds__(256) void k_upload(const UploadBlob b, unsigned int* __restrict__ dst,
                                                int nw) {
  for (int i = threadIdx.x; i < nw; i += 256) dst[i] = b.w[i];
}

void launch_upload(const UploadBlob& b, unsigned int* dst, int nw, hipStream_t s) {
  PR_CHECK(nw > 0 && nw <= kUploadWords, "upload of at most kUploadWords words");
  hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, s, b, dst, nw);
  PR_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Block whitening (WhitenDesc). One workgroup of 64 threads per item.
__global__ __launch_bounds__(64) void k_block_whiten(const WhitenDesc* __restrict__ descs) {
  const WhitenDesc& d = descs[blockIdx.x];
  __shared__ double A[kWhitenMaxCols][kWhitenMaxCols + 1];
  __shared__ double Ts[kWhitenMaxCols * 32];
  __shared__ int mb[kWhitenMaxCols];
  const int tid = threadIdx.x;
  const int nb = d.nb, bs = d.bs, nc = nb * bs;
  for (int e = tid; e < nc * nc; e += 64) A[e / nc][e % nc] = d.G[(long long)(e / nc) * d.ldg + e % nc];
  if (tid < nb) mb[tid] = d.m[tid] ? min(*d.m[tid], bs) : bs;
  __syncthreads();
  // Cholesky of each diagonal block, one thread per block (rows in order)
  if (tid < nb) {
    const int o = tid * bs;
    double* T = Ts + tid * bs * bs;
    int m = mb[tid];
    for (int j = 0; j < m; ++j) {
      double dj = A[o + j][o + j];
      for (int k = 0; k < j; ++k) dj -= T[k * bs + j] * T[k * bs + j];
      if (!(dj > kDropPivot)) {
        m = j;
        break;
      }
      const double tjj = sqrt(dj);
      T[j * bs + j] = tjj;
      for (int i = j + 1; i < m; ++i) {
        double v = A[o + j][o + i];
        for (int k = 0; k < j; ++k) v -= T[k * bs + j] * T[k * bs + i];
        T[j * bs + i] = v / tjj;
      }
    }
    mb[tid] = m;
  }
  __syncthreads();
  // left: column c of each block row b <- T_b^{-T} (forward substitution);
  // rows beyond the kept columns become zero
  if (tid < nc) {
    const int c = tid;
    for (int b = 0; b < nb; ++b) {
      const int o = b * bs, m = mb[b];
      const double* T = Ts + b * bs * bs;
      for (int i = 0; i < bs; ++i) {
        if (i >= m) {
          A[o + i][c] = 0.0;
          continue;
        }
        double v = A[o + i][c];
        for (int k = 0; k < i; ++k) v -= T[k * bs + i] * A[o + k][c];
        A[o + i][c] = v / T[i * bs + i];
      }
    }
  }
  __syncthreads();
  // right: row r of each block column b <- (.) T_b^{-1}
  if (tid < nc) {
    const int r = tid;
    for (int b = 0; b < nb; ++b) {
      const int o = b * bs, m = mb[b];
      const double* T = Ts + b * bs * bs;
      for (int i = 0; i < bs; ++i) {
        if (i >= m) {
          A[r][o + i] = 0.0;
          continue;
        }
        double v = A[r][o + i];
        for (int k = 0; k < i; ++k) v -= A[r][o + k] * T[k * bs + i];
        A[r][o + i] = v / T[i * bs + i];
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < nc * nc; e += 64) d.G[(long long)(e / nc) * d.ldg + e % nc] = A[e / nc][e % nc];
  for (int e = tid; e < nb * bs * bs; e += 64) d.T[e] = Ts[e];
  if (tid < nb) d.meff[tid] = mb[tid];
}

// coef rows of block b <- T_b^{-1} (back substitution), one thread per column
__global__ __launch_bounds__(64) void k_block_unwhiten(const WhitenDesc* __restrict__ descs) {
  const WhitenDesc& d = descs[blockIdx.x];
  const int nb = d.nb, bs = d.bs;
  for (int j = threadIdx.x; j < d.ncoef; j += 64) {
    for (int b = 0; b < nb; ++b) {
      const int o = b * bs, m = d.meff[b];
      const double* T = d.T + b * bs * bs;
      for (int i = m - 1; i >= 0; --i) {
        double v = d.coef[(long long)(o + i) * d.ld_coef + j];
        for (int k = i + 1; k < m; ++k) v -= T[i * bs + k] * d.coef[(long long)(o + k) * d.ld_coef + j];
        d.coef[(long long)(o + i) * d.ld_coef + j] = v / T[i * bs + i];
      }
      for (int i = m; i < bs; ++i) d.coef[(long long)(o + i) * d.ld_coef + j] = 0.0;
    }
  }
}

void launch_block_whiten(const WhitenDesc* d, int nd, hipStream_t s) {
  if (nd <= 0) return;
  hipLaunchKernelGGL(k_block_whiten, dim3(nd), dim3(64), 0, s, d);
  PR_HIP(hipGetLastError());
}

void launch_block_unwhiten(const WhitenDesc* d, int nd, hipStream_t s) {
  if (nd <= 0) return;
  hipLaunchKernelGGL(k_block_unwhiten, dim3(nd), dim3(64), 0, s, d);
  PR_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Reduced system helpers shared by the sweep and the k = 0 recurrence.
struct RedShared {
  double M[kMaxQ + 1][kMaxQ + 2];
  double K[kMaxQ + 1][kMaxQ + 2];
  double B[kMaxQ + 1][kMaxQ + 2];
  double T[kMaxQ + 1][kMaxQ + 2];
  double beta[2][kMaxQ + 1];
  double tmp[2][kMaxQ + 1];
  // forced flows: g_j = M_r^{-1} f_r,j and the RK4 stage vectors
  double g[kMaxPieces][kMaxQ + 1];
  double y[2][kMaxQ + 1];
  double kv[2][kMaxQ + 1];
  double acc[2][kMaxQ + 1];
  int idx[kMaxQ + 1];
  double red[256];
  int q, n_c, bad;
};

// This thread's entries (row, column) of a q x q reduced system, e = tid +
// 256 r for r < 4 (q <= 32): fixed for a kernel, so the loops over the
// system's entries do no index division.
struct QSlots {
  int i[4], j[4];
};
static_assert(kMaxQ * kMaxQ <= 4 * 256, "four entries per thread cover the largest system");
__device__ __forceinline__ QSlots q_slots(int q) {
  QSlots sl;
  const int tid = threadIdx.x;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int e = tid + 256 * r;
    sl.i[r] = e < q * q ? e / q : -1;
    sl.j[r] = e < q * q ? e % q : 0;
  }
  return sl;
}

// Cholesky in place of sh.M (q x q, lower); sets bad on a non-positive (or
// NaN) pivot, which is then clamped only so the factorisation completes: the
// callers turn bad into NaN coefficients. Right-looking elimination on the
// unscaled pivot column (one barrier per column: after step j - 1, column j
// and its pivot are final), then one pass scales the columns by the square
// roots of their pivots.
__device__ void red_cholesky(RedShared& sh, int q, const QSlots& sl) {
  const int tid = threadIdx.x;
  for (int j = 0; j < q; ++j) {
    const double inv = 1.0 / fmax(sh.M[j][j], 1e-300);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = sl.i[r], k = sl.j[r];
      if (i < 0) break;
      if (k > j && k <= i) sh.M[i][k] -= (sh.M[i][j] * inv) * sh.M[k][j];
    }
    __syncthreads();
  }
  if (tid < q) {
    const double dj = sh.M[tid][tid];
    if (!(dj > 0.0)) sh.bad = 1;
    sh.tmp[0][tid] = sqrt(fmax(dj, 1e-300));
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = sl.i[r], k = sl.j[r];
    if (i < 0) break;
    if (k < i) sh.M[i][k] /= sh.tmp[0][k];
    else if (k == i) sh.M[i][i] = sh.tmp[0][i];
  }
  __syncthreads();
}

// Solve (L L^T) x = b in place for a vector held by one thread.
__device__ void red_solve(const RedShared& sh, int q, double* x, int stride) {
  for (int i = 0; i < q; ++i) {
    double s = x[i * stride];
    for (int k = 0; k < i; ++k) s -= sh.M[i][k] * x[k * stride];
    x[i * stride] = s / sh.M[i][i];
  }
  for (int i = q - 1; i >= 0; --i) {
    double s = x[i * stride];
    for (int k = i + 1; k < q; ++k) s -= sh.M[k][i] * x[k * stride];
    x[i * stride] = s / sh.M[i][i];
  }
}

// Given sh.M (Cholesky factor) and sh.K holding L_r, turn sh.K into
// M_r^{-1} L_r, apply the guard and form sh.B = P4(h K) by Horner.
__device__ void red_propagator(RedShared& sh, int q, double dT, int n_c0, const QSlots& sl) {
  const int tid = threadIdx.x;
  if (tid < q) red_solve(sh, q, &sh.K[0][tid], kMaxQ + 2);
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (sl.i[r] < 0) break;
    const double v = sh.K[sl.i[r]][sl.j[r]];
    s += v * v;
  }
  sh.red[tid] = s;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int i = 0; i < 256; ++i) t += sh.red[i];
    const double nrm = sqrt(t);
    int n_c = max(1, n_c0);
    while ((dT / n_c) * nrm > kGuard && n_c < (1 << 16)) n_c *= 2;
    sh.n_c = n_c;
  }
  __syncthreads();
  const double h = dT / sh.n_c;
  // B = I + (h/4) K
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = sl.i[r], j = sl.j[r];
    if (i < 0) break;
    sh.B[i][j] = (i == j ? 1.0 : 0.0) + 0.25 * h * sh.K[i][j];
  }
  __syncthreads();
  const double cf[3] = {h / 3.0, h / 2.0, h};
  for (int st = 0; st < 3; ++st) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = sl.i[r], j = sl.j[r];
      if (i < 0) break;
      double acc = 0.0;
      for (int k = 0; k < q; ++k) acc += sh.K[i][k] * sh.B[k][j];
      sh.T[i][j] = (i == j ? 1.0 : 0.0) + cf[st] * acc;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (sl.i[r] < 0) break;
      sh.B[sl.i[r]][sl.j[r]] = sh.T[sl.i[r]][sl.j[r]];
    }
    __syncthreads();
  }
}

// Forced flows: the pieces K_j = M_r^{-1} L_r,j sit in sh.K, sh.B, sh.T (j =
// 0, 1, 2) and g_j = M_r^{-1} f_r,j in sh.g[j], given sh.M (Cholesky factor)
// and the unsolved L_r,j / f_r,j in the same places. Solves in place and sets
// sh.n_c by the guard on sum_j ||K_j||_F (|theta_j| <= 1 bounds
// ||K(t)||_F by it at every t).
__device__ void red_forced_setup(RedShared& sh, int q, int np, double dT, int n_c0,
                                 const QSlots& sl) {
  const int tid = threadIdx.x;
  double (*P[kMaxPieces])[kMaxQ + 2] = {sh.K, sh.B, sh.T};
  for (int e = tid; e < np * q; e += 256) red_solve(sh, q, &P[e / q][0][e % q], kMaxQ + 2);
  if (tid < np) red_solve(sh, q, sh.g[tid], 1);
  __syncthreads();
  double nrm = 0.0;
  for (int j = 0; j < np; ++j) {
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (sl.i[r] < 0) break;
      const double v = P[j][sl.i[r]][sl.j[r]];
      s += v * v;
    }
    sh.red[tid] = s;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int i = 0; i < 256; ++i) t += sh.red[i];
      sh.tmp[0][0] = sqrt(t);
    }
    __syncthreads();
    nrm += sh.tmp[0][0];
    __syncthreads();
  }
  if (tid == 0) {
    int n_c = max(1, n_c0);
    while ((dT / n_c) * nrm > kGuard && n_c < (1 << 16)) n_c *= 2;
    sh.n_c = n_c;
  }
  __syncthreads();
}

// Forced flows: n_c classical RK4 steps of beta' = sum_j theta_j(t)
// (K_j beta + g_j) over [t0, t0 + dT] for beta[v], v < nv; stages at t,
// t + h/2, t + h/2, t + h.
__device__ void red_advance_forced(RedShared& sh, int q, int nv, int np, int kind, double w,
                                   double t0, double dT) {
  const int tid = threadIdx.x;
  double (*P[kMaxPieces])[kMaxQ + 2] = {sh.K, sh.B, sh.T};
  const double h = dT / sh.n_c;
  const bool act = tid < nv * q;
  const int v = act ? tid / q : 0, i = act ? tid % q : 0;
  const double cst[4] = {0.0, 0.5, 0.5, 1.0};     // stage time offsets
  const double cin[4] = {0.0, 0.5, 0.5, 1.0};     // stage input weights (of h)
  const double cacc[4] = {1.0, 2.0, 2.0, 1.0};
  for (int it = 0; it < sh.n_c; ++it) {
    const double t = t0 + it * h;
    for (int st = 0; st < 4; ++st) {
      if (act) sh.y[v][i] = st == 0 ? sh.beta[v][i] : fma(cin[st] * h, sh.kv[v][i], sh.beta[v][i]);
      __syncthreads();
      if (act) {
        const double ta = t + cst[st] * h;
        double k = 0.0;
        for (int j = 0; j < np; ++j) {
          double r = sh.g[j][i];
          for (int l = 0; l < q; ++l) r = fma(P[j][i][l], sh.y[v][l], r);
          k = fma(theta_of(kind, w, j, ta), r, k);
        }
        sh.kv[v][i] = k;
        sh.acc[v][i] = st == 0 ? k : fma(cacc[st], k, sh.acc[v][i]);
      }
      __syncthreads();
    }
    if (act) sh.beta[v][i] = fma(h / 6.0, sh.acc[v][i], sh.beta[v][i]);
    __syncthreads();
  }
}

// beta[v] <- B^{n_c} beta[v] for v < nv.
__device__ void red_advance(RedShared& sh, int q, int nv) {
  const int tid = threadIdx.x;
  const bool act = tid < nv * q;
  const int v = act ? tid / q : 0, i = act ? tid % q : 0;
  for (int it = 0; it < sh.n_c; ++it) {
    if (act) {
      double acc = 0.0;
      for (int k = 0; k < q; ++k) acc += sh.B[i][k] * sh.beta[v][k];
      sh.tmp[v][i] = acc;
    }
    __syncthreads();
    if (act) sh.beta[v][i] = sh.tmp[v][i];
    __syncthreads();
  }
}

// sh.B <- B^{n_c} by binary powering of the one-step propagator (sh.K and
// sh.T serve as work matrices; K is not needed after the propagator is
// formed). One barrier per product.
__device__ void red_power(RedShared& sh, int q, const QSlots& sl) {
  if (sh.n_c == 1) return;
  double (*A[3])[kMaxQ + 2] = {sh.B, sh.K, sh.T};
  int ib = 0, ir = 1, it = 2;   // base, result, spare (the same in every thread)
  bool have = false;
  auto mul = [&](int x, int y, int z) {   // A[z] = A[x] A[y]
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = sl.i[r], j = sl.j[r];
      if (i < 0) break;
      double acc = 0.0;
      for (int k = 0; k < q; ++k) acc += A[x][i][k] * A[y][k][j];
      A[z][i][j] = acc;
    }
    __syncthreads();
  };
  for (int e = sh.n_c; e > 0; e >>= 1) {
    if (e & 1) {
      if (!have) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (sl.i[r] < 0) break;
          A[ir][sl.i[r]][sl.j[r]] = A[ib][sl.i[r]][sl.j[r]];
        }
        __syncthreads();
        have = true;
      } else {
        mul(ir, ib, it);
        const int t = ir;
        ir = it;
        it = t;
      }
    }
    if (e > 1) {
      mul(ib, ib, it);
      const int t = ib;
      ib = it;
      it = t;
    }
  }
  if (ir != 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (sl.i[r] < 0) break;
      sh.B[sl.i[r]][sl.j[r]] = A[ir][sl.i[r]][sl.j[r]];
    }
    __syncthreads();
  }
}

// beta[v] <- P beta[v] for v < nv, P = sh.B (after red_power: B^{n_c}).
__device__ void red_apply(RedShared& sh, int q, int nv) {
  const int tid = threadIdx.x;
  const bool act = tid < nv * q;
  const int v = act ? tid / q : 0, i = act ? tid % q : 0;
  if (act) {
    double acc = 0.0;
    for (int k = 0; k < q; ++k) acc += sh.B[i][k] * sh.beta[v][k];
    sh.tmp[v][i] = acc;
  }
  __syncthreads();
  if (act) sh.beta[v][i] = sh.tmp[v][i];
  __syncthreads();
}

// Products of a binary power cost about three matrix-vector steps each: the
// power pays from this many steps on.
constexpr int kPowerMinSteps = 64;

__device__ void reduced_run(const ReducedDesc& d) {
  __shared__ RedShared sh;
  const int tid = threadIdx.x;
  if (tid == 0) {
    const int m = *d.m;
    const int aug = d.aug ? *d.aug : 0;
    int q = 0;
    for (int a = 0; a < m; ++a) sh.idx[q++] = a;
    if (aug) sh.idx[q++] = d.cap;
    sh.q = q;
    sh.bad = 0;
  }
  __syncthreads();
  const int q = sh.q;
  const int np = d.forced ? d.npieces : 1;
  const int ps = d.ld_piece > 0 ? d.ld_piece : 32;
  for (int e = tid; e < q * q; e += 256) {
    const int a = e / q, b = e % q;
    const double* row = d.S + (long long)sh.idx[a] * d.ld;
    sh.M[a][b] = row[d.off_M + sh.idx[b]];
    sh.K[a][b] = row[d.off_L + sh.idx[b]];
    if (np > 1) sh.B[a][b] = row[d.off_L + ps + sh.idx[b]];
    if (np > 2) sh.T[a][b] = row[d.off_L + 2 * ps + sh.idx[b]];
  }
  if (tid < d.n_in * q) {
    const int v = tid / q, a = tid % q;
    sh.beta[v][a] = d.S[(long long)sh.idx[a] * d.ld + d.off_U + v];
  }
  if (d.forced && tid < np * q) {
    const int j = tid / q, a = tid % q;
    sh.g[j][a] = d.S[(long long)sh.idx[a] * d.ld + d.off_F + j];
  }
  __syncthreads();
  const QSlots sl = q_slots(q);
  red_cholesky(sh, q, sl);
  if (tid < d.n_in) red_solve(sh, q, sh.beta[tid], 1);
  __syncthreads();
  // M_r not positive definite (a NaN or a breakdown): the coefficients become
  // NaN, so the correction and its jump norm carry the failure to the host
  if (sh.bad && tid < d.n_in * q) sh.beta[tid / q][tid % q] = NAN;
  __syncthreads();
  if (d.forced) {
    red_forced_setup(sh, q, np, d.dT, d.n_c, sl);
    red_advance_forced(sh, q, d.n_in, np, d.forced, d.w, d.t0, d.dT);
  } else {
    red_propagator(sh, q, d.dT, d.n_c, sl);
    if (sh.n_c >= kPowerMinSteps) {
      red_power(sh, q, sl);
      red_apply(sh, q, d.n_in);
    } else {
      red_advance(sh, q, d.n_in);
    }
  }
  const int w = d.cap + 1;
  for (int e = tid; e < d.n_in * w; e += 256) d.beta[e] = 0.0;
  if (d.coef)
    for (int e = tid; e < w; e += 256) d.coef[e] = 0.0;
  __syncthreads();
  if (tid < d.n_in * q) {
    const int v = tid / q, a = tid % q;
    d.beta[v * w + sh.idx[a]] = sh.beta[v][a];
  }
  if (d.coef && tid < q) {
    const double c = (d.n_in > 1) ? sh.beta[0][tid] - sh.beta[1][tid] : sh.beta[0][tid];
    d.coef[sh.idx[tid]] = c;
  }
  if (tid == 0) {
    if (d.n_c_out) *d.n_c_out = sh.n_c;
  }
}

__global__ __launch_bounds__(256) void k_reduced(const ReducedDesc* __restrict__ descs) {
  const ReducedDesc d = descs[blockIdx.x];
  reduced_run(d);
}

// One system, its descriptor passed as the kernel argument (no staging copy).
__global__ __launch_bounds__(256) void k_reduced_one(const ReducedDesc d) { reduced_run(d); }

void launch_reduced(const ReducedDesc* d, int nd, hipStream_t s) {
  if (nd <= 0) return;
  hipLaunchKernelGGL(k_reduced, dim3(nd), dim3(256), 0, s, d);
  PR_HIP(hipGetLastError());
}

void launch_reduced_one(const ReducedDesc& d, hipStream_t s) {
  hipLaunchKernelGGL(k_reduced_one, dim3(1), dim3(256), 0, s, d);
  PR_HIP(hipGetLastError());
}

__global__ __launch_bounds__(256) void k_reduced0(const Reduced0Desc* __restrict__ dp) {
  const Reduced0Desc d = *dp;
  __shared__ RedShared sh;
  const int tid = threadIdx.x;
  if (tid == 0) {
    const int m = *d.m;
    for (int a = 0; a < m; ++a) sh.idx[a] = a;
    sh.q = m;
    sh.bad = 0;
  }
  __syncthreads();
  const int q = sh.q;
  const int np = d.forced ? d.npieces : 1;
  const int ps = d.ld_piece > 0 ? d.ld_piece : 32;
  for (int e = tid; e < q * q; e += 256) {
    const int a = e / q, b = e % q;
    const double* row = d.S + (long long)a * d.ld;
    sh.M[a][b] = row[d.off_M + b];
    sh.K[a][b] = row[d.off_L + b];
    if (np > 1) sh.B[a][b] = row[d.off_L + ps + b];
    if (np > 2) sh.T[a][b] = row[d.off_L + 2 * ps + b];
  }
  if (tid < q) sh.beta[0][tid] = d.S[(long long)tid * d.ld + d.off_U];
  if (d.forced && tid < np * q) sh.g[tid / q][tid % q] = d.S[(long long)(tid % q) * d.ld + d.off_F + tid / q];
  __syncthreads();
  const QSlots sl = q_slots(q);
  red_cholesky(sh, q, sl);
  if (tid == 0) red_solve(sh, q, sh.beta[0], 1);
  __syncthreads();
  if (sh.bad && tid < q) sh.beta[0][tid] = NAN;   // as in reduced_run
  __syncthreads();
  // the same propagator for every subinterval: its n_c-th power once, then
  // one product per subinterval
  if (d.forced) {
    red_forced_setup(sh, q, np, d.dT, d.n_c, sl);
  } else {
    red_propagator(sh, q, d.dT, d.n_c, sl);
    red_power(sh, q, sl);
  }
  for (int n = 0; n < d.count; ++n) {
    // subinterval n runs over [(n + n_warm) dT, (n + n_warm + 1) dT]
    if (d.forced)
      red_advance_forced(sh, q, 1, np, d.forced, d.w, (double)(n + d.n_warm) * d.dT, d.dT);
    else red_apply(sh, q, 1);
    for (int e = tid; e < d.ld_out; e += 256)
      d.betas[(long long)n * d.ld_out + e] = (e < q) ? sh.beta[0][e] : 0.0;
  }
  if (tid == 0 && d.n_c_out) *d.n_c_out = sh.n_c;
}

void launch_reduced0(const Reduced0Desc* d, hipStream_t s) {
  hipLaunchKernelGGL(k_reduced0, dim3(1), dim3(256), 0, s, d);
  PR_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
__global__ void k_negate(const double* __restrict__ in, double* __restrict__ out, int n) {
  if ((int)threadIdx.x < n) out[threadIdx.x] = -in[threadIdx.x];
}

void launch_negate(const double* in, double* out, int n, hipStream_t s) {
  if (n <= 0) return;
  PR_CHECK(n <= 256, "negate: at most 256 values");
  hipLaunchKernelGGL(k_negate, dim3(1), dim3(256), 0, s, in, out, n);
  PR_HIP(hipGetLastError());
}

// out = max over i, j < min(*m, cap) of |G[i ld + j] - delta_ij| (NaN if any
// entry is NaN): the loss of M-orthonormality of a basis from its Gram.
__global__ void k_orth_defect(const double* __restrict__ G, int ld, const int* __restrict__ m,
                              int cap, double* out) {
  __shared__ double red[256];
  const int q = min(*m, cap);
  double v = 0.0;
  for (int e = threadIdx.x; e < q * q; e += 256) {
    const int i = e / q, j = e % q;
    const double d = fabs(G[(size_t)i * ld + j] - (i == j ? 1.0 : 0.0));
    if (!(d <= v)) v = d;   // keeps a NaN
  }
  red[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int t = 0; t < 256; ++t)
      if (!(red[t] <= r)) r = red[t];
    out[0] = r;
  }
}

void launch_orth_defect(const double* G, int ld, const int* m, int cap, double* out,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_orth_defect, dim3(1), dim3(256), 0, s, G, ld, m, cap, out);
  PR_HIP(hipGetLastError());
}

}  // namespace pr
