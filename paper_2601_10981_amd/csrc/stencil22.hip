// Fused RK4 step with 2 x 2 register blocking: the same step, stage pipeline
// and per-point arithmetic as k_rk4_fused (stencil.hip), but every thread owns
// a 2 x 2 block of (y, z) columns instead of one column.
//
// Of each point's four in-plane neighbours two are then in the thread's own
// registers, so a stage evaluation exchanges 24 B per point through LDS (one
// 8 B write, two 8 B reads) instead of 40 B (one write, four reads), and the
// per-block descriptors (offsets, velocity coefficients) are shared by four
// columns.
//
// LDS layout. A stage plane of the (TY + 8) x (TZ + 8) region is stored as two
// sub-planes, even z and odd z, of (TY + 8 + 2) rows x SZ columns (one guard
// row above and below, guard columns beside): point (ry, rz) at row ry + 1,
// column rz / 2 + 1 of sub-plane rz % 2. A block's four LDS neighbours of one
// kind (the two y-neighbours above its first row, the two z-neighbours left
// of its first column, ...) then lie in one sub-plane at lane stride 8 B, and
// pairs of them sit a fixed number of rows apart, so each pair is one
// ds_read2 and a block-stage takes four reads and two writes. SZ is odd, so
// lanes walking down a column of blocks (the halo ring's sides) hit distinct
// banks, and lanes along a row read consecutive values.
//
// Blocks are numbered interior first, then the block ring at distance 1 from
// the edge, then the outermost ring. A block at distance d >= 2 holds only
// interior points; d = 1 holds halo levels 2 and 1, d = 0 levels 4 and 3.
// Stage 1 runs on every block, stages 2 and 3 on d >= 1, the output stage on
// d >= 2. A point of a block whose stage its level does not need reads guard
// or stale LDS values; what it computes is never read by a point that does.
#include <type_traits>

#include "pr_internal.h"
#include "stencil_dev.h"

namespace pr {

namespace {

// Position p of the ring order over an IY x IZ interior with H rings around
// it: the interior row-major, then ring by ring, each ring as four
// contiguous segments (top row, bottom row, left column, right column) so
// that neighbouring lanes stay on neighbouring LDS rows or columns. Region
// coordinates and ring level (0 = interior); lev = 99 beyond the region.
template <int IY, int IZ, int H>
__device__ __forceinline__ void ring_pos(int p, int& ry, int& rz, int& lev) {
  if (p < IY * IZ) {
    ry = H + p / IZ;
    rz = H + p % IZ;
    lev = 0;
    return;
  }
  int start = IY * IZ;
#pragma unroll
  for (int L = 1; L <= H; ++L) {
    const int WY = IY + 2 * L, WZ = IZ + 2 * L;
    const int ring = 2 * WZ + 2 * (WY - 2);
    if (p < start + ring) {
      const int q = p - start;
      int by, bz;
      if (q < 2 * WZ) {            // top row, then bottom row
        by = q < WZ ? 0 : WY - 1;
        bz = q < WZ ? q : q - WZ;
      } else {                     // left column, then right column
        const int c = q - 2 * WZ;
        by = 1 + (c < WY - 2 ? c : c - (WY - 2));
        bz = c < WY - 2 ? 0 : WZ - 1;
      }
      ry = by + H - L;
      rz = bz + H - L;
      lev = L;
      return;
    }
    start += ring;
  }
  ry = rz = 0;
  lev = 99;
}

template <int P>
using Ph = std::integral_constant<int, P>;

template <int P, int END, typename F>
__device__ __forceinline__ void run_all(F& f) {
  if constexpr (P < END) {
    f(Ph<P>{}, std::false_type{});
    run_all<P + 1, END>(f);
  }
}
template <int P, int END, typename F>
__device__ __forceinline__ void run_upto(F& f, int left) {
  if constexpr (P < END) {
    if (left > 0) {
      f(Ph<P>{}, std::false_type{});
      run_upto<P + 1, END>(f, left - 1);
    }
  }
}

// L at one point from its six neighbours; the same operations in the same
// order as lop / lop_x of stencil_dev.h, so every value is bitwise the one
// k_rk4_fused computes.
template <typename T>
__device__ __forceinline__ T lop6(T xm, T c, T xp, T ym, T yp, T zm, T zp, T clap, T vx, T vy,
                                  T vz) {
#pragma clang fp contract(off)
  const T lap = fma((T)-6, c, ((xp + xm) + (yp + ym)) + (zp + zm));
  const T adv = fma(vz, zp - zm, fma(vy, yp - ym, vx * (xp - xm)));
  return fma(clap, lap, -adv);
}
template <typename T>
__device__ __forceinline__ T lop6_x(T xm, T c, T xp, T ym, T yp, T zm, T zp, T clap, T e, T a,
                                    T b) {
#pragma clang fp contract(off)
  const T syz = (yp + ym) + (zp + zm);
  return fma(a, xp, fma(b, xm, fma(clap, syz, e * c)));
}

}  // namespace

// x planes per workgroup at most (the host caps the chunk; the per-plane
// velocity table in LDS is sized for it)
constexpr int kB22Chunk = kBlockedChunk;

// Geometry of the blocked LDS planes for an output tile TY x TZ.
template <typename T, int TY, int TZ>
struct B22 {
  static constexpr int H = kFusedHalo;
  static constexpr int RY = TY + 2 * H, RZ = TZ + 2 * H;
  static constexpr int BY = RY / 2, BZ = RZ / 2;          // blocks
  static constexpr int NB = BY * BZ;
  static constexpr int SZ = (BZ + 2) | 1;                  // sub-plane row: odd, >= BZ + 2
  static constexpr int SR = RY + 2;                       // sub-plane rows
  static constexpr int SUB = SR * SZ;                     // values per sub-plane
  static constexpr int PLANE = 2 * SUB;                   // even + odd
  static_assert(TY % 2 == 0 && TZ % 2 == 0, "blocks of 2 x 2");
  static_assert(SZ >= BZ + 2, "guard columns");
};

template <typename T, int TY, int TZ, int NT, bool XONLY, int RING, bool SPLIT>
__device__ __forceinline__ void rk4_tile22(const FineDesc<T>& d, int step, long long lt, T* lds,
                                           T (*vxt)[kB22Chunk + 10]) {
#pragma clang fp contract(off)
  using G = B22<T, TY, TZ>;
  using V2 = T __attribute__((ext_vector_type(2)));
  constexpr int H = G::H, SZ = G::SZ, SUB = G::SUB, PLANE = G::PLANE;
  static_assert(RING % 3 == 0 && RING >= 6, "the y ring is a whole number of W-ring periods");
  const int tz = (int)(lt % d.tiles_z);
  const long long rest = lt / d.tiles_z;
  const int ty = (int)(rest % d.tiles_y);
  const int tx = (int)(rest / d.tiles_y);
  const int n = d.g.n;
  const long long plane = (long long)n * n;
  const int y0 = ty * TY, z0 = tz * TZ;
  const int x0 = tx * d.xc, x1 = min(n, x0 + d.xc);
  const int nst = d.n_steps;
  const PR_GLOBAL T* src = gptr((step == 0) ? d.first_src : (const T*)d.buf[(nst - step) % 2]);
  PR_GLOBAL T* dst = gptr(d.buf[(nst - 1 - step) % 2]);
  PR_GLOBAL T* snap = nullptr;
  if (d.snaps != nullptr && (step + 1) % d.snap_every == 0)
    snap = gptr(d.snaps + (long long)((step + 1) / d.snap_every) * d.snap_ld);
  const PR_GLOBAL T* tab = gptr(tab_of<T>(d.g));
  const T clap = (T)d.g.c_lap;
  const T e6 = (T)-6 * clap;
  const T dt = (T)d.dt;
  const T c1 = dt * (T)0.25, c2 = dt / (T)3, c3 = dt * (T)0.5, c4 = dt;

  // this thread's block: block-region coordinates (by, bz), block ring
  int by, bz, blev;
  ring_pos<TY / 2, TZ / 2, H / 2>((int)threadIdx.x, by, bz, blev);
  const bool live = blev <= 2;            // a block of the region
  const bool mid = blev <= 1;             // stages 2 and 3
  const bool inner = blev == 0;           // output stage
  // first point of the block in the region and on the grid
  const int ry = 2 * by, rz = 2 * bz;
  const bool outp = inner && y0 + ry - H < n && z0 + rz - H < n;
  const int gy0 = wrapi(y0 + ry - H, n), gy1 = wrapi(y0 + ry - H + 1, n);
  const int gz = wrapi(z0 + rz - H, n);   // even: the pair gz, gz + 1 is contiguous
  const int off0 = live ? gy0 * n + gz : 0, off1 = live ? gy1 * n + gz : 0;
  // LDS index of the block's first point in the even sub-plane
  const int li = (ry + 1) * SZ + bz + 1;

  // velocity: point k = 2 i + j is (row i, column j) of the block
  T va[4], vb[4], vyz[2], vzy[2];
  {
    const int gzz[2] = {gz, gz + 1};
    const int gyy[2] = {gy0, gy1};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const T vx = tab[gyy[k >> 1]] + tab[n + gzz[k & 1]];
      va[k] = XONLY ? clap - vx : vx;
      vb[k] = XONLY ? clap + vx : (T)0;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      vyz[j] = XONLY ? (T)0 : tab[3 * n + gzz[j]];
      vzy[j] = XONLY ? (T)0 : tab[5 * n + gyy[j]];
    }
  }
  if (!XONLY)
    for (int i = threadIdx.x; i < x1 - x0 + 10; i += NT) {
      const int x = wrapi(x0 - 6 + i, n);
      vxt[0][i] = tab[2 * n + x];
      vxt[1][i] = tab[4 * n + x];
    }

  // A wave whose 64 blocks are all interior output blocks runs every stage on
  // every lane: its copy of the march has no per-lane stage gating (SPLIT:
  // the tilings whose register budget holds both copies without spilling).
  constexpr bool kSplit = SPLIT && XONLY;
  const bool full = kSplit && __ballot(!(inner && outp)) == 0ull;
  auto body = [&](auto fullc) {
  constexpr bool FULL = decltype(fullc)::value;
  const bool live_ = FULL || live, mid_ = FULL || mid, outp_ = FULL || outp;
  // rings as in rk4_tile, per point of the block
  T Y[4][RING], W1[4][3], W2[4][3], W3[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int r = 0; r < RING; ++r) Y[k][r] = (T)0;
#pragma unroll
    for (int r = 0; r < 3; ++r) W1[k][r] = W2[k][r] = W3[k][r] = (T)0;
  }
  // y of plane x into ring entry r of the four points: two pair loads,
  // unconditional (blocks beyond the region read offset 0)
#define PR_B22_LOAD(base, r)                                            \
  do {                                                                  \
    const V2 u_ = *(const PR_GLOBAL V2*)(src + (base) + off0);          \
    const V2 w_ = *(const PR_GLOBAL V2*)(src + (base) + off1);          \
    Y[0][r] = u_.x;                                                     \
    Y[1][r] = u_.y;                                                     \
    Y[2][r] = w_.x;                                                     \
    Y[3][r] = w_.y;                                                     \
  } while (0)
#pragma unroll
  for (int r = 2; r <= RING - 2; ++r) {
    const long long pk = (long long)wrapi(x0 - 6 + r, n) * plane;
    PR_B22_LOAD(pk, r);
  }
  long long ol = (long long)wrapi(x0 - 7 + RING, n) * plane;
  long long od = (long long)wrapi(x0 - 6, n) * plane;
  const long long ng = plane * n;
  int tt = x0 - 6;

  auto march = [&](auto phase, auto warm) {
    constexpr int PH = decltype(phase)::value;
    constexpr bool WARM = decltype(warm)::value;
    constexpr bool s2 = !WARM || PH >= 2, s3 = !WARM || PH >= 4, s4 = !WARM;
    __builtin_amdgcn_sched_barrier(0);
    constexpr int k0 = PH % RING, k1 = (1 + PH) % RING, k2 = (2 + PH) % RING,
                  k3 = (3 + PH) % RING, k4 = (4 + PH) % RING, kl = (RING - 1 + PH) % RING;
    constexpr int j0 = PH % 3, j1 = (1 + PH) % 3, j2 = (2 + PH) % 3;
    // the two LDS plane sets alternate with the step (not the ring phase:
    // RING may be odd)
    T* pl = lds + ((tt - x0) & 1) * 4 * PLANE;
    PR_B22_LOAD(ol, kl);   // y(tt + RING - 1)
    // current plane of every stage into LDS: even sub-plane then odd, rows
    // 0 and 1 of the block one sub-plane row apart
    auto put = [&](T* p, T a0, T a1, T a2, T a3) {
      p[li] = a0;
      p[li + SZ] = a2;
      p[SUB + li] = a1;
      p[SUB + li + SZ] = a3;
    };
    if (live_) put(pl, Y[0][k3], Y[1][k3], Y[2][k3], Y[3][k3]);
    if (live_) put(pl + PLANE, W1[0][j1], W1[1][j1], W1[2][j1], W1[3][j1]);
    if (mid_) put(pl + 2 * PLANE, W2[0][j1], W2[1][j1], W2[2][j1], W2[3][j1]);
    if (mid_) put(pl + 3 * PLANE, W3[0][j1], W3[1][j1], W3[2][j1], W3[3][j1]);
    __syncthreads();
    const int iv = tt - (x0 - 6);
    T vy_p[4], vz_p[4];   // per-plane velocity parts of stages 1..4
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      vy_p[s] = XONLY ? (T)0 : vxt[0][iv + 3 - s];
      vz_p[s] = XONLY ? (T)0 : vxt[1][iv + 3 - s];
    }
    // the eight LDS neighbours of the block in stage plane p: above row 0 and
    // below row 1 (columns 0, 1), left of column 0 and right of column 1
    // (rows 0, 1)
    struct Nb {
      T yu0, yu1, yd0, yd1, zl0, zl1, zr0, zr1;
    };
    auto rd = [&](const T* p) {
      Nb q;
      q.yu0 = p[li - SZ];
      q.yu1 = p[SUB + li - SZ];
      q.yd0 = p[li + 2 * SZ];
      q.yd1 = p[SUB + li + 2 * SZ];
      q.zl0 = p[SUB + li - 1];
      q.zl1 = p[SUB + li - 1 + SZ];
      q.zr0 = p[li + 1];
      q.zr1 = p[li + 1 + SZ];
      return q;
    };
    // one stage on the block: input planes xm / c / xp (4 values each), the
    // centre plane's LDS neighbours, per-plane velocity parts; L[k] = L at
    // point k
    auto comp = [&](const T* xm, const T* c, const T* xp, const Nb& q, T vyp, T vzp, T* L) {
      // neighbours (ym, yp, zm, zp) of points 0..3
      const T ym[4] = {q.yu0, q.yu1, c[0], c[1]};
      const T yp[4] = {c[2], c[3], q.yd0, q.yd1};
      const T zm[4] = {q.zl0, c[0], q.zl1, c[2]};
      const T zp[4] = {c[1], q.zr0, c[3], q.zr1};
#pragma unroll
      for (int k = 0; k < 4; ++k)
        L[k] = XONLY ? lop6_x<T>(xm[k], c[k], xp[k], ym[k], yp[k], zm[k], zp[k], clap, e6, va[k],
                                 vb[k])
                     : lop6<T>(xm[k], c[k], xp[k], ym[k], yp[k], zm[k], zp[k], clap, va[k],
                               vyp + vyz[k & 1], vzp + vzy[k >> 1]);
    };
    T a[4], b[4], e[4], L[4];
    // stage s's inputs: x neighbours and centre from the rings
    auto in1 = [&]() {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        a[k] = Y[k][k2];
        b[k] = Y[k][k3];
        e[k] = Y[k][k4];
      }
    };
    auto inW = [&](T (*R)[3]) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        a[k] = R[k][j0];
        b[k] = R[k][j1];
        e[k] = R[k][j2];
      }
    };
    auto store = [&]() {
      V2 r0, r1;
      r0.x = fma(c4, L[0], Y[0][k0]);
      r0.y = fma(c4, L[1], Y[1][k0]);
      r1.x = fma(c4, L[2], Y[2][k0]);
      r1.y = fma(c4, L[3], Y[3][k0]);
      *(PR_GLOBAL V2*)(dst + od + off0) = r0;
      *(PR_GLOBAL V2*)(dst + od + off1) = r1;
      if (snap) {
        *(PR_GLOBAL V2*)(snap + od + off0) = r0;
        *(PR_GLOBAL V2*)(snap + od + off1) = r1;
      }
    };
    {
      // stage 1 at plane tt + 3 (every block)
      in1();
      T w1[4] = {(T)0, (T)0, (T)0, (T)0};
      if (live_) {
        comp(a, b, e, rd(pl), vy_p[0], vz_p[0], L);
#pragma unroll
        for (int k = 0; k < 4; ++k) w1[k] = fma(c1, L[k], Y[k][k3]);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) W1[k][j2] = w1[k];
      // stage 2 at plane tt + 2
      T w2[4] = {(T)0, (T)0, (T)0, (T)0};
      if (s2 && mid_) {
        inW(W1);
        comp(a, b, e, rd(pl + PLANE), vy_p[1], vz_p[1], L);
#pragma unroll
        for (int k = 0; k < 4; ++k) w2[k] = fma(c2, L[k], Y[k][k2]);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) W2[k][j2] = w2[k];
      // stage 3 at plane tt + 1
      T w3[4] = {(T)0, (T)0, (T)0, (T)0};
      if (s3 && mid_) {
        inW(W2);
        comp(a, b, e, rd(pl + 2 * PLANE), vy_p[2], vz_p[2], L);
#pragma unroll
        for (int k = 0; k < 4; ++k) w3[k] = fma(c3, L[k], Y[k][k1]);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) W3[k][j2] = w3[k];
      // output stage at plane tt
      if (s4 && outp_) {
        inW(W3);
        comp(a, b, e, rd(pl + 3 * PLANE), vy_p[3], vz_p[3], L);
        store();
      }
    }
    ol += plane;
    if (ol == ng) ol = 0;
    od += plane;
    if (od == ng) od = 0;
    ++tt;
  };

  using W = std::true_type;
  __syncthreads();   // vxt visible
  march(Ph<0>{}, W{}); march(Ph<1>{}, W{}); march(Ph<2>{}, W{});
  march(Ph<3>{}, W{}); march(Ph<4>{}, W{}); march(Ph<5>{}, W{});
  int left = x1 - x0;
  run_upto<6, RING>(march, left);
  left -= min(left, RING - 6);
  for (; left >= RING; left -= RING) run_all<0, RING>(march);
  run_upto<0, RING>(march, left);
  };
  if constexpr (kSplit) {
    if (full) body(std::true_type{});
    else body(std::false_type{});
  } else {
    body(std::false_type{});
  }
#undef PR_B22_LOAD
}

template <typename T, int TY, int TZ, int NT, bool XO>
constexpr int b22_waves_per_simd() {
  using G = B22<T, TY, TZ>;
  constexpr long long lds =
      (2LL * 4 * G::PLANE + (XO ? 0 : 2LL * (kB22Chunk + 10))) * (long long)sizeof(T);
  constexpr long long wgs = (160LL * 1024) / lds;
  constexpr long long w = (wgs * (NT / 64) + 3) / 4;
  return w < 1 ? 1 : (w > 4 ? 4 : (int)w);
}

// XO = 1: every field of the launch has a velocity along x only, and the
// per-plane velocity table is not needed (more workgroups fit a CU);
// XO = 0: each field takes its own operator form. SPLIT (with XO = 1): fully
// interior waves take a march without per-lane stage gating.
template <typename T, int TY, int TZ, int NT, int RING, bool XO, bool SPLIT>
__global__ __launch_bounds__(NT, (b22_waves_per_simd<T, TY, TZ, NT, XO>())) void k_rk4_b22(
    const FineDesc<T>* __restrict__ descs, int nd, int step, long long total, long long per_xcd) {
  using G = B22<T, TY, TZ>;
  static_assert(G::NB <= NT, "one block per thread");
  // two sets of the four stage planes, alternating per march step
  __shared__ T lds[2 * 4 * G::PLANE];
  __shared__ T vxt[XO ? 1 : 2][XO ? 1 : kB22Chunk + 10];
  const long long b = blockIdx.x;
  const long long t = (b % 8) * per_xcd + b / 8;
  if (t >= total) return;
  const int f = find_desc(descs, nd, t);
  const FineDesc<T>& d = descs[f];
  if (step >= d.n_steps) return;
  if (XO || d.g.xonly)
    rk4_tile22<T, TY, TZ, NT, true, RING, XO && SPLIT>(d, step, t - d.tile_begin, lds,
                                                       (T (*)[kB22Chunk + 10])vxt);
  else
    rk4_tile22<T, TY, TZ, NT, false, RING, false>(d, step, t - d.tile_begin, lds,
                                                  (T (*)[kB22Chunk + 10])vxt);
}

// The y ring: nine planes, loads four steps ahead of their first use (on
// 63 x 128^3 FP64, 32 x 32 tiles: six planes 229, nine 245, twelve 242 GPts/s;
// twelve nears the register limit).
constexpr int kB22Ring = 9;

// Tilings whose fully interior waves take the ungated march: FP64 with 32
// columns along z (both copies of the march fit 256 VGPRs without spilling;
// at 64 columns they do not, and FP32 runs at more waves per SIMD).
template <typename T, int TY, int TZ>
constexpr bool b22_split() {
  return sizeof(T) == 8 && TZ == 32;
}

template <typename T, int TY, int TZ, int NT, bool XO>
static void launch_b22_xo(const FineDesc<T>* d, int nd, long long total, int step,
                          hipStream_t s) {
  const long long g8 = (total + 7) / 8 * 8;
  hipLaunchKernelGGL((k_rk4_b22<T, TY, TZ, NT, kB22Ring, XO, b22_split<T, TY, TZ>()>),
                     dim3((unsigned)g8), dim3(NT), 0, s,
                     d, nd, step, total, g8 / 8);
}

template <typename T, int TY, int TZ, int NT>
static void launch_b22(const FineDesc<T>* d, int nd, long long total, int step, bool xo,
                       hipStream_t s) {
  if (xo) launch_b22_xo<T, TY, TZ, NT, true>(d, nd, total, step, s);
  else launch_b22_xo<T, TY, TZ, NT, false>(d, nd, total, step, s);
}

template <typename T, int TY, int TZ, int NT, bool XO>
static int occ_b22_xo() {
  int v = 0;
  PR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &v, k_rk4_b22<T, TY, TZ, NT, kB22Ring, XO, b22_split<T, TY, TZ>()>, NT, 0));
  return v;
}

template <typename T, int TY, int TZ, int NT>
static int occ_b22(bool xo) {
  return xo ? occ_b22_xo<T, TY, TZ, NT, true>() : occ_b22_xo<T, TY, TZ, NT, false>();
}

// Blocked tilings (kFusedCfgs entries with blocked = 1), by tiling index.
template <typename T>
static void b22_step(const FineDesc<T>* d, int nd, long long total, int step, int cfg, bool xo,
                     hipStream_t s) {
  if (total <= 0) return;
  switch (cfg) {
    case 8: launch_b22<T, 32, 32, 448>(d, nd, total, step, xo, s); break;
    case 9: launch_b22<T, 16, 64, 512>(d, nd, total, step, xo, s); break;
    case 10: launch_b22<T, 16, 32, 256>(d, nd, total, step, xo, s); break;
    default: fail(PR_EINVAL, "unknown blocked stencil configuration");
  }
  PR_HIP(hipGetLastError());
}

template <typename T>
static int b22_occ(int cfg, bool xo) {
  switch (cfg) {
    case 8: return occ_b22<T, 32, 32, 448>(xo);
    case 9: return occ_b22<T, 16, 64, 512>(xo);
    case 10: return occ_b22<T, 16, 32, 256>(xo);
    default: fail(PR_EINVAL, "unknown blocked stencil configuration");
  }
  return 0;
}

void launch_b22_step_f64(const FineDesc<double>* d, int nd, long long total, int step, int cfg,
                         bool xo, hipStream_t s) {
  b22_step<double>(d, nd, total, step, cfg, xo, s);
}
void launch_b22_step_f32(const FineDesc<float>* d, int nd, long long total, int step, int cfg,
                         bool xo, hipStream_t s) {
  b22_step<float>(d, nd, total, step, cfg, xo, s);
}
int b22_blocks_per_cu(int cfg, bool f32, bool xo) {
  return f32 ? b22_occ<float>(cfg, xo) : b22_occ<double>(cfg, xo);
}

}  // namespace pr
