// Fine propagator kernels of the periodic FD advection-diffusion operator
// (L u)_p = kappa sum_d (u_{p+e_d} - 2 u_p + u_{p-e_d}) / h^2
//           - sum_d v_d(p) (u_{p+e_d} - u_{p-e_d}) / (2 h).
//
// For this linear autonomous operator one classical RK4 step is P4(dt L) y
// with P4(z) = 1 + z + z^2/2 + z^3/6 + z^4/24, evaluated in Horner form as
// four stencil stages that all use y as base:
//   w1 = y + dt/4 L y,  w2 = y + dt/3 L w1,  w3 = y + dt/2 L w2,
//   y_new = y + dt L w3.
//
// k_rk4_fused runs all four stages of one step in one pass over HBM (read y,
// write y_new: 2 x s_f bytes per point instead of 11 x s_f for four separate
// sweeps). A workgroup owns a tile of the (y, z) plane (the tiling is a
// template parameter, chosen per batch by timing) and marches along x
// through a chunk of planes. Stage s is evaluated on the tile grown by 4 - s
// halo layers, so the 4-layer halo of y suffices; the stages form a skewed
// pipeline along x (at march step t: w1 at plane t + 3, w2 at t + 2, w3 at
// t + 1, y_new at t). Workgroups are mapped to XCDs in contiguous tile ranges
// so neighbouring tiles share an L2.
#include <type_traits>

#include "pr_internal.h"
#include "stencil_dev.h"

namespace pr {

// (L u) at one point from its centre c0, x neighbours cm / cp, y neighbours
// ym / yp and z neighbours zm / zp, velocity (vx, vy, vz).
template <typename T>
__device__ __forceinline__ T l_point(T cm, T c0, T cp, T ym, T yp, T zm, T zp, T vx, T vy, T vz,
                                     T clap) {
  const T lap = ((cp + cm) + (yp + ym) + (zp + zm)) - (T)6 * c0;
  const T adv = vx * (cp - cm) + vy * (yp - ym) + vz * (zp - zm);
  return clap * lap - adv;
}

// Evaluate (L in) along x for one (j, k) column over planes [x0, x1),
// calling emit(x, p, Lv) for each plane. Periodic wrap on every axis. The
// loads of four planes are issued before any of them is used, so a thread
// waits for memory once per four planes rather than once per plane.
template <typename T, typename Emit>
__device__ __forceinline__ void march_L(const Geom& g, const PR_GLOBAL T* __restrict__ in, int j,
                                        int k, int x0, int x1, Emit emit) {
  const int n = g.n;
  const long long plane = (long long)n * n;
  const PR_GLOBAL T* tab = gptr(tab_of<T>(g));
  const T clap = (T)g.c_lap;
  const int jm = (j == 0) ? n - 1 : j - 1, jp = (j == n - 1) ? 0 : j + 1;
  const int km = (k == 0) ? n - 1 : k - 1, kp = (k == n - 1) ? 0 : k + 1;
  const T vx = tab[0 * n + j] + tab[1 * n + k];
  const T vy_z = tab[3 * n + k];
  const T vz_y = tab[5 * n + j];
  const int q = j * n + k;
  const int oym = jm * n + k, oyp = jp * n + k, ozm = j * n + km, ozp = j * n + kp;
  const int xm0 = (x0 == 0) ? n - 1 : x0 - 1;
  T cm = in[(long long)xm0 * plane + q];
  T c0 = in[(long long)x0 * plane + q];
  auto point = [&](int x, T cp, T ym, T yp, T zm, T zp, T ty, T tz) {
    emit(x, (long long)x * plane + q,
         l_point<T>(cm, c0, cp, ym, yp, zm, zp, vx, ty + vy_z, tz + vz_y, clap));
    cm = c0;
    c0 = cp;
  };
  constexpr int U = 4;
  int x = x0;
  for (; x + U <= x1; x += U) {
    T cp[U], ym[U], yp[U], zm[U], zp[U], ty[U], tz[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int xx = x + u;
      const int xp = (xx == n - 1) ? 0 : xx + 1;
      const long long base = (long long)xx * plane;
      cp[u] = in[(long long)xp * plane + q];
      ym[u] = in[base + oym];
      yp[u] = in[base + oyp];
      zm[u] = in[base + ozm];
      zp[u] = in[base + ozp];
      ty[u] = tab[2 * n + xx];
      tz[u] = tab[4 * n + xx];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) point(x + u, cp[u], ym[u], yp[u], zm[u], zp[u], ty[u], tz[u]);
  }
  for (; x < x1; ++x) {
    const int xp = (x == n - 1) ? 0 : x + 1;
    const long long base = (long long)x * plane;
    point(x, in[(long long)xp * plane + q], in[base + oym], in[base + oyp], in[base + ozm],
          in[base + ozp], tab[2 * n + x], tab[4 * n + x]);
  }
}

// ---------------------------------------------------------------------------
// Fused RK4 step.

template <int P>
using Phase = std::integral_constant<int, P>;

// Steady march steps of phases P, P + 1, ..., END - 1 (all of them), or only
// the first `left` of them.
template <int P, int END, typename F>
__device__ __forceinline__ void march_all(F& f) {
  if constexpr (P < END) {
    f(Phase<P>{}, std::false_type{});
    march_all<P + 1, END>(f);
  }
}
template <int P, int END, typename F>
__device__ __forceinline__ void march_upto(F& f, int left) {
  if constexpr (P < END) {
    if (left > 0) {
      f(Phase<P>{}, std::false_type{});
      march_upto<P + 1, END>(f, left - 1);
    }
  }
}

// One fused RK4 step of one workgroup tile. The stages form a skewed
// pipeline along x: at march step tt, w1 at plane tt + 3, w2 at tt + 2, w3 at
// tt + 1 and y_new at tt. Each thread holds SL columns (slots); for each it
// keeps the planes every stage still needs in registers and exchanges the
// current plane of every stage through LDS for the y and z neighbours.
// The per-slot plane windows are rings of registers indexed by the march
// step modulo their length (RING for y, whose last entries are loads in
// flight, 3 for the stages), and the march is unrolled by RING so every ring
// index is a compile-time constant (no register shuffling per step). Slots
// wholly inside the interior are known at compile time and skip the ring
// tests.
template <typename T, int TY, int TZ, int NT, bool XONLY, int RING>
__device__ __forceinline__ void rk4_tile(const FineDesc<T>& d, int step, long long lt,
                                         T (*lds)[4][(TY + 2 * kFusedHalo) * (TZ + 2 * kFusedHalo)],
                                         T (*vxt)[kMaxChunk + 10]) {
#pragma clang fp contract(off)
  constexpr int H = kFusedHalo;
  constexpr int RY = TY + 2 * H, RZ = TZ + 2 * H;
  constexpr int NR = RY * RZ;
  constexpr int SL = (NR + NT - 1) / NT;
  constexpr int NI = TY * TZ;
  static_assert(RING % 6 == 0, "the y ring is a whole number of W-ring periods and even");
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

  int ci[SL];    // row-major LDS index of the slot's column
  int off[SL];   // gy * n + gz of the slot's column
  int lev[SL];   // ring level (0 = interior), 99 = no column
  bool outp[SL];
  T va[SL], vb[SL], vyz[SL], vzy[SL];   // XONLY: a, b; else v_x and the y/z parts
#pragma unroll
  for (int s = 0; s < SL; ++s) {
    int ry, rz, lv;
    ring_col<TY, TZ>((int)threadIdx.x + s * NT, ry, rz, lv);
    lev[s] = lv;
    ci[s] = ry * RZ + rz;
    const int dy = ry - H, dz = rz - H;
    outp[s] = lv == 0 && y0 + dy < n && z0 + dz < n;
    const int gy = wrapi(y0 + dy, n), gz = wrapi(z0 + dz, n);
    off[s] = lv <= H ? gy * n + gz : 0;
    const T vx = tab[gy] + tab[n + gz];
    va[s] = XONLY ? clap - vx : vx;
    vb[s] = XONLY ? clap + vx : (T)0;
    vyz[s] = XONLY ? (T)0 : tab[3 * n + gz];
    vzy[s] = XONLY ? (T)0 : tab[5 * n + gy];
  }
  if (!XONLY)
    for (int i = threadIdx.x; i < x1 - x0 + 10; i += NT) {
      const int x = wrapi(x0 - 6 + i, n);
      vxt[0][i] = tab[2 * n + x];
      vxt[1][i] = tab[4 * n + x];
    }

  // Rings, at march step tt with phase ph = (tt - x0 + 6) % RING, logical
  // index k at physical (k + ph) % RING: Y: y(tt + k), k = 0..RING-1 (k =
  // RING - 1 is loaded during the step, RING - 5 steps ahead of use); W1:
  // w1(tt + 1 + k), W2: w2(tt + k), W3: w3(tt - 1 + k), k = 0..2 at physical
  // (k + ph) % 3.
  T Y[SL][RING], W1[SL][3], W2[SL][3], W3[SL][3];
#pragma unroll
  for (int s = 0; s < SL; ++s) {
#pragma unroll
    for (int k = 0; k < RING; ++k) Y[s][k] = (T)0;
#pragma unroll
    for (int k = 0; k < 3; ++k) W1[s][k] = W2[s][k] = W3[s][k] = (T)0;
  }
  // y(tt + k) for k = 2 .. RING - 2 before the first step (tt = x0 - 6);
  // each step then loads y(tt + RING - 1), RING - 5 steps ahead of its
  // first use. Unconditional loads (slots without a column read offset 0):
  // a conditional load would merge values across lanes and wait at once.
#pragma unroll
  for (int k = 2; k <= RING - 2; ++k) {
    const long long pk = (long long)wrapi(x0 - 6 + k, n) * plane;
#pragma unroll
    for (int s = 0; s < SL; ++s) Y[s][k] = src[pk + off[s]];
  }
  // plane offsets of x = tt + RING - 1 (load) and x = tt (store), wrapped by
  // stepping instead of dividing
  long long o5 = (long long)wrapi(x0 - 7 + RING, n) * plane;
  long long od = (long long)wrapi(x0 - 6, n) * plane;
  const long long ng = plane * n;
  int tt = x0 - 6;

  // phase: march step modulo RING; warm: the first six steps of the chunk,
  // where stage s only starts once its input planes exist (w2 from the third
  // step, w3 from the fifth, y_new after the sixth)
  auto march = [&](auto phase, auto warm) {
    constexpr int PH = decltype(phase)::value;
    constexpr bool WARM = decltype(warm)::value;
    constexpr bool s2 = !WARM || PH >= 2, s3 = !WARM || PH >= 4, s4 = !WARM;
    // keep the scheduler from interleaving consecutive steps (which would
    // stretch live ranges across the unrolled round)
    __builtin_amdgcn_sched_barrier(0);
    // Y ring positions (period 6) and W ring positions (period 3)
    constexpr int k0 = PH % RING, k1 = (1 + PH) % RING, k2 = (2 + PH) % RING,
                  k3 = (3 + PH) % RING, k4 = (4 + PH) % RING, kl = (RING - 1 + PH) % RING;
    constexpr int j0 = PH % 3, j1 = (1 + PH) % 3, j2 = (2 + PH) % 3;
    T (*pl)[NR] = lds[PH & 1];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      const bool inner = (s + 1) * NT <= NI;
      Y[s][kl] = src[o5 + off[s]];   // y(tt + RING - 1), used RING - 5 steps later
      if (inner || lev[s] <= H) pl[0][ci[s]] = Y[s][k3];
      if (inner || lev[s] <= H - 1) pl[1][ci[s]] = W1[s][j1];
      if (inner || lev[s] <= H - 2) pl[2][ci[s]] = W2[s][j1];
      if (inner || lev[s] <= H - 3) pl[3][ci[s]] = W3[s][j1];
    }
    __syncthreads();
    const int iv = tt - (x0 - 6);
    T vy_a = 0, vz_a = 0, vy_b = 0, vz_b = 0, vy_c = 0, vz_c = 0, vy_d = 0, vz_d = 0;
    if (!XONLY) {
      vy_a = vxt[0][iv + 3]; vz_a = vxt[1][iv + 3];
      vy_b = vxt[0][iv + 2]; vz_b = vxt[1][iv + 2];
      vy_c = vxt[0][iv + 1]; vz_c = vxt[1][iv + 1];
      vy_d = vxt[0][iv];     vz_d = vxt[1][iv];
    }
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      const bool inner = (s + 1) * NT <= NI;
      const int c = ci[s];
      const int lv = lev[s];
      // every ring entry is overwritten each step (zero where the stage is
      // skipped), so no stale entry stays live across the march
      T w1 = (T)0, w2 = (T)0, w3 = (T)0;
      if (inner || lv <= H - 1) {
        const T L1 = XONLY ? lop_x<T, RZ>(Y[s][k2], Y[s][k3], Y[s][k4], pl[0], c, clap, e6, va[s],
                                          vb[s])
                           : lop<T, RZ>(Y[s][k2], Y[s][k3], Y[s][k4], pl[0], c, clap, va[s],
                                        vy_a + vyz[s], vz_a + vzy[s]);
        w1 = fma(c1, L1, Y[s][k3]);
      }
      W1[s][j2] = w1;
      if (s2 && (inner || lv <= H - 2)) {
        const T L2 = XONLY ? lop_x<T, RZ>(W1[s][j0], W1[s][j1], W1[s][j2], pl[1], c, clap, e6,
                                          va[s], vb[s])
                           : lop<T, RZ>(W1[s][j0], W1[s][j1], W1[s][j2], pl[1], c, clap, va[s],
                                        vy_b + vyz[s], vz_b + vzy[s]);
        w2 = fma(c2, L2, Y[s][k2]);
      }
      W2[s][j2] = w2;
      if (s3 && (inner || lv <= H - 3)) {
        const T L3 = XONLY ? lop_x<T, RZ>(W2[s][j0], W2[s][j1], W2[s][j2], pl[2], c, clap, e6,
                                          va[s], vb[s])
                           : lop<T, RZ>(W2[s][j0], W2[s][j1], W2[s][j2], pl[2], c, clap, va[s],
                                        vy_c + vyz[s], vz_c + vzy[s]);
        w3 = fma(c3, L3, Y[s][k1]);
      }
      W3[s][j2] = w3;
      if (s4 && outp[s]) {
        const T L4 = XONLY ? lop_x<T, RZ>(W3[s][j0], W3[s][j1], W3[s][j2], pl[3], c, clap, e6,
                                          va[s], vb[s])
                           : lop<T, RZ>(W3[s][j0], W3[s][j1], W3[s][j2], pl[3], c, clap, va[s],
                                        vy_d + vyz[s], vz_d + vzy[s]);
        const T yn = fma(c4, L4, Y[s][k0]);
        dst[od + off[s]] = yn;
        if (snap) snap[od + off[s]] = yn;
      }
    }
    o5 += plane;
    if (o5 == ng) o5 = 0;
    od += plane;
    if (od == ng) od = 0;
    ++tt;
  };
  using W = std::true_type;

  __syncthreads();   // vxt visible
  // (x1 - x0) + 6 march steps: the six warm-up steps (phases 0..5), the rest
  // of the first round of RING phases, whole rounds, then the remainder
  // (phases continue from 0, the phase after a whole round)
  march(Phase<0>{}, W{}); march(Phase<1>{}, W{}); march(Phase<2>{}, W{});
  march(Phase<3>{}, W{}); march(Phase<4>{}, W{}); march(Phase<5>{}, W{});
  int left = x1 - x0;
  march_upto<6, RING>(march, left);
  left -= min(left, RING - 6);
  for (; left >= RING; left -= RING) march_all<0, RING>(march);
  march_upto<0, RING>(march, left);
}

// Waves per SIMD that the tiling's LDS allows on a CU (160 KiB of LDS, four
// SIMDs), capped at 4: the register budget the kernel is compiled for.
template <typename T, int TY, int TZ, int NT>
constexpr int fused_waves_per_simd() {
  constexpr long long lds = (2LL * 4 * (TY + 2 * kFusedHalo) * (TZ + 2 * kFusedHalo) +
                             2LL * (kMaxChunk + 10)) * (long long)sizeof(T);
  constexpr long long wgs = (160LL * 1024) / lds;
  constexpr long long w = wgs * (NT / 64) / 4;
  return w < 1 ? 1 : (w > 4 ? 4 : (int)w);
}

// TY x TZ output tile per workgroup of NT threads; the region with the
// 4-layer halo has (TY + 8) x (TZ + 8) columns.
template <typename T, int TY, int TZ, int NT, int RING>
__global__ __launch_bounds__(NT, (fused_waves_per_simd<T, TY, TZ, NT>())) void k_rk4_fused(const FineDesc<T>* __restrict__ descs, int nd,
                                                  int step, long long total, long long per_xcd) {
  constexpr int NR = (TY + 2 * kFusedHalo) * (TZ + 2 * kFusedHalo);
  // two sets of the four stage planes, alternating per march step, so one
  // barrier per step suffices (a set is rewritten two steps later, after
  // every thread has passed the intermediate barrier)
  __shared__ T lds[2][4][NR];
  // v_y(x) and v_z(x) parts of the velocity for the chunk's planes
  // x0 - 6 .. x0 + kMaxChunk + 3
  __shared__ T vxt[2][kMaxChunk + 10];

  // blocks b, b + 8, b + 16, ... run on one XCD: give them consecutive tiles
  const long long b = blockIdx.x;
  const long long t = (b % 8) * per_xcd + b / 8;
  if (t >= total) return;
  const int f = find_desc(descs, nd, t);
  const FineDesc<T>& d = descs[f];
  if (step >= d.n_steps) return;
  if (d.g.xonly)
    rk4_tile<T, TY, TZ, NT, true, RING>(d, step, t - d.tile_begin, lds, vxt);
  else
    rk4_tile<T, TY, TZ, NT, false, RING>(d, step, t - d.tile_begin, lds, vxt);
}

// Launch of one fused step in tile configuration cfg (kFusedCfgs).
// The y ring of six planes (one step of prefetch): a ring of twelve measured
// 5 % slower on 63 x 128^3 FP64 in the tiling with two columns per thread
// (spills) and 13 % faster only in the one-column tiling.
constexpr int kFusedRing = 6;

template <typename T, int TY, int TZ, int NT>
static void launch_cfg(const FineDesc<T>* d, int nd, long long total, int step, hipStream_t s) {
  const long long g8 = (total + 7) / 8 * 8;
  hipLaunchKernelGGL((k_rk4_fused<T, TY, TZ, NT, kFusedRing>), dim3((unsigned)g8), dim3(NT), 0, s,
                     d, nd, step, total, g8 / 8);
}

template <typename T>
static void launch_step_impl(const FineDesc<T>* d, int nd, long long total, int step, int cfg,
                             hipStream_t s) {
  if (total <= 0) return;
  static_assert(kNumColumnCfgs == 8, "one case per configuration");
  switch (cfg) {
    case 0: launch_cfg<T, 32, 32, 512>(d, nd, total, step, s); break;
    case 1: launch_cfg<T, 16, 32, 256>(d, nd, total, step, s); break;
    case 2: launch_cfg<T, 16, 32, 512>(d, nd, total, step, s); break;
    case 3: launch_cfg<T, 32, 32, 1024>(d, nd, total, step, s); break;
    case 4: launch_cfg<T, 8, 32, 256>(d, nd, total, step, s); break;
    case 5: launch_cfg<T, 16, 64, 512>(d, nd, total, step, s); break;
    case 6: launch_cfg<T, 8, 64, 512>(d, nd, total, step, s); break;
    case 7: launch_cfg<T, 16, 32, 1024>(d, nd, total, step, s); break;
    default: fail(PR_EINVAL, "unknown fused stencil configuration");
  }
}

template <typename T, int TY, int TZ, int NT>
static int occ_cfg() {
  int n = 0;
  PR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_rk4_fused<T, TY, TZ, NT, kFusedRing>,
                                                       NT, 0));
  return n;
}

template <typename T>
static int occ_impl(int cfg) {
  switch (cfg) {
    case 0: return occ_cfg<T, 32, 32, 512>();
    case 1: return occ_cfg<T, 16, 32, 256>();
    case 2: return occ_cfg<T, 16, 32, 512>();
    case 3: return occ_cfg<T, 32, 32, 1024>();
    case 4: return occ_cfg<T, 8, 32, 256>();
    case 5: return occ_cfg<T, 16, 64, 512>();
    case 6: return occ_cfg<T, 8, 64, 512>();
    case 7: return occ_cfg<T, 16, 32, 1024>();
    default: fail(PR_EINVAL, "unknown fused stencil configuration");
  }
  return 0;
}

int fused_blocks_per_cu(int cfg, bool f32, bool xonly) {
  if (kFusedCfgs[cfg].blocked) return b22_blocks_per_cu(cfg, f32, xonly);
  return f32 ? occ_impl<float>(cfg) : occ_impl<double>(cfg);
}

void launch_fine_step_f64(const FineDesc<double>* d, int nd, long long total, int step, int cfg,
                          bool xonly, hipStream_t s) {
  if (kFusedCfgs[cfg].blocked) return launch_b22_step_f64(d, nd, total, step, cfg, xonly, s);
  launch_step_impl<double>(d, nd, total, step, cfg, s);
  PR_HIP(hipGetLastError());
}
void launch_fine_step_f32(const FineDesc<float>* d, int nd, long long total, int step, int cfg,
                          bool xonly, hipStream_t s) {
  if (kFusedCfgs[cfg].blocked) return launch_b22_step_f32(d, nd, total, step, cfg, xonly, s);
  launch_step_impl<float>(d, nd, total, step, cfg, s);
  PR_HIP(hipGetLastError());
}

void launch_fine_f64(const FineDesc<double>* d, int nd, long long total, int max_steps, int cfg,
                     bool xonly, hipStream_t s) {
  for (int step = 0; step < max_steps; ++step)
    launch_fine_step_f64(d, nd, total, step, cfg, xonly, s);
}
void launch_fine_f32(const FineDesc<float>* d, int nd, long long total, int max_steps, int cfg,
                     bool xonly, hipStream_t s) {
  for (int step = 0; step < max_steps; ++step)
    launch_fine_step_f32(d, nd, total, step, cfg, xonly, s);
}

// out = L(in) for each valid column; invalid columns are written as zero.
template <typename T>
__global__ __launch_bounds__(kTileQ) void k_apply_L(const ApplyLDesc<T>* __restrict__ descs,
                                                    int nd) {
  const long long t = blockIdx.x;
  const int f = find_desc(descs, nd, t);
  const ApplyLDesc<T> d = descs[f];
  const long long lt = t - d.tile_begin;
  const int per_col = d.tiles_q * d.tiles_x;
  const int col = (int)(lt / per_col);
  const int r = (int)(lt - (long long)col * per_col);
  const int tq = r % d.tiles_q, tx = r / d.tiles_q;
  const int n = d.g.n;
  const int q = tq * kTileQ + threadIdx.x;
  if (q >= n * n) return;
  const int j = q / n, k = q - (q / n) * n;
  const int x0 = tx * d.chunk_x, x1 = min(n, x0 + d.chunk_x);
  const PR_GLOBAL T* in = gptr(d.in) + (long long)col * d.ld;
  PR_GLOBAL T* out = gptr(d.out) + (long long)col * d.ld;
  const bool valid = (d.mptr == nullptr) || (col < *d.mptr);
  if (!valid) {
    if (d.skip_tail) return;
    const long long plane = (long long)n * n;
    for (int x = x0; x < x1; ++x) out[(long long)x * plane + q] = (T)0;
    return;
  }
  march_L<T>(d.g, in, j, k, x0, x1, [&](int, long long p, T Lv) { out[p] = Lv; });
}

// out = L(in) through an LDS window of each plane, for kWinMinN <= n <=
// kWinMaxN (a window index then wraps at most once either way). A workgroup
// owns kWinQ consecutive points q = j n + k of the (y, z) plane and marches
// along x. Plane x's window holds the points q0 - n .. q0 + kWinQ + n
// (periodic in q), which covers every y and z neighbour of the owned points,
// so a point costs (kWinQ + 2 n) / kWinQ loads instead of five. Two window
// buffers hold planes x and x + 1; plane x + 2 is loaded into registers while
// plane x is computed. Same arithmetic per point as k_apply_L.
template <typename T>
__global__ __launch_bounds__(256) void k_apply_L_win(const ApplyLDesc<T>* __restrict__ descs,
                                                     int nd) {
  constexpr int U = kWinQ / 256;                      // points per thread
  constexpr int NW = (kWinQ + 2 * kWinMaxN + 255) / 256;   // window loads per thread (at most)
  __shared__ T win[2][kWinQ + 2 * kWinMaxN];
  const long long t = blockIdx.x;
  const int f = find_desc(descs, nd, t);
  const ApplyLDesc<T> d = descs[f];
  const long long lt = t - d.tile_begin;
  const int per_col = d.tiles_q * d.tiles_x;
  const int col = (int)(lt / per_col);
  const int r = (int)(lt - (long long)col * per_col);
  const int tq = r % d.tiles_q, tx = r / d.tiles_q;
  const int n = d.g.n;
  const int plane = n * n;
  const int tid = threadIdx.x;
  const int q0 = tq * kWinQ;
  const int x0 = tx * d.chunk_x, x1 = min(n, x0 + d.chunk_x);
  const PR_GLOBAL T* in = gptr(d.in) + (long long)col * d.ld;
  PR_GLOBAL T* out = gptr(d.out) + (long long)col * d.ld;
  const bool valid = (d.mptr == nullptr) || (col < *d.mptr);
  if (!valid) {
    if (d.skip_tail) return;
    for (int u = 0; u < U; ++u) {
      const int q = q0 + tid + 256 * u;
      if (q < plane)
        for (int x = x0; x < x1; ++x) out[(long long)x * plane + q] = (T)0;
    }
    return;
  }
  const PR_GLOBAL T* tab = gptr(tab_of<T>(d.g));
  const T clap = (T)d.g.c_lap;
  const int W = kWinQ + 2 * n;
  // this thread's points: window index of the centre and of the z neighbours
  bool ok[U];
  int q[U], wc[U], wzm[U], wzp[U];
  T vx[U], vyz[U], vzy[U], cm[U];
  const int xm0 = (x0 == 0) ? n - 1 : x0 - 1;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int l = tid + 256 * u;
    q[u] = q0 + l;
    ok[u] = q[u] < plane;
    const int qq = ok[u] ? q[u] : 0;
    const int j = qq / n, k = qq - j * n;
    wc[u] = n + l;
    wzm[u] = (k > 0) ? wc[u] - 1 : wc[u] + n - 1;
    wzp[u] = (k < n - 1) ? wc[u] + 1 : wc[u] - (n - 1);
    vx[u] = tab[0 * n + j] + tab[1 * n + k];
    vyz[u] = tab[3 * n + k];
    vzy[u] = tab[5 * n + j];
    cm[u] = ok[u] ? in[(long long)xm0 * plane + qq] : (T)0;
  }
  T reg[NW];
  auto load = [&](int x) {
    const PR_GLOBAL T* p = in + (long long)x * plane;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const int w = tid + 256 * i;
      int qq = q0 - n + w;
      qq = qq < 0 ? qq + plane : (qq >= plane ? qq - plane : qq);
      reg[i] = w < W ? p[qq] : (T)0;
    }
  };
  auto store = [&](int b) {
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const int w = tid + 256 * i;
      if (w < W) win[b][w] = reg[i];
    }
  };
  load(x0);
  store(0);
  load(x0 == n - 1 ? 0 : x0 + 1);
  store(1);
  __syncthreads();
  for (int x = x0; x < x1; ++x) {
    const int cur = (x - x0) & 1, nxt = cur ^ 1;
    const bool more = x + 1 < x1;   // plane x + 1 is computed, so plane x + 2 is needed
    if (more) load(x + 2 >= n ? x + 2 - n : x + 2);
    const T ty = tab[2 * n + x], tz = tab[4 * n + x];
    const T* wcur = win[cur];
    const T* wnxt = win[nxt];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!ok[u]) continue;
      const T c0 = wcur[wc[u]];
      const T Lv = l_point<T>(cm[u], c0, wnxt[wc[u]], wcur[wc[u] - n], wcur[wc[u] + n],
                              wcur[wzm[u]], wcur[wzp[u]], vx[u], ty + vyz[u], tz + vzy[u], clap);
      out[(long long)x * plane + q[u]] = Lv;
      cm[u] = c0;
    }
    if (more) {
      __syncthreads();   // every read of plane x's window is done
      store(cur);
      __syncthreads();
    }
  }
}

void launch_applyL_f64(const ApplyLDesc<double>* d, int nd, long long tt, bool win,
                       hipStream_t s) {
  if (tt <= 0) return;
  if (win)
    hipLaunchKernelGGL(k_apply_L_win<double>, dim3((unsigned)tt), dim3(256), 0, s, d, nd);
  else
    hipLaunchKernelGGL(k_apply_L<double>, dim3((unsigned)tt), dim3(kTileQ), 0, s, d, nd);
  PR_HIP(hipGetLastError());
}
void launch_applyL_f32(const ApplyLDesc<float>* d, int nd, long long tt, bool win,
                       hipStream_t s) {
  if (tt <= 0) return;
  if (win)
    hipLaunchKernelGGL(k_apply_L_win<float>, dim3((unsigned)tt), dim3(256), 0, s, d, nd);
  else
    hipLaunchKernelGGL(k_apply_L<float>, dim3((unsigned)tt), dim3(kTileQ), 0, s, d, nd);
  PR_HIP(hipGetLastError());
}

__global__ void k_f64_to_f32(const double* __restrict__ in, float* __restrict__ out, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}
__global__ void k_f32_to_f64(const float* __restrict__ in, double* __restrict__ out, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = (double)in[i];
}

static unsigned grid_for(long long n) {
  long long g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  return (unsigned)(g < 1 ? 1 : g);
}

void launch_convert_f64_to_f32(const double* in, float* out, long long n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_f64_to_f32, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
  PR_HIP(hipGetLastError());
}
void launch_convert_f32_to_f64(const float* in, double* out, long long n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_f32_to_f64, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
  PR_HIP(hipGetLastError());
}

__global__ void k_scale_into(const double* __restrict__ in, void* out, int out_f32, long long n,
                             const double* __restrict__ scale) {
  const double a = *scale;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double v = a * in[i];
    if (out_f32) ((float*)out)[i] = (float)v;
    else ((double*)out)[i] = v;
  }
}
void launch_scale_into(const double* in, void* out, int out_f32, long long n, const double* scale,
                       hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scale_into, dim3(grid_for(n)), dim3(256), 0, s, in, out, out_f32, n, scale);
  PR_HIP(hipGetLastError());
}

}  // namespace pr
