// Fine propagator kernel of the forced flows of Sec. 4 (time-dependent
// velocity and forcing) and the forcing fields of their time-space pieces.
#include <type_traits>

#include "pr_internal.h"
#include "stencil_dev.h"

namespace pr {

// Fused RK4 step for the forced flows: du/dt = L(t) u + f(t). One classical
// RK4 step from t, with stage times t, t + dt/2, t + dt/2, t + dt:
//   k1 = L(t) y + f(t),                 w1 = y + dt/2 k1
//   k2 = L(t + dt/2) w1 + f(t + dt/2),  w2 = y + dt/2 k2
//   k3 = L(t + dt/2) w2 + f(t + dt/2),  w3 = y + dt k3
//   k4 = L(t + dt) w3 + f(t + dt),      y_new = y + dt/6 (k1 + 2 k2 + 2 k3 + k4)
// The operators differ per stage, so the Horner form of the steady kernel
// does not apply; the stages keep the same skewed pipeline along x and add an
// accumulator per plane, A = dt/2 (k1 + 2 k2 + 2 k3), started at stage 2 as
// (w1 - y) + dt k2 (w1 - y = dt/2 k1) and completed by stage 3, so that
// y_new = y + (A + dt/2 k4) / 3. A lives from stage 2 to stage 4 of its
// plane (three march steps): a ring of three registers per column.
// The velocity and forcing at each of the three stage times are formed once
// per workgroup: their (y, z) parts per column in registers, their x parts
// per plane in LDS.
template <typename T>
__device__ __forceinline__ const T* ptab_of(const Geom& g);
template <>
__device__ __forceinline__ const double* ptab_of<double>(const Geom& g) { return g.ptab64; }
template <>
__device__ __forceinline__ const float* ptab_of<float>(const Geom& g) { return g.ptab32; }

template <typename T, int TY, int TZ, int NT>
__device__ __forceinline__ void rk4_tile_forced(
    const FineDesc<T>& d, int step, long long lt,
    T (*lds)[4][(TY + 2 * kFusedHalo) * (TZ + 2 * kFusedHalo)], T (*xt)[kForcedChunk + 10],
    T (*thl)[kMaxPieces]) {
#pragma clang fp contract(off)
  constexpr int H = kFusedHalo;
  constexpr int RY = TY + 2 * H, RZ = TZ + 2 * H;
  constexpr int NR = RY * RZ;
  constexpr int SL = (NR + NT - 1) / NT;
  constexpr int NI = TY * TZ;
  constexpr int RING = 6;
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
  const PR_GLOBAL T* pt = gptr(ptab_of<T>(d.g));
  const int np = d.g.npieces;
  const long long pstride = 9LL * n;
  const T clap = (T)d.g.c_lap;
  const T dt = (T)d.dt;
  const T hdt = dt * (T)0.5;
  const T third = (T)1 / (T)3;

  // theta_j at the stage times t, t + dt/2, t + dt, evaluated once per
  // workgroup (forcing weights zero for the homogeneous propagator)
  if (threadIdx.x < 3 * kMaxPieces) {
    const int a = threadIdx.x / kMaxPieces, j = threadIdx.x % kMaxPieces;
    const double t = d.t0 + (double)step * d.dt;
    const double ta = (a == 0) ? t : (a == 1 ? t + 0.5 * d.dt : t + d.dt);
    thl[a][j] = j < np ? (T)theta_of(d.g.forced, d.g.w, j, ta) : (T)0;
  }
  __syncthreads();
  T th[3][kMaxPieces], tf[3][kMaxPieces];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int j = 0; j < kMaxPieces; ++j) {
      const T v = thl[a][j];
      th[a][j] = v;
      tf[a][j] = d.with_forcing ? v : (T)0;
    }
  }
  // sum_j theta_j table_j[i] in a fixed order
  auto mix = [&](const T* w, int tab, int i) {
    T acc = (T)0;
    for (int j = 0; j < np; ++j) acc = fma(w[j], pt[j * pstride + (long long)tab * n + i], acc);
    return acc;
  };

  int ci[SL];
  int off[SL];
  int lev[SL];
  bool outp[SL];
  // per column and stage time: v_x, the z part of v_y, the y part of v_z and
  // the (y, z) part of f
  T vx[SL][3], vyz[SL][3], vzy[SL][3], fyz[SL][3];
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
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      vx[s][a] = mix(th[a], 0, gy) + mix(th[a], 1, gz);
      vyz[s][a] = mix(th[a], 3, gz);
      vzy[s][a] = mix(th[a], 5, gy);
      fyz[s][a] = mix(tf[a], 7, gy) + mix(tf[a], 8, gz);
    }
  }
  // per plane x0 - 6 .. and stage time a: xt[3a] = v_y x part, xt[3a + 1] =
  // v_z x part, xt[3a + 2] = f x part
  for (int i = threadIdx.x; i < x1 - x0 + 10; i += NT) {
    const int x = wrapi(x0 - 6 + i, n);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      xt[3 * a][i] = mix(th[a], 2, x);
      xt[3 * a + 1][i] = mix(th[a], 4, x);
      xt[3 * a + 2][i] = mix(tf[a], 6, x);
    }
  }

  // Rings as in rk4_tile; A: A(tt + k), k = 0..2, at (k + ph) % 3.
  T Y[SL][RING], W1[SL][3], W2[SL][3], W3[SL][3], A[SL][3];
#pragma unroll
  for (int s = 0; s < SL; ++s) {
#pragma unroll
    for (int k = 0; k < RING; ++k) Y[s][k] = (T)0;
#pragma unroll
    for (int k = 0; k < 3; ++k) W1[s][k] = W2[s][k] = W3[s][k] = A[s][k] = (T)0;
  }
  {
    const long long pa = (long long)wrapi(x0 - 4, n) * plane;
    const long long pb = (long long)wrapi(x0 - 3, n) * plane;
    const long long pc = (long long)wrapi(x0 - 2, n) * plane;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      Y[s][2] = src[pa + off[s]];
      Y[s][3] = src[pb + off[s]];
      Y[s][4] = src[pc + off[s]];
    }
  }
  long long o5 = (long long)wrapi(x0 - 1, n) * plane;
  long long od = (long long)wrapi(x0 - 6, n) * plane;
  const long long ng = plane * n;
  int tt = x0 - 6;

  auto march = [&](auto phase, auto warm) {
    constexpr int PH = decltype(phase)::value;
    constexpr bool WARM = decltype(warm)::value;
    constexpr bool s2 = !WARM || PH >= 2, s3 = !WARM || PH >= 4, s4 = !WARM;
    __builtin_amdgcn_sched_barrier(0);
    constexpr int k0 = PH % RING, k1 = (1 + PH) % RING, k2 = (2 + PH) % RING,
                  k3 = (3 + PH) % RING, k4 = (4 + PH) % RING, k5 = (5 + PH) % RING;
    constexpr int j0 = PH % 3, j1 = (1 + PH) % 3, j2 = (2 + PH) % 3;
    T (*pl)[NR] = lds[PH & 1];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      const bool inner = (s + 1) * NT <= NI;
      Y[s][k5] = src[o5 + off[s]];
      if (inner || lev[s] <= H) pl[0][ci[s]] = Y[s][k3];
      if (inner || lev[s] <= H - 1) pl[1][ci[s]] = W1[s][j1];
      if (inner || lev[s] <= H - 2) pl[2][ci[s]] = W2[s][j1];
      if (inner || lev[s] <= H - 3) pl[3][ci[s]] = W3[s][j1];
    }
    __syncthreads();
    const int iv = tt - (x0 - 6);
    // x parts: stage 1 at plane tt + 3 (time a = 0), stages 2 and 3 at
    // tt + 2 and tt + 1 (a = 1), stage 4 at tt (a = 2)
    const T vy1 = xt[0][iv + 3], vz1 = xt[1][iv + 3], f1 = xt[2][iv + 3];
    const T vy2 = xt[3][iv + 2], vz2 = xt[4][iv + 2], f2 = xt[5][iv + 2];
    const T vy3 = xt[3][iv + 1], vz3 = xt[4][iv + 1], f3 = xt[5][iv + 1];
    const T vy4 = xt[6][iv], vz4 = xt[7][iv], f4 = xt[8][iv];
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      const bool inner = (s + 1) * NT <= NI;
      const int c = ci[s];
      const int lv = lev[s];
      T w1 = (T)0, w2 = (T)0, w3 = (T)0, a2 = (T)0, a3 = (T)0;
      if (inner || lv <= H - 1) {
        const T k1 = lop<T, RZ>(Y[s][k2], Y[s][k3], Y[s][k4], pl[0], c, clap, vx[s][0],
                                vy1 + vyz[s][0], vz1 + vzy[s][0]) + (f1 + fyz[s][0]);
        w1 = fma(hdt, k1, Y[s][k3]);
      }
      W1[s][j2] = w1;
      if (s2 && (inner || lv <= H - 2)) {
        const T k2v = lop<T, RZ>(W1[s][j0], W1[s][j1], W1[s][j2], pl[1], c, clap, vx[s][1],
                                 vy2 + vyz[s][1], vz2 + vzy[s][1]) + (f2 + fyz[s][1]);
        w2 = fma(hdt, k2v, Y[s][k2]);
        a2 = fma(dt, k2v, W1[s][j1] - Y[s][k2]);
      }
      W2[s][j2] = w2;
      A[s][j2] = a2;
      if (s3 && (inner || lv <= H - 3)) {
        const T k3v = lop<T, RZ>(W2[s][j0], W2[s][j1], W2[s][j2], pl[2], c, clap, vx[s][1],
                                 vy3 + vyz[s][1], vz3 + vzy[s][1]) + (f3 + fyz[s][1]);
        w3 = fma(dt, k3v, Y[s][k1]);
        a3 = fma(dt, k3v, A[s][j1]);
      }
      W3[s][j2] = w3;
      A[s][j1] = a3;
      if (s4 && outp[s]) {
        const T k4v = lop<T, RZ>(W3[s][j0], W3[s][j1], W3[s][j2], pl[3], c, clap, vx[s][2],
                                 vy4 + vyz[s][2], vz4 + vzy[s][2]) + (f4 + fyz[s][2]);
        const T yn = fma(fma(hdt, k4v, A[s][j0]), third, Y[s][k0]);
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
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;
  using I4 = std::integral_constant<int, 4>;
  using I5 = std::integral_constant<int, 5>;
  using W = std::true_type;
  using S = std::false_type;

  __syncthreads();   // xt visible
  march(I0{}, W{}); march(I1{}, W{}); march(I2{}, W{});
  march(I3{}, W{}); march(I4{}, W{}); march(I5{}, W{});
  const int nstep = x1 - x0;
  for (int r = 0; r + RING <= nstep; r += RING) {
    march(I0{}, S{}); march(I1{}, S{}); march(I2{}, S{});
    march(I3{}, S{}); march(I4{}, S{}); march(I5{}, S{});
  }
  const int rem = nstep % RING;
  if (rem > 0) march(I0{}, S{});
  if (rem > 1) march(I1{}, S{});
  if (rem > 2) march(I2{}, S{});
  if (rem > 3) march(I3{}, S{});
  if (rem > 4) march(I4{}, S{});
}

template <typename T, int TY, int TZ, int NT>
constexpr int forced_waves_per_simd() {
  constexpr long long lds = (2LL * 4 * (TY + 2 * kFusedHalo) * (TZ + 2 * kFusedHalo) +
                             9LL * (kForcedChunk + 10)) * (long long)sizeof(T);
  constexpr long long wgs = (160LL * 1024) / lds;
  constexpr long long w = wgs * (NT / 64) / 4;
  // registers: FP64 keeps every column's rings and coefficients resident at
  // two waves per SIMD (more would spill)
  constexpr int cap = sizeof(T) == 8 ? 2 : 3;
  return w < 1 ? 1 : (w > cap ? cap : (int)w);
}

template <typename T, int TY, int TZ, int NT>
__global__ __launch_bounds__(NT, (forced_waves_per_simd<T, TY, TZ, NT>())) void k_rk4_forced(
    const FineDesc<T>* __restrict__ descs, int nd, int step, long long total, long long per_xcd) {
  constexpr int NR = (TY + 2 * kFusedHalo) * (TZ + 2 * kFusedHalo);
  __shared__ T lds[2][4][NR];
  __shared__ T xt[9][kForcedChunk + 10];
  __shared__ T thl[3][kMaxPieces];
  const long long b = blockIdx.x;
  const long long t = (b % 8) * per_xcd + b / 8;
  if (t >= total) return;
  const int f = find_desc(descs, nd, t);
  const FineDesc<T>& d = descs[f];
  if (step >= d.n_steps) return;
  rk4_tile_forced<T, TY, TZ, NT>(d, step, t - d.tile_begin, lds, xt, thl);
}

template <typename T, int TY, int TZ, int NT>
static void launch_forced_cfg(const FineDesc<T>* d, int nd, long long total, int step,
                              hipStream_t s) {
  const long long g8 = (total + 7) / 8 * 8;
  hipLaunchKernelGGL((k_rk4_forced<T, TY, TZ, NT>), dim3((unsigned)g8), dim3(NT), 0, s, d, nd,
                     step, total, g8 / 8);
}

template <typename T>
static void launch_forced_impl(const FineDesc<T>* d, int nd, long long total, int step, int cfg,
                               hipStream_t s) {
  if (total <= 0) return;
  static_assert(kNumForcedCfgs == 5, "one case per forced configuration");
  switch (cfg) {
    case 2: launch_forced_cfg<T, 16, 32, 512>(d, nd, total, step, s); break;
    case 3: launch_forced_cfg<T, 32, 32, 1024>(d, nd, total, step, s); break;
    case 4: launch_forced_cfg<T, 8, 32, 256>(d, nd, total, step, s); break;
    case 6: launch_forced_cfg<T, 8, 64, 512>(d, nd, total, step, s); break;
    case 7: launch_forced_cfg<T, 16, 32, 1024>(d, nd, total, step, s); break;
    default: fail(PR_EINVAL, "tiling not available for the forced-flow stencil");
  }
}

template <typename T, int TY, int TZ, int NT>
static int occ_forced_cfg() {
  int n = 0;
  PR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_rk4_forced<T, TY, TZ, NT>, NT, 0));
  return n;
}

template <typename T>
static int occ_forced_impl(int cfg) {
  switch (cfg) {
    case 2: return occ_forced_cfg<T, 16, 32, 512>();
    case 3: return occ_forced_cfg<T, 32, 32, 1024>();
    case 4: return occ_forced_cfg<T, 8, 32, 256>();
    case 6: return occ_forced_cfg<T, 8, 64, 512>();
    case 7: return occ_forced_cfg<T, 16, 32, 1024>();
    default: fail(PR_EINVAL, "tiling not available for the forced-flow stencil");
  }
  return 0;
}

int forced_blocks_per_cu(int cfg, bool f32) {
  return f32 ? occ_forced_impl<float>(cfg) : occ_forced_impl<double>(cfg);
}

void launch_forced_step_f64(const FineDesc<double>* d, int nd, long long total, int step, int cfg,
                            hipStream_t s) {
  launch_forced_impl<double>(d, nd, total, step, cfg, s);
  PR_HIP(hipGetLastError());
}
void launch_forced_step_f32(const FineDesc<float>* d, int nd, long long total, int step, int cfg,
                            hipStream_t s) {
  launch_forced_impl<float>(d, nd, total, step, cfg, s);
  PR_HIP(hipGetLastError());
}

// f_j(x, y, z) = t[6][x] + t[7][y] + t[8][z] of piece j as a field.
__global__ void k_forcing_field(const double* __restrict__ pt, int n, void* out, int out_f32) {
  const long long ng = (long long)n * n * n;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < ng;
       p += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(p % n), j = (int)((p / n) % n), i = (int)(p / ((long long)n * n));
    const double v = (pt[6 * n + i] + pt[7 * n + j]) + pt[8 * n + k];
    if (out_f32) ((float*)out)[p] = (float)v;
    else ((double*)out)[p] = v;
  }
}

void launch_forcing_field(const Geom& g, int piece, void* out, int out_f32, hipStream_t s) {
  const long long ng = (long long)g.n * g.n * g.n;
  long long blocks = (ng + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_forcing_field, dim3((unsigned)blocks), dim3(256), 0, s,
                     g.ptab64 + 9LL * g.n * piece, g.n, out, out_f32);
  PR_HIP(hipGetLastError());
}

}  // namespace pr
