// Fine propagator kernels: RK4 stages of the periodic FD advection-diffusion
// operator, batched over fields of different sizes in one launch per stage.
//
// For the linear autonomous operator L one classical RK4 step is
// P4(dt L) y with P4(z) = 1 + z + z^2/2 + z^3/6 + z^4/24, evaluated here in
// Horner form as four stencil sweeps that all use y as base:
//   w1 = y + dt/4 L y,  w2 = y + dt/3 L w1,  w3 = y + dt/2 L w2,
//   y <- y + dt L w3.
// Stage traffic per grid point: read y (and the previous stage), write one
// field. Each thread owns one (y, z) column of a tile and marches along x,
// keeping the x-1, x, x+1 values of the stage input in registers; the y and
// z neighbours come from the L1/L2 caches (z fastest, so a tile's z rows are
// 256 consecutive points and fully coalesced).
#include "pr_internal.h"

namespace pr {

template <typename T>
__device__ __forceinline__ const T* tab_of(const Geom& g);
template <>
__device__ __forceinline__ const double* tab_of<double>(const Geom& g) { return g.tab64; }
template <>
__device__ __forceinline__ const float* tab_of<float>(const Geom& g) { return g.tab32; }

// Locate the descriptor owning global tile `t` (descriptors sorted by
// tile_begin): binary search over uniform data.
template <typename D>
__device__ __forceinline__ int find_desc(const D* d, int nd, long long t) {
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].tile_begin <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Evaluate (L in) along x for one (j, k) column over planes [x0, x1),
// calling emit(x, p, Lv) for each plane. Periodic wrap on every axis.
template <typename T, typename Emit>
__device__ __forceinline__ void march_L(const Geom& g, const T* __restrict__ in, int j, int k,
                                        int x0, int x1, Emit emit) {
  const int n = g.n;
  const long long plane = (long long)n * n;
  const T* tab = tab_of<T>(g);
  const T clap = (T)g.c_lap;
  const int jm = (j == 0) ? n - 1 : j - 1, jp = (j == n - 1) ? 0 : j + 1;
  const int km = (k == 0) ? n - 1 : k - 1, kp = (k == n - 1) ? 0 : k + 1;
  const T vx = tab[0 * n + j] + tab[1 * n + k];
  const T vy_z = tab[3 * n + k];
  const T vz_y = tab[5 * n + j];
  const int q = j * n + k;
  const int xm0 = (x0 == 0) ? n - 1 : x0 - 1;
  T cm = in[(long long)xm0 * plane + q];
  T c0 = in[(long long)x0 * plane + q];
  for (int x = x0; x < x1; ++x) {
    const int xp = (x == n - 1) ? 0 : x + 1;
    const long long base = (long long)x * plane;
    const T cp = in[(long long)xp * plane + q];
    const T ym = in[base + jm * n + k];
    const T yp = in[base + jp * n + k];
    const T zm = in[base + j * n + km];
    const T zp = in[base + j * n + kp];
    const T vy = tab[2 * n + x] + vy_z;
    const T vz = tab[4 * n + x] + vz_y;
    const T lap = ((cp + cm) + (yp + ym) + (zp + zm)) - (T)6 * c0;
    const T adv = vx * (cp - cm) + vy * (yp - ym) + vz * (zp - zm);
    emit(x, base + q, clap * lap - adv);
    cm = c0;
    c0 = cp;
  }
}

// One RK4 stage for every field of the batch with step < n_steps.
template <typename T>
__global__ __launch_bounds__(kTileQ) void k_fine_stage(const FineDesc<T>* __restrict__ descs,
                                                       int nd, int step, int stage) {
  const long long t = blockIdx.x;
  const int f = find_desc(descs, nd, t);
  const FineDesc<T> d = descs[f];
  if (step >= d.n_steps) return;
  const long long lt = t - d.tile_begin;
  const int tq = (int)(lt % d.tiles_q);
  const int tx = (int)(lt / d.tiles_q);
  const int n = d.g.n;
  const int q = tq * kTileQ + threadIdx.x;
  if (q >= n * n) return;
  const int j = q / n, k = q - (q / n) * n;
  const int x0 = tx * kChunkX;
  const int x1 = min(n, x0 + kChunkX);
  const T* in;
  T* out;
  T coef;
  const T dt = (T)d.dt;
  switch (stage) {
    case 0: in = d.y;  out = d.wa; coef = dt * (T)0.25; break;
    case 1: in = d.wa; out = d.wb; coef = dt / (T)3; break;
    case 2: in = d.wb; out = d.wa; coef = dt * (T)0.5; break;
    default: in = d.wa; out = d.y; coef = dt; break;
  }
  const T* y = d.y;
  const bool snap = (stage == 3) && d.snaps != nullptr && ((step + 1) % d.snap_every == 0);
  const long long ng = (long long)n * n * n;
  T* snapcol = snap ? d.snaps + (long long)((step + 1) / d.snap_every) * ng : nullptr;
  march_L<T>(d.g, in, j, k, x0, x1, [&](int, long long p, T Lv) {
    const T v = y[p] + coef * Lv;
    out[p] = v;
    if (snap) snapcol[p] = v;
  });
}

template <typename T>
static void launch_fine_impl(const FineDesc<T>* d, int nd, long long total_tiles, int max_steps,
                             hipStream_t s) {
  if (total_tiles <= 0) return;
  for (int step = 0; step < max_steps; ++step)
    for (int stage = 0; stage < 4; ++stage)
      hipLaunchKernelGGL(k_fine_stage<T>, dim3((unsigned)total_tiles), dim3(kTileQ), 0, s, d, nd,
                         step, stage);
  PR_HIP(hipGetLastError());
}

void launch_fine_f64(const FineDesc<double>* d, int nd, long long tt, int ms, hipStream_t s) {
  launch_fine_impl<double>(d, nd, tt, ms, s);
}
void launch_fine_f32(const FineDesc<float>* d, int nd, long long tt, int ms, hipStream_t s) {
  launch_fine_impl<float>(d, nd, tt, ms, s);
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
  const int x0 = tx * kChunkX, x1 = min(n, x0 + kChunkX);
  const long long ng = (long long)n * n * n;
  const T* in = d.in + (long long)col * ng;
  T* out = d.out + (long long)col * ng;
  const bool valid = (d.mptr == nullptr) || (col < *d.mptr);
  if (!valid) {
    const long long plane = (long long)n * n;
    for (int x = x0; x < x1; ++x) out[(long long)x * plane + q] = (T)0;
    return;
  }
  march_L<T>(d.g, in, j, k, x0, x1, [&](int, long long p, T Lv) { out[p] = Lv; });
}

void launch_applyL_f64(const ApplyLDesc<double>* d, int nd, long long tt, hipStream_t s) {
  if (tt <= 0) return;
  hipLaunchKernelGGL(k_apply_L<double>, dim3((unsigned)tt), dim3(kTileQ), 0, s, d, nd);
  PR_HIP(hipGetLastError());
}
void launch_applyL_f32(const ApplyLDesc<float>* d, int nd, long long tt, hipStream_t s) {
  if (tt <= 0) return;
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
