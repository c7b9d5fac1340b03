// Grid transfers of the coarse-grid coarse propagator (the comparison method
// "Parareal-II" of Sec. 4, which solves the same equation on a coarser
// mesh): the n/2 node-centred grid of the same periodic box, coarse node I
// on fine node 2I.
//
//   restriction (full weighting), per axis
//       c[I] = 1/4 f[2I - 1] + 1/2 f[2I] + 1/4 f[2I + 1]
//   prolongation (linear interpolation), per axis
//       f[2I] = c[I],  f[2I + 1] = (c[I] + c[I + 1]) / 2
//
// both periodic and separable (trilinear in 3-D). k_restrict restricts the
// difference of two fine fields (the coarse propagator is linear, so the
// parareal correction needs G(U^k_n) - G(U^{k-1}_n) = G(U^k_n - U^{k-1}_n));
// k_prolong_add writes P(c) + F with the jump and error partials of the
// correction kernel.
#include "pr_internal.h"

namespace pr {

__device__ __forceinline__ int wrapm(int v, int m) { return v < 0 ? v + m : (v >= m ? v - m : v); }

__global__ __launch_bounds__(256) void k_restrict(const RestrictDesc* __restrict__ dd) {
  const RestrictDesc d = *dd;
  const int m = d.m, n = 2 * m;
  const long long mc = (long long)m * m * m;
  const PR_GLOBAL double* a = gptr(d.a);
  const PR_GLOBAL double* b = d.b ? gptr(d.b) : nullptr;
  PR_GLOBAL double* out = gptr(d.out);
  const double w[3] = {0.25, 0.5, 0.25};
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < mc;
       q += (long long)gridDim.x * blockDim.x) {
    const int K = (int)(q % m), J = (int)((q / m) % m), I = (int)(q / ((long long)m * m));
    double acc = 0.0;
    for (int dx = -1; dx <= 1; ++dx) {
      const long long px = (long long)wrapm(2 * I + dx, n) * n * n;
      double ax = 0.0;
      for (int dy = -1; dy <= 1; ++dy) {
        const long long py = px + (long long)wrapm(2 * J + dy, n) * n;
        double ay = 0.0;
        for (int dz = -1; dz <= 1; ++dz) {
          const long long p = py + wrapm(2 * K + dz, n);
          const double v = b ? a[p] - b[p] : a[p];
          ay += w[dz + 1] * v;
        }
        ax += w[dy + 1] * ay;
      }
      acc += w[dx + 1] * ax;
    }
    out[q] = acc;
  }
}

// out = P(c) + fine (nullable) with per-workgroup partials of |out - prev|^2,
// |out|^2, |out - ref|^2 and |ref|^2 (layout of the correction kernel).
__global__ __launch_bounds__(256) void k_prolong_add(const ProlongDesc* __restrict__ dd) {
  __shared__ double red[4][4];
  const ProlongDesc d = *dd;
  const int m = d.m, n = 2 * m;
  const long long ng = (long long)n * n * n;
  const PR_GLOBAL double* c = gptr(d.c);
  const PR_GLOBAL double* fine = d.fine ? gptr(d.fine) : nullptr;
  const PR_GLOBAL double* prev = d.prev ? gptr(d.prev) : nullptr;
  const PR_GLOBAL double* ref = d.ref ? gptr(d.ref) : nullptr;
  PR_GLOBAL double* out = gptr(d.out);
  const long long per = (ng + d.nwg - 1) / d.nwg;
  const long long r0 = (long long)blockIdx.x * per, r1 = min(ng, r0 + per);
  double s_jump = 0, s_u = 0, s_err = 0, s_ref = 0;
  for (long long p = r0 + threadIdx.x; p < r1; p += 256) {
    const int k = (int)(p % n), j = (int)((p / n) % n), i = (int)(p / ((long long)n * n));
    // per axis: the coarse points and weights of the interpolation
    const int ia = i >> 1, ja = j >> 1, ka = k >> 1;
    const int ib = (i & 1) ? wrapm(ia + 1, m) : ia;
    const int jb = (j & 1) ? wrapm(ja + 1, m) : ja;
    const int kb = (k & 1) ? wrapm(ka + 1, m) : ka;
    const double wi = (i & 1) ? 0.5 : 1.0, wj = (j & 1) ? 0.5 : 1.0, wk = (k & 1) ? 0.5 : 1.0;
    auto at = [&](int x, int y, int z) { return c[((long long)x * m + y) * m + z]; };
    auto line = [&](int x, int y) {
      return (k & 1) ? wk * (at(x, y, ka) + at(x, y, kb)) : at(x, y, ka);
    };
    auto plane = [&](int x) { return (j & 1) ? wj * (line(x, ja) + line(x, jb)) : line(x, ja); };
    const double pv = (i & 1) ? wi * (plane(ia) + plane(ib)) : plane(ia);
    const double v = fine ? pv + fine[p] : pv;
    out[p] = v;
    s_u += v * v;
    if (prev) {
      const double dj = v - prev[p];
      s_jump += dj * dj;
    }
    if (ref) {
      const double r = ref[p];
      const double de = v - r;
      s_err += de * de;
      s_ref += r * r;
    }
  }
  for (int o = 32; o >= 1; o >>= 1) {
    s_jump += __shfl_xor(s_jump, o, 64);
    s_u += __shfl_xor(s_u, o, 64);
    s_err += __shfl_xor(s_err, o, 64);
    s_ref += __shfl_xor(s_ref, o, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[wave][0] = s_jump;
    red[wave][1] = s_u;
    red[wave][2] = s_err;
    red[wave][3] = s_ref;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int e = threadIdx.x;
    gptr(d.partial)[(long long)blockIdx.x * 4 + e] = (red[0][e] + red[1][e]) + (red[2][e] + red[3][e]);
  }
}

void launch_restrict(const RestrictDesc* d, long long coarse_points, hipStream_t s) {
  if (coarse_points <= 0) return;
  long long g = (coarse_points + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_restrict, dim3((unsigned)g), dim3(256), 0, s, d);
  PR_HIP(hipGetLastError());
}

void launch_prolong_add(const ProlongDesc* d, int nwg, hipStream_t s) {
  if (nwg <= 0) return;
  hipLaunchKernelGGL(k_prolong_add, dim3((unsigned)nwg), dim3(256), 0, s, d);
  PR_HIP(hipGetLastError());
}

}  // namespace pr
