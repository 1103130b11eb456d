// Rayleigh-Sommerfeld source plane (BabelBrain Section 2.3): the field of the
// transducer's surface elements radiating into water, at the cell centres of
// the source plane, e^{+i omega t}:
//   S(x) = (i omega rho_w / 2 pi) sum_e u0 A_e exp(-i k R_e) / R_e.
// One thread per plane point; element tiles are staged through LDS and shared
// by the block.  Distances and phases are FP64 (k R reaches a few hundred
// radians), the phase is reduced to [-pi, pi] in FP64 and only the sine and
// cosine of the reduced phase are FP32; sums accumulate in FP64.  ALU bound.
#include "bbfd_dev.h"

namespace bbfd {

constexpr int kRayThreads = 256;

// blockIdx.y selects the plane z = z0 + blockIdx.y * dx; out is [planes][ny][nx].
__global__ void __launch_bounds__(kRayThreads)
    k_rayleigh(const double4 *__restrict__ el, int n_el, int nx, int ny, double dx, double z0,
               double kw, double pre, float2 *__restrict__ out) {
  __shared__ double4 tile[kRayThreads];
  const int q = blockIdx.x * kRayThreads + threadIdx.x;
  const bool live = q < nx * ny;
  const int i = live ? q % nx : 0, j = live ? q / nx : 0;
  const double x = i * dx, y = j * dx, z = z0 + blockIdx.y * dx;
  out += (long long)blockIdx.y * nx * ny;
  const double two_pi = 6.283185307179586476925286766559;
  double sr = 0.0, si = 0.0;
  for (int t0 = 0; t0 < n_el; t0 += kRayThreads) {
    const int t = t0 + threadIdx.x;
    tile[threadIdx.x] = t < n_el ? el[t] : make_double4(0.0, 0.0, 0.0, 0.0);
    __syncthreads();
    const int m = min(kRayThreads, n_el - t0);
    for (int e = 0; e < m; ++e) {
      const double4 p = tile[e];
      const double ddx = x - p.x, ddy = y - p.y, ddz = z - p.z;
      const double R = sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
      double ph = kw * R;
      ph -= two_pi * rint(ph * (1.0 / two_pi));
      float s, c;
      sincosf((float)ph, &s, &c);
      const double w = p.w / R;
      sr += w * s;  // i exp(-i k R) = sin(kR) + i cos(kR)
      si += w * c;
    }
    __syncthreads();
  }
  if (live) out[q] = make_float2((float)(pre * sr), (float)(pre * si));
}

hipError_t launch_rayleigh(const double4 *el, int n_el, int nx, int ny, int planes, double dx,
                           double z0, double kw, double pre, float2 *out, hipStream_t s) {
  const int blocks = (nx * ny + kRayThreads - 1) / kRayThreads;
  hipLaunchKernelGGL(k_rayleigh, dim3(blocks, planes), dim3(kRayThreads), 0, s, el, n_el, nx, ny,
                     dx, z0, kw, pre, out);
  return hipGetLastError();
}

}  // namespace bbfd
