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
// With W, each element carries a complex drive weight wts[e] (phased arrays).
template <bool W>
__global__ void __launch_bounds__(kRayThreads)
    k_rayleigh(const double4 *__restrict__ el, const double2 *__restrict__ wts, int n_el, int nx,
               int ny, double dx, double z0, double kw, double pre, float2 *__restrict__ out) {
  __shared__ double4 tile[kRayThreads];
  __shared__ double2 wtile[W ? kRayThreads : 1];
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
    if (W) wtile[threadIdx.x] = t < n_el ? wts[t] : make_double2(0.0, 0.0);
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
      if (W) {  // (a + i b) (sin kR + i cos kR)
        const double2 q = wtile[e];
        sr += w * (q.x * s - q.y * c);
        si += w * (q.x * c + q.y * s);
      } else {
        sr += w * s;  // i exp(-i k R) = sin(kR) + i cos(kR)
        si += w * c;
      }
    }
    __syncthreads();
  }
  if (live) out[q] = make_float2((float)(pre * sr), (float)(pre * si));
}

hipError_t launch_rayleigh(const double4 *el, int n_el, int nx, int ny, int planes, double dx,
                           double z0, double kw, double pre, float2 *out, hipStream_t s,
                           const double2 *wts) {
  const int blocks = (nx * ny + kRayThreads - 1) / kRayThreads;
  if (wts)
    hipLaunchKernelGGL(k_rayleigh<true>, dim3(blocks, planes), dim3(kRayThreads), 0, s, el, wts,
                       n_el, nx, ny, dx, z0, kw, pre, out);
  else
    hipLaunchKernelGGL(k_rayleigh<false>, dim3(blocks, planes), dim3(kRayThreads), 0, s, el, wts,
                       n_el, nx, ny, dx, z0, kw, pre, out);
  return hipGetLastError();
}

// ---------------------------------------------------------- back-propagation
// Rayleigh integral from a plane of complex normal velocity (the recorded
// field of a point source, one value per cell of area dx^2 at z = zp) to a
// few points (the elements of a phased array):
//   p(r) = (i omega rho_w / 2 pi) sum_cells v dx^2 exp(-i k R) / R.
// Few points and many plane cells: block (point, row chunk) sums its rows in
// FP64 and reduces in LDS; k_backprop_final adds the chunks in a fixed order.
constexpr int kBpThreads = 256;
constexpr int kBpChunks = 64;

__global__ void __launch_bounds__(kBpThreads)
    k_backprop(const float2 *__restrict__ plane, int nx, int ny, double dx, double zp,
               const double4 *__restrict__ pts, double kw, double2 *__restrict__ part) {
  __shared__ double sr[kBpThreads], si[kBpThreads];
  const double4 p = pts[blockIdx.x];
  const double two_pi = 6.283185307179586476925286766559;
  double ar = 0.0, ai = 0.0;
  const int rows = (ny + kBpChunks - 1) / kBpChunks;
  const int j0 = blockIdx.y * rows, j1 = min(j0 + rows, ny);
  for (int q = threadIdx.x; q < (j1 - j0) * nx; q += kBpThreads) {
    const int i = q % nx, j = j0 + q / nx;
    const float2 v = plane[(long long)j * nx + i];
    const double ddx = i * dx - p.x, ddy = j * dx - p.y, ddz = zp - p.z;
    const double R = sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
    double ph = kw * R;
    ph -= two_pi * rint(ph * (1.0 / two_pi));
    float s, c;
    sincosf((float)ph, &s, &c);
    const double w = 1.0 / R;
    ar += w * ((double)v.x * s - (double)v.y * c);
    ai += w * ((double)v.x * c + (double)v.y * s);
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int st = kBpThreads / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      sr[threadIdx.x] += sr[threadIdx.x + st];
      si[threadIdx.x] += si[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long long)blockIdx.x * kBpChunks + blockIdx.y] = make_double2(sr[0], si[0]);
}

__global__ void k_backprop_final(const double2 *__restrict__ part, int n_pts, double pre,
                                 double2 *__restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_pts) return;
  double r = 0.0, i = 0.0;
  for (int c = 0; c < kBpChunks; ++c) {
    r += part[(long long)e * kBpChunks + c].x;
    i += part[(long long)e * kBpChunks + c].y;
  }
  out[e] = make_double2(pre * r, pre * i);
}

int backprop_partials(int n_pts) { return n_pts * kBpChunks; }

// part: backprop_partials(n_pts) double2; out: n_pts double2 (device).
hipError_t launch_backprop(const float2 *plane, int nx, int ny, double dx, double zp,
                           const double4 *pts, int n_pts, double kw, double pre, double2 *part,
                           double2 *out, hipStream_t s) {
  hipLaunchKernelGGL(k_backprop, dim3(n_pts, kBpChunks), dim3(kBpThreads), 0, s, plane, nx, ny, dx,
                     zp, pts, kw, part);
  hipLaunchKernelGGL(k_backprop_final, dim3((n_pts + 127) / 128), dim3(128), 0, s, part, n_pts, pre,
                     out);
  return hipGetLastError();
}

// Complex phasor of v_z on one plane of faces (z = (k + 1/2) dx), accumulated
// over the steps of the last period: ph += v_z (c + i s) with c + i s =
// (2 / N_T) exp(-i omega t_n) (host FP64).
__global__ void k_record_plane(const float *__restrict__ vz, long long base, int pitch, int nx,
                               int ny, float c, float s, float2 *__restrict__ ph) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nx * ny) return;
  const int i = q % nx, j = q / nx;
  const float v = vz[base + (long long)j * pitch + i];
  float2 a = ph[q];
  a.x = fmaf(v, c, a.x);
  a.y = fmaf(v, s, a.y);
  ph[q] = a;
}

hipError_t launch_record_plane(const float *vz, long long base, int pitch, int nx, int ny, float c,
                               float s, float2 *ph, hipStream_t st) {
  hipLaunchKernelGGL(k_record_plane, dim3((nx * ny + 255) / 256), dim3(256), 0, st, vz, base,
                     pitch, nx, ny, c, s, ph);
  return hipGetLastError();
}

}  // namespace bbfd
