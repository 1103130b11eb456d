// Energy-loss factor of a transcranial solve (BabelBrain Section 2.4, Eq. 2)
// and the pressure transmission T_S = sqrt(E_L) (Section 3.2): the ratio of
// the pulse-average intensity p^2 / (2 rho c) summed over one x-y plane of the
// skull solve to the same sum over the water-only solve, on the plane z_m of
// the water-only field's maximum.  Sums run over the plane's cells outside the
// absorbing layer.  The plane index comes either from the caller or from the
// peak voxel the argmax kernels stored for the water-only map.
//
// Two launches with a deterministic result: each block accumulates its
// grid-stride share of cells in FP64 and reduces it in LDS; one block then adds
// the block partials in a fixed order.  HBM-bound and tiny (two planes of
// float and of uint8: 10 B per plane cell).
#include "bbfd_dev.h"

namespace bbfd {

constexpr int kEnThreads = 256;
constexpr int kEnBlocks = 128;

struct EnergyOut {
  double e_l, t_s, z_m, num, den;
};

__device__ __forceinline__ int energy_plane(int z_m, const Status *st, int nx, int ny) {
  return z_m >= 0 ? z_m : (int)(st->peak_index / ((long long)nx * ny));
}

__device__ __forceinline__ int map_at(const uint8_t *m, long long c, int idx16) {
  return idx16 ? (int)reinterpret_cast<const uint16_t *>(m)[c] : (int)m[c];
}

// iz: 1 / (2 rho c_l) per material (FP64, host-derived); maps of uint8 or
// (idx16) uint16 indices.
__global__ void __launch_bounds__(kEnThreads)
    k_plane_energy(const uint8_t *__restrict__ mat_s, const float *__restrict__ p_s,
                   const uint8_t *__restrict__ mat_w, const float *__restrict__ p_w, int nx,
                   int ny, int L, int z_m, const Status *st, const double *__restrict__ iz,
                   int n_mat, int idx16, double2 *__restrict__ part) {
  __shared__ double sn[kEnThreads], sd[kEnThreads];
  const int k = energy_plane(z_m, st, nx, ny);
  const int wx = nx - 2 * L, wy = ny - 2 * L;
  const long long base = (long long)k * nx * ny;
  double num = 0.0, den = 0.0;
  for (int q = blockIdx.x * kEnThreads + threadIdx.x; q < wx * wy; q += gridDim.x * kEnThreads) {
    const int i = L + q % wx, j = L + q / wx;
    const long long c = base + (long long)j * nx + i;
    const double a = p_s[c], b = p_w[c];
    const int ms = map_at(mat_s, c, idx16), mw = map_at(mat_w, c, idx16);
    num += a * a * (ms < n_mat ? iz[ms] : 0.0);
    den += b * b * (mw < n_mat ? iz[mw] : 0.0);
  }
  sn[threadIdx.x] = num;
  sd[threadIdx.x] = den;
  __syncthreads();
  for (int s = kEnThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sn[threadIdx.x] += sn[threadIdx.x + s];
      sd[threadIdx.x] += sd[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = make_double2(sn[0], sd[0]);
}

__global__ void __launch_bounds__(kEnBlocks)
    k_plane_energy_final(const double2 *__restrict__ part, int nx, int ny, int z_m,
                         const Status *st, EnergyOut *out) {
  __shared__ double sn[kEnBlocks], sd[kEnBlocks];
  sn[threadIdx.x] = part[threadIdx.x].x;
  sd[threadIdx.x] = part[threadIdx.x].y;
  __syncthreads();
  for (int s = kEnBlocks / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sn[threadIdx.x] += sn[threadIdx.x + s];
      sd[threadIdx.x] += sd[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double e = sn[0] / sd[0];
    out->e_l = e;
    out->t_s = sqrt(e);
    out->z_m = (double)energy_plane(z_m, st, nx, ny);
    out->num = sn[0];
    out->den = sd[0];
  }
}

// inv_z (dev): n_mat doubles; part: kEnBlocks double2; out: one EnergyOut (device).
hipError_t launch_plane_energy(const uint8_t *mat_s, const float *p_s, const uint8_t *mat_w,
                               const float *p_w, int nx, int ny, int L, int z_m, const Status *st,
                               const double *inv_z, int n_mat, int idx16, double2 *part,
                               double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_plane_energy, dim3(kEnBlocks), dim3(kEnThreads), 0, s, mat_s, p_s, mat_w,
                     p_w, nx, ny, L, z_m, st, inv_z, n_mat, idx16, part);
  hipLaunchKernelGGL(k_plane_energy_final, dim3(1), dim3(kEnBlocks), 0, s, part, nx, ny, z_m, st,
                     reinterpret_cast<EnergyOut *>(out));
  return hipGetLastError();
}

int energy_out_doubles() { return (int)(sizeof(EnergyOut) / sizeof(double)); }
int energy_partials() { return kEnBlocks; }

}  // namespace bbfd
