// Thermal step of the pipeline (BabelBrain Section 2.4): the Pennes bio-heat
// transfer equation
//   rho C dT/dt = div(k grad T) - w rho_b C_b (T - T_a) + Q
// by explicit finite differences on the acoustic grid (7-point Laplacian,
// harmonic-mean face conductivities, the outermost cells held at T_a), with
// the running maximal temperature and the CEM43 thermal dose
//   dose += dt/60 * R^(43 - T),  R = 0.5 at T >= 43 degC, 0.25 below.
// Q = 2 h alpha_l p^2 / (2 rho c_l) from the acoustic peak-pressure map, with h
// the share of the attenuation that heats (0.16 in bone), times the caller's
// intensity scale and, while the ultrasound is on, the duty cycle.
//
// One launch per time step.  Each wave owns a 64-cell x segment of one row
// and marches over a chunk of z planes, keeping the z neighbours of its column
// (temperature and material) in registers; x and y neighbours are cache hits
// of this and the neighbouring waves.  Per cell update it moves T in and out,
// Q, the material byte, and the maximum and dose in and out: 29 bytes.
// HBM-bound.  The material table (k, and dt-scaled coefficients) sits in LDS.
#include "bbfd_dev.h"

namespace bbfd {

constexpr int kThRows = 4;     // rows per block (one wave each)
constexpr int kThPlanes = 16;  // z planes per block

// Per material: k, a = dt / (rho C dx^2), b = dt w rho_b C_b / (rho C), c = dt / (rho C).
struct ThermRow {
  float k, a, b, c;
};

// The kernels carry the temperature rise theta = T - T_a (zero on the border
// and at the start), which keeps FP32 resolution for the small per-step
// increments; outputs are converted back to degC at the end.
struct ThermArgs {
  int nx, ny, nz;
  int n_mat;
  const ThermRow *tab;
  const uint8_t *mat;
  const float *q;      // heat source, W/m^3 (before the duty cycle)
  const float *t_in;   // theta of the current step
  float *t_out;        // theta of the next step
  float *t_max;        // running maximum of theta
  float *dose;         // CEM43, minutes
  float q_scale;       // duty cycle while on, 0 while off
  float d43;           // 43 degC - T_a
  float dose_dt;       // dt / 60
};

__device__ __forceinline__ float face_k(float ka, float kb) {
  const float s = ka + kb;
  return s > 0.f ? 2.f * ka * kb / s : 0.f;
}

__global__ void __launch_bounds__(64 * kThRows)
    k_bhte_step(ThermArgs A) {
  __shared__ ThermRow s_tab[kMaxMaterials];
  const int t0 = threadIdx.y * 64 + threadIdx.x;
  for (int m = t0; m < A.n_mat; m += 64 * kThRows) s_tab[m] = A.tab[m];
  __syncthreads();
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * kThRows + threadIdx.y;
  const int k0 = blockIdx.z * kThPlanes, k1 = min(k0 + kThPlanes, A.nz);
  if (i >= A.nx || j >= A.ny) return;
  const long long row = (long long)A.nx, plane = (long long)A.nx * A.ny;
  const bool bxy = i == 0 || j == 0 || i == A.nx - 1 || j == A.ny - 1;
  long long c = (long long)k0 * plane + (long long)j * row + i;
  // z window of this column: theta and material at k-1, k, k+1
  float tm = k0 > 0 ? A.t_in[c - plane] : 0.f, t0c = A.t_in[c];
  int mm = k0 > 0 ? A.mat[c - plane] : 0, m0 = A.mat[c];
  for (int k = k0; k < k1; ++k, c += plane) {
    const bool last = k == A.nz - 1;
    const float tp = last ? 0.f : A.t_in[c + plane];
    const int mp = last ? 0 : A.mat[c + plane];
    float tn = 0.f;  // border cells stay at the body temperature
    if (!(bxy || k == 0 || last)) {
      const float txm = A.t_in[c - 1], txp = A.t_in[c + 1];
      const float tym = A.t_in[c - row], typ = A.t_in[c + row];
      const int mxm = A.mat[c - 1], mxp = A.mat[c + 1], mym = A.mat[c - row], myp = A.mat[c + row];
      const float q = A.q[c];
      const ThermRow r = s_tab[m0];
      float div = face_k(r.k, s_tab[mm].k) * (tm - t0c);
      div += face_k(r.k, s_tab[mp].k) * (tp - t0c);
      div += face_k(r.k, s_tab[mym].k) * (tym - t0c);
      div += face_k(r.k, s_tab[myp].k) * (typ - t0c);
      div += face_k(r.k, s_tab[mxm].k) * (txm - t0c);
      div += face_k(r.k, s_tab[mxp].k) * (txp - t0c);
      tn = t0c + (r.a * div - r.b * t0c + r.c * (A.q_scale * q));
    }
    A.t_out[c] = tn;
    A.t_max[c] = fmaxf(A.t_max[c], tn);
    // log2 of R^(43 - T): R = 0.5 at T >= 43, 0.25 below
    const float e = tn >= A.d43 ? (tn - A.d43) : 2.f * (tn - A.d43);
    A.dose[c] += A.dose_dt * exp2f(e);
    tm = t0c;
    t0c = tp;
    mm = m0;
    m0 = mp;
  }
}

// Back to degC: t_final = theta + T_a, t_max += T_a.
__global__ void k_bhte_finish(const float *__restrict__ theta, float *__restrict__ t_final,
                              float *__restrict__ t_max, long long n, float t_body) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x) {
    t_final[t] = theta[t] + t_body;
    t_max[t] = t_max[t] + t_body;
  }
}

// Q per cell: scale * 2 h alpha_l p^2 / (2 rho c_l); coef[m] = scale * h alpha_l / (rho c_l).
__global__ void k_bhte_source(const uint8_t *__restrict__ mat, const float *__restrict__ peak,
                              const float *__restrict__ coef, long long n, float *__restrict__ q) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x) {
    const float p = peak[t];
    q[t] = coef[mat[t]] * (p * p);
  }
}

__global__ void k_bhte_fill(float *__restrict__ a, float *__restrict__ b, float *__restrict__ c,
                            long long n, float va, float vb, float vc) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x) {
    a[t] = va;
    b[t] = vb;
    c[t] = vc;
  }
}

hipError_t launch_bhte_source(const uint8_t *mat, const float *peak, const float *coef, long long n,
                              float *q, hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_bhte_source, dim3((unsigned)blocks), dim3(256), 0, s, mat, peak, coef, n, q);
  return hipGetLastError();
}

hipError_t launch_bhte_fill(float *a, float *b, float *c, long long n, float va, float vb, float vc,
                            hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_bhte_fill, dim3((unsigned)blocks), dim3(256), 0, s, a, b, c, n, va, vb, vc);
  return hipGetLastError();
}

hipError_t launch_bhte_step(int nx, int ny, int nz, int n_mat, const void *tab, const uint8_t *mat,
                            const float *q, const float *t_in, float *t_out, float *t_max,
                            float *dose, float q_scale, float d43, float dose_dt, hipStream_t s) {
  ThermArgs A;
  A.nx = nx; A.ny = ny; A.nz = nz; A.n_mat = n_mat;
  A.tab = (const ThermRow *)tab;
  A.mat = mat; A.q = q; A.t_in = t_in; A.t_out = t_out; A.t_max = t_max; A.dose = dose;
  A.q_scale = q_scale; A.d43 = d43; A.dose_dt = dose_dt;
  const dim3 grid((nx + 63) / 64, (ny + kThRows - 1) / kThRows, (nz + kThPlanes - 1) / kThPlanes);
  hipLaunchKernelGGL(k_bhte_step, grid, dim3(64, kThRows, 1), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_bhte_finish(const float *theta, float *t_final, float *t_max, long long n,
                              float t_body, hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_bhte_finish, dim3((unsigned)blocks), dim3(256), 0, s, theta, t_final, t_max,
                     n, t_body);
  return hipGetLastError();
}

int bhte_row_floats() { return (int)(sizeof(ThermRow) / sizeof(float)); }

}  // namespace bbfd
