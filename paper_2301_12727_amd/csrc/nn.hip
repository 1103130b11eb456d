// Kernels of the learned surrogate: a generic batched strided GEMM on the
// gfx950 BF16 matrix cores (v_mfma_f32_32x32x16_bf16, FP32 accumulation) and
// the element-wise pieces of a Fourier neural operator (GELU and its
// gradient, per-mode complex channel mixing, loss, Adam).
//
// GEMM: C[b](m, n) = alpha * sum_k A[b](m, k) * B[b](k, n) + beta * C[b](m, n)
// (+ bias[m]).  Operands are FP32 in memory, rounded to BF16 when staged into
// LDS ("FP32 in, BF16 MFMA, FP32 accumulate").  Element addresses are fully
// strided, and K may be split into two segments held at different offsets
// (k >= seg_k reads from base + seg_off), which lets the real and imaginary
// planes of a complex operand form one contraction.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nn_dev.h"

namespace bbsur {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kBM = 64, kBN = 64, kBK = 32, kPad = 8;
constexpr int kThreads = 256;

__device__ __forceinline__ long long a_off(const GemmArgs &g, int m, int k) {
  const int seg = k >= g.a_seg_k;
  return (long long)m * g.sAm + (long long)(k - seg * g.a_seg_k) * g.sAk + seg * g.a_seg_off;
}

__device__ __forceinline__ long long b_off(const GemmArgs &g, int k, int n) {
  const int seg = k >= g.b_seg_k;
  return (long long)(k - seg * g.b_seg_k) * g.sBk + (long long)n * g.sBn + seg * g.b_seg_off;
}

__global__ void __launch_bounds__(kThreads) k_gemm(GemmArgs g) {
  __shared__ __bf16 As[kBM][kBK + kPad];  // [m][k]
  __shared__ __bf16 Bs[kBN][kBK + kPad];  // [n][k]
  const int b = blockIdx.z;
  const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
  const float *A = g.A + (long long)b * g.sAb;
  const float *B = g.B + (long long)b * g.sBb;
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  f32x16 acc;
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  for (int k0 = 0; k0 < g.K; k0 += kBK) {
    // stage A (64 x 32) and B (32 x 64): 8 elements per thread each, the
    // unit-stride axis mapped to consecutive threads
    for (int r = 0; r < 8; ++r) {
      const int e = t + kThreads * r;
      int m, k;
      if (g.a_kfast) { m = e >> 5; k = e & 31; } else { m = e & 63; k = e >> 6; }
      const int gm = m0 + m, gk = k0 + k;
      const float v = (gm < g.M && gk < g.K) ? A[a_off(g, gm, gk)] : 0.f;
      As[m][k] = (__bf16)v;
    }
    for (int r = 0; r < 8; ++r) {
      const int e = t + kThreads * r;
      int n, k;
      if (g.b_nfast) { n = e & 63; k = e >> 6; } else { n = e >> 5; k = e & 31; }
      const int gn = n0 + n, gk = k0 + k;
      const float v = (gn < g.N && gk < g.K) ? B[b_off(g, gk, gn)] : 0.f;
      Bs[n][k] = (__bf16)v;
    }
    __syncthreads();
    for (int kk = 0; kk < kBK; kk += 16) {
      // lane l holds rows/cols l % 32 and the 8 consecutive k of half l / 32
      const int kq = kk + 8 * (lane >> 5);
      const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&As[wm + (lane & 31)][kq]);
      const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(&Bs[wn + (lane & 31)][kq]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bv, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  float *C = g.C + (long long)b * g.sCb;
  const int col = n0 + wn + (lane & 31);
  if (col >= g.N) return;
  for (int r = 0; r < 16; ++r) {
    const int row = m0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (row >= g.M) continue;
    float *c = C + (long long)row * g.sCm + (long long)col * g.sCn;
    float v = g.alpha * acc[r];
    if (g.beta != 0.f) v += g.beta * *c;
    if (g.bias) v += g.bias[row];
    *c = v;
  }
}

// ---------------------------------------------------------------- element-wise

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__global__ void k_gelu(const float *__restrict__ z, float *__restrict__ h, long long n) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x)
    h[t] = gelu(z[t]);
}

__global__ void k_gelu_bwd(const float *__restrict__ z, const float *__restrict__ dh,
                           float *__restrict__ dz, long long n) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x)
    dz[t] = dh[t] * gelu_grad(z[t]);
}

__global__ void k_fill(float *__restrict__ p, long long n, float v) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x)
    p[t] = v;
}

// Per-mode complex channel mixing.  U, V: [b][ch][2][Q] (real plane, then
// imaginary plane); R: [2][Q][C][O].
//   V[b][o][q] = sum_c R[q][c][o] U[b][c][q]
__global__ void k_mix(const float *__restrict__ U, const float *__restrict__ R,
                      float *__restrict__ V, int B, int C, int O, int Q) {
  const long long total = (long long)B * O * Q;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int q = (int)(t % Q);
    const int o = (int)((t / Q) % O);
    const int b = (int)(t / ((long long)Q * O));
    float vr = 0.f, vi = 0.f;
    const float *u = U + (long long)b * C * 2 * Q + q;
    const float *rr = R + (long long)q * C * O + o;
    const float *ri = rr + (long long)Q * C * O;
    for (int c = 0; c < C; ++c) {
      const float ur = u[(long long)c * 2 * Q], ui = u[(long long)c * 2 * Q + Q];
      const float ar = rr[c * O], ai = ri[c * O];
      vr += ar * ur - ai * ui;
      vi += ar * ui + ai * ur;
    }
    float *v = V + ((long long)b * O + o) * 2 * Q + q;
    v[0] = vr;
    v[Q] = vi;
  }
}

//   dU[b][c][q] = sum_o conj-transpose action:  dUr = sum (Rr dVr + Ri dVi),
//   dUi = sum (Rr dVi - Ri dVr)
__global__ void k_mix_bwd_data(const float *__restrict__ dV, const float *__restrict__ R,
                               float *__restrict__ dU, int B, int C, int O, int Q) {
  const long long total = (long long)B * C * Q;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int q = (int)(t % Q);
    const int c = (int)((t / Q) % C);
    const int b = (int)(t / ((long long)Q * C));
    float gr = 0.f, gi = 0.f;
    const float *dv = dV + (long long)b * O * 2 * Q + q;
    const float *rr = R + ((long long)q * C + c) * O;
    const float *ri = rr + (long long)Q * C * O;
    for (int o = 0; o < O; ++o) {
      const float vr = dv[(long long)o * 2 * Q], vi = dv[(long long)o * 2 * Q + Q];
      gr += rr[o] * vr + ri[o] * vi;
      gi += rr[o] * vi - ri[o] * vr;
    }
    float *du = dU + ((long long)b * C + c) * 2 * Q + q;
    du[0] = gr;
    du[Q] = gi;
  }
}

//   dRr[q][c][o] = sum_b (Ur dVr + Ui dVi),  dRi = sum_b (Ur dVi - Ui dVr)
__global__ void k_mix_bwd_weight(const float *__restrict__ U, const float *__restrict__ dV,
                                 float *__restrict__ dR, int B, int C, int O, int Q) {
  const long long total = (long long)Q * C * O;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int o = (int)(t % O);
    const int c = (int)((t / O) % C);
    const int q = (int)(t / ((long long)O * C));
    float gr = 0.f, gi = 0.f;
    for (int b = 0; b < B; ++b) {
      const float *u = U + ((long long)b * C + c) * 2 * Q + q;
      const float *v = dV + ((long long)b * O + o) * 2 * Q + q;
      gr += u[0] * v[0] + u[Q] * v[Q];
      gi += u[0] * v[Q] - u[Q] * v[0];
    }
    dR[t] = gr;
    dR[t + (long long)Q * C * O] = gi;
  }
}

// out[m] = sum_r in[r * M + m]  (fixed order: deterministic)
// out[m] = sum over r of in[r][m].  A block owns 64 consecutive m; its 16
// thread rows take every 16th r, and the 16 partial sums are added in a
// fixed order, so the result does not depend on scheduling.
constexpr int kSumCols = 64, kSumRows = 16;
__global__ void __launch_bounds__(kSumCols * kSumRows)
    k_sum_rows(const float *__restrict__ in, float *__restrict__ out, int R, int M) {
  __shared__ float part[kSumRows][kSumCols];
  const int m = blockIdx.x * kSumCols + threadIdx.x;
  float acc = 0.f;
  if (m < M)
    for (int r = threadIdx.y; r < R; r += kSumRows) acc += in[(long long)r * M + m];
  part[threadIdx.y][threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.y == 0 && m < M) {
    float s = 0.f;
    for (int q = 0; q < kSumRows; ++q) s += part[q][threadIdx.x];
    out[m] = s;
  }
}

// Squared-error loss: dy = 2 (y - t) / count, per-block partial sums of (y - t)^2.
constexpr int kLossThreads = 256;
__global__ void __launch_bounds__(kLossThreads)
    k_loss(const float *__restrict__ y, const float *__restrict__ tgt, float *__restrict__ dy,
           float *__restrict__ partial, long long n, float inv_count, float focus) {
  __shared__ float sh[kLossThreads];
  float acc = 0.f;
  for (long long t = blockIdx.x * (long long)kLossThreads + threadIdx.x; t < n;
       t += (long long)gridDim.x * kLossThreads) {
    const float w = focus > 0.f ? 1.f + focus * expf(tgt[t]) : 1.f;
    const float d = y[t] - tgt[t];
    dy[t] = 2.f * w * d * inv_count;
    acc += w * d * d;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s2 = kLossThreads / 2; s2 > 0; s2 >>= 1) {
    if (threadIdx.x < s2) sh[threadIdx.x] += sh[threadIdx.x + s2];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void k_loss_final(const float *__restrict__ partial, int n, float inv_count,
                             float *__restrict__ loss) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float acc = 0.f;
    for (int i = 0; i < n; ++i) acc += partial[i];
    *loss = acc * inv_count;
  }
}

// Adam with bias correction folded into lr_t = lr sqrt(1 - b2^t) / (1 - b1^t).
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, long long n, float lr_t, float b1, float b2,
                       float eps_t) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x) {
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.f - b1) * gt;
    const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    p[t] -= lr_t * mt / (sqrtf(vt) + eps_t);
  }
}

// Input channels of one sample: [c / c_w - 1, rho / rho_w - 1, cos phase,
// sin phase], each [cells]; table holds the first two per material (indices
// beyond it read as water, 0).
__global__ void k_features(const uint8_t *__restrict__ mat, const float2 *__restrict__ table,
                           int n_table, const float2 *__restrict__ field, float *__restrict__ x,
                           long long cells) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < cells;
       t += (long long)gridDim.x * blockDim.x) {
    const int mi = mat[t];
    const float2 tb = mi < n_table ? table[mi] : make_float2(0.f, 0.f);
    const float2 f = field[t];
    const float a = sqrtf(f.x * f.x + f.y * f.y);
    x[t] = tb.x;
    x[t + cells] = tb.y;
    x[t + 2 * cells] = a > 0.f ? f.x / a : 1.f;
    x[t + 3 * cells] = a > 0.f ? f.y / a : 0.f;
  }
}

static unsigned grid_for(long long n) {
  long long b = (n + 255) / 256;
  return (unsigned)(b > 16384 ? 16384 : (b < 1 ? 1 : b));
}

hipError_t launch_gelu(const float *z, float *h, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_gelu, dim3(grid_for(n)), dim3(256), 0, s, z, h, n);
  return hipGetLastError();
}
hipError_t launch_gelu_bwd(const float *z, const float *dh, float *dz, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_gelu_bwd, dim3(grid_for(n)), dim3(256), 0, s, z, dh, dz, n);
  return hipGetLastError();
}
hipError_t launch_fill(float *p, long long n, float v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_mix(const float *U, const float *R, float *V, int B, int C, int O, int Q,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_mix, dim3(grid_for((long long)B * O * Q)), dim3(256), 0, s, U, R, V, B, C, O, Q);
  return hipGetLastError();
}
hipError_t launch_mix_bwd(const float *U, const float *dV, const float *R, float *dU, float *dR,
                          int B, int C, int O, int Q, hipStream_t s) {
  hipLaunchKernelGGL(k_mix_bwd_data, dim3(grid_for((long long)B * C * Q)), dim3(256), 0, s, dV, R,
                     dU, B, C, O, Q);
  hipLaunchKernelGGL(k_mix_bwd_weight, dim3(grid_for((long long)Q * C * O)), dim3(256), 0, s, U,
                     dV, dR, B, C, O, Q);
  return hipGetLastError();
}
hipError_t launch_sum_rows(const float *in, float *out, int R, int M, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_rows, dim3((M + kSumCols - 1) / kSumCols), dim3(kSumCols, kSumRows), 0, s,
                     in, out, R, M);
  return hipGetLastError();
}
constexpr int kLossBlocks = 1024;
int loss_partials() { return kLossBlocks; }
hipError_t launch_loss(const float *y, const float *t, float *dy, float *partial, float *loss,
                       float focus, long long n, hipStream_t s) {
  const float inv = 1.f / (float)n;
  hipLaunchKernelGGL(k_loss, dim3(kLossBlocks), dim3(kLossThreads), 0, s, y, t, dy, partial, n, inv,
                     focus);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, partial, kLossBlocks, inv, loss);
  return hipGetLastError();
}
hipError_t launch_adam(float *p, const float *g, float *m, float *v, long long n, float lr_t,
                       float b1, float b2, float eps_t, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, s, p, g, m, v, n, lr_t, b1, b2, eps_t);
  return hipGetLastError();
}
hipError_t launch_features(const uint8_t *mat, const float2 *table, int n_table,
                           const float2 *field, float *x, long long cells, hipStream_t s) {
  hipLaunchKernelGGL(k_features, dim3(grid_for(cells)), dim3(256), 0, s, mat, table, n_table,
                     field, x, cells);
  return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.K <= 0 || g.batch <= 0) return hipSuccess;
  dim3 grid((g.N + kBN - 1) / kBN, (g.M + kBM - 1) / kBM, g.batch);
  hipLaunchKernelGGL(k_gemm, grid, dim3(kThreads), 0, s, g);
  return hipGetLastError();
}

}  // namespace bbsur
