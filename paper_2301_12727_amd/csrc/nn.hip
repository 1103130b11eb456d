// Kernels of the learned surrogate: a generic batched strided GEMM on the
// gfx950 BF16 matrix cores (v_mfma_f32_32x32x16_bf16, FP32 accumulation) and
// the element-wise pieces of a Fourier neural operator (GELU gradient,
// per-mode complex channel mixing, loss, Adam; GELU itself is applied in the
// GEMM epilogue).
//
// GEMM: C[b](m, n) = alpha * sum_k A[b](m, k) * B[b](k, n) + beta * C[b](m, n)
// (+ bias[m]); optionally GELU(C) into a second output as well, or, for the
// backward pass, C * GELU'(z) into the second output in place of C.  Operands are FP32 in memory, rounded to BF16 when staged into
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

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

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

// Staging of one 64 x 32 operand tile.  Mode 0: one element per load, any
// strides.  Mode 1: four consecutive k per load (k unit-stride).  Mode 2: four
// consecutive m (or n) per load.  Modes 1 and 2 need the vectorised axis'
// extent, the other strides and the base 16-byte aligned (checked on the host,
// see launch_gemm), so a float4 is either wholly inside the operand or wholly
// outside it.  Modes 3 and 4 are modes 1 and 2 for a BF16 operand: eight
// values per 16-byte load, stored to LDS as they are (the FP32 modes round to
// BF16 on the way in, so an operand kept in BF16 gives the same products).
// Every thread holds 8 values of the next tile in registers while the matrix
// cores work on the current one.
struct Stage {
  float v[8];
  uint4 raw;  // eight BF16 values (modes 3, 4)
};

__device__ __forceinline__ const float *fp(const void *p) { return static_cast<const float *>(p); }
__device__ __forceinline__ const uint4 *bp(const void *p, long long off) {
  return reinterpret_cast<const uint4 *>(static_cast<const __bf16 *>(p) + off);
}
__device__ __forceinline__ __bf16 bf_at(const uint4 &r, int i) {
  const uint32_t w = (&r.x)[i >> 1];
  const unsigned short h = (unsigned short)((i & 1) ? (w >> 16) : (w & 0xffffu));
  return __builtin_bit_cast(__bf16, h);
}

template <int MODE>
__device__ __forceinline__ void load_a(const GemmArgs &g, const void *A, int m0, int k0, int t,
                                       Stage &r) {
  if (MODE >= 3) {
    int m, k;
    if (MODE == 3) { m = t >> 2; k = (t & 3) << 3; } else { k = t >> 3; m = (t & 7) << 3; }
    const int gm = m0 + m, gk = k0 + k;
    r.raw = make_uint4(0u, 0u, 0u, 0u);
    if (gm < g.M && gk < g.K) r.raw = *bp(A, a_off(g, gm, gk));
  } else if (MODE == 0) {
    for (int q = 0; q < 8; ++q) {
      const int e = t + kThreads * q;
      int m, k;
      if (g.a_kfast) { m = e >> 5; k = e & 31; } else { m = e & 63; k = e >> 6; }
      const int gm = m0 + m, gk = k0 + k;
      r.v[q] = (gm < g.M && gk < g.K) ? fp(A)[a_off(g, gm, gk)] : 0.f;
    }
  } else {
    for (int q = 0; q < 2; ++q) {
      const int e = t + kThreads * q;
      int m, k;
      if (MODE == 1) { m = e >> 3; k = (e & 7) << 2; } else { k = e >> 4; m = (e & 15) << 2; }
      const int gm = m0 + m, gk = k0 + k;
      float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
      if (gm < g.M && gk < g.K) x = *reinterpret_cast<const float4 *>(fp(A) + a_off(g, gm, gk));
      r.v[4 * q] = x.x; r.v[4 * q + 1] = x.y; r.v[4 * q + 2] = x.z; r.v[4 * q + 3] = x.w;
    }
  }
}

template <int MODE>
__device__ __forceinline__ void store_a(__bf16 (*As)[kBK + kPad], int t, const Stage &r,
                                        const GemmArgs &g) {
  if (MODE == 3) {
    *reinterpret_cast<uint4 *>(&As[t >> 2][(t & 3) << 3]) = r.raw;
  } else if (MODE == 4) {
    const int k = t >> 3, m = (t & 7) << 3;
    for (int i = 0; i < 8; ++i) As[m + i][k] = bf_at(r.raw, i);
  } else if (MODE == 0) {
    for (int q = 0; q < 8; ++q) {
      const int e = t + kThreads * q;
      int m, k;
      if (g.a_kfast) { m = e >> 5; k = e & 31; } else { m = e & 63; k = e >> 6; }
      As[m][k] = (__bf16)r.v[q];
    }
  } else {
    for (int q = 0; q < 2; ++q) {
      const int e = t + kThreads * q;
      if (MODE == 1) {
        const int m = e >> 3, k = (e & 7) << 2;
        for (int i = 0; i < 4; ++i) As[m][k + i] = (__bf16)r.v[4 * q + i];
      } else {
        const int k = e >> 4, m = (e & 15) << 2;
        for (int i = 0; i < 4; ++i) As[m + i][k] = (__bf16)r.v[4 * q + i];
      }
    }
  }
}

// B tile (32 k x 64 n), staged as Bs[n][k].  Mode 1: four consecutive n per
// load (n unit-stride); mode 2: four consecutive k; modes 3, 4 the same with
// eight BF16 values.
template <int MODE>
__device__ __forceinline__ void load_b(const GemmArgs &g, const void *B, int n0, int k0, int t,
                                       Stage &r) {
  if (MODE >= 3) {
    int n, k;
    if (MODE == 3) { k = t >> 3; n = (t & 7) << 3; } else { n = t >> 2; k = (t & 3) << 3; }
    const int gn = n0 + n, gk = k0 + k;
    r.raw = make_uint4(0u, 0u, 0u, 0u);
    if (gn < g.N && gk < g.K) r.raw = *bp(B, b_off(g, gk, gn));
  } else if (MODE == 0) {
    for (int q = 0; q < 8; ++q) {
      const int e = t + kThreads * q;
      int n, k;
      if (g.b_nfast) { n = e & 63; k = e >> 6; } else { n = e >> 5; k = e & 31; }
      const int gn = n0 + n, gk = k0 + k;
      r.v[q] = (gn < g.N && gk < g.K) ? fp(B)[b_off(g, gk, gn)] : 0.f;
    }
  } else {
    for (int q = 0; q < 2; ++q) {
      const int e = t + kThreads * q;
      int n, k;
      if (MODE == 1) { k = e >> 4; n = (e & 15) << 2; } else { n = e >> 3; k = (e & 7) << 2; }
      const int gn = n0 + n, gk = k0 + k;
      float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
      if (gn < g.N && gk < g.K) x = *reinterpret_cast<const float4 *>(fp(B) + b_off(g, gk, gn));
      r.v[4 * q] = x.x; r.v[4 * q + 1] = x.y; r.v[4 * q + 2] = x.z; r.v[4 * q + 3] = x.w;
    }
  }
}

template <int MODE>
__device__ __forceinline__ void store_b(__bf16 (*Bs)[kBK + kPad], int t, const Stage &r,
                                        const GemmArgs &g) {
  if (MODE == 3) {
    const int k = t >> 3, n = (t & 7) << 3;
    for (int i = 0; i < 8; ++i) Bs[n + i][k] = bf_at(r.raw, i);
  } else if (MODE == 4) {
    *reinterpret_cast<uint4 *>(&Bs[t >> 2][(t & 3) << 3]) = r.raw;
  } else if (MODE == 0) {
    for (int q = 0; q < 8; ++q) {
      const int e = t + kThreads * q;
      int n, k;
      if (g.b_nfast) { n = e & 63; k = e >> 6; } else { n = e >> 5; k = e & 31; }
      Bs[n][k] = (__bf16)r.v[q];
    }
  } else {
    for (int q = 0; q < 2; ++q) {
      const int e = t + kThreads * q;
      if (MODE == 1) {
        const int k = e >> 4, n = (e & 15) << 2;
        for (int i = 0; i < 4; ++i) Bs[n + i][k] = (__bf16)r.v[4 * q + i];
      } else {
        const int n = e >> 3, k = (e & 7) << 2;
        for (int i = 0; i < 4; ++i) Bs[n][k + i] = (__bf16)r.v[4 * q + i];
      }
    }
  }
}

// Output stores: FP32, or BF16 (rounded to nearest even) when bf16 is set;
// off counts elements of the output's own type.
__device__ __forceinline__ void store1(float *p, long long off, float v, int bf16) {
  if (bf16) reinterpret_cast<__bf16 *>(p)[off] = (__bf16)v;
  else p[off] = v;
}
__device__ __forceinline__ void store4(float *p, long long off, float4 v, int bf16) {
  if (bf16) {
    __bf16 *q = reinterpret_cast<__bf16 *>(p) + off;
    q[0] = (__bf16)v.x; q[1] = (__bf16)v.y; q[2] = (__bf16)v.z; q[3] = (__bf16)v.w;
  } else {
    *reinterpret_cast<float4 *>(p + off) = v;
  }
}

// LDS: the two operand tiles during the K loop; the 64 x 64 FP32 result
// (transposed) in the column-major epilogue, after the loop.
constexpr int kOpBytes = kBM * (kBK + kPad) * 2;
constexpr int kCPitch = kBM + 4;
constexpr int kSmem = kBN * kCPitch * 4 > 2 * kOpBytes ? kBN * kCPitch * 4 : 2 * kOpBytes;

template <int AMODE, int BMODE>
__global__ void __launch_bounds__(kThreads) k_gemm(GemmArgs g) {
  __shared__ __align__(16) char smem[kSmem];
  auto As = reinterpret_cast<__bf16 (*)[kBK + kPad]>(smem);             // [m][k]
  auto Bs = reinterpret_cast<__bf16 (*)[kBK + kPad]>(smem + kOpBytes);  // [n][k]
  const int b = blockIdx.z;
  const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
  const void *A = AMODE >= 3 ? (const void *)((const __bf16 *)g.A + (long long)b * g.sAb)
                             : (const void *)(g.A + (long long)b * g.sAb);
  const void *B = BMODE >= 3 ? (const void *)((const __bf16 *)g.B + (long long)b * g.sBb)
                             : (const void *)(g.B + (long long)b * g.sBb);
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  f32x16 acc;
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  Stage ra, rb;
  load_a<AMODE>(g, A, m0, 0, t, ra);
  load_b<BMODE>(g, B, n0, 0, t, rb);
  for (int k0 = 0; k0 < g.K; k0 += kBK) {
    store_a<AMODE>(As, t, ra, g);
    store_b<BMODE>(Bs, t, rb, g);
    __syncthreads();
    if (k0 + kBK < g.K) {  // next tile's loads fly while the matrix cores work
      load_a<AMODE>(g, A, m0, k0 + kBK, t, ra);
      load_b<BMODE>(g, B, n0, k0 + kBK, t, rb);
    }
    for (int kk = 0; kk < kBK; kk += 16) {
      // lane l holds rows/cols l % 32 and the 8 consecutive k of half l / 32
      const int kq = kk + 8 * (lane >> 5);
      const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&As[wm + (lane & 31)][kq]);
      const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(&Bs[wn + (lane & 31)][kq]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bv, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const long long cb = (long long)b * g.sCb;
  if (g.c_mfast) {
    // column-major C: transpose the tile through LDS, then each thread writes
    // four consecutive rows of one column at once
    auto Cs = reinterpret_cast<float (*)[kCPitch]>(smem);  // [n][m]
    for (int r = 0; r < 16; ++r)
      Cs[wn + (lane & 31)][wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)] = acc[r];
    __syncthreads();
    for (int q = 0; q < 4; ++q) {
      const int e = t + kThreads * q;
      const int n = e >> 4, m = (e & 15) << 2;
      const int gn = n0 + n, gm = m0 + m;
      if (gn >= g.N || gm >= g.M) continue;
      const float4 c = *reinterpret_cast<const float4 *>(&Cs[n][m]);
      const long long go = cb + (long long)gn * g.sCn + gm;
      float4 v = make_float4(g.alpha * c.x, g.alpha * c.y, g.alpha * c.z, g.alpha * c.w);
      if (g.beta != 0.f) {  // FP32 C only (checked by the launcher)
        const float4 o = *reinterpret_cast<const float4 *>(g.C + go);
        v.x += g.beta * o.x; v.y += g.beta * o.y; v.z += g.beta * o.z; v.w += g.beta * o.w;
      }
      if (g.bias) {
        v.x += g.bias[gm]; v.y += g.bias[gm + 1]; v.z += g.bias[gm + 2]; v.w += g.bias[gm + 3];
      }
      if (g.gelu_z) {
        const float4 zz = *reinterpret_cast<const float4 *>(g.gelu_z + go);
        *reinterpret_cast<float4 *>(g.gelu_out + go) =
            make_float4(v.x * gelu_grad(zz.x), v.y * gelu_grad(zz.y), v.z * gelu_grad(zz.z),
                        v.w * gelu_grad(zz.w));
        continue;
      }
      store4(g.C, go, v, g.c_bf16);
      if (g.gelu_out)
        store4(g.gelu_out, go, make_float4(gelu(v.x), gelu(v.y), gelu(v.z), gelu(v.w)),
               g.gelu_bf16);
    }
    return;
  }
  const int col = n0 + wn + (lane & 31);
  if (col >= g.N) return;
  for (int r = 0; r < 16; ++r) {
    const int row = m0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (row >= g.M) continue;
    const long long go = cb + (long long)row * g.sCm + (long long)col * g.sCn;
    float v = g.alpha * acc[r];
    if (g.beta != 0.f) v += g.beta * g.C[go];
    if (g.bias) v += g.bias[row];
    if (g.gelu_z) {
      g.gelu_out[go] = v * gelu_grad(g.gelu_z[go]);
      continue;
    }
    store1(g.C, go, v, g.c_bf16);
    if (g.gelu_out) store1(g.gelu_out, go, gelu(v), g.gelu_bf16);
  }
}

// ---------------------------------------------------------------- element-wise



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
// One thread per (b, q, o), o fastest: a wave reads R[q][c][.] as whole rows
// and U[b][c][q] as one broadcast value per mode.
__global__ void k_mix(const float *__restrict__ U, const float *__restrict__ R,
                      float *__restrict__ V, int B, int C, int O, int Q) {
  const long long total = (long long)B * O * Q;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int o = (int)(t % O);
    const int q = (int)((t / O) % Q);
    const int b = (int)(t / ((long long)O * Q));
    const float *rr = R + (long long)q * C * O + o;
    const float *ri = rr + (long long)Q * C * O;
    const float *u = U + (long long)b * C * 2 * Q + q;
    float vr = 0.f, vi = 0.f;
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
// One thread per (b, q, c), c fastest: each lane walks its own row R[q][c][.]
// (one cache line) and dV[b][.][q] is a broadcast per mode.
__global__ void k_mix_bwd_data(const float *__restrict__ dV, const float *__restrict__ R,
                               float *__restrict__ dU, int B, int C, int O, int Q) {
  const long long total = (long long)B * C * Q;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(t % C);
    const int q = (int)((t / C) % Q);
    const int b = (int)(t / ((long long)C * Q));
    const float *rr = R + ((long long)q * C + c) * O;
    const float *ri = rr + (long long)Q * C * O;
    const float *dv = dV + (long long)b * O * 2 * Q + q;
    float gr = 0.f, gi = 0.f;
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

// LDS versions of the two mixing gradients, one block per mode q: the block
// gathers the mode's strided spectra once into LDS (and, for the data
// gradient, the mode's weight rows), so every global load of the inner loops
// becomes an LDS read.  Same sums in the same order as the kernels above.
constexpr int kMixThreads = 256;

__global__ void __launch_bounds__(kMixThreads)
    k_mix_bwd_data_lds(const float *__restrict__ dV, const float *__restrict__ R,
                       float *__restrict__ dU, int B, int C, int O, int Q) {
  extern __shared__ float sm[];
  const int q = blockIdx.x;
  const int OP = O + 1;                       // padded row: lanes of one o hit distinct banks
  float *rre = sm, *rim = sm + C * OP;        // [C][O + 1]
  float *vre = sm + 2 * C * OP, *vim = vre + B * O;  // [B][O]
  const float *Rq = R + (long long)q * C * O;
  const long long QCO = (long long)Q * C * O;
  for (int e = threadIdx.x; e < C * O; e += kMixThreads) {
    const int c = e / O, o = e % O;
    rre[c * OP + o] = Rq[e];
    rim[c * OP + o] = Rq[QCO + e];
  }
  for (int e = threadIdx.x; e < B * O; e += kMixThreads) {
    const float *dv = dV + (long long)e * 2 * Q + q;  // e = b * O + o
    vre[e] = dv[0];
    vim[e] = dv[Q];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < B * C; e += kMixThreads) {
    const int b = e / C, c = e % C;
    const float *rr = rre + c * OP, *ri = rim + c * OP;
    const float *vr_ = vre + b * O, *vi_ = vim + b * O;
    float gr = 0.f, gi = 0.f;
    for (int o = 0; o < O; ++o) {
      const float vr = vr_[o], vi = vi_[o];
      gr += rr[o] * vr + ri[o] * vi;
      gi += rr[o] * vi - ri[o] * vr;
    }
    float *du = dU + ((long long)b * C + c) * 2 * Q + q;
    du[0] = gr;
    du[Q] = gi;
  }
}

__global__ void __launch_bounds__(kMixThreads)
    k_mix_bwd_weight_lds(const float *__restrict__ U, const float *__restrict__ dV,
                         float *__restrict__ dR, int B, int C, int O, int Q) {
  extern __shared__ float sm[];
  const int q = blockIdx.x;
  float *ure = sm, *uim = sm + B * C;            // [B][C]
  float *vre = sm + 2 * B * C, *vim = vre + B * O;  // [B][O]
  for (int e = threadIdx.x; e < B * C; e += kMixThreads) {
    const float *u = U + (long long)e * 2 * Q + q;  // e = b * C + c
    ure[e] = u[0];
    uim[e] = u[Q];
  }
  for (int e = threadIdx.x; e < B * O; e += kMixThreads) {
    const float *v = dV + (long long)e * 2 * Q + q;
    vre[e] = v[0];
    vim[e] = v[Q];
  }
  __syncthreads();
  const long long QCO = (long long)Q * C * O;
  for (int e = threadIdx.x; e < C * O; e += kMixThreads) {
    const int c = e / O, o = e % O;
    float gr = 0.f, gi = 0.f;
    for (int b = 0; b < B; ++b) {
      const float ur = ure[b * C + c], ui = uim[b * C + c];
      const float vr = vre[b * O + o], vi = vim[b * O + o];
      gr += ur * vr + ui * vi;
      gi += ur * vi - ui * vr;
    }
    const long long t = (long long)q * C * O + e;
    dR[t] = gr;
    dR[t + QCO] = gi;
  }
}

// out[m] = sum over r of in[r][m], in a fixed order (deterministic).  Block
// (x, g) owns 64 consecutive m and the rows [g * rows, (g + 1) * rows); its 16
// thread rows take every 16th of them and the 16 partial sums are added in a
// fixed order.  With more than one row group the group sums go to tmp and a
// second launch of the same kernel adds them.
constexpr int kSumCols = 64, kSumRows = 16, kSumGroups = 64;
__global__ void __launch_bounds__(kSumCols * kSumRows)
    k_sum_rows(const float *__restrict__ in, float *__restrict__ out, int R, int M, int rows) {
  __shared__ float part[kSumRows][kSumCols];
  const int m = blockIdx.x * kSumCols + threadIdx.x;
  const int r0 = blockIdx.y * rows, r1 = min(R, r0 + rows);
  float acc = 0.f;
  if (m < M)
    for (int r = r0 + threadIdx.y; r < r1; r += kSumRows) acc += in[(long long)r * M + m];
  part[threadIdx.y][threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.y == 0 && m < M) {
    float s = 0.f;
    for (int q = 0; q < kSumRows; ++q) s += part[q][threadIdx.x];
    out[(long long)blockIdx.y * M + m] = s;
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

// Sum of the per-block partials: each thread adds a strided share in a fixed
// order, then a fixed pairwise tree in LDS (deterministic).
constexpr int kLossFinal = 256;
__global__ void __launch_bounds__(kLossFinal)
    k_loss_final(const float *__restrict__ partial, int n, float inv_count,
                 float *__restrict__ loss) {
  __shared__ float sh[kLossFinal];
  float acc = 0.f;
  for (int i = threadIdx.x; i < n; i += kLossFinal) acc += partial[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kLossFinal / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = sh[0] * inv_count;
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
  const size_t lds_data = (size_t)(2 * C * (O + 1) + 2 * B * O) * sizeof(float);
  const size_t lds_weight = (size_t)(2 * B * C + 2 * B * O) * sizeof(float);
  constexpr size_t kLdsMax = 48 * 1024;
  if (lds_data <= kLdsMax)
    hipLaunchKernelGGL(k_mix_bwd_data_lds, dim3(Q), dim3(kMixThreads), lds_data, s, dV, R, dU, B, C,
                       O, Q);
  else
    hipLaunchKernelGGL(k_mix_bwd_data, dim3(grid_for((long long)B * C * Q)), dim3(256), 0, s, dV, R,
                       dU, B, C, O, Q);
  if (lds_weight <= kLdsMax)
    hipLaunchKernelGGL(k_mix_bwd_weight_lds, dim3(Q), dim3(kMixThreads), lds_weight, s, U, dV, dR,
                       B, C, O, Q);
  else
    hipLaunchKernelGGL(k_mix_bwd_weight, dim3(grid_for((long long)Q * C * O)), dim3(256), 0, s, U,
                       dV, dR, B, C, O, Q);
  return hipGetLastError();
}
// Row groups: enough blocks to spread over the chip (about 512), at most
// kSumGroups groups, so tmp needs kSumGroups * M floats.
int sum_rows_groups() { return kSumGroups; }
hipError_t launch_sum_rows(const float *in, float *out, int R, int M, float *tmp, hipStream_t s) {
  if (R <= 0 || M <= 0) return hipSuccess;
  const int cb = (M + kSumCols - 1) / kSumCols;
  int g = 512 / cb;
  g = g < 1 ? 1 : (g > kSumGroups ? kSumGroups : g);
  if (g > R) g = R;
  const int rows = (R + g - 1) / g;
  g = (R + rows - 1) / rows;
  if (g == 1) {
    hipLaunchKernelGGL(k_sum_rows, dim3(cb, 1), dim3(kSumCols, kSumRows), 0, s, in, out, R, M, R);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_sum_rows, dim3(cb, g), dim3(kSumCols, kSumRows), 0, s, in, tmp, R, M, rows);
  hipLaunchKernelGGL(k_sum_rows, dim3(cb, 1), dim3(kSumCols, kSumRows), 0, s, tmp, out, g, M, g);
  return hipGetLastError();
}
constexpr int kLossBlocks = 1024;
int loss_partials() { return kLossBlocks; }
hipError_t launch_loss(const float *y, const float *t, float *dy, float *partial, float *loss,
                       float focus, long long n, hipStream_t s) {
  const float inv = 1.f / (float)n;
  hipLaunchKernelGGL(k_loss, dim3(kLossBlocks), dim3(kLossThreads), 0, s, y, t, dy, partial, n, inv,
                     focus);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kLossFinal), 0, s, partial, kLossBlocks, inv, loss);
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

static bool al4(long long v) { return v % 4 == 0; }

// Picks the staging modes: float4 loads along an operand's unit-stride axis
// when that axis' extent, the other strides, the segment offset and the base
// are all multiples of four floats; the column-major epilogue when C is
// unit-stride along m under the same conditions (and gelu_out, if any, 16-byte
// aligned).
static bool al8(long long v) { return v % 8 == 0; }

template <int AM>
static void launch_b(const GemmArgs &g, int bm, dim3 grid, hipStream_t s) {
  switch (bm) {
    case 0: hipLaunchKernelGGL((k_gemm<AM, 0>), grid, dim3(kThreads), 0, s, g); break;
    case 1: hipLaunchKernelGGL((k_gemm<AM, 1>), grid, dim3(kThreads), 0, s, g); break;
    case 2: hipLaunchKernelGGL((k_gemm<AM, 2>), grid, dim3(kThreads), 0, s, g); break;
    case 3: hipLaunchKernelGGL((k_gemm<AM, 3>), grid, dim3(kThreads), 0, s, g); break;
    default: hipLaunchKernelGGL((k_gemm<AM, 4>), grid, dim3(kThreads), 0, s, g); break;
  }
}

hipError_t launch_gemm(const GemmArgs &g0, hipStream_t s) {
  if (g0.M <= 0 || g0.N <= 0 || g0.K <= 0 || g0.batch <= 0) return hipSuccess;
  GemmArgs g = g0;
  int am = 0, bm = 0;
  if (g.a_bf16) {  // BF16 operand: eight-element loads only
    const bool ok = (uintptr_t)g.A % 16 == 0 && al8(g.sAb) && al8(g.a_seg_off) &&
                    (g.a_seg_k >= g.K || al8(g.a_seg_k));
    if (ok && g.sAk == 1 && al8(g.K) && al8(g.sAm)) am = 3;
    else if (ok && g.sAm == 1 && al8(g.M) && al8(g.sAk)) am = 4;
    else return hipErrorInvalidValue;
  } else {
    const bool a16 = (uintptr_t)g.A % 16 == 0 && al4(g.sAb) && al4(g.a_seg_off) &&
                     (g.a_seg_k >= g.K || al4(g.a_seg_k));
    if (a16 && g.sAk == 1 && al4(g.K) && al4(g.sAm)) am = 1;
    else if (a16 && g.sAm == 1 && al4(g.M) && al4(g.sAk)) am = 2;
  }
  if (g.b_bf16) {
    const bool ok = (uintptr_t)g.B % 16 == 0 && al8(g.sBb) && al8(g.b_seg_off) &&
                    (g.b_seg_k >= g.K || al8(g.b_seg_k));
    if (ok && g.sBn == 1 && al8(g.N) && al8(g.sBk)) bm = 3;
    else if (ok && g.sBk == 1 && al8(g.K) && al8(g.sBn)) bm = 4;
    else return hipErrorInvalidValue;
  } else {
    const bool b16 = (uintptr_t)g.B % 16 == 0 && al4(g.sBb) && al4(g.b_seg_off) &&
                     (g.b_seg_k >= g.K || al4(g.b_seg_k));
    if (b16 && g.sBn == 1 && al4(g.N) && al4(g.sBk)) bm = 1;
    else if (b16 && g.sBk == 1 && al4(g.K) && al4(g.sBn)) bm = 2;
  }
  if ((g.c_bf16 && g.beta != 0.f) || (g.gelu_z && g.gelu_bf16)) return hipErrorInvalidValue;
  g.c_mfast = (g.sCm == 1 && g.sCn != 1 && al4(g.M) && al4(g.sCn) && al4(g.sCb) &&
               (uintptr_t)g.C % 16 == 0 && (uintptr_t)g.gelu_out % 16 == 0 &&
               (uintptr_t)g.gelu_z % 16 == 0) ? 1 : 0;
  dim3 grid((g.N + kBN - 1) / kBN, (g.M + kBM - 1) / kBM, g.batch);
  switch (am) {
    case 0: launch_b<0>(g, bm, grid, s); break;
    case 1: launch_b<1>(g, bm, grid, s); break;
    case 2: launch_b<2>(g, bm, grid, s); break;
    case 3: launch_b<3>(g, bm, grid, s); break;
    default: launch_b<4>(g, bm, grid, s); break;
  }
  return hipGetLastError();
}

}  // namespace bbsur
