// Device-side argument blocks of the surrogate kernels (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

namespace bbsur {

// C[b](m, n) = alpha * sum_k A[b](m, k) B[b](k, n) + beta * C[b](m, n) + bias[m]
//   A(m, k) at A + b*sAb + m*sAm + (k mod seg)*sAk + [k >= a_seg_k]*a_seg_off
//   B(k, n) at B + b*sBb + (k mod seg)*sBk + n*sBn + [k >= b_seg_k]*b_seg_off
//   C(m, n) at C + b*sCb + m*sCm + n*sCn
// a_seg_k / b_seg_k must be multiples of 32 (or >= K for one segment).
struct GemmArgs {
  const float *A, *B;
  float *C;
  const float *bias;
  int M, N, K, batch;
  long long sAb, sAm, sAk, a_seg_off;
  long long sBb, sBk, sBn, b_seg_off;
  long long sCb, sCm, sCn;
  int a_seg_k, b_seg_k;
  int a_kfast, b_nfast;  // which axis is unit-stride (staging order of the scalar path)
  int c_mfast;           // set by the launcher: column-major epilogue
  float alpha, beta;
  float *gelu_out;       // optional second output, with C's strides: GELU(C(m, n)), or
                         // with gelu_z set C(m, n) * GELU'(gelu_z(m, n)) instead of C
  const float *gelu_z;
  // BF16 storage (the pointers above then address __bf16 elements): operand A
  // or B (staged with eight-element loads; the launcher rejects layouts that do
  // not allow them), output C (not with beta != 0), the GELU output
  int a_bf16, b_bf16, c_bf16, gelu_bf16;
};

}  // namespace bbsur
