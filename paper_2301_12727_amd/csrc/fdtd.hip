// Viscoelastic FDTD step kernels for gfx950 (BabelBrain Section 2.3, Eq. 1).
//
// One time step is two launches:
//   k_velocity : v^{n-1/2} -> v^{n+1/2}   (Eq. 1 rows 1-3)
//   k_stress   : sigma^n -> sigma^{n+1}, Zener memory variables, soft source
//                on plane ks, peak |p| capture (Eq. 1 rows 4-9, Section 3.2)
// Both are HBM-bandwidth bound stencils.  A block is a 64x4 x-y tile of
// columns marching over a chunk of z; x is the fastest (coalesced) axis.  The
// absorbing layer (CPML) is applied per cell behind a slab test that is uniform
// across most waves.
#include "bbfd_dev.h"

namespace bbfd {

#define C1 (9.0f / 8.0f)
#define C2 (-1.0f / 24.0f)
// 4th-order staggered differences (times dx): forward one sits at +1/2 of the
// centre sample, backward one at the centre from samples stored at +1/2.
#define DP(a, c, s) (C1 * ((a)[(c) + (s)] - (a)[(c)]) + C2 * ((a)[(c) + 2 * (s)] - (a)[(c) - (s)]))
#define DM(a, c, s) (C1 * ((a)[(c)] - (a)[(c) - (s)]) + C2 * ((a)[(c) + (s)] - (a)[(c) - 2 * (s)]))

__device__ __forceinline__ float cpml(float *psi, long long c, float b, float a, float d) {
  float p = b * psi[c] + a * d;
  psi[c] = p;
  return d + p;
}

__device__ __forceinline__ bool in_layer(int i, int n, int L) { return i < L || i >= n - L; }

__global__ void __launch_bounds__(256) k_velocity(StepArgs A) {
  const Grid g = A.g;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const int k0 = blockIdx.z * A.kchunk;
  const int k1 = min(k0 + A.kchunk, g.nz);
  const long long P = g.pitch, PL = g.plane;
  const float *__restrict__ sxx = A.f[SXX], *__restrict__ syy = A.f[SYY];
  const float *__restrict__ szz = A.f[SZZ], *__restrict__ sxy = A.f[SXY];
  const float *__restrict__ sxz = A.f[SXZ], *__restrict__ syz = A.f[SYZ];
  float *__restrict__ vx = A.f[VX], *__restrict__ vy = A.f[VY], *__restrict__ vz = A.f[VZ];
  const uint8_t *__restrict__ idx = A.idx;
  const float *__restrict__ lut = A.lut;
  const bool px = in_layer(i, g.nx, g.L), py = in_layer(j, g.ny, g.L);
  const float4 tx = px ? A.pml.x[i] : make_float4(1.f, 0.f, 1.f, 0.f);
  const float4 ty = py ? A.pml.y[j] : make_float4(1.f, 0.f, 1.f, 0.f);
  for (int k = k0; k < k1; ++k) {
    const long long c = g.off(i, j, k);
    const float r0 = lut[idx[c] * kLutW + kRhoS];
    const float bx = 2.f / (r0 + lut[idx[c + 1] * kLutW + kRhoS]);
    const float by = 2.f / (r0 + lut[idx[c + P] * kLutW + kRhoS]);
    const float bz = 2.f / (r0 + lut[idx[c + PL] * kLutW + kRhoS]);
    float d1 = DP(sxx, c, 1), d2 = DM(sxy, c, P), d3 = DM(sxz, c, PL);
    float e1 = DM(sxy, c, 1), e2 = DP(syy, c, P), e3 = DM(syz, c, PL);
    float f1 = DM(sxz, c, 1), f2 = DM(syz, c, P), f3 = DP(szz, c, PL);
    const bool pz = in_layer(k, g.nz, g.L);
    if (px) {
      d1 = cpml(A.psi[0], c, tx.z, tx.w, d1);
      e1 = cpml(A.psi[3], c, tx.x, tx.y, e1);
      f1 = cpml(A.psi[6], c, tx.x, tx.y, f1);
    }
    if (py) {
      d2 = cpml(A.psi[1], c, ty.x, ty.y, d2);
      e2 = cpml(A.psi[4], c, ty.z, ty.w, e2);
      f2 = cpml(A.psi[7], c, ty.x, ty.y, f2);
    }
    if (pz) {
      const float4 tz = A.pml.z[k];
      d3 = cpml(A.psi[2], c, tz.x, tz.y, d3);
      e3 = cpml(A.psi[5], c, tz.x, tz.y, e3);
      f3 = cpml(A.psi[8], c, tz.z, tz.w, f3);
    }
    vx[c] += bx * (d1 + d2 + d3);
    vy[c] += by * (e1 + e2 + e3);
    vz[c] += bz * (f1 + f2 + f3);
  }
}

// Zener update of one stress component: memory variable relaxes by
// Crank-Nicolson toward -target, stress takes the elastic increment plus the
// mean of the old and new memory value (all pre-scaled by dt).
__device__ __forceinline__ float zener(float &s, float &r, float elastic, float target, float ra,
                                       float rb) {
  const float rn = ra * r - rb * target;
  s += elastic + 0.5f * (r + rn);
  r = rn;
  return s;
}

__device__ __forceinline__ void edge(float &s, float &r, float e, const float *lut, int m0, int m1,
                                     int m2, int m3, float ra, float rb) {
  const float *a = lut + m0 * kLutW, *b = lut + m1 * kLutW, *c = lut + m2 * kLutW,
              *d = lut + m3 * kLutW;
  const float mue = 4.f / (a[kInvMu] + b[kInvMu] + c[kInvMu] + d[kInvMu]);
  const float te = 0.25f * (a[kTauS] + b[kTauS] + c[kTauS] + d[kTauS]);
  zener(s, r, mue * (1.f + te) * e, mue * te * e, ra, rb);
}

__global__ void __launch_bounds__(256) k_stress(StepArgs A) {
  const Grid g = A.g;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const int k0 = blockIdx.z * A.kchunk;
  const int k1 = min(k0 + A.kchunk, g.nz);
  const long long P = g.pitch, PL = g.plane;
  const float *__restrict__ vx = A.f[VX], *__restrict__ vy = A.f[VY], *__restrict__ vz = A.f[VZ];
  float *__restrict__ sxxp = A.f[SXX], *__restrict__ syyp = A.f[SYY], *__restrict__ szzp = A.f[SZZ];
  float *__restrict__ sxyp = A.f[SXY], *__restrict__ sxzp = A.f[SXZ], *__restrict__ syzp = A.f[SYZ];
  float *__restrict__ rxxp = A.f[RXX], *__restrict__ ryyp = A.f[RYY], *__restrict__ rzzp = A.f[RZZ];
  float *__restrict__ rxyp = A.f[RXY], *__restrict__ rxzp = A.f[RXZ], *__restrict__ ryzp = A.f[RYZ];
  const uint8_t *__restrict__ idx = A.idx;
  const float *__restrict__ lut = A.lut;
  const float ra = A.relax_a, rb = A.relax_b;
  const bool px = in_layer(i, g.nx, g.L), py = in_layer(j, g.ny, g.L);
  const float4 tx = px ? A.pml.x[i] : make_float4(1.f, 0.f, 1.f, 0.f);
  const float4 ty = py ? A.pml.y[j] : make_float4(1.f, 0.f, 1.f, 0.f);
  for (int k = k0; k < k1; ++k) {
    const long long c = g.off(i, j, k);
    float exx = DM(vx, c, 1), eyy = DM(vy, c, P), ezz = DM(vz, c, PL);
    float dyvx = DP(vx, c, P), dxvy = DP(vy, c, 1);
    float dzvx = DP(vx, c, PL), dxvz = DP(vz, c, 1);
    float dzvy = DP(vy, c, PL), dyvz = DP(vz, c, P);
    const bool pz = in_layer(k, g.nz, g.L);
    if (px) {
      exx = cpml(A.psi[9], c, tx.x, tx.y, exx);
      dxvy = cpml(A.psi[13], c, tx.z, tx.w, dxvy);
      dxvz = cpml(A.psi[15], c, tx.z, tx.w, dxvz);
    }
    if (py) {
      eyy = cpml(A.psi[10], c, ty.x, ty.y, eyy);
      dyvx = cpml(A.psi[12], c, ty.z, ty.w, dyvx);
      dyvz = cpml(A.psi[17], c, ty.z, ty.w, dyvz);
    }
    if (pz) {
      const float4 tz = A.pml.z[k];
      ezz = cpml(A.psi[11], c, tz.x, tz.y, ezz);
      dzvx = cpml(A.psi[14], c, tz.z, tz.w, dzvx);
      dzvy = cpml(A.psi[16], c, tz.z, tz.w, dzvy);
    }
    const int m0 = idx[c], mx = idx[c + 1], my = idx[c + P], mz = idx[c + PL];
    const int mxy = idx[c + 1 + P], mxz = idx[c + 1 + PL], myz = idx[c + P + PL];
    const float *L0 = lut + m0 * kLutW;
    const float th = exx + eyy + ezz;
    float sxx = sxxp[c], syy = syyp[c], szz = szzp[c];
    float rxx = rxxp[c], ryy = ryyp[c], rzz = rzzp[c];
    {
      const float piu = L0[kPiU], muu2 = 2.f * L0[kMuU];
      const float pit = L0[kPiTau], mut2 = 2.f * L0[kMuTau];
      float lat = eyy + ezz;
      zener(sxx, rxx, piu * th - muu2 * lat, pit * th - mut2 * lat, ra, rb);
      lat = exx + ezz;
      zener(syy, ryy, piu * th - muu2 * lat, pit * th - mut2 * lat, ra, rb);
      lat = exx + eyy;
      zener(szz, rzz, piu * th - muu2 * lat, pit * th - mut2 * lat, ra, rb);
    }
    float sxy = sxyp[c], sxz = sxzp[c], syz = syzp[c];
    float rxy = rxyp[c], rxz = rxzp[c], ryz = ryzp[c];
    edge(sxy, rxy, dyvx + dxvy, lut, m0, mx, my, mxy, ra, rb);
    edge(sxz, rxz, dzvx + dxvz, lut, m0, mx, mz, mxz, ra, rb);
    edge(syz, ryz, dzvy + dyvz, lut, m0, my, mz, myz, ra, rb);
    if (k == g.ks) {
      const float2 s = A.src[(long long)j * g.nx + i];
      const float dp = A.src_c * s.x - A.src_s * s.y;
      sxx -= dp;
      syy -= dp;
      szz -= dp;
    }
    sxxp[c] = sxx; syyp[c] = syy; szzp[c] = szz;
    rxxp[c] = rxx; ryyp[c] = ryy; rzzp[c] = rzz;
    sxyp[c] = sxy; sxzp[c] = sxz; syzp[c] = syz;
    rxyp[c] = rxy; rxzp[c] = rxz; ryzp[c] = ryz;
    if (A.capture) {
      const long long q = ((long long)k * g.ny + j) * g.nx + i;
      const float a = fabsf(sxx + syy + szz) / 3.f;
      const float p = A.peak[q];
      if (a > p || a != a) A.peak[q] = a;
    }
  }
}

// Padded uint8 index map with edge-replicated ghosts; flags out-of-range
// indices (which are replaced by 0 so the solve stays in bounds).
__global__ void k_pack_idx(const uint8_t *__restrict__ mat, uint8_t *__restrict__ idx, Grid g,
                           int n_mat, int *flags) {
  const long long total = (long long)g.rows * (g.nz + 2 * kGhost) * g.pitch;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const long long r = t / g.pitch;
    const int i = min(max((int)(t - r * g.pitch) - kGhost, 0), g.nx - 1);
    const int j = min(max((int)(r % g.rows) - kGhost, 0), g.ny - 1);
    const int k = min(max((int)(r / g.rows) - kGhost, 0), g.nz - 1);
    int m = mat[((long long)k * g.ny + j) * g.nx + i];
    if (m >= n_mat) {
      atomicOr(flags, kStatusIndex);
      m = 0;
    }
    idx[kX0 - kGhost + t] = (uint8_t)m;
  }
}

__global__ void k_fill(float4 *__restrict__ p, long long n4, float v) {
  const float4 z = make_float4(v, v, v, v);
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n4;
       t += (long long)gridDim.x * blockDim.x)
    p[t] = z;
}

__global__ void k_fill_tail(float *p, long long n, float v) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x)
    p[t] = v;
}

// Argmax over the interior outside the layer (lowest linear index on ties) and
// finiteness over the whole map: per-block partials, then one block.
constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 512;

__device__ __forceinline__ bool better(float v, long long i, float bv, long long bi) {
  return v > bv || (v == bv && i < bi);
}

__global__ void __launch_bounds__(kRedThreads)
    k_argmax_partial(const float *__restrict__ P, int nx, int ny, int nz, int L,
                     float *__restrict__ pv, long long *__restrict__ pi, int *flags) {
  __shared__ float sv[kRedThreads];
  __shared__ long long si[kRedThreads];
  __shared__ int sbad;
  if (threadIdx.x == 0) sbad = 0;
  __syncthreads();
  float bv = -1.f;
  long long bi = -1;
  int bad = 0;
  const long long n = (long long)nx * ny * nz;
  for (long long q = blockIdx.x * (long long)kRedThreads + threadIdx.x; q < n;
       q += (long long)gridDim.x * kRedThreads) {
    const float v = P[q];
    if (!isfinite(v)) {
      bad = 1;
      continue;
    }
    const long long r = q / nx;
    const int i = (int)(q - r * nx), j = (int)(r % ny), k = (int)(r / ny);
    if (i < L || i >= nx - L || j < L || j >= ny - L || k < L || k >= nz - L) continue;
    if (better(v, q, bv, bi)) {
      bv = v;
      bi = q;
    }
  }
  if (bad) atomicOr(&sbad, 1);
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const float v = sv[threadIdx.x + s];
      const long long q = si[threadIdx.x + s];
      if (q >= 0 && (si[threadIdx.x] < 0 || better(v, q, sv[threadIdx.x], si[threadIdx.x]))) {
        sv[threadIdx.x] = v;
        si[threadIdx.x] = q;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = sv[0];
    pi[blockIdx.x] = si[0];
    if (sbad) atomicOr(flags, kStatusDiverged);
  }
}

__global__ void __launch_bounds__(kRedThreads)
    k_argmax_final(const float *__restrict__ pv, const long long *__restrict__ pi, int nparts,
                   Status *st) {
  __shared__ float sv[kRedThreads];
  __shared__ long long si[kRedThreads];
  float bv = -1.f;
  long long bi = -1;
  for (int t = threadIdx.x; t < nparts; t += kRedThreads) {
    if (pi[t] >= 0 && (bi < 0 || better(pv[t], pi[t], bv, bi))) {
      bv = pv[t];
      bi = pi[t];
    }
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const float v = sv[threadIdx.x + s];
      const long long q = si[threadIdx.x + s];
      if (q >= 0 && (si[threadIdx.x] < 0 || better(v, q, sv[threadIdx.x], si[threadIdx.x]))) {
        sv[threadIdx.x] = v;
        si[threadIdx.x] = q;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    st->peak_value = sv[0];
    st->peak_index = si[0];
  }
}

// ------------------------------------------------------------------ launchers

static constexpr int kBX = 64, kBY = 4;

static dim3 step_grid(const StepArgs &a) {
  return dim3((a.g.nx + kBX - 1) / kBX, (a.g.ny + kBY - 1) / kBY,
              (a.g.nz + a.kchunk - 1) / a.kchunk);
}

hipError_t launch_velocity(const StepArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_velocity, step_grid(a), dim3(kBX, kBY, 1), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_stress(const StepArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_stress, step_grid(a), dim3(kBX, kBY, 1), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_step(const StepArgs &a, hipStream_t s) {
  hipError_t e = launch_velocity(a, s);
  if (e != hipSuccess) return e;
  return launch_stress(a, s);
}

hipError_t launch_pack(const uint8_t *mat, uint8_t *idx, const Grid &g, int n_mat, int *flags,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_pack_idx, dim3(2048), dim3(256), 0, s, mat, idx, g, n_mat, flags);
  return hipGetLastError();
}

hipError_t launch_fill(float *p, long long n, float v, hipStream_t s) {
  const long long n4 = ((uintptr_t)p % 16 == 0) ? n / 4 : 0;
  if (n4 > 0) {
    long long blocks = (n4 + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, (float4 *)p, n4, v);
  }
  const long long rest = n - 4 * n4;
  if (rest > 0) {
    long long blocks = (rest + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_fill_tail, dim3((unsigned)blocks), dim3(256), 0, s, p + 4 * n4, rest, v);
  }
  return hipGetLastError();
}

int argmax_partials() { return kRedBlocks; }

hipError_t launch_argmax(const float *P, int nx, int ny, int nz, int L, float *pv, long long *pi,
                         Status *st, hipStream_t s) {
  hipLaunchKernelGGL(k_argmax_partial, dim3(kRedBlocks), dim3(kRedThreads), 0, s, P, nx, ny, nz,
                     L, pv, pi, &st->flags);
  hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(kRedThreads), 0, s, pv, pi, kRedBlocks, st);
  return hipGetLastError();
}

}  // namespace bbfd
