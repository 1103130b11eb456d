// Viscoelastic FDTD step kernels for gfx950 (BabelBrain Section 2.3, Eq. 1).
//
// One time step is two launches:
//   k_velocity : v^{n-1/2} -> v^{n+1/2} (Eq. 1 rows 1-3) and the source force
//                on the v_z faces of plane ks (Section 2.3)
//   k_stress   : sigma^n -> sigma^{n+1}, Zener memory variables, peak |p|
//                capture (Eq. 1 rows 4-9, Section 3.2)
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

// Velocity update (Eq. 1 rows 1-3) of one tile: x segment bx (one cell per
// lane), rows by * blockDim.y + threadIdx.y, planes [k0, k1).  On plane ks the
// v_z faces also receive the source force (src_c Re S - src_s Im S, scaled by
// the face buoyancy): a normal-traction jump of 2 S across z = (ks + 1/2) dx.
__device__ __forceinline__ void velocity_tile(const StepArgs &A, int bx, int by, int k0, int k1,
                                              float src_c, float src_s) {
  const Grid g = A.g;
  const int i = bx * kSeg + threadIdx.x;
  const int j = by * blockDim.y + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
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
  const int seg = bx;  // blockDim.x == kSeg: one wave = one row segment
  for (int k = k0; k < k1; ++k) {
    const long long c = g.off(i, j, k);
    const bool pz = in_layer(k, g.nz, g.L);
    const int cl = __builtin_amdgcn_readfirstlane(A.cls[((long long)k * g.ny + j) * A.nseg + seg]);
    if (cl) {
      // acoustic path: the three normal stresses are equal and the shear
      // stresses vanish throughout the stencil's reach
      const float b = 1.f / lut[(cl - 1) * kLutW + kRhoS];
      float d1 = DP(sxx, c, 1), e2 = DP(sxx, c, P), f3 = DP(sxx, c, PL);
      if (px) d1 = cpml(A.psi[0], c, tx.z, tx.w, d1);
      if (py) e2 = cpml(A.psi[4], c, ty.z, ty.w, e2);
      if (pz) f3 = cpml(A.psi[8], c, A.pml.z[k].z, A.pml.z[k].w, f3);
      vx[c] += b * d1;
      vy[c] += b * e2;
      if (k == g.ks) {
        const float2 q = A.src[(long long)j * g.nx + i];
        f3 += src_c * q.x - src_s * q.y;
      }
      vz[c] += b * f3;
      continue;
    }
    const float r0 = lut[idx[c] * kLutW + kRhoS];
    const float bx = 2.f / (r0 + lut[idx[c + 1] * kLutW + kRhoS]);
    const float by = 2.f / (r0 + lut[idx[c + P] * kLutW + kRhoS]);
    const float bz = 2.f / (r0 + lut[idx[c + PL] * kLutW + kRhoS]);
    float d1 = DP(sxx, c, 1), d2 = DM(sxy, c, P), d3 = DM(sxz, c, PL);
    float e1 = DM(sxy, c, 1), e2 = DP(syy, c, P), e3 = DM(syz, c, PL);
    float f1 = DM(sxz, c, 1), f2 = DM(syz, c, P), f3 = DP(szz, c, PL);
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
    float fz = f1 + f2 + f3;
    if (k == g.ks) {  // traction source: force layer on the v_z faces of plane ks
      const float2 q = A.src[(long long)j * g.nx + i];
      fz += src_c * q.x - src_s * q.y;
    }
    vz[c] += bz * fz;
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

// Stress + memory update (Eq. 1 rows 4-9) and peak capture of one tile;
// capture is this step's flag.
__device__ __forceinline__ void stress_tile(const StepArgs &A, int bx, int by, int k0, int k1,
                                            int capture) {
  const Grid g = A.g;
  const int i = bx * kSeg + threadIdx.x;
  const int j = by * blockDim.y + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
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
  const int seg = bx;
  for (int k = k0; k < k1; ++k) {
    const long long c = g.off(i, j, k);
    const bool pz = in_layer(k, g.nz, g.L);
    const int cl = __builtin_amdgcn_readfirstlane(A.cls[((long long)k * g.ny + j) * A.nseg + seg]);
    if (cl) {
      // acoustic path: only the (equal) normal stresses change
      float exx = DM(vx, c, 1), eyy = DM(vy, c, P), ezz = DM(vz, c, PL);
      if (px) exx = cpml(A.psi[9], c, tx.x, tx.y, exx);
      if (py) eyy = cpml(A.psi[10], c, ty.x, ty.y, eyy);
      if (pz) ezz = cpml(A.psi[11], c, A.pml.z[k].x, A.pml.z[k].y, ezz);
      const float sn = sxxp[c] + lut[(cl - 1) * kLutW + kPiU] * (exx + eyy + ezz);
      sxxp[c] = sn;
      syyp[c] = sn;
      szzp[c] = sn;
      if (capture) {
        const long long q = ((long long)k * g.ny + j) * g.nx + i;
        const float a = fabsf(sn + sn + sn) / 3.f;
        const float p = A.peak[q];
        if (a > p || a != a) A.peak[q] = a;
      }
      continue;
    }
    float exx = DM(vx, c, 1), eyy = DM(vy, c, P), ezz = DM(vz, c, PL);
    float dyvx = DP(vx, c, P), dxvy = DP(vy, c, 1);
    float dzvx = DP(vx, c, PL), dxvz = DP(vz, c, 1);
    float dzvy = DP(vy, c, PL), dyvz = DP(vz, c, P);
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
    sxxp[c] = sxx; syyp[c] = syy; szzp[c] = szz;
    rxxp[c] = rxx; ryyp[c] = ryy; rzzp[c] = rzz;
    sxyp[c] = sxy; sxzp[c] = sxz; syzp[c] = syz;
    rxyp[c] = rxy; rxzp[c] = rxz; ryzp[c] = ryz;
    if (capture) {
      const long long q = ((long long)k * g.ny + j) * g.nx + i;
      const float a = fabsf(sxx + syy + szz) / 3.f;
      const float p = A.peak[q];
      if (a > p || a != a) A.peak[q] = a;
    }
  }
}

__global__ void __launch_bounds__(256) k_velocity(StepArgs A) {
  const int k0 = blockIdx.z * A.kchunk;
  velocity_tile(A, blockIdx.x, blockIdx.y, k0, min(k0 + A.kchunk, A.g.nz), A.src_c, A.src_s);
}

__global__ void __launch_bounds__(256) k_stress(StepArgs A) {
  const int k0 = blockIdx.z * A.kchunk;
  stress_tile(A, blockIdx.x, blockIdx.y, k0, min(k0 + A.kchunk, A.g.nz), A.capture);
}

// Persistent batched step kernels: a fixed grid walks the live prefix of the
// (solve, tile) table; every solve keeps its own grid, tables, step count and
// source coefficients.  The per-cell arithmetic is the single-solve tile code.
template <int BY>
__global__ void __launch_bounds__(kSeg * BY)
    k_velocity_batched(const StepArgs *__restrict__ desc, const BatchTile *__restrict__ tiles,
                       int n_tiles, const float2 *__restrict__ coef, int max_steps, int n) {
  for (int t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const BatchTile tl = tiles[t];
    const float2 cs = coef[(long long)tl.solve * max_steps + n];
    velocity_tile(desc[tl.solve], tl.bx, tl.by, tl.k0, tl.k1, cs.x, cs.y);
  }
}

template <int BY>
__global__ void __launch_bounds__(kSeg * BY)
    k_stress_batched(const StepArgs *__restrict__ desc, const BatchTile *__restrict__ tiles,
                     int n_tiles, const int *__restrict__ cap, int n) {
  for (int t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const BatchTile tl = tiles[t];
    stress_tile(desc[tl.solve], tl.bx, tl.by, tl.k0, tl.k1, (n + 1 >= cap[tl.solve]) ? 1 : 0);
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

// Segment classes (see kSeg): m + 1 if every cell within two cells of the
// segment holds lossless fluid m, else 0.  Reads the padded, ghost-replicated
// index map, so cells outside the grid count as their edge neighbour.
__global__ void k_classify(const uint8_t *__restrict__ idx, uint8_t *__restrict__ cls, Grid g,
                           int nseg, const float *__restrict__ lut) {
  const long long total = (long long)nseg * g.ny * g.nz;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int sg = (int)(t % nseg);
    const long long r = t / nseg;
    const int j = (int)(r % g.ny), k = (int)(r / g.ny);
    const int x0 = sg * kSeg;
    const int xa = x0 - kGhost, xb = min(x0 + kSeg - 1, g.nx - 1) + kGhost;
    const int m = idx[g.off(x0, j, k)];
    bool ok = m < 255 && lut[m * kLutW + kLossless] != 0.f;
    for (int dk = -kGhost; ok && dk <= kGhost; ++dk)
      for (int dj = -kGhost; ok && dj <= kGhost; ++dj) {
        const uint8_t *row = idx + g.off(0, j + dj, k + dk);
        for (int x = xa; x <= xb; ++x)
          if (row[x] != m) {
            ok = false;
            break;
          }
      }
    cls[t] = ok ? (uint8_t)(m + 1) : (uint8_t)0;
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

static constexpr int kBX = kSeg, kBY = 4;

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

hipError_t launch_classify(const uint8_t *idx, uint8_t *cls, const Grid &g, int nseg,
                           const float *lut, hipStream_t s) {
  hipLaunchKernelGGL(k_classify, dim3(4096), dim3(256), 0, s, idx, cls, g, nseg, lut);
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

template <int BY>
static hipError_t batched_step(const StepArgs *desc, const BatchTile *tiles, int n_tiles,
                               const float2 *coef, const int *cap, int max_steps, int n,
                               int blocks, hipStream_t s) {
  const dim3 grid(min(blocks, n_tiles)), block(kSeg, BY, 1);
  hipLaunchKernelGGL(k_velocity_batched<BY>, grid, block, 0, s, desc, tiles, n_tiles, coef,
                     max_steps, n);
  hipLaunchKernelGGL(k_stress_batched<BY>, grid, block, 0, s, desc, tiles, n_tiles, cap, n);
  return hipGetLastError();
}

hipError_t launch_batched_step(int by, const StepArgs *desc, const BatchTile *tiles, int n_tiles,
                               const float2 *coef, const int *cap, int max_steps, int n,
                               int blocks, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  switch (by) {
    case 1: return batched_step<1>(desc, tiles, n_tiles, coef, cap, max_steps, n, blocks, s);
    case 2: return batched_step<2>(desc, tiles, n_tiles, coef, cap, max_steps, n, blocks, s);
    case 4: return batched_step<4>(desc, tiles, n_tiles, coef, cap, max_steps, n, blocks, s);
    case 8: return batched_step<8>(desc, tiles, n_tiles, coef, cap, max_steps, n, blocks, s);
    default: return hipErrorInvalidValue;
  }
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
