// Viscoelastic FDTD step kernels for gfx950 (BabelBrain Section 2.3, Eq. 1).
//
// One time step is two launches:
//   k_velocity : v^{n-1/2} -> v^{n+1/2} (Eq. 1 rows 1-3) and the source force
//                on the v_z faces of plane ks (Section 2.3)
//   k_stress   : sigma^n -> sigma^{n+1}, Zener memory variables, peak |p|
//                capture (Eq. 1 rows 4-9, Section 3.2)
// Both are HBM-bandwidth-bound stencils.  A tile is a 64 x 4 block of x-y
// columns marching over a chunk of z; x is the fastest (coalesced) axis and
// each wave owns one 64-cell row segment, so the segment class (acoustic or
// elastic branch) is wave-uniform.  Per block the material table is staged
// in LDS, so the material gathers of a cell are LDS reads rather than a
// second dependent trip to the cache hierarchy, and the class bytes of a
// segment's z column are read four at a time through the scalar cache, one
// group ahead.  Tiles are assigned so that each XCD works on a contiguous
// band of them, keeping the halo rows of neighbouring tiles in one L2.  The
// absorbing layer (CPML) is applied per cell behind a slab test that is
// uniform across most waves.
#include "bbfd_dev.h"

namespace bbfd {

#define C1 (9.0f / 8.0f)
#define C2 (-1.0f / 24.0f)
// 4th-order staggered differences (times dx): forward one sits at +1/2 of the
// centre sample, backward one at the centre from samples stored at +1/2.
#define DP(a, c, s) (C1 * ((a)[(c) + (s)] - (a)[(c)]) + C2 * ((a)[(c) + 2 * (s)] - (a)[(c) - (s)]))
#define DM(a, c, s) (C1 * ((a)[(c)] - (a)[(c) - (s)]) + C2 * ((a)[(c) + (s)] - (a)[(c) - 2 * (s)]))

typedef __attribute__((address_space(4))) const uint32_t ScalarU32;

// CPML memory update and corrected derivative: psi <- b psi + a d, d + psi.
__device__ __forceinline__ float cpml_apply(float *__restrict__ psi, long long c, float &q, float b,
                                            float a, float d) {
  q = b * q + a * d;
  psi[c] = q;
  return d + q;
}

__device__ __forceinline__ bool in_layer(int i, int n, int L) { return i < L || i >= n - L; }

// Blocks are dispatched to the 8 XCDs round-robin; this maps dispatch order b
// of n blocks onto tile ids so that XCD x owns the contiguous tile range
// [x * (n / 8) + min(x, n % 8), ...) (a bijection on [0, n)).
__device__ __forceinline__ int xcd_band(int b, int n) {
  const int per = n >> 3, rem = n & 7, x = b & 7, r = b >> 3;
  return x * per + min(x, rem) + r;
}

// Copies the material table of a solve into LDS (whole block; caller syncs).
__device__ __forceinline__ void stage_lut(float *s_lut, const float *lut, int n_mat) {
  const int nt = blockDim.x * blockDim.y, t0 = threadIdx.y * blockDim.x + threadIdx.x;
  for (int t = t0; t < n_mat * kLutW; t += nt) s_lut[t] = lut[t];
}

// Wave-uniform class reader of one segment's z column: bytes are fetched as
// 32-bit words through the scalar cache, the next word one group early.
struct ClassColumn {
  const ScalarU32 *w;
  uint32_t cur, nxt;
  __device__ __forceinline__ ClassColumn(const StepArgs &A, int j, int seg, int k0) {
    w = (const ScalarU32 *)(A.cls + ((long long)j * A.nseg + seg) * A.kpad);
    cur = w[k0 >> 2];
    nxt = w[(k0 >> 2) + 1];
  }
  __device__ __forceinline__ int at(int k, int k0) {
    if ((k & 3) == 0 && k != k0) {
      cur = nxt;
      nxt = w[(k >> 2) + 1];
    }
    return (int)((cur >> ((k & 3) * 8)) & 0xffu);
  }
};

// Every cell update below first issues all of its loads (stencil values, own
// state, layer memories, material indices) and only then computes and
// stores, so a wave has one round trip to memory per cell instead of a chain
// of load-wait-store steps.

// Velocity update (Eq. 1 rows 1-3) of one tile: x segment bx (one cell per
// lane), row j (wave-uniform), planes [k0, k1); lut is the LDS copy of the
// material table.  On plane ks the v_z faces also receive the source force
// (src_c Re S - src_s Im S, scaled by the face buoyancy): a normal-traction
// jump of 2 S across z = (ks + 1/2) dx.
__device__ __forceinline__ void velocity_tile(const StepArgs &A, const float *lut, int bx, int j,
                                              int k0, int k1, float src_c, float src_s) {
  const Grid g = A.g;
  const int i = bx * kSeg + threadIdx.x;
  if (i >= g.nx || j >= g.ny) return;
  const long long P = g.pitch, PL = g.plane;
  const float *__restrict__ sxx = A.f[SXX], *__restrict__ syy = A.f[SYY];
  const float *__restrict__ szz = A.f[SZZ], *__restrict__ sxy = A.f[SXY];
  const float *__restrict__ sxz = A.f[SXZ], *__restrict__ syz = A.f[SYZ];
  float *__restrict__ vx = A.f[VX], *__restrict__ vy = A.f[VY], *__restrict__ vz = A.f[VZ];
  float *__restrict__ p0 = A.psi[0], *__restrict__ p1 = A.psi[1], *__restrict__ p2 = A.psi[2];
  float *__restrict__ p3 = A.psi[3], *__restrict__ p4 = A.psi[4], *__restrict__ p5 = A.psi[5];
  float *__restrict__ p6 = A.psi[6], *__restrict__ p7 = A.psi[7], *__restrict__ p8 = A.psi[8];
  const uint8_t *__restrict__ idx = A.idx;
  const float2 *__restrict__ srcp = A.src + (long long)j * g.nx + i;
  const bool px = in_layer(i, g.nx, g.L), py = in_layer(j, g.ny, g.L);
  const float4 tx = px ? A.pml.x[i] : make_float4(1.f, 0.f, 1.f, 0.f);
  const float4 ty = py ? A.pml.y[j] : make_float4(1.f, 0.f, 1.f, 0.f);
  ClassColumn col(A, j, bx, k0);
  for (int k = k0; k < k1; ++k) {
    const long long c = g.off(i, j, k);
    const bool pz = in_layer(k, g.nz, g.L);
    const bool on_src = k == g.ks;
    const int cl = col.at(k, k0);
    if (cl) {
      // acoustic path: the three normal stresses are equal and the shear
      // stresses vanish throughout the stencil's reach
      float d1 = DP(sxx, c, 1), e2 = DP(sxx, c, P), f3 = DP(sxx, c, PL);
      const float vxo = vx[c], vyo = vy[c], vzo = vz[c];
      float q0 = 0.f, q4 = 0.f, q8 = 0.f;
      if (px) q0 = p0[c];
      if (py) q4 = p4[c];
      if (pz) q8 = p8[c];
      float2 sq = make_float2(0.f, 0.f);
      if (on_src) sq = *srcp;
      const float4 tz = pz ? A.pml.z[k] : make_float4(1.f, 0.f, 1.f, 0.f);
      const float b = 1.f / lut[(cl - 1) * kLutW + kRhoS];
      if (px) d1 = cpml_apply(p0, c, q0, tx.z, tx.w, d1);
      if (py) e2 = cpml_apply(p4, c, q4, ty.z, ty.w, e2);
      if (pz) f3 = cpml_apply(p8, c, q8, tz.z, tz.w, f3);
      vx[c] = vxo + b * d1;
      vy[c] = vyo + b * e2;
      if (on_src) f3 += src_c * sq.x - src_s * sq.y;
      vz[c] = vzo + b * f3;
      continue;
    }
    const int m0 = idx[c], mx = idx[c + 1], my = idx[c + P], mz = idx[c + PL];
    float d1 = DP(sxx, c, 1), d2 = DM(sxy, c, P), d3 = DM(sxz, c, PL);
    float e1 = DM(sxy, c, 1), e2 = DP(syy, c, P), e3 = DM(syz, c, PL);
    float f1 = DM(sxz, c, 1), f2 = DM(syz, c, P), f3 = DP(szz, c, PL);
    const float vxo = vx[c], vyo = vy[c], vzo = vz[c];
    float q0 = 0.f, q1 = 0.f, q2 = 0.f, q3 = 0.f, q4 = 0.f, q5 = 0.f, q6 = 0.f, q7 = 0.f, q8 = 0.f;
    if (px) { q0 = p0[c]; q3 = p3[c]; q6 = p6[c]; }
    if (py) { q1 = p1[c]; q4 = p4[c]; q7 = p7[c]; }
    if (pz) { q2 = p2[c]; q5 = p5[c]; q8 = p8[c]; }
    float2 sq = make_float2(0.f, 0.f);
    if (on_src) sq = *srcp;
    const float4 tz = pz ? A.pml.z[k] : make_float4(1.f, 0.f, 1.f, 0.f);
    const float r0 = lut[m0 * kLutW + kRhoS];
    const float bx = 2.f / (r0 + lut[mx * kLutW + kRhoS]);
    const float by = 2.f / (r0 + lut[my * kLutW + kRhoS]);
    const float bz = 2.f / (r0 + lut[mz * kLutW + kRhoS]);
    if (px) {
      d1 = cpml_apply(p0, c, q0, tx.z, tx.w, d1);
      e1 = cpml_apply(p3, c, q3, tx.x, tx.y, e1);
      f1 = cpml_apply(p6, c, q6, tx.x, tx.y, f1);
    }
    if (py) {
      d2 = cpml_apply(p1, c, q1, ty.x, ty.y, d2);
      e2 = cpml_apply(p4, c, q4, ty.z, ty.w, e2);
      f2 = cpml_apply(p7, c, q7, ty.x, ty.y, f2);
    }
    if (pz) {
      d3 = cpml_apply(p2, c, q2, tz.x, tz.y, d3);
      e3 = cpml_apply(p5, c, q5, tz.x, tz.y, e3);
      f3 = cpml_apply(p8, c, q8, tz.z, tz.w, f3);
    }
    vx[c] = vxo + bx * (d1 + d2 + d3);
    vy[c] = vyo + by * (e1 + e2 + e3);
    float fz = f1 + f2 + f3;
    if (on_src) fz += src_c * sq.x - src_s * sq.y;  // traction source on the v_z faces of plane ks
    vz[c] = vzo + bz * fz;
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

__device__ __forceinline__ float2 edge_in(const float *lut, int m) {
  return *reinterpret_cast<const float2 *>(lut + m * kLutW + kInvMu);
}

// Shear component on an edge shared by cells with edge inputs a, b, c, d
// ({1/mu, tau_S} each): harmonic-mean modulus, arithmetic-mean tau_S.
__device__ __forceinline__ void edge(float &s, float &r, float e, float2 a, float2 b, float2 c,
                                     float2 d, float ra, float rb) {
  const float mue = 4.f / (a.x + b.x + c.x + d.x);
  const float te = 0.25f * (a.y + b.y + c.y + d.y);
  zener(s, r, mue * (1.f + te) * e, mue * te * e, ra, rb);
}

__device__ __forceinline__ void capture_peak(float *__restrict__ peak, long long q, float old,
                                             float s3) {
  const float a = fabsf(s3) / 3.f;
  if (a > old || a != a) peak[q] = a;
}

// Stress + memory update (Eq. 1 rows 4-9) and peak capture of one tile;
// capture is this step's flag.
__device__ __forceinline__ void stress_tile(const StepArgs &A, const float *lut, int bx, int j,
                                            int k0, int k1, int capture) {
  const Grid g = A.g;
  const int i = bx * kSeg + threadIdx.x;
  if (i >= g.nx || j >= g.ny) return;
  const long long P = g.pitch, PL = g.plane;
  const float *__restrict__ vx = A.f[VX], *__restrict__ vy = A.f[VY], *__restrict__ vz = A.f[VZ];
  float *__restrict__ sxxp = A.f[SXX], *__restrict__ syyp = A.f[SYY], *__restrict__ szzp = A.f[SZZ];
  float *__restrict__ sxyp = A.f[SXY], *__restrict__ sxzp = A.f[SXZ], *__restrict__ syzp = A.f[SYZ];
  float *__restrict__ rxxp = A.f[RXX], *__restrict__ ryyp = A.f[RYY], *__restrict__ rzzp = A.f[RZZ];
  float *__restrict__ rxyp = A.f[RXY], *__restrict__ rxzp = A.f[RXZ], *__restrict__ ryzp = A.f[RYZ];
  float *__restrict__ p9 = A.psi[9], *__restrict__ p10 = A.psi[10], *__restrict__ p11 = A.psi[11];
  float *__restrict__ p12 = A.psi[12], *__restrict__ p13 = A.psi[13], *__restrict__ p14 = A.psi[14];
  float *__restrict__ p15 = A.psi[15], *__restrict__ p16 = A.psi[16], *__restrict__ p17 = A.psi[17];
  float *__restrict__ peak = A.peak;
  const uint8_t *__restrict__ idx = A.idx;
  const float ra = A.relax_a, rb = A.relax_b;
  const bool px = in_layer(i, g.nx, g.L), py = in_layer(j, g.ny, g.L);
  const float4 tx = px ? A.pml.x[i] : make_float4(1.f, 0.f, 1.f, 0.f);
  const float4 ty = py ? A.pml.y[j] : make_float4(1.f, 0.f, 1.f, 0.f);
  ClassColumn col(A, j, bx, k0);
  for (int k = k0; k < k1; ++k) {
    const long long c = g.off(i, j, k);
    const long long q = ((long long)k * g.ny + j) * g.nx + i;
    const bool pz = in_layer(k, g.nz, g.L);
    const int cl = col.at(k, k0);
    if (cl) {
      // acoustic path: only the (equal) normal stresses change
      float exx = DM(vx, c, 1), eyy = DM(vy, c, P), ezz = DM(vz, c, PL);
      const float so = sxxp[c];
      float q9 = 0.f, q10 = 0.f, q11 = 0.f, pk = 0.f;
      if (px) q9 = p9[c];
      if (py) q10 = p10[c];
      if (pz) q11 = p11[c];
      if (capture) pk = peak[q];
      const float4 tz = pz ? A.pml.z[k] : make_float4(1.f, 0.f, 1.f, 0.f);
      if (px) exx = cpml_apply(p9, c, q9, tx.x, tx.y, exx);
      if (py) eyy = cpml_apply(p10, c, q10, ty.x, ty.y, eyy);
      if (pz) ezz = cpml_apply(p11, c, q11, tz.x, tz.y, ezz);
      const float sn = so + lut[(cl - 1) * kLutW + kPiU] * (exx + eyy + ezz);
      sxxp[c] = sn;
      syyp[c] = sn;
      szzp[c] = sn;
      if (capture) capture_peak(peak, q, pk, sn + sn + sn);
      continue;
    }
    const int m0 = idx[c], mx = idx[c + 1], my = idx[c + P], mz = idx[c + PL];
    const int mxy = idx[c + 1 + P], mxz = idx[c + 1 + PL], myz = idx[c + P + PL];
    float exx = DM(vx, c, 1), eyy = DM(vy, c, P), ezz = DM(vz, c, PL);
    float dyvx = DP(vx, c, P), dxvy = DP(vy, c, 1);
    float dzvx = DP(vx, c, PL), dxvz = DP(vz, c, 1);
    float dzvy = DP(vy, c, PL), dyvz = DP(vz, c, P);
    float sxx = sxxp[c], syy = syyp[c], szz = szzp[c];
    float rxx = rxxp[c], ryy = ryyp[c], rzz = rzzp[c];
    float sxy = sxyp[c], sxz = sxzp[c], syz = syzp[c];
    float rxy = rxyp[c], rxz = rxzp[c], ryz = ryzp[c];
    float q9 = 0.f, q10 = 0.f, q11 = 0.f, q12 = 0.f, q13 = 0.f, q14 = 0.f, q15 = 0.f, q16 = 0.f,
          q17 = 0.f, pk = 0.f;
    if (px) { q9 = p9[c]; q13 = p13[c]; q15 = p15[c]; }
    if (py) { q10 = p10[c]; q12 = p12[c]; q17 = p17[c]; }
    if (pz) { q11 = p11[c]; q14 = p14[c]; q16 = p16[c]; }
    if (capture) pk = peak[q];
    const float4 tz = pz ? A.pml.z[k] : make_float4(1.f, 0.f, 1.f, 0.f);
    if (px) {
      exx = cpml_apply(p9, c, q9, tx.x, tx.y, exx);
      dxvy = cpml_apply(p13, c, q13, tx.z, tx.w, dxvy);
      dxvz = cpml_apply(p15, c, q15, tx.z, tx.w, dxvz);
    }
    if (py) {
      eyy = cpml_apply(p10, c, q10, ty.x, ty.y, eyy);
      dyvx = cpml_apply(p12, c, q12, ty.z, ty.w, dyvx);
      dyvz = cpml_apply(p17, c, q17, ty.z, ty.w, dyvz);
    }
    if (pz) {
      ezz = cpml_apply(p11, c, q11, tz.x, tz.y, ezz);
      dzvx = cpml_apply(p14, c, q14, tz.z, tz.w, dzvx);
      dzvy = cpml_apply(p16, c, q16, tz.z, tz.w, dzvy);
    }
    const float4 L0 = *reinterpret_cast<const float4 *>(lut + m0 * kLutW);  // piU muU piTau muTau
    const float th = exx + eyy + ezz;
    {
      const float piu = L0.x, muu2 = 2.f * L0.y;
      const float pit = L0.z, mut2 = 2.f * L0.w;
      float lat = eyy + ezz;
      zener(sxx, rxx, piu * th - muu2 * lat, pit * th - mut2 * lat, ra, rb);
      lat = exx + ezz;
      zener(syy, ryy, piu * th - muu2 * lat, pit * th - mut2 * lat, ra, rb);
      lat = exx + eyy;
      zener(szz, rzz, piu * th - muu2 * lat, pit * th - mut2 * lat, ra, rb);
    }
    const float2 e0 = edge_in(lut, m0), ex = edge_in(lut, mx);
    const float2 ey = edge_in(lut, my), ez = edge_in(lut, mz);
    edge(sxy, rxy, dyvx + dxvy, e0, ex, ey, edge_in(lut, mxy), ra, rb);
    edge(sxz, rxz, dzvx + dxvz, e0, ex, ez, edge_in(lut, mxz), ra, rb);
    edge(syz, ryz, dzvy + dyvz, e0, ey, ez, edge_in(lut, myz), ra, rb);
    sxxp[c] = sxx; syyp[c] = syy; szzp[c] = szz;
    rxxp[c] = rxx; ryyp[c] = ryy; rzzp[c] = rzz;
    sxyp[c] = sxy; sxzp[c] = sxz; syzp[c] = syz;
    rxyp[c] = rxy; rxzp[c] = rxz; ryzp[c] = ryz;
    if (capture) capture_peak(peak, q, pk, sxx + syy + szz);
  }
}

// Tile t of a single solve: x segment fastest, then row block, then z chunk.
__device__ __forceinline__ void tile_coords(const StepArgs &A, int t, int &bx, int &by, int &k0,
                                            int &k1) {
  bx = t % A.nseg;
  const int r = t / A.nseg;
  by = r % A.nby;
  k0 = (r / A.nby) * A.kchunk;
  k1 = min(k0 + A.kchunk, A.g.nz);
}

__device__ __forceinline__ int wave_row() { return __builtin_amdgcn_readfirstlane(threadIdx.y); }

// Dynamic LDS of the step kernels: the material table, n_mat * kLutW floats.
extern __shared__ __align__(16) float s_lut[];

__global__ void __launch_bounds__(kSeg * kRows) k_velocity(StepArgs A) {
  stage_lut(s_lut, A.lut, A.n_mat);
  __syncthreads();
  int bx, by, k0, k1;
  tile_coords(A, xcd_band(blockIdx.x, gridDim.x), bx, by, k0, k1);
  velocity_tile(A, s_lut, bx, by * kRows + wave_row(), k0, k1, A.src_c, A.src_s);
}

__global__ void __launch_bounds__(kSeg * kRows) k_stress(StepArgs A) {
  stage_lut(s_lut, A.lut, A.n_mat);
  __syncthreads();
  int bx, by, k0, k1;
  tile_coords(A, xcd_band(blockIdx.x, gridDim.x), bx, by, k0, k1);
  stress_tile(A, s_lut, bx, by * kRows + wave_row(), k0, k1, A.capture);
}

// Persistent batched step kernels: a fixed grid walks the live prefix of the
// (solve, tile) table, each XCD over its own contiguous band of every round;
// every solve keeps its own grid, tables, step count and source
// coefficients.  The per-cell arithmetic is the single-solve tile code.
template <int BY>
__global__ void __launch_bounds__(kSeg * BY)
    k_velocity_batched(const StepArgs *__restrict__ desc, const BatchTile *__restrict__ tiles,
                       int n_tiles, const float2 *__restrict__ coef, int max_steps, int n) {
  int staged = -1;
  const int b = xcd_band(blockIdx.x, gridDim.x);
  for (int t = b; t < n_tiles; t += gridDim.x) {
    const BatchTile tl = tiles[t];
    if (tl.solve != staged) {
      __syncthreads();
      stage_lut(s_lut, desc[tl.solve].lut, desc[tl.solve].n_mat);
      __syncthreads();
      staged = tl.solve;
    }
    const float2 cs = coef[(long long)tl.solve * max_steps + n];
    velocity_tile(desc[tl.solve], s_lut, tl.bx, tl.by * BY + wave_row(), tl.k0, tl.k1, cs.x, cs.y);
  }
}

template <int BY>
__global__ void __launch_bounds__(kSeg * BY)
    k_stress_batched(const StepArgs *__restrict__ desc, const BatchTile *__restrict__ tiles,
                     int n_tiles, const int *__restrict__ cap, int n) {
  int staged = -1;
  const int b = xcd_band(blockIdx.x, gridDim.x);
  for (int t = b; t < n_tiles; t += gridDim.x) {
    const BatchTile tl = tiles[t];
    if (tl.solve != staged) {
      __syncthreads();
      stage_lut(s_lut, desc[tl.solve].lut, desc[tl.solve].n_mat);
      __syncthreads();
      staged = tl.solve;
    }
    stress_tile(desc[tl.solve], s_lut, tl.bx, tl.by * BY + wave_row(), tl.k0, tl.k1,
                (n + 1 >= cap[tl.solve]) ? 1 : 0);
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
// index map, so cells outside the grid count as their edge neighbour.  Written
// as one z column of kpad bytes per (row, segment).
__global__ void k_classify(const uint8_t *__restrict__ idx, uint8_t *__restrict__ cls, Grid g,
                           int nseg, int kpad, const float *__restrict__ lut) {
  const long long total = (long long)nseg * g.ny * g.nz;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(t % g.nz);
    const long long r = t / g.nz;
    const int sg = (int)(r % nseg), j = (int)(r / nseg);
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
    cls[r * kpad + k] = ok ? (uint8_t)(m + 1) : (uint8_t)0;
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

static size_t lut_bytes(int n_mat) { return (size_t)n_mat * kLutW * sizeof(float); }

hipError_t launch_velocity(const StepArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_velocity, dim3(a.n_tiles), dim3(kSeg, kRows, 1), lut_bytes(a.n_mat), s, a);
  return hipGetLastError();
}

hipError_t launch_stress(const StepArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_stress, dim3(a.n_tiles), dim3(kSeg, kRows, 1), lut_bytes(a.n_mat), s, a);
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

hipError_t launch_classify(const uint8_t *idx, uint8_t *cls, const Grid &g, int nseg, int kpad,
                           const float *lut, hipStream_t s) {
  hipLaunchKernelGGL(k_classify, dim3(4096), dim3(256), 0, s, idx, cls, g, nseg, kpad, lut);
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
                               int blocks, int max_mat, hipStream_t s) {
  const dim3 grid(min(blocks, n_tiles)), block(kSeg, BY, 1);
  hipLaunchKernelGGL(k_velocity_batched<BY>, grid, block, lut_bytes(max_mat), s, desc, tiles,
                     n_tiles, coef, max_steps, n);
  hipLaunchKernelGGL(k_stress_batched<BY>, grid, block, lut_bytes(max_mat), s, desc, tiles,
                     n_tiles, cap, n);
  return hipGetLastError();
}

hipError_t launch_batched_step(int by, const StepArgs *desc, const BatchTile *tiles, int n_tiles,
                               const float2 *coef, const int *cap, int max_steps, int n,
                               int blocks, int max_mat, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  switch (by) {
    case 1: return batched_step<1>(desc, tiles, n_tiles, coef, cap, max_steps, n, blocks, max_mat, s);
    case 2: return batched_step<2>(desc, tiles, n_tiles, coef, cap, max_steps, n, blocks, max_mat, s);
    case 4: return batched_step<4>(desc, tiles, n_tiles, coef, cap, max_steps, n, blocks, max_mat, s);
    case 8: return batched_step<8>(desc, tiles, n_tiles, coef, cap, max_steps, n, blocks, max_mat, s);
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
