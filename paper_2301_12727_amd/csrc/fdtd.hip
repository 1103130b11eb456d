// Viscoelastic FDTD step kernels for gfx950 (BabelBrain Section 2.3, Eq. 1).
//
// One time step is up to five launches over the tiles of a solve (64 x 4 x-y
// columns marching over up to 8 planes of z), split once per solve into
// acoustic tiles (every row segment a single lossless fluid throughout the
// stencil's reach), deep tiles (acoustic, with the fused step's whole reach in
// one fluid) and general tiles:
//   k_velocity_ac, k_velocity : v^{n-1/2} -> v^{n+1/2} (Eq. 1 rows 1-3) and
//                the source force on the v_z faces of plane ks (Section 2.3)
//   k_stress_ac, k_stress     : sigma^n -> sigma^{n+1}, Zener memory
//                variables, peak |p| capture (Eq. 1 rows 4-9, Section 3.2)
//   k_step_deep               : both half-steps of a deep tile in one pass
// All are HBM-bandwidth-bound stencils.  x is the fastest (coalesced) axis
// and each wave owns one 64-cell row segment, so the segment class (acoustic
// or elastic branch) is wave-uniform, and in the fused step and the velocity
// kernels the x neighbours of a whole segment come by lane shifts.  Per block
// the material table (for 16-bit maps, the columns gathered per neighbour) is
// staged in LDS, so the material gathers of a cell are LDS reads rather than
// a second dependent trip to the cache hierarchy, and the class bytes of a
// segment's z column are read four at a time through the scalar cache, one
// group ahead.  Tiles are assigned so that each XCD works on a contiguous
// band of them, keeping the halo rows of neighbouring tiles in one L2.  The
// absorbing layer (CPML) is applied per cell behind a slab test that is
// uniform across most waves.  Batched sweeps run the same tile code from
// per-kind tables that span many solves.
#include "bbfd_dev.h"

namespace bbfd {

// Every floating-point operation of a cell update is spelled out here and in
// the helpers below (fused multiply-adds only where written as fmaf: this
// file is compiled with -ffp-contract=off), and every code path (general
// tiles, acoustic tiles, register windows, batched tiles) goes through the
// same helpers, so a cell's value does not depend on which kernel or tiling
// updated it.

#define C1 (9.0f / 8.0f)
#define C2 (-1.0f / 24.0f)
// 4th-order staggered differences (times dx) from four samples: the forward
// one sits at +1/2 of sample p0, the backward one at p0 from samples stored
// at +1/2.
__device__ __forceinline__ float dfw(float m1, float p0, float p1, float p2) {
  return fmaf(C1, p1 - p0, C2 * (p2 - m1));
}
__device__ __forceinline__ float dbw(float m2, float m1, float p0, float p1) {
  return fmaf(C1, p0 - m1, C2 * (p1 - m2));
}
// Source force on a v_z face: c Re S - s Im S.
__device__ __forceinline__ float src_force(float c, float s, float2 q) {
  return fmaf(c, q.x, -(s * q.y));
}

// Read-only data the kernels index uniformly, read through the scalar cache.
typedef __attribute__((address_space(4))) const uint32_t ScalarU32;
typedef __attribute__((address_space(4))) const int ScalarI32;

// Copy of a uniformly indexed read-only object, dword by dword through the
// scalar cache.
template <class T>
__device__ __forceinline__ T scalar_copy(const T *p) {
  static_assert(sizeof(T) % 4 == 0, "dword-sized object");
  T v;
  const ScalarU32 *src = (const ScalarU32 *)p;
  uint32_t *dst = reinterpret_cast<uint32_t *>(&v);
#pragma unroll
  for (int w = 0; w < (int)(sizeof(T) / 4); ++w) dst[w] = src[w];
  return v;
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
// Copies n floats into LDS (whole block; caller syncs).
__device__ __forceinline__ void stage_floats(float *dst, const float *src, int n) {
  const int nt = blockDim.x * blockDim.y, t0 = threadIdx.y * blockDim.x + threadIdx.x;
  for (int t = t0; t < n; t += nt) dst[t] = src[t];
}

// Wave-uniform class reader of one segment's z column: bytes are fetched as
// 32-bit words through the scalar cache, the next word one group early.
struct ClassColumn {
  const ScalarU32 *w;
  uint32_t cur, nxt;
  __device__ __forceinline__ ClassColumn(const StepArgs &A, int j, int seg, int k0,
                                         const uint8_t *bytes = nullptr) {
    w = (const ScalarU32 *)((bytes ? bytes : A.cls) + ((long long)j * A.nseg + seg) * A.kpad);
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

// Element access by 32-bit byte offset from a uniform base: the loads and
// stores take the scalar-base + 32-bit vector-offset addressing form, so each
// neighbour costs one 32-bit register (x and, for pitches up to 1023 floats, y
// neighbours fold into the instruction's immediate offset).  Stencil values,
// which neighbouring cells of the same and nearby tiles read again, are
// ordinary loads; values a cell reads once (its own state, layer memories,
// peak) and all stores carry the non-temporal hint, so the streams that are
// touched once do not push the stencil data out of the caches (measured:
// +11 % on the whole step).
__device__ __forceinline__ float ldb(const float *base, uint32_t off) {
  return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(base) + off);
}
__device__ __forceinline__ float ldb_once(const float *base, uint32_t off) {
  return __builtin_nontemporal_load(
      reinterpret_cast<const float *>(reinterpret_cast<const char *>(base) + off));
}
__device__ __forceinline__ void stb(float *base, uint32_t off, float v) {
  __builtin_nontemporal_store(v, reinterpret_cast<float *>(reinterpret_cast<char *>(base) + off));
}
__device__ __forceinline__ float cpml_b(float *psi, uint32_t off, float q, float b, float a, float d) {
  q = fmaf(b, q, a * d);
  stb(psi, off, q);
  return d + q;
}

// Every cell update below first issues all of its loads (stencil values, own
// state, layer memories, material indices) and only then computes and
// stores, so a wave has one round trip to memory per cell instead of a chain
// of load-wait-store steps.  Addresses are 32-bit byte offsets from uniform
// bases (see ldb).

#define DPB(a, o, s4) dfw(ldb(a, (o) - (s4)), ldb(a, o), ldb(a, (o) + (s4)), ldb(a, (o) + 2 * (s4)))
#define DMB(a, o, s4) dbw(ldb(a, (o) - 2 * (s4)), ldb(a, (o) - (s4)), ldb(a, o), ldb(a, (o) + (s4)))
// The same with the centre value c = a at o already in a register.
#define DPBC(a, o, s4, c) dfw(ldb(a, (o) - (s4)), c, ldb(a, (o) + (s4)), ldb(a, (o) + 2 * (s4)))
#define DMBC(a, o, s4, c) dbw(ldb(a, (o) - 2 * (s4)), ldb(a, (o) - (s4)), c, ldb(a, (o) + (s4)))

// x stencils without x-shifted loads.  In a wave whose 64 lanes are one whole
// row segment inside the grid, the x neighbours of a cell are the
// neighbouring lanes' values: whole-wave lane shifts (DPP wave_shr:1 /
// wave_shl:1) move them, and only the two lanes at the segment's ends take a
// cell of the neighbouring segment, a wave-uniform value read once per row
// through the scalar cache.  The values and the arithmetic are those of the
// loads they replace, so results are identical bit for bit.
typedef __attribute__((address_space(4))) const float ScalarF32;
// A float at a wave-uniform byte offset, through the scalar cache.
__device__ __forceinline__ float ld_uniform(const float *base, uint32_t off) {
  return *(const ScalarF32 *)(reinterpret_cast<const char *>(base) + off);
}
// Lane l receives lane l - 1's v (lane_up) or lane l + 1's (lane_down); the
// lane with no such neighbour (0, resp. 63) receives edge.  Every lane of the
// wave must be active.
__device__ __forceinline__ float lane_up(float v, float edge) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                               __builtin_bit_cast(int, v), 0x138,
                                                               0xf, 0xf, false));
}
__device__ __forceinline__ float lane_down(float v, float edge) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                               __builtin_bit_cast(int, v), 0x130,
                                                               0xf, 0xf, false));
}
// Byte offset of the row's first cell (lane 0's o; wave-uniform).
__device__ __forceinline__ uint32_t row_start(uint32_t o) {
  return __builtin_amdgcn_readfirstlane(o - 4u * threadIdx.x);
}
// DPB / DMB along x of field a, centre value c, row start ro.
__device__ __forceinline__ float dpb_x(const float *a, uint32_t ro, float c) {
  const float p1 = lane_down(c, ld_uniform(a, ro + 4 * kSeg));
  return dfw(lane_up(c, ld_uniform(a, ro - 4)), c, p1,
             lane_down(p1, ld_uniform(a, ro + 4 * kSeg + 4)));
}
__device__ __forceinline__ float dmb_x(const float *a, uint32_t ro, float c) {
  const float m1 = lane_up(c, ld_uniform(a, ro - 4));
  return dbw(lane_up(m1, ld_uniform(a, ro - 8)), m1, c, lane_down(c, ld_uniform(a, ro + 4 * kSeg)));
}

// Material index of the cell at element offset off of the padded index map
// (uint8 entries, or uint16 for 12-bit CT maps).
template <typename IdxT>
__device__ __forceinline__ int ldi(const uint8_t *idx, uint32_t off) {
  return reinterpret_cast<const IdxT *>(idx)[off];
}

// Velocity update (Eq. 1 rows 1-3) of one tile: x segment bx (one cell per
// lane), row j (wave-uniform), planes [k0, k1); lut is the LDS copy of the
// material table.  On plane ks the v_z faces also receive the source force
// (src_c Re S - src_s Im S, scaled by the face buoyancy): a normal-traction
// jump of 2 S across z = (ks + 1/2) dx.
// XD: the wave's row segment lies wholly inside the grid (x stencils by lane
// shifts).
// lut: for 8-bit maps the material table (rows of kLutW); for 16-bit maps
// the buoyancy column (one float per material), both in LDS.
template <typename IdxT = uint8_t, bool XD = false>
__device__ __forceinline__ void velocity_tile(const StepArgs &A, const float *lut, int bx, int j,
                                              int k0, int k1, float src_c, float src_s) {
  constexpr int RS = sizeof(IdxT) == 1 ? kLutW : 1;  // floats from one material's kRhoS to the next
  const float *rho = sizeof(IdxT) == 1 ? lut + kRhoS : lut;
  const Grid &g = A.g;
  const int i = bx * kSeg + threadIdx.x;
  if (i >= g.nx || j >= g.ny) return;
  const uint32_t P = (uint32_t)g.pitch, PL = (uint32_t)g.plane, P4 = 4 * P, PL4 = 4 * PL;
  const float *sxx = A.f[SXX], *syy = A.f[SYY], *szz = A.f[SZZ];
  const float *sxy = A.f[SXY], *sxz = A.f[SXZ], *syz = A.f[SYZ];
  const float *vx = A.f[VX], *vy = A.f[VY], *vz = A.f[VZ];
  float *vxw = A.fo[VX], *vyw = A.fo[VY], *vzw = A.fo[VZ];
  const uint8_t *idx = A.idx;
  const uint32_t so = (uint32_t)(j * g.nx + i) * 8u;
  const bool px = in_layer(i, g.nx, g.L), py = in_layer(j, g.ny, g.L);
  const float4 tx = px ? A.pml.x[i] : make_float4(1.f, 0.f, 1.f, 0.f);
  const float4 ty = py ? A.pml.y[j] : make_float4(1.f, 0.f, 1.f, 0.f);
  ClassColumn col(A, j, bx, k0);
  uint32_t c = (uint32_t)g.off(i, j, k0);
  for (int k = k0; k < k1; ++k, c += PL) {
    const uint32_t o = 4 * c;
    const uint32_t ro = XD ? row_start(o) : 0u;
    const bool pz = in_layer(k, g.nz, g.L);
    const bool on_src = k == g.ks;
    const int cl = col.at(k, k0);
    const float4 tz = pz ? A.pml.z[k] : make_float4(1.f, 0.f, 1.f, 0.f);
    float2 sq = make_float2(0.f, 0.f);
    if (on_src) sq = *reinterpret_cast<const float2 *>(reinterpret_cast<const char *>(A.src) + so);
    if (cl) {
      // acoustic path: the three normal stresses are equal and the shear
      // stresses vanish throughout the stencil's reach
      const float s0 = ldb(sxx, o);
      float d1 = XD ? dpb_x(sxx, ro, s0) : DPBC(sxx, o, 4, s0);
      float e2 = DPBC(sxx, o, P4, s0), f3 = DPBC(sxx, o, PL4, s0);
      const float vxo = ldb_once(vx, o), vyo = ldb_once(vy, o), vzo = ldb_once(vz, o);
      const float q0 = px ? ldb_once(A.psi[0], o) : 0.f;
      const float q4 = py ? ldb_once(A.psi[4], o) : 0.f;
      const float q8 = pz ? ldb_once(A.psi[8], o) : 0.f;
      const float b = 1.f / rho[(cl - 1) * RS];
      if (px) d1 = cpml_b(A.psi[0], o, q0, tx.z, tx.w, d1);
      if (py) e2 = cpml_b(A.psi[4], o, q4, ty.z, ty.w, e2);
      if (pz) f3 = cpml_b(A.psi[8], o, q8, tz.z, tz.w, f3);
      stb(vxw, o, fmaf(b, d1, vxo));
      stb(vyw, o, fmaf(b, e2, vyo));
      if (on_src) f3 += src_force(src_c, src_s, sq);
      stb(vzw, o, fmaf(b, f3, vzo));
      continue;
    }
    const int m0 = ldi<IdxT>(idx, c), mx = ldi<IdxT>(idx, c + 1), my = ldi<IdxT>(idx, c + P),
              mz = ldi<IdxT>(idx, c + PL);
    const float cxx = ldb(sxx, o), cxy = ldb(sxy, o), cxz = ldb(sxz, o);
    float d1 = XD ? dpb_x(sxx, ro, cxx) : DPBC(sxx, o, 4, cxx);
    float d2 = DMBC(sxy, o, P4, cxy), d3 = DMBC(sxz, o, PL4, cxz);
    float e1 = XD ? dmb_x(sxy, ro, cxy) : DMBC(sxy, o, 4, cxy);
    float e2 = DPB(syy, o, P4), e3 = DMB(syz, o, PL4);
    float f1 = XD ? dmb_x(sxz, ro, cxz) : DMBC(sxz, o, 4, cxz);
    float f2 = DMB(syz, o, P4), f3 = DPB(szz, o, PL4);
    const float vxo = ldb_once(vx, o), vyo = ldb_once(vy, o), vzo = ldb_once(vz, o);
    float q0 = 0.f, q1 = 0.f, q2 = 0.f, q3 = 0.f, q4 = 0.f, q5 = 0.f, q6 = 0.f, q7 = 0.f, q8 = 0.f;
    if (px) { q0 = ldb_once(A.psi[0], o); q3 = ldb_once(A.psi[3], o); q6 = ldb_once(A.psi[6], o); }
    if (py) { q1 = ldb_once(A.psi[1], o); q4 = ldb_once(A.psi[4], o); q7 = ldb_once(A.psi[7], o); }
    if (pz) { q2 = ldb_once(A.psi[2], o); q5 = ldb_once(A.psi[5], o); q8 = ldb_once(A.psi[8], o); }
    const float r0 = rho[m0 * RS];
    const float bx = 2.f / (r0 + rho[mx * RS]);
    const float by = 2.f / (r0 + rho[my * RS]);
    const float bz = 2.f / (r0 + rho[mz * RS]);
    if (px) {
      d1 = cpml_b(A.psi[0], o, q0, tx.z, tx.w, d1);
      e1 = cpml_b(A.psi[3], o, q3, tx.x, tx.y, e1);
      f1 = cpml_b(A.psi[6], o, q6, tx.x, tx.y, f1);
    }
    if (py) {
      d2 = cpml_b(A.psi[1], o, q1, ty.x, ty.y, d2);
      e2 = cpml_b(A.psi[4], o, q4, ty.z, ty.w, e2);
      f2 = cpml_b(A.psi[7], o, q7, ty.x, ty.y, f2);
    }
    if (pz) {
      d3 = cpml_b(A.psi[2], o, q2, tz.x, tz.y, d3);
      e3 = cpml_b(A.psi[5], o, q5, tz.x, tz.y, e3);
      f3 = cpml_b(A.psi[8], o, q8, tz.z, tz.w, f3);
    }
    stb(vxw, o, fmaf(bx, d1 + d2 + d3, vxo));
    stb(vyw, o, fmaf(by, e1 + e2 + e3, vyo));
    float fz = f1 + f2 + f3;
    if (on_src) fz += src_force(src_c, src_s, sq);  // traction source on the v_z faces of plane ks
    stb(vzw, o, fmaf(bz, fz, vzo));
  }
}

// Zener update of one stress component: memory variable relaxes by
// Crank-Nicolson toward -target, stress takes the elastic increment plus the
// mean of the old and new memory value (all pre-scaled by dt).
__device__ __forceinline__ float zener(float &s, float &r, float elastic, float target, float ra,
                                       float rb) {
  const float rn = fmaf(ra, r, -(rb * target));
  s += elastic + 0.5f * (r + rn);
  r = rn;
  return s;
}

// Edge inputs {1/mu, tau_S} of material m: from the table's rows (es =
// kLutW / 2 float2 per material, starting at kInvMu) or from a column (es = 1).
__device__ __forceinline__ float2 edge_in(const float2 *edge, int es, int m) {
  return edge[m * es];
}

// Shear component on an edge shared by cells with edge inputs a, b, c, d
// ({1/mu, tau_S} each): harmonic-mean modulus, arithmetic-mean tau_S.
__device__ __forceinline__ void edge(float &s, float &r, float e, float2 a, float2 b, float2 c,
                                     float2 d, float ra, float rb) {
  const float mue = 4.f / (a.x + b.x + c.x + d.x);
  const float te = 0.25f * (a.y + b.y + c.y + d.y);
  zener(s, r, (mue * (1.f + te)) * e, (mue * te) * e, ra, rb);
}


// Stress + memory update (Eq. 1 rows 4-9) and peak capture of one tile;
// capture is this step's flag.  lut: the material table's rows (in LDS for
// 8-bit maps); edge_col: for 16-bit maps, the edge-input column in LDS.
template <typename IdxT = uint8_t>
__device__ __forceinline__ void stress_tile(const StepArgs &A, const float *lut, int bx, int j,
                                            int k0, int k1, int capture,
                                            const float2 *edge_col = nullptr) {
  constexpr int ES = sizeof(IdxT) == 1 ? kLutW / 2 : 1;
  const float2 *edge_tab =
      sizeof(IdxT) == 1 ? reinterpret_cast<const float2 *>(lut + kInvMu) : edge_col;
  const Grid &g = A.g;
  const int i = bx * kSeg + threadIdx.x;
  if (i >= g.nx || j >= g.ny) return;
  const uint32_t P = (uint32_t)g.pitch, PL = (uint32_t)g.plane, P4 = 4 * P, PL4 = 4 * PL;
  const uint32_t QL4 = (uint32_t)(g.ny * g.nx) * 4u;
  const float *vx = A.f[VX], *vy = A.f[VY], *vz = A.f[VZ];
  const float *sxxp = A.f[SXX], *syyp = A.f[SYY], *szzp = A.f[SZZ];
  float *sxxw = A.fo[SXX], *syyw = A.fo[SYY], *szzw = A.fo[SZZ];
  float *sxyp = A.f[SXY], *sxzp = A.f[SXZ], *syzp = A.f[SYZ];
  float *rxxp = A.f[RXX], *ryyp = A.f[RYY], *rzzp = A.f[RZZ];
  float *rxyp = A.f[RXY], *rxzp = A.f[RXZ], *ryzp = A.f[RYZ];
  const uint8_t *idx = A.idx;
  const float ra = A.relax_a, rb = A.relax_b;
  const bool px = in_layer(i, g.nx, g.L), py = in_layer(j, g.ny, g.L);
  const float4 tx = px ? A.pml.x[i] : make_float4(1.f, 0.f, 1.f, 0.f);
  const float4 ty = py ? A.pml.y[j] : make_float4(1.f, 0.f, 1.f, 0.f);
  ClassColumn col(A, j, bx, k0);
  uint32_t c = (uint32_t)g.off(i, j, k0);
  uint32_t qo = ((uint32_t)k0 * (uint32_t)(g.ny * g.nx) + (uint32_t)(j * g.nx + i)) * 4u;
  // z windows of this column, one new plane loaded per step in z: v_z at
  // planes k-2..k+1 (z0..z3), v_x and v_y at k-1..k+2 (x0..x3, y0..y3).  The
  // velocities are not written by this kernel, so the window stays valid.
  float z0, z1, z2, z3, x0, x1, x2, x3, y0, y1, y2, y3, zn = 0.f, xn = 0.f, yn = 0.f;
  {
    const uint32_t o = 4 * c;
    z0 = ldb(vz, o - 2 * PL4); z1 = ldb(vz, o - PL4); z2 = ldb(vz, o); z3 = ldb(vz, o + PL4);
    x0 = ldb(vx, o - PL4); x1 = ldb(vx, o); x2 = ldb(vx, o + PL4); x3 = ldb(vx, o + 2 * PL4);
    y0 = ldb(vy, o - PL4); y1 = ldb(vy, o); y2 = ldb(vy, o + PL4); y3 = ldb(vy, o + 2 * PL4);
  }
  for (int k = k0; k < k1; ++k, c += PL, qo += QL4) {
    const uint32_t o = 4 * c;
    if (k != k0) {
      z0 = z1; z1 = z2; z2 = z3; z3 = zn;
      x0 = x1; x1 = x2; x2 = x3; x3 = xn;
      y0 = y1; y1 = y2; y2 = y3; y3 = yn;
    }
    if (k + 1 < k1) {  // the next plane's new window entries
      zn = ldb(vz, o + 2 * PL4);
      xn = ldb(vx, o + 3 * PL4);
      yn = ldb(vy, o + 3 * PL4);
    }
    const bool pz = in_layer(k, g.nz, g.L);
    const int cl = col.at(k, k0);
    const float4 tz = pz ? A.pml.z[k] : make_float4(1.f, 0.f, 1.f, 0.f);
    const float pk = capture ? ldb_once(A.peak, qo) : 0.f;
    if (cl) {
      // acoustic path: only the (equal) normal stresses change
      float exx = DMB(vx, o, 4), eyy = DMB(vy, o, P4), ezz = dbw(z0, z1, z2, z3);
      const float so = ldb_once(sxxp, o);
      const float q9 = px ? ldb_once(A.psi[9], o) : 0.f;
      const float q10 = py ? ldb_once(A.psi[10], o) : 0.f;
      const float q11 = pz ? ldb_once(A.psi[11], o) : 0.f;
      if (px) exx = cpml_b(A.psi[9], o, q9, tx.x, tx.y, exx);
      if (py) eyy = cpml_b(A.psi[10], o, q10, ty.x, ty.y, eyy);
      if (pz) ezz = cpml_b(A.psi[11], o, q11, tz.x, tz.y, ezz);
      const float sn = fmaf(lut[(cl - 1) * kLutW + kPiU], exx + eyy + ezz, so);
      stb(sxxw, o, sn);
      stb(syyw, o, sn);
      stb(szzw, o, sn);
      if (capture) {
        const float a = fabsf(sn + sn + sn) / 3.f;
        if (a > pk || a != a) stb(A.peak, qo, a);
      }
      continue;
    }
    const int m0 = ldi<IdxT>(idx, c), mx = ldi<IdxT>(idx, c + 1), my = ldi<IdxT>(idx, c + P),
              mz = ldi<IdxT>(idx, c + PL);
    const int mxy = ldi<IdxT>(idx, c + 1 + P), mxz = ldi<IdxT>(idx, c + 1 + PL),
              myz = ldi<IdxT>(idx, c + P + PL);
    float exx = DMB(vx, o, 4), eyy = DMB(vy, o, P4), ezz = dbw(z0, z1, z2, z3);
    float dyvx = DPB(vx, o, P4), dxvy = DPB(vy, o, 4);
    float dzvx = dfw(x0, x1, x2, x3), dxvz = DPB(vz, o, 4);
    float dzvy = dfw(y0, y1, y2, y3), dyvz = DPB(vz, o, P4);
    float sxx = ldb_once(sxxp, o), syy = ldb_once(syyp, o), szz = ldb_once(szzp, o);
    float rxx = ldb_once(rxxp, o), ryy = ldb_once(ryyp, o), rzz = ldb_once(rzzp, o);
    float sxy = ldb_once(sxyp, o), sxz = ldb_once(sxzp, o), syz = ldb_once(syzp, o);
    float rxy = ldb_once(rxyp, o), rxz = ldb_once(rxzp, o), ryz = ldb_once(ryzp, o);
    float q9 = 0.f, q10 = 0.f, q11 = 0.f, q12 = 0.f, q13 = 0.f, q14 = 0.f, q15 = 0.f, q16 = 0.f,
          q17 = 0.f;
    if (px) { q9 = ldb_once(A.psi[9], o); q13 = ldb_once(A.psi[13], o); q15 = ldb_once(A.psi[15], o); }
    if (py) { q10 = ldb_once(A.psi[10], o); q12 = ldb_once(A.psi[12], o); q17 = ldb_once(A.psi[17], o); }
    if (pz) { q11 = ldb_once(A.psi[11], o); q14 = ldb_once(A.psi[14], o); q16 = ldb_once(A.psi[16], o); }
    if (px) {
      exx = cpml_b(A.psi[9], o, q9, tx.x, tx.y, exx);
      dxvy = cpml_b(A.psi[13], o, q13, tx.z, tx.w, dxvy);
      dxvz = cpml_b(A.psi[15], o, q15, tx.z, tx.w, dxvz);
    }
    if (py) {
      eyy = cpml_b(A.psi[10], o, q10, ty.x, ty.y, eyy);
      dyvx = cpml_b(A.psi[12], o, q12, ty.z, ty.w, dyvx);
      dyvz = cpml_b(A.psi[17], o, q17, ty.z, ty.w, dyvz);
    }
    if (pz) {
      ezz = cpml_b(A.psi[11], o, q11, tz.x, tz.y, ezz);
      dzvx = cpml_b(A.psi[14], o, q14, tz.z, tz.w, dzvx);
      dzvy = cpml_b(A.psi[16], o, q16, tz.z, tz.w, dzvy);
    }
    const float4 L0 = *reinterpret_cast<const float4 *>(lut + m0 * kLutW);  // piU muU piTau muTau
    const float th = exx + eyy + ezz;
    {
      const float piu = L0.x, muu2 = 2.f * L0.y;
      const float pit = L0.z, mut2 = 2.f * L0.w;
      float lat = eyy + ezz;
      zener(sxx, rxx, fmaf(piu, th, -(muu2 * lat)), fmaf(pit, th, -(mut2 * lat)), ra, rb);
      lat = exx + ezz;
      zener(syy, ryy, fmaf(piu, th, -(muu2 * lat)), fmaf(pit, th, -(mut2 * lat)), ra, rb);
      lat = exx + eyy;
      zener(szz, rzz, fmaf(piu, th, -(muu2 * lat)), fmaf(pit, th, -(mut2 * lat)), ra, rb);
    }
    const float2 e0 = edge_in(edge_tab, ES, m0), ex = edge_in(edge_tab, ES, mx);
    const float2 ey = edge_in(edge_tab, ES, my), ez = edge_in(edge_tab, ES, mz);
    edge(sxy, rxy, dyvx + dxvy, e0, ex, ey, edge_in(edge_tab, ES, mxy), ra, rb);
    edge(sxz, rxz, dzvx + dxvz, e0, ex, ez, edge_in(edge_tab, ES, mxz), ra, rb);
    edge(syz, ryz, dzvy + dyvz, e0, ey, ez, edge_in(edge_tab, ES, myz), ra, rb);
    stb(sxxw, o, sxx); stb(syyw, o, syy); stb(szzw, o, szz);
    stb(rxxp, o, rxx); stb(ryyp, o, ryy); stb(rzzp, o, rzz);
    stb(sxyp, o, sxy); stb(sxzp, o, sxz); stb(syzp, o, syz);
    stb(rxyp, o, rxy); stb(rxzp, o, rxz); stb(ryzp, o, ryz);
    if (capture) {
      const float a = fabsf(sxx + syy + szz) / 3.f;
      if (a > pk || a != a) stb(A.peak, qo, a);
    }
  }
}

// ------------------------------------------------------------ acoustic tiles
// A tile whose every row segment is of a lossless-fluid class on every plane
// of its chunk runs these leaner kernels: no index map, no shear or memory
// state, and the z-neighbours of the one z-differenced field held in a
// register window (one new plane loaded per step in z), at a fraction of the
// general kernels' registers.  The arithmetic is the acoustic branch of the
// general tile code, operation for operation.

struct AcCtx {
  const StepArgs *A;
  uint32_t P4, PL4;  // row and plane strides in bytes
  bool px, py;
  float4 tx, ty;
};

// One plane of the acoustic velocity update at byte offset o.  z0..z3: sxx at
// planes k-1, k, k+1, k+2 of this column.  XD: the wave's row segment lies
// wholly inside the grid; the x neighbours come by lane shifts from z1 and
// the segment-edge cells xm, xp, xp2 (of lanes 0, 63, 63) from the scalar cache.
template <bool XD>
struct VelAc {
  float xm, xp, xp2, ym, yp, yp2, vx, vy, vz, q0, q4, q8;
  float2 sq;
  float4 tz;
  int cl;
  bool pz, src;
  __device__ __forceinline__ void load(const AcCtx &C, uint32_t o, int k, int cls, uint32_t so) {
    const StepArgs &A = *C.A;
    const float *sxx = A.f[SXX];
    cl = cls;
    pz = in_layer(k, A.g.nz, A.g.L);
    src = k == A.g.ks;
    if (XD) {
      const uint32_t ro = row_start(o);
      xm = ld_uniform(sxx, ro - 4); xp = ld_uniform(sxx, ro + 4 * kSeg);
      xp2 = ld_uniform(sxx, ro + 4 * kSeg + 4);
    } else {
      xm = ldb(sxx, o - 4); xp = ldb(sxx, o + 4); xp2 = ldb(sxx, o + 8);
    }
    ym = ldb(sxx, o - C.P4); yp = ldb(sxx, o + C.P4); yp2 = ldb(sxx, o + 2 * C.P4);
    vx = ldb_once(A.f[VX], o); vy = ldb_once(A.f[VY], o); vz = ldb_once(A.f[VZ], o);
    q0 = C.px ? ldb_once(A.psi[0], o) : 0.f;
    q4 = C.py ? ldb_once(A.psi[4], o) : 0.f;
    q8 = pz ? ldb_once(A.psi[8], o) : 0.f;
    tz = pz ? A.pml.z[k] : make_float4(1.f, 0.f, 1.f, 0.f);
    sq = src ? *reinterpret_cast<const float2 *>(reinterpret_cast<const char *>(A.src) + so)
             : make_float2(0.f, 0.f);
  }
  __device__ __forceinline__ void finish(const AcCtx &C, const float *lut, uint32_t o, float z0,
                                         float z1, float z2, float z3, float src_c, float src_s) {
    const StepArgs &A = *C.A;
    if (XD) {
      const float p1 = lane_down(z1, xp);
      xp2 = lane_down(p1, xp2);
      xm = lane_up(z1, xm);
      xp = p1;
    }
    float d1 = dfw(xm, z1, xp, xp2), e2 = dfw(ym, z1, yp, yp2), f3 = dfw(z0, z1, z2, z3);
    const float b = 1.f / lut[(cl - 1) * kLutW + kRhoS];
    if (C.px) d1 = cpml_b(A.psi[0], o, q0, C.tx.z, C.tx.w, d1);
    if (C.py) e2 = cpml_b(A.psi[4], o, q4, C.ty.z, C.ty.w, e2);
    if (pz) f3 = cpml_b(A.psi[8], o, q8, tz.z, tz.w, f3);
    stb(A.fo[VX], o, fmaf(b, d1, vx));
    stb(A.fo[VY], o, fmaf(b, e2, vy));
    if (src) f3 += src_force(src_c, src_s, sq);
    stb(A.fo[VZ], o, fmaf(b, f3, vz));
  }
};

__device__ __forceinline__ bool ac_setup(AcCtx &C, const StepArgs &A, int i, int j) {
  const Grid &g = A.g;
  if (i >= g.nx || j >= g.ny) return false;
  C.A = &A;
  C.P4 = (uint32_t)g.pitch * 4u;
  C.PL4 = (uint32_t)g.plane * 4u;
  C.px = in_layer(i, g.nx, g.L);
  C.py = in_layer(j, g.ny, g.L);
  C.tx = C.px ? A.pml.x[i] : make_float4(1.f, 0.f, 1.f, 0.f);
  C.ty = C.py ? A.pml.y[j] : make_float4(1.f, 0.f, 1.f, 0.f);
  return true;
}

// The loads of plane k + 1 are issued before the stores of plane k: the wait
// for them then does not include the completion of those stores (vector
// memory operations retire in issue order), so each plane costs about one
// memory latency instead of a load latency plus a store latency.
template <bool XD = false>
__device__ __forceinline__ void velocity_ac_tile(const StepArgs &A, const float *lut, int bx, int j,
                                                 int k0, int k1, float src_c, float src_s) {
  const int i = bx * kSeg + threadIdx.x;
  AcCtx C;
  if (!ac_setup(C, A, i, j)) return;
  const float *sxx = A.f[SXX];
  const uint32_t so = (uint32_t)(j * A.g.nx + i) * 8u;
  ClassColumn col(A, j, bx, k0);
  uint32_t o = (uint32_t)A.g.off(i, j, k0) * 4u;
  float z0 = ldb(sxx, o - C.PL4), z1 = ldb(sxx, o), z2 = ldb(sxx, o + C.PL4),
        z3 = ldb(sxx, o + 2 * C.PL4);
  VelAc<XD> cur;
  cur.load(C, o, k0, col.at(k0, k0), so);
  float h = (k0 + 1 < k1) ? ldb(sxx, o + 3 * C.PL4) : 0.f;  // plane k0 + 3, if used
  for (int k = k0; k < k1; ++k, o += C.PL4) {
    VelAc<XD> nxt;
    float hn = 0.f;
    if (k + 1 < k1) {
      nxt.load(C, o + C.PL4, k + 1, col.at(k + 1, k0), so);
      if (k + 2 < k1) hn = ldb(sxx, o + 4 * C.PL4);          // plane k + 4
    }
    cur.finish(C, lut, o, z0, z1, z2, z3, src_c, src_s);
    z0 = z1; z1 = z2; z2 = z3; z3 = h;
    h = hn;
    cur = nxt;
  }
}

// One plane of the acoustic stress update.  w0..w3: vz at planes k-2, k-1,
// k, k+1 of this column.
struct StrAc {
  float xm2, xm1, x0, xp1, ym2, ym1, y0, yp1, s, q9, q10, q11, pk;
  float4 tz;
  int cl, keep;
  bool pz;
  __device__ __forceinline__ void load(const AcCtx &C, uint32_t o, uint32_t qo, int k, int cls,
                                       int kp, int capture) {
    const StepArgs &A = *C.A;
    const float *vx = A.f[VX], *vy = A.f[VY];
    cl = cls;
    keep = kp;
    pz = in_layer(k, A.g.nz, A.g.L);
    xm2 = ldb(vx, o - 8); xm1 = ldb(vx, o - 4); x0 = ldb(vx, o); xp1 = ldb(vx, o + 4);
    ym2 = ldb(vy, o - 2 * C.P4); ym1 = ldb(vy, o - C.P4); y0 = ldb(vy, o); yp1 = ldb(vy, o + C.P4);
    s = ldb_once(A.f[SXX], o);
    q9 = C.px ? ldb_once(A.psi[9], o) : 0.f;
    q10 = C.py ? ldb_once(A.psi[10], o) : 0.f;
    q11 = pz ? ldb_once(A.psi[11], o) : 0.f;
    tz = pz ? A.pml.z[k] : make_float4(1.f, 0.f, 1.f, 0.f);
    pk = capture ? ldb_once(A.peak, qo) : 0.f;
  }
  __device__ __forceinline__ void finish(const AcCtx &C, const float *lut, uint32_t o, uint32_t qo,
                                         float w0, float w1, float w2, float w3, int capture) {
    const StepArgs &A = *C.A;
    float exx = dbw(xm2, xm1, x0, xp1), eyy = dbw(ym2, ym1, y0, yp1), ezz = dbw(w0, w1, w2, w3);
    if (C.px) exx = cpml_b(A.psi[9], o, q9, C.tx.x, C.tx.y, exx);
    if (C.py) eyy = cpml_b(A.psi[10], o, q10, C.ty.x, C.ty.y, eyy);
    if (pz) ezz = cpml_b(A.psi[11], o, q11, tz.x, tz.y, ezz);
    const float sn = fmaf(lut[(cl - 1) * kLutW + kPiU], exx + eyy + ezz, s);
    stb(A.fo[SXX], o, sn);
    if (keep) {  // read by an elastic neighbour: keep the three normal stresses equal
      stb(A.fo[SYY], o, sn);
      stb(A.fo[SZZ], o, sn);
    }
    if (capture) {
      const float a = fabsf(sn + sn + sn) / 3.f;
      if (a > pk || a != a) stb(A.peak, qo, a);
    }
  }
};

__device__ __forceinline__ void stress_ac_tile(const StepArgs &A, const float *lut, int bx, int j,
                                               int k0, int k1, int capture) {
  const int i = bx * kSeg + threadIdx.x;
  AcCtx C;
  if (!ac_setup(C, A, i, j)) return;
  const float *vz = A.f[VZ];
  const uint32_t QL4 = (uint32_t)(A.g.ny * A.g.nx) * 4u;
  ClassColumn col(A, j, bx, k0);
  uint32_t o = (uint32_t)A.g.off(i, j, k0) * 4u;
  uint32_t qo = ((uint32_t)k0 * (uint32_t)(A.g.ny * A.g.nx) + (uint32_t)(j * A.g.nx + i)) * 4u;
  float w0 = ldb(vz, o - 2 * C.PL4), w1 = ldb(vz, o - C.PL4), w2 = ldb(vz, o), w3 = ldb(vz, o + C.PL4);
  StrAc cur;
  ClassColumn kcol(A, j, bx, k0, A.keep);
  cur.load(C, o, qo, k0, col.at(k0, k0), kcol.at(k0, k0), capture);
  float h = ldb(vz, o + 2 * C.PL4);  // plane k0 + 2 <= nz + 1
  for (int k = k0; k < k1; ++k, o += C.PL4, qo += QL4) {
    StrAc nxt;
    float hn = 0.f;
    if (k + 1 < k1) {
      nxt.load(C, o + C.PL4, qo + QL4, k + 1, col.at(k + 1, k0), kcol.at(k + 1, k0), capture);
      hn = ldb(vz, o + 3 * C.PL4);  // plane k + 3 <= nz + 1
    }
    cur.finish(C, lut, o, qo, w0, w1, w2, w3, capture);
    w0 = w1; w1 = w2; w2 = w3; w3 = h;
    h = hn;
    cur = nxt;
  }
}

// ------------------------------------------------------------- deep tiles
// A deep tile (see k_tile_kinds) takes a whole time step in one pass: each
// cell recomputes the new velocities its stress update needs (v_x at x-2..x+1,
// v_y at y-2..y+1, v_z at z-2..z+1, the last in a register window along the
// march) from the current normal stress and velocities, stores its own new
// velocity and stress, and never waits for another tile.  Inputs come from the
// current buffers and outputs go to the other ones, so neighbouring tiles may
// run in any order.  Every recomputed value is the acoustic velocity update
// of the velocity kernels, operation for operation (with the CPML memory term
// for faces in the x layer, see XFace), so the results equal the two-pass step
// bit for bit.  It moves 32 bytes per cell update (sigma_xx and v read,
// written) instead of 48.  Away from the x layer the x stencils of sigma_xx
// and v_x come by lane shifts (9 of the 22 loads of a plane), which the
// memory pipeline, the kernel's first limit, no longer has to serve.
__device__ __forceinline__ float vnew(float vold, float b, float m1, float p0, float p1, float p2) {
  return fmaf(b, dfw(m1, p0, p1, p2), vold);
}

// XL: some face v_x(p), p = i-2 .. i+1, of the wave's recomputed velocities
// lies in the x absorbing layer or outside the grid.  Inside the layer the
// recomputation and the own cell's updates add the CPML memory terms exactly
// as the velocity and stress kernels do (the memories of the faces the wave
// recomputes but does not own are read only; the tile test keeps them inside
// the wave's own segment); outside the grid v_x is the zero ghost face, which
// no kernel updates.
struct XFace {
  bool in, ly;   // inside the grid; inside the x layer
  float tb, ta;  // CPML b and a at the half position p + 1/2
  __device__ __forceinline__ void set(const StepArgs &A, int p) {
    const Grid &g = A.g;
    in = p >= 0 && p < g.nx;
    ly = in && in_layer(p, g.nx, g.L);
    const float4 t = ly ? A.pml.x[p] : make_float4(1.f, 0.f, 1.f, 0.f);
    tb = t.z;
    ta = t.w;
  }
  // new v_x of this face from its x derivative d, memory q and old value
  __device__ __forceinline__ float vnew(float d, float q, float bu, float vold) const {
    if (!in) return 0.f;
    if (ly) d = d + fmaf(tb, q, ta * d);
    return fmaf(bu, d, vold);
  }
};

template <bool XL>
__device__ __forceinline__ void deep_tile(const StepArgs &A, const float *lut, int bx, int j, int k0,
                                          int k1, float src_c, float src_s, int capture) {
  const Grid &g = A.g;
  const int i = bx * kSeg + threadIdx.x;  // deep tiles are whole row blocks
  if (i >= g.nx) return;                   // the grid's last x segment may be partial
  const uint32_t P4 = 4u * (uint32_t)g.pitch, PL4 = 4u * (uint32_t)g.plane;
  const uint32_t QL4 = (uint32_t)(g.ny * g.nx) * 4u;
  const float *sxx = A.f[SXX], *vx = A.f[VX], *vy = A.f[VY], *vz = A.f[VZ];
  ClassColumn col(A, j, bx, k0);
  const int cl = col.at(k0, k0);  // one fluid class over the tile and its reach
  const float b = 1.f / lut[(cl - 1) * kLutW + kRhoS];
  const float piu = lut[(cl - 1) * kLutW + kPiU];
  const uint32_t so = (uint32_t)(j * g.nx + i) * 8u;
  const float2 sq = (g.ks >= k0 - 2 && g.ks <= k1)
                        ? *reinterpret_cast<const float2 *>(reinterpret_cast<const char *>(A.src) + so)
                        : make_float2(0.f, 0.f);
  uint32_t o = (uint32_t)g.off(i, j, k0) * 4u;
  uint32_t qo = ((uint32_t)k0 * (uint32_t)(g.ny * g.nx) + (uint32_t)(j * g.nx + i)) * 4u;
  // sxx of this column at planes k-3 .. k+3 (s0..s6), new v_z at k-2 .. k+1 (w0..w3)
  float s0 = ldb(sxx, o - 3 * PL4), s1 = ldb(sxx, o - 2 * PL4), s2 = ldb(sxx, o - PL4),
        s3 = ldb(sxx, o), s4 = ldb(sxx, o + PL4), s5 = ldb(sxx, o + 2 * PL4),
        s6 = ldb(sxx, o + 3 * PL4);
  auto vz_face = [&](int kk, float vold, float m1, float p0, float p1, float p2) {
    float f3 = dfw(m1, p0, p1, p2);
    if (kk == g.ks) f3 += src_force(src_c, src_s, sq);
    return fmaf(b, f3, vold);
  };
  float w0 = vz_face(k0 - 2, ldb(vz, o - 2 * PL4), s0, s1, s2, s3);
  float w1 = vz_face(k0 - 1, ldb(vz, o - PL4), s1, s2, s3, s4);
  float w2 = vz_face(k0, ldb(vz, o), s2, s3, s4, s5);
  float w3 = vz_face(k0 + 1, ldb(vz, o + PL4), s3, s4, s5, s6);
  XFace f2, f1, f0, fp;  // faces i-2, i-1, i, i+1 (XL only)
  bool lc = false;       // this cell inside the x layer (CPML of exx)
  float4 tc = make_float4(1.f, 0.f, 1.f, 0.f);
  if (XL) {
    f2.set(A, i - 2); f1.set(A, i - 1); f0.set(A, i); fp.set(A, i + 1);
    lc = in_layer(i, g.nx, g.L);
    if (lc) tc = A.pml.x[i];
  }
  for (int k = k0; k < k1; ++k, o += PL4, qo += QL4) {
    // x stencil of sxx on this row and plane, y stencil on this column
    float xm3, xm2, xm1, xp1, xp2, xp3, ux2, ux1, ux0, uxp;
    if (!XL) {  // every lane of the wave is inside the grid: lane shifts
      const uint32_t ro = row_start(o);
      xm1 = lane_up(s3, ld_uniform(sxx, ro - 4));
      xm2 = lane_up(xm1, ld_uniform(sxx, ro - 8));
      xm3 = lane_up(xm2, ld_uniform(sxx, ro - 12));
      xp1 = lane_down(s3, ld_uniform(sxx, ro + 4 * kSeg));
      xp2 = lane_down(xp1, ld_uniform(sxx, ro + 4 * kSeg + 4));
      xp3 = lane_down(xp2, ld_uniform(sxx, ro + 4 * kSeg + 8));
      ux0 = ldb(vx, o);
      ux1 = lane_up(ux0, ld_uniform(vx, ro - 4));
      ux2 = lane_up(ux1, ld_uniform(vx, ro - 8));
      uxp = lane_down(ux0, ld_uniform(vx, ro + 4 * kSeg));
    } else {
      xm3 = ldb(sxx, o - 12); xm2 = ldb(sxx, o - 8); xm1 = ldb(sxx, o - 4);
      xp1 = ldb(sxx, o + 4); xp2 = ldb(sxx, o + 8); xp3 = ldb(sxx, o + 12);
      ux2 = ldb(vx, o - 8); ux1 = ldb(vx, o - 4); ux0 = ldb(vx, o); uxp = ldb(vx, o + 4);
    }
    const float ym3 = ldb(sxx, o - 3 * P4), ym2 = ldb(sxx, o - 2 * P4), ym1 = ldb(sxx, o - P4);
    const float yp1 = ldb(sxx, o + P4), yp2 = ldb(sxx, o + 2 * P4), yp3 = ldb(sxx, o + 3 * P4);
    const float uy2 = ldb(vy, o - 2 * P4), uy1 = ldb(vy, o - P4), uy0 = ldb(vy, o),
                uyp = ldb(vy, o + P4);
    const bool more = k + 1 < k1;
    const float s7 = more ? ldb(sxx, o + 4 * PL4) : 0.f;    // plane k + 4
    const float vzn = more ? ldb(vz, o + 2 * PL4) : 0.f;    // plane k + 2
    const float pk = capture ? ldb_once(A.peak, qo) : 0.f;
    // new velocities around the cell (the velocity kernels' acoustic update)
    float nx2, nx1, nx0, nxp;
    if (XL) {
      float *psx = A.psi[0];
      const float q2 = f2.ly ? ldb(psx, o - 8) : 0.f, q1 = f1.ly ? ldb(psx, o - 4) : 0.f;
      const float q0 = f0.ly ? ldb_once(psx, o) : 0.f, qp = fp.ly ? ldb(psx, o + 4) : 0.f;
      const float d0 = dfw(xm1, s3, xp1, xp2);
      nx2 = f2.vnew(dfw(xm3, xm2, xm1, s3), q2, b, ux2);
      nx1 = f1.vnew(dfw(xm2, xm1, s3, xp1), q1, b, ux1);
      nx0 = f0.vnew(d0, q0, b, ux0);
      nxp = fp.vnew(dfw(s3, xp1, xp2, xp3), qp, b, uxp);
      if (f0.ly) stb(psx, o, fmaf(f0.tb, q0, f0.ta * d0));  // this face's memory
    } else {
      nx2 = vnew(ux2, b, xm3, xm2, xm1, s3); nx1 = vnew(ux1, b, xm2, xm1, s3, xp1);
      nx0 = vnew(ux0, b, xm1, s3, xp1, xp2); nxp = vnew(uxp, b, s3, xp1, xp2, xp3);
    }
    const float ny2 = vnew(uy2, b, ym3, ym2, ym1, s3), ny1 = vnew(uy1, b, ym2, ym1, s3, yp1);
    const float ny0 = vnew(uy0, b, ym1, s3, yp1, yp2), nyp = vnew(uyp, b, s3, yp1, yp2, yp3);
    // stress update (the acoustic stress kernels' arithmetic)
    float exx = dbw(nx2, nx1, nx0, nxp);
    const float eyy = dbw(ny2, ny1, ny0, nyp), ezz = dbw(w0, w1, w2, w3);
    if (XL && lc) {
      const float q9 = ldb_once(A.psi[9], o);
      exx = cpml_b(A.psi[9], o, q9, tc.x, tc.y, exx);
    }
    const float sn = fmaf(piu, exx + eyy + ezz, s3);
    stb(A.fo[VX], o, nx0);
    stb(A.fo[VY], o, ny0);
    stb(A.fo[VZ], o, w2);
    stb(A.fo[SXX], o, sn);
    if (capture) {
      const float a = fabsf(sn + sn + sn) / 3.f;
      if (a > pk || a != a) stb(A.peak, qo, a);
    }
    if (more) {
      const float w4 = vz_face(k + 2, vzn, s4, s5, s6, s7);
      s0 = s1; s1 = s2; s2 = s3; s3 = s4; s4 = s5; s5 = s6; s6 = s7;
      w0 = w1; w1 = w2; w2 = w3; w3 = w4;
    }
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

// Single-solve step kernels.  The tiles of a solve are split once per solve
// into three lists (acoustic / general / deep, each in tile order); block b
// of a launch takes list entry xcd_band(b, count) and blocks beyond the
// list's length exit at once.
// General kernels: the material table of an 8-bit map is staged in LDS.  Of
// the up to 4096 rows of a 16-bit map's table, the columns gathered for the
// neighbours of a cell (buoyancy for the velocity update, edge inputs for the
// shear update) are staged in LDS; the moduli, one float4 per cell, and the
// fluid rows of the acoustic branches are read through the caches.
template <typename IdxT>
__global__ void __launch_bounds__(kSeg * kRows)
    k_velocity(StepArgs A, const int *__restrict__ list, const int *__restrict__ count) {
  const int n = *count;
  if ((int)blockIdx.x >= n) return;
  if (sizeof(IdxT) == 1)
    stage_lut(s_lut, A.lut, A.n_mat);  // the whole table
  else
    stage_floats(s_lut, rho_column(A.lut), A.n_mat);  // its buoyancy column
  __syncthreads();
  int bx, by, k0, k1;
  tile_coords(A, list[xcd_band(blockIdx.x, n)], bx, by, k0, k1);
  const float *lut = s_lut;
  if ((bx + 1) * kSeg <= A.g.nx)  // whole segment inside the grid: lane shifts
    velocity_tile<IdxT, true>(A, lut, bx, by * kRows + wave_row(), k0, k1, A.src_c, A.src_s);
  else
    velocity_tile<IdxT, false>(A, lut, bx, by * kRows + wave_row(), k0, k1, A.src_c, A.src_s);
}

template <typename IdxT>
__global__ void __launch_bounds__(kSeg * kRows)
    k_stress(StepArgs A, const int *__restrict__ list, const int *__restrict__ count) {
  const int n = *count;
  if ((int)blockIdx.x >= n) return;
  const bool lds = sizeof(IdxT) == 1;
  if (lds)
    stage_lut(s_lut, A.lut, A.n_mat);  // the whole table
  else  // its edge-input column (the moduli rows are read through the caches)
    stage_floats(s_lut, reinterpret_cast<const float *>(edge_column(A.lut)), 2 * A.n_mat);
  __syncthreads();
  int bx, by, k0, k1;
  tile_coords(A, list[xcd_band(blockIdx.x, n)], bx, by, k0, k1);
  stress_tile<IdxT>(A, lds ? s_lut : A.lut, bx, by * kRows + wave_row(), k0, k1, A.capture,
                    reinterpret_cast<const float2 *>(s_lut));
}

// Rows the fluid-only kernels read: those of the lossless fluids that have a
// segment class (class m + 1 fits a byte, so m < 255), up to the last one.
__device__ __forceinline__ int fluid_rows(const StepArgs &A) { return A.n_fluid; }

__global__ void __launch_bounds__(kSeg * kRows)
    k_velocity_ac(StepArgs A, const int *__restrict__ list, const int *__restrict__ count) {
  const int n = *count;
  if ((int)blockIdx.x >= n) return;
  stage_lut(s_lut, A.lut, fluid_rows(A));
  __syncthreads();
  int bx, by, k0, k1;
  tile_coords(A, list[xcd_band(blockIdx.x, n)], bx, by, k0, k1);
  if ((bx + 1) * kSeg <= A.g.nx)
    velocity_ac_tile<true>(A, s_lut, bx, by * kRows + wave_row(), k0, k1, A.src_c, A.src_s);
  else
    velocity_ac_tile<false>(A, s_lut, bx, by * kRows + wave_row(), k0, k1, A.src_c, A.src_s);
}

__global__ void __launch_bounds__(kSeg * kRows)
    k_stress_ac(StepArgs A, const int *__restrict__ list, const int *__restrict__ count) {
  const int n = *count;
  if ((int)blockIdx.x >= n) return;
  stage_lut(s_lut, A.lut, fluid_rows(A));
  __syncthreads();
  int bx, by, k0, k1;
  tile_coords(A, list[xcd_band(blockIdx.x, n)], bx, by, k0, k1);
  stress_ac_tile(A, s_lut, bx, by * kRows + wave_row(), k0, k1, A.capture);
}

__global__ void __launch_bounds__(kSeg * kRows)
    k_step_deep(StepArgs A, const int *__restrict__ list, const int *__restrict__ count) {
  const int n = *count;
  if ((int)blockIdx.x >= n) return;
  stage_lut(s_lut, A.lut, fluid_rows(A));
  __syncthreads();
  int bx, by, k0, k1;
  tile_coords(A, list[xcd_band(blockIdx.x, n)], bx, by, k0, k1);
  const int i0 = bx * kSeg;
  if (i0 - 2 < A.g.L || i0 + kSeg >= A.g.nx - A.g.L)  // faces i0-2 .. i0+64 touch the x layer
    deep_tile<true>(A, s_lut, bx, by * kRows + wave_row(), k0, k1, A.src_c, A.src_s, A.capture);
  else
    deep_tile<false>(A, s_lut, bx, by * kRows + wave_row(), k0, k1, A.src_c, A.src_s, A.capture);
}

// Tile kinds of a single solve: 1 when every row segment of the tile has a
// fluid class on every plane of its chunk (acoustic tile), 2 (deep tile) when
// moreover
//  * the tile's rows and planes and 3 around them lie inside the grid and
//    outside the absorbing layer; in x the tile may reach into the x layer or
//    past the grid's edge, as long as every layer face it recomputes is one
//    of its own (deep_x_ok),
//  * every cell of that reach inside the grid holds the tile's fluid: the
//    classes of the segments one row and one plane around the tile cover it up
//    to two cells beyond their segment in x, and the index map is read for the
//    third, and
//  * no elastic segment reads sigma_yy or sigma_zz of the tile (keep flags 0:
//    the fused step stores sigma_xx alone),
// else 0 (and never 2 where the plan does not launch the fused step, A.deep
// = 0).  Within that reach every other kernel's velocity update reduces to
// the acoustic one (shear stresses of fluid edges are zero), so the fused
// step's recomputed neighbours equal the values the neighbouring tiles store.
constexpr int kReach = kDeepReach;
// x extent of a deep tile: a segment (the last one may be partial) whose
// recomputed faces beyond it (i0-2, i0-1, i0+64) are outside the grid or
// outside the x layer, so that every layer face it touches is its own.
__device__ __forceinline__ bool deep_x_ok(const Grid &g, int i0) {
  auto ok = [&](int p) { return p < 0 || p >= g.nx || !in_layer(p, g.nx, g.L); };
  return ok(i0 - 2) && ok(i0 - 1) && ok(i0 + kSeg);
}
__device__ __forceinline__ int idx_at(const StepArgs &A, long long off) {
  return A.idx16 ? reinterpret_cast<const uint16_t *>(A.idx)[off] : A.idx[off];
}
__global__ void k_tile_kinds(StepArgs A, uint8_t *__restrict__ kind) {
  const Grid &g = A.g;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < A.n_tiles; t += gridDim.x * blockDim.x) {
    int bx, by, k0, k1;
    tile_coords(A, t, bx, by, k0, k1);
    bool ac = true;
    for (int r = 0; ac && r < kRows; ++r) {
      const int j = by * kRows + r;
      if (j >= g.ny) break;
      const uint8_t *colp = A.cls + ((long long)j * A.nseg + bx) * A.kpad;
      for (int k = k0; k < k1; ++k)
        if (colp[k] == 0) {
          ac = false;
          break;
        }
    }
    int kd = ac ? 1 : 0;
    const int i0 = bx * kSeg, j0 = by * kRows;
    if (ac && A.deep && deep_x_ok(g, i0) && j0 - kReach >= g.L && j0 + kRows - 1 + kReach < g.ny - g.L &&
        k0 - kReach >= g.L && k1 - 1 + kReach < g.nz - g.L) {
      const int c = A.cls[((long long)j0 * A.nseg + bx) * A.kpad + k0];
      bool deep = true;
      for (int j = j0 - 1; deep && j <= j0 + kRows; ++j) {
        const long long col = ((long long)j * A.nseg + bx) * A.kpad;
        const bool inner = j >= j0 && j < j0 + kRows;
        for (int k = k0 - 1; k <= k1; ++k)
          if (A.cls[col + k] != c || (inner && k >= k0 && k < k1 && A.keep[col + k] != 0)) {
            deep = false;
            break;
          }
      }
      // third cell in x beyond the segment, where it is inside the grid (outside
      // it the fused step reads only zero ghost faces and stresses)
      const bool xl = i0 - kReach >= 0, xr = i0 + kSeg - 1 + kReach < g.nx;
      for (int k = k0 - kReach; deep && k < k1 + kReach; ++k)
        for (int j = j0 - kReach; j < j0 + kRows + kReach; ++j)
          if ((xl && idx_at(A, g.off(i0 - kReach, j, k)) != c - 1) ||
              (xr && idx_at(A, g.off(i0 + kSeg - 1 + kReach, j, k)) != c - 1)) {
            deep = false;
            break;
          }
      if (deep) kd = 2;
    }
    kind[t] = (uint8_t)kd;
  }
}

// Stable split of the tile ids by kind: lists[0] acoustic, lists[1] general,
// lists[2] deep; counts[0..2] their lengths.  One block; chunked block-wide
// prefix sums.
constexpr int kListThreads = 1024;
__global__ void __launch_bounds__(kListThreads)
    k_tile_lists(const uint8_t *__restrict__ kind, int n, int *__restrict__ list_ac,
                 int *__restrict__ list_gen, int *__restrict__ list_deep, int *__restrict__ counts) {
  __shared__ int sa[kListThreads], sd[kListThreads];
  __shared__ int base_a, base_d;
  const int t = threadIdx.x;
  if (t == 0) base_a = base_d = 0;
  __syncthreads();
  for (int c0 = 0; c0 < n; c0 += kListThreads) {
    const int id = c0 + t;
    const int kd = id < n ? kind[id] : 0;
    const int fa = kd == 1 ? 1 : 0, fd = kd == 2 ? 1 : 0;
    sa[t] = fa;
    sd[t] = fd;
    __syncthreads();
    for (int o = 1; o < kListThreads; o <<= 1) {  // inclusive Hillis-Steele scans
      const int va = t >= o ? sa[t - o] : 0, vd = t >= o ? sd[t - o] : 0;
      __syncthreads();
      sa[t] += va;
      sd[t] += vd;
      __syncthreads();
    }
    const int ba = base_a + sa[t] - fa, bd = base_d + sd[t] - fd;  // earlier tiles of each kind
    if (id < n) {
      if (fa) list_ac[ba] = id;
      else if (fd) list_deep[bd] = id;
      else list_gen[id - ba - bd] = id;
    }
    __syncthreads();
    if (t == kListThreads - 1) {
      base_a += sa[t];
      base_d += sd[t];
    }
    __syncthreads();
  }
  if (t == 0) {
    counts[0] = base_a;
    counts[1] = n - base_a - base_d;
    counts[2] = base_d;
  }
}

// Batched step kernels: a grid of persistent blocks, or of one block per tile
// (when the grid is at least as long as the table), walks the live part of
// one of the two per-kind tile tables (acoustic / general, each in solve order, so
// the tiles of the solves still running are a prefix whose length,
// table_len[live], the device computed in the prologue); each XCD takes a
// contiguous band of every round.  Every solve keeps its own grid, tables,
// step count and source coefficients; the per-cell arithmetic is the
// single-solve tile code.
template <int BY, bool AC>
__global__ void __launch_bounds__(kSeg * BY)
    k_velocity_batched(BatchWalk W, const float2 *__restrict__ coef, int max_steps, int n) {
  const int len = ((const ScalarI32 *)W.table_len)[W.live];
  int staged = -1, t, stride;
  if ((int)gridDim.x >= len) {  // one block per tile
    if ((int)blockIdx.x >= len) return;
    t = xcd_band(blockIdx.x, len);
    stride = len;
  } else {                      // persistent blocks
    t = xcd_band(blockIdx.x, gridDim.x);
    stride = gridDim.x;
  }
  for (; t < len; t += stride) {
    // uniform reads through the scalar cache: the tile, then its solve's arguments
    const BatchTile tl = scalar_copy(W.tiles + ((const ScalarI32 *)W.table)[t]);
    const StepArgs A = scalar_copy(W.desc + tl.solve);
    if (tl.solve != staged) {
      __syncthreads();
      stage_lut(s_lut, A.lut, A.n_mat);
      __syncthreads();
      staged = tl.solve;
    }
    const float2 cs = coef[(long long)tl.solve * max_steps + n];
    if (AC)
      velocity_ac_tile(A, s_lut, tl.bx, tl.by * BY + wave_row(), tl.k0, tl.k1, cs.x, cs.y);
    else
      velocity_tile(A, s_lut, tl.bx, tl.by * BY + wave_row(), tl.k0, tl.k1, cs.x, cs.y);
  }
}

template <int BY, bool AC>
__global__ void __launch_bounds__(kSeg * BY)
    k_stress_batched(BatchWalk W, const int *__restrict__ cap, int n) {
  const int len = ((const ScalarI32 *)W.table_len)[W.live];
  int staged = -1, t, stride;
  if ((int)gridDim.x >= len) {  // one block per tile
    if ((int)blockIdx.x >= len) return;
    t = xcd_band(blockIdx.x, len);
    stride = len;
  } else {                      // persistent blocks
    t = xcd_band(blockIdx.x, gridDim.x);
    stride = gridDim.x;
  }
  for (; t < len; t += stride) {
    // uniform reads through the scalar cache: the tile, then its solve's arguments
    const BatchTile tl = scalar_copy(W.tiles + ((const ScalarI32 *)W.table)[t]);
    const StepArgs A = scalar_copy(W.desc + tl.solve);
    if (tl.solve != staged) {
      __syncthreads();
      stage_lut(s_lut, A.lut, A.n_mat);
      __syncthreads();
      staged = tl.solve;
    }
    const int capture = (n + 1 >= cap[tl.solve]) ? 1 : 0;
    if (AC)
      stress_ac_tile(A, s_lut, tl.bx, tl.by * BY + wave_row(), tl.k0, tl.k1, capture);
    else
      stress_tile(A, s_lut, tl.bx, tl.by * BY + wave_row(), tl.k0, tl.k1, capture);
  }
}

// Stable split of the batch tile table by kind, and the live lengths of both
// tables: len[kind][q] = tiles of that kind among the first q solves
// (solve_end[q - 1] = end of solve q - 1's tiles in the table).  One block.
__global__ void __launch_bounds__(kListThreads)
    k_batch_split(const BatchTile *__restrict__ tiles, int n, const int *__restrict__ solve_end,
                  int n_solves, int *__restrict__ table_ac, int *__restrict__ table_gen,
                  int *__restrict__ scan, int *__restrict__ len_ac, int *__restrict__ len_gen) {
  __shared__ int sc[kListThreads];
  __shared__ int base;
  const int t = threadIdx.x;
  if (t == 0) base = 0;
  __syncthreads();
  for (int c0 = 0; c0 < n; c0 += kListThreads) {
    const int id = c0 + t;
    const int f = (id < n && tiles[id].kind) ? 1 : 0;
    sc[t] = f;
    __syncthreads();
    for (int o = 1; o < kListThreads; o <<= 1) {
      const int v = t >= o ? sc[t - o] : 0;
      __syncthreads();
      sc[t] += v;
      __syncthreads();
    }
    const int incl = base + sc[t];
    if (id < n) {
      scan[id] = incl;
      if (f) table_ac[incl - 1] = id;
      else table_gen[id - incl] = id;
    }
    __syncthreads();
    if (t == kListThreads - 1) base += sc[t];
    __syncthreads();
  }
  for (int q = t; q <= n_solves; q += kListThreads) {
    const int end = q == 0 ? 0 : solve_end[q - 1];
    const int ac = end == 0 ? 0 : scan[end - 1];
    len_ac[q] = ac;
    len_gen[q] = end - ac;
  }
}

// Kinds of the batch tile table (rows of by rows each), as k_tile_kinds.
__global__ void k_batch_kinds(const StepArgs *__restrict__ desc, BatchTile *__restrict__ tiles,
                              int n_tiles, int by) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n_tiles; t += gridDim.x * blockDim.x) {
    BatchTile &tl = tiles[t];
    const StepArgs &A = desc[tl.solve];
    bool ac = true;
    for (int r = 0; ac && r < by; ++r) {
      const int j = tl.by * by + r;
      if (j >= A.g.ny) break;
      const uint8_t *colp = A.cls + ((long long)j * A.nseg + tl.bx) * A.kpad;
      for (int k = tl.k0; k < tl.k1; ++k)
        if (colp[k] == 0) {
          ac = false;
          break;
        }
    }
    tl.kind = ac ? 1 : 0;
  }
}

// Padded index map (uint8, or uint16 for 16-bit maps) with edge-replicated
// ghosts; flags out-of-range indices (which are replaced by 0 so the solve
// stays in bounds).
__global__ void k_pack_idx(const uint8_t *__restrict__ mat, uint8_t *__restrict__ idx, Grid g,
                           int n_mat, int idx16, int *flags) {
  const long long total = (long long)g.rows * (g.nz + 2 * kGhost) * g.pitch;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const long long r = t / g.pitch;
    const int i = min(max((int)(t - r * g.pitch) - kGhost, 0), g.nx - 1);
    const int j = min(max((int)(r % g.rows) - kGhost, 0), g.ny - 1);
    const int k = min(max((int)(r / g.rows) - kGhost, 0), g.nz - 1);
    const long long q = ((long long)k * g.ny + j) * g.nx + i;
    int m = idx16 ? reinterpret_cast<const uint16_t *>(mat)[q] : mat[q];
    if (m >= n_mat) {
      atomicOr(flags, kStatusIndex);
      m = 0;
    }
    if (idx16)
      reinterpret_cast<uint16_t *>(idx)[kX0 - kGhost + t] = (uint16_t)m;
    else
      idx[kX0 - kGhost + t] = (uint8_t)m;
  }
}

// Segment classes (see kSeg): m + 1 if every cell within two cells of the
// segment holds lossless fluid m, else 0.  Reads the padded, ghost-replicated
// index map, so cells outside the grid count as their edge neighbour.  Two
// passes: k_row_uniform finds, for every row of the padded grid (two ghost
// rows and planes on each side) and segment, the index all of the segment's
// cells and two more on each side in x share (255 where they differ);
// k_classify then asks the 5 x 5 rows around the segment's own row to agree.
// Written as one z column of kpad bytes per (row, segment).  rowu holds 16-bit
// entries (0xffff where the cells differ) for either index width; only
// fluids of index below 255 get a class of their own (classes are bytes).
constexpr int kRowMixed = 0xffff;
__global__ void k_row_uniform(const uint8_t *__restrict__ idx, uint16_t *__restrict__ rowu, Grid g,
                              int nseg, int idx16) {
  const long long total = (long long)nseg * (g.ny + 4) * (g.nz + 4);
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int sg = (int)(t % nseg);
    const long long r = t / nseg;
    const int j = (int)(r % (g.ny + 4)) - kGhost, k = (int)(r / (g.ny + 4)) - kGhost;
    const int x0 = sg * kSeg;
    const int xa = x0 - kGhost, xb = min(x0 + kSeg - 1, g.nx - 1) + kGhost;
    const long long row = g.off(0, j, k);
    auto at = [&](int x) {
      return idx16 ? (int)reinterpret_cast<const uint16_t *>(idx)[row + x] : (int)idx[row + x];
    };
    const int m = at(xa);
    bool same = true;
    for (int x = xa + 1; same && x <= xb; ++x) same = at(x) == m;
    rowu[t] = same ? (uint16_t)m : (uint16_t)kRowMixed;
  }
}

__global__ void k_classify(const uint16_t *__restrict__ rowu, uint8_t *__restrict__ cls, Grid g,
                           int nseg, int kpad, const float *__restrict__ lut) {
  const long long total = (long long)nseg * g.ny * g.nz;
  const long long rstride = (long long)(g.ny + 4) * nseg;  // one padded plane of rowu
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(t % g.nz);
    const long long r = t / g.nz;
    const int sg = (int)(r % nseg), j = (int)(r / nseg);
    const uint16_t *c = rowu + (long long)(k + kGhost) * rstride + (long long)(j + kGhost) * nseg + sg;
    const int m = *c;
    bool ok = m < 255 && lut[m * kLutW + kLossless] != 0.f;
    for (int dk = -kGhost; ok && dk <= kGhost; ++dk)
      for (int dj = -kGhost; ok && dj <= kGhost; ++dj)
        ok = c[dk * rstride + (long long)dj * nseg] == m;
    cls[r * kpad + k] = ok ? (uint8_t)(m + 1) : (uint8_t)0;
  }
}

// Keep flags (see StepArgs::keep): 1 where a class-0 (elastic) segment of the
// same x segment lies within rows j-2..j+1 of the same plane (it reads
// sigma_yy here) or within planes k-2..k+1 of the same row (sigma_zz).
__global__ void k_keep(const uint8_t *__restrict__ cls, uint8_t *__restrict__ keep, Grid g,
                       int nseg, int kpad) {
  const long long total = (long long)nseg * g.ny * g.nz;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(t % g.nz);
    const long long r = t / g.nz;
    const int sg = (int)(r % nseg), j = (int)(r / nseg);
    bool need = false;
    for (int jj = max(j - 2, 0); !need && jj <= min(j + 1, g.ny - 1); ++jj)
      need = cls[((long long)jj * nseg + sg) * kpad + k] == 0;
    for (int kk = max(k - 2, 0); !need && kk <= min(k + 1, g.nz - 1); ++kk)
      need = cls[r * kpad + kk] == 0;
    keep[r * kpad + k] = need ? 1 : 0;
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
// LDS of a launch: for the general kernels the whole table of an 8-bit map,
// or the column of a 16-bit map's table that the kernel gathers per neighbour
// (buoyancy: up to 16 KB; edge inputs: up to 32 KB); the fluid rows for the
// acoustic kernels and the fused step.
static size_t lds_velocity(const StepArgs &a) {
  return a.idx16 ? (size_t)a.n_mat * sizeof(float) : lut_bytes(a.n_mat);
}
static size_t lds_stress(const StepArgs &a) {
  return a.idx16 ? (size_t)a.n_mat * sizeof(float2) : lut_bytes(a.n_mat);
}
static size_t lds_fluid(const StepArgs &a) { return lut_bytes(a.n_fluid); }

// The buoyancy and edge-input columns of a 16-bit map's table (rows [0,
// n_mat)), written after its rows; see rho_column / edge_column.
__global__ void k_lut_columns(float *lut, int n_mat) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_mat) return;
  const float *row = lut + (size_t)m * kLutW;
  const_cast<float *>(rho_column(lut))[m] = row[kRhoS];
  const_cast<float2 *>(edge_column(lut))[m] = make_float2(row[kInvMu], row[kTauS]);
}

hipError_t launch_lut_columns(float *lut, int n_mat, hipStream_t s) {
  hipLaunchKernelGGL(k_lut_columns, dim3((n_mat + 255) / 256), dim3(256), 0, s, lut, n_mat);
  return hipGetLastError();
}

// lists: [0] acoustic tile ids, [1] general tile ids (n_tiles ints each);
// counts: their lengths (device).  Each launch has n_tiles blocks.
hipError_t launch_velocity(const StepArgs &a, const int *const *lists, const int *counts,
                           int which, hipStream_t s) {
  if (which == 0)
    hipLaunchKernelGGL(k_velocity_ac, dim3(a.n_tiles), dim3(kSeg, kRows, 1), lds_fluid(a), s, a,
                       lists[0], counts);
  else if (a.idx16)
    hipLaunchKernelGGL(k_velocity<uint16_t>, dim3(a.n_tiles), dim3(kSeg, kRows, 1), lds_velocity(a),
                       s, a, lists[1], counts + 1);
  else
    hipLaunchKernelGGL(k_velocity<uint8_t>, dim3(a.n_tiles), dim3(kSeg, kRows, 1), lds_velocity(a),
                       s, a, lists[1], counts + 1);
  return hipGetLastError();
}

// Fused step of the deep tiles (lists[2], counts[2]).
hipError_t launch_deep(const StepArgs &a, const int *const *lists, const int *counts,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_step_deep, dim3(a.n_tiles), dim3(kSeg, kRows, 1), lds_fluid(a), s, a,
                     lists[2], counts + 2);
  return hipGetLastError();
}

hipError_t launch_stress(const StepArgs &a, const int *const *lists, const int *counts, int which,
                         hipStream_t s) {
  if (which == 0)
    hipLaunchKernelGGL(k_stress_ac, dim3(a.n_tiles), dim3(kSeg, kRows, 1), lds_fluid(a), s, a,
                       lists[0], counts);
  else if (a.idx16)
    hipLaunchKernelGGL(k_stress<uint16_t>, dim3(a.n_tiles), dim3(kSeg, kRows, 1), lds_stress(a), s,
                       a, lists[1], counts + 1);
  else
    hipLaunchKernelGGL(k_stress<uint8_t>, dim3(a.n_tiles), dim3(kSeg, kRows, 1), lds_stress(a), s,
                       a, lists[1], counts + 1);
  return hipGetLastError();
}

hipError_t launch_batch_kinds(const StepArgs *desc, BatchTile *tiles, int n_tiles, int by,
                              hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  int blocks = (n_tiles + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_batch_kinds, dim3(blocks), dim3(256), 0, s, desc, tiles, n_tiles, by);
  return hipGetLastError();
}

hipError_t launch_tile_lists(const StepArgs &a, uint8_t *kind, int *const *lists, int *counts,
                             hipStream_t s) {
  int blocks = (a.n_tiles + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_tile_kinds, dim3(blocks), dim3(256), 0, s, a, kind);
  hipLaunchKernelGGL(k_tile_lists, dim3(1), dim3(kListThreads), 0, s, kind, a.n_tiles, lists[0],
                     lists[1], lists[2], counts);
  return hipGetLastError();
}

hipError_t launch_pack(const uint8_t *mat, uint8_t *idx, const Grid &g, int n_mat, int idx16,
                       int *flags, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_idx, dim3(2048), dim3(256), 0, s, mat, idx, g, n_mat, idx16, flags);
  return hipGetLastError();
}

hipError_t launch_classify(const uint8_t *idx, uint16_t *rowu, uint8_t *cls, uint8_t *keep,
                           const Grid &g, int nseg, int kpad, const float *lut, int idx16,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_row_uniform, dim3(4096), dim3(256), 0, s, idx, rowu, g, nseg, idx16);
  hipLaunchKernelGGL(k_classify, dim3(4096), dim3(256), 0, s, rowu, cls, g, nseg, kpad, lut);
  hipLaunchKernelGGL(k_keep, dim3(4096), dim3(256), 0, s, cls, keep, g, nseg, kpad);
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

// Batched step: the four persistent kernels over the live parts of the two
// per-kind tables.  W[0] walks the acoustic table, W[1] the general one.
template <int BY>
static hipError_t batched_step(const BatchWalk *W, const float2 *coef, const int *cap,
                               int max_steps, int n, int blocks, int max_mat, hipStream_t s) {
  const dim3 grid(blocks), block(kSeg, BY, 1);
  const size_t lds = lut_bytes(max_mat);
  hipLaunchKernelGGL((k_velocity_batched<BY, true>), grid, block, lds, s, W[0], coef, max_steps, n);
  hipLaunchKernelGGL((k_velocity_batched<BY, false>), grid, block, lds, s, W[1], coef, max_steps, n);
  hipLaunchKernelGGL((k_stress_batched<BY, true>), grid, block, lds, s, W[0], cap, n);
  hipLaunchKernelGGL((k_stress_batched<BY, false>), grid, block, lds, s, W[1], cap, n);
  return hipGetLastError();
}

hipError_t launch_batched_step(int by, const BatchWalk *W, const float2 *coef, const int *cap,
                               int max_steps, int n, int blocks, int max_mat, hipStream_t s) {
  switch (by) {
    case 1: return batched_step<1>(W, coef, cap, max_steps, n, blocks, max_mat, s);
    case 2: return batched_step<2>(W, coef, cap, max_steps, n, blocks, max_mat, s);
    case 4: return batched_step<4>(W, coef, cap, max_steps, n, blocks, max_mat, s);
    case 8: return batched_step<8>(W, coef, cap, max_steps, n, blocks, max_mat, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_batch_split(const BatchTile *tiles, int n, const int *solve_end, int n_solves,
                              int *table_ac, int *table_gen, int *scan, int *len_ac, int *len_gen,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_batch_split, dim3(1), dim3(kListThreads), 0, s, tiles, n, solve_end,
                     n_solves, table_ac, table_gen, scan, len_ac, len_gen);
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
