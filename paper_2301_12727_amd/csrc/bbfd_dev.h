// Device-side data layout shared by the HIP kernels and the host side of the
// library.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bbfd {

// Padded field layout: every field array holds the interior (nx, ny, nz) plus
// two zero ghost cells on each side, x fastest.  Rows are `pitch` floats apart
// (pitch >= nx + 4, multiple of 32) and every row's interior starts on a
// 128-byte boundary, so interior cell (i, j, k) sits at
//   kX0 + ((k + 2) * rows + (j + 2)) * pitch + i,   rows = ny + 4.
// Ghost slots i = -2, -1 of a row alias the unused tail of the previous row.
constexpr int kX0 = 32;
constexpr int kGhost = 2;

struct Grid {
  int nx, ny, nz;
  int pitch;      // floats between consecutive rows
  int rows;       // ny + 4
  int L;          // absorbing layer thickness (cells)
  int ks;         // source plane
  long long plane;   // pitch * rows
  long long stride;  // elements per padded array (multiple of 64)
  __host__ __device__ long long off(int i, int j, int k) const {
    return kX0 + ((long long)(k + kGhost) * rows + (j + kGhost)) * pitch + i;
  }
};

// Per-material FP32 table (host-derived in FP64, scaled by dt/dx).  The four
// moduli of a cell centre and the two edge-average inputs are adjacent so the
// kernels fetch them as one float4 and one float2.
enum LutField {
  kPiU = 0,    // pi_U * dt / dx          (unrelaxed P modulus)
  kMuU = 1,    // mu_U * dt / dx          (unrelaxed shear modulus)
  kPiTau = 2,  // pi_R * tau_P * dt / dx  (memory-variable target, normal part)
  kMuTau = 3,  // mu_R * tau_S * dt / dx  (memory-variable target, shear part)
  kInvMu = 4,  // dx / (mu_R * dt), +inf for fluids (edge harmonic mean)
  kTauS = 5,   // tau_S                   (edge average)
  kRhoS = 6,   // rho * dx / dt           (buoyancy of a face: 2 / (rhoS_a + rhoS_b))
  kLossless = 7,  // 1 for a fluid without attenuation (no shear, no memory), else 0
  kLutW = 8
};
constexpr int kMaxMaterials = 256;      // rows of an 8-bit map's table (staged in LDS)
constexpr int kMaxMaterials16 = 4096;   // rows of a 16-bit map's table (12-bit CT levels)
// A 16-bit map's table region holds, after its kMaxMaterials16 rows, two
// columns of it that the general kernels stage in LDS: the buoyancy input
// kRhoS (one float per material) and the edge inputs kInvMu, kTauS (one
// float2 per material).  kLutW + 3 floats per material in all.
constexpr int kLutW16 = kLutW + 3;
__host__ __device__ inline const float *rho_column(const float *lut) {
  return lut + (size_t)kMaxMaterials16 * kLutW;
}
__host__ __device__ inline const float2 *edge_column(const float *lut) {
  return reinterpret_cast<const float2 *>(lut + (size_t)kMaxMaterials16 * (kLutW + 1));
}

// Row segments: the kernels' waves cover 64 consecutive x cells of one row.
// A segment's class is m + 1 when every cell within two cells of it (the
// reach of both stencils, ghosts included) holds the same lossless fluid m;
// then shear stresses and memory variables there stay exactly zero and the
// three normal stresses stay equal, so the wave takes the acoustic path.
// Class 0 (mixed) takes the full viscoelastic path.
constexpr int kSeg = 64;

// State array slots inside the workspace.
enum Field {
  VX = 0, VY, VZ, SXX, SYY, SZZ, SXY, SXZ, SYZ, RXX, RYY, RZZ, RXY, RXZ, RYZ, kNState
};
// The first kNOut fields (v and the normal stresses) can be double-buffered.
constexpr int kNOut = 6;
// 18 CPML memories: 9 for the stress derivatives of the velocity update and 9
// for the velocity derivatives of the stress update.
constexpr int kNPsi = 18;

// CPML coefficient table per axis: 4 floats per index
//   [b at integer position, a at integer, b at half position i+1/2, a at half]
// with b = exp(-(d + alpha) dt), a = d/(d + alpha) (b - 1) (frequency-shifted
// CPML); b = 1, a = 0 where the profile is zero.
struct PmlTab {
  const float4 *x, *y, *z;
};

struct StepArgs {
  Grid g;
  const uint8_t *idx;     // padded, replicated ghosts; uint8 or (idx16) uint16 entries
  const uint8_t *cls;     // segment classes, [ny][nseg][kpad]: one z column per segment
  int nseg;               // ceil(nx / kSeg)
  int kpad;               // round_up(nz, 4) + 4 bytes per class column
  const uint8_t *keep;    // same layout: 1 where an elastic segment reads sigma_yy or
                          // sigma_zz of this segment (within 2 rows / 2 planes)
  const float *lut;       // kLutW floats per material
  int n_mat;              // materials in lut
  int n_fluid;            // rows [0, n_fluid) hold every fluid that has a segment class
  PmlTab pml;
  float *f[kNState];      // padded state arrays (read; shear stresses and memories
                          // are also written in place)
  float *fo[kNOut];       // where the velocity (VX..VZ) and normal-stress
                          // (SXX..SZZ) updates write: f itself (in place) or
                          // the other buffer of a double-buffered pair
  float *psi[kNPsi];      // padded CPML memories (touched in the layer only)
  const float2 *src;      // [ny][nx] source plane
  float *peak;            // [nz][ny][nx]
  float relax_a;          // (1 - h) / (1 + h), h = omega dt / 2
  float relax_b;          // 2 h / (1 + h)
  float src_c, src_s;     // per step: v_z face force src_c * Re S - src_s * Im S (x b_z)
  int capture;            // 1: update the peak map after this step
  int kchunk;             // z cells per tile
  int nby;                // row blocks per plane (rows per block: kRows)
  int n_tiles;            // x segments * row blocks * z chunks
  int deep;               // 1: tiles may be classified deep (fused step launched)
  int idx16;              // 1: 16-bit material indices (12-bit CT maps), table in global memory
};

// Rows of a single-solve tile (one wave per row).
constexpr int kRows = 4;
// Cells around a deep tile that its fused velocity + stress step reads.
constexpr int kDeepReach = 3;

// Batched sweeps: one entry per (solve, tile); solves are ordered by
// decreasing step count so the live tiles of step n are a prefix of the table.
struct BatchTile {
  int solve;
  int bx, by;   // x segment and row-block index inside the solve
  int k0, k1;   // z range
  int kind;     // 1: acoustic tile (set on the device once the classes are known)
  int pad[2];
};

// One persistent batched launch walks the live part of one per-kind tile table.
struct BatchWalk {
  const StepArgs *desc;
  const BatchTile *tiles;
  const int *table;       // tile indices of one kind, in solve order
  const int *table_len;   // [live solves] -> live length of table
  int live;               // solves still running at this step
};

// Device status block at the front of the workspace.
struct Status {
  int flags;       // bit 0: index out of range; bit 1: non-finite peak
  int pad;
  float peak_value;
  int pad2;
  long long peak_index;
};
constexpr int kStatusIndex = 1;
constexpr int kStatusDiverged = 2;

}  // namespace bbfd
