// Host side of libbbfd: problem validation, FP64 derivation of the material,
// time-step and absorbing-layer constants, workspace layout, graph capture of
// the time loop and the C ABI declared in include/bbfd.h.
#include "bbfd.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <fstream>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "bbfd_dev.h"

namespace bbfd {
hipError_t launch_velocity(const StepArgs &a, const int *const *lists, const int *counts,
                           int which, hipStream_t s);
hipError_t launch_stress(const StepArgs &a, const int *const *lists, const int *counts, int which,
                         hipStream_t s);
hipError_t launch_tile_lists(const StepArgs &a, uint8_t *kind, int *const *lists, int *counts,
                             hipStream_t s);
hipError_t launch_deep(const StepArgs &a, const int *const *lists, const int *counts,
                       hipStream_t s);
hipError_t launch_lut_columns(float *lut, int n_mat, hipStream_t s);
hipError_t launch_batch_kinds(const StepArgs *desc, BatchTile *tiles, int n_tiles, int by,
                              hipStream_t s);
hipError_t launch_pack(const uint8_t *mat, uint8_t *idx, const Grid &g, int n_mat, int idx16,
                       int *flags, hipStream_t s);
hipError_t launch_fill(float *p, long long n, float v, hipStream_t s);
hipError_t launch_classify(const uint8_t *idx, uint16_t *rowu, uint8_t *cls, uint8_t *keep,
                           const Grid &g, int nseg, int kpad, const float *lut, int idx16,
                           hipStream_t s);
hipError_t launch_argmax(const float *P, int nx, int ny, int nz, int L, float *pv, long long *pi,
                         Status *st, hipStream_t s);
int argmax_partials();
hipError_t launch_rayleigh(const double4 *el, int n_el, int nx, int ny, int planes, double dx,
                           double z0, double kw, double pre, float2 *out, hipStream_t s,
                           const double2 *wts = nullptr);
hipError_t launch_backprop(const float2 *plane, int nx, int ny, double dx, double zp,
                           const double4 *pts, int n_pts, double kw, double pre, double2 *part,
                           double2 *out, hipStream_t s);
int backprop_partials(int n_pts);
hipError_t launch_record_plane(const float *vz, long long base, int pitch, int nx, int ny, float c,
                               float s, float2 *ph, hipStream_t st);
hipError_t launch_batched_step(int by, const BatchWalk *W, const float2 *coef, const int *cap,
                               int max_steps, int n, int blocks, int max_mat, hipStream_t s);
hipError_t launch_batch_split(const BatchTile *tiles, int n, const int *solve_end, int n_solves,
                              int *table_ac, int *table_gen, int *scan, int *len_ac, int *len_gen,
                              hipStream_t s);
hipError_t launch_plane_energy(const uint8_t *mat_s, const float *p_s, const uint8_t *mat_w,
                               const float *p_w, int nx, int ny, int L, int z_m, const Status *st,
                               const double *inv_z, int n_mat, int idx16, double2 *part,
                               double *out, hipStream_t s);
int energy_out_doubles();
int energy_partials();
}  // namespace bbfd

using namespace bbfd;

namespace {

constexpr double kCw = 1500.0;   // water speed (Table 1), also fixes dx from PPW
constexpr double kRhoW = 1000.0; // water density (Table 1)
constexpr double kPi = 3.14159265358979323846;
constexpr double kC1 = 9.0 / 8.0, kC2 = -1.0 / 24.0;
constexpr double kPmlR0 = 1e-3;  // design reflection of the absorbing layer

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(BBFD_EHIP, "%s: %s", what, hipGetErrorString(e));
}

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

namespace bbfd {
// Shared error reporting for the other translation units of the library.
int set_error(int code, const char *msg) { return fail(code, "%s", msg); }
}  // namespace bbfd

namespace {

// Zener element relaxing at omega0 with strength tau: factor applied to rho c^2
// so that the phase speed at omega0 equals the tabulated speed.
double relaxed_factor(double tau) {
  const std::complex<double> m = std::complex<double>(1.0, 1.0 + tau) / std::complex<double>(1.0, 1.0);
  const double re = std::real(1.0 / std::sqrt(m));
  return re * re;
}

}  // namespace

struct bbfd_plan {
  bbfd_problem prob{};
  std::vector<bbfd_material> mats;
  double dx = 0, dt = 0, omega = 0, cmax = 0, d0 = 0;
  int nt = 0, cap = 0, ks = 0;
  std::vector<double> consts;  // 9 per material
  std::vector<double> inv_z;   // 1 / (2 rho c_l) per material (plane intensity sums)
  Grid g{};
  std::vector<float> lut;      // n_materials x kLutW
  std::vector<float4> pmltab;  // nx + ny + nz entries
  float *h_lut = nullptr;      // pinned copies, made at the first solve
  float4 *h_pml = nullptr;
  float relax_a = 0, relax_b = 0;
  std::vector<float> src_c, src_s;
  int kchunk = 1;
  int nseg = 1;
  int kpad = 4;                // bytes per class column (round_up(nz, 4) + 4)
  size_t off_status = 0, off_lut = 0, off_pml = 0, off_pv = 0, off_pi = 0, off_idx = 0,
         off_cls = 0, off_keep = 0, off_rowu = 0, off_alt = 0, off_kind = 0, off_lists = 0, off_counts = 0, off_state = 0, off_psi = 0,
         off_energy = 0, off_aux = 0,
         ws_bytes = 0;
  int n_tiles = 0;
  int n_fluid = 1;      // table rows the fluid-only kernels stage (see build_tables)
  bool deep = false;    // some tile can be deep: the fused step is launched
  bool branch = false;  // the captured steps run as two branches
  std::mutex mu;
  hipStream_t cap_stream = nullptr;
  hipStream_t side_stream = nullptr;  // second branch of the captured steps
  hipEvent_t fork = nullptr, join = nullptr;
  // Captured time loops, one per pointer set (mat, src, peak, workspace), at
  // most kGraphCache of them, least recently used replaced first.  `done` is
  // recorded after every launch; a graph is destroyed only once it has run.
  struct Captured {
    const void *key[4];
    hipGraph_t graph;
    hipGraphExec_t exec;
    hipEvent_t done;
    uint64_t used;
  };
  std::vector<Captured> graphs;
  uint64_t clock = 0;
  uint64_t captures = 0;
};

namespace {

int validate_and_derive(const bbfd_problem *p, bbfd_plan *pl) {
  if (!p) return fail(BBFD_EINVAL, "null problem");
  if (p->nx <= 0 || p->ny <= 0 || p->nz <= 0 || p->pml < 0 || p->n_steps <= 0)
    return fail(BBFD_EINVAL, "sizes must be positive (nx %d ny %d nz %d pml %d steps %d)", p->nx,
                p->ny, p->nz, p->pml, p->n_steps);
  if (2 * p->pml >= p->nx || 2 * p->pml >= p->ny || 2 * p->pml >= p->nz)
    return fail(BBFD_EINVAL, "absorbing layer of %d cells does not fit the grid", p->pml);
  if ((long long)p->nx * p->ny > (1LL << 30))
    return fail(BBFD_EINVAL, "plane too large");
  if (!(p->freq_hz > 0) || !(p->ppw > 0) || !(p->qc > 0) || !(p->cfl_safety > 0))
    return fail(BBFD_EINVAL, "frequency, ppw, qc and cfl_safety must be positive");
  if (p->index_bits != 0 && p->index_bits != 8 && p->index_bits != 16)
    return fail(BBFD_EINVAL, "index_bits must be 8 or 16, not %d", p->index_bits);
  const int max_mat = p->index_bits == 16 ? kMaxMaterials16 : kMaxMaterials;
  if (p->n_materials < 1 || p->n_materials > max_mat || !p->materials)
    return fail(BBFD_EINVAL, "need 1..%d materials for %d-bit maps", max_mat,
                p->index_bits == 16 ? 16 : 8);
  pl->prob = *p;
  pl->mats.assign(p->materials, p->materials + p->n_materials);
  pl->prob.materials = pl->mats.data();

  const double dx = kCw / (p->freq_hz * p->ppw);  // PPW counted in water
  const double w0 = 2.0 * kPi * p->freq_hz;
  const double T = 1.0 / p->freq_hz;
  double cmax = 0.0;
  pl->consts.assign(9 * (size_t)p->n_materials, 0.0);
  for (int m = 0; m < p->n_materials; ++m) {
    const bbfd_material &q = pl->mats[m];
    if (!(q.rho > 0) || !(q.c_l > 0) || !(q.c_s >= 0) || !(q.alpha_l >= 0) || !(q.alpha_s >= 0))
      return fail(BBFD_EMATERIAL, "material %d: non-positive density/speed or negative attenuation", m);
    double nu = 0.5;  // fluid
    if (q.c_s > 0) {
      const double l2 = q.c_l * q.c_l, s2 = q.c_s * q.c_s;
      if (!(l2 > s2)) return fail(BBFD_EMATERIAL, "material %d: shear speed >= longitudinal", m);
      nu = (l2 - 2.0 * s2) / (2.0 * (l2 - s2));
      if (nu < -1.0 || nu >= 0.5)
        return fail(BBFD_EMATERIAL, "material %d: Poisson ratio %g outside [-1, 0.5)", m, nu);
    }
    // Q = qc * omega / (2 c alpha) (Eq. 3 with the correction factor); no loss -> Q infinite.
    const double qp = q.alpha_l > 0 ? p->qc * w0 / (2.0 * q.c_l * q.alpha_l) : HUGE_VAL;
    const double qs = (q.c_s > 0 && q.alpha_s > 0) ? p->qc * w0 / (2.0 * q.c_s * q.alpha_s) : HUGE_VAL;
    if (!(qp > 1.0) || !(qs > 1.0))
      return fail(BBFD_EMATERIAL, "material %d: quality factor <= 1 (Q_P %g, Q_S %g)", m, qp, qs);
    // One Zener mechanism at omega0: Q(omega0) = (2 + tau)/tau  ->  tau = 2/(Q - 1).
    const double tp = std::isinf(qp) ? 0.0 : 2.0 / (qp - 1.0);
    const double ts = std::isinf(qs) ? 0.0 : 2.0 / (qs - 1.0);
    const double pir = q.rho * q.c_l * q.c_l * relaxed_factor(tp);
    const double mur = q.rho * q.c_s * q.c_s * relaxed_factor(ts);
    const double piu = pir * (1.0 + tp), muu = mur * (1.0 + ts);
    cmax = std::fmax(cmax, std::sqrt(piu / q.rho));
    double *o = &pl->consts[9 * (size_t)m];
    o[0] = qp; o[1] = qs; o[2] = tp; o[3] = ts; o[4] = pir; o[5] = mur; o[6] = piu; o[7] = muu;
    o[8] = nu;
  }
  // Stability of the 4th-order staggered leapfrog in 3D: c dt/dx <= 1/(sqrt(3)(|c1|+|c2|)).
  const double dt_max = dx / (std::sqrt(3.0) * (kC1 - kC2) * cmax);
  const int nt = (int)std::ceil(T / (p->cfl_safety * dt_max));
  const double dt = T / nt;
  const int ks = p->source_k < 0 ? p->pml : p->source_k;
  if (ks < p->pml || ks >= p->nz - p->pml)
    return fail(BBFD_EGEOMETRY, "source plane %d inside the absorbing layer", ks);
  int cap = p->capture_start < 0 ? p->n_steps - 2 * nt : p->capture_start;
  if (cap < 0) cap = 0;
  if (cap > p->n_steps) return fail(BBFD_EINVAL, "capture_start beyond n_steps");
  pl->dx = dx; pl->dt = dt; pl->omega = w0; pl->cmax = cmax; pl->nt = nt; pl->cap = cap; pl->ks = ks;
  pl->d0 = p->pml > 0 ? 3.0 * cmax * std::log(1.0 / kPmlR0) / (2.0 * p->pml * dx) : 0.0;
  return BBFD_OK;
}

// Frequency-shifted CPML at coordinate xi (cells, integer or half-integer)
// along an axis of n cells with an L-cell layer: quadratic damping
// d = d0 (l/L)^2 and shift alpha = pi f0 (1 - l/L) at depth l;
// b = exp(-(d + alpha) dt), a = d/(d + alpha) (b - 1); b = 1, a = 0 outside.
void pml_coeff(const bbfd_plan *pl, int n, double xi, float *b, float *a) {
  const int L = pl->prob.pml;
  double depth = 0.0;
  if (L > 0) depth = std::fmax(0.0, std::fmax((L - 0.5) - xi, xi - (n - L - 0.5)));
  if (depth <= 0.0) {
    *b = 1.0f;
    *a = 0.0f;
    return;
  }
  const double d = pl->d0 * (depth / L) * (depth / L);
  const double al = kPi * pl->prob.freq_hz * (1.0 - depth / L);
  *b = (float)std::exp(-(d + al) * pl->dt);
  *a = (float)(d / (d + al) * std::expm1(-(d + al) * pl->dt));
}

int build_tables(bbfd_plan *pl) {
  const bbfd_problem &p = pl->prob;
  pl->lut.assign((size_t)p.n_materials * kLutW, 0.0f);
  pl->inv_z.resize(p.n_materials);
  for (int m = 0; m < p.n_materials; ++m)
    pl->inv_z[m] = 1.0 / (2.0 * pl->mats[m].rho * pl->mats[m].c_l);
  pl->pmltab.resize((size_t)p.nx + p.ny + p.nz);
  const double s = pl->dt / pl->dx;
  for (int m = 0; m < p.n_materials; ++m) {
    const double *c = &pl->consts[9 * (size_t)m];
    float *o = pl->lut.data() + m * kLutW;
    o[kRhoS] = (float)(pl->mats[m].rho / s);
    o[kPiU] = (float)(c[6] * s);
    o[kMuU] = (float)(c[7] * s);
    o[kPiTau] = (float)(c[4] * c[2] * s);
    o[kMuTau] = (float)(c[5] * c[3] * s);
    o[kTauS] = (float)c[3];
    o[kInvMu] = c[5] > 0 ? (float)(1.0 / (c[5] * s)) : INFINITY;
    o[kLossless] = (c[5] == 0.0 && c[2] == 0.0) ? 1.0f : 0.0f;  // no shear, no P memory
  }
  // Only lossless fluids of index below 255 get a segment class, and the
  // acoustic kernels and the fused step read the table rows of those classes
  // alone: they stage the rows up to the last such fluid (a 12-bit CT table
  // holds its fluid in row 0 and bone in the 4095 rows after it).
  pl->n_fluid = 1;
  for (int m = 0; m < std::min(p.n_materials, kMaxMaterials - 1); ++m)
    if (pl->lut[(size_t)m * kLutW + kLossless] != 0.0f) pl->n_fluid = m + 1;
  const int dims[3] = {p.nx, p.ny, p.nz};
  float4 *t = pl->pmltab.data();
  for (int ax = 0; ax < 3; ++ax)
    for (int i = 0; i < dims[ax]; ++i, ++t) {
      pml_coeff(pl, dims[ax], (double)i, &t->x, &t->y);
      pml_coeff(pl, dims[ax], i + 0.5, &t->z, &t->w);
    }
  const double h = 0.5 * pl->omega * pl->dt;  // dt / (2 tau_sigma), tau_sigma = 1/omega0
  pl->relax_a = (float)((1.0 - h) / (1.0 + h));
  pl->relax_b = (float)(2.0 * h / (1.0 + h));
  // Source: a normal-traction jump of 2 S across z = (ks + 1/2) dx, i.e. a
  // force layer on the v_z faces there, applied with the velocity update of
  // step n at t = n dt with a two-period sin^2 ramp.  In the scaled kernel
  // variables the face gains b_z * (src_c Re S - src_s Im S).
  pl->src_c.resize(p.n_steps);
  pl->src_s.resize(p.n_steps);
  const double T = 1.0 / p.freq_hz;
  for (int n = 0; n < p.n_steps; ++n) {
    const double t = n * pl->dt;
    double w = 1.0;
    if (t < 2.0 * T) {
      const double q = std::sin(kPi * t / (4.0 * T));
      w = q * q;
    }
    pl->src_c[n] = (float)(2.0 * w * std::cos(pl->omega * t));
    pl->src_s[n] = (float)(2.0 * w * std::sin(pl->omega * t));
  }
  return BBFD_OK;
}

// Tiles from which a single solve uses the fused step and two branches.
constexpr int kLargeTiles = 2048;
// Captured time loops a plan keeps (distinct pointer sets).
constexpr int kGraphCache = 4;

void layout(bbfd_plan *pl) {
  const bbfd_problem &p = pl->prob;
  Grid &g = pl->g;
  g.nx = p.nx; g.ny = p.ny; g.nz = p.nz; g.L = p.pml; g.ks = pl->ks;
  g.pitch = (int)round_up((size_t)p.nx + 2 * kGhost, 32);
  g.rows = p.ny + 2 * kGhost;
  g.plane = (long long)g.pitch * g.rows;
  g.stride = (long long)round_up(kX0 + (size_t)g.plane * (p.nz + 2 * kGhost), 64);
  const long long nbxy = (long long)((p.nx + kSeg - 1) / kSeg) * ((p.ny + kRows - 1) / kRows);
  // z cells per tile: at least ~8192 tiles (a few rounds of blocks over the
  // 256 CUs) and at most 8 planes, the shortest march that measured fastest
  // on the 400x400x520 workload (longer marches gain no reuse: every plane's
  // loads are issued afresh)
  const long long kc = std::min(8LL, (nbxy * p.nz) / 8192);
  pl->kchunk = (int)std::max(1LL, std::min<long long>(kc, p.nz));
  size_t o = 0;
  pl->off_status = o; o += 256;
  const bool idx16 = p.index_bits == 16;
  pl->off_lut = o;
  o += round_up((size_t)(idx16 ? kMaxMaterials16 * kLutW16 : kMaxMaterials * kLutW) * sizeof(float),
                256);
  pl->off_pml = o; o += round_up(((size_t)p.nx + p.ny + p.nz) * sizeof(float4), 256);
  pl->off_pv = o; o += round_up(argmax_partials() * sizeof(float), 256);
  pl->off_pi = o; o += round_up(argmax_partials() * sizeof(long long), 256);
  pl->off_idx = o; o += round_up((size_t)g.stride * (idx16 ? 2 : 1), 256);
  pl->nseg = (p.nx + kSeg - 1) / kSeg;
  pl->kpad = (int)round_up((size_t)p.nz, 4) + 4;
  pl->off_cls = o; o += round_up((size_t)pl->nseg * p.ny * pl->kpad, 256);
  pl->off_keep = o; o += round_up((size_t)pl->nseg * p.ny * pl->kpad, 256);
  pl->off_rowu = o; o += round_up((size_t)pl->nseg * (p.ny + 4) * (p.nz + 4) * 2, 256);
  pl->n_tiles = pl->nseg * (int)((p.ny + kRows - 1) / kRows) * ((p.nz + pl->kchunk - 1) / pl->kchunk);
  // A deep tile needs a whole x segment, a row block and a z chunk with
  // kDeepReach cells around them inside the grid and outside the layer; where
  // no tile can be deep the fused step is not launched at all.
  auto fits = [&](int n, int len) {
    for (int a = 0; a < n; a += len)
      if (a + len <= n && a - kDeepReach >= p.pml && a + len - 1 + kDeepReach < n - p.pml) return true;
    return false;
  };
  // in x a segment suffices whose recomputed faces beyond it are outside the
  // grid or outside the layer (the fused step handles the x layer)
  auto x_face_ok = [&](int q) { return q < 0 || q >= p.nx || (q >= p.pml && q < p.nx - p.pml); };
  bool xfit = false;
  for (int a = 0; a < p.nx; a += kSeg)
    xfit = xfit || (x_face_ok(a - 2) && x_face_ok(a - 1) && x_face_ok(a + kSeg));
  // Small grids are bound by launch and dependency latency, not by bytes: a
  // fifth launch per step costs more than the fused step saves, and
  // side-by-side branches only fill the tails of launches that take many
  // rounds of blocks.  Both are used from kLargeTiles tiles up.
  pl->deep = xfit && fits(p.ny, kRows) && fits(p.nz, pl->kchunk) && pl->n_tiles >= kLargeTiles;
  pl->branch = pl->n_tiles >= kLargeTiles;
  pl->off_kind = o; o += round_up((size_t)pl->n_tiles, 256);
  pl->off_lists = o; o += round_up(3 * (size_t)pl->n_tiles * sizeof(int), 256);
  pl->off_counts = o; o += 256;
  // energy-loss reduction: a status block for the water map's peak voxel, the
  // result, the block partials
  // phased-array refocusing: a point-source plane and the recorded phasor plane
  pl->off_aux = o; o += round_up(2 * (size_t)p.nx * p.ny * sizeof(float2), 256);
  pl->off_energy = o;
  o += round_up(256 + 256 + (size_t)energy_partials() * 16 + (size_t)p.n_materials * 8, 256);
  pl->off_state = o; o += (size_t)kNState * g.stride * sizeof(float);
  pl->off_psi = o; o += (size_t)kNPsi * g.stride * sizeof(float);
  pl->off_alt = o; o += (size_t)kNOut * g.stride * sizeof(float);  // second buffers of v, sigma_ii
  pl->ws_bytes = o;
}

int check_ws(const bbfd_plan *pl, const void *ws, uint64_t bytes) {
  if (!ws) return fail(BBFD_ENOMEM, "null workspace");
  if ((uintptr_t)ws % 256) return fail(BBFD_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < pl->ws_bytes)
    return fail(BBFD_ENOMEM, "workspace of %llu bytes, need %llu", (unsigned long long)bytes,
                (unsigned long long)pl->ws_bytes);
  return BBFD_OK;
}

StepArgs step_args(const bbfd_plan *pl, const uint8_t *, const float *src, float *peak, char *ws) {
  StepArgs a{};
  a.g = pl->g;
  a.idx = (const uint8_t *)(ws + pl->off_idx);
  a.cls = (const uint8_t *)(ws + pl->off_cls);
  a.nseg = pl->nseg;
  a.kpad = pl->kpad;
  a.keep = (const uint8_t *)(ws + pl->off_keep);
  a.lut = (const float *)(ws + pl->off_lut);
  a.n_mat = pl->prob.n_materials;
  a.n_fluid = pl->n_fluid;
  const float4 *t = (const float4 *)(ws + pl->off_pml);
  a.pml.x = t;
  a.pml.y = t + pl->prob.nx;
  a.pml.z = t + pl->prob.nx + pl->prob.ny;
  for (int f = 0; f < kNState; ++f)
    a.f[f] = (float *)(ws + pl->off_state) + (size_t)f * pl->g.stride;
  for (int f = 0; f < kNPsi; ++f)
    a.psi[f] = (float *)(ws + pl->off_psi) + (size_t)f * pl->g.stride;
  for (int f = 0; f < kNOut; ++f) a.fo[f] = a.f[f];  // in place unless the caller pairs buffers
  a.src = (const float2 *)src;
  a.peak = peak;
  a.relax_a = pl->relax_a;
  a.relax_b = pl->relax_b;
  a.kchunk = pl->kchunk;
  a.nby = (pl->prob.ny + kRows - 1) / kRows;
  a.n_tiles = pl->n_tiles;
  a.deep = pl->deep ? 1 : 0;
  a.idx16 = pl->prob.index_bits == 16 ? 1 : 0;
  return a;
}

// Pinned staging copies of the host tables (device uploads stay asynchronous
// and capturable); made once, at the first solve, under the plan's mutex.
int ensure_pinned(bbfd_plan *pl) {
  if (pl->h_lut) return BBFD_OK;
  hipError_t e;
  float *lut = nullptr;
  float4 *pml = nullptr;
  if ((e = hipHostMalloc((void **)&lut, pl->lut.size() * sizeof(float), hipHostMallocDefault)) !=
      hipSuccess)
    return hip_fail(e, "pinned LUT allocation");
  if ((e = hipHostMalloc((void **)&pml, pl->pmltab.size() * sizeof(float4), hipHostMallocDefault)) !=
      hipSuccess) {
    (void)hipHostFree(lut);
    return hip_fail(e, "pinned layer-table allocation");
  }
  std::memcpy(lut, pl->lut.data(), pl->lut.size() * sizeof(float));
  std::memcpy(pml, pl->pmltab.data(), pl->pmltab.size() * sizeof(float4));
  pl->h_pml = pml;
  pl->h_lut = lut;
  return BBFD_OK;
}

// Per-solve prologue: tables, cleared state/peak/status, packed index map,
// segment classes.
// With pinned = false the tables are uploaded from the plan's own (pageable)
// host vectors instead of its pinned copies, so no pinned staging is needed.
int enqueue_prologue(const bbfd_plan *pl, const uint8_t *mat, float *peak, char *ws, hipStream_t s,
                     bool pinned = true) {
  const bbfd_problem &p = pl->prob;
  hipError_t e;
  if ((e = hipMemcpyAsync(ws + pl->off_lut, pinned ? pl->h_lut : pl->lut.data(),
                          (size_t)p.n_materials * kLutW * sizeof(float),
                          hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_fail(e, "LUT upload");
  if ((e = hipMemcpyAsync(ws + pl->off_pml, pinned ? pl->h_pml : pl->pmltab.data(),
                          ((size_t)p.nx + p.ny + p.nz) * sizeof(float4), hipMemcpyHostToDevice,
                          s)) != hipSuccess)
    return hip_fail(e, "layer-table upload");
  if (p.index_bits == 16 &&
      (e = launch_lut_columns((float *)(ws + pl->off_lut), p.n_materials, s)) != hipSuccess)
    return hip_fail(e, "table columns");
  if ((e = launch_fill((float *)(ws + pl->off_status), 256 / sizeof(float), 0.f, s)) != hipSuccess)
    return hip_fail(e, "status clear");
  if ((e = launch_fill((float *)(ws + pl->off_state),
                       (long long)(kNState + kNPsi + kNOut) * pl->g.stride, 0.f, s)) != hipSuccess)
    return hip_fail(e, "state clear");
  const long long cells = (long long)p.nx * p.ny * p.nz;
  if ((e = launch_fill(peak, cells, 0.f, s)) != hipSuccess) return hip_fail(e, "peak clear");
  Status *st = (Status *)(ws + pl->off_status);
  const int idx16 = p.index_bits == 16 ? 1 : 0;
  if ((e = launch_pack(mat, (uint8_t *)(ws + pl->off_idx), pl->g, p.n_materials, idx16, &st->flags,
                       s)) != hipSuccess)
    return hip_fail(e, "index pack");
  if ((e = launch_classify((const uint8_t *)(ws + pl->off_idx), (uint16_t *)(ws + pl->off_rowu),
                           (uint8_t *)(ws + pl->off_cls),
                           (uint8_t *)(ws + pl->off_keep), pl->g, pl->nseg, pl->kpad,
                           (const float *)(ws + pl->off_lut), idx16, s)) != hipSuccess)
    return hip_fail(e, "segment classes");
  StepArgs a = step_args(pl, mat, nullptr, peak, ws);
  int *lists[3] = {(int *)(ws + pl->off_lists), (int *)(ws + pl->off_lists) + pl->n_tiles,
                   (int *)(ws + pl->off_lists) + 2 * (size_t)pl->n_tiles};
  if ((e = launch_tile_lists(a, (uint8_t *)(ws + pl->off_kind), lists, (int *)(ws + pl->off_counts),
                             s)) != hipSuccess)
    return hip_fail(e, "tile lists");
  return BBFD_OK;
}

// Per-solve epilogue: peak voxel and finiteness into the status block.
int enqueue_epilogue(const bbfd_plan *pl, float *peak, char *ws, hipStream_t s) {
  const bbfd_problem &p = pl->prob;
  hipError_t e = launch_argmax(peak, p.nx, p.ny, p.nz, p.pml, (float *)(ws + pl->off_pv),
                               (long long *)(ws + pl->off_pi), (Status *)(ws + pl->off_status), s);
  if (e != hipSuccess) return hip_fail(e, "argmax launch");
  return BBFD_OK;
}

// Make `to` wait for the work enqueued so far on `from`.
hipError_t link(hipStream_t from, hipStream_t to, hipEvent_t ev) {
  hipError_t e = hipEventRecord(ev, from);
  return e != hipSuccess ? e : hipStreamWaitEvent(to, ev, 0);
}

// Enqueue one whole solve on s (no synchronisation).  With ev != NULL (direct
// launches only), ev[2 (5n + q)] / ev[2 (5n + q) + 1] bracket kernel q of step
// n (q: 0 acoustic velocity, 1 general velocity, 2 acoustic stress, 3 general
// stress, 4 fused step of the deep tiles).  With side != NULL (graph capture
// only, under the plan's lock), each step forks in two branches: the fused
// step of the deep tiles runs on `side` beside the velocity kernels, then the
// acoustic stress kernel beside the general one; the kernels of a branch pair
// touch disjoint outputs, so running them side by side fills the tail of one
// with blocks of the other.
constexpr int kStepKernels = 5;
// A solve that records, instead of capturing peaks: the source on plane ks
// (overriding the plan's), and the complex phasor of v_z on the faces of plane
// k_rec over the last period, (2 / N_T) sum v_z exp(-i omega t_n) with
// t_n = (n + 1/2) dt (the time level of the velocities of step n).
struct Record {
  int ks;
  int k_rec;
  float2 *phasor;  // [ny][nx], cleared here unless accumulate
  bool accumulate = false;
};

// Steps [n0, n1) of a solve whose prologue has been enqueued (arguments as
// enqueue_solve).
int enqueue_steps(const bbfd_plan *pl, const uint8_t *mat, const float *src, float *peak,
                  char *ws, hipStream_t s, int n0, int n1, hipEvent_t *ev = nullptr,
                  hipStream_t side = nullptr, const Record *rec = nullptr) {
  const bbfd_problem &p = pl->prob;
  hipError_t e;
  StepArgs a = step_args(pl, mat, src, peak, ws);
  if (rec) a.g.ks = rec->ks;
  const int *lists[3] = {(const int *)(ws + pl->off_lists),
                         (const int *)(ws + pl->off_lists) + pl->n_tiles,
                         (const int *)(ws + pl->off_lists) + 2 * (size_t)pl->n_tiles};
  const int *counts = (const int *)(ws + pl->off_counts);
  // v and the normal stresses alternate between two buffers: the velocity
  // update reads cur and writes nxt; the stress update reads the new velocity
  // (nxt) and the current stresses (cur) and writes the stresses to nxt; the
  // fused step of the deep tiles reads cur and writes nxt.
  float *cur[kNOut], *nxt[kNOut];
  for (int f = 0; f < kNOut; ++f) {
    cur[f] = a.f[f];
    nxt[f] = (float *)(ws + pl->off_alt) + (size_t)f * pl->g.stride;
    if (n0 % 2) std::swap(cur[f], nxt[f]);  // step n reads the buffers of parity n
  }
  for (int n = n0; n < n1; ++n) {
    a.src_c = pl->src_c[n];
    a.src_s = pl->src_s[n];
    a.capture = (n + 1 >= pl->cap) ? 1 : 0;
    StepArgs av = a, as = a, ad = a;
    for (int f = 0; f < kNOut; ++f) {
      const bool vel = f <= VZ;
      av.f[f] = cur[f];
      av.fo[f] = vel ? nxt[f] : cur[f];
      as.f[f] = vel ? nxt[f] : cur[f];
      as.fo[f] = nxt[f];
      ad.f[f] = cur[f];
      ad.fo[f] = nxt[f];
    }
    if (side) {
      if ((e = link(s, side, pl->fork)) != hipSuccess ||
          (pl->deep && (e = launch_deep(ad, lists, counts, side)) != hipSuccess) ||
          (e = launch_velocity(av, lists, counts, 0, s)) != hipSuccess ||
          (e = launch_velocity(av, lists, counts, 1, s)) != hipSuccess ||
          (e = link(side, s, pl->join)) != hipSuccess ||
          (e = link(s, side, pl->fork)) != hipSuccess ||
          (e = launch_stress(as, lists, counts, 0, side)) != hipSuccess ||
          (e = launch_stress(as, lists, counts, 1, s)) != hipSuccess ||
          (e = link(side, s, pl->join)) != hipSuccess)
        return hip_fail(e, "step launch");
      for (int f = 0; f < kNOut; ++f) std::swap(cur[f], nxt[f]);
      continue;
    }
    // order: both velocity kernels and the fused step (all read only cur),
    // then the stress kernels (they read the new velocity of every tile)
    static const int order[kStepKernels] = {0, 1, 4, 2, 3};
    for (int qi = 0; qi < kStepKernels; ++qi) {
      const int q = order[qi];
      if (ev) (void)hipEventRecord(ev[2 * (kStepKernels * n + q)], s);
      if (q < 2) e = launch_velocity(av, lists, counts, q, s);
      else if (q < 4) e = launch_stress(as, lists, counts, q - 2, s);
      else if (pl->deep) e = launch_deep(ad, lists, counts, s);
      if (e != hipSuccess) return hip_fail(e, "step launch");
      if (ev) (void)hipEventRecord(ev[2 * (kStepKernels * n + q) + 1], s);
    }
    for (int f = 0; f < kNOut; ++f) std::swap(cur[f], nxt[f]);
    if (rec && n >= p.n_steps - pl->nt) {
      const double t = (n + 0.5) * pl->dt, w = 2.0 / pl->nt;
      if ((e = launch_record_plane(cur[VZ], pl->g.off(0, 0, rec->k_rec), pl->g.pitch, p.nx, p.ny,
                                   (float)(w * std::cos(pl->omega * t)),
                                   (float)(-w * std::sin(pl->omega * t)), rec->phasor, s)) !=
          hipSuccess)
        return hip_fail(e, "phasor record");
    }
  }
  return BBFD_OK;
}

int enqueue_solve(const bbfd_plan *pl, const uint8_t *mat, const float *src, float *peak,
                  char *ws, hipStream_t s, hipEvent_t *ev = nullptr, hipStream_t side = nullptr,
                  bool pinned = true, const Record *rec = nullptr) {
  const bbfd_problem &p = pl->prob;
  int rc = enqueue_prologue(pl, mat, peak, ws, s, pinned);
  if (rc) return rc;
  if (rec && !rec->accumulate) {
    hipError_t e = launch_fill((float *)rec->phasor, 2LL * p.nx * p.ny, 0.f, s);
    if (e != hipSuccess) return hip_fail(e, "phasor clear");
  }
  if ((rc = enqueue_steps(pl, mat, src, peak, ws, s, 0, p.n_steps, ev, side, rec))) return rc;
  return enqueue_epilogue(pl, peak, ws, s);
}

// The second branch of captured steps (stream and fork/join events), made at
// the first capture, under the plan's mutex.
int ensure_branch(bbfd_plan *pl) {
  hipError_t e;
  if (!pl->side_stream &&
      (e = hipStreamCreateWithFlags(&pl->side_stream, hipStreamNonBlocking)) != hipSuccess)
    return hip_fail(e, "capture stream");
  if (!pl->fork && (e = hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming)) != hipSuccess)
    return hip_fail(e, "capture event");
  if (!pl->join && (e = hipEventCreateWithFlags(&pl->join, hipEventDisableTiming)) != hipSuccess)
    return hip_fail(e, "capture event");
  return BBFD_OK;
}

// Waits for the last launch of a cached graph, then frees it.
void release_graph(bbfd_plan::Captured &c) {
  if (c.done) {
    (void)hipEventSynchronize(c.done);
    (void)hipEventDestroy(c.done);
  }
  if (c.exec) (void)hipGraphExecDestroy(c.exec);
  if (c.graph) (void)hipGraphDestroy(c.graph);
  c = bbfd_plan::Captured{};
}

int check_solve_args(const bbfd_plan *pl, const uint8_t *mat, const float *src, float *peak,
                     void *ws, uint64_t bytes) {
  if (!pl) return fail(BBFD_EINVAL, "null plan");
  if (!mat || !src || !peak) return fail(BBFD_EINVAL, "null device pointer");
  return check_ws(pl, ws, bytes);
}

// Ring decomposition of the radiating surface (Section 2.3): rings no wider
// than lambda/4, each split into the fewest equal elements of area at most
// lambda^2/16.  e1 is e_x projected off the axis (e_y when the axis lies within
// ~26 degrees of x); e2 = axis x e1.
int make_elements(const bbfd_transducer *t, double freq, std::vector<double> &out) {
  if (!t) return fail(BBFD_EINVAL, "null transducer");
  if (!(t->radius_m > 0)) return fail(BBFD_EINVAL, "transducer radius must be positive");
  double ax[3] = {t->axis[0], t->axis[1], t->axis[2]};
  const double an = std::sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
  if (!(an > 0)) return fail(BBFD_EINVAL, "zero transducer axis");
  for (double &v : ax) v /= an;
  double ref[3] = {1.0, 0.0, 0.0};
  if (std::fabs(ax[0]) >= 0.9) { ref[0] = 0.0; ref[1] = 1.0; }
  const double dr = ref[0] * ax[0] + ref[1] * ax[1] + ref[2] * ax[2];
  double e1[3], e2[3];
  for (int a = 0; a < 3; ++a) e1[a] = ref[a] - dr * ax[a];
  const double n1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  for (double &v : e1) v /= n1;
  e2[0] = ax[1] * e1[2] - ax[2] * e1[1];
  e2[1] = ax[2] * e1[0] - ax[0] * e1[2];
  e2[2] = ax[0] * e1[1] - ax[1] * e1[0];
  const double lam = kCw / freq;
  const double area_max = lam * lam / 16.0, width = lam / 4.0;
  out.clear();
  auto push = [&](const double p[3], double area) {
    out.push_back(p[0]); out.push_back(p[1]); out.push_back(p[2]); out.push_back(area);
  };
  if (t->kind == 0) {
    const int nr = (int)std::ceil(t->radius_m / width);
    const double dr_ = t->radius_m / nr;
    for (int r = 0; r < nr; ++r) {
      const double r0 = r * dr_, r1 = (r + 1) * dr_, rm = 0.5 * (r0 + r1);
      const double ring = kPi * (r1 * r1 - r0 * r0);
      const long nphi = std::max(1L, (long)std::ceil(ring / area_max));
      for (long q = 0; q < nphi; ++q) {
        const double ph = 2.0 * kPi * (q + 0.5) / nphi, c = std::cos(ph), s = std::sin(ph);
        double p[3];
        for (int a = 0; a < 3; ++a) p[a] = t->apex_m[a] + rm * (c * e1[a] + s * e2[a]);
        push(p, ring / nphi);
      }
    }
  } else if (t->kind == 1) {
    const double F = t->focal_m;
    if (!(F >= t->radius_m)) return fail(BBFD_EINVAL, "bowl aperture radius exceeds its curvature radius");
    const double thmax = std::asin(t->radius_m / F);
    const int nr = (int)std::ceil(F * thmax / width);
    const double dth = thmax / nr;
    double focus[3];
    for (int a = 0; a < 3; ++a) focus[a] = t->apex_m[a] + F * ax[a];
    for (int r = 0; r < nr; ++r) {
      const double t0 = r * dth, t1 = (r + 1) * dth, tm = 0.5 * (t0 + t1);
      const double ring = 2.0 * kPi * F * F * (std::cos(t0) - std::cos(t1));
      const long nphi = std::max(1L, (long)std::ceil(ring / area_max));
      const double ct = std::cos(tm), st = std::sin(tm);
      for (long q = 0; q < nphi; ++q) {
        const double ph = 2.0 * kPi * (q + 0.5) / nphi, c = std::cos(ph), s = std::sin(ph);
        double p[3];
        for (int a = 0; a < 3; ++a) p[a] = focus[a] + F * (-ct * ax[a] + st * (c * e1[a] + s * e2[a]));
        push(p, ring / nphi);
      }
    }
  } else {
    return fail(BBFD_EINVAL, "unknown transducer kind %d", t->kind);
  }
  return BBFD_OK;
}

}  // namespace

extern "C" {

const char *bbfd_last_error(void) { return g_err.c_str(); }

int bbfd_plan_create(const bbfd_problem *problem, bbfd_plan **out) {
  if (!out) return fail(BBFD_EINVAL, "null output pointer");
  *out = nullptr;
  bbfd_plan *pl = new (std::nothrow) bbfd_plan();
  if (!pl) return fail(BBFD_EINVAL, "out of host memory");
  int rc = validate_and_derive(problem, pl);
  if (rc == BBFD_OK) rc = build_tables(pl);
  if (rc != BBFD_OK) {
    bbfd_plan_destroy(pl);
    return rc;
  }
  layout(pl);
  // the step kernels address every array by 32-bit byte offsets
  const uint64_t cells = (uint64_t)problem->nx * problem->ny * problem->nz;
  if ((uint64_t)pl->g.stride * sizeof(float) > 0xffffffffull ||
      cells * sizeof(float) > 0xffffffffull) {
    bbfd_plan_destroy(pl);
    return fail(BBFD_EINVAL, "grid of %llu cells exceeds the 4 GiB per-array limit of the step kernels",
                (unsigned long long)cells);
  }
  *out = pl;
  return BBFD_OK;
}

void bbfd_plan_destroy(bbfd_plan *pl) {
  if (!pl) return;
  for (auto &c : pl->graphs) release_graph(c);
  if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
  if (pl->side_stream) (void)hipStreamDestroy(pl->side_stream);
  if (pl->fork) (void)hipEventDestroy(pl->fork);
  if (pl->join) (void)hipEventDestroy(pl->join);
  if (pl->h_lut) (void)hipHostFree(pl->h_lut);
  if (pl->h_pml) (void)hipHostFree(pl->h_pml);
  delete pl;
}

int bbfd_plan_get_info(const bbfd_plan *pl, bbfd_plan_info *out) {
  if (!pl || !out) return fail(BBFD_EINVAL, "null argument");
  out->dx = pl->dx;
  out->dt = pl->dt;
  out->c_max = pl->cmax;
  out->steps_per_period = pl->nt;
  out->capture_start = pl->cap;
  out->source_k = pl->ks;
  out->pitch = pl->g.pitch;
  out->workspace_bytes = pl->ws_bytes;
  out->cells = (uint64_t)pl->prob.nx * pl->prob.ny * pl->prob.nz;
  out->tile_rows = kRows;
  out->tile_planes = pl->kchunk;
  out->graph_captures = pl->captures;
  return BBFD_OK;
}

int bbfd_material_constants(const bbfd_plan *pl, double *out, int32_t n_rows) {
  if (!pl || !out) return fail(BBFD_EINVAL, "null argument");
  if (n_rows < pl->prob.n_materials) return fail(BBFD_EINVAL, "need %d rows", pl->prob.n_materials);
  std::memcpy(out, pl->consts.data(), pl->consts.size() * sizeof(double));
  return BBFD_OK;
}

int bbfd_transducer_elements(const bbfd_plan *pl, const bbfd_transducer *t, double *xyza,
                             int64_t cap, int64_t *n_out) {
  if (!pl || !n_out) return fail(BBFD_EINVAL, "null argument");
  std::vector<double> el;
  int rc = make_elements(t, pl->prob.freq_hz, el);
  if (rc) return rc;
  const int64_t n = (int64_t)(el.size() / 4);
  *n_out = n;
  if (xyza) std::memcpy(xyza, el.data(), (size_t)std::min(n, cap) * 4 * sizeof(double));
  return BBFD_OK;
}

// Elements of t staged in the workspace, then the Rayleigh sum on `planes`
// planes starting at z0 (cell-centre x, y).
static int rayleigh_planes(const bbfd_plan *pl, const bbfd_transducer *t, float *out,
                           void *workspace, uint64_t bytes, void *stream, int planes, double z0,
                           double z_limit) {
  if (!pl || !out) return fail(BBFD_EINVAL, "null argument");
  int rc = check_ws(pl, workspace, bytes);
  if (rc) return rc;
  std::vector<double> el;
  if ((rc = make_elements(t, pl->prob.freq_hz, el))) return rc;
  const size_t n = el.size() / 4;
  for (size_t e = 0; e < n; ++e)
    if (!(el[4 * e + 2] < z_limit))
      return fail(BBFD_EGEOMETRY, "transducer element %zu at z %.4g m is not before the source plane (%.4g m)",
                  e, el[4 * e + 2], z_limit);
  const size_t need = n * sizeof(double4);
  if (need > (size_t)kNState * pl->g.stride * sizeof(float))
    return fail(BBFD_ENOMEM, "too many elements (%zu) for the workspace", n);
  hipStream_t s = (hipStream_t)stream;
  char *ws = (char *)workspace;
  hipError_t e = hipMemcpyAsync(ws + pl->off_state, el.data(), need, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "element upload");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "element upload sync");
  const double kw = pl->omega / kCw;
  const double pre = pl->omega * kRhoW * t->u0 / (2.0 * kPi);
  e = launch_rayleigh((const double4 *)(ws + pl->off_state), (int)n, pl->prob.nx, pl->prob.ny,
                      planes, pl->dx, z0, kw, pre, (float2 *)out, s);
  if (e != hipSuccess) return hip_fail(e, "rayleigh launch");
  return BBFD_OK;
}

int bbfd_source_rayleigh(const bbfd_plan *pl, const bbfd_transducer *t, float *src,
                         void *workspace, uint64_t bytes, void *stream) {
  if (!pl) return fail(BBFD_EINVAL, "null plan");
  return rayleigh_planes(pl, t, src, workspace, bytes, stream, 1, (pl->ks + 0.5) * pl->dx,
                         pl->ks * pl->dx);
}

int bbfd_rayleigh_volume(const bbfd_plan *pl, const bbfd_transducer *t, float *field,
                         void *workspace, uint64_t bytes, void *stream) {
  if (!pl) return fail(BBFD_EINVAL, "null plan");
  return rayleigh_planes(pl, t, field, workspace, bytes, stream, pl->prob.nz, 0.0,
                         pl->ks * pl->dx);
}

// ---------------------------------------------------------- phased arrays
// Every element of an array is a flat circular piston decomposed like the
// single piston (rings no wider than lambda/4, equal parts of at most
// lambda^2/16); its sub-elements carry the element's complex drive.
static int array_subelements(const bbfd_plan *pl, const bbfd_element *el, int32_t n,
                             std::vector<double> &xyza, std::vector<double> &w) {
  if (!pl) return fail(BBFD_EINVAL, "null plan");
  if (!el || n < 1) return fail(BBFD_EINVAL, "need at least one array element");
  xyza.clear();
  w.clear();
  for (int e = 0; e < n; ++e) {
    bbfd_transducer t{};
    t.kind = 0;
    t.radius_m = el[e].radius_m;
    for (int a = 0; a < 3; ++a) {
      t.apex_m[a] = el[e].centre_m[a];
      t.axis[a] = el[e].axis[a];
    }
    t.u0 = 1.0;
    std::vector<double> sub;
    int rc = make_elements(&t, pl->prob.freq_hz, sub);
    if (rc) {
      std::string msg = g_err;
      return fail(rc, "array element %d: %s", e, msg.c_str());
    }
    xyza.insert(xyza.end(), sub.begin(), sub.end());
    for (size_t q = 0; q < sub.size() / 4; ++q) {
      w.push_back(el[e].w_re);
      w.push_back(el[e].w_im);
    }
  }
  return BBFD_OK;
}

int bbfd_array_elements(const bbfd_plan *pl, const bbfd_element *el, int32_t n, double *out,
                        int64_t cap, int64_t *n_out) {
  if (!n_out) return fail(BBFD_EINVAL, "null count output");
  std::vector<double> xyza, w;
  int rc = array_subelements(pl, el, n, xyza, w);
  if (rc) return rc;
  const int64_t m = (int64_t)(xyza.size() / 4);
  *n_out = m;
  if (out)
    for (int64_t q = 0; q < std::min(m, cap); ++q) {
      for (int a = 0; a < 4; ++a) out[6 * q + a] = xyza[4 * q + a];
      out[6 * q + 4] = w[2 * q];
      out[6 * q + 5] = w[2 * q + 1];
    }
  return BBFD_OK;
}

int bbfd_array_rayleigh(const bbfd_plan *pl, const bbfd_element *el, int32_t n, float *src,
                        void *workspace, uint64_t bytes, void *stream) {
  if (!pl || !src) return fail(BBFD_EINVAL, "null argument");
  int rc = check_ws(pl, workspace, bytes);
  if (rc) return rc;
  std::vector<double> xyza, w;
  if ((rc = array_subelements(pl, el, n, xyza, w))) return rc;
  const size_t m = xyza.size() / 4;
  const double zs = pl->ks * pl->dx;
  for (size_t q = 0; q < m; ++q)
    if (!(xyza[4 * q + 2] < zs))
      return fail(BBFD_EGEOMETRY, "array sub-element %zu at z %.4g m is not before the source plane (%.4g m)",
                  q, xyza[4 * q + 2], zs);
  const size_t need = m * (sizeof(double4) + sizeof(double2));
  if (need > (size_t)kNState * pl->g.stride * sizeof(float))
    return fail(BBFD_ENOMEM, "too many array sub-elements (%zu) for the workspace", m);
  hipStream_t s = (hipStream_t)stream;
  char *ws = (char *)workspace;
  double4 *del = (double4 *)(ws + pl->off_state);
  double2 *dw = (double2 *)(ws + pl->off_state + m * sizeof(double4));
  hipError_t e;
  if ((e = hipMemcpyAsync(del, xyza.data(), m * sizeof(double4), hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(dw, w.data(), m * sizeof(double2), hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_fail(e, "array element upload");
  const double kw = pl->omega / kCw, pre = pl->omega * kRhoW / (2.0 * kPi);
  if ((e = launch_rayleigh(del, (int)m, pl->prob.nx, pl->prob.ny, 1, pl->dx, (pl->ks + 0.5) * pl->dx, kw,
                           pre, (float2 *)src, s, dw)) != hipSuccess)
    return hip_fail(e, "array rayleigh launch");
  return BBFD_OK;
}

int bbfd_array_steer(const bbfd_plan *pl, const bbfd_element *el, int32_t n, const double *target,
                     double *w) {
  if (!pl || !el || n < 1 || !target || !w) return fail(BBFD_EINVAL, "null or empty argument");
  const double k = pl->omega / kCw;
  for (int e = 0; e < n; ++e) {
    double r2 = 0.0;
    for (int a = 0; a < 3; ++a) r2 += (el[e].centre_m[a] - target[a]) * (el[e].centre_m[a] - target[a]);
    const double ph = k * std::sqrt(r2);
    w[2 * e] = std::cos(ph);
    w[2 * e + 1] = std::sin(ph);
  }
  return BBFD_OK;
}

int bbfd_array_refocus(const bbfd_plan *cpl, const uint8_t *mat, const bbfd_element *el, int32_t n,
                       const int32_t *cell, float *peak, double *w, double *field,
                       void *workspace, uint64_t bytes, void *stream) {
  int rc = check_solve_args(cpl, mat, (const float *)mat, peak, workspace, bytes);
  if (rc) return rc;
  if (!el || n < 1 || !cell || !w) return fail(BBFD_EINVAL, "null or empty argument");
  bbfd_plan *pl = const_cast<bbfd_plan *>(cpl);
  const bbfd_problem &p = pl->prob;
  const int it = cell[0], jt = cell[1], kt = cell[2];
  if (it < p.pml || it >= p.nx - p.pml || jt < p.pml || jt >= p.ny - p.pml || kt <= pl->ks + 1 ||
      kt >= p.nz - p.pml)
    return fail(BBFD_EINVAL,
                "target cell (%d, %d, %d) must lie in the interior, two planes beyond the source plane",
                it, jt, kt);
  {
    std::lock_guard<std::mutex> lock(pl->mu);
    if ((rc = ensure_pinned(pl))) return rc;
  }
  hipStream_t s = (hipStream_t)stream;
  char *ws = (char *)workspace;
  float2 *point = (float2 *)(ws + pl->off_aux);
  float2 *ph = point + (size_t)p.nx * p.ny;
  hipError_t e;
  // the point source: unit z forces pushing outward on the two v_z faces of
  // the target cell, +1 on the face above it (plane kt) and -1 on the face
  // below (plane kt - 1), recorded by two solves into one phasor (the record
  // is linear in the source)
  if ((e = launch_fill((float *)point, 2LL * p.nx * p.ny, 0.f, s)) != hipSuccess ||
      (e = launch_fill((float *)(point + (size_t)jt * p.nx + it), 1, 1.f, s)) != hipSuccess)
    return hip_fail(e, "point source");
  Record rec{kt, pl->ks, ph};
  if ((rc = enqueue_solve(pl, mat, (const float *)point, peak, ws, s, nullptr, nullptr, true, &rec)))
    return rc;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "record solve");
  if ((rc = bbfd_status(pl, ws, nullptr, nullptr, stream))) return rc;
  if ((e = launch_fill((float *)(point + (size_t)jt * p.nx + it), 1, -1.f, s)) != hipSuccess)
    return hip_fail(e, "point source");
  Record below{kt - 1, pl->ks, ph, true};
  if ((rc = enqueue_solve(pl, mat, (const float *)point, peak, ws, s, nullptr, nullptr, true, &below)))
    return rc;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "record solve");
  if ((rc = bbfd_status(pl, ws, nullptr, nullptr, stream))) return rc;
  // back-propagate the recorded plane to the element centres (Rayleigh)
  const size_t need = (size_t)n * sizeof(double4) + (size_t)backprop_partials(n) * sizeof(double2) +
                      (size_t)n * sizeof(double2);
  if (need > (size_t)kNState * pl->g.stride * sizeof(float))
    return fail(BBFD_ENOMEM, "too many array elements (%d) for the workspace", n);
  std::vector<double> pts(4 * (size_t)n, 0.0);
  for (int q = 0; q < n; ++q)
    for (int a = 0; a < 3; ++a) pts[4 * q + a] = el[q].centre_m[a];
  double4 *dpts = (double4 *)(ws + pl->off_state);
  double2 *part = (double2 *)(dpts + n);
  double2 *out = part + backprop_partials(n);
  std::vector<double> pe(2 * (size_t)n);
  const double kw = pl->omega / kCw, pre = pl->omega * kRhoW * pl->dx * pl->dx / (2.0 * kPi);
  if ((e = hipMemcpyAsync(dpts, pts.data(), pts.size() * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess ||
      (e = launch_backprop(ph, p.nx, p.ny, pl->dx, (pl->ks + 0.5) * pl->dx, dpts, n, kw, pre, part, out,
                           s)) != hipSuccess ||
      (e = hipMemcpyAsync(pe.data(), out, pe.size() * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_fail(e, "back-propagation");
  for (int q = 0; q < n; ++q) {
    const double re = pe[2 * q], im = pe[2 * q + 1], a = std::hypot(re, im);
    w[2 * q] = a > 0 ? re / a : 0.0;          // phase conjugation: exp(-i arg p_e)
    w[2 * q + 1] = a > 0 ? -im / a : 0.0;
    if (field) {
      field[2 * q] = re;
      field[2 * q + 1] = im;
    }
  }
  return BBFD_OK;
}

int bbfd_solve_direct(const bbfd_plan *cpl, const uint8_t *mat, const float *src, float *peak,
                      void *workspace, uint64_t bytes, void *stream) {
  int rc = check_solve_args(cpl, mat, src, peak, workspace, bytes);
  if (rc) return rc;
  bbfd_plan *pl = const_cast<bbfd_plan *>(cpl);  // pinned staging only
  {
    std::lock_guard<std::mutex> lock(pl->mu);
    if ((rc = ensure_pinned(pl))) return rc;
  }
  return enqueue_solve(pl, mat, src, peak, (char *)workspace, (hipStream_t)stream);
}

int bbfd_solve_profiled(const bbfd_plan *cpl, const uint8_t *mat, const float *src, float *peak,
                        void *workspace, uint64_t bytes, void *stream, double *ms_out) {
  int rc = check_solve_args(cpl, mat, src, peak, workspace, bytes);
  if (rc) return rc;
  if (!ms_out) return fail(BBFD_EINVAL, "null timing output");
  bbfd_plan *pl = const_cast<bbfd_plan *>(cpl);
  {
    std::lock_guard<std::mutex> lock(pl->mu);
    if ((rc = ensure_pinned(pl))) return rc;
  }
  const int n = pl->prob.n_steps;
  std::vector<hipEvent_t> ev(2 * kStepKernels * (size_t)n, nullptr);
  hipError_t e = hipSuccess;
  for (auto &x : ev)
    if ((e = hipEventCreate(&x)) != hipSuccess) break;
  if (e == hipSuccess) {
    hipStream_t s = (hipStream_t)stream;
    rc = enqueue_solve(pl, mat, src, peak, (char *)workspace, s, ev.data());
    if (rc == BBFD_OK && (e = hipStreamSynchronize(s)) != hipSuccess)
      rc = hip_fail(e, "profiled solve sync");
    double t[kStepKernels] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int k = 0; rc == BBFD_OK && k < kStepKernels * n; ++k) {
      float a = 0.f;
      if (hipEventElapsedTime(&a, ev[2 * k], ev[2 * k + 1]) != hipSuccess) {
        rc = fail(BBFD_EHIP, "event timing");
        break;
      }
      t[k % kStepKernels] += a;
    }
    for (int q = 0; q < kStepKernels; ++q) ms_out[q] = t[q];
  } else {
    rc = hip_fail(e, "event create");
  }
  for (auto &x : ev)
    if (x) (void)hipEventDestroy(x);
  return rc;
}

int bbfd_solve(const bbfd_plan *cpl, const uint8_t *mat, const float *src, float *peak,
               void *workspace, uint64_t bytes, void *stream) {
  int rc = check_solve_args(cpl, mat, src, peak, workspace, bytes);
  if (rc) return rc;
  bbfd_plan *pl = const_cast<bbfd_plan *>(cpl);  // graph cache only
  std::lock_guard<std::mutex> lock(pl->mu);
  if ((rc = ensure_pinned(pl))) return rc;
  const void *key[4] = {mat, src, peak, workspace};
  bbfd_plan::Captured *hit = nullptr;
  for (auto &c : pl->graphs)
    if (std::memcmp(key, c.key, sizeof key) == 0) hit = &c;
  if (!hit) {
    hipError_t e;
    if (!pl->cap_stream &&
        (e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking)) != hipSuccess)
      return hip_fail(e, "capture stream");
    if ((rc = ensure_branch(pl))) return rc;
    if (pl->graphs.size() >= (size_t)kGraphCache) {  // replace the least recently used
      size_t lru = 0;
      for (size_t q = 1; q < pl->graphs.size(); ++q)
        if (pl->graphs[q].used < pl->graphs[lru].used) lru = q;
      release_graph(pl->graphs[lru]);
      pl->graphs.erase(pl->graphs.begin() + (long)lru);
    }
    bbfd_plan::Captured c{};
    std::memcpy(c.key, key, sizeof key);
    if ((e = hipEventCreateWithFlags(&c.done, hipEventDisableTiming)) != hipSuccess)
      return hip_fail(e, "graph event");
    if ((e = hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
      release_graph(c);
      return hip_fail(e, "begin capture");
    }
    rc = enqueue_solve(pl, mat, src, peak, (char *)workspace, pl->cap_stream, nullptr,
                       pl->branch ? pl->side_stream : nullptr);
    e = hipStreamEndCapture(pl->cap_stream, &c.graph);
    if (rc || e != hipSuccess) {
      release_graph(c);
      return rc ? rc : hip_fail(e, "end capture");
    }
    if ((e = hipGraphInstantiate(&c.exec, c.graph, nullptr, nullptr, 0)) != hipSuccess) {
      c.exec = nullptr;
      release_graph(c);
      return hip_fail(e, "graph instantiate");
    }
    ++pl->captures;
    pl->graphs.push_back(c);
    hit = &pl->graphs.back();
  }
  hit->used = ++pl->clock;
  hipError_t e = hipGraphLaunch(hit->exec, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  if ((e = hipEventRecord(hit->done, (hipStream_t)stream)) != hipSuccess)
    return hip_fail(e, "graph event record");
  return BBFD_OK;
}

// ------------------------------------------------ solve without allocation
// Device memory of bbfd_solve_static: one file-scope array per GPU, holding
// the whole workspace of a solve (state, tables, classes, status).  Host code
// never uses the array's name as an address: its device address is looked up
// once per device (with that device current) and kept in g_scratch_ptr.
constexpr size_t kScratchBytes = (size_t)96 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static void *g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

static int scratch_address(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "current device");
  if (dev < 0 || dev >= kMaxDevices) return fail(BBFD_EINVAL, "device %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess)
      return hip_fail(e, "scratch symbol address");
    if (!p || (uintptr_t)p % 256) return fail(BBFD_EHIP, "scratch array misplaced");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return BBFD_OK;
}

int bbfd_solve_static(const bbfd_plan *pl, const uint8_t *mat, const float *src, float *peak,
                      void *stream, int64_t *peak_index, float *peak_value) {
  if (!pl) return fail(BBFD_EINVAL, "null plan");
  if (!mat || !src || !peak) return fail(BBFD_EINVAL, "null device pointer");
  if (pl->ws_bytes > kScratchBytes)
    return fail(BBFD_ENOMEM,
                "solve needs %llu bytes of device workspace; bbfd_solve_static holds at most %llu "
                "(use bbfd_solve with a caller workspace)",
                (unsigned long long)pl->ws_bytes, (unsigned long long)kScratchBytes);
  void *ws = nullptr;
  int rc = scratch_address(&ws);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if ((rc = enqueue_solve(pl, mat, src, peak, (char *)ws, s, nullptr, nullptr, false))) return rc;
  if (peak_index || peak_value) return bbfd_status(pl, ws, peak_index, peak_value, stream);
  return BBFD_OK;
}

int bbfd_energy_loss(const bbfd_plan *pl, const uint8_t *mat_skull, const float *peak_skull,
                     const uint8_t *mat_water, const float *peak_water, int32_t z_m,
                     void *workspace, uint64_t bytes, void *stream, double *out) {
  if (!pl || !out) return fail(BBFD_EINVAL, "null argument");
  if (!mat_skull || !peak_skull || !mat_water || !peak_water)
    return fail(BBFD_EINVAL, "null device pointer");
  int rc = check_ws(pl, workspace, bytes);
  if (rc) return rc;
  const bbfd_problem &p = pl->prob;
  if (z_m >= 0 && (z_m < p.pml || z_m >= p.nz - p.pml))
    return fail(BBFD_EINVAL, "plane %d outside the interior [%d, %d)", z_m, p.pml, p.nz - p.pml);
  hipStream_t s = (hipStream_t)stream;
  char *ws = (char *)workspace;
  Status *st = (Status *)(ws + pl->off_energy);
  double *res = (double *)(ws + pl->off_energy + 256);
  double2 *part = (double2 *)(ws + pl->off_energy + 512);
  double *iz = (double *)(ws + pl->off_energy + 512 + (size_t)energy_partials() * 16);
  hipError_t e;
  if ((e = hipMemcpyAsync(iz, pl->inv_z.data(), pl->inv_z.size() * sizeof(double),
                          hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_fail(e, "impedance table upload");
  if (z_m < 0) {  // plane of the water-only map's peak voxel
    if ((e = launch_fill((float *)st, 256 / sizeof(float), 0.f, s)) != hipSuccess ||
        (e = launch_argmax(peak_water, p.nx, p.ny, p.nz, p.pml, (float *)(ws + pl->off_pv),
                           (long long *)(ws + pl->off_pi), st, s)) != hipSuccess)
      return hip_fail(e, "water peak voxel");
  }
  if ((e = launch_plane_energy(mat_skull, peak_skull, mat_water, peak_water, p.nx, p.ny, p.pml, z_m,
                               st, iz, p.n_materials, p.index_bits == 16 ? 1 : 0, part, res,
                               s)) != hipSuccess)
    return hip_fail(e, "plane energy launch");
  double h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int nd = energy_out_doubles();
  if ((e = hipMemcpyAsync(h, res, (size_t)nd * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_fail(e, "energy read");
  for (int q = 0; q < 5; ++q) out[q] = h[q];
  if (!(h[4] > 0.0) || !std::isfinite(h[3]) || !std::isfinite(h[4]))
    return fail(BBFD_EDIVERGED, "water-only plane sum %g is not positive and finite", h[4]);
  return BBFD_OK;
}

int bbfd_status(const bbfd_plan *pl, const void *workspace, int64_t *peak_index,
                float *peak_value, void *stream) {
  if (!pl || !workspace) return fail(BBFD_EINVAL, "null argument");
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "stream sync");
  Status st{};
  e = hipMemcpy(&st, (const char *)workspace + pl->off_status, sizeof st, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "status read");
  if (peak_index) *peak_index = st.peak_index;
  if (peak_value) *peak_value = st.peak_value;
  if (st.flags & kStatusIndex) return fail(BBFD_EINDEX, "material index >= n_materials in the map");
  if (st.flags & kStatusDiverged) return fail(BBFD_EDIVERGED, "non-finite peak pressure (diverged)");
  return BBFD_OK;
}

int bbfd_tile_counts(const bbfd_plan *pl, const void *workspace, int32_t *counts, void *stream) {
  if (!pl || !workspace || !counts) return fail(BBFD_EINVAL, "null argument");
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "stream sync");
  int c[3] = {0, 0, 0};
  e = hipMemcpy(c, (const char *)workspace + pl->off_counts, sizeof c, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "tile count read");
  for (int q = 0; q < 3; ++q) counts[q] = c[q];
  return BBFD_OK;
}

int bbfd_segment_classes(const bbfd_plan *pl, const void *workspace, uint8_t *classes,
                         uint64_t n, void *stream) {
  if (!pl || !workspace || !classes) return fail(BBFD_EINVAL, "null argument");
  const int nx = pl->nseg, ny = pl->g.ny, nz = pl->g.nz, kp = pl->kpad;
  if (n < (uint64_t)nx * ny * nz) return fail(BBFD_EINVAL, "classes buffer holds fewer than nseg*ny*nz bytes");
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "stream sync");
  std::vector<uint8_t> col((size_t)nx * ny * kp);  // device layout: [ny][nseg][kpad]
  e = hipMemcpy(col.data(), (const char *)workspace + pl->off_cls, col.size(), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "class read");
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int sg = 0; sg < nx; ++sg)
        classes[((size_t)k * ny + j) * nx + sg] = col[((size_t)j * nx + sg) * kp + k];
  return BBFD_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches

struct bbfd_batch {
  std::vector<bbfd_plan *> plans;
  std::vector<int> order;       // solves by decreasing step count
  std::vector<size_t> sub_off;  // per-solve workspace offset
  size_t off_desc = 0, off_tiles = 0, off_coef = 0, off_cap = 0, off_tab = 0, off_scan = 0,
         off_len = 0, off_end = 0, ws_bytes = 0;
  int max_steps = 0;
  size_t max_tiles = 0;         // capacity of the tile table region
  // launch shape (autotuned): rows per block, persistent blocks, z cells per
  // tile; by = 0 runs every solve with its own step kernels instead (the
  // per-solve shape, blocks = kchunk = 0)
  int by = 4, blocks = 1024, kchunk = 16;
  int max_mat = 1;              // largest material table (LDS staging size)
  std::vector<BatchTile> tiles;
  std::vector<int> solve_end;   // end of each solve's tiles in the table (solve order)
  std::vector<int> live_solves; // solves still running at each step (a prefix of the order)
  StepArgs *h_desc = nullptr;   // pinned staging, made at the first solve
  BatchTile *h_tiles = nullptr;
  float2 *h_coef = nullptr;
  int *h_cap = nullptr;
  int *h_end = nullptr;
  // Recorded after every enqueue that reads the pinned staging above (graph
  // launches included: their table uploads read it when they execute).  The
  // staging is rewritten, and a graph destroyed, only once it has completed.
  hipEvent_t staged = nullptr;
  std::mutex mu;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const void *> key;
  int key_shape[3] = {0, 0, 0};
};

namespace {

// z cells per tile for a solve: the shape's kchunk, capped at nz.
void build_tiles(bbfd_batch *b) {
  b->tiles.clear();
  b->solve_end.clear();
  b->live_solves.clear();
  if (b->by == 0) return;  // the per-solve shape walks no table
  for (int s : b->order) {
    const bbfd_problem &p = b->plans[s]->prob;
    const int kc = std::max(1, std::min(b->kchunk, p.nz));
    const int nbx = (p.nx + kSeg - 1) / kSeg, nby = (p.ny + b->by - 1) / b->by;
    for (int k0 = 0; k0 < p.nz; k0 += kc)
      for (int y = 0; y < nby; ++y)
        for (int x = 0; x < nbx; ++x) {
          BatchTile t{};
          t.solve = s;
          t.bx = x;
          t.by = y;
          t.k0 = k0;
          t.k1 = std::min(k0 + kc, p.nz);
          b->tiles.push_back(t);
        }
    b->solve_end.push_back((int)b->tiles.size());
  }
  b->live_solves.assign(b->max_steps, 0);
  for (int n = 0; n < b->max_steps; ++n) {
    int live = 0;
    for (size_t q = 0; q < b->order.size(); ++q)
      if (b->plans[b->order[q]]->prob.n_steps > n) live = (int)q + 1;
    b->live_solves[n] = live;
  }
}

size_t tiles_capacity(const bbfd_batch *b) {
  // the finest shape the tuner tries (1 row, 4 planes) bounds the table size
  size_t n = 0;
  for (const bbfd_plan *pl : b->plans) {
    const bbfd_problem &p = pl->prob;
    n += (size_t)((p.nx + kSeg - 1) / kSeg) * p.ny * ((p.nz + 3) / 4);
  }
  return n;
}

int batch_pinned(bbfd_batch *b) {
  if (b->h_desc) return BBFD_OK;
  const size_t n = b->plans.size();
  hipError_t e;
  if ((e = hipHostMalloc((void **)&b->h_desc, n * sizeof(StepArgs), hipHostMallocDefault)) != hipSuccess)
    return hip_fail(e, "pinned descriptor allocation");
  if ((e = hipHostMalloc((void **)&b->h_tiles, b->max_tiles * sizeof(BatchTile), hipHostMallocDefault)) !=
      hipSuccess)
    return hip_fail(e, "pinned tile-table allocation");
  if ((e = hipHostMalloc((void **)&b->h_coef, n * (size_t)b->max_steps * sizeof(float2),
                         hipHostMallocDefault)) != hipSuccess)
    return hip_fail(e, "pinned coefficient allocation");
  if ((e = hipHostMalloc((void **)&b->h_cap, n * sizeof(int), hipHostMallocDefault)) != hipSuccess)
    return hip_fail(e, "pinned capture allocation");
  if ((e = hipHostMalloc((void **)&b->h_end, n * sizeof(int), hipHostMallocDefault)) != hipSuccess)
    return hip_fail(e, "pinned tile-range allocation");
  if ((e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming)) != hipSuccess)
    return hip_fail(e, "staging event");
  for (size_t s = 0; s < n; ++s) {
    const bbfd_plan *pl = b->plans[s];
    for (int k = 0; k < b->max_steps; ++k) {
      const bool on = k < pl->prob.n_steps;
      b->h_coef[s * b->max_steps + k] = make_float2(on ? pl->src_c[k] : 0.f, on ? pl->src_s[k] : 0.f);
    }
    b->h_cap[s] = pl->cap;
  }
  for (bbfd_plan *pl : b->plans) {
    std::lock_guard<std::mutex> lock(pl->mu);
    int rc = ensure_pinned(pl);
    if (rc) return rc;
  }
  return BBFD_OK;
}

int check_batch_args(const bbfd_batch *b, const uint8_t *const *mat, const float *const *src,
                     float *const *peak, void *ws, uint64_t bytes) {
  if (!b || !mat || !src || !peak) return fail(BBFD_EINVAL, "null argument");
  for (size_t s = 0; s < b->plans.size(); ++s)
    if (!mat[s] || !src[s] || !peak[s]) return fail(BBFD_EINVAL, "null device pointer for solve %zu", s);
  if (!ws) return fail(BBFD_ENOMEM, "null workspace");
  if ((uintptr_t)ws % 256) return fail(BBFD_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < b->ws_bytes)
    return fail(BBFD_ENOMEM, "batch workspace of %llu bytes, need %llu", (unsigned long long)bytes,
                (unsigned long long)b->ws_bytes);
  return BBFD_OK;
}

// Descriptor and table uploads, every solve's prologue, `steps` batched steps
// (all of them when steps < 0), every solve's epilogue (when complete).
// Grid of the batched step kernels: the persistent block count, or (blocks =
// 0) one block per tile of the whole table, an upper bound on either kind's
// live length.
int batch_grid(const bbfd_batch *b) {
  return b->blocks > 0 ? b->blocks : std::max(1, (int)b->tiles.size());
}

// The two walks (acoustic, general) of step k over the per-kind tables.
void batch_walks(const bbfd_batch *b, char *ws, int k, BatchWalk *W) {
  const int *tab = (const int *)(ws + b->off_tab);
  const int *len = (const int *)(ws + b->off_len);
  const size_t n = b->plans.size();
  for (int q = 0; q < 2; ++q) {
    W[q].desc = (const StepArgs *)(ws + b->off_desc);
    W[q].tiles = (const BatchTile *)(ws + b->off_tiles);
    W[q].table = tab + (size_t)q * b->max_tiles;
    W[q].table_len = len + (size_t)q * (n + 1);
    W[q].live = b->live_solves[k];
  }
}

// Blocks until every earlier enqueue that reads the pinned staging has run.
int wait_staging(bbfd_batch *b) {
  if (!b->staged) return BBFD_OK;
  hipError_t e = hipEventSynchronize(b->staged);
  return e == hipSuccess ? BBFD_OK : hip_fail(e, "staging wait");
}

int mark_staging(bbfd_batch *b, hipStream_t s) {
  hipError_t e = hipEventRecord(b->staged, s);
  return e == hipSuccess ? BBFD_OK : hip_fail(e, "staging event record");
}

// The per-solve shape: each solve's prologue, steps (in two branches, as a
// captured single solve) and epilogue, one solve after the other, in the order
// of the problems.  Graph capture only, under the batch's lock.
int enqueue_per_solve(bbfd_batch *b, const uint8_t *const *mat, const float *const *src,
                      float *const *peak, char *ws, hipStream_t s) {
  for (size_t q = 0; q < b->plans.size(); ++q) {
    bbfd_plan *pl = b->plans[q];
    std::lock_guard<std::mutex> lock(pl->mu);
    int rc = ensure_branch(pl);
    if (!rc)
      rc = enqueue_solve(pl, mat[q], src[q], peak[q], ws + b->sub_off[q], s, nullptr,
                         pl->branch ? pl->side_stream : nullptr);
    if (rc) return rc;
  }
  return BBFD_OK;
}

int enqueue_batch(bbfd_batch *b, const uint8_t *const *mat, const float *const *src,
                  float *const *peak, char *ws, hipStream_t s, int steps = -1) {
  const size_t n = b->plans.size();
  if (b->by == 0) return enqueue_per_solve(b, mat, src, peak, ws, s);
  // callers have waited for the staging (drop_graph precedes every capture and
  // every tuning pass)
  for (size_t q = 0; q < n; ++q)
    b->h_desc[q] = step_args(b->plans[q], mat[q], src[q], peak[q], ws + b->sub_off[q]);
  std::copy(b->tiles.begin(), b->tiles.end(), b->h_tiles);
  std::copy(b->solve_end.begin(), b->solve_end.end(), b->h_end);
  hipError_t e;
  if ((e = hipMemcpyAsync(ws + b->off_desc, b->h_desc, n * sizeof(StepArgs), hipMemcpyHostToDevice, s)) ||
      (e = hipMemcpyAsync(ws + b->off_tiles, b->h_tiles, b->tiles.size() * sizeof(BatchTile),
                          hipMemcpyHostToDevice, s)) ||
      (e = hipMemcpyAsync(ws + b->off_coef, b->h_coef, n * (size_t)b->max_steps * sizeof(float2),
                          hipMemcpyHostToDevice, s)) ||
      (e = hipMemcpyAsync(ws + b->off_cap, b->h_cap, n * sizeof(int), hipMemcpyHostToDevice, s)) ||
      (e = hipMemcpyAsync(ws + b->off_end, b->h_end, n * sizeof(int), hipMemcpyHostToDevice, s)))
    return hip_fail(e, "batch table upload");
  for (size_t q = 0; q < n; ++q) {
    int rc = enqueue_prologue(b->plans[q], mat[q], peak[q], ws + b->sub_off[q], s);
    if (rc) return rc;
  }
  if ((e = launch_batch_kinds((const StepArgs *)(ws + b->off_desc), (BatchTile *)(ws + b->off_tiles),
                              (int)b->tiles.size(), b->by, s)) != hipSuccess)
    return hip_fail(e, "batch tile kinds");
  {
    int *tab = (int *)(ws + b->off_tab), *len = (int *)(ws + b->off_len);
    if ((e = launch_batch_split((const BatchTile *)(ws + b->off_tiles), (int)b->tiles.size(),
                                (const int *)(ws + b->off_end), (int)n, tab, tab + b->max_tiles,
                                (int *)(ws + b->off_scan), len, len + n + 1, s)) != hipSuccess)
      return hip_fail(e, "batch tile split");
  }
  const int last = steps < 0 ? b->max_steps : std::min(steps, b->max_steps);
  for (int k = 0; k < last; ++k) {
    BatchWalk W[2];
    batch_walks(b, ws, k, W);
    if ((e = launch_batched_step(b->by, W, (const float2 *)(ws + b->off_coef),
                                 (const int *)(ws + b->off_cap), b->max_steps, k, batch_grid(b),
                                 b->max_mat, s)) != hipSuccess)
      return hip_fail(e, "batched step launch");
  }
  if (steps >= 0) return BBFD_OK;
  for (size_t q = 0; q < n; ++q) {
    int rc = enqueue_epilogue(b->plans[q], peak[q], ws + b->sub_off[q], s);
    if (rc) return rc;
  }
  return BBFD_OK;
}

// Autotuner probe of the per-solve shape: every solve's prologue, then one
// captured graph of probe steps of every solve (its own step kernels, two
// branches), launched once untimed and once between e0 and e1.
int probe_per_solve(bbfd_batch *b, const uint8_t *const *mat, const float *const *src,
                    float *const *peak, char *ws, hipStream_t s, int probe, hipEvent_t e0,
                    hipEvent_t e1, float *ms) {
  hipError_t e;
  if (!b->cap_stream && (e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking)) != hipSuccess)
    return hip_fail(e, "capture stream");
  const size_t n = b->plans.size();
  for (size_t q = 0; q < n; ++q) {
    bbfd_plan *pl = b->plans[q];
    std::lock_guard<std::mutex> lock(pl->mu);
    int rc = ensure_branch(pl);
    if (!rc) rc = enqueue_prologue(pl, mat[q], peak[q], ws + b->sub_off[q], s);
    if (rc) return rc;
  }
  if ((e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return hip_fail(e, "begin capture");
  int rc = BBFD_OK;
  for (size_t q = 0; q < n && !rc; ++q) {
    bbfd_plan *pl = b->plans[q];
    std::lock_guard<std::mutex> lock(pl->mu);
    rc = enqueue_steps(pl, mat[q], src[q], peak[q], ws + b->sub_off[q], b->cap_stream, 0,
                       std::min(probe, pl->prob.n_steps), nullptr,
                       pl->branch ? pl->side_stream : nullptr);
  }
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->cap_stream, &g);
  if (rc || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return rc ? rc : hip_fail(e, "end capture");
  }
  hipGraphExec_t x = nullptr;
  if ((e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0)) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(e, "graph instantiate");
  }
  *ms = 0.f;
  if ((e = hipGraphLaunch(x, s)) != hipSuccess || (e = hipEventRecord(e0, s)) != hipSuccess ||
      (e = hipGraphLaunch(x, s)) != hipSuccess || (e = hipEventRecord(e1, s)) != hipSuccess ||
      (e = hipEventSynchronize(e1)) != hipSuccess || (e = hipEventElapsedTime(ms, e0, e1)) != hipSuccess)
    rc = hip_fail(e, "per-solve probe");
  (void)hipGraphExecDestroy(x);
  (void)hipGraphDestroy(g);
  return rc;
}

void drop_graph(bbfd_batch *b) {
  (void)wait_staging(b);  // a launch of the graph may still be queued
  if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  b->key.clear();
}

std::string batch_key(const bbfd_batch *b) {
  // size class of the sweep: solve count, total cells (to 1 %) and the longest run
  unsigned long long cells = 0;
  for (const bbfd_plan *pl : b->plans) cells += (unsigned long long)pl->prob.nx * pl->prob.ny * pl->prob.nz;
  double lg = std::log(std::max(1.0, (double)cells)) / std::log(1.01);
  std::ostringstream os;
  os << "gfx950:n" << b->plans.size() << ":c" << (long long)std::floor(lg) << ":s" << b->max_steps;
  return os.str();
}

}  // namespace

extern "C" {

int bbfd_batch_create(const bbfd_problem *probs, int32_t n, bbfd_batch **out) {
  if (!out) return fail(BBFD_EINVAL, "null output pointer");
  *out = nullptr;
  if (!probs || n <= 0) return fail(BBFD_EINVAL, "need at least one problem");
  bbfd_batch *b = new (std::nothrow) bbfd_batch();
  if (!b) return fail(BBFD_EINVAL, "out of host memory");
  for (int s = 0; s < n; ++s) {
    bbfd_plan *pl = nullptr;
    int rc = bbfd_plan_create(&probs[s], &pl);
    if (rc) {
      std::string msg = g_err;
      bbfd_batch_destroy(b);
      return fail(rc, "problem %d: %s", s, msg.c_str());
    }
    b->plans.push_back(pl);
    if (pl->prob.index_bits == 16) {
      bbfd_batch_destroy(b);
      return fail(BBFD_EINVAL, "problem %d: batched sweeps take 8-bit maps", s);
    }
    b->max_steps = std::max(b->max_steps, pl->prob.n_steps);
    b->max_mat = std::max(b->max_mat, pl->prob.n_materials);
  }
  b->order.resize(n);
  for (int s = 0; s < n; ++s) b->order[s] = s;
  std::stable_sort(b->order.begin(), b->order.end(), [&](int a, int c) {
    return b->plans[a]->prob.n_steps > b->plans[c]->prob.n_steps;
  });
  b->max_tiles = tiles_capacity(b);
  size_t o = 0;
  b->off_desc = o; o += round_up((size_t)n * sizeof(StepArgs), 256);
  b->off_tiles = o; o += round_up(b->max_tiles * sizeof(BatchTile), 256);
  b->off_coef = o; o += round_up((size_t)n * b->max_steps * sizeof(float2), 256);
  b->off_cap = o; o += round_up((size_t)n * sizeof(int), 256);
  b->off_tab = o; o += round_up(2 * b->max_tiles * sizeof(int), 256);
  b->off_scan = o; o += round_up(b->max_tiles * sizeof(int), 256);
  b->off_len = o; o += round_up(2 * ((size_t)n + 1) * sizeof(int), 256);
  b->off_end = o; o += round_up((size_t)n * sizeof(int), 256);
  for (int s = 0; s < n; ++s) {
    b->sub_off.push_back(o);
    o += round_up(b->plans[s]->ws_bytes, 256);
  }
  b->ws_bytes = o;
  build_tiles(b);
  *out = b;
  return BBFD_OK;
}

void bbfd_batch_destroy(bbfd_batch *b) {
  if (!b) return;
  drop_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->staged) (void)hipEventDestroy(b->staged);
  if (b->h_desc) (void)hipHostFree(b->h_desc);
  if (b->h_tiles) (void)hipHostFree(b->h_tiles);
  if (b->h_coef) (void)hipHostFree(b->h_coef);
  if (b->h_cap) (void)hipHostFree(b->h_cap);
  if (b->h_end) (void)hipHostFree(b->h_end);
  for (bbfd_plan *pl : b->plans) bbfd_plan_destroy(pl);
  delete b;
}

int bbfd_batch_info(const bbfd_batch *b, uint64_t *workspace_bytes, int32_t *shape) {
  if (!b || !workspace_bytes) return fail(BBFD_EINVAL, "null argument");
  *workspace_bytes = b->ws_bytes;
  if (shape) {
    shape[0] = b->by;
    shape[1] = b->blocks;
    shape[2] = b->kchunk;
    shape[3] = (int32_t)b->tiles.size();
  }
  return BBFD_OK;
}

const bbfd_plan *bbfd_batch_plan(const bbfd_batch *b, int32_t i) {
  if (!b || i < 0 || i >= (int32_t)b->plans.size()) {
    fail(BBFD_EINVAL, "solve index out of range");
    return nullptr;
  }
  return b->plans[i];
}

uint64_t bbfd_batch_offset(const bbfd_batch *b, int32_t i) {
  if (!b || i < 0 || i >= (int32_t)b->plans.size()) return 0;
  return b->sub_off[i];
}

int bbfd_batch_set_shape(bbfd_batch *b, int32_t by, int32_t blocks, int32_t kchunk) {
  if (!b) return fail(BBFD_EINVAL, "null batch");
  if (by == 0) {  // per-solve shape
    std::lock_guard<std::mutex> lock(b->mu);
    b->by = b->blocks = b->kchunk = 0;
    build_tiles(b);
    drop_graph(b);
    return BBFD_OK;
  }
  if (!(by == 1 || by == 2 || by == 4 || by == 8) || blocks < 0 || kchunk < 1)
    return fail(BBFD_EINVAL, "bad launch shape (%d, %d, %d)", by, blocks, kchunk);
  size_t ntiles = 0;
  for (const bbfd_plan *pl : b->plans) {
    const bbfd_problem &p = pl->prob;
    const int kc = std::max(1, std::min((int)kchunk, p.nz));
    ntiles += (size_t)((p.nx + kSeg - 1) / kSeg) * ((p.ny + by - 1) / by) * ((p.nz + kc - 1) / kc);
  }
  if (ntiles > b->max_tiles)
    return fail(BBFD_EINVAL, "shape (%d, %d, %d) needs %zu tiles, table holds %zu", by, blocks, kchunk,
                ntiles, b->max_tiles);
  std::lock_guard<std::mutex> lock(b->mu);
  b->by = by;
  b->blocks = blocks;
  b->kchunk = kchunk;
  build_tiles(b);
  drop_graph(b);
  return BBFD_OK;
}

int bbfd_batch_solve(bbfd_batch *b, const uint8_t *const *mat, const float *const *src,
                     float *const *peak, void *workspace, uint64_t bytes, void *stream) {
  int rc = check_batch_args(b, mat, src, peak, workspace, bytes);
  if (rc) return rc;
  std::lock_guard<std::mutex> lock(b->mu);
  if ((rc = batch_pinned(b))) return rc;
  const size_t n = b->plans.size();
  std::vector<const void *> key;
  for (size_t q = 0; q < n; ++q) {
    key.push_back(mat[q]);
    key.push_back(src[q]);
    key.push_back(peak[q]);
  }
  key.push_back(workspace);
  const int shape[3] = {b->by, b->blocks, b->kchunk};
  if (!b->exec || key != b->key || std::memcmp(shape, b->key_shape, sizeof shape) != 0) {
    drop_graph(b);
    hipError_t e;
    if (!b->cap_stream && (e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking)) != hipSuccess)
      return hip_fail(e, "capture stream");
    if ((e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return hip_fail(e, "begin capture");
    rc = enqueue_batch(b, mat, src, peak, (char *)workspace, b->cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->cap_stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    b->graph = g;
    if ((e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0)) != hipSuccess) {
      b->exec = nullptr;
      return hip_fail(e, "graph instantiate");
    }
    b->key = key;
    std::memcpy(b->key_shape, shape, sizeof shape);
  }
  hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  return mark_staging(b, (hipStream_t)stream);
}

int bbfd_batch_status(const bbfd_batch *b, const void *workspace, int32_t i, int64_t *peak_index,
                      float *peak_value, void *stream) {
  if (!b || i < 0 || i >= (int32_t)b->plans.size()) return fail(BBFD_EINVAL, "solve index out of range");
  return bbfd_status(b->plans[i], (const char *)workspace + b->sub_off[i], peak_index, peak_value,
                     stream);
}

int bbfd_batch_autotune(bbfd_batch *b, const uint8_t *const *mat, const float *const *src,
                        float *const *peak, void *workspace, uint64_t bytes, void *stream,
                        const char *cache_path, int32_t probe_steps, double *best_ms) {
  int rc = check_batch_args(b, mat, src, peak, workspace, bytes);
  if (rc) return rc;
  const std::string key = batch_key(b);
  if (cache_path && *cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string k;
      int by, blocks, kc;
      double ms;
      if ((ls >> k >> by >> blocks >> kc >> ms) && k == key) {
        if (best_ms) *best_ms = ms;
        return bbfd_batch_set_shape(b, by, blocks, kc);
      }
    }
  }
  if (probe_steps < 1) probe_steps = 1;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(BBFD_EHIP, "event create");
  double best = 1e300;
  int bb_ = b->by, bl_ = b->blocks, kc_ = b->kchunk;
  const int bys[] = {1, 2, 4, 8};
  const int kcs[] = {4, 8, 16, 32};
  const int bls[] = {0, 1024, 2048, 4096};
  {
    std::lock_guard<std::mutex> lock(b->mu);
    if ((rc = batch_pinned(b))) goto done;
  }
  for (int by : bys)
    for (int kc : kcs)
      for (int bl : bls) {
        if ((rc = bbfd_batch_set_shape(b, by, bl, kc))) {
          rc = BBFD_OK;  // shape not representable: skip it
          continue;
        }
        std::lock_guard<std::mutex> lock(b->mu);
        // warm-up pass (prologue + probe steps), then the timed probe steps
        if ((rc = enqueue_batch(b, mat, src, peak, (char *)workspace, s, probe_steps)) ||
            (rc = mark_staging(b, s)))
          goto done;
        (void)hipEventRecord(e0, s);
        for (int k = 0; k < probe_steps; ++k) {
          BatchWalk W[2];
          batch_walks(b, (char *)workspace, k, W);
          hipError_t e = launch_batched_step(b->by, W, (const float2 *)((char *)workspace + b->off_coef),
                                             (const int *)((char *)workspace + b->off_cap), b->max_steps, k,
                                             batch_grid(b), b->max_mat, s);
          if (e != hipSuccess) {
            rc = hip_fail(e, "tuning launch");
            goto done;
          }
        }
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) {
          rc = fail(BBFD_EHIP, "tuning sync");
          goto done;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
          best = ms;
          bb_ = by;
          bl_ = bl;
          kc_ = kc;
        }
      }
  {
    std::lock_guard<std::mutex> lock(b->mu);
    float ms = 0.f;
    if ((rc = probe_per_solve(b, mat, src, peak, (char *)workspace, s, probe_steps, e0, e1, &ms)))
      goto done;
    if (ms < best) {
      best = ms;
      bb_ = bl_ = kc_ = 0;
    }
  }
  rc = bbfd_batch_set_shape(b, bb_, bl_, kc_);
  if (rc == BBFD_OK && best_ms) *best_ms = best;
  if (rc == BBFD_OK && cache_path && *cache_path) {
    std::ofstream outf(cache_path, std::ios::app);
    outf << key << " " << bb_ << " " << bl_ << " " << kc_ << " " << best << "\n";
  }
done:
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // extern "C"
