// Host side of the thermal step (BHTE, BabelBrain Section 2.4): validation,
// the FP64 derivation of the per-material coefficients and the stability
// limit of the explicit scheme, the workspace layout, and the time loop of
// bbfd_bhte_run (one step kernel per time step, the source switched by the
// sonication regime).  C ABI in include/bbfd.h.
#include "bbfd.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>
#include <string>
#include <vector>

#include "bbfd_dev.h"

namespace bbfd {
int set_error(int code, const char *msg);
hipError_t launch_bhte_source(const uint8_t *mat, const float *peak, const float *coef, long long n,
                              float *q, hipStream_t s);
hipError_t launch_bhte_fill(float *a, float *b, float *c, long long n, float va, float vb, float vc,
                            hipStream_t s);
hipError_t launch_bhte_step(int nx, int ny, int nz, int n_mat, const void *tab, const uint8_t *mat,
                            const float *q, const float *t_in, float *t_out, float *t_max,
                            float *dose, float q_scale, float d43, float dose_dt, hipStream_t s);
hipError_t launch_bhte_finish(const float *theta, float *t_final, float *t_max, long long n,
                              float t_body, hipStream_t s);
int bhte_row_floats();
}  // namespace bbfd

using namespace bbfd;

namespace {

constexpr double kRhoCBlood = 1050.0 * 3617.0;  // blood density x specific heat

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return bbfd::set_error(code, buf);
}

int hip_fail(hipError_t e, const char *what) {
  return fail(BBFD_EHIP, "%s: %s", what, hipGetErrorString(e));
}

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct bbfd_bhte {
  bbfd_bhte_problem prob{};
  std::vector<bbfd_material> acoustic;
  std::vector<bbfd_thermal> thermal;
  std::vector<float> tab;   // per material: k, dt/(rho C dx^2), dt w rho_b C_b/(rho C), dt/(rho C)
  std::vector<float> coef;  // per material: scale h alpha_l / (rho c_l)
  double dt_max = 0;
  size_t off_tab = 0, off_coef = 0, off_t0 = 0, off_t1 = 0, off_q = 0, ws_bytes = 0;
};

extern "C" {

int bbfd_bhte_create(const bbfd_bhte_problem *p, bbfd_bhte **out) {
  if (!out) return fail(BBFD_EINVAL, "null output pointer");
  *out = nullptr;
  if (!p) return fail(BBFD_EINVAL, "null problem");
  if (p->nx < 3 || p->ny < 3 || p->nz < 3)
    return fail(BBFD_EINVAL, "grid %dx%dx%d: need at least 3 cells per axis", p->nx, p->ny, p->nz);
  if (!(p->dx > 0) || !(p->dt > 0)) return fail(BBFD_EINVAL, "dx and dt must be positive");
  if (p->n_on < 0 || p->n_off < 0 || p->n_on + p->n_off < 1)
    return fail(BBFD_EINVAL, "need n_on, n_off >= 0 and at least one step");
  if (!(p->duty > 0 && p->duty <= 1)) return fail(BBFD_EINVAL, "duty cycle %g outside (0, 1]", p->duty);
  if (!(p->intensity_scale >= 0) || !std::isfinite(p->t_body))
    return fail(BBFD_EINVAL, "bad intensity scale or body temperature");
  if (p->n_materials < 1 || p->n_materials > kMaxMaterials || !p->acoustic || !p->thermal)
    return fail(BBFD_EINVAL, "need 1..%d materials with both tables", kMaxMaterials);
  bbfd_bhte *b = new (std::nothrow) bbfd_bhte();
  if (!b) return fail(BBFD_EINVAL, "out of host memory");
  b->prob = *p;
  b->acoustic.assign(p->acoustic, p->acoustic + p->n_materials);
  b->thermal.assign(p->thermal, p->thermal + p->n_materials);
  b->prob.acoustic = b->acoustic.data();
  b->prob.thermal = b->thermal.data();
  const double dx2 = p->dx * p->dx;
  double dt_max = INFINITY;
  for (int m = 0; m < p->n_materials; ++m) {
    const bbfd_material &a = b->acoustic[m];
    const bbfd_thermal &t = b->thermal[m];
    if (!(a.rho > 0) || !(a.c_l > 0) || !(a.alpha_l >= 0) || !(t.c > 0) || !(t.k >= 0) ||
        !(t.perfusion >= 0) || !(t.heat_frac >= 0 && t.heat_frac <= 1)) {
      delete b;
      return fail(BBFD_EMATERIAL, "material %d: bad thermal or acoustic properties", m);
    }
    const double rc = a.rho * t.c;
    dt_max = std::min(dt_max, rc / (6.0 * t.k / dx2 + t.perfusion * kRhoCBlood));
    b->tab.push_back((float)t.k);
    b->tab.push_back((float)(p->dt / (rc * dx2)));
    b->tab.push_back((float)(p->dt * t.perfusion * kRhoCBlood / rc));
    b->tab.push_back((float)(p->dt / rc));
    b->coef.push_back((float)(p->intensity_scale * t.heat_frac * a.alpha_l / (a.rho * a.c_l)));
  }
  b->dt_max = dt_max;
  if (!(p->dt < dt_max)) {
    delete b;
    return fail(BBFD_EINVAL, "dt %g s at or above the explicit stability limit %g s", p->dt, dt_max);
  }
  const size_t cells = (size_t)p->nx * p->ny * p->nz;
  size_t o = 0;
  b->off_tab = o; o += round_up((size_t)kMaxMaterials * bhte_row_floats() * sizeof(float), 256);
  b->off_coef = o; o += round_up((size_t)kMaxMaterials * sizeof(float), 256);
  b->off_t0 = o; o += round_up(cells * sizeof(float), 256);
  b->off_t1 = o; o += round_up(cells * sizeof(float), 256);
  b->off_q = o; o += round_up(cells * sizeof(float), 256);
  b->ws_bytes = o;
  *out = b;
  return BBFD_OK;
}

void bbfd_bhte_destroy(bbfd_bhte *b) { delete b; }

int bbfd_bhte_info(const bbfd_bhte *b, uint64_t *workspace_bytes, double *dt_max) {
  if (!b) return fail(BBFD_EINVAL, "null thermal plan");
  if (workspace_bytes) *workspace_bytes = b->ws_bytes;
  if (dt_max) *dt_max = b->dt_max;
  return BBFD_OK;
}

int bbfd_bhte_run(const bbfd_bhte *b, const uint8_t *mat, const float *peak, float *t_final,
                  float *t_max, float *dose, void *workspace, uint64_t bytes, void *stream) {
  if (!b) return fail(BBFD_EINVAL, "null thermal plan");
  if (!mat || !peak || !t_final || !t_max || !dose) return fail(BBFD_EINVAL, "null device pointer");
  if (!workspace) return fail(BBFD_ENOMEM, "null workspace");
  if ((uintptr_t)workspace % 256) return fail(BBFD_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < b->ws_bytes)
    return fail(BBFD_ENOMEM, "workspace of %llu bytes, need %llu", (unsigned long long)bytes,
                (unsigned long long)b->ws_bytes);
  const bbfd_bhte_problem &p = b->prob;
  hipStream_t s = (hipStream_t)stream;
  char *ws = (char *)workspace;
  const long long n = (long long)p.nx * p.ny * p.nz;
  float *th[2] = {(float *)(ws + b->off_t0), (float *)(ws + b->off_t1)};
  float *q = (float *)(ws + b->off_q);
  hipError_t e;
  if ((e = hipMemcpyAsync(ws + b->off_tab, b->tab.data(), b->tab.size() * sizeof(float),
                          hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(ws + b->off_coef, b->coef.data(), b->coef.size() * sizeof(float),
                          hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_fail(e, "thermal table upload");
  if ((e = launch_bhte_fill(th[0], t_max, dose, n, 0.f, 0.f, 0.f, s)) != hipSuccess ||
      (e = launch_bhte_source(mat, peak, (const float *)(ws + b->off_coef), n, q, s)) != hipSuccess)
    return hip_fail(e, "thermal prologue");
  const int steps = p.n_on + p.n_off;
  const float d43 = (float)(43.0 - p.t_body), dose_dt = (float)(p.dt / 60.0);
  for (int k = 0; k < steps; ++k) {
    const float qs = k < p.n_on ? (float)p.duty : 0.f;
    if ((e = launch_bhte_step(p.nx, p.ny, p.nz, p.n_materials, ws + b->off_tab, mat, q, th[k & 1],
                              th[(k + 1) & 1], t_max, dose, qs, d43, dose_dt, s)) != hipSuccess)
      return hip_fail(e, "thermal step launch");
  }
  if ((e = launch_bhte_finish(th[steps & 1], t_final, t_max, n, (float)p.t_body, s)) != hipSuccess)
    return hip_fail(e, "thermal epilogue");
  return BBFD_OK;
}

}  // extern "C"
