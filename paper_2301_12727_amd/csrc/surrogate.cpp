// Host side of the learned surrogate (include/bbsur.h): the Fourier neural
// operator's forward and backward passes as sequences of strided BF16-MFMA
// GEMMs and element-wise kernels.
//
// The truncated 3D Fourier transforms are three successive GEMMs against
// small constant matrices.  Each stage contracts the innermost (unit-stride)
// axis of its input and writes the new frequency (or space) index outermost,
// so every stage reads and writes with plain strides:
//   forward  x:[z][y][x] -> [p,kx][z][y] -> [p,ky][kx][z] -> [p,kz][ky][kx]
//   inverse    [p][kz][ky][kx] -> [p,x][kz][ky] -> [p,y][x][kz] -> [z][y][x]
// (p = real/imaginary plane; complex contractions read both planes as one K
// axis of two segments).  The backward pass reuses the same stages: the
// adjoint of the inverse transform is the forward one with Hermitian weights
// c_k / n^3 folded in, and the adjoint of the forward transform is the inverse
// one without them.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <random>
#include <vector>

#include "bbfd.h"
#include "bbsur.h"
#include "nn_dev.h"

namespace bbfd {
int set_error(int code, const char *msg);
}

namespace bbsur {
hipError_t launch_gemm(const GemmArgs &g, hipStream_t s);
hipError_t launch_gelu_bwd(const float *z, const float *dh, float *dz, long long n, hipStream_t s);
hipError_t launch_fill(float *p, long long n, float v, hipStream_t s);
hipError_t launch_mix(const float *U, const float *R, float *V, int B, int C, int O, int Q,
                      hipStream_t s);
hipError_t launch_mix_bwd(const float *U, const float *dV, const float *R, float *dU, float *dR,
                          int B, int C, int O, int Q, hipStream_t s);
hipError_t launch_sum_rows(const float *in, float *out, int R, int M, float *tmp, hipStream_t s);
int sum_rows_groups();
int loss_partials();
hipError_t launch_loss(const float *y, const float *t, float *dy, float *partial, float *loss,
                       float focus, long long n, hipStream_t s);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, long long n, float lr_t,
                       float b1, float b2, float eps_t, hipStream_t s);
hipError_t launch_features(const uint8_t *mat, const float2 *table, int n_table,
                           const float2 *field, float *x, long long cells, hipStream_t s);
}  // namespace bbsur

using namespace bbsur;

namespace {

constexpr double kPi = 3.14159265358979323846;

int fail(int code, const char *msg) { return bbfd::set_error(code, msg); }

int hipchk(hipError_t e, const char *what) {
  if (e == hipSuccess) return BBFD_OK;
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return bbfd::set_error(BBFD_EHIP, m.c_str());
}

}  // namespace

struct bbsur_model {
  bbsur_config c{};
  int n = 0, cin = 0, W = 0, L = 0, mx = 0, my = 0, mz = 0;
  long long n2 = 0, P = 0, Q = 0;
  // constant transform matrices (FP32), concatenated
  std::vector<float> mats;
  size_t o_fx = 0, o_fxs = 0, o_fy = 0, o_fz = 0, o_gx = 0, o_gxu = 0, o_gy = 0, o_gz = 0;
  float *h_mats = nullptr;  // pinned copy, made at the first device call
  std::mutex mu;
  // parameter offsets (floats)
  size_t p_lw = 0, p_lb = 0, p_pw = 0, p_pb = 0, n_params = 0;
  std::vector<size_t> p_r, p_w, p_b;
};

namespace {

// Workspace layout for a batch (offsets in floats).
struct Layout {
  size_t mats, ones, h, z, U, T1, T2, V, I1, I2, y, dy, lossp, loss, dh, dh2, dz, dV, dU, part,
      bpart, red, total;
  long long Kc, S;  // split-K chunk and chunk count (Kc * S = n^3)
};

Layout layout(const bbsur_model *m, int B) {
  Layout o{};
  size_t a = 0;
  auto take = [&](size_t n) {
    size_t r = a;
    a += (n + 63) / 64 * 64;
    return r;
  };
  const long long BW = (long long)B * m->W;
  // weight gradients contract over all n^3 cells: split them into chunks of
  // n^2 / 16 cells (n^2 for small n) so a gradient launch has 16n blocks
  // (a multiple of 8 cells: the BF16 activations are staged eight at a time)
  o.Kc = (m->n2 % 128 == 0 && m->n2 >= 4096) ? m->n2 / 16 : m->n2;
  o.S = m->P / o.Kc;
  o.mats = take(m->mats.size());
  o.ones = take(o.Kc);
  o.h = take(((size_t)(m->L + 1) * BW * m->P + 1) / 2);  // BF16 activations h_0..h_L
  o.z = take((size_t)m->L * BW * m->P);
  o.U = take((size_t)m->L * BW * 2 * m->Q);
  o.T1 = take((size_t)BW * 2 * m->mx * m->n2);
  o.T2 = take((size_t)BW * 4 * m->my * m->mx * m->n);
  o.V = take((size_t)BW * 2 * m->Q);
  o.I1 = take((size_t)BW * 2 * m->n * 2 * m->mz * 2 * m->my);
  o.I2 = take((size_t)BW * 2 * m->n * m->n * 2 * m->mz);
  o.y = take((size_t)B * m->P);
  o.dy = take((size_t)B * m->P);
  o.lossp = take(loss_partials());
  o.loss = take(1);
  o.dh = take((size_t)BW * m->P);
  o.dh2 = take((size_t)BW * m->P);
  o.dz = take((size_t)BW * m->P);
  o.dV = take((size_t)BW * 2 * m->Q);
  o.dU = take((size_t)BW * 2 * m->Q);
  const size_t mw = (size_t)std::max(m->W, m->cin);
  o.part = take((size_t)B * o.S * mw * mw);
  o.bpart = take((size_t)B * o.S * mw);
  o.red = take((size_t)sum_rows_groups() * mw * mw);  // row-group sums of a gradient
  o.total = a;
  return o;
}

void build_mats(bbsur_model *m) {
  const int n = m->n, mx = m->mx, my = m->my, mz = m->mz;
  const double n3 = (double)n * n * n;
  auto sfreq = [](int kp, int mm) { return kp < mm ? kp : kp - 2 * mm; };  // signed frequency
  std::vector<float> &M = m->mats;
  auto add = [&](size_t count) {
    size_t o = M.size();
    M.resize(o + count, 0.f);
    return o;
  };
  // forward x: [x][(p, kx)], e^{-i theta}
  m->o_fx = add((size_t)n * 2 * mx);
  m->o_fxs = add((size_t)n * 2 * mx);
  for (int x = 0; x < n; ++x)
    for (int k = 0; k < mx; ++k) {
      const double th = 2.0 * kPi * k * x / n, w = (k == 0 ? 1.0 : 2.0) / n3;
      M[m->o_fx + x * 2 * mx + k] = (float)std::cos(th);
      M[m->o_fx + x * 2 * mx + mx + k] = (float)-std::sin(th);
      M[m->o_fxs + x * 2 * mx + k] = (float)(w * std::cos(th));
      M[m->o_fxs + x * 2 * mx + mx + k] = (float)(-w * std::sin(th));
    }
  // forward complex y / z: rows (p, s), cols (p', k'), e^{-i theta}
  auto fwd_complex = [&](int mm) {
    const size_t o = add((size_t)2 * n * 4 * mm);
    const int cols = 4 * mm;
    for (int s = 0; s < n; ++s)
      for (int kp = 0; kp < 2 * mm; ++kp) {
        const double th = 2.0 * kPi * sfreq(kp, mm) * s / n;
        const float c = (float)std::cos(th), sn = (float)std::sin(th);
        M[o + (size_t)s * cols + kp] = c;                           // Re <- Re
        M[o + (size_t)(n + s) * cols + kp] = sn;                    // Re <- Im
        M[o + (size_t)s * cols + 2 * mm + kp] = -sn;                // Im <- Re
        M[o + (size_t)(n + s) * cols + 2 * mm + kp] = c;            // Im <- Im
      }
    return o;
  };
  m->o_fy = fwd_complex(my);
  m->o_fz = fwd_complex(mz);
  // inverse x: rows (p, kx), cols (p', x), e^{+i theta}, weight w
  auto inv_x = [&](bool weighted) {
    const size_t o = add((size_t)2 * mx * 2 * n);
    for (int k = 0; k < mx; ++k)
      for (int x = 0; x < n; ++x) {
        const double th = 2.0 * kPi * k * x / n;
        const double w = weighted ? (k == 0 ? 1.0 : 2.0) / n3 : 1.0;
        const float c = (float)(w * std::cos(th)), sn = (float)(w * std::sin(th));
        M[o + (size_t)k * 2 * n + x] = c;
        M[o + (size_t)(mx + k) * 2 * n + x] = -sn;
        M[o + (size_t)k * 2 * n + n + x] = sn;
        M[o + (size_t)(mx + k) * 2 * n + n + x] = c;
      }
    return o;
  };
  m->o_gx = inv_x(true);
  m->o_gxu = inv_x(false);
  // inverse y: rows (p, ky'), cols (p', y)
  m->o_gy = add((size_t)4 * my * 2 * n);
  for (int kp = 0; kp < 2 * my; ++kp)
    for (int y = 0; y < n; ++y) {
      const double th = 2.0 * kPi * sfreq(kp, my) * y / n;
      const float c = (float)std::cos(th), sn = (float)std::sin(th);
      M[m->o_gy + (size_t)kp * 2 * n + y] = c;
      M[m->o_gy + (size_t)(2 * my + kp) * 2 * n + y] = -sn;
      M[m->o_gy + (size_t)kp * 2 * n + n + y] = sn;
      M[m->o_gy + (size_t)(2 * my + kp) * 2 * n + n + y] = c;
    }
  // inverse z, real part only: rows (p, kz'), cols z
  m->o_gz = add((size_t)4 * mz * n);
  for (int kp = 0; kp < 2 * mz; ++kp)
    for (int z = 0; z < n; ++z) {
      const double th = 2.0 * kPi * sfreq(kp, mz) * z / n;
      M[m->o_gz + (size_t)kp * n + z] = (float)std::cos(th);
      M[m->o_gz + (size_t)(2 * mz + kp) * n + z] = (float)-std::sin(th);
    }
}

// Which GEMM operands are stored as BF16 (the GELU outputs h_l are: every
// consumer of h_l is a matrix-core operand, rounded to BF16 anyway).
constexpr unsigned kBfA = 1, kBfB = 2, kBfC = 4, kBfGelu = 8;
typedef uint16_t bf16_t;  // storage of one BF16 value in host code
inline float *as_f(bf16_t *p) { return reinterpret_cast<float *>(p); }
inline const float *as_f(const bf16_t *p) { return reinterpret_cast<const float *>(p); }

// One strided GEMM launch (A may be two-segment along K).
struct G {
  hipStream_t s;
  int run(int batch, int M, int N, int K, const float *A, long long sAb, long long sAm,
          long long sAk, int aseg, long long asegoff, const float *B, long long sBb, long long sBk,
          long long sBn, float *C, long long sCb, long long sCm, long long sCn, float beta = 0.f,
          const float *bias = nullptr, float *gelu_out = nullptr,
          const float *gelu_z = nullptr, unsigned bf = 0) const {
    GemmArgs g{};
    g.A = A; g.B = B; g.C = C; g.bias = bias;
    g.M = M; g.N = N; g.K = K; g.batch = batch;
    g.sAb = sAb; g.sAm = sAm; g.sAk = sAk; g.a_seg_k = aseg > 0 ? aseg : K; g.a_seg_off = asegoff;
    g.sBb = sBb; g.sBk = sBk; g.sBn = sBn; g.b_seg_k = K; g.b_seg_off = 0;
    g.sCb = sCb; g.sCm = sCm; g.sCn = sCn;
    g.a_kfast = (sAk == 1) ? 1 : 0;
    g.b_nfast = (sBn == 1) ? 1 : 0;
    g.alpha = 1.f;
    g.beta = beta;
    g.gelu_out = gelu_out;
    g.gelu_z = gelu_z;
    g.a_bf16 = (bf & kBfA) ? 1 : 0;
    g.b_bf16 = (bf & kBfB) ? 1 : 0;
    g.c_bf16 = (bf & kBfC) ? 1 : 0;
    g.gelu_bf16 = (bf & kBfGelu) ? 1 : 0;
    return hipchk(launch_gemm(g, s), "gemm");
  }
};

struct Ctx {
  const bbsur_model *m;
  float *ws;
  Layout o;
  int B;
  hipStream_t s;
  const float *mat(size_t off) const { return ws + o.mats + off; }
};

// Truncated forward transform of nb volumes `in` ([nb][n^3]) into spectra
// `out` ([nb][2][Q]); fx selects plain or Hermitian-weighted x matrix.
// `in` holds BF16 values when in_bf16 (the activations h_l).
int spectral_forward(const Ctx &c, const float *in, float *out, size_t fx, int nb,
                     bool in_bf16 = false) {
  const bbsur_model *m = c.m;
  const int n = m->n, mx = m->mx, my = m->my, mz = m->mz;
  const long long n2 = m->n2;
  G g{c.s};
  float *T1 = c.ws + c.o.T1, *T2 = c.ws + c.o.T2;
  int rc = g.run(nb, (int)n2, 2 * mx, n, in, m->P, n, 1, 0, 0, c.mat(fx), 0, 2 * mx, 1, T1,
                 2LL * mx * n2, 1, n2, 0.f, nullptr, nullptr, nullptr, in_bf16 ? kBfA : 0);
  if (!rc)
    rc = g.run(nb, mx * n, 4 * my, 2 * n, T1, 2LL * mx * n2, n, 1, n, (long long)mx * n2,
               c.mat(m->o_fy), 0, 4 * my, 1, T2, 4LL * my * mx * n, 1, (long long)mx * n);
  if (!rc)
    rc = g.run(nb, 2 * my * mx, 4 * mz, 2 * n, T2, 4LL * my * mx * n, n, 1, n,
               2LL * my * mx * n, c.mat(m->o_fz), 0, 4 * mz, 1, out, 2 * m->Q, 1,
               2LL * my * mx);
  return rc;
}

// Inverse transform of spectra `in` ([nb][2][Q]) onto volumes `out`
// ([nb][n^3], accumulated when beta = 1); gx selects the weighted (forward
// pass) or unweighted (gradient) x matrix.  With act != NULL the last stage
// also stores GELU of the result there (same layout); with zpre != NULL as
// well it stores result * GELU'(zpre) there instead of the result.
int spectral_inverse(const Ctx &c, const float *in, float *out, size_t gx, int nb, float beta,
                     float *act = nullptr, const float *zpre = nullptr, bool act_bf16 = false) {
  const bbsur_model *m = c.m;
  const int n = m->n, mx = m->mx, my = m->my, mz = m->mz;
  const long long n2 = m->n2;
  G g{c.s};
  float *I1 = c.ws + c.o.I1, *I2 = c.ws + c.o.I2;
  const long long kzy = 4LL * mz * my;  // 2mz * 2my
  int rc = g.run(nb, (int)kzy, 2 * n, 2 * mx, in, 2 * m->Q, mx, 1, mx, m->Q, c.mat(gx), 0, 2 * n,
                 1, I1, 2LL * n * kzy, 1, kzy);
  if (!rc)
    rc = g.run(nb, n * 2 * mz, 2 * n, 4 * my, I1, 2LL * n * kzy, 2 * my, 1, 2 * my,
               (long long)n * kzy, c.mat(m->o_gy), 0, 2 * n, 1, I2, 2LL * n * n * 2 * mz, 1,
               (long long)n * 2 * mz);
  if (!rc)
    rc = g.run(nb, (int)n2, n, 4 * mz, I2, 2LL * n * n * 2 * mz, 2 * mz, 1, 2 * mz,
               n2 * 2 * mz, c.mat(m->o_gz), 0, n, 1, out, m->P, 1, n2, beta, nullptr, act, zpre,
               act_bf16 ? kBfGelu : 0);
  return rc;
}

// grad (M x N) = sum_b sum_p D[b][m][p] H[b][n][p]: split-K partials + fixed-order sum.
int weight_grad(const Ctx &c, const float *D, const float *H, int M, int N, float *grad,
                bool h_bf16 = false) {
  const bbsur_model *m = c.m;
  G g{c.s};
  float *part = c.ws + c.o.part;
  for (int b = 0; b < c.B; ++b) {
    const float *Hb = h_bf16 ? as_f(reinterpret_cast<const bf16_t *>(H) + (size_t)b * N * m->P)
                             : H + (size_t)b * N * m->P;
    int rc = g.run((int)c.o.S, M, N, (int)c.o.Kc, D + (size_t)b * M * m->P, c.o.Kc, m->P, 1, 0, 0,
                   Hb, c.o.Kc, 1, m->P, part + (size_t)b * c.o.S * M * N, (long long)M * N, N, 1,
                   0.f, nullptr, nullptr, nullptr, h_bf16 ? kBfB : 0);
    if (rc) return rc;
  }
  return hipchk(launch_sum_rows(part, grad, (int)(c.B * c.o.S), M * N, c.ws + c.o.red, c.s),
                "grad sum");
}

// grad (M) = sum_b sum_p D[b][m][p]
int bias_grad(const Ctx &c, const float *D, int M, float *grad) {
  const bbsur_model *m = c.m;
  G g{c.s};
  float *bpart = c.ws + c.o.bpart;
  for (int b = 0; b < c.B; ++b) {
    int rc = g.run((int)c.o.S, M, 1, (int)c.o.Kc, D + (size_t)b * M * m->P, c.o.Kc, m->P, 1, 0, 0,
                   c.ws + c.o.ones, 0, 1, 0, bpart + (size_t)b * c.o.S * M, M, 1, 0);
    if (rc) return rc;
  }
  return hipchk(launch_sum_rows(bpart, grad, (int)(c.B * c.o.S), M, c.ws + c.o.red, c.s),
                "bias sum");
}

int prepare(const bbsur_model *cm, void *ws, uint64_t bytes, int B, hipStream_t s, Ctx *c) {
  bbsur_model *m = const_cast<bbsur_model *>(cm);  // pinned staging only
  if (!m || !ws) return fail(BBFD_EINVAL, "null model or workspace");
  if (B < 1) return fail(BBFD_EINVAL, "batch must be >= 1");
  if ((uintptr_t)ws % 256) return fail(BBFD_EINVAL, "workspace must be 256-byte aligned");
  c->m = m;
  c->ws = (float *)ws;
  c->o = layout(m, B);
  c->B = B;
  c->s = s;
  if (bytes < c->o.total * sizeof(float)) return fail(BBFD_ENOMEM, "surrogate workspace too small");
  {
    std::lock_guard<std::mutex> lock(m->mu);
    if (!m->h_mats) {
      float *p = nullptr;
      hipError_t e = hipHostMalloc((void **)&p, m->mats.size() * sizeof(float), hipHostMallocDefault);
      if (e != hipSuccess) return hipchk(e, "pinned matrices");
      std::memcpy(p, m->mats.data(), m->mats.size() * sizeof(float));
      m->h_mats = p;
    }
  }
  int rc = hipchk(hipMemcpyAsync(c->ws + c->o.mats, m->h_mats, m->mats.size() * sizeof(float),
                                 hipMemcpyHostToDevice, s), "matrix upload");
  if (!rc) rc = hipchk(launch_fill(c->ws + c->o.ones, c->o.Kc, 1.f, s), "ones");
  return rc;
}

// Forward pass keeping h_l, z_l and the spectra U_l in the workspace.
int forward(const Ctx &c, const float *prm, const float *x) {
  const bbsur_model *m = c.m;
  const int B = c.B, W = m->W;
  const long long BWP = (long long)B * W * m->P;
  G g{c.s};
  bf16_t *h = reinterpret_cast<bf16_t *>(c.ws + c.o.h);
  float *z = c.ws + c.o.z, *U = c.ws + c.o.U;
  int rc = g.run(B, W, (int)m->P, m->cin, prm + m->p_lw, 0, m->cin, 1, 0, 0, x,
                 (long long)m->cin * m->P, m->P, 1, as_f(h), (long long)W * m->P, m->P, 1, 0.f,
                 prm + m->p_lb, nullptr, nullptr, kBfC);
  for (int l = 0; !rc && l < m->L; ++l) {
    const bf16_t *hin = h + l * BWP;
    float *zl = z + l * BWP;
    float *Ul = U + (size_t)l * B * W * 2 * m->Q;
    rc = g.run(B, W, (int)m->P, W, prm + m->p_w[l], 0, W, 1, 0, 0, as_f(hin),
               (long long)W * m->P, m->P, 1, zl, (long long)W * m->P, m->P, 1, 0.f,
               prm + m->p_b[l], nullptr, nullptr, kBfB);
    if (!rc) rc = spectral_forward(c, as_f(hin), Ul, m->o_fx, B * W, true);
    if (!rc)
      rc = hipchk(launch_mix(Ul, prm + m->p_r[l], c.ws + c.o.V, B, W, W, (int)m->Q, c.s), "mix");
    // z_l accumulates the inverse transform; h_{l+1} = GELU(z_l) in the same epilogue
    if (!rc)
      rc = spectral_inverse(c, c.ws + c.o.V, zl, m->o_gx, B * W, 1.f, as_f(h + (l + 1) * BWP),
                            nullptr, true);
  }
  if (!rc)
    rc = g.run(B, 1, (int)m->P, W, prm + m->p_pw, 0, W, 1, 0, 0, as_f(h + m->L * BWP),
               (long long)W * m->P, m->P, 1, c.ws + c.o.y, m->P, m->P, 1, 0.f, prm + m->p_pb,
               nullptr, nullptr, kBfB);
  return rc;
}

// Backward pass from dy (in the workspace) using the forward tape.
int backward(const Ctx &c, const float *prm, const float *x, const float *dy, float *grad) {
  const bbsur_model *m = c.m;
  const int B = c.B, W = m->W;
  const long long BWP = (long long)B * W * m->P;
  G g{c.s};
  const bf16_t *h = reinterpret_cast<const bf16_t *>(c.ws + c.o.h);
  float *z = c.ws + c.o.z, *U = c.ws + c.o.U;
  float *dh = c.ws + c.o.dh, *dh2 = c.ws + c.o.dh2, *dz = c.ws + c.o.dz;
  int rc = weight_grad(c, dy, as_f(h + m->L * BWP), 1, W, grad + m->p_pw, true);
  if (!rc) rc = bias_grad(c, dy, 1, grad + m->p_pb);
  if (!rc)
    rc = g.run(B, W, (int)m->P, 1, prm + m->p_pw, 0, 1, W, 0, 0, dy, m->P, m->P, 1, dh,
               (long long)W * m->P, m->P, 1);
  for (int l = m->L - 1; !rc && l >= 0; --l) {
    const bf16_t *hin = h + l * BWP;
    const float *zl = z + l * BWP;
    const float *Ul = U + (size_t)l * B * W * 2 * m->Q;
    // dz = dh * GELU'(z_l): for the top layer here, below it in the epilogue of
    // the previous iteration's last inverse-transform stage
    if (l == m->L - 1) rc = hipchk(launch_gelu_bwd(zl, dh, dz, BWP, c.s), "gelu grad");
    if (!rc) rc = weight_grad(c, dz, as_f(hin), W, W, grad + m->p_w[l], true);
    if (!rc) rc = bias_grad(c, dz, W, grad + m->p_b[l]);
    if (!rc)
      rc = g.run(B, W, (int)m->P, W, prm + m->p_w[l], 0, 1, W, 0, 0, dz, (long long)W * m->P,
                 m->P, 1, dh2, (long long)W * m->P, m->P, 1);
    if (!rc) rc = spectral_forward(c, dz, c.ws + c.o.dV, m->o_fxs, B * W);
    if (!rc)
      rc = hipchk(launch_mix_bwd(Ul, c.ws + c.o.dV, prm + m->p_r[l], c.ws + c.o.dU,
                                 grad + m->p_r[l], B, W, W, (int)m->Q, c.s), "mix grad");
    // dh2 = dL/dh_l; below the bottom layer h_l = GELU(z_{l-1}), so the next
    // iteration's dz is formed here (dz_l is no longer read)
    if (!rc && l > 0)
      rc = spectral_inverse(c, c.ws + c.o.dU, dh2, m->o_gxu, B * W, 1.f, dz, z + (l - 1) * BWP);
    else if (!rc)
      rc = spectral_inverse(c, c.ws + c.o.dU, dh2, m->o_gxu, B * W, 1.f);
    std::swap(dh, dh2);
  }
  if (!rc) rc = weight_grad(c, dh, x, W, m->cin, grad + m->p_lw);
  if (!rc) rc = bias_grad(c, dh, W, grad + m->p_lb);
  return rc;
}

}  // namespace

extern "C" {

int bbsur_create(const bbsur_config *cfg, bbsur_model **out) {
  if (!out) return fail(BBFD_EINVAL, "null output pointer");
  *out = nullptr;
  if (!cfg) return fail(BBFD_EINVAL, "null config");
  const bbsur_config &c = *cfg;
  if (c.n < 8 || c.n > 256 || c.n % 8 != 0 || c.cin < 1 || c.width < 1 || c.width > 256 ||
      c.layers < 1 ||
      c.mx < 1 || c.my < 1 || c.mz < 1 || 2 * c.mx > c.n || 2 * c.my > c.n || 2 * c.mz > c.n ||
      !(c.loss_focus >= 0.f))
    return fail(BBFD_EINVAL, "bad surrogate configuration");
  bbsur_model *m = new (std::nothrow) bbsur_model();
  if (!m) return fail(BBFD_EINVAL, "out of host memory");
  m->c = c;
  m->n = c.n; m->cin = c.cin; m->W = c.width; m->L = c.layers;
  m->mx = c.mx; m->my = c.my; m->mz = c.mz;
  m->n2 = (long long)c.n * c.n;
  m->P = m->n2 * c.n;
  m->Q = (long long)c.mx * 2 * c.my * 2 * c.mz;
  size_t o = 0;
  m->p_lw = o; o += (size_t)c.width * c.cin;
  m->p_lb = o; o += c.width;
  for (int l = 0; l < c.layers; ++l) {
    m->p_r.push_back(o); o += 2 * (size_t)m->Q * c.width * c.width;
    m->p_w.push_back(o); o += (size_t)c.width * c.width;
    m->p_b.push_back(o); o += c.width;
  }
  m->p_pw = o; o += c.width;
  m->p_pb = o; o += 1;
  m->n_params = o;
  build_mats(m);
  *out = m;
  return BBFD_OK;
}

void bbsur_destroy(bbsur_model *m) {
  if (!m) return;
  if (m->h_mats) (void)hipHostFree(m->h_mats);
  delete m;
}

int bbsur_sizes(const bbsur_model *m, int32_t batch, uint64_t *n_params, uint64_t *ws_bytes) {
  if (!m || batch < 1) return fail(BBFD_EINVAL, "null model or batch < 1");
  if (n_params) *n_params = m->n_params;
  if (ws_bytes) *ws_bytes = layout(m, batch).total * sizeof(float);
  return BBFD_OK;
}

int bbsur_init_params(const bbsur_model *m, float *params, uint64_t seed, void *stream) {
  if (!m || !params) return fail(BBFD_EINVAL, "null argument");
  std::vector<float> p(m->n_params, 0.f);
  std::mt19937_64 rng(seed);
  auto normal = [&](size_t off, size_t cnt, double sd) {
    std::normal_distribution<double> d(0.0, sd);
    for (size_t i = 0; i < cnt; ++i) p[off + i] = (float)d(rng);
  };
  const int W = m->W;
  normal(m->p_lw, (size_t)W * m->cin, 1.0 / std::sqrt((double)m->cin));
  for (int l = 0; l < m->L; ++l) {
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    const size_t cnt = 2 * (size_t)m->Q * W * W;
    const double sc = 1.0 / W;
    for (size_t i = 0; i < cnt; ++i) p[m->p_r[l] + i] = (float)(sc * u(rng));
    normal(m->p_w[l], (size_t)W * W, 1.0 / std::sqrt((double)W));
  }
  normal(m->p_pw, W, 1.0 / std::sqrt((double)W));
  hipStream_t s = (hipStream_t)stream;
  int rc = hipchk(hipMemcpyAsync(params, p.data(), p.size() * sizeof(float), hipMemcpyHostToDevice, s),
                  "parameter upload");
  if (!rc) rc = hipchk(hipStreamSynchronize(s), "parameter upload sync");
  return rc;
}

int bbsur_forward(const bbsur_model *m, const float *params, const float *x, float *y,
                  int32_t batch, void *ws, uint64_t bytes, void *stream) {
  if (!params || !x || !y) return fail(BBFD_EINVAL, "null device pointer");
  Ctx c{};
  int rc = prepare(m, ws, bytes, batch, (hipStream_t)stream, &c);
  if (!rc) rc = forward(c, params, x);
  if (!rc)
    rc = hipchk(hipMemcpyAsync(y, c.ws + c.o.y, (size_t)batch * m->P * sizeof(float),
                               hipMemcpyDeviceToDevice, c.s), "output copy");
  return rc;
}

int bbsur_backward(const bbsur_model *m, const float *params, const float *x, const float *dy,
                   float *grad, int32_t batch, void *ws, uint64_t bytes, void *stream) {
  if (!params || !x || !dy || !grad) return fail(BBFD_EINVAL, "null device pointer");
  Ctx c{};
  int rc = prepare(m, ws, bytes, batch, (hipStream_t)stream, &c);
  if (!rc) rc = forward(c, params, x);
  if (!rc) rc = backward(c, params, x, dy, grad);
  return rc;
}

int bbsur_train_step(const bbsur_model *m, float *params, float *grad, float *mom, float *var,
                     int32_t step, float lr, const float *x, const float *target, int32_t batch,
                     float *loss_dev, void *ws, uint64_t bytes, void *stream) {
  if (!params || !grad || !mom || !var || !x || !target || !loss_dev)
    return fail(BBFD_EINVAL, "null device pointer");
  if (step < 1) return fail(BBFD_EINVAL, "step counts from 1");
  Ctx c{};
  int rc = prepare(m, ws, bytes, batch, (hipStream_t)stream, &c);
  if (!rc) rc = forward(c, params, x);
  if (!rc)
    rc = hipchk(launch_loss(c.ws + c.o.y, target, c.ws + c.o.dy, c.ws + c.o.lossp, loss_dev,
                            m->c.loss_focus, (long long)batch * m->P, c.s), "loss");
  if (!rc) rc = backward(c, params, x, c.ws + c.o.dy, grad);
  if (!rc) {
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    const double c2 = std::sqrt(1.0 - std::pow(b2, step));
    const double lr_t = lr * c2 / (1.0 - std::pow(b1, step));
    rc = hipchk(launch_adam(params, grad, mom, var, (long long)m->n_params, (float)lr_t, (float)b1,
                            (float)b2, (float)(eps * c2), c.s), "adam");
  }
  return rc;
}

int bbsur_features(const uint8_t *mat, const float *table, int32_t n_table, const float *field,
                   float *x, int64_t cells, void *stream) {
  if (!mat || !table || !field || !x || cells <= 0 || n_table < 1)
    return fail(BBFD_EINVAL, "bad argument");
  return hipchk(launch_features(mat, (const float2 *)table, n_table, (const float2 *)field, x,
                                cells, (hipStream_t)stream), "features");
}

int bbsur_gemm(const float *A, const int64_t *as, const float *B, const int64_t *bs, float *C,
               const int64_t *cs, const float *bias, int32_t M, int32_t N, int32_t K,
               int32_t batch, float alpha, float beta, void *stream) {
  if (!A || !B || !C || !as || !bs || !cs) return fail(BBFD_EINVAL, "null argument");
  if (M < 0 || N < 0 || K < 0 || batch < 0) return fail(BBFD_EINVAL, "negative size");
  GemmArgs g{};
  g.A = A; g.B = B; g.C = C; g.bias = bias;
  g.M = M; g.N = N; g.K = K; g.batch = batch;
  g.sAb = as[0]; g.sAm = as[1]; g.sAk = as[2]; g.a_seg_k = K > 0 ? K : 1; g.a_seg_off = 0;
  g.sBb = bs[0]; g.sBk = bs[1]; g.sBn = bs[2]; g.b_seg_k = K > 0 ? K : 1; g.b_seg_off = 0;
  g.sCb = cs[0]; g.sCm = cs[1]; g.sCn = cs[2];
  g.a_kfast = g.sAk == 1;
  g.b_nfast = g.sBn == 1;
  g.alpha = alpha;
  g.beta = beta;
  return hipchk(launch_gemm(g, (hipStream_t)stream), "gemm");
}

}  // extern "C"
