/*
 * bbref -- plain FP64 CPU oracle for the transcranial viscoelastic FDTD solve.
 *
 * TEST INFRASTRUCTURE ONLY: the checker of the HIP library, never part of it.
 * Written for readability against the paper, not for speed: every field access
 * goes through a bounds-checked accessor, material coefficients and staggered
 * averages are recomputed where they are used (only the absorbing profile is
 * tabulated once), and the loops run in the order the method states them.
 *
 * What it computes (paper Section 2.3, Eq. 1, with the pieces the paper defers
 * to its solver library filled in by the readings below):
 *
 *  - velocity-stress viscoelastic system of Eq. 1 on a Virieux staggered grid,
 *    4th order in space (Levander coefficients 9/8, -1/24), leapfrog in time;
 *  - attenuation through one standard-linear-solid (Zener) mechanism per wave
 *    type relaxing at the drive frequency, sized from Q = q_c * omega/(2 c alpha)
 *    (Section 3.2, Eq. 3 and the q_c correction);
 *  - convolutional PML with frequency shift (quadratic damping profile,
 *    R0 = 1e-3, shift alpha = pi f0 decreasing linearly to 0 at the wall);
 *  - the Rayleigh-Sommerfeld field S of the transducer (Section 2.3) entering
 *    as a normal-stress (traction) jump of 2S across the plane
 *    z = (k_s + 1/2) dx, i.e. a force layer on the v_z faces there;
 *  - capture of max |p|, p = -(sxx+syy+szz)/3, over the last two periods.
 */
#include "bbref.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define C1 (9.0 / 8.0)
#define C2 (-1.0 / 24.0)
#define RHO_W 1000.0
#define C_W 1500.0
#define PML_R0 1e-3

/* ------------------------------------------------------------------ setup */

/* Relaxed-modulus factor of a Zener element with relaxation strength tau whose
   relaxation time is 1/omega0: the squared real part of M(omega0)/M_R to the
   power -1/2.  Scaling the table speed's modulus by it makes the phase speed at
   the drive frequency equal the table speed. */
static double relaxed_factor(double tau) {
  double complex m = (1.0 + I * (1.0 + tau)) / (1.0 + I);
  double complex s = 1.0 / csqrt(m);
  return creal(s) * creal(s);
}

int bbref_setup(const bbref_problem *p, bbref_info *info, bbref_matconst *mc) {
  if (!p || !info) return BBREF_EINVAL;
  if (p->nx <= 0 || p->ny <= 0 || p->nz <= 0 || p->pml < 0 || p->n_steps <= 0)
    return BBREF_EINVAL;
  if (!(p->freq_hz > 0) || !(p->ppw > 0) || !(p->qc > 0) || !(p->cfl_safety > 0))
    return BBREF_EINVAL;
  if (p->index_bits != 0 && p->index_bits != 8 && p->index_bits != 16) return BBREF_EINVAL;
  const int max_mat = p->index_bits == 16 ? 4096 : 256;
  if (p->n_materials <= 0 || p->n_materials > max_mat || !p->materials) return BBREF_EINVAL;
  int periodic = (p->mode & BBREF_LATERAL_PERIODIC) != 0;
  if (2 * p->pml >= p->nz) return BBREF_EINVAL;
  if (!periodic && (2 * p->pml >= p->nx || 2 * p->pml >= p->ny)) return BBREF_EINVAL;

  double dx = C_W / (p->freq_hz * p->ppw);
  double w0 = 2.0 * M_PI * p->freq_hz;
  double T = 1.0 / p->freq_hz;
  double cmax = 0.0;
  for (int m = 0; m < p->n_materials; ++m) {
    const bbref_material *q = &p->materials[m];
    if (!(q->rho > 0) || !(q->c_l > 0) || !(q->c_s >= 0) || !(q->alpha_l >= 0) ||
        !(q->alpha_s >= 0))
      return BBREF_EMATERIAL;
    double nu = 0.5;
    if (q->c_s > 0) {
      if (!(q->c_l > q->c_s)) return BBREF_EMATERIAL;
      nu = (q->c_l * q->c_l - 2 * q->c_s * q->c_s) / (2 * (q->c_l * q->c_l - q->c_s * q->c_s));
      if (nu < -1.0 || nu >= 0.5) return BBREF_EMATERIAL; /* Section 3.2.2 range */
    }
    /* Eq. 3 with the q_c correction; no attenuation -> Q infinite. */
    double qp = q->alpha_l > 0 ? p->qc * w0 / (2 * q->c_l * q->alpha_l) : INFINITY;
    double qs = (q->c_s > 0 && q->alpha_s > 0) ? p->qc * w0 / (2 * q->c_s * q->alpha_s) : INFINITY;
    if (!(qp > 1.0) || !(qs > 1.0)) return BBREF_EMATERIAL;
    double tp = isinf(qp) ? 0.0 : 2.0 / (qp - 1.0);
    double ts = isinf(qs) ? 0.0 : 2.0 / (qs - 1.0);
    double pir = q->rho * q->c_l * q->c_l * relaxed_factor(tp);
    double mur = q->rho * q->c_s * q->c_s * relaxed_factor(ts);
    double piu = pir * (1 + tp), muu = mur * (1 + ts);
    double cu = sqrt(piu / q->rho);
    if (cu > cmax) cmax = cu;
    if (mc) {
      bbref_matconst *o = &mc[m];
      o->q_p = qp; o->q_s = qs; o->tau_p = tp; o->tau_s = ts;
      o->pi_r = pir; o->mu_r = mur; o->pi_u = piu; o->mu_u = muu; o->nu = nu;
    }
  }
  /* 3D stability limit of the 4th-order staggered leapfrog, then an integer
     number of steps per period. */
  double dt_max = dx / (sqrt(3.0) * (C1 - C2) * cmax);
  int nt = (int)ceil(T / (p->cfl_safety * dt_max));
  double dt = T / nt;

  int ks = p->source_k < 0 ? p->pml : p->source_k;
  if (ks < p->pml || ks >= p->nz - p->pml) return BBREF_EGEOMETRY;
  int cap = p->capture_start;
  if (cap < 0) {
    cap = p->n_steps - 2 * nt;
    if (cap < 0) cap = 0;
  }
  if (cap > p->n_steps) return BBREF_EINVAL;

  info->dx = dx;
  info->dt = dt;
  info->omega = w0;
  info->c_max = cmax;
  info->d0 = p->pml > 0 ? 3.0 * cmax * log(1.0 / PML_R0) / (2.0 * p->pml * dx) : 0.0;
  info->steps_per_period = nt;
  info->capture_start = cap;
  info->source_k = ks;
  return BBREF_OK;
}

/* -------------------------------------------------------------- simulator */

struct bbref_sim {
  bbref_problem p;
  bbref_info info;
  int nx, ny, nz, L, periodic, shear_src;
  size_t n;
  uint16_t *mat; /* material index per cell (from a uint8 or uint16 map) */
  int nm;
  double *rho, *pi_u, *mu_u, *pi_tau, *mu_tau, *tau_s, *mu;
  double *f[BBREF_NFIELDS];
  double *pml_b[3]; /* per axis, index 2*xi+1: exp(-(d + alpha) dt), or 0 outside the layer */
  double *pml_a[3]; /* per axis, index 2*xi+1: d/(d + alpha) (b - 1) */
  double *psi_v[9]; /* CPML memories of the 9 stress derivatives */
  double *psi_s[9]; /* CPML memories of the 9 velocity derivatives */
};

static size_t lin(const bbref_sim *s, int i, int j, int k) {
  return ((size_t)k * s->ny + j) * s->nx + i;
}

static int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

static int clampi(int i, int n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }

/* Field value; zero outside the grid (rigid wall behind the absorbing layer),
   periodic in x and y in the lateral-periodic test mode. */
static double F(const bbref_sim *s, const double *a, int i, int j, int k) {
  if (s->periodic) {
    i = wrap(i, s->nx);
    j = wrap(j, s->ny);
  } else if (i < 0 || j < 0 || i >= s->nx || j >= s->ny) {
    return 0.0;
  }
  if (k < 0 || k >= s->nz) return 0.0;
  return a[lin(s, i, j, k)];
}

/* Material index of a cell; outside the grid the edge cell is replicated. */
static int M(const bbref_sim *s, int i, int j, int k) {
  if (s->periodic) {
    i = wrap(i, s->nx);
    j = wrap(j, s->ny);
  } else {
    i = clampi(i, s->nx);
    j = clampi(j, s->ny);
  }
  k = clampi(k, s->nz);
  return s->mat[lin(s, i, j, k)];
}

/* 4th-order staggered differences along axis ax (0 x, 1 y, 2 z).
   dplus: value at (index + 1/2) from values stored at integer offsets.
   dminus: value at the integer index from values stored at (offset + 1/2). */
static double dplus(const bbref_sim *s, const double *a, int i, int j, int k, int ax) {
  int di = ax == 0, dj = ax == 1, dk = ax == 2;
  return (C1 * (F(s, a, i + di, j + dj, k + dk) - F(s, a, i, j, k)) +
          C2 * (F(s, a, i + 2 * di, j + 2 * dj, k + 2 * dk) - F(s, a, i - di, j - dj, k - dk))) /
         s->info.dx;
}

static double dminus(const bbref_sim *s, const double *a, int i, int j, int k, int ax) {
  int di = ax == 0, dj = ax == 1, dk = ax == 2;
  return (C1 * (F(s, a, i, j, k) - F(s, a, i - di, j - dj, k - dk)) +
          C2 * (F(s, a, i + di, j + dj, k + dk) - F(s, a, i - 2 * di, j - 2 * dj, k - 2 * dk))) /
         s->info.dx;
}

/* Depth (in cells) into the absorbing layer of a derivative evaluated at
   coordinate xi (in cells; integer or half-integer) along axis ax. */
static double pml_depth(const bbref_sim *s, int ax, double xi) {
  if (s->L == 0 || (s->periodic && ax < 2)) return 0.0;
  int N = ax == 0 ? s->nx : (ax == 1 ? s->ny : s->nz);
  double lo = (s->L - 0.5) - xi;
  double hi = xi - (N - s->L - 0.5);
  double l = lo > hi ? lo : hi;
  return l > 0 ? l : 0.0;
}

/* Frequency-shifted CPML coefficients at depth l > 0 (cells): damping
   d = d0 (l/L)^2, shift alpha = pi f0 (1 - l/L); per step b = exp(-(d + alpha) dt)
   and a = d/(d + alpha) (b - 1).  b = 0 marks a coordinate outside the layer. */
static void pml_coeffs(const bbref_sim *s, int ax, double xi, double *b, double *a) {
  double l = pml_depth(s, ax, xi);
  if (l <= 0) {
    *b = 0.0;
    *a = 0.0;
    return;
  }
  double d = s->info.d0 * (l / s->L) * (l / s->L);
  double al = M_PI * s->p.freq_hz * (1.0 - l / s->L);
  *b = exp(-(d + al) * s->info.dt);
  *a = d / (d + al) * (*b - 1.0);
}

/* Convolutional PML (kappa = 1): psi <- b psi + a d, and the derivative used by
   the update becomes d + psi. */
static double cpml(const bbref_sim *s, double *psi, size_t c, int ax, double xi, double d) {
  int m = (int)(2.0 * xi) + 1;
  double b = s->pml_b[ax][m];
  if (b == 0.0) return d;
  psi[c] = b * psi[c] + s->pml_a[ax][m] * d;
  return d + psi[c];
}

int bbref_sim_create(const bbref_problem *p, const void *map, bbref_sim **out) {
  if (!out || !map) return BBREF_EINVAL;
  *out = NULL;
  bbref_info info;
  int rc = bbref_setup(p, &info, NULL);
  if (rc) return rc;
  bbref_matconst *mc = (bbref_matconst *)calloc((size_t)p->n_materials, sizeof(bbref_matconst));
  bbref_setup(p, &info, mc);
  size_t n = (size_t)p->nx * p->ny * p->nz;
  uint16_t *mat = (uint16_t *)malloc(n * sizeof(uint16_t));
  for (size_t c = 0; c < n; ++c)
    mat[c] = p->index_bits == 16 ? ((const uint16_t *)map)[c] : ((const uint8_t *)map)[c];
  for (size_t c = 0; c < n; ++c)
    if (mat[c] >= p->n_materials) {
      free(mc);
      free(mat);
      return BBREF_EINDEX;
    }
  bbref_sim *s = (bbref_sim *)calloc(1, sizeof(bbref_sim));
  s->p = *p;
  s->info = info;
  s->nx = p->nx; s->ny = p->ny; s->nz = p->nz; s->L = p->pml;
  s->periodic = (p->mode & BBREF_LATERAL_PERIODIC) != 0;
  s->shear_src = (p->mode & BBREF_SOURCE_SHEAR_XZ) != 0;
  s->n = n;
  s->mat = mat;
  s->nm = p->n_materials;
  double **tabs[] = {&s->rho, &s->pi_u, &s->mu_u, &s->pi_tau, &s->mu_tau, &s->tau_s, &s->mu};
  for (int t = 0; t < 7; ++t) *tabs[t] = (double *)calloc((size_t)s->nm, sizeof(double));
  for (int m = 0; m < s->nm; ++m) {
    s->rho[m] = p->materials[m].rho;
    s->pi_u[m] = mc[m].pi_u;
    s->mu_u[m] = mc[m].mu_u;
    s->pi_tau[m] = mc[m].pi_r * mc[m].tau_p;
    s->mu_tau[m] = mc[m].mu_r * mc[m].tau_s;
    s->tau_s[m] = mc[m].tau_s;
    s->mu[m] = mc[m].mu_r;
  }
  free(mc);
  for (int ax = 0; ax < 3; ++ax) {
    int N = ax == 0 ? s->nx : (ax == 1 ? s->ny : s->nz);
    s->pml_b[ax] = (double *)calloc((size_t)(2 * N + 2), sizeof(double));
    s->pml_a[ax] = (double *)calloc((size_t)(2 * N + 2), sizeof(double));
    for (int m = 0; m < 2 * N + 2; ++m)
      pml_coeffs(s, ax, 0.5 * (m - 1), &s->pml_b[ax][m], &s->pml_a[ax][m]);
  }
  for (int f = 0; f < BBREF_NFIELDS; ++f) s->f[f] = (double *)calloc(n, sizeof(double));
  for (int f = 0; f < 9; ++f) {
    s->psi_v[f] = (double *)calloc(n, sizeof(double));
    s->psi_s[f] = (double *)calloc(n, sizeof(double));
  }
  *out = s;
  return BBREF_OK;
}

void bbref_sim_destroy(bbref_sim *s) {
  if (!s) return;
  free(s->mat);
  free(s->rho); free(s->pi_u); free(s->mu_u); free(s->pi_tau); free(s->mu_tau);
  free(s->tau_s); free(s->mu);
  for (int f = 0; f < BBREF_NFIELDS; ++f) free(s->f[f]);
  for (int ax = 0; ax < 3; ++ax) {
    free(s->pml_b[ax]);
    free(s->pml_a[ax]);
  }
  for (int f = 0; f < 9; ++f) {
    free(s->psi_v[f]);
    free(s->psi_s[f]);
  }
  free(s);
}

double *bbref_sim_field(bbref_sim *s, int32_t id) {
  if (!s || id < 0 || id >= BBREF_NFIELDS) return NULL;
  return s->f[id];
}

/* Eq. 1, rows 1-3: v^{n-1/2} -> v^{n+1/2} from sigma^n.  Buoyancy on the
   staggered velocity node is the inverse of the arithmetic mean density of the
   two cells it joins. */
static void velocity_update(bbref_sim *s) {
  double *vx = s->f[BBREF_VX], *vy = s->f[BBREF_VY], *vz = s->f[BBREF_VZ];
  const double *sxx = s->f[BBREF_SXX], *syy = s->f[BBREF_SYY], *szz = s->f[BBREF_SZZ];
  const double *sxy = s->f[BBREF_SXY], *sxz = s->f[BBREF_SXZ], *syz = s->f[BBREF_SYZ];
  const double dt = s->info.dt;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < s->nz; ++k)
    for (int j = 0; j < s->ny; ++j)
      for (int i = 0; i < s->nx; ++i) {
        size_t c = lin(s, i, j, k);
        double rho0 = s->rho[M(s, i, j, k)];
        { /* v_x at (i+1/2, j, k) */
          double b = 2.0 / (rho0 + s->rho[M(s, i + 1, j, k)]);
          double d1 = cpml(s, s->psi_v[0], c, 0, i + 0.5, dplus(s, sxx, i, j, k, 0));
          double d2 = cpml(s, s->psi_v[1], c, 1, j, dminus(s, sxy, i, j, k, 1));
          double d3 = cpml(s, s->psi_v[2], c, 2, k, dminus(s, sxz, i, j, k, 2));
          vx[c] += dt * b * (d1 + d2 + d3);
        }
        { /* v_y at (i, j+1/2, k) */
          double b = 2.0 / (rho0 + s->rho[M(s, i, j + 1, k)]);
          double d1 = cpml(s, s->psi_v[3], c, 0, i, dminus(s, sxy, i, j, k, 0));
          double d2 = cpml(s, s->psi_v[4], c, 1, j + 0.5, dplus(s, syy, i, j, k, 1));
          double d3 = cpml(s, s->psi_v[5], c, 2, k, dminus(s, syz, i, j, k, 2));
          vy[c] += dt * b * (d1 + d2 + d3);
        }
        { /* v_z at (i, j, k+1/2) */
          double b = 2.0 / (rho0 + s->rho[M(s, i, j, k + 1)]);
          double d1 = cpml(s, s->psi_v[6], c, 0, i, dminus(s, sxz, i, j, k, 0));
          double d2 = cpml(s, s->psi_v[7], c, 1, j, dminus(s, syz, i, j, k, 1));
          double d3 = cpml(s, s->psi_v[8], c, 2, k + 0.5, dplus(s, szz, i, j, k, 2));
          vz[c] += dt * b * (d1 + d2 + d3);
        }
      }
}

/* Crank-Nicolson step of one Zener memory variable relaxing (time constant
   1/omega0) toward -target, then the stress increment using the mean of its old
   and new value. */
static void relax_and_stress(double *sig, double *r, size_t c, double dt, double h,
                             double elastic_rate, double target) {
  double rn = ((1.0 - h) * r[c] - 2.0 * h * target) / (1.0 + h);
  sig[c] += dt * (elastic_rate + 0.5 * (r[c] + rn));
  r[c] = rn;
}

/* Shear stress on an edge: harmonic mean of the four cells' relaxed shear
   moduli (zero as soon as one cell is fluid), arithmetic mean of their shear
   relaxation strengths. */
static void shear_update(const bbref_sim *s, double *sig, double *r, size_t c, double e,
                         int m0, int m1, int m2, int m3) {
  double inv = 1.0 / s->mu[m0] + 1.0 / s->mu[m1] + 1.0 / s->mu[m2] + 1.0 / s->mu[m3];
  double mu_e = 4.0 / inv;
  double tau_e = 0.25 * (s->tau_s[m0] + s->tau_s[m1] + s->tau_s[m2] + s->tau_s[m3]);
  double h = 0.5 * s->info.omega * s->info.dt;
  relax_and_stress(sig, r, c, s->info.dt, h, mu_e * (1.0 + tau_e) * e, mu_e * tau_e * e);
}

/* Eq. 1, rows 4-9, with memory variables: sigma^n -> sigma^{n+1} from v^{n+1/2}. */
static void stress_update(bbref_sim *s) {
  const double *vx = s->f[BBREF_VX], *vy = s->f[BBREF_VY], *vz = s->f[BBREF_VZ];
  double **f = s->f;
  const double dt = s->info.dt;
  const double h = 0.5 * s->info.omega * dt;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < s->nz; ++k)
    for (int j = 0; j < s->ny; ++j)
      for (int i = 0; i < s->nx; ++i) {
        size_t c = lin(s, i, j, k);
        int m = M(s, i, j, k);
        double exx = cpml(s, s->psi_s[0], c, 0, i, dminus(s, vx, i, j, k, 0));
        double eyy = cpml(s, s->psi_s[1], c, 1, j, dminus(s, vy, i, j, k, 1));
        double ezz = cpml(s, s->psi_s[2], c, 2, k, dminus(s, vz, i, j, k, 2));
        double th = exx + eyy + ezz;
        const double lat[3] = {eyy + ezz, exx + ezz, exx + eyy};
        for (int a = 0; a < 3; ++a)
          relax_and_stress(f[BBREF_SXX + a], f[BBREF_RXX + a], c, dt, h,
                           s->pi_u[m] * th - 2.0 * s->mu_u[m] * lat[a],
                           s->pi_tau[m] * th - 2.0 * s->mu_tau[m] * lat[a]);
        /* sigma_xy at (i+1/2, j+1/2, k) */
        double exy = cpml(s, s->psi_s[3], c, 1, j + 0.5, dplus(s, vx, i, j, k, 1)) +
                     cpml(s, s->psi_s[4], c, 0, i + 0.5, dplus(s, vy, i, j, k, 0));
        shear_update(s, f[BBREF_SXY], f[BBREF_RXY], c, exy, m, M(s, i + 1, j, k),
                     M(s, i, j + 1, k), M(s, i + 1, j + 1, k));
        /* sigma_xz at (i+1/2, j, k+1/2) */
        double exz = cpml(s, s->psi_s[5], c, 2, k + 0.5, dplus(s, vx, i, j, k, 2)) +
                     cpml(s, s->psi_s[6], c, 0, i + 0.5, dplus(s, vz, i, j, k, 0));
        shear_update(s, f[BBREF_SXZ], f[BBREF_RXZ], c, exz, m, M(s, i + 1, j, k),
                     M(s, i, j, k + 1), M(s, i + 1, j, k + 1));
        /* sigma_yz at (i, j+1/2, k+1/2) */
        double eyz = cpml(s, s->psi_s[7], c, 2, k + 0.5, dplus(s, vy, i, j, k, 2)) +
                     cpml(s, s->psi_s[8], c, 1, j + 0.5, dplus(s, vz, i, j, k, 1));
        shear_update(s, f[BBREF_SYZ], f[BBREF_RYZ], c, eyz, m, M(s, i, j + 1, k),
                     M(s, i, j, k + 1), M(s, i, j + 1, k + 1));
      }
}

/* Source (Section 2.3: the incident field enters as a stress source on a
   plane perpendicular to the axis): a normal-traction jump of 2 S across the
   plane z = (k_s + 1/2) dx, i.e. a force layer on the v_z faces there, applied
   with the velocity update at t = n dt.  S is the incident complex pressure
   (e^{+i omega t}) at that plane, ramped in over two periods; each side then
   carries +-S for every angular component.  In the shear test mode the force
   acts on v_x of plane k_s instead. */
static void source_inject(bbref_sim *s, int n, const double *src) {
  if (!src) return;
  const double dt = s->info.dt, T = 2.0 * M_PI / s->info.omega;
  double t = n * dt;
  double tr = 2.0 * T;
  double w = 1.0;
  if (t < tr) {
    double q = sin(M_PI * t / (2.0 * tr));
    w = q * q;
  }
  double cs = cos(s->info.omega * t), sn = sin(s->info.omega * t);
  int ks = s->info.source_k;
  for (int j = 0; j < s->ny; ++j)
    for (int i = 0; i < s->nx; ++i) {
      size_t q = (size_t)j * s->nx + i;
      double force = 2.0 * w * (src[2 * q] * cs - src[2 * q + 1] * sn) / s->info.dx;
      size_t c = lin(s, i, j, ks);
      if (s->shear_src) {
        double b = 2.0 / (s->rho[M(s, i, j, ks)] + s->rho[M(s, i + 1, j, ks)]);
        s->f[BBREF_VX][c] += dt * b * force;
      } else {
        double b = 2.0 / (s->rho[M(s, i, j, ks)] + s->rho[M(s, i, j, ks + 1)]);
        s->f[BBREF_VZ][c] += dt * b * force;
      }
    }
}

/* Peak |p| with p the negative mean normal stress; a NaN is kept once seen so
   that divergence shows in the output. */
static void capture(bbref_sim *s) {
  const double *sxx = s->f[BBREF_SXX], *syy = s->f[BBREF_SYY], *szz = s->f[BBREF_SZZ];
  double *P = s->f[BBREF_PEAK];
#pragma omp parallel for schedule(static)
  for (long c = 0; c < (long)s->n; ++c) {
    double a = fabs(-(sxx[c] + syy[c] + szz[c]) / 3.0);
    if (a > P[c] || a != a) P[c] = a;
  }
}

void bbref_sim_step(bbref_sim *s, int32_t n, const double *src_re_im) {
  velocity_update(s);
  source_inject(s, n, src_re_im);
  stress_update(s);
  if (n + 1 >= s->info.capture_start) capture(s);
}

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

int bbref_solve(const bbref_problem *p, const void *mat, const double *src_re_im,
                double *peak, int64_t *peak_index, double *seconds) {
  bbref_sim *s = NULL;
  int rc = bbref_sim_create(p, mat, &s);
  if (rc) return rc;
  double t0 = now_s();
  for (int n = 0; n < p->n_steps; ++n) bbref_sim_step(s, n, src_re_im);
  if (seconds) *seconds = now_s() - t0;
  const double *P = s->f[BBREF_PEAK];
  if (peak) memcpy(peak, P, s->n * sizeof(double));
  rc = BBREF_OK;
  for (size_t c = 0; c < s->n; ++c)
    if (!isfinite(P[c])) rc = BBREF_EDIVERGED;
  if (peak_index) {
    int lx = s->periodic ? 0 : s->L, ly = s->periodic ? 0 : s->L, lz = s->L;
    int64_t best = -1;
    double bv = -1.0;
    for (int k = lz; k < s->nz - lz; ++k)
      for (int j = ly; j < s->ny - ly; ++j)
        for (int i = lx; i < s->nx - lx; ++i) {
          double v = P[lin(s, i, j, k)];
          if (v > bv) {
            bv = v;
            best = (int64_t)lin(s, i, j, k);
          }
        }
    *peak_index = best;
  }
  bbref_sim_destroy(s);
  return rc;
}

/* --------------------------------------------------------------- Rayleigh */

/* Orthonormal pair perpendicular to the unit axis: e1 is the projection of
   e_x (of e_y when the axis is within ~26 degrees of x), e2 = axis x e1. */
static void perp_basis(const double ax[3], double e1[3], double e2[3]) {
  double ref[3] = {1, 0, 0};
  if (fabs(ax[0]) >= 0.9) {
    ref[0] = 0;
    ref[1] = 1;
  }
  double d = ref[0] * ax[0] + ref[1] * ax[1] + ref[2] * ax[2];
  for (int a = 0; a < 3; ++a) e1[a] = ref[a] - d * ax[a];
  double nrm = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  for (int a = 0; a < 3; ++a) e1[a] /= nrm;
  e2[0] = ax[1] * e1[2] - ax[2] * e1[1];
  e2[1] = ax[2] * e1[0] - ax[0] * e1[2];
  e2[2] = ax[0] * e1[1] - ax[1] * e1[0];
}

int bbref_elements(const bbref_transducer *t, double freq_hz, double area_div, double *xyza,
                   int64_t cap, int64_t *n_out) {
  if (!t || !n_out || !(freq_hz > 0) || !(area_div > 0) || !(t->radius > 0)) return BBREF_EINVAL;
  double ax[3] = {t->axis[0], t->axis[1], t->axis[2]};
  double an = sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
  if (!(an > 0)) return BBREF_EINVAL;
  for (int a = 0; a < 3; ++a) ax[a] /= an;
  double e1[3], e2[3];
  perp_basis(ax, e1, e2);
  double lam = C_W / freq_hz;
  double target = lam * lam / area_div; /* element area (Section 2.3: lambda^2/16) */
  double width = sqrt(target);          /* ring width: lambda/4 at lambda^2/16 */
  int64_t n = 0;
  if (t->kind == 0) { /* flat piston: concentric rings */
    int nr = (int)ceil(t->radius / width);
    double dr = t->radius / nr;
    for (int r = 0; r < nr; ++r) {
      double r0 = r * dr, r1 = (r + 1) * dr;
      double ar = M_PI * (r1 * r1 - r0 * r0);
      long nphi = (long)ceil(ar / target);
      if (nphi < 1) nphi = 1;
      double rm = 0.5 * (r0 + r1);
      for (long q = 0; q < nphi; ++q, ++n) {
        if (!xyza || n >= cap) continue;
        double ph = 2.0 * M_PI * (q + 0.5) / nphi;
        for (int a = 0; a < 3; ++a)
          xyza[4 * n + a] = t->apex[a] + rm * (cos(ph) * e1[a] + sin(ph) * e2[a]);
        xyza[4 * n + 3] = ar / nphi;
      }
    }
  } else if (t->kind == 1) { /* spherical cap: rings equally spaced in polar angle */
    double Fo = t->focal;
    if (!(Fo >= t->radius)) return BBREF_EINVAL;
    double thmax = asin(t->radius / Fo);
    int nr = (int)ceil(Fo * thmax / width);
    double dth = thmax / nr;
    double focus[3];
    for (int a = 0; a < 3; ++a) focus[a] = t->apex[a] + Fo * ax[a];
    for (int r = 0; r < nr; ++r) {
      double t0 = r * dth, t1 = (r + 1) * dth;
      double ar = 2.0 * M_PI * Fo * Fo * (cos(t0) - cos(t1));
      long nphi = (long)ceil(ar / target);
      if (nphi < 1) nphi = 1;
      double tm = 0.5 * (t0 + t1);
      for (long q = 0; q < nphi; ++q, ++n) {
        if (!xyza || n >= cap) continue;
        double ph = 2.0 * M_PI * (q + 0.5) / nphi;
        for (int a = 0; a < 3; ++a)
          xyza[4 * n + a] = focus[a] + Fo * (-cos(tm) * ax[a] +
                                             sin(tm) * (cos(ph) * e1[a] + sin(ph) * e2[a]));
        xyza[4 * n + 3] = ar / nphi;
      }
    }
  } else {
    return BBREF_EINVAL;
  }
  *n_out = n;
  return BBREF_OK;
}

/* p(x) = (i omega rho_w / 2 pi) sum_e u0 A_e exp(-i k R_e) / R_e  (e^{+i omega t}). */
void bbref_rayleigh(const double *xyza, int64_t n_el, double freq_hz, double u0,
                    const double *pts, int64_t n_pts, double *out_re_im) {
  double w = 2.0 * M_PI * freq_hz;
  double k = w / C_W;
  double pre = w * RHO_W * u0 / (2.0 * M_PI);
#pragma omp parallel for schedule(static)
  for (long q = 0; q < (long)n_pts; ++q) {
    double sr = 0.0, si = 0.0;
    for (int64_t e = 0; e < n_el; ++e) {
      double dx = pts[3 * q] - xyza[4 * e];
      double dy = pts[3 * q + 1] - xyza[4 * e + 1];
      double dz = pts[3 * q + 2] - xyza[4 * e + 2];
      double R = sqrt(dx * dx + dy * dy + dz * dz);
      /* i * exp(-ikR) = sin(kR) + i cos(kR) */
      sr += xyza[4 * e + 3] * sin(k * R) / R;
      si += xyza[4 * e + 3] * cos(k * R) / R;
    }
    out_re_im[2 * q] = pre * sr;
    out_re_im[2 * q + 1] = pre * si;
  }
}
