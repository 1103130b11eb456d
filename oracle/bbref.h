/*
 * bbref -- plain FP64 CPU oracle for the transcranial viscoelastic FDTD solve
 * (BabelBrain, Section 2.3, Eq. 1; attenuation by quality factor, Section 3.2,
 * Eq. 3; Rayleigh-Sommerfeld source on the incident plane, Section 2.3).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the checker of the HIP path: only
 * the test suite, the smoke entry and the benchmark's CPU-baseline leg may load
 * it.  It shares no code, header, table or helper with the HIP library.
 *
 * Units are SI.  Every 3D array is C-order [nz][ny][nx] (x fastest).  All
 * pointers are host pointers owned by the caller unless stated otherwise.
 * Functions return 0 on success or a negative code (below).
 */
#ifndef BBREF_H
#define BBREF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BBREF_OK 0
#define BBREF_EINVAL (-1)
#define BBREF_EMATERIAL (-2)
#define BBREF_EINDEX (-3)
#define BBREF_EGEOMETRY (-4)
#define BBREF_EDIVERGED (-5)

/* Test modes (bit flags in bbref_problem.mode). */
#define BBREF_LATERAL_PERIODIC 1 /* x and y wrap periodically, no x/y absorbing layer */
#define BBREF_SOURCE_SHEAR_XZ 2  /* source force along x on the v_x of plane k_s (shear waves) */

typedef struct {
  double rho, c_l, c_s, alpha_l, alpha_s; /* alpha in Np/m at the drive frequency */
} bbref_material;

typedef struct {
  int32_t nx, ny, nz, pml;
  double freq_hz, ppw, qc, cfl_safety;
  int32_t n_steps, capture_start, source_k; /* < 0 -> defaults (last 2 periods; pml) */
  int32_t n_materials;
  const bbref_material *materials;
  int32_t mode;
  int32_t index_bits; /* 8 (or 0): uint8 map, <= 256 materials; 16: uint16 map, <= 4096 */
} bbref_problem;

typedef struct {
  double dx, dt, omega, c_max, d0;
  int32_t steps_per_period, capture_start, source_k;
} bbref_info;

typedef struct {
  double q_p, q_s, tau_p, tau_s, pi_r, mu_r, pi_u, mu_u, nu;
} bbref_matconst;

/* Field ids for bbref_sim_field. */
enum {
  BBREF_VX, BBREF_VY, BBREF_VZ,
  BBREF_SXX, BBREF_SYY, BBREF_SZZ, BBREF_SXY, BBREF_SXZ, BBREF_SYZ,
  BBREF_RXX, BBREF_RYY, BBREF_RZZ, BBREF_RXY, BBREF_RXZ, BBREF_RYZ,
  BBREF_PEAK, BBREF_NFIELDS
};

typedef struct bbref_sim bbref_sim;

/* Derived constants (grid, time step, per-material moduli).  mc may be NULL. */
int bbref_setup(const bbref_problem *p, bbref_info *info, bbref_matconst *mc);

/* Stateful stepping (fields start at zero). */
int bbref_sim_create(const bbref_problem *p, const void *mat, bbref_sim **out);
void bbref_sim_destroy(bbref_sim *s);
double *bbref_sim_field(bbref_sim *s, int32_t id); /* nz*ny*nx doubles, writable */
/* Advance from t_n to t_{n+1}: velocity, source (force layer), stress+memory,
   capture.  src_re_im: complex incident pressure at z = (k_s + 1/2) dx, [ny][nx]. */
void bbref_sim_step(bbref_sim *s, int32_t n, const double *src_re_im);

/* Whole solve: n_steps steps from rest, peak |p| map and its argmax over the
   non-absorbing interior (lowest linear index on ties). */
int bbref_solve(const bbref_problem *p, const void *mat, const double *src_re_im,
                double *peak, int64_t *peak_index, double *seconds);

/* Transducer surface elements (x, y, z, area): rings no wider than
   lambda/sqrt(area_div), each split into the fewest equal elements of area
   <= lambda^2/area_div (the paper uses 16, Section 2.3). */
typedef struct {
  int32_t kind; /* 0 flat piston, 1 spherical bowl */
  double radius, focal, apex[3], axis[3], u0;
} bbref_transducer;
int bbref_elements(const bbref_transducer *t, double freq_hz, double area_div,
                   double *xyza, int64_t cap, int64_t *n_out);

/* First Rayleigh integral at n_pts points: complex pressure (re, im). */
void bbref_rayleigh(const double *xyza, int64_t n_el, double freq_hz, double u0,
                    const double *pts, int64_t n_pts, double *out_re_im);

#ifdef __cplusplus
}
#endif
#endif
