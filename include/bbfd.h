/*
 * bbfd -- MI355X (gfx950) viscoelastic FDTD for transcranial ultrasound.
 *
 * C ABI of the hot path of BabelBrain's acoustic step (arXiv 2301.12727,
 * Section 2.3): a material map plus property table, a transducer, a frequency
 * and points-per-wavelength in; the transmitted peak-pressure map out.
 *
 * Conventions
 *  - SI units.  3D arrays are C-order [nz][ny][nx] (x fastest), z is the
 *    acoustic axis; cell (i, j, k) has its centre at (i dx, j dx, k dx).
 *  - "dev" marks a device pointer.  The caller allocates and owns every device
 *    buffer, including the workspace (size from bbfd_plan_get_info); the library
 *    allocates no device memory.  Plans own only host data and, once a solve
 *    has been captured, a HIP graph.
 *  - "stream" is a hipStream_t (NULL = legacy default stream).  Device work is
 *    enqueued asynchronously unless stated otherwise.
 *  - Every call returns BBFD_OK (0) or a negative code; no C++ exception
 *    crosses the ABI.  bbfd_last_error() describes the last failure of the
 *    calling thread.
 *  - A plan is immutable once created and may be shared across threads; two
 *    solves in flight at the same time need distinct workspaces.
 */
#ifndef BBFD_H
#define BBFD_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BBFD_OK 0
#define BBFD_EINVAL (-1)    /* bad size, pointer, step count, layer thickness */
#define BBFD_EMATERIAL (-2) /* rho <= 0, Q <= 1, Poisson ratio outside [-1, 0.5) */
#define BBFD_EINDEX (-3)    /* device found a material index >= n_materials */
#define BBFD_EGEOMETRY (-4) /* source plane inside the layer; element at/after it */
#define BBFD_EDIVERGED (-5) /* non-finite value in the peak map */
#define BBFD_EHIP (-6)      /* HIP runtime error */
#define BBFD_ENOMEM (-7)    /* workspace missing or too small */

/* One row of the property table (paper Section 2.2.1, Table 1): density,
   longitudinal and shear speed, longitudinal and shear attenuation in Np/m at
   the drive frequency.  c_s = 0 marks a fluid. */
typedef struct {
  double rho, c_l, c_s, alpha_l, alpha_s;
} bbfd_material;

/* Problem statement (Sections 2.2-2.3 and 3.2).
   dx = 1500 / (freq_hz * ppw) (Section 2.2, PPW in water).
   qc: attenuation correction, Q = Q0 * qc (Section 3.2; 1 = none).
   cfl_safety: fraction of the 3D stability limit used to size dt (0.95).
   pml: absorbing-layer thickness in cells on every face (8 by default).
   capture_start: first step whose end state enters the peak map
                  (< 0: n_steps - 2 periods).
   source_k: plane of the soft stress source (< 0: pml, the first interior
             plane).  The property table is copied at plan creation.
   index_bits: 8 (or 0): the material map is uint8 and the table has up to 256
             rows; 16: the map is uint16 and the table has up to 4096 rows (CT
             values quantised at 12 bits, Section 2.2.2).  With 16-bit maps the
             general kernels stage only the table's buoyancy and edge-input
             columns in LDS (the workspace holds them after the rows) and read
             each cell's moduli through the caches, and only fluids of index
             below 255 take the acoustic kernels. */
typedef struct {
  int32_t nx, ny, nz, pml;
  double freq_hz, ppw, qc, cfl_safety;
  int32_t n_steps, capture_start, source_k;
  int32_t n_materials; /* 1..256 (8-bit maps) or 1..4096 (16-bit maps) */
  const bbfd_material *materials;
  int32_t index_bits;  /* 8 (0 = 8) or 16 */
} bbfd_problem;

/* Single-element transducer (Section 2, "Single").  kind 0: flat piston,
   radius_m = face radius, apex_m = face centre.  kind 1: spherical bowl,
   radius_m = aperture radius, focal_m = radius of curvature, apex_m = apex on
   the axis.  axis: propagation direction (normalised by the library).
   u0: normal surface velocity amplitude (m/s). */
typedef struct {
  int32_t kind;
  double radius_m, focal_m, apex_m[3], axis[3], u0;
} bbfd_transducer;

typedef struct {
  double dx, dt, c_max;       /* grid spacing, time step, fastest unrelaxed speed */
  int32_t steps_per_period;   /* dt = period / steps_per_period */
  int32_t capture_start, source_k, pitch;
  uint64_t workspace_bytes;   /* device workspace a solve needs */
  uint64_t cells;             /* nx * ny * nz */
  int32_t tile_rows;          /* step-kernel tile: 64 x tile_rows x tile_planes cells */
  int32_t tile_planes;
  uint64_t graph_captures;    /* time loops captured so far by bbfd_solve on this plan */
} bbfd_plan_info;

typedef struct bbfd_plan bbfd_plan;

/* Validates the problem and derives, in FP64 on the host, the per-material
   Zener constants (Q from Eq. 3 times qc, one relaxation mechanism at the drive
   frequency), the time step and the absorbing-layer profile; packs them as the
   FP32 device tables.  *out is NULL on failure.  BBFD_EINVAL also when a
   padded field array would exceed 4 GiB (about 1e9 cells): the step kernels
   address arrays by 32-bit byte offsets. */
int bbfd_plan_create(const bbfd_problem *problem, bbfd_plan **out);
int bbfd_plan_get_info(const bbfd_plan *plan, bbfd_plan_info *out);
void bbfd_plan_destroy(bbfd_plan *plan);

/* Host copy of the FP64 per-material constants: n_materials rows of
   (Q_P, Q_S, tau_P, tau_S, pi_R, mu_R, pi_U, mu_U, nu). */
int bbfd_material_constants(const bbfd_plan *plan, double *out, int32_t n_rows);

/* Surface decomposition of the transducer (Section 2.3: elements of area
   lambda^2/16): rings no wider than lambda/4, each split into the fewest
   equal elements no larger than lambda^2/16.  Writes up to cap rows of
   (x, y, z, area) to host memory xyza (may be NULL to count); *n_out gets the
   element count. */
int bbfd_transducer_elements(const bbfd_plan *plan, const bbfd_transducer *t, double *xyza,
                             int64_t cap, int64_t *n_out);

/* Rayleigh-Sommerfeld field of the transducer radiating into water (Section
   2.3) on the source plane z = (source_k + 1/2) dx at the (x, y) cell centres:
     S(x) = (i omega rho_w / 2 pi) sum_e u0 A_e exp(-i k R_e) / R_e
   (e^{+i omega t}); src_re_im (dev) receives 2*nx*ny floats, (re, im)
   interleaved, [ny][nx].  Uses the front of the workspace to stage the
   elements and blocks until they are uploaded.  BBFD_EGEOMETRY if an element
   lies at or beyond the source plane. */
int bbfd_source_rayleigh(const bbfd_plan *plan, const bbfd_transducer *t, float *src_re_im,
                         void *workspace, uint64_t workspace_bytes, void *stream);

/* The same Rayleigh-Sommerfeld field in water at every cell centre of the
   grid, field (dev) = 2*nx*ny*nz floats, complex [nz][ny][nx] (the free
   field of the transducer; its phase is one of the surrogate's inputs).  Same
   staging, blocking and geometry check as bbfd_source_rayleigh. */
int bbfd_rayleigh_volume(const bbfd_plan *plan, const bbfd_transducer *t, float *field,
                         void *workspace, uint64_t workspace_bytes, void *stream);

/* ---- Phased arrays (Section 2: the multi-element transducers, with
   electronic steering and, for refocusing, a point source at the target
   back-propagated to the domain interface and then by Rayleigh-Sommerfeld to
   the elements, Section 2.3).  An element is a flat circular piston driven
   with a complex normal velocity; its surface is decomposed like the single
   piston (rings no wider than lambda/4, equal parts of at most lambda^2/16),
   every part carrying the element's drive. */
typedef struct {
  double radius_m;     /* face radius */
  double centre_m[3];  /* face centre */
  double axis[3];      /* radiating direction (normalised by the library) */
  double w_re, w_im;   /* drive: normal surface velocity u e^{i phi}, m/s */
} bbfd_element;

/* Sub-element decomposition of n elements: up to cap rows of
   (x, y, z, area, w_re, w_im) into host memory out (may be NULL to count);
   *n_out receives the number of sub-elements. */
int bbfd_array_elements(const bbfd_plan *plan, const bbfd_element *elements, int32_t n, double *out,
                        int64_t cap, int64_t *n_out);
/* Rayleigh-Sommerfeld field of the driven array on the source plane, as
   bbfd_source_rayleigh (same layout, staging, blocking and geometry check):
     S(x) = (i omega rho_w / 2 pi) sum_parts w_e A exp(-i k R) / R. */
int bbfd_array_rayleigh(const bbfd_plan *plan, const bbfd_element *elements, int32_t n,
                        float *src_re_im, void *workspace, uint64_t workspace_bytes, void *stream);
/* Electronic steering in water to target (host, m): unit drives with phase
   k |c_e - target| (c_e the element centre), so that every element's wave
   arrives at the target in phase.  w (host) receives 2 n doubles (re, im). */
int bbfd_array_steer(const bbfd_plan *plan, const bbfd_element *elements, int32_t n,
                     const double *target, double *w);
/* Refocusing through the map (time reversal).  (1) The point source at the
   target cell (i, j, k) (k at least two planes beyond the source plane, inside
   the interior), in place of the transducer source: unit z forces pushing
   outward on the two v_z faces of the cell (+1 on face k, -1 on face k - 1),
   which for the near-axial waves a focus collects acts as a monopole, so the
   record is the transfer to the pressure at the target (a single z force
   would give the transfer to v_z, whose sign flips for waves reflected back
   from beyond the target); two solves, one per face, record the complex
   phasor of v_z on the faces of the source plane over the last period,
   (2/N_T) sum v_z exp(-i omega t_n), t_n = (n + 1/2) dt, summed; (2) the Rayleigh
   integral of that plane (normal velocity, cells of area dx^2 at
   z = (source_k + 1/2) dx) to every element centre, p_e; (3) the drives
   w_e = conj(p_e) / |p_e| (host, 2 n doubles).  field (host, may be NULL)
   receives the p_e.  peak (dev) receives the second point-source solve's peak map;
   workspace as bbfd_solve.  Synchronises stream. */
int bbfd_array_refocus(const bbfd_plan *plan, const uint8_t *mat, const bbfd_element *elements,
                       int32_t n, const int32_t *cell, float *peak, double *w, double *field,
                       void *workspace, uint64_t workspace_bytes, void *stream);

/* Full FDTD solve (Eq. 1 with memory variables, absorbing layer, source,
   peak capture), enqueued on stream.  The source field enters as a
   normal-traction jump of 2 S across z = (source_k + 1/2) dx (a force layer on
   the v_z faces there), ramped in over two periods.  Arguments:
     mat (dev)        [nz][ny][nx] material indices into the table: uint8, or
                      uint16 when the problem's index_bits is 16
     src_re_im (dev)  complex source plane as written by bbfd_source_rayleigh
     peak (dev)       float [nz][ny][nx], receives max |p| over the capture
                      window, p = -(sxx + syy + szz)/3
     workspace (dev)  >= workspace_bytes, 256-byte aligned; no need to clear
   The first solve with a given (mat, src, peak, workspace) captures the time
   loop into a HIP graph owned by the plan; later solves with the same
   pointers replay it.  A plan keeps the graphs of its 4 most recently used
   pointer sets (so a skull solve and its water-only companion, or two
   workspaces, alternate without re-capture; bbfd_plan_info.graph_captures
   counts captures) and frees a replaced graph only after its last launch
   has completed.  For plans of 2048 tiles or more, each captured step
   runs as two branches on a second stream the plan owns (the fused step of
   the deep tiles beside the velocity kernels, then the two stress kernels
   side by side); the result is the same bit for bit.  Index and divergence
   errors are detected on the device and reported by bbfd_status. */
int bbfd_solve(const bbfd_plan *plan, const uint8_t *mat, const float *src_re_im, float *peak,
               void *workspace, uint64_t workspace_bytes, void *stream);

/* Same as bbfd_solve but launches kernels directly (no graph). */
int bbfd_solve_direct(const bbfd_plan *plan, const uint8_t *mat, const float *src_re_im,
                      float *peak, void *workspace, uint64_t workspace_bytes, void *stream);

/* Profiling variant of bbfd_solve_direct: records a HIP event before and after
   every kernel of the time loop on stream, waits for the solve, and writes the
   summed kernel times in milliseconds to ms_out[0..4]: the velocity update
   (Eq. 1 rows 1-3) of the acoustic tiles [0] and of the general tiles [1],
   the stress/memory update (rows 4-9) of the acoustic tiles [2] and of the
   general tiles [3], and the fused velocity + stress step of the deep tiles
   [4].  A tile (64 x tile_rows x tile_planes cells, see bbfd_plan_info) is
   acoustic when every one of its row segments is of a lossless-fluid class
   (bbfd_segment_classes) on every plane, and deep when moreover its rows and
   planes clear the y and z absorbing layers by 3 cells, every layer face its
   fused step recomputes in x is one of its own, all cells within 3 of it
   inside the grid hold one fluid and no elastic segment within two rows or
   planes reads its sigma_yy or sigma_zz; such tiles run kernels specialised
   to those cases (bbfd_tile_counts).  Plans of fewer than 2048 tiles run no
   fused step.  Results are identical to bbfd_solve. */
int bbfd_solve_profiled(const bbfd_plan *plan, const uint8_t *mat, const float *src_re_im,
                        float *peak, void *workspace, uint64_t workspace_bytes, void *stream,
                        double *ms_out);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the solve of
   bbfd_solve_direct with the workspace taken from a fixed device array the
   library holds on every GPU it runs on (96 MiB per GPU, held until the
   process ends; enough for grids up to about 64^3 with the default layer).
   Calls no allocating routine: the material and layer tables are uploaded from
   the plan's own host memory.  The caller still passes mat, src and peak
   (layouts as bbfd_solve).  Every call on one GPU shares that GPU's array and
   clears what it needs at the start, so calls that overlap on one GPU (two
   streams, two threads) race: serialise them.  When peak_index or
   peak_value is non-NULL the call waits for stream and returns the status as
   bbfd_status would (BBFD_EINDEX, BBFD_EDIVERGED); otherwise it returns once
   the solve is enqueued.  BBFD_ENOMEM, without enqueuing anything, when the
   plan's workspace_bytes exceeds the array. */
int bbfd_solve_static(const bbfd_plan *plan, const uint8_t *mat, const float *src_re_im,
                      float *peak, void *stream, int64_t *peak_index, float *peak_value);

/* Waits for stream, then reads the device status of the last solve in this
   workspace: BBFD_EINDEX, BBFD_EDIVERGED or BBFD_OK.  peak_index receives the
   linear index (x fastest) of the largest peak value over the interior outside
   the absorbing layer (lowest index on ties), peak_value that value.  Either
   output may be NULL. */
int bbfd_status(const bbfd_plan *plan, const void *workspace, int64_t *peak_index,
                float *peak_value, void *stream);

/* Energy-loss factor of a transcranial solve against its water-only companion
   (Section 2.4, Eq. 2) and the pressure transmission T_S = sqrt(E_L) (Section
   3.2):
     E_L = sum_{x,y} I(x, y, z_m | skull) / sum_{x,y} I(x, y, z_m | water),
     I = P^2 / (2 rho c_l)   (P the peak-pressure map, rho and c_l of the
                              cell's material in the table of plan)
   with the sums over the plane's cells outside the absorbing layer.  Arguments
   (dev, layouts and index width as bbfd_solve, both solved with this plan's
   grid and table):
     mat_skull, peak_skull   map and peak map of the transcranial solve
     mat_water, peak_water   map (typically all water) and peak map of the
                             water-only solve
     z_m                     plane index in [pml, nz - pml), or < 0 for the
                             plane of the water-only map's peak voxel (largest
                             value outside the layer, lowest index on ties)
     workspace (dev)         a solve workspace of this plan; only its
                             reduction scratch is used (enqueue after, or on the
                             stream of, the solves that share it)
     out (host)              5 doubles: E_L, T_S, z_m, the skull sum, the
                             water sum (W m^-2 summed over cells)
   Waits for stream.  BBFD_EDIVERGED when the water-only sum is not positive
   and finite; BBFD_EINVAL for a plane outside the interior. */
int bbfd_energy_loss(const bbfd_plan *plan, const uint8_t *mat_skull, const float *peak_skull,
                     const uint8_t *mat_water, const float *peak_water, int32_t z_m,
                     void *workspace, uint64_t workspace_bytes, void *stream, double *out);

/* Diagnostic: the row-segment classes the last solve in this workspace used.
   Row segment s of row (j, k) covers cells x in [64 s, min(64 s + 64, nx)); its
   class is m + 1 when every cell within two cells of the segment (x, y and z,
   edge cells standing in for cells beyond the grid) holds the same lossless
   fluid material m (zero shear speed and zero attenuation), else 0.  Class m + 1
   segments take the acoustic branch of the step kernels (one normal stress read,
   no memory variables); the result is the same either way.  classes (host)
   receives nseg * ny * nz bytes, nseg = ceil(nx / 64), ordered [nz][ny][nseg];
   n is its size (BBFD_EINVAL if smaller).  Synchronises stream. */
int bbfd_segment_classes(const bbfd_plan *plan, const void *workspace, uint8_t *classes,
                         uint64_t n, void *stream);

/* Diagnostic: the number of tiles of each kind in the last solve in this
   workspace, counts (host, 3 values): acoustic tiles run by the acoustic
   velocity and stress kernels [0], general tiles [1], deep tiles run by the
   fused step [2] (tile kinds as described at bbfd_solve_profiled; their sum is
   the plan's tile count).  Synchronises stream. */
int bbfd_tile_counts(const bbfd_plan *plan, const void *workspace, int32_t *counts, void *stream);

/* ---- Batched sweeps: many independent solves of uneven size in one launch.
   Each problem keeps its own grid, frequency, time step, tables and step count.
   Per time step, four kernels (velocity and stress, each for acoustic and for
   general tiles) walk ragged per-kind (solve, tile) tables ordered by
   decreasing step count, so solves drop out of them once their own step count
   is reached; the blocks are persistent or one per tile (autotuned), and the
   whole sweep is captured in one HIP graph.  For sweeps of solves that each
   fill the GPU, the per-solve shape instead captures every solve's own step
   kernels (acoustic, general and fused deep tiles, as bbfd_solve) one solve
   after the other into the batch's graph.  Results equal those of the same
   problems solved one by one with bbfd_solve, bit for bit. */
typedef struct bbfd_batch bbfd_batch;

/* Creates one plan per problem (same validation and errors as
   bbfd_plan_create, message prefixed with the problem index); batched sweeps
   take 8-bit maps (BBFD_EINVAL for index_bits 16).  A sweep of the
   attenuation correction q_c (Section 3.2) over one map is a batch of problems
   that differ only in qc. */
int bbfd_batch_create(const bbfd_problem *problems, int32_t n, bbfd_batch **out);
void bbfd_batch_destroy(bbfd_batch *batch);
/* workspace_bytes: device workspace of a batched solve (all solves plus the
   tile/descriptor tables).  shape (may be NULL, 4 ints): rows per block,
   persistent blocks (0: one block per tile), z cells per tile, number of
   tiles; all four 0 for the per-solve shape. */
int bbfd_batch_info(const bbfd_batch *batch, uint64_t *workspace_bytes, int32_t *shape);
/* Plan of solve i (owned by the batch) and the byte offset of its part of the
   batch workspace, e.g. for bbfd_source_rayleigh on that solve. */
const bbfd_plan *bbfd_batch_plan(const bbfd_batch *batch, int32_t i);
uint64_t bbfd_batch_offset(const bbfd_batch *batch, int32_t i);
/* Launch shape: by in {1, 2, 4, 8} rows per 64-wide block; blocks >= 1
   persistent blocks, or 0 for one block per tile; kchunk >= 1 z cells per
   tile (>= 4 when by = 1).  by = 0 selects the per-solve shape (blocks and
   kchunk are then ignored).  BBFD_EINVAL for any other shape. */
int bbfd_batch_set_shape(bbfd_batch *batch, int32_t by, int32_t blocks, int32_t kchunk);
/* mat, src, peak: host arrays of n device pointers (layouts as bbfd_solve).
   Captures on first use per pointer set and launch shape; enqueued on stream. */
int bbfd_batch_solve(bbfd_batch *batch, const uint8_t *const *mat, const float *const *src,
                     float *const *peak, void *workspace, uint64_t workspace_bytes, void *stream);
/* bbfd_status for solve i of the last batched solve in this workspace. */
int bbfd_batch_status(const bbfd_batch *batch, const void *workspace, int32_t i,
                      int64_t *peak_index, float *peak_value, void *stream);
/* Tile-shape autotuner: if cache_path names a file holding a line for this
   sweep's size class ("gfx950:n<solves>:c<log1.01 cells>:s<max steps>"), applies
   its shape; otherwise times probe_steps batched steps for every candidate
   tiled shape (direct launches) and probe_steps steps of every solve in the
   per-solve shape (one captured graph) on these inputs (synchronising
   stream), applies the fastest, appends it to cache_path (if given) and
   writes its time to *best_ms.  The workspace contents are overwritten. */
int bbfd_batch_autotune(bbfd_batch *batch, const uint8_t *const *mat, const float *const *src,
                        float *const *peak, void *workspace, uint64_t workspace_bytes,
                        void *stream, const char *cache_path, int32_t probe_steps,
                        double *best_ms);

/* ---- Thermal step (Section 2.4): the Pennes bio-heat transfer equation
     rho C dT/dt = div(k grad T) - w rho_b C_b (T - T_a) + Q
   (rho_b C_b = 1050 * 3617 J m^-3 K^-1 for blood) by explicit finite
   differences on the acoustic grid: Euler steps of dt, the 7-point Laplacian
   with each face's conductivity the harmonic mean of its two cells', and the
   outermost cells of the grid held at T_a (the paper's 37 degC border).  The
   heat source is Q = 2 h alpha_l I, I = p^2 / (2 rho c_l) with p the
   acoustic peak-pressure map, h the share of the longitudinal attenuation
   that turns into heat (the paper uses 0.16 in skull bone) and the result
   times intensity_scale; Q is applied times the duty cycle during the first
   n_on steps and not at all during the n_off steps after them.  Outputs are
   the final temperature, the maximal temperature and the CEM43 thermal dose
     dose = sum over steps of dt/60 * R^(43 - T),  R = 0.5 at T >= 43 degC,
            0.25 below  (minutes; T at the end of each step). */
typedef struct {
  double k;         /* thermal conductivity, W m^-1 K^-1 */
  double c;         /* specific heat, J kg^-1 K^-1 */
  double perfusion; /* blood perfusion w, s^-1 */
  double heat_frac; /* share h of alpha_l turned into heat, in [0, 1] */
} bbfd_thermal;

typedef struct {
  int32_t nx, ny, nz;       /* >= 3 each */
  double dx, dt;            /* grid spacing (m) and time step (s) */
  int32_t n_on, n_off;      /* steps with the ultrasound on, then off */
  double duty;              /* duty cycle while on, in (0, 1] */
  double t_body;            /* T_a: border and initial temperature, degC */
  double intensity_scale;   /* multiplies I (e.g. to reach a requested intensity) */
  int32_t n_materials;      /* 1..256 rows of both tables, indexed like the map */
  const bbfd_material *acoustic; /* rho, c_l and alpha_l (Np/m) are used */
  const bbfd_thermal *thermal;
} bbfd_bhte_problem;

typedef struct bbfd_bhte bbfd_bhte;

/* Validates the problem (BBFD_EINVAL for sizes, steps, duty cycle, or a dt at
   or above the explicit stability limit min over the table of
   rho C / (6 k / dx^2 + w rho_b C_b); BBFD_EMATERIAL for bad properties) and
   derives the per-material coefficients in FP64.  Tables are copied. */
int bbfd_bhte_create(const bbfd_bhte_problem *problem, bbfd_bhte **out);
void bbfd_bhte_destroy(bbfd_bhte *plan);
/* Device workspace a run needs and the stability limit of dt (either may be
   NULL). */
int bbfd_bhte_info(const bbfd_bhte *plan, uint64_t *workspace_bytes, double *dt_max);
/* Runs all n_on + n_off steps on stream (asynchronous).  mat (dev) uint8
   [nz][ny][nx] indices into the tables, peak (dev) float peak-pressure map
   (Pa) of the acoustic solve; outputs (dev, float [nz][ny][nx]): t_final and
   t_max in degC, dose in CEM43 minutes.  workspace (dev, 256-byte aligned)
   >= workspace_bytes.  Indices >= n_materials are not checked here (the
   acoustic solve of the same map reports them). */
int bbfd_bhte_run(const bbfd_bhte *plan, const uint8_t *mat, const float *peak, float *t_final,
                  float *t_max, float *dose, void *workspace, uint64_t workspace_bytes,
                  void *stream);

/* Message of the last error on the calling thread ("" if none). */
const char *bbfd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
