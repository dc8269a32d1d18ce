/*
 * lbm.h - C ABI of the MI355X (gfx950) D2Q37 thermal lattice Boltzmann hot path.
 *
 * The operations follow Calore et al., "Massively parallel Lattice Boltzmann
 * codes on large GPU clusters" (arXiv:1703.00185):
 *   - Sec. 2: the D2Q37 model, the discrete master equation (Eq. 6) with the
 *     shifted equilibrium (Eqs. 4-5), the moments, and the pull form (Eq. 10);
 *   - Sec. 2 (kernel list) and Sec. 4 (Single-GPU Implementation): per time
 *     step, pbc (periodic-x halo columns), propagate, bc (thermal walls on
 *     rows 0..2 and Ly-3..Ly-1) and collide, on a structure-of-arrays lattice
 *     (each population of each column one contiguous run, y fastest; runs
 *     ordered column-major or plane by plane, lbm_layout_kind) in two
 *     copies.  The fused path does propagate + bc + collide in one kernel
 *     and takes periodic x by wrapping instead of pbc.
 * Where the paper is silent the library takes these readings: the 37 hops
 * are the shells (0,0) (1,0) (1,1) (2,0) (2,1) (2,2) (3,0) (3,1) with all
 * images; the weights solve the isotropy conditions through order 8; the
 * equilibrium is the 4th-order Hermite projection of the Maxwellian; a
 * population whose pull source lies beyond a wall is taken from the opposite
 * population of the same site, and bc then resets each wall-row site to
 * rho * K_l(T_wall) (its density times the zero-velocity equilibrium at the
 * wall temperature).  Units: time step 1, hop e_l sites, velocity c_l = r e_l.
 *
 * Conventions for every call:
 *   - Every call returns an lbm_status (0 = success) unless stated; no call
 *     throws.  lbm_last_error() gives the reason of the last failure.
 *   - Device memory is owned by the caller: one block of at least
 *     lbm_required_bytes() bytes, 256-byte aligned, that must outlive the
 *     handle.  The library never allocates or frees device memory (its
 *     one static array, the staging of lbm_get_sites_noalloc, is part of
 *     its code object).
 *   - The HIP stream is owned by the caller.  Calls documented as
 *     asynchronous only enqueue work on it; calls that take or fill host
 *     arrays synchronise it before returning.
 *   - Host arrays are owned by the caller.  Field arrays are [x][y] (y
 *     fastest, Lx*Ly doubles); population arrays are [l][x][y] (37*Lx*Ly
 *     doubles) in the population order returned by lbm_tables().
 *   - A handle is not thread-safe: one thread, one stream per handle.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_NPOP 37

typedef struct lbm_handle lbm_handle;

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,  /* bad argument: NULL pointer, invalid config, n < 0 */
  LBM_ENOMEM = -2,  /* caller's device block too small or misaligned */
  LBM_EDEVICE = -3, /* a HIP call failed (message in lbm_last_error) */
  LBM_ESTATE = -4   /* lattice not initialised (init_rt / set_populations) */
} lbm_status;

/* Storage type of the populations.  Arithmetic is binary64 for all.
 *   LBM_FP32: widened exactly on load, rounded to nearest binary32 on store.
 *   LBM_FP16DEV: binary16 scaled deviation from a per-row reference, the
 *     zero-velocity equilibrium of a reference state with density
 *     rho_ref(y) per row and temperature T_lo on rows y < y_split, T_hi on
 *     rows y >= y_split: c = K_l(T(y)) rho_ref(y) (K_l as in
 *     lbm_wall_factors), stored d = f16(f32((f - c) * (K_l(T(y))^-1 *
 *     rho_ref(y)^-1))), read back as c (1 + d).  The reference comes from
 *     lbm_init_rt (the density of the Rayleigh-Taylor state with a flat
 *     interface, the wall temperatures as the layers, split at the first row
 *     above the interface) or lbm_set_reference.
 * Bytes per population: 8, 4, 2. */
typedef enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16DEV = 2 } lbm_storage;

/* Kernel sequence of lbm_step (Sec. 2 kernel list; fusion as in Sec. 5). */
typedef enum {
  LBM_PATH_SEPARATE = 0, /* pbc, propagate, bc, collide: four kernels */
  LBM_PATH_FUSED = 1,    /* one kernel doing propagate+bc+collide, periodic
                            x by wrapping the source column (no pbc launch,
                            halo columns unused); LBM_FP16DEV lattices whose
                            reference layer boundary lies inside the lattice
                            add a small launch over the (at most two)
                            wavefronts per column that straddle it */
  LBM_PATH_REGIONS = 2,  /* region split (Sec. 5, 1-D tiling): the fused
                            kernel on the bulk columns 3..Lx-4 runs on the
                            bound stream while a second stream refreshes
                            the halos (pbc) and steps the 3 + 3 border
                            columns, ordered by events across steps only;
                            same results as LBM_PATH_FUSED bit for bit */
  LBM_PATH_FUSED2 = 3    /* two steps per launch (temporal blocking; the
                            fusion of Sec. 5 carried across two steps):
                            each wavefront marches along x over a strip of
                            64 rows, steps each column once and the column
                            three behind it a second time, keeping the
                            intermediate populations in registers and LDS,
                            so each site is read and written once per two
                            steps.  LBM_FP64 storage only (EINVAL
                            otherwise); same results as LBM_PATH_FUSED bit
                            for bit.  Interior strips run on the bound
                            stream, the strips holding wall rows on a
                            second stream beside them.  The last step of
                            an lbm_step call with an odd count, and every
                            step of a lattice lower than 64 rows, takes
                            the fused kernel.  Faster than LBM_PATH_FUSED
                            on lattices of several million sites (1.15x at
                            2048 x 8192), slower on small ones */
} lbm_path;

/* Population layout in each lattice copy.  Columns X = 0 .. Lx+5 include
 * 3 halo columns per side (physical column x is X = x + 3); each
 * population of a column is a run of NY contiguous rows (NY >= Ly, rows
 * >= Ly unused), so the lanes of a wavefront, which take consecutive rows,
 * touch one contiguous segment per population: the structure-of-arrays
 * principle of Sec. 4 (Data Structure Analysis).  Element (l, X, y) sits at
 * l * pstride + X * cstride + y (lbm_layout reports both strides). */
typedef enum {
  LBM_LAYOUT_COLUMN = 0, /* f[X][l][y]: the 37 runs of a column back to
                            back (pstride = NY, cstride = 37 NY + pad);
                            the default: a work-group's tile streams
                            through one contiguous column block */
  LBM_LAYOUT_PLANAR = 1  /* f[l][X][y]: one plane per population, as in
                            Sec. 4 (cstride = NY, pstride = (Lx + 6) NY
                            rounded up to 64, + pad) */
} lbm_layout_kind;

/* Single phases for lbm_run_phase and the timing counters. */
typedef enum {
  LBM_PHASE_PBC = 0,       /* copy the periodic-x halo columns (in place) */
  LBM_PHASE_PROPAGATE = 1, /* pull gather into the other buffer */
  LBM_PHASE_BC = 2,        /* thermal walls on the 6 wall rows (in place) */
  LBM_PHASE_COLLIDE = 3,   /* collision into the other buffer */
  LBM_PHASE_FUSED = 4,     /* propagate + bc + collide into the other buffer,
                              periodic x by wrapping (reads no halo) */
  LBM_PHASE_FUSED_BULK = 5,   /* timing only: region path, bulk columns */
  LBM_PHASE_FUSED_BORDER = 6, /* timing only: region path, border columns */
  LBM_PHASE_FUSED2 = 7,       /* timing only: two-step path, interior
                                 strips (one launch per two steps) */
  LBM_NPHASES = 8
} lbm_phase;

typedef struct {
  int32_t lx, ly;    /* physical lattice, Lx >= 3 (halo of 3), Ly >= 6 */
  double tau;        /* relaxation time, > 0.5 */
  double gx, gy;     /* body force per unit mass (lattice units per step) */
  double t_bottom;   /* wall temperature of rows 0..2 (> 0) */
  double t_top;      /* wall temperature of rows Ly-3..Ly-1 (> 0) */
  int32_t storage;   /* lbm_storage */
  int32_t path;      /* lbm_path used by lbm_step */
  int32_t layout;    /* lbm_layout_kind */
  int32_t block;     /* work-group size of the lattice kernels: 64, 128,
                        256, 512 or 1024; 0 selects the default: 64 when
                        Lx * ceil(Ly / 64) < 1024 (fewer wavefronts than
                        SIMDs), else 512 (FP64), 256 (FP32), 64 (FP16DEV),
                        lowered to the smallest power of two >= Ly when
                        that is less */
  int32_t ny_pad;    /* extra elements in the row pitch NY; < 0 default */
  int64_t stride_pad; /* extra elements on the outer stride (cstride for
                         the column layout, pstride for the planar one);
                         < 0 default */
} lbm_config;

/* Rayleigh-Taylor initial state (the initial assignment of Sec. 2; the
 * Rayleigh-Taylor runs of Sec. 6, Overview of Physics Results):
 * T(x,y) = T_m - a tanh((y - y_center - h(x)) / width), with T_m and a
 * the mean and half difference of the wall temperatures, h(x) = sum_k
 * amp[k-1] cos(2 pi k x / Lx + phase[k-1]), k = 1..n_modes, pressure rho T in
 * hydrostatic balance d ln p / dy = r gy / T with p = 1 on the interface,
 * zero velocity, populations at equilibrium. */
typedef struct {
  double width;        /* interface width in sites, > 0 */
  double y_center;     /* interface height in sites */
  int32_t n_modes;     /* 0..LBM_MAX_MODES */
  const double *amp;   /* host array of n_modes amplitudes (sites) */
  const double *phase; /* host array of n_modes phases (radians) */
} lbm_rt_params;

#define LBM_MAX_MODES 32

/* Fill *cfg with defaults for an lx x ly lattice: tau 0.8, g = (0, -1e-4),
 * walls 1.05 (bottom) / 0.95 (top), FP64, fused path, column layout,
 * default tiling. */
int lbm_config_default(lbm_config *cfg, int32_t lx, int32_t ly);

/* Bytes of device memory needed for cfg (two lattice copies with halos,
 * plus the reference of deviation storage: 16 bytes per row and 512); 0
 * if cfg is invalid. */
size_t lbm_required_bytes(const lbm_config *cfg);

/* Bind a lattice to caller memory dev_mem (dev_bytes long) and to the HIP
 * stream `stream` (a hipStream_t; NULL is the null stream).  *out receives
 * the handle.  No GPU work is enqueued.  Errors: EINVAL (NULL arguments,
 * invalid config), ENOMEM (dev_bytes too small or dev_mem not 256-byte
 * aligned), EDEVICE (no usable device). */
int lbm_create(const lbm_config *cfg, void *dev_mem, size_t dev_bytes,
               void *stream, lbm_handle **out);

/* Rebind the handle to another stream (asynchronous calls go there).
 * Errors: EINVAL (NULL handle), ESTATE (the lattice is in an engine). */
int lbm_set_stream(lbm_handle *h, void *stream);

/* Set the Rayleigh-Taylor initial state (see lbm_rt_params); computed on
 * the GPU.  Asynchronous.  Errors: EINVAL (NULL, width <= 0, n_modes out of
 * range, non-finite amp/phase/y_center), EDEVICE. */
int lbm_init_rt(lbm_handle *h, const lbm_rt_params *rt);

/* Advance n >= 0 time steps (Eq. 6: propagate, bc, collide per step, x
 * periodic) with the configured lbm_path.  Asynchronous.  Errors: EINVAL
 * (n < 0), ESTATE (no state yet), EDEVICE. */
int lbm_step(lbm_handle *h, int32_t n);

/* Same steps as lbm_step, replayed from a HIP graph: the first call for a
 * given n and current buffer captures the n steps from this handle's
 * stream (launches only, nothing else may be enqueued on that stream
 * meanwhile) and keeps the instantiated graph until lbm_destroy; later
 * calls launch it.  Removes the per-launch host cost of short steps.
 * Asynchronous.  Errors: EINVAL (n < 0, timing enabled), ESTATE, EDEVICE. */
int lbm_step_captured(lbm_handle *h, int32_t n);

/* Run one phase on the current state (test and profiling hook): PBC and BC
 * work in place, PROPAGATE, COLLIDE and FUSED write the other copy, which
 * then becomes current.  Phases 0..4 only.  Asynchronous.  Errors: EINVAL,
 * ESTATE, EDEVICE. */
int lbm_run_phase(lbm_handle *h, int32_t phase);

/* Per-site moments of the current populations (Sec. 2, under Eq. 6):
 * rho = sum f, rho u = sum c f, 2 rho T = sum |c - u|^2 f, into host arrays
 * of Lx*Ly doubles each ([x][y]); any of them may be NULL.  Uses the idle
 * lattice copy as scratch.  Synchronises the stream. */
int lbm_moments(lbm_handle *h, double *rho, double *ux, double *uy, double *T);

/* Global sums of the current state: out[0] mass sum f, out[1..2] momentum
 * sum c f, out[3] energy (1/2) sum |c|^2 f, out[4] number of populations that
 * are NaN or infinite.  Deterministic (fixed reduction order).  Uses the
 * idle lattice copy as scratch.  Synchronises the stream. */
int lbm_conservation(lbm_handle *h, double out[5]);

/* Copy the current populations to / from a host array [37][Lx][Ly]
 * (checkpoint and restore; restore marks the state initialised), through
 * the storage codec, one population at a time staged in the idle lattice
 * copy.
 * Synchronise the stream.  Deviation storage needs a reference first. */
int lbm_get_populations(lbm_handle *h, double *host);
int lbm_set_populations(lbm_handle *h, const double *host);

/* Populations of n selected sites of the current state: out[l * n + i] =
 * f_l(xs[i], ys[i]), host arrays, 0 <= xs[i] < Lx, 0 <= ys[i] < Ly (checked
 * on the host: EINVAL otherwise).  n may be at most lbm_layout()[4] / 304.
 * Uses the idle lattice copy as scratch.  Synchronises the stream. */
int lbm_get_sites(lbm_handle *h, int32_t n, const int32_t *xs, const int32_t *ys, double *out);

/* For callers that cannot allocate device memory or use the lattice's idle
 * copy (code that must not call hipMalloc, tight serving loops): the same
 * gather as lbm_get_sites, same arguments and results bit for bit, with
 * its device staging (the gathered populations and the coordinates) in a
 * fixed array of the library, one per GPU, held from the first call on that
 * GPU until the process ends: LBM_NOALLOC_MAX_SITES * 304 bytes (2.4 MiB).
 * Calls no allocating routine; the idle lattice copy is not touched.
 * n may be at most LBM_NOALLOC_MAX_SITES (EINVAL otherwise).  Every call on
 * one GPU shares that array: calls that overlap on one GPU (other threads,
 * other streams) race and must be serialised by the caller.  Nothing in the
 * array needs to start cleared.  Synchronises the stream. */
#define LBM_NOALLOC_MAX_SITES 8192
int lbm_get_sites_noalloc(lbm_handle *h, int32_t n, const int32_t *xs, const int32_t *ys, double *out);

/* Deviation storage only: set / read the reference state: rho_ref[Ly]
 * (host array, finite and > 0), the layer temperatures t_lo (rows
 * y < y_split) and t_hi (rows y >= y_split), finite, > 0 and with every
 * K_l(t) > 0, and 0 <= y_split <= Ly (t_lo = t_hi = 1 gives c =
 * w_l rho_ref(y)).  Setting it uploads rho_ref, 1 / rho_ref and the 32
 * layer factors into the caller's block after the two lattice copies,
 * synchronises the stream and invalidates the stored state (set
 * populations or init again).  On get, t_layers and y_split may be NULL.
 * Errors: EINVAL (other storage, bad values), ESTATE (no reference yet,
 * get only). */
int lbm_set_reference(lbm_handle *h, const double *rho_ref, double t_lo, double t_hi, int32_t y_split);
int lbm_get_reference(lbm_handle *h, double *rho_ref, double t_layers[2], int32_t *y_split);

/* Per-phase kernel timing with HIP events recorded on the bound stream
 * around every launch while enabled.  lbm_read_timing synchronises the
 * stream, writes the summed milliseconds and launch counts per lbm_phase,
 * and resets the counters. */
int lbm_set_timing(lbm_handle *h, int32_t enable);
int lbm_read_timing(lbm_handle *h, double ms[LBM_NPHASES], int64_t count[LBM_NPHASES]);

/* Geometry of the bound lattice: out[0] columns NX = Lx + 6 (3 halo
 * columns each side), out[1] row pitch NY (elements), out[2] pstride and
 * out[3] cstride (elements; element (l, X, y) at l pstride + X cstride + y),
 * out[4] bytes of one lattice copy, out[5] work-group size in use. */
int lbm_layout(const lbm_handle *h, int64_t out[6]);

/* Model constants as the library uses them (host only, no GPU): hops
 * e[37][2], opposite index opp[37], weights w[37], velocity scale r.  Any
 * pointer may be NULL. */
int lbm_tables(int32_t *e, int32_t *opp, double *w, double *r);

/* Wall factors K_l(T) = w_l [1 + th (C_l-2)/2 + th^2 (C_l^2 - 8 C_l + 8)/8],
 * th = T - 1, C_l = r^2 |e_l|^2, as bc applies them (host only). */
int lbm_wall_factors(double t_wall, double out[LBM_NPOP]);

/* Bandwidth probe: the copy micro-benchmark of Sec. 4 (Fig. misalignment)
 * that chose pull over push.  Copies between two caller device buffers of
 * `bytes` bytes (a multiple of 16, both 16-byte aligned) on `stream`,
 * asynchronously:
 *   LBM_PROBE_COPY: dst[i] = src[i], all bytes, in 16-byte vectors (four
 *                   per lane per pass, non-temporal loads and stores);
 *   LBM_PROBE_MRAW: dst[64 + i] = src[64 + i + shift] (misaligned read);
 *   LBM_PROBE_ARMW: dst[64 + i + shift] = src[64 + i] (misaligned write);
 * for MRAW/ARMW elements are doubles, i < bytes / 8 - 128 and |shift| <= 64,
 * so every access stays inside both buffers.  bytes >= 2048.  It touches no
 * lattice state.
 * Errors: EINVAL (NULL, misaligned, bad mode or shift), EDEVICE. */
typedef enum { LBM_PROBE_COPY = 0, LBM_PROBE_MRAW = 1, LBM_PROBE_ARMW = 2 } lbm_probe;
int lbm_probe_bandwidth(int32_t mode, const void *src, void *dst, size_t bytes, int32_t shift,
                        void *stream);

/* ------------------------------------------------------------------------
 * Ensemble engine: many independent lattices stepped together, one
 * persistent launch per time step (the step of Eq. 6 for every lattice,
 * fused as above, periodic x by wrapping the source column instead of pbc),
 * replayed from a HIP graph built once.  Lattices are existing handles
 * (LBM_FP64 or LBM_FP32 storage, any sizes, each with its own tau, g and
 * walls); each keeps its own step count and stops when it reaches zero.
 * The engine owns no lattice memory: its own device block (caller-owned,
 * lbm_engine_required_bytes) holds the slot table only.
 *
 * While a lattice is in an engine, the engine steps it on the engine's
 * stream (the handle is rebound to that stream, and back to its own when it
 * leaves the engine); lbm_set_stream, lbm_step, lbm_run_phase, lbm_init_rt,
 * lbm_set_populations and lbm_set_reference on it fail with ESTATE; reads (moments, conservation, populations, sites) first
 * synchronise with the engine.  lbm_destroy of such a handle removes it
 * from its engine first.
 * ---------------------------------------------------------------------- */
typedef struct lbm_engine lbm_engine;

/* Engine schedules (how the persistent grid takes tiles): CHUNKED = one
 * contiguous run of tiles per work-group, dealt to its wavefronts in turn;
 * STRIDED = tiles dealt round-robin over all wavefronts.  A tile is one
 * wavefront: 64 rows of one column of one lattice. */
typedef enum { LBM_SCHED_CHUNKED = 0, LBM_SCHED_STRIDED = 1 } lbm_schedule;

/* Bytes of device memory for an engine with max_slots lattices; 0 if
 * max_slots is outside [1, 2^20]. */
size_t lbm_engine_required_bytes(int32_t max_slots);

/* Create an engine on caller memory (256-byte aligned) and stream.
 * Default tiling: block 256, 256 work-groups per compute unit, STRIDED.
 * Errors: EINVAL, ENOMEM (block too small / misaligned), EDEVICE. */
int lbm_engine_create(int32_t max_slots, void *dev_mem, size_t dev_bytes, void *stream,
                      lbm_engine **out);

/* Add lattice h with `steps` steps to run; *slot receives its slot index.
 * Synchronises h's stream first.  Errors: EINVAL (NULL, other storage,
 * other device, steps < 0), ESTATE (h not initialised or already in an
 * engine), ENOMEM (no free slot), EDEVICE. */
int lbm_engine_add(lbm_engine *e, lbm_handle *h, int32_t steps, int32_t *slot);

/* Take the lattice of `slot` out of the engine (its state stays in its
 * handle, at the step it reached) and rebind the handle to the stream it
 * had when it was added.  Synchronises the engine stream. */
int lbm_engine_remove(lbm_engine *e, int32_t slot);

/* Enqueue n engine steps (asynchronous): each lattice with steps left
 * advances one step per engine step. */
int lbm_engine_step(lbm_engine *e, int32_t n);

/* Synchronise and report steps left per slot (steps_left[max_slots];
 * -1 for a free slot; may be NULL).  Finished lattices leave the tile table. */
int lbm_engine_status(lbm_engine *e, int32_t *steps_left);

/* Tiling: block (work-group size 64, 128, 256 or 512: 1 to 8 wavefronts),
 * persistent groups, and lbm_schedule.  set_tiling rebuilds the step
 * graph. */
int lbm_engine_set_tiling(lbm_engine *e, int32_t block, int32_t groups, int32_t schedule);
int lbm_engine_get_tiling(const lbm_engine *e, int32_t out[3]);

/* Autotune the tiling on the current lattices: times `reps` step launches
 * (without advancing any lattice: each launch rewrites the idle buffer from
 * the current one) for every block in {64,128,256,512}, groups in
 * {2,4,...,1024} x compute units and both schedules; keeps the fastest.
 * out[3] = chosen (block, groups, schedule), *best_ms = its time per step
 * (either may be NULL).  Errors: ESTATE (no active lattice), EDEVICE. */
int lbm_engine_tune(lbm_engine *e, int32_t reps, int32_t out[3], double *best_ms);

/* Reason of the last engine failure (per engine, or per thread for NULL). */
const char *lbm_engine_last_error(const lbm_engine *e);

/* Release the engine; its lattices keep their state (cur written back). */
void lbm_engine_destroy(lbm_engine *e);

/* Reason of the last failure on h, or of the last failed lbm_create /
 * lbm_required_bytes on this thread when h is NULL.  Never NULL. */
const char *lbm_last_error(const lbm_handle *h);

/* Release the host-side handle (not the caller's memory or stream).  Waits
 * for the handle's pending work.  NULL is accepted. */
void lbm_destroy(lbm_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
