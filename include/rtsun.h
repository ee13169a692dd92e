/*
 * rtsun.h -- C ABI of the MI355X library for refractive radio ray tracing
 * through a gridded corona with step-wise ray-tube magnification and thermal
 * free-free transfer.
 *
 * Paper: "Modeling the Thermal Low-Frequency Radio Sun with Ray Tracing".
 * The calls follow its statement of the problem: a coronal grid of electron
 * density and temperature (Sec. 3.1), frequencies in 40-800 MHz (Sec. 1) and
 * an observer image plane (Sec. 3.2) go in; brightness-temperature maps
 * (Sec. 3.3) and optionally the recorded ray paths with their geometric
 * factors (Sec. 3.2, Figs. 4 and 6) come out.
 *
 * Units: lengths in solar radii (6.957e10 cm), n_e in cm^-3, T in K,
 * frequencies in Hz, brightness temperatures in K.
 *
 * Conventions shared by every call:
 *  - Status codes only; nothing throws across the ABI.  On failure the
 *    thread-local message of rt_last_error_message() says why.
 *  - Every argument and host-side value is validated before any device work.
 *    RT_OK from a trace call means the work is enqueued on `hip_stream`
 *    (a hipStream_t, NULL = the null stream); device faults surface at the next
 *    call or at the caller's synchronisation as RT_E_DEVICE.
 *  - Per-ray outcomes (exit, hit, miss, step limit) are data in rt_ray_info,
 *    not errors.
 *  - The caller owns every input and output buffer.  The library owns an
 *    rt_model's device copy until rt_model_free, and its own scratch.
 *  - Library scratch (per-pixel launch table, work counters, path-ray list,
 *    beam intermediate, adjoint workspace) is kept per device and per stream:
 *    calls on one stream run in order and share it, calls on different streams
 *    use their own, so calls on different streams do not race.  Scratch grows
 *    on demand; an outgrown table is retired, not freed, so that a HIP graph
 *    that captured a trace call stays valid after later, larger calls (the
 *    adjoint workspace is freed when outgrown, and rt_trace_adjoint refuses
 *    graph capture).  A captured graph uses the tables of the stream it was
 *    captured on: replaying it while another call runs on that stream races.
 *  - A call on a model makes the model's device the calling thread's current
 *    HIP device (and leaves it so); rt_model_load makes `device` current.
 *  - Grid limits (RT_E_CAPACITY): n0 * n1 < 2^24, the packed row length
 *    (n2 + 1 for spherical grids, n2 for Cartesian) < 2^24, and
 *    n0 * n1 * (packed row length) <= 2^31 - 1.
 */
#ifndef RTSUN_H
#define RTSUN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RT_ABI_VERSION 1u

typedef enum {
  RT_OK = 0,
  RT_E_INVALID_ARG = 1,      /* bad pointer, size, descriptor field or version */
  RT_E_NONFINITE_INPUT = 2,  /* NaN/Inf, n_e < 0 or T <= 0 in model values */
  RT_E_OUT_OF_MEMORY = 3,    /* device allocation failed or RT_MAX_DEVICE_BYTES exceeded */
  RT_E_DEVICE = 4,           /* no device, or a HIP runtime error */
  RT_E_UNSUPPORTED = 5,      /* valid but not implemented combination */
  RT_E_CAPACITY = 6,         /* a fixed-size limit of the library was exceeded */
  RT_E_INTERNAL = 7
} rt_status;

/* Per-ray termination codes (rt_ray_info.code). */
enum {
  RT_RAY_EXIT_OUTER = 1,  /* left through the outer sphere r = r_max */
  RT_RAY_HIT_INNER = 2,   /* reached the inner sphere r = r_in */
  RT_RAY_MISS = 3,        /* impact parameter >= r_max: never entered */
  RT_RAY_MAX_STEPS = 4,   /* step limit reached */
  RT_RAY_NONFINITE = 5    /* state became NaN/Inf */
};
/* rt_ray_info.flags */
enum { RT_RAY_FLAG_MARGINAL = 2 /* last-step fraction lambda within 1e-4 of 0 or 1 */ };

/* ------------------------------------------------------------------------
 * Model (Sec. 3.1: global corona on a spherical (r, theta, phi) grid).
 * ------------------------------------------------------------------------ */
typedef enum {
  /* vertices r_a = r_in (r_max/r_in)^(a/(n0-1)), theta_b = (b+1/2) pi/n1,
     phi_c = 2 pi c/n2 (periodic); n0, n1 >= 2, n2 >= 3 */
  RT_GRID_SPHERICAL_LOGR = 0,
  /* vertices origin[k] + i*spacing[k], edge-clamped; n0, n1, n2 >= 2 */
  RT_GRID_CARTESIAN = 1
} rt_grid_kind;

typedef struct {
  uint32_t abi_version;   /* RT_ABI_VERSION */
  uint32_t kind;          /* rt_grid_kind */
  int32_t n0, n1, n2;     /* (N_r, N_theta, N_phi) or (N_x, N_y, N_z) */
  int32_t _reserved;
  double r_in, r_max;     /* termination spheres; spherical grids span [r_in, r_max].
                             For Cartesian grids r_in <= 0 disables the inner sphere. */
  double origin[3];       /* Cartesian only */
  double spacing[3];      /* Cartesian only, > 0 */
} rt_grid_desc;

typedef struct rt_model rt_model;  /* opaque: device-resident packed model */

/* Load a model.  ne, te: HOST arrays, float32, C-order [n0][n1][n2], read
 * before the call returns.  Values must be finite, ne >= 0, te > 0.
 * The packed device copy (n_e, index-space vertex gradient, T) is built on
 * `device`, ordered on `hip_stream`; the call synchronises that stream.
 * On success *out owns the device memory until rt_model_free. */
rt_status rt_model_load(const rt_grid_desc* desc, const float* ne, const float* te, int32_t device,
                        void* hip_stream, rt_model** out);

/* Replace a model's values (same shape).  on_device = 0: host pointers,
 * validated on the host; on_device = 1: device pointers on the model's device,
 * validated by a device reduction (this synchronises `hip_stream`);
 * on_device = 2: device pointers to the natural logarithms ln n_e, ln T (the
 * variables of the differentiable forward), exponentiated on the device and
 * then validated like on_device = 1.  Must not race a trace that reads the same
 * model. */
rt_status rt_model_update(rt_model* model, const float* ne, const float* te, int32_t on_device,
                          void* hip_stream);

/* Free a model (NULL is a no-op).  Synchronises the device first. */
void rt_model_free(rt_model* model);

/* ------------------------------------------------------------------------
 * Observer image plane (Sec. 3.2): parallel rays launched from the observer.
 * o = obs_dir / |obs_dir| (Sun -> observer), u = up x o (normalised), v = o x u.
 * Pixel (j, i), j along u, i along v, has centre (-half_u + (j+1/2) 2 half_u/nu,
 * -half_v + (i+1/2) 2 half_v/nv).  The ray starts on the r_max sphere and
 * travels along -o; impact parameter >= r_max gives RT_RAY_MISS.
 * ------------------------------------------------------------------------ */
typedef struct {
  double obs_dir[3];
  double up[3];
  int32_t nu, nv;
  double half_u, half_v;
} rt_image_desc;

/* rt_params.flags */
enum {
  RT_USE_MAGNIFICATION = 1u << 0,  /* geometric d ln S/ds term (Eqs. 2-3, 7-12) */
  RT_USE_REFRACTION = 1u << 1,     /* off: straight lines of sight, n taken as 1 (Sec. 3.3) */
  RT_PREC_ALL_FP32 = 1u << 2,      /* everything in FP32: ray state, step increments, grid
                                      index (cell + FP32 fraction), the area estimate of
                                      Eqs. 9-11 and the transfer accumulators.  Default
                                      (no precision flag): model evaluations in FP32,
                                      state, increments, grid index, area and transfer in
                                      FP64 */
  RT_SCHED_PLAIN = 1u << 3,        /* one launch per (model, frequency) image instead of
                                      one persistent launch over all of them */
  RT_DETERMINISTIC_GRAD = 1u << 4, /* reserved (rt_trace_adjoint: RT_E_UNSUPPORTED) */
  RT_CARRIED_TUBE = 1u << 5,       /* the ray-tube cross-section S of Eqs. 2-3 from two
                                      neighbour rays launched perturb_ratio*ds_max away
                                      across the initial direction (Eq. 6 basis) and
                                      stepped beside the ray for its whole length, in
                                      place of the per-step retrace of Eqs. 7-11:
                                      ln M of a step = ln(S_{i+1}/S_i), S = |(dr_a x dr_b)
                                      . p/|p||, dr the separations at equal t.  Needs
                                      RT_USE_REFRACTION | RT_USE_MAGNIFICATION
                                      (RT_E_INVALID_ARG otherwise); default precision only
                                      (RT_E_UNSUPPORTED with RT_PREC_ALL_FP32 or
                                      RT_PREC_FP32_STEP); always one
                                      launch per image; rt_autotune: RT_E_INVALID_ARG;
                                      rt_trace_adjoint: RT_E_UNSUPPORTED */
  RT_PREC_FP32_STEP = 1u << 6,     /* FP32 stepping: ray state, step increments and grid
                                      index in FP32; the area estimate (differences of
                                      perturbed neighbour rays, Eqs. 9-11) and the optical
                                      depth / brightness accumulation (Eqs. 2-3, 12) in
                                      FP64.  RT_PREC_ALL_FP32 takes precedence */
  RT_TEST_NO_ABSORPTION = 1u << 30 /* kappa = 0 (tests of I*S = const, Eq. 1) */
};

typedef struct {
  uint32_t abi_version;     /* RT_ABI_VERSION */
  uint32_t flags;
  double ds_max;            /* step rule dt = ds_max / max(n(r_i), n_floor) (arc length <= ds_max) */
  double n_floor;           /* in (0, 1]; 1 gives the fixed dt = ds_max of Sec. 2.1 */
  int32_t max_steps;        /* >= 1 */
  int32_t checkpoint_every; /* adjoint: ray-state checkpoint interval K (>= 1; 0 selects 64) */
  double perturb_ratio;     /* eta of Eq. 8, > 0 */
  double tb_inner_K;        /* boundary brightness behind a ray that reaches r_in */
  double tb_sky_K;          /* boundary brightness behind a ray that leaves (or misses) */
} rt_params;

/* Fill *p with defaults: magnification + refraction, ds_max 0.005, n_floor 1,
 * max_steps 200000, checkpoint_every 64, eta 1e-2, tb_inner 1e4 K, tb_sky 0. */
void rt_params_default(rt_params* p);

typedef struct {
  int32_t n_steps;      /* central steps taken, the truncated last one included */
  int8_t code;          /* RT_RAY_* */
  int8_t flags;         /* RT_RAY_FLAG_* */
  int8_t _pad[2];
  float exit_pos[3];    /* end point (on the crossed sphere for EXIT/HIT) */
  float tau;            /* total optical depth */
  float ln_s_end;       /* ln(S_end / S_0) = sum lambda_i ln M_i (Fig. 6) */
  float r_min;          /* smallest |r| among step points */
} rt_ray_info;          /* 32 bytes */

typedef struct {
  unsigned long long ray_steps;   /* sum of n_steps over all rays of the call */
  unsigned int max_steps;         /* largest n_steps */
  unsigned int code_count[6];     /* rays per code (index = code) */
  unsigned int _pad;
} rt_trace_stats;                 /* 40 bytes */

/* Launch tuning of the persistent (batched) trace.  Every setting gives
 * bitwise-identical maps: each lane traces its own ray with the same
 * arithmetic, only the order in which rays are taken up changes.
 *  refill_min_idle: a wave takes up new rays once at least this many of its
 *    64 lanes are idle (1..64; 64 = whole waves only).
 *  blocks_per_cu: 256-thread blocks per compute unit (0 = the most that fit).
 *  xcd_bands: 8 = the tiles are split into 8 contiguous bands of image rows,
 *    one per die, each with its own claim counter (waves of a die start in
 *    their band and take from the others when it is empty); 1 = one queue. */
typedef struct {
  uint32_t abi_version;     /* RT_ABI_VERSION */
  int32_t refill_min_idle;
  int32_t blocks_per_cu;
  int32_t xcd_bands;
} rt_tuning;

/* Defaults: refill_min_idle 64, blocks_per_cu 0, xcd_bands 8. */
void rt_tuning_default(rt_tuning* t);

/* Per-device tuning used by later persistent traces on `device` (the library
 * keeps one per device; rt_get_tuning reads it back).  RT_E_INVALID_ARG for
 * values out of range. */
rt_status rt_set_tuning(int device, const rt_tuning* t);
rt_status rt_get_tuning(int device, rt_tuning* t);

/* Autotuner: times every candidate tuning (refill_min_idle in {64, 32, 16, 8,
 * 1} x blocks_per_cu in {1 .. the most that fit} x xcd_bands in {8, 1}) on a
 * sample of the call - the same models and image, at most `max_freqs`
 * frequencies spread over freq_hz - and installs the fastest as the device's
 * tuning.  Each candidate's maps are compared with the first candidate's and
 * must be bitwise identical (RT_E_INTERNAL otherwise).  best (HOST, may be
 * NULL) receives the chosen tuning, best_ms and default_ms (HOST, may be NULL)
 * the sample's time with it and with the defaults.  Synchronises hip_stream;
 * allocates its own device buffers for the sample's maps. */
rt_status rt_autotune(const rt_model* const* models, int32_t n_models, const double* freq_hz, int32_t n_freq,
                      const rt_image_desc* image, const rt_params* params, int32_t max_freqs, rt_tuning* best,
                      double* best_ms, double* default_ms, void* hip_stream);

/* Trace maps for every (model, frequency) pair.
 *  models[n_models]: all on one device (the call makes it current), sharing
 *    one grid descriptor; at most 16.  n_freq <= 128.
 *  freq_hz[n_freq]: HOST array, each > 0.
 *  tb_out: DEVICE float32 [n_models][n_freq][nv][nu] (required).
 *  info_out: DEVICE rt_ray_info with the same shape, or NULL.
 *  stats_out: DEVICE rt_trace_stats, or NULL; overwritten.
 *  Paths (optional, all NULL/0 to disable): path_rays = HOST sorted, distinct
 *  flat ray indices into the tb_out shape; path_out = DEVICE float32
 *  [n_path_rays][path_capacity][9] records (x, y, z, s, ln M, d ln S/ds,
 *  tau, n_e, T) per step after the step; path_len_out = DEVICE int32
 *  [n_path_rays] (steps recorded, <= path_capacity; longer paths are
 *  truncated and the ray's flags are unaffected).
 * RT_SCHED_PLAIN selects one launch per image; otherwise one persistent launch
 * covers all rays and refills lanes whose ray has finished.  Both give
 * bitwise-identical results. */
rt_status rt_trace_maps(const rt_model* const* models, int32_t n_models, const double* freq_hz,
                        int32_t n_freq, const rt_image_desc* image, const rt_params* params,
                        float* tb_out, rt_ray_info* info_out, rt_trace_stats* stats_out,
                        const int32_t* path_rays, int32_t n_path_rays, int32_t path_capacity,
                        float* path_out, int32_t* path_len_out, void* hip_stream);

/* rt_trace_maps without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments and results as rt_trace_maps (bitwise
 * equal), without path outputs.  The per-call tables (claim counters, the
 * per-pixel launch table, n_e at the start points) live in a fixed device array
 * of RT_STATIC_SCRATCH_BYTES per device, held from the library's first use on
 * that device until the process ends; a call needs
 * 256 + ceil256(48 nu nv) + 4 nu nv n_models bytes of it (RT_E_CAPACITY beyond:
 * a 1024 x 1024 image with up to 3 models fits).  Every call of this entry
 * point on a device shares that array and leaves its contents behind: calls
 * that overlap in time on one device (different streams, or a replayed graph
 * beside another call) race; issue them on one stream.  Errors as
 * rt_trace_maps. */
#define RT_STATIC_SCRATCH_BYTES (64u << 20)
rt_status rt_trace_maps_static(const rt_model* const* models, int32_t n_models, const double* freq_hz,
                               int32_t n_freq, const rt_image_desc* image, const rt_params* params,
                               float* tb_out, rt_ray_info* info_out, rt_trace_stats* stats_out,
                               void* hip_stream);

/* Reverse-mode gradient of L = sum_{f,i,j} w[f][i][j] T_b[f][i][j] with
 * respect to ln n_e and ln T at every grid vertex, for one model: the exact
 * derivative of the discrete forward of rt_trace_maps (Sec. 2.1 Eq. 4 ray
 * equations, Eqs. 5-11 perturbation retracing and magnification, Eqs. 2-3 and
 * 12 transfer with the geometric term), every discrete choice (cells, step
 * count, termination) held fixed.
 *  freq_hz[n_freq]: HOST array, each > 0 (n_freq <= 128).
 *  weights: DEVICE float32 [n_freq][nv][nu] (caller-owned; rays with w = 0 are
 *    traced forward for the loss but not swept backward).
 *  loss_out: DEVICE double scalar, overwritten with L.
 *  grad_ln_ne, grad_ln_te: DEVICE float32 [n0][n1][n2] (C order), overwritten.
 *  tb_out: DEVICE float32 [n_freq][nv][nu] or NULL; the maps of rt_trace_maps
 *    with the same params, up to rounding (the adjoint kernels are compiled
 *    per tracing mode, so their arithmetic may be contracted differently).
 * Each ray is traced forward with its state checkpointed every
 * params->checkpoint_every steps (0 selects 64); a ray longer than 128
 * checkpoints doubles its interval.  The reverse sweep recomputes each chunk of
 * steps from its checkpoint, recording every step's start state and the model
 * values its adjoint needs (188 bytes a step), and then sweeps the chunk
 * backward from that record.  The image tiles (8 x 8 pixels of one frequency)
 * are traced and swept in batches whose checkpoints (up to 10 KB a ray) fit an
 * 8 GiB budget (the environment variable RT_ADJOINT_CHECKPOINT_BYTES, read at
 * each call, sets another; at least one tile is taken per batch).  Channel
 * adjoints are accumulated per lane and cell in FP32 and added into an FP64
 * per-vertex accumulator with atomics, so the last bits can vary between runs.  Default precision only: RT_PREC_ALL_FP32, RT_PREC_FP32_STEP,
 * RT_DETERMINISTIC_GRAD and RT_TEST_NO_ABSORPTION return RT_E_UNSUPPORTED.  The
 * library keeps a workspace per device and stream (checkpoints, chunk
 * records, accumulator), grown on demand and kept until the process ends; a
 * call issued while `hip_stream` is being captured into a graph returns
 * RT_E_UNSUPPORTED.
 * Errors: RT_E_INVALID_ARG for NULL or inconsistent arguments, RT_E_CAPACITY,
 * RT_E_OUT_OF_MEMORY, RT_E_DEVICE; nothing is written on a validation error. */
rt_status rt_trace_adjoint(const rt_model* model, const double* freq_hz, int32_t n_freq,
                           const rt_image_desc* image, const rt_params* params, const float* weights,
                           double* loss_out, float* grad_ln_ne, float* grad_ln_te, float* tb_out,
                           void* hip_stream);

/* Beam FWHM in R_sun of an interferometer with maximum baseline `baseline_m`
 * (metres) at each frequency: lambda / B radians over the angle 1 R_sun
 * subtends at 1 au (the beam scale of the paper's convolved maps, Sec. 3.3;
 * the form lambda / B is this library's reading).  freq_hz, fwhm_out: HOST
 * [n].  Errors: RT_E_INVALID_ARG for NULL pointers, n < 1, a baseline or a
 * frequency that is not finite and > 0. */
rt_status rt_beam_fwhm(const double* freq_hz, int32_t n, double baseline_m, double* fwhm_out);

/* Maps convolved with a Gaussian beam (the interferometric beam the paper
 * applies to its synthetic maps, Sec. 3.3).  maps_in, maps_out: DEVICE float32
 * [n_maps][nv][nu] in the rt_trace_maps layout (pixel centres
 * -half + (j + 1/2) 2 half / n), distinct.  fwhm: HOST [n_maps] beam full
 * width at half maximum in R_sun (0: the map is copied).  The beam is sampled
 * at pixel offsets, w(k) ~ exp(-k^2 / 2 sigma^2) with sigma = FWHM /
 * (2 sqrt(2 ln 2)) in pixels along each axis, cut at |k| <= ceil(5 sigma) and
 * normalised to sum 1; it is applied along u, then along v, with zero beyond
 * the image edges.  n_maps <= 128.  Uses library scratch of the maps' size.
 * Errors: RT_E_INVALID_ARG, RT_E_CAPACITY, RT_E_OUT_OF_MEMORY, RT_E_DEVICE. */
rt_status rt_beam_convolve(const float* maps_in, float* maps_out, int32_t n_maps, int32_t nu, int32_t nv,
                           double half_u, double half_v, const double* fwhm, void* hip_stream);

/* Mean T_b of each map over the pixels whose centre lies within `radius`
 * (R_sun) of the image centre: the disc-centre brightness-temperature spectrum
 * when the maps are the frequencies of one model (Sec. 3.4.1).  maps: DEVICE
 * float32 [n_maps][nv][nu]; mean_out: DEVICE double [n_maps] (0 when no pixel
 * centre is inside).  Sums in FP64.  Errors: RT_E_INVALID_ARG, RT_E_CAPACITY,
 * RT_E_DEVICE. */
rt_status rt_disc_mean(const float* maps, int32_t n_maps, int32_t nu, int32_t nv, double half_u, double half_v,
                       double radius, double* mean_out, void* hip_stream);

/* Measurement probe (not part of the method): the streaming read bandwidth
 * that the tracer's gathers are compared with.  Allocates a device buffer of
 * `bytes` on `device` (zero-filled; freed before return) and launches `blocks`
 * 256-thread blocks, each reading `span_bytes` of it with float4 loads `reps`
 * times: span_bytes = bytes makes every block read the whole buffer (from one
 * die's L2 when bytes is at most its 4 MiB); span_bytes = bytes / blocks
 * partitions it (from the 256 MB Infinity Cache or from HBM, by size).
 * gbps_out: HOST double, bytes requested / kernel time (hipEvents around one
 * launch after an untimed one) in GB/s.  Synchronises the stream.  Errors:
 * RT_E_INVALID_ARG (bytes or span_bytes not a positive multiple of 16,
 * span_bytes > bytes, blocks outside [1, 2^20], reps outside [1, 4096]),
 * RT_E_OUT_OF_MEMORY, RT_E_DEVICE. */
rt_status rt_probe_read_bandwidth(int32_t device, int64_t bytes, int64_t span_bytes, int32_t blocks, int32_t reps,
                                  double* gbps_out, void* hip_stream);

/* Measurement probe: cell keys of recorded ray paths, the input of
 * rt_probe_gather_replay.  path, path_len: DEVICE, as written by rt_trace_maps
 * ([n_walks][path_capacity][9] float32 records, int32 lengths); keys_out: DEVICE
 * int32 [path_capacity][n_walks], for record s of walk w the key
 * (a n1 + b) n2p + c of the model cell holding its point (the tracer's cell
 * clamping; n2p = n2 + 1 on spherical grids, n2 otherwise), -1 from the walk's
 * length on.  Errors: RT_E_INVALID_ARG, RT_E_CAPACITY (n_walks x path_capacity
 * above 2^31-1), RT_E_DEVICE. */
rt_status rt_probe_path_keys(const rt_model* model, const float* path, const int32_t* path_len, int32_t n_walks,
                             int32_t path_capacity, int32_t* keys_out, void* hip_stream);

/* Measurement probe: gather-only replay of recorded cell walks with the model's
 * layout and the tracer's per-lane cell cache (8 corners of float4 n_e/gradient
 * and float T gathered into LDS when a walk's key changes, read back every
 * step), one lane per walk, no ray arithmetic.  keys: DEVICE int32
 * [path_capacity][n_walks] from rt_probe_path_keys (a key < 0 or beyond the
 * grid ends the walk).  ms_out: HOST double, kernel time of one launch after
 * an untimed one (hipEvents).  Synchronises the stream.  Errors:
 * RT_E_INVALID_ARG, RT_E_CAPACITY, RT_E_OUT_OF_MEMORY, RT_E_DEVICE. */
rt_status rt_probe_gather_replay(const rt_model* model, const int32_t* keys, int32_t n_walks, int32_t path_capacity,
                                 double* ms_out, void* hip_stream);

const char* rt_status_string(rt_status s);
const char* rt_last_error_message(void);
uint32_t rt_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RTSUN_H */
