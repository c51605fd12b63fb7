/*
 * rs.h -- C ABI of librs, MI355X (gfx950) synthesis of FMCW TDM-MIMO beat
 * cubes where every rendered pixel is a point scatterer.
 *
 * Signal model (Sec. II).  For an M-Tx / N-Rx array, eq. (1) gives the beat
 * signal of Tx m and Rx r at fast-time sample n_s and TDM block l as a
 * sigma-weighted exp(j 2 pi (2 mu R / c * (n_s - 1)/F_s - f_D (l - 1) T_b));
 * eq. (2) sums that over the N_az x N_el rendered pixels.  This library keeps
 * every virtual channel c = m*N + r separate and uses exact per-channel ranges
 * (not eq. (2)'s far-field angle term), 0-based indices:
 *
 *   Y[c][l][n] = sum_p a_p exp(j 2 pi (psi_{p,c} + b_{p,c} n - beta_p l))
 *
 *   R_{p,c}   = (|x_p - tx_m| + |x_p - rx_r|) / 2       (eq. (1)'s R_{m,n})
 *   psi_{p,c} = 2 fc R_{p,c} / c0   carrier phase carried by sigma; 0 when
 *                                    rs_radar.carrier_phase == 0 (sigma = a)
 *   b_{p,c}   = 2 mu R_{p,c} / (c0 Fs)   beat frequency, cycles per sample
 *   beta_p    = 2 fc v_p Tb / c0         Doppler f_D = 2 v fc / c0 times T_b
 *
 * a_p is the pixel strength (eq. (2)'s P_r, applied as an amplitude) and v_p
 * its radial velocity (eq. (2)'s V), positive when approaching.  T_b is the
 * TDM block period (one block holds M chirps).  The intra-block Tx slot
 * offset, residual video phase, intra-chirp Doppler and a strength that
 * changes from block to block are not in this form of eq. (1); each is
 * available as a variant (rs_model_flags).
 *
 * Two forms compute Y:
 *   RS_FORM_FP64_DIRECT   binary64 phasors and binary64 complex
 *                         multiply-accumulate on the vector ALUs;
 *   RS_FORM_MFMA_SPLIT16  binary64 phase arguments reduced mod 1, binary32
 *                         phasors split into hi + lo binary16 parts, and the
 *                         per-channel complex contraction
 *                         Y_c = F_c^T diag(sigma_c) D done on fp16 matrix
 *                         cores with fp32 accumulation (hi*hi + hi*lo +
 *                         lo*hi).  Typical relative L2 error vs an exact
 *                         binary64 sum: 1e-6 .. 1e-5.
 *   RS_FORM_NUFFT         per channel a two-dimensional type-1 non-uniform
 *                         FFT from the points (b, -beta) onto the Ns x L
 *                         modes: binary64 phase arguments, float32
 *                         spreading with an exponential-of-semicircle
 *                         kernel onto a grid oversampled >= 2x, float32
 *                         FFTs and deconvolution.  An approximation sized
 *                         by a tolerance (rs_cube_plan_nufft; 1e-6 from
 *                         rs_cube_plan): relative L2 error vs the exact sum
 *                         of about the tolerance, float32 rounding
 *                         (~1e-6) below.  Work grows with P C w^2 +
 *                         C Ns L log, not P C Ns L.  The grid sums are
 *                         formed in a fixed order (bitwise reproducible)
 *                         while each 256-pixel block's box of grid cells
 *                         (or its two sub-boxes, for a block whose points
 *                         fall into two row groups) fits 1,024 cells and
 *                         512 columns; larger boxes are added with atomics
 *                         and then the last bits vary from run to run.
 *                         Workspace grows with P (8 KiB per block and
 *                         channel).  Limits: Ns, L <= 2048, strengths
 *                         constant over the blocks; batches run frame by
 *                         frame, sessions are refused (RS_E_UNSUPPORTED).
 *
 * Conventions
 *   - Every call returns rs_status; nothing throws or aborts across the ABI.
 *     rs_last_error() gives thread-local text for the last non-OK status.
 *   - Pixel and cube buffers are caller-owned DEVICE memory on the plan's
 *     device.  Calls taking a `hip_stream` (a hipStream_t, NULL = the null
 *     stream) only enqueue work: buffers must stay valid until the stream has
 *     passed the work.
 *   - Cube layout: [C = M*N][L][Ns] row-major, n fastest, interleaved
 *     (re, im); complex64 (2 x float32) or complex128 (2 x float64).
 *   - Pixel positions are metres in the radar frame, float32 structure of
 *     arrays.  Per-pixel values are not validated (NaN in gives NaN out).
 *     Aliasing is not an error: beat frequencies above Fs and |f_D T_b| > 1/2
 *     wrap as the equation defines.
 *   - P = 0 is valid and writes an exact zero cube.
 */
#ifndef RS_H
#define RS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RS_OK = 0,
    RS_E_INVALID = 1,     /* bad argument; nothing was launched or written      */
    RS_E_NOMEM = 2,       /* device or host allocation failed                   */
    RS_E_DEVICE = 3,      /* a HIP runtime call failed (text: rs_last_error)     */
    RS_E_UNSUPPORTED = 4, /* valid request this build cannot serve               */
    RS_E_BUSY = 5,        /* session queue full (back-pressure); retry later     */
    RS_E_NOT_FOUND = 6    /* unknown session ticket                              */
} rs_status;

typedef enum { RS_FORM_FP64_DIRECT = 0, RS_FORM_MFMA_SPLIT16 = 1, RS_FORM_NUFFT = 2 } rs_form;
typedef enum { RS_C64 = 0, RS_C128 = 1 } rs_dtype; /* interleaved (re, im) */

/* Signal-model variants (bit flags, rs_radar.model; 0 = the model above).
 * Each changes only the per-(pixel, channel) phase arguments psi and b, in
 * binary64, in this order:
 *   RS_MODEL_FAR_FIELD    eq. (2): the beat frequency and the carrier
 *                         phase use the range from the array origin
 *                         Rp = |x|, and the channels differ by eq. (2)'s
 *                         angle-of-arrival term, the first-order path
 *                         change across the array:
 *                         psi = Rp Kc - s (2 fc / c0), b = Rp Kb, with
 *                         s = u.(tx_m + rx_r)/2 and u = x / Rp.  With
 *                         carrier_phase = 0 (Kc = 0) this is eq. (2) as
 *                         printed: sigma = a, and channel c = m N + r of a
 *                         lambda/2 ULA on +x gets the phase c sin(theta)/2
 *                         with sin(theta) = -u_x (theta measured toward -x).
 *                         With carrier_phase = 1 it is the far-field limit
 *                         of the exact model.  Pixels must not sit at the
 *                         origin.
 *   RS_MODEL_RVP          residual video phase of the dechirped echo,
 *                         -mu tau^2 / 2 with tau = 2 R / c0:
 *                         psi -= R^2 (2 mu / c0^2), R the beat range
 *   RS_MODEL_TDM_SLOT     Tx m transmits in slot m of each block, at
 *                         l Tb + m Tb / M (eq. (1) uses l Tb for all Tx):
 *                         psi -= beta m / M
 *   RS_MODEL_INTRA_CHIRP  Doppler shift within the chirp, with the sign of
 *                         the slow-time term: b -= v (2 fc / (c0 Fs))
 * and one changes the strength instead:
 *   RS_MODEL_BLOCK_STRENGTH  eq. (1)'s sigma_{m,n,l} varies with the TDM
 *                         block l (the same for every channel): a_p becomes
 *                         a_{p,l}, and rs_pixels.amp points to float32
 *                         [L][P], the strength of pixel p in block l at
 *                         amp[l * P + p] (L * P values per frame).
 * Range migration over the CPI is not modelled by any variant. */
typedef enum {
    RS_MODEL_FAR_FIELD = 1,
    RS_MODEL_TDM_SLOT = 2,
    RS_MODEL_INTRA_CHIRP = 4,
    RS_MODEL_RVP = 8,
    RS_MODEL_BLOCK_STRENGTH = 16
} rs_model_flags;

/* eq. (1) signal model, SI units.  tx_xyz / rx_xyz are HOST arrays
 * [M][3] / [N][3] of antenna positions in metres; they are copied by
 * rs_cube_plan and may be freed on return. */
typedef struct {
    int32_t M, N, Ns, L;     /* Tx, Rx, fast-time samples, TDM blocks (>= 1)   */
    double fc, mu, Fs, Tb, c0; /* Hz, Hz/s, Hz, s, m/s (Fs, Tb, c0 > 0)        */
    const double *tx_xyz, *rx_xyz;
    int32_t carrier_phase;   /* 1: sigma = a exp(j 2 pi 2 fc R / c0); 0: a     */
    int32_t model;           /* rs_model_flags, 0 = eq. (1) as above            */
} rs_radar;

/* One frame of rendered pixels, caller-owned DEVICE pointers, float32 SoA:
 * x, y, z, vr hold P values; amp holds P values, or L * P ([L][P]) when the
 * plan's model has RS_MODEL_BLOCK_STRENGTH.  Array lengths cannot be
 * checked: shorter arrays are read out of bounds. */
typedef struct {
    int64_t P; /* >= 0; pointers may be NULL when P == 0 */
    const float *x, *y, *z, *amp, *vr;
} rs_pixels;

typedef struct rs_plan rs_plan;
typedef struct rs_session rs_session;

/* ---------------------------------------------------------------- plans -- */

/* Validate `radar`, derive the phase constants, copy the antenna geometry to
 * the current HIP device and choose the tile configuration.  max_pixels
 * bounds P for every later call on this plan (>= 0).
 * Errors: RS_E_INVALID (M, N, Ns or L < 1, M*N*L*Ns > 2^31, Fs, Tb or c0 <= 0,
 * unknown model flags,
 * any non-finite parameter, NULL tx/rx, bad form or dtype, max_pixels < 0),
 * RS_E_NOMEM, RS_E_DEVICE.  On success *out owns device memory until
 * rs_plan_destroy.  A plan is immutable and may be used from several threads
 * and streams at once. */
rs_status rs_cube_plan(const rs_radar *radar, rs_form form, rs_dtype dtype,
                       int64_t max_pixels, rs_plan **out);

/* A plan of the NUFFT form for a tolerance in [1e-7, 0.5): kernel width
 * w = ceil(log10(1/tolerance)) + 1 cells (at most 8), shape beta = 2.30 w,
 * grid the smallest power of two >= max(2 Ns, 2 w) by >= max(2 L, 2 w).
 * Errors: as rs_cube_plan, RS_E_INVALID for a tolerance outside the range,
 * RS_E_UNSUPPORTED for RS_MODEL_BLOCK_STRENGTH, Ns or L > 2048, more than
 * 65,535 channels, max_pixels >= 2^31, or channels x grid rows (in l) or
 * channels x Ns reaching 2^24. */
rs_status rs_cube_plan_nufft(const rs_radar *radar, rs_dtype dtype, int64_t max_pixels,
                             double tolerance, rs_plan **out);

/* Bytes of device workspace rs_beat_synthesize_ws needs for P pixels
 * (0 <= P <= max_pixels).  Errors: RS_E_INVALID. */
rs_status rs_plan_workspace_bytes(const rs_plan *plan, int64_t P, size_t *bytes);

/* Matrix-core tile configurations are named "WNxTLxNW" -- rows per wave x
 * columns (l) x waves per workgroup; the library builds 64x128x4, 32x128x4,
 * 32x128x8, 32x64x4, 32x64x8, 64x64x4, 64x64x8 and 128x64x4 -- with an
 * optional suffix 'i' on the 8-wave shapes.  8-wave shapes run two waves
 * per SIMD with their matrix and vector work phase-shifted against each
 * other; with 'i' they run the software-pipelined interleave (each wave
 * alternates matrix groups with staged slices of phasor work), which the
 * 4-wave shapes always run (the suffix is accepted there and changes
 * nothing).  The two schedules of a shape give the same cube bit for bit;
 * different shapes chunk the pixels differently and so differ in the last
 * bits, all within the form's error. */

/* Sets the matrix-core tile configuration of `plan` (see above).  It changes
 * the plan: call it before the plan is shared, never while other calls use
 * it.  Errors: RS_E_INVALID (NULL plan, or a string that is not a built
 * configuration), RS_E_UNSUPPORTED (plans of the other forms). */
rs_status rs_plan_set_tile(rs_plan *plan, const char *tile);

/* Chooses the matrix-core tile configuration of `plan` by measurement:
 * every built configuration (the eight shapes, and the three 8-wave shapes
 * again with 'i') synthesises `pixels` into `cube` once to warm up and
 * `reps` times timed with HIP events on `hip_stream`, and the one with the
 * smallest mean time is kept (the plan's own choice otherwise comes from a
 * rule measured on the frame and batch workloads).  The call synchronises
 * the stream and leaves the last synthesis in `cube`.  It changes the plan:
 * call it before the plan is shared, never while other calls use it.  Plans
 * of the other forms are left unchanged.  chosen (may be NULL) receives the
 * configuration string (an empty string for the other forms).
 * Errors: as rs_beat_synthesize, RS_E_INVALID for reps < 1. */
rs_status rs_plan_tune(rs_plan *plan, const rs_pixels *pixels, void *cube, int32_t reps,
                       void *hip_stream, char *chosen, size_t chosen_len);

/* rs_plan_tune with a persistent cache of its choices: a text file at
 * cache_path (host path), one entry per line "C Ns L Pb TILE" keyed by the
 * channel count, N_s, L and Pb, the pixel count rounded up to a power of
 * two, TILE a configuration string as above.  On a hit (the last
 * well-formed line with the plan's key and a built configuration) the plan
 * takes that configuration and nothing is launched; on a miss the
 * configuration is tuned as rs_plan_tune does (the cube is synthesised) and
 * the entry appended with one write.  A missing file is an empty cache;
 * lines that do not parse are skipped.  Concurrent callers may both tune
 * and both append; the later line wins.  Plans of the other forms are left
 * unchanged (chosen: empty string, no file access).
 * Errors: as rs_plan_tune, RS_E_INVALID for a NULL cache_path; a file that
 * exists but cannot be read or appended to gives RS_E_INVALID. */
rs_status rs_plan_tune_cached(rs_plan *plan, const rs_pixels *pixels, void *cube, int32_t reps,
                              void *hip_stream, const char *cache_path, char *chosen, size_t chosen_len);

/* Human-readable description of the plan (form, tile, chunking) into buf
 * (always NUL-terminated when len > 0).  Errors: RS_E_INVALID. */
rs_status rs_plan_describe(const rs_plan *plan, int64_t P, char *buf, size_t len);

/* Enqueue the synthesis of one cube on `hip_stream`.  Split-K workspace is
 * taken from the device's stream-ordered pool and returned in stream order.
 * Errors: RS_E_INVALID (NULL plan/pixels/cube, P < 0 or > max_pixels, NULL
 * pixel pointer with P > 0), RS_E_NOMEM, RS_E_DEVICE. */
rs_status rs_beat_synthesize(rs_plan *plan, const rs_pixels *pixels, void *cube,
                             void *hip_stream);

/* As rs_beat_synthesize with caller-provided device workspace of at least
 * rs_plan_workspace_bytes(plan, P) bytes (256-byte aligned).  The workspace
 * must not be used by other work until the stream has passed this call. */
rs_status rs_beat_synthesize_ws(rs_plan *plan, const rs_pixels *pixels, void *cube,
                                void *workspace, size_t workspace_bytes, void *hip_stream);

/* Size of the static device array that rs_beat_synthesize_noalloc uses as
 * its workspace (one array per device, held until the process ends). */
#define RS_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * rs_beat_synthesize with no allocation at all.  The workspace that
 * rs_beat_synthesize_ws takes from the caller (rs_plan_workspace_bytes) comes
 * from a static device array of RS_STATIC_SCRATCH_BYTES bytes per device
 * instead; the kernels and their chunking are those of rs_beat_synthesize,
 * so the cube is bitwise the same.  The caller still passes the pixels and
 * the cube.  The array's address is looked up once per device, on the first
 * call there (hipGetSymbolAddress).  Every call on one device shares that
 * device's array and nothing in it carries over from call to call (each call
 * writes every workspace entry it reads), but calls that overlap in time on
 * one device -- different streams, or threads without ordering -- race on it
 * and give wrong cubes; calls in order on one stream are safe.  Calls on
 * different devices use different arrays.
 * Errors: as rs_beat_synthesize_ws; RS_E_INVALID (nothing launched) when the
 * plan's workspace for P pixels exceeds RS_STATIC_SCRATCH_BYTES (the
 * matrix-core plan of a 3 x 4 array with Ns 256 and L 128 needs at most
 * 63 MiB whatever P, its binary64 plain form twice that, which is refused);
 * RS_E_UNSUPPORTED for device ordinals >= 64. */
rs_status rs_beat_synthesize_noalloc(rs_plan *plan, const rs_pixels *pixels, void *cube,
                                     void *hip_stream);

/* Enqueue `nframes` cubes that share one plan (e.g. consecutive animation
 * frames with different pixel counts) as ONE persistent launch over all
 * frames' work items plus one reduction launch (NUFFT plans: the frames'
 * launches one after another on one workspace).  frames: HOST array of
 * nframes rs_pixels (device pointers inside); cubes: device buffer of
 * nframes consecutive cubes.  Each frame's cube is bitwise identical to
 * rs_beat_synthesize on that frame alone (for the NUFFT form where every
 * box fits its tile slot, as there).
 * Errors: as rs_beat_synthesize, plus nframes < 0. */
rs_status rs_beat_synthesize_batch(rs_plan *plan, const rs_pixels *frames, int32_t nframes,
                                   void *cubes, void *hip_stream);

void rs_plan_destroy(rs_plan *plan);

/* ------------------------------------------------------------- sessions -- */
/* A session is a serving loop with continuous batching: a scheduler thread
 * admits queued cube requests while a slot is free and the request's split-K
 * partial sums fit the session's HBM arena (hbm_budget), cuts the admitted
 * requests' work into time slices of about slice_terms terms, and runs each
 * slice as persistent MFMA-form launches that mix work items of all admitted
 * requests.  A request that arrives while others run is admitted as soon as
 * memory and a slot free up; requests that fit may overtake one that does
 * not (at most 64 times, then it is admitted first), unless strict_fifo is
 * set.  A request's cube is bitwise identical whatever else runs beside it.
 *
 * Shares of a slice (policy):
 *   RS_SCHED_SHORTEST  slices as large as equal shares would make them,
 *                      given to the requests with the least work left first
 *                      (shortest remaining processing time) after a floor of
 *                      1/8 of an equal share for every admitted request so
 *                      that none stalls: small requests finish within a
 *                      slice or two, large ones take the rest of each slice;
 *   RS_SCHED_EQUAL     an equal share of slice_terms for each admitted
 *                      request with work left (processor sharing); a slice
 *                      is shorter when the requests need less than that. */

typedef enum { RS_SCHED_SHORTEST = 0, RS_SCHED_EQUAL = 1 } rs_sched_policy;

typedef struct {
    int32_t device;       /* HIP device ordinal                                  */
    size_t hbm_budget;    /* bytes of session workspace (partial sums) in flight */
    int32_t max_slots;    /* requests admitted at once (>= 1)                    */
    int32_t queue_cap;    /* requests queued before submit returns RS_E_BUSY     */
    int32_t slice_items;  /* > 0: per request and slice about this many work
                             items x 256-pixel steps (overrides slice_terms)      */
    int32_t policy;       /* rs_sched_policy                                      */
    int32_t strict_fifo;  /* 1: admit in arrival order only                       */
    int32_t reserved;     /* 0 */
    double slice_terms;   /* terms per slice; 0 = 1.2e11 (~2 ms of matrix work)  */
} rs_session_opts;

typedef enum {
    RS_REQ_QUEUED = 0, RS_REQ_RUNNING = 1, RS_REQ_DONE = 2, RS_REQ_FAILED = 3,
    RS_REQ_CANCELLED = 4
} rs_request_state;

typedef struct {
    int64_t t_submit_ns, t_admit_ns, t_done_ns; /* host CLOCK_MONOTONIC */
} rs_timing;

/* footprint_*: arena bytes held by admitted requests (what admission
 * counts: the session allocates nothing else per request).  request_bytes_*:
 * the HBM the admitted requests use in all -- their pixels (20 B per pixel,
 * L x 4 + 16 B with strengths per block) and cubes, which the caller owns,
 * plus the arena bytes.  device_error: 1 once a device error has stopped
 * the session (text: rs_last_error after a failing submit). */
typedef struct {
    int64_t submitted, admitted, done, failed, cancelled, launches;
    int64_t queued_now, running_now;
    size_t footprint_now, footprint_peak;
    double terms_done;
    size_t request_bytes_now, request_bytes_peak;
    int32_t device_error, reserved;
} rs_session_stats;

/* Start a session and its scheduler thread on opts->device.
 * Errors: RS_E_INVALID (bad options: max_slots outside 1..4096, queue_cap
 * < 1, slice_items < 0, unknown policy, slice_terms < 0 or not finite),
 * RS_E_NOMEM, RS_E_DEVICE.
 * After a device error (a failed launch reported by the device, or a failing
 * completion query) the session stops: every admitted and queued request
 * ends RS_REQ_FAILED, its arena range is freed, later submits return
 * RS_E_DEVICE, and drain and destroy still return. */
rs_status rs_session_create(const rs_session_opts *opts, rs_session **out);

/* Queue one request: synthesize `pixels` with `plan` (which must use
 * RS_FORM_MFMA_SPLIT16 and outlive the request) into `cube`.  The pixel and
 * cube device buffers are borrowed until poll reports DONE, FAILED or
 * CANCELLED; pixel data must already be complete on the device.
 * Errors: RS_E_INVALID (bad arguments, or a footprint that can never fit
 * hbm_budget), RS_E_BUSY (queue full), RS_E_UNSUPPORTED (plan form). */
rs_status rs_session_submit(rs_session *s, const rs_plan *plan, const rs_pixels *pixels,
                            void *cube, uint64_t *ticket);

/* State of a ticket (rs_request_state) and its timestamps (timing may be
 * NULL).  Errors: RS_E_NOT_FOUND. */
rs_status rs_session_poll(rs_session *s, uint64_t ticket, int32_t *state, rs_timing *timing);

/* Cancel a request that is still queued.  Errors: RS_E_NOT_FOUND,
 * RS_E_BUSY (already admitted). */
rs_status rs_session_cancel(rs_session *s, uint64_t ticket);

/* Block until every submitted request has finished. */
rs_status rs_session_drain(rs_session *s);

rs_status rs_session_stats_get(rs_session *s, rs_session_stats *out);

/* Drain, stop the scheduler thread and free the session. */
void rs_session_destroy(rs_session *s);

/* Test hook: make the next `count` launches of this session report failure
 * without running, so their requests end FAILED (host-side; no kernel is
 * affected). */
rs_status rs_session_inject_failure(rs_session *s, int32_t count);

/* Test hook: the next completion check of this session reports a device
 * error (host-side; the device is not touched), which stops the session as a
 * real one would. */
rs_status rs_session_inject_device_error(rs_session *s);

/* ------------------------------------------------- scenes on the device -- */
/* The paper obtains each frame's pixels (range, strength, angle, velocity)
 * from a rendered image (Sec. II, the paragraph after eq. (1)).  These calls
 * ray-cast the synthetic stand-in scene on the device instead, so that a
 * batch of frames never passes through host memory: an axis-aligned room
 * [-W/2, W/2] x [0, D] x [-H/2, H/2] seen from the origin (boresight +y,
 * array axis +x) and an optional ellipsoid pedestrian.
 *   pixel p = j * g_az + i, azimuth -60 + 120 (i + 1/2) / g_az degrees,
 *   elevation -30 + 60 (j + 1/2) / g_el degrees, unit ray
 *   u = (cos el sin az, cos el cos az, sin el);
 *   t = nearest positive hit on the walls x = +-W/2, y = D, z = +-H/2, or on
 *   the ellipsoid |(x - c) / s| = 1 when that is nearer (it occludes);
 *   position t u, strength |cos incidence| / t^2 * noise[p], radial velocity
 *   -(v . u) on the pedestrian, 0 on the walls.
 * Geometry in binary64, stored as float32 structure of arrays. */
typedef struct {
    double room_w, room_d, room_h;  /* metres */
    int32_t pedestrian;             /* 1: the ellipsoid below is present */
    int32_t reserved;               /* 0 */
    double centre[3];               /* ellipsoid centre, metres */
    double velocity[3];             /* m/s */
    double semi_axes[3];            /* metres, > 0 */
} rs_scene;

/* Render `nframes` scenes over one g_az x g_el grid (P = g_az g_el pixels
 * per frame).  scenes: HOST array [nframes] (copied in stream order).
 * noise: device [nframes][P] strength factors (e.g. lognormal draws), or
 * NULL for 1.  x, y, z, amp, vr: device [nframes][P] outputs, frame f at
 * offset f P -- ready for rs_pixels / rs_beat_synthesize_batch.
 * Errors: RS_E_INVALID (NULL scenes or outputs with nframes > 0,
 * nframes < 0, g_az or g_el < 1, P * nframes > 2^31, non-positive or
 * non-finite room or semi-axes), RS_E_NOMEM, RS_E_DEVICE. */
rs_status rs_render_scenes(const rs_scene *scenes, int32_t nframes, int32_t g_az, int32_t g_el,
                           const float *noise, float *x, float *y, float *z, float *amp, float *vr,
                           void *hip_stream);

/* -------------------------------------------------- range-Doppler maps -- */
/* The processing the paper applies to each simulated cube (Sec. III): an FFT
 * over each coherent processing interval (one cube) gives the range-Doppler
 * map, and the velocity of the map's strongest cell, one per CPI, forms the
 * Doppler-time series that is compared with the ground-truth velocity.
 *
 *   X_c[k][d] = sum_l sum_n Y[c][l][n] exp(-j2pi k n / Ns) exp(+j2pi d l / L)
 *   power[k][d] = sum_c |X_c[k][d]|^2         (non-coherent over channels)
 *
 * Range: forward DFT over fast time, bin k at range k c0 Fs / (2 mu Ns).
 * Doppler: inverse-sign DFT over blocks, so that a scatterer approaching at
 * v (Y ~ exp(-j2pi beta l), beta = 2 fc Tb v / c0) peaks at bin d = beta L;
 * bins are in natural order, d >= L/2 meaning d - L, velocity
 * d_signed c0 / (2 fc Tb L).  Rectangular window, no normalisation.
 * The peak is the largest power over all (k, d) -- over d != 0 when
 * skip_static is set, which removes scatterers at rest (a static scatterer
 * lands exactly in bin d = 0) -- ties going to the smallest k L + d. */
typedef struct {
    int32_t range_bin;    /* k, 0 .. Ns-1 */
    int32_t doppler_bin;  /* signed d, -L/2 .. L/2-1; > 0 approaching */
    float power;          /* power[k][d] */
    float range_m;        /* k c0 Fs / (2 mu Ns) */
    float velocity_mps;   /* d c0 / (2 fc Tb L) */
    float reserved;       /* 0 */
} rs_rd_peak;

/* Range-Doppler processing of `nframes` consecutive cubes made with `plan`
 * (its radar and output dtype; either form).  cubes: device
 * [nframes][C][L][Ns] as written by the synthesis calls.  Outputs, all
 * device memory, each may be NULL:
 *   power         float32 [nframes][Ns][L]  (range-major, Doppler fastest)
 *   doppler_time  float32 [nframes][L]      power[k_peak][.] of each frame:
 *                                           its velocity spectrum at the peak
 *   peaks         rs_rd_peak [nframes]
 * Arithmetic in float32 with twiddles from binary64: for Ns = 256 and
 * L in 16..128 each channel's 2-D FFT runs in registers and LDS within one
 * workgroup and the channels' power is summed in registers (partial maps
 * of the workgroups that share a frame are added in a fixed order); other
 * shapes take two passes of radix-2 LDS FFTs.  Deterministic.
 * Needs Ns and L powers of two, Ns <= 4096, L <= 1024 (else
 * RS_E_UNSUPPORTED).  Temporary device memory
 * (rs_range_doppler_workspace_bytes) is allocated and freed in stream
 * order.
 * Errors: RS_E_INVALID (NULL plan or cubes with nframes > 0, nframes < 0),
 * RS_E_UNSUPPORTED, RS_E_NOMEM, RS_E_DEVICE.  nframes = 0 does nothing. */
rs_status rs_range_doppler(rs_plan *plan, const void *cubes, int32_t nframes, int32_t skip_static,
                           float *power, float *doppler_time, rs_rd_peak *peaks, void *hip_stream);

/* Device bytes of temporary memory that rs_range_doppler uses for
 * `nframes` cubes of `plan`, with (power_given = 1) or without a caller's
 * power map; 0 for nframes <= 0 or a NULL plan. */
size_t rs_range_doppler_workspace_bytes(const rs_plan *plan, int32_t nframes, int32_t power_given);

/* rs_range_doppler with the temporary memory in `workspace` (device memory
 * of workspace_bytes >= rs_range_doppler_workspace_bytes(plan, nframes,
 * power != NULL), 256-byte aligned, owned by the caller and not used by
 * anything else until the stream reaches the end of the call): no
 * allocation.  Same results bit for bit.  Errors: as rs_range_doppler, and
 * RS_E_INVALID for a NULL, misaligned or too small workspace. */
rs_status rs_range_doppler_ws(rs_plan *plan, const void *cubes, int32_t nframes, int32_t skip_static,
                              float *power, float *doppler_time, rs_rd_peak *peaks, void *workspace,
                              size_t workspace_bytes, void *hip_stream);

/* --------------------------------------------------------- kernel timer -- */
/* Per-launch timing of the main (contraction) kernel with HIP events, for
 * profiling.  A timer attached to the calling thread records an event pair
 * around every main-kernel launch made by rs_beat_synthesize* and
 * rs_beat_synthesize_batch, and around the ray-cast kernel of
 * rs_render_scenes, from that thread, on the launch's stream, until
 * `capacity` launches are recorded.  Create and read on the plan's device. */
typedef struct rs_kernel_timer rs_kernel_timer;

/* Errors: RS_E_INVALID (capacity < 1), RS_E_NOMEM, RS_E_DEVICE. */
rs_status rs_kernel_timer_create(int32_t capacity, rs_kernel_timer **out);
/* Attach to / detach from the calling thread (NULL detaches). */
rs_status rs_kernel_timer_attach(rs_kernel_timer *t);
/* Wait for the recorded launches and copy up to `max` durations in
 * milliseconds into ms (may be NULL); *count = launches recorded.  Resets the
 * timer.  Errors: RS_E_INVALID, RS_E_DEVICE. */
rs_status rs_kernel_timer_read(rs_kernel_timer *t, double *ms, int32_t max, int32_t *count);
void rs_kernel_timer_destroy(rs_kernel_timer *t);

/* ---------------------------------------------------------------- misc -- */
const char *rs_last_error(void);
const char *rs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RS_H */
