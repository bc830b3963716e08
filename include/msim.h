/*
 * msim: moving-source image-source synthesis on MI355X (gfx950).
 *
 * C-ABI of the synthesis library.  Implements the moving image-source model of
 * "Fast Algorithm for Moving Sound Source" (arXiv 2508.03065):
 *
 *   y_c[n] = sum_i g_i(n) * (x fractionally delayed by D_i(n) samples)       (Eq. 2, Eq. 8)
 *
 * over every image source i of a shoebox room with total reflection order
 * |mx|+|my|+|mz| <= K (image-source method, Sec. II-A, Eq. 1), with
 *   D_i(n) = fs * tau_i(n),  tau_i = d_i / c                                   (Sec. II-C-3)
 *   g_i(n) = beta_i / (4 pi c tau_i(n)),  beta_i = prod of wall coefficients   (Sec. II-A, after Eq. 2)
 * The delay is sampled on an order-tiered grid (low orders at the audio rate,
 * high orders decimated) and interpolated back to the audio rate (Sec. II-C-3).
 * The fractional delay is a T-tap Kaiser-windowed sinc, an FIR truncation of the
 * ideal sinc response of Sec. II-B, read from an oversampled table.
 *
 * Conventions
 *  - Geometry in FP64, SI units; signals in FP32.
 *  - Walls are ordered x=0, x=Lx, y=0, y=Ly, z=0, z=Lz.
 *  - Taps j = -T/2+1 .. T/2 around floor(D); x is zero outside [0, n_in).
 *  - Signal buffers are DEVICE pointers.  All scenes of a plan are packed back to
 *    back: x holds scene 0's n_in samples, then scene 1's, ...; y holds, per
 *    scene in order, n_mics rows of n_out samples (scene-major, mic, time).
 *    msim_plan_layout() returns the offsets.
 *  - Every entry point returns a status; nothing is thrown across the ABI.  On a
 *    non-OK status msim_last_error() describes the failure (thread-local string).
 *  - msim_forward / msim_backward enqueue work on the caller's stream and return
 *    without synchronising; they allocate no device memory (all scratch lives in
 *    the caller's workspace).  Plan creation allocates and synchronises.
 */
#ifndef MSIM_H
#define MSIM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MSIM_OK = 0,
    MSIM_E_INVALID_ARG = 1,   /* a NULL pointer, a size <= 0, beta outside [0,1], T odd or outside 8..128, ... */
    MSIM_E_OUTSIDE_ROOM = 2,  /* a knot or circle of a trajectory (or a mic) lies outside the room */
    MSIM_E_TOO_CLOSE = 3,     /* source and a mic closer than 1 mm at a knot time */
    MSIM_E_SUPERSONIC = 4,    /* a trajectory segment faster than c/10 */
    MSIM_E_WORKSPACE = 5,     /* workspace NULL or smaller than msim_workspace_size() */
    MSIM_E_UNSUPPORTED = 6,   /* a valid request the library does not implement */
    MSIM_E_HIP = 7,           /* a HIP runtime call failed */
    MSIM_E_DEVICE = 8         /* a device-side check failed (see msim_device_status) */
} msim_status;

enum { MSIM_TRAJ_PWL = 0, MSIM_TRAJ_CIRCLE = 1 };
enum { MSIM_DELAY_RETARDED = 0, MSIM_DELAY_INSTANTANEOUS = 1 };
enum { MSIM_TIER_ORDER = 0, MSIM_TIER_ADAPTIVE = 1 };
enum { MSIM_ADJX_GATHER = 0, MSIM_ADJX_TRANSPOSE = 1 };

/* A trajectory.  PWL: positions p[3k..3k+2] at strictly increasing times t[k],
 * linear in between, held constant before t[0] and after t[n_points-1]; one knot
 * is a static point.  CIRCLE: center + radius (cos(w t + phase0), sin(w t + phase0), 0),
 * w = speed / radius.  Pointers are host memory, read during msim_plan_create only. */
typedef struct {
    int32_t kind;
    int32_t n_points;
    const double* t;
    const double* p;
    double center[3];
    double radius;
    double speed;
    double phase0;
} msim_traj;

/* One scene: a room, a source path, a receiver path with n_mics microphones at
 * fixed offsets from the receiver point, and the signal lengths. */
typedef struct {
    double size[3];             /* Lx, Ly, Lz (m) */
    double beta[6];             /* wall reflection coefficients in [0, 1] */
    msim_traj src;
    msim_traj rcv;
    int32_t n_mics;
    const double* mic_offset;   /* host, [n_mics*3] */
    int32_t max_order;          /* K >= 0 */
    int64_t n_in;               /* source samples */
    int64_t n_out;              /* output samples per mic */
} msim_scene;

/* Synthesis parameters shared by every scene of a plan. */
typedef struct {
    double c;                   /* speed of sound, m/s */
    double fs;                  /* sample rate, Hz */
    int32_t taps;               /* T: even, 8..128, multiple of 8 */
    double kaiser_beta;         /* Kaiser window shape */
    double cutoff;              /* normalised cutoff in (0, 0.5] cycles/sample */
    int32_t table_phases;       /* L: phases per unit delay of the FD table, interpolated
                                   quadratically (power of two, 16..1024), or 0 (the
                                   default): the planner takes 128, or 64 where that lets
                                   two outputs share a lane within the error budget */
    int32_t n_tiers;            /* 0: every image at the audio rate; 1..4 tiers below */
    int32_t tier_max_order[4];  /* tier k holds orders <= tier_max_order[k] not in an earlier tier */
    int32_t tier_decim[4];      /* decimation of tier k's delay grid (1 = audio rate), 1..4096 */
    int32_t delay_model;        /* MSIM_DELAY_RETARDED (emission-time delay) or _INSTANTANEOUS */
    int32_t fd_kind;            /* MSIM_FD_TABLE (default) or MSIM_FD_FARROW */
    int32_t farrow_order;       /* M, 4..11: degree of the Farrow polynomial in the fractional delay */
    double knot_slack;          /* m, 0..10: how far msim_plan_update may move a source knot from the
                                   plan's path (every delay bound is planned that much wider) */
    int32_t tier_mode;          /* MSIM_TIER_ORDER: decimations by reflection order (n_tiers ...);
                                   MSIM_TIER_ADAPTIVE: per image, from a bound on its delay track's
                                   third derivative (Sec. II-C-1/2: the motion's bandwidth, and the
                                   near field of a close image), see msim_plan_create */
    double tier_tol;            /* adaptive: bound on the interpolated delay's error, samples (> 0) */
    int32_t tier_rmax;          /* adaptive: largest decimation, 1..4096 */
    int32_t adjx_mode;          /* dL/dx in the backward.  MSIM_ADJX_GATHER (default): every
                                   source position gathers the image samples that read it and
                                   the Farrow filter bank is transposed (Sec. II-B, Eq. 3-5;
                                   in the table form this is the transpose of the Farrow fit of
                                   the same kernel, within its error of the table's); taken
                                   unless the Farrow fit exceeds the error budget or a
                                   delay group's gather window does not fit LDS.
                                   MSIM_ADJX_TRANSPOSE:
                                   the table form's exact transpose.  farrow_order 4..11. */
} msim_params;

/* How the T-tap Kaiser-windowed sinc h(j - mu) is applied.
 *  MSIM_FD_TABLE:  an oversampled table of h in LDS, interpolated quadratically
 *                  between phases, one gather of T taps per image sample; the
 *                  adjoint is the exact transpose and derivative of that interpolant.
 *  MSIM_FD_FARROW: the Farrow structure of Sec. II-B (Eq. 3-5): h(j - mu) is fitted
 *                  by a degree-M polynomial in s = 2 mu - 1 for every tap j
 *                  (Chebyshev interpolation of the same kernel), the M+1 filtered
 *                  signals v_k = x * c_k are computed once per source, and each image
 *                  sample reads v_0..v_M at n - floor(D) and evaluates the polynomial
 *                  by Horner's rule.  Both approximate the same h; with M = 9 the
 *                  polynomial's error is below FP32 rounding of the output. */
enum { MSIM_FD_TABLE = 0, MSIM_FD_FARROW = 1 };

typedef struct msim_plan msim_plan;

/* Fills defaults: c 343, fs 16000, T 64, Kaiser beta 8, cutoff 0.5, L 128,
 * three tiers (orders <=2 at the audio rate, 3-6 decimated by 16, the rest by 160),
 * retarded delays. */
msim_status msim_default_params(msim_params* p);

/* Number of images with |mx|+|my|+|mz| <= max_order. */
msim_status msim_count_images(int32_t max_order, int64_t* n);

/* An output length that holds every contribution: n_in + ceil(fs * d_max / c) + T,
 * with d_max the largest distance from the room to an image cell of order <= K. */
msim_status msim_suggest_n_out(const msim_scene* scene, const msim_params* p, int64_t* n_out);

/* Adaptive decimation (tier_mode MSIM_TIER_ADAPTIVE).  Image i may err in its
 * delay by delta_i = tier_tol * max(d_i, 0.1 m) / beta_i samples: tier_tol for an
 * image as loud as a unit source at 1 m, more for a fainter one (its gain is
 * beta_i / (4 pi d)), d_i the smallest distance from the image's box over the
 * path to the mics' box.  The delay d_i(t) = |S_i p(t) - r(t)| / c has a third
 * derivative of at most
 *   K3_i = ( (2/sqrt 3) u^3 / d_i^2 + 3 u a / d_i + j ) / (1 - u/c)^3      (m/s^3)
 * with u, a, j the source's plus the receiver's largest speed, acceleration and
 * jerk (a circle: v, v^2/r, v^3/r^2; a PWL path read as samples of a smooth
 * path: the piece speeds, the velocity change at each inner knot over the mean
 * of its two pieces' durations, no jerk): the near field (small d_i) raises it,
 * far images keep the motion's own bandwidth (Sec. II-C-1/2).  Uniform
 * Catmull-Rom through decimation R errs by at most about R^3 D3_i / 24 samples,
 * D3_i = K3_i / (c fs^2), on smooth motion, and by up to (3/16) R dv / (c - u) at
 * a knot whose velocity changes by dv (the largest inner-knot change of the
 * source plus the receiver).  Image i takes the largest R of 1, 4, 8, 16, ...
 * (not above tier_rmax) that keeps both within delta_i.  The paths' first and
 * last knots (where motion starts and stops) are not counted. */

/* Validates the scenes, enumerates their images, sorts them by delay, builds the
 * fractional-delay table and uploads the plan's device descriptors.  Runs on the
 * current HIP device and synchronises.  *plan is owned by the caller and released
 * with msim_plan_destroy. */
msim_status msim_plan_create(const msim_scene* scenes, int32_t n_scenes, const msim_params* p, msim_plan** plan);

msim_status msim_plan_destroy(msim_plan* plan);

/* Packed layout: x_off[s], y_off[s] (element offsets) for each scene, and totals. */
msim_status msim_plan_layout(const msim_plan* plan, int64_t* x_off, int64_t* y_off, int64_t* x_total, int64_t* y_total);

/* Image count of every scene, and the forward tap count
 * sum over scenes, mics, images of (n_in + T - 1) * T. */
msim_status msim_plan_stats(const msim_plan* plan, int64_t* n_images, double* forward_taps);

/* Bytes of device workspace msim_forward (with_grad = 0) or msim_backward
 * (with_grad = 1) needs; the caller allocates it (256-byte aligned). */
msim_status msim_workspace_size(const msim_plan* plan, int32_t with_grad, size_t* bytes);

/* Forward synthesis, one scene after another with ordinary launches.
 * x: device [x_total] FP32; y: device [y_total] FP32, fully overwritten. */
msim_status msim_forward(msim_plan* plan, const float* x, float* y, void* ws, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): msim_forward without a
 * caller workspace.  Its scratch (track slots, partial outputs, the ticket
 * counter) is a fixed 64 MiB array on each GPU, held from the first plan
 * created on that GPU until the process ends; the call allocates nothing.
 * MSIM_E_WORKSPACE when the plan needs more than that (msim_workspace_size(plan,
 * 0) > 64 MiB).  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (two streams, or two host threads) race and must be
 * serialised by the caller.  Everything a call reads from the array it first
 * writes in the same call.  Same result as msim_forward, bit for bit. */
msim_status msim_forward_noalloc(msim_plan* plan, const float* x, float* y, hipStream_t stream);

/* Batched forward: the same result as msim_forward (bit for bit: both sum every
 * delay group in the same order), computed by three launches over all scenes
 * at once: the delay tracks of every scene, one persistent synthesis kernel
 * whose fixed grid of workgroups loads the fractional-delay table once and then
 * takes (scene, mic, tile, delay group) work items in decreasing-cost order from
 * a ticket counter, and the group reduction.  With use_graph != 0 the three
 * launches are captured once into a HIP graph (per x, y, ws triple) and replayed
 * on `stream`; use_graph = 0 launches them directly.  ws holds
 * msim_batched_workspace_size() bytes (all scenes' tracks at once). */
msim_status msim_batched_workspace_size(const msim_plan* plan, size_t* bytes);
msim_status msim_forward_batched(msim_plan* plan, const float* x, float* y, void* ws, size_t ws_bytes,
                                 hipStream_t stream, int32_t use_graph);

/* Launch shape: output samples per workgroup (512 or 1024), images per delay
 * group (0: the form's default, 96 table / 256 Farrow), adjacent output samples per lane of the
 * forward (a lane's samples share one track segment, so every tier decimation
 * must be 1 or a multiple of it; the table form takes 1 or 2 and its two samples
 * also share table rows, which needs the delay to drift by at most ~0.8 table rows
 * per sample: source plus receiver speed below 2.2 m/s at 128 phases, 4.4 m/s at
 * 64; the Farrow form takes 1, 2 or 4; 0: the form's default, 2 for the table form
 * where allowed, else 1), and the persistent grid size it implies. */
typedef struct {
    int32_t threads;
    int32_t group_cap;
    int32_t outputs_per_lane;
    int32_t workgroups;   /* output only */
    double ms;            /* output only: the batched forward time that chose it */
    int32_t adjx_gather;  /* output only: 1 when the backward's dL/dx is the Farrow gather */
} msim_tuning;

msim_status msim_get_tuning(const msim_plan* plan, msim_tuning* t);
/* Predicted relative L2 error of one image's output for a white source signal,
 * per approximation of the truncated Kaiser-windowed sinc (Sec. II-B), computed
 * from the kernel at the plan's taps, kaiser_beta, cutoff, table_phases and
 * farrow_order: `table`, the quadratic phase table as stored (table form);
 * `pair`, the edge tap that two outputs per lane omit where they straddle an
 * integer delay, at the scenes' largest source plus receiver speed (table form);
 * `farrow`, the Farrow polynomials' fit (Farrow form); 0 where the form is not
 * the plan's.  msim_plan_create refuses a form whose figure exceeds `budget`
 * (MSIM_E_UNSUPPORTED, with the figure in the message) and keeps the table form
 * at one output per lane where table and pair together, in quadrature, would. */
typedef struct {
    double table;
    double pair;
    double farrow;
    double budget;
    int32_t table_phases;   /* the table's phase count (the planner's choice when
                               table_phases was 0) */
} msim_fd_error;

msim_status msim_get_fd_error(const msim_plan* plan, msim_fd_error* out);

/* The images of scene `scene` (plan order): out[4 i .. 4 i + 3] = (mx, my, mz,
 * decimation R of the image's delay track); *n_img gets the count.  With
 * out = NULL only the count is written; else capacity must hold n_img rows. */
msim_status msim_get_images(const msim_plan* plan, int32_t scene, int32_t* out, int64_t capacity, int64_t* n_img);

/* Replaces the wall reflection coefficients (beta [n_scenes*6], or NULL) and the
 * PWL source knot positions (knots [src_total*3] in the gradient layout of
 * msim_plan_grad_layout, or NULL; knot times stay) of every scene in place,
 * without planning again: the image gains beta_i = prod_w beta_w^hits_w (Sec.
 * II-A) and the knots are rewritten in the plan's device buffers on `stream`
 * (synchronised before return), so captured graphs stay valid.  The delay
 * groups keep the bounds planned for the original path widened by
 * params.knot_slack: a knot moved further than that from the plan's original
 * position gives MSIM_E_UNSUPPORTED (plan again); coefficients outside [0, 1],
 * knots leaving the room or moving at >= c/10 give the statuses of
 * msim_plan_create.  On any error nothing changes.  Calls that overlap a
 * launch on another stream race with it. */
msim_status msim_plan_update(msim_plan* plan, const double* beta, const double* knots, hipStream_t stream);
/* Regroups the plan for a launch shape; workspace sizes change with it. */
msim_status msim_set_tuning(msim_plan* plan, const msim_tuning* t);
/* Largest batched workspace over the shapes msim_autotune tries. */
msim_status msim_autotune_workspace_size(msim_plan* plan, size_t* bytes);
/* Times the batched forward (direct launches, 3 runs after 1 warm-up) for each
 * launch shape that fits ws and keeps the fastest; the choice is read from and
 * appended to the JSON-lines file cache_path (may be NULL), keyed by the
 * fractional-delay form, table shape, scene count, image count and output size.  Synchronises `stream`;
 * x and y are scratch for the timing runs (y is overwritten). */
msim_status msim_autotune(msim_plan* plan, const float* x, float* y, void* ws, size_t ws_bytes,
                          hipStream_t stream, const char* cache_path, msim_tuning* best);

/* Reverse mode of msim_forward for a scalar loss L, given gy = dL/dy (device,
 * [y_total] FP32).  Recomputes the delay tracks (nothing is kept from the
 * forward) and writes, each only when its pointer is non-NULL (device memory):
 *   gx    [x_total] FP32: dL/dx, the transpose time-varying fractional delay;
 *   gbeta [n_scenes*6] FP64: dL/dbeta_w through beta_i = prod_w beta_w^hits_w;
 *   gsrc  [src_total*3] FP64: dL/d(source knot position) for PWL sources, through
 *         the Catmull-Rom delay interpolation and the implicit derivative of the
 *         retarded delay (Sec. II-A, II-C-3); knots are packed per scene as
 *         msim_plan_grad_layout reports (circle sources have none).
 * Knot times, mic and receiver positions get no gradient.  ws holds
 * msim_workspace_size(plan, 1) bytes.  Both fractional-delay forms have their
 * adjoint: with MSIM_FD_TABLE dL/dx is scattered tap by tap into per-wave LDS
 * windows; with MSIM_FD_FARROW each source position gathers the sums
 * u_k = sum gy g s^k of the image samples that read it, and dL/dx is the
 * transposed filter bank sum_k c_k (x) u_k.  Every output is summed in a fixed
 * order, so repeated calls give identical bits.  MSIM_E_UNSUPPORTED: a scene
 * whose delay groups leave no LDS for the adjoint, or a source with more than
 * 32 knots when gsrc is requested. */
msim_status msim_backward(msim_plan* plan, const float* x, const float* gy, float* gx, double* gbeta,
                          double* gsrc, void* ws, size_t ws_bytes, hipStream_t stream);

/* Batched reverse mode: the same gradients as msim_backward (bit for bit: both
 * sum every partial in the same order), computed by one launch per kernel over
 * all scenes at once (persistent workgroups taking (scene, mic, tile,
 * supergroup) items from a ticket counter).  With use_graph != 0 the launches
 * are captured once into a HIP graph (per argument set: x, gy, gx, gbeta, gsrc,
 * ws) and replayed on `stream`.  ws holds msim_batched_workspace_size() bytes. */
msim_status msim_backward_batched(msim_plan* plan, const float* x, const float* gy, float* gx, double* gbeta,
                                  double* gsrc, void* ws, size_t ws_bytes, hipStream_t stream, int32_t use_graph);

/* Offsets (in knots) of each scene's source knots in gsrc, and their total. */
msim_status msim_plan_grad_layout(const msim_plan* plan, int64_t* src_off, int64_t* src_total);

/* Reads and clears the plan's device-side status flags (synchronises the stream).
 * Bit 0: a delay left the window the plan bounded for it (output not trusted). */
msim_status msim_device_status(msim_plan* plan, hipStream_t stream, int32_t* flags);

/* Per-kernel timing.  Between msim_profile_begin and msim_profile_end every
 * kernel the plan launches is bracketed by HIP events on its stream;
 * msim_profile_end waits for them and returns the summed durations (ms) and
 * launch counts per kernel kind.  Profiling adds host work per launch only. */
typedef struct {
    double synth_ms;           /* forward synthesis (k_synth, k_farrow; tracks solved inside) */
    double reduce_ms;          /* the forward's supergroup reduction */
    double adjx_ms;            /* dL/dx: k_adjx or k_farrow_u with their reductions */
    double adjp_ms;            /* gain/delay adjoints with the in-tile parameter sums (k_adjp, k_farrow_gd) */
    double params_ms;          /* reduction of the parameter rows */
    double graph_ms;           /* replays of a batched graph */
    double filter_ms;          /* the Farrow filter bank v_k = x * c_k */
    int32_t synth_launches, reduce_launches, adjx_launches, adjp_launches, params_launches, graph_launches,
        filter_launches;
} msim_profile;

msim_status msim_profile_begin(msim_plan* plan);
msim_status msim_profile_end(msim_plan* plan, msim_profile* out);

/* Thread-local description of the last failure. */
const char* msim_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MSIM_H */
