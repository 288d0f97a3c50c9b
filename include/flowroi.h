/*
 * flowroi.h — C ABI of the MI355X (gfx950) FlowRoI hot path.
 *
 * FlowRoI (Method section, "Optical flow extraction" and "Region of Interest
 * extraction") turns a pair of adjacent grayscale frames into a dense optical
 * flow field with Farneback's estimator, keeps the pixels whose motion
 * exceeds a threshold, and cleans the result with morphology into a binary
 * RoI mask that a host-side JPEG2000 RoI encoder consumes. This library runs
 * that path as HIP kernels; the estimator is the two-frame polynomial-
 * expansion method (Farneback, SCIA 2003), whose constants the paper leaves
 * open; the defaults below are the frozen reading.
 *
 * Conventions shared by every entry point
 *   - Frames are row-major, h rows by w columns, `pitch` elements between
 *     the starts of consecutive rows (pitch >= w). Element type: roi_dtype.
 *   - x is the column, y the row. Flow is interleaved float (dx, dy) per
 *     pixel, h*w*2 floats with row pitch w, pointing from prev to next:
 *     next(x + d) ~ prev(x).
 *   - The mask is h*w uint8 values in {0, 1}, row pitch w.
 *   - Every pointer named "device" is device memory on the current HIP
 *     device, owned by the caller; the library never frees or retains it.
 *     Host pointers are read during the call only.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream)
 *     and runs asynchronously. Parameter errors are detected on the host
 *     before anything is enqueued; on any error status nothing was enqueued
 *     (except ROI_EDEVICE, which reports a failed launch).
 *   - No entry point allocates device memory except roi_stream_create and
 *     roi_server_create (and roi_server_open_stream, inside the server's
 *     HBM budget). Scratch comes from a caller-provided workspace of at
 *     least roi_workspace_size() bytes, 256-byte aligned. roi_mask_batched
 *     keeps its instantiated HIP graphs, and the batched path and the
 *     server their own streams and events, until the process ends (or the
 *     server is destroyed).
 *   - Calls that share a workspace or a stream context must not overlap.
 */
#ifndef FLOWROI_H
#define FLOWROI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ROI_OK = 0,
    ROI_PRIMED = 1,          /* stream push: first frame stored, no flow/mask yet */
    ROI_EINVAL = -1,         /* bad pointer, size or parameter */
    ROI_ENOMEM = -2,         /* workspace too small / device allocation failed */
    ROI_EDEVICE = -3,        /* a HIP call or kernel launch failed */
    ROI_EUNSUPPORTED = -4    /* valid request outside what the kernels handle */
} roi_status;

typedef enum { ROI_U8 = 0, ROI_U16 = 1, ROI_F32 = 2 } roi_dtype;

enum {
    ROI_THRESH_ABS = 0,      /* keep |d| > thresh (pixels) */
    ROI_THRESH_TOP = 1       /* keep the top `thresh` fraction of |d| (RoI threshold, Table 1) */
};

enum {
    /* Mask rule. MAGNITUDE: pre = [|d| above the threshold]. SALIENCY
     * (Method, Region of Interest extraction): motion saliency S combines
     * the flow magnitude M = |d| with its spatial gradient G = |grad M|
     * (central differences, replicated edges) with weight sal_weight on M,
     * each term divided by its maximum over the frame, and S divided by its
     * own maximum (the normalisation); pre = [S above the threshold] (TOP:
     * the top `thresh` fraction of S, as the paper's RoI threshold of 0.2
     * keeps the top 20 %; ABS: normalised S > thresh), then opening and
     * closing with the (2 morph_radius + 1)^2 square, then removal of the
     * 8-connected components smaller than min_area pixels. Both rules end
     * with the dilation (dilate_radius, se_shape). */
    ROI_RULE_MAGNITUDE = 0,
    ROI_RULE_SALIENCY = 1
};

enum {
    ROI_SE_SQUARE = 0,       /* (2r+1)^2 square */
    ROI_SE_DISC = 1          /* offsets with u^2 + v^2 <= r^2 */
};

enum {
    ROI_USE_INITIAL_FLOW = 1u, /* `flow` holds an initial flow on entry (see roi_mask) */
    ROI_FP16_STORAGE = 2u,     /* per-level expansions (the planes every iteration reads) stored as FP16;
                                  pyramid images stay FP64, all arithmetic FP32/FP64 as without it */
    ROI_STABILIZE = 4u         /* register next to prev before the flow (Method, optical flow extraction:
                                  phase-correlation alignment, after denoising); see roi_phase_correlation */
};

/* Parameters of the path. Farneback's constants are not given by the paper
 * (it only names the "dense Farneback" estimator); the RoI threshold is
 * Table 1's (the paper's example: 0.2 keeps the top 20 %). */
typedef struct roi_params {
    int32_t levels;        /* pyramid levels, 1..10; level l+1 = binomial-blurred level l at even pixels */
    int32_t winsize;       /* side of the square pooling window, odd, 1..15 */
    int32_t iterations;    /* displacement updates per level, 1..64 */
    int32_t poly_n;        /* expansion neighbourhood side, 3, 5 or 7 */
    float poly_sigma;      /* Gaussian applicability sigma (pixels), > 0 */
    float eps;             /* regulariser: den = max(det G, eps (tr G)^2), > 0 */
    int32_t thresh_mode;   /* ROI_THRESH_ABS or ROI_THRESH_TOP */
    float thresh;          /* ABS: pixels, >= 0; TOP: fraction in (0, 1) */
    int32_t dilate_radius; /* structuring-element radius, 0..32 */
    int32_t se_shape;      /* ROI_SE_SQUARE or ROI_SE_DISC */
    uint32_t flags;        /* ROI_USE_INITIAL_FLOW | ROI_FP16_STORAGE | ROI_STABILIZE */
    /* Denoising pre-stage (Method, Optical flow extraction: median then
     * bilateral filtering; Table 1 "Denoise" on/off), applied to both
     * frames before the pyramid. */
    int32_t denoise;          /* 0 off, 1 on */
    int32_t median_radius;    /* 0..2: (2r+1)^2 median, 0 skips it */
    int32_t bilateral_radius; /* 0..3: (2r+1)^2 bilateral window, 0 skips it */
    float sigma_space;        /* bilateral spatial sigma (pixels), > 0 */
    float sigma_range;        /* bilateral range sigma (grey levels of the input), > 0 */
    /* Adjacent factor (Table 1; Region of Interest extraction: masks of
     * neighbouring frames join the current one when motion is weak). Stream
     * contexts only: the mask of frame t becomes the union of its own mask
     * and those of the previous `adjacent` frames of the stream. 0..8. */
    int32_t adjacent;
    /* Mask rule (ROI_RULE_*). Under ROI_RULE_SALIENCY, thresh applies to
     * the saliency: TOP fraction in (0, 1), or ABS level on the normalised
     * saliency (>= 0). */
    int32_t rule;
    float sal_weight;      /* weight of the magnitude term, [0, 1] (the paper's 0.7) */
    int32_t morph_radius;  /* opening/closing square radius, 0..2 (0 skips them) */
    int32_t min_area;      /* smallest kept component, pixels, >= 0 (0 or 1 keeps all) */
} roi_params;

/* Defaults: levels 3, winsize 15, iterations 3, poly_n 5, poly_sigma 1.1,
 * eps 1e-3, ABS threshold 1.0 px, square dilation of radius 2, no flags,
 * denoising off (when on: 3x3 median, 5x5 bilateral, sigma_space 1.5,
 * sigma_range 20), adjacent 0, magnitude rule (saliency rule settings:
 * sal_weight 0.7, morph_radius 1, min_area 32). */
void roi_default_params(roi_params *p);

/* Host-only check of a request (no device work). ROI_OK, ROI_EINVAL for a
 * bad value, ROI_EUNSUPPORTED for valid values the kernels do not handle.
 * h or w equal to 0 is valid (empty frame: every call is a no-op). */
roi_status roi_validate(int32_t h, int32_t w, roi_dtype dtype, const roi_params *p);

/* Workspace bytes roi_mask needs for this request (0 if roi_validate fails). */
size_t roi_workspace_size(int32_t h, int32_t w, roi_dtype dtype, const roi_params *p);

/* The hot path for one frame pair: flow prev -> next, the magnitude
 * threshold, and the dilation into the RoI mask.
 *   prev, next  device, h x w frames of `dtype`, row pitch `pitch` elements.
 *   flow        device, h*w*2 floats, output. With ROI_USE_INITIAL_FLOW it
 *               is also read first: the coarsest level L-1 starts from
 *               flow(min(2^(L-1) y, h-1), min(2^(L-1) x, w-1)) / 2^(L-1).
 *   mask        device, h*w uint8, output: 1 inside the RoI, 0 elsewhere.
 *               May be NULL to skip threshold and dilation.
 *   ws          device workspace of ws_bytes >= roi_workspace_size(...).
 * Returns ROI_OK once the work is enqueued. */
roi_status roi_mask(const void *prev, const void *next, int32_t h, int32_t w, int64_t pitch,
                    roi_dtype dtype, const roi_params *p, float *flow, uint8_t *mask, void *ws,
                    size_t ws_bytes, void *stream);

/* Squared threshold tau^2 that the last roi_mask / roi_mask_batched call on
 * this workspace applied (ABS: thresh^2; TOP: the (k+1)-th largest |d|^2
 * with k = floor(q h w)), copied to the host after synchronising `stream`.
 * For a batched call, `index` selects the pair. Under the saliency rule
 * with TOP it is the (k+1)-th largest saliency before normalisation (S,
 * not squared); under the saliency rule with ABS it is 0. */
roi_status roi_read_tau2(const void *ws, int32_t index, float *tau2_out, void *stream);

/* Translation (sy, sx) that stabilisation applied in the last roi_mask,
 * roi_mask_batched (pair `index`) or roi_phase_correlation call on this
 * workspace, and the correlation peak (peak may be NULL); copied to the
 * host after synchronising `stream`. Meaningful only after a call that ran
 * stabilisation. */
roi_status roi_read_shift(const void *ws, int32_t index, int32_t *sy, int32_t *sx, float *peak, void *stream);

/* ---- Stabilisation (Method, optical flow extraction) --------------------
 * Registration of a frame to its predecessor by phase correlation. Both
 * frames are cut to the centred P x P window, P = roi_phase_size(h, w)
 * (the largest power of two <= min(h, w, 2048); 0 for frames thinner than
 * 2 pixels: no estimate, zero shift), multiplied by the separable Hann
 * window 0.5 (1 - cos(2 pi i / (P - 1))); with A, B their 2-D DFTs the
 * surface r = IDFT(B conj(A) / |B conj(A)|) (0 where the product is 0)
 * peaks at the translation s of next against prev (next(x) = prev(x - s)):
 * its largest value (first in row-major order on ties), indices at or above
 * P/2 read as negative. The registered frame is next moved back by s,
 * out(y, x) = next(y + sy, x + sx), coordinates clamped into the frame.
 * Under ROI_STABILIZE, roi_mask computes the flow from prev to the
 * registered next (after the denoising pre-stage when it is on); a stream
 * registers each frame to its registered predecessor (the first is kept). */
int32_t roi_phase_size(int32_t h, int32_t w);
size_t roi_phase_workspace_size(int32_t h, int32_t w);

/* The stabilisation step alone.
 *   prev, next  device h x w frames of `dtype`, row pitch `pitch` elements.
 *   surface     device P*P floats (row-major, P = roi_phase_size), output of
 *               the correlation surface; may be NULL.
 *   aligned     device h*w floats (pitch w), output of the registered next
 *               frame; may be NULL.
 *   ws          device workspace >= roi_phase_workspace_size(h, w) bytes,
 *               256-byte aligned; roi_read_shift(ws, 0, ...) reads the shift. */
roi_status roi_phase_correlation(const void *prev, const void *next, int32_t h, int32_t w, int64_t pitch,
                                 roi_dtype dtype, float *surface, float *aligned, void *ws, size_t ws_bytes,
                                 void *stream);

/* Workspace bytes roi_mask_from_flow needs (0 if the parameters fail the
 * checks of roi_validate that concern the mask stage). */
size_t roi_flow_mask_workspace_size(int32_t h, int32_t w, const roi_params *p);

/* The mask stage alone, on a given flow field: the rule p->rule with its
 * threshold, then the dilation, exactly as roi_mask applies them after its
 * last update (the same kernels and per-pixel arithmetic, so a flow from
 * roi_mask gives back roi_mask's mask).
 *   flow      device, h*w*2 floats (pitch w), input.
 *   mask      device, h*w uint8, output.
 *   saliency  device, h*w floats (pitch w), output of the normalised
 *             saliency under ROI_RULE_SALIENCY; may be NULL; ignored under
 *             ROI_RULE_MAGNITUDE.
 *   ws        device workspace of ws_bytes >= roi_flow_mask_workspace_size,
 *             256-byte aligned; roi_read_tau2(ws, 0, ...) reads its threshold.
 * Only the mask-stage fields of p are used (thresh_mode, thresh,
 * dilate_radius, se_shape, rule, sal_weight, morph_radius, min_area). */
roi_status roi_mask_from_flow(const float *flow, int32_t h, int32_t w, const roi_params *p, uint8_t *mask,
                              float *saliency, void *ws, size_t ws_bytes, void *stream);

/* ---- Single steps, for testing each step in isolation ------------------ */

/* One pyramid step (step a2): dst(i, j) = sum_{u,v} k(u) k(v) src(2i+u, 2j+v),
 * k = [1 4 6 4 1]/16, replicate border. src device h x w floats (pitch w),
 * dst device ceil(h/2) x ceil(w/2) floats (pitch ceil(w/2)). */
roi_status roi_pyr_down(const float *src, int32_t h, int32_t w, float *dst, void *stream);

/* Polynomial expansion (step a3) of one frame: weighted least-squares fit
 * of f ~ x^T A x + b^T x + c over the poly_n x poly_n neighbourhood with
 * Gaussian applicability (poly_sigma), replicate border. Output `coef` is
 * device 5 x h x w floats (plane stride h*w): b_x, b_y, A_xx, A_yy, A_xy
 * (A_xy is the off-diagonal entry, half the x*y coefficient). Uses
 * p->poly_n, p->poly_sigma and p->flags & ROI_FP16_STORAGE (rounds the
 * stored values to FP16 precision). */
roi_status roi_poly_expand(const void *img, int32_t h, int32_t w, int64_t pitch, roi_dtype dtype,
                           const roi_params *p, float *coef, void *stream);

/* Denoising pre-stage of one frame: median of radius p->median_radius, then
 * bilateral of radius p->bilateral_radius (sigma_space, sigma_range), both
 * with replicated borders. out: device h*w floats (pitch w). Applies
 * whatever p->denoise says (the stage runs regardless). */
roi_status roi_denoise(const void *img, int32_t h, int32_t w, int64_t pitch, roi_dtype dtype, const roi_params *p,
                       float *out, void *stream);

/* ---- Batched: several pairs of uneven sizes in one captured launch ------ */

typedef struct roi_pair {
    const void *prev;      /* device frame */
    const void *next;      /* device frame */
    float *flow;           /* device h*w*2 floats */
    uint8_t *mask;         /* device h*w uint8 (must not be NULL) */
    int32_t h, w;
    int64_t pitch;         /* elements */
} roi_pair;

/* Workspace for roi_mask_batched over these pairs (0 on invalid input). */
size_t roi_batched_workspace_size(int32_t n, const roi_pair *pairs, roi_dtype dtype, const roi_params *p);

/* All n pairs through the whole path. Each pair's result is the one roi_mask
 * gives for it alone (the same per-pixel arithmetic, bit for bit). The
 * expansions, the full-resolution updates and the mask stages run as
 * independent per-pair branches; each coarse-level update is one launch
 * over up to 16 pairs at once, so the coarse levels of many pairs fill the
 * GPU together. The launch
 * sequence for a given (pairs, dtype, params, ws) is captured into a HIP
 * graph on first use and replayed afterwards. n in 1..256. */
roi_status roi_mask_batched(int32_t n, const roi_pair *pairs, roi_dtype dtype, const roi_params *p,
                            void *ws, size_t ws_bytes, void *stream);

/* ---- Streaming: one context per camera stream --------------------------- */

/* Allocates the resident state of one stream (the previous frame's pyramid
 * expansions and the flow/mask scratch) on the current device. */
roi_status roi_stream_create(int32_t h, int32_t w, roi_dtype dtype, const roi_params *p, void **out_ctx);

/* Pushes the next frame. The first push after create (or reset) stores the
 * frame and returns ROI_PRIMED without writing flow/mask. Later pushes write
 * the flow from the previous frame to this one and its mask, exactly as
 * roi_mask(previous, frame) would, and return ROI_OK. */
roi_status roi_stream_push(void *ctx, const void *frame, int64_t pitch, float *flow, uint8_t *mask,
                           void *stream);

/* Forget the stored frame: the next push primes again. */
roi_status roi_stream_reset(void *ctx);

/* Resident device bytes of a stream context with these settings. */
size_t roi_stream_state_bytes(int32_t h, int32_t w, roi_dtype dtype, const roi_params *p);

void roi_stream_destroy(void *ctx);

/* The translation stabilisation applied to the last frame pushed to this
 * stream (0, 0 for its first frame), as roi_read_shift. */
roi_status roi_stream_read_shift(void *ctx, int32_t *sy, int32_t *sx, float *peak, void *stream);

/* Several stream contexts advanced together: frames[i] is pushed into
 * ctxs[i], all in one batched launch sequence on `stream`; the coarse-level
 * updates of all contexts that produce a flow share grids of up to 16.
 * status[i] gets ROI_PRIMED or ROI_OK per context, and each result is the
 * one roi_stream_push gives. Contexts must share dtype and params and be
 * distinct (ROI_EINVAL otherwise). n in 1..256. */
roi_status roi_stream_push_many(int32_t n, void *const *ctxs, const void *const *frames,
                                const int64_t *pitches, float *const *flows, uint8_t *const *masks,
                                int32_t *status, void *stream);

/* ---- Serving: continuous batching over many camera streams -------------- */

/* A server owns up to max_streams stream contexts of one frame size, dtype
 * and parameter set. Frames are submitted from host memory as they arrive;
 * a scheduler thread forms steps of at most one ready frame per stream
 * (oldest arrival first, at most max_batch frames), copies them to the
 * device on a copy stream and runs them on four compute streams (each
 * server stream always on the same one, which keeps its frames in order).
 * Up to max_inflight steps are on the GPU at once; frames that arrive
 * while a step runs join a later step. A completion thread stamps each
 * frame's completion time. Every result equals what roi_stream_push gives
 * for that stream alone. */
typedef struct roi_server_config {
    int32_t h, w;
    roi_dtype dtype;
    roi_params params;
    size_t hbm_budget;      /* device bytes the server may hold (stream state + staging) */
    int32_t max_streams;    /* 1..256 */
    int32_t max_batch;      /* frames per step, 1..256 */
    int32_t max_inflight;   /* steps on the GPU at once, 1..4 */
    int32_t queue_depth;    /* frames a stream may have queued, 1..64 */
} roi_server_config;

typedef struct roi_server_result {
    uint64_t tag;           /* the caller's tag from roi_server_submit */
    int32_t stream;         /* server stream id */
    int32_t status;         /* ROI_OK, ROI_PRIMED (first frame), or an error */
    double t_arrival;       /* seconds on the steady clock, at submit */
    double t_done;          /* seconds, when the GPU finished the frame's step */
    int32_t batch;          /* frames in the step that carried it */
    int32_t pad;
} roi_server_result;

/* Validates the config and starts the threads; allocates nothing on the
 * device until streams open. */
roi_status roi_server_create(const roi_server_config *cfg, void **out_srv);

/* Admission: opens a stream if its resident state fits in what is left of
 * the HBM budget (ROI_ENOMEM otherwise: the caller may retry once another
 * stream closes). Allocates the stream's context and two device frame
 * slots. */
roi_status roi_server_open_stream(void *srv, int32_t *out_id);

/* Closes a stream after its queued frames complete; frees its memory. */
roi_status roi_server_close_stream(void *srv, int32_t id);

/* Device bytes one stream holds (context + frame slots). */
size_t roi_server_stream_bytes(const roi_server_config *cfg);

/* Queues one frame for stream `id`. host_frame (h rows, `pitch` elements
 * per row) must stay valid and unchanged until the frame's result has been
 * polled; pinned memory gives asynchronous copies. flow (h*w*2 floats) and
 * mask (h*w uint8) are device buffers the caller owns; they are written
 * when the frame completes (not for a ROI_PRIMED first frame). Returns
 * ROI_EINVAL for a bad id or pointer and ROI_ENOMEM when the stream's
 * queue is full (the frame is then not queued). The arrival time is taken
 * here. */
roi_status roi_server_submit(void *srv, int32_t id, const void *host_frame, int64_t pitch, float *flow,
                             uint8_t *mask, uint64_t tag);

/* Moves up to `max` completed results (in completion order) into `out`;
 * returns how many. Non-blocking. */
int32_t roi_server_poll(void *srv, roi_server_result *out, int32_t max);

/* Blocks until every submitted frame has completed (or an error stops the
 * server); ROI_OK or the first error seen. */
roi_status roi_server_drain(void *srv);

/* Stops the threads (after draining) and frees everything. */
void roi_server_destroy(void *srv);

/* ---- Kernel timing ------------------------------------------------------ */

/* Timing of the iteration kernel (warp + update + window + solve, the
 * dominant kernel) with HIP events on the stream it is launched on.
 * mode 1: events around every launch; mode 2: one pair of events around
 * each call's run of iteration launches (they are back to back on the
 * stream, so the bracket is their kernel time plus the dispatch gaps
 * between them, and the call records far fewer events); 0: off. Events come
 * from a pool that roi_timing_read refills; mode 1 or 2 pre-creates `ROI_
 * TIMING_POOL` of them when the pool is smaller. roi_timing_read
 * synchronises the pending events and returns, summed since the last reset:
 * kernel time (ms), launches, output pixels, and algorithmic bytes
 * (expansion planes of both frames at the storage width + prior flow read +
 * flow written + the mask stage's input written, each counted once per
 * output pixel). Launches captured into graphs are not timed. */
#define ROI_TIMING_POOL 4096
void roi_timing_enable(int32_t mode);
roi_status roi_timing_read(double *total_ms, int64_t *launches, int64_t *pixels, double *bytes);
void roi_timing_reset(void);

/* Mode 2 brackets only every `every`-th call (counted from the last
 * roi_timing_reset; values below 1 mean 1, the default). Recording an event
 * leaves the GPU idle for a few microseconds between the kernels around it,
 * so sampling the calls keeps that cost out of a throughput measurement
 * while the sampled calls still give the kernel's launch times. */
void roi_timing_sample(int32_t every);

/* Records behind roi_timing_read (same synchronisation): fills up to `max`
 * entries of kernel ms, output pixels and algorithmic bytes, one per launch
 * (mode 1) or per call (mode 2), in order, and returns the number of
 * records available. */
int32_t roi_timing_records(double *ms, int64_t *pixels, double *bytes, int32_t max);

/* ---- Tuning -------------------------------------------------------------- */

/* The iteration kernel walks strips of 64 columns; the strip height only
 * changes how the work is split, never the result (bitwise). mode 1
 * (default): the first uncaptured launch for a new (level size, window,
 * storage) times the candidate heights {8, 16, ..., 256} on the real data
 * and keeps the fastest; mode 0: a size heuristic; mode 2: like 1 after
 * forgetting every tuned entry. */
void roi_autotune(int32_t mode);

/* Force every iteration launch to one strip height (a multiple of 8), or 0
 * to return to tuned/heuristic heights. ROI_EINVAL for other values. */
roi_status roi_set_strip(int32_t strip);

/* Tuned strip height for a level of h x w with this window and storage
 * (fp16 != 0: FP16), or 0 if that shape has not been tuned yet. Strips are
 * tuned per prior mode; this returns the one of the launches that start
 * from the same level's flow, else from the upsampled coarser flow, else
 * from zero. */
int32_t roi_tuned_strip(int32_t h, int32_t w, int32_t winsize, int32_t fp16);

const char *roi_status_str(roi_status s);

#ifdef __cplusplus
}
#endif

#endif /* FLOWROI_H */
