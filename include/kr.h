/*
 * kr.h -- C ABI of libkr, MI355X (gfx950) bilinear resampling kernels.
 *
 * The operators are the image-transformation hot path of kornia-rs
 * (arXiv 2505.12425): resize up and down (Sec. III, the benchmarked
 * "geometric transformations"), affine warping (Sec. II-A, kornia-imgproc
 * "geometric transforms"), on interleaved Image<T, C> buffers (Sec. II-B.2),
 * with caller-owned, pre-allocated outputs and no allocation on the call path
 * (Sec. II-B.4 and the "no implicit allocations" point of Listing 1).
 * The paper prints no resampling formula; the definitions fixed here are:
 *
 *  - layout: HWC-contiguous, C interleaved channels (1 <= C <= 4), row pitch
 *    W*C elements (sources may also be views with a larger pitch, see the
 *    *_view entry points), u8 or f32 samples;
 *  - half-pixel centres: resize source x = (dx + 1/2) * W_in / W_out - 1/2,
 *    evaluated exactly as a rational; warp destination pixel (x, y) maps to
 *    xs = fma(A, x, fma(B, y, C)), ys = fma(D, x, fma(E, y, F)) in binary64,
 *    where [[A, B, C], [D, E, F]] is the inverse map;
 *  - per-tap borders: a tap outside the source reads the constant border value
 *    (KR_BORDER_CONSTANT) or the nearest edge pixel (KR_BORDER_REPLICATE);
 *  - u8 output: 11-bit per-axis weights w1 = round-half-even(2048 * frac),
 *    w0 = 2048 - w1, exact integer sum, out = (acc + 2^21) >> 22;
 *  - f32 output: unquantised weights, values on the 0..255 scale, optionally
 *    normalised per channel as (v / 255 - mean_c) / std_c.
 *
 * Conventions shared by every entry point:
 *  - src, dst, workspace are DEVICE pointers, 16-byte aligned, owned by the
 *    caller; the library never frees or retains them.  src and dst must not
 *    overlap.
 *  - stream is a hipStream_t (NULL = the legacy default stream).  Work is
 *    enqueued asynchronously; the call returns once it is enqueued.
 *  - Arguments are validated synchronously before anything is enqueued; on a
 *    validation failure nothing is enqueued and a kr_status other than KR_OK
 *    is returned.  kr_last_error() then describes it (per calling thread).
 *  - Launch failures return KR_ERR_HIP.  Faults during execution surface at
 *    the caller's next synchronisation, as for any HIP kernel.
 *  - Sizes: 1 <= H, W <= 32767.  Supported (src, dst) types: (U8, U8),
 *    (U8, F32), (F32, F32).  norm is only accepted with an F32 destination.
 *    For a U8 source the border value must be an integer in [0, 255].
 *  - All entry points are reentrant; no C++ exception crosses the ABI.
 *  - Outputs are written with non-temporal stores: they go to HBM rather than
 *    staying in the GPU caches, so a kernel that reads them next fetches them
 *    from HBM (the bits are the same either way).
 */
#ifndef KR_H
#define KR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KR_OK = 0,
    KR_ERR_INVALID_ARGUMENT = 1, /* null/misaligned pointer, bad size, overlap, bad border value */
    KR_ERR_UNSUPPORTED = 2,      /* dtype pair, channel count or border mode not provided */
    KR_ERR_SINGULAR_MATRIX = 3,  /* non-finite or (numerically) singular affine matrix */
    KR_ERR_WORKSPACE_TOO_SMALL = 4,
    KR_ERR_OUT_OF_BUDGET = 5,    /* a request larger than the serving memory budget */
    KR_ERR_HIP = 6               /* a HIP runtime call failed */
} kr_status;

typedef enum { KR_U8 = 0, KR_F32 = 1 } kr_dtype;

typedef enum { KR_BORDER_CONSTANT = 0, KR_BORDER_REPLICATE = 1 } kr_border;

/* Per-channel normalisation on the [0, 1] scale: out_c = (v / 255 - mean[c]) / std[c].
 * Only the first C entries are read.  std[c] must be finite and non-zero. */
typedef struct {
    float mean[4];
    float std[4];
} kr_normalize;

/* kr_warp_affine / batch item flag: m is already the inverse map
 * (destination pixel centre -> source coordinate). */
#define KR_WARP_INVERSE_MAP 1

/*
 * Bilinear resize of one image (Sec. III "upsizing" and "downsizing").
 * src: src_h x src_w x c samples of type src_t.  dst: dst_h x dst_w x c
 * samples of type dst_t; the destination size is the target size (the
 * paper's ops take a pre-sized output, Sec. IV-B/IV-C listings).
 * border / border_value: tap rule for taps outside the source (only reached
 * when upsampling; OpenCV-style resizes use KR_BORDER_REPLICATE).
 * norm: NULL, or per-channel normalisation (F32 destination only).
 */
kr_status kr_resize_bilinear(const void *src, int src_h, int src_w, int c, kr_dtype src_t,
                             void *dst, int dst_h, int dst_w, kr_dtype dst_t,
                             kr_border border, float border_value, const kr_normalize *norm,
                             void *stream);

/*
 * Nearest-neighbour resize of one image (the paper's other benchmarked
 * resize, Sec. III): output pixel (x, y) copies the source sample at column
 * floor((x + 1/2) * src_w / dst_w) and row floor((y + 1/2) * src_h / dst_h),
 * exact integer quotients (never outside the source, so no border rule).
 * Same arguments and type pairs as kr_resize_bilinear without the border;
 * an F32 destination takes v * 1 or the normalisation of norm.
 */
kr_status kr_resize_nearest(const void *src, int src_h, int src_w, int c, kr_dtype src_t,
                            void *dst, int dst_h, int dst_w, kr_dtype dst_t,
                            const kr_normalize *norm, void *stream);

/*
 * Flip of one image (Sec. III "horizontal flip"): dst(x, y) = src(flip_x ?
 * w-1-x : x, flip_y ? h-1-y : y), every channel; src and dst have the same
 * size and type t (U8 or F32; f32 samples are moved bit for bit).
 * flip_x, flip_y: 0 or 1.
 */
kr_status kr_flip(const void *src, int h, int w, int c, kr_dtype t, void *dst, int flip_x, int flip_y,
                  void *stream);

/*
 * RGB to gray of one image (Sec. III "RGB to grayscale"), ITU-R BT.601 luma:
 * src h x w x 3, dst h x w x 1.  U8 -> U8: (4899 R + 9617 G + 1868 B + 2^13)
 * >> 14 (OpenCV-style 14-bit weights summing to 2^14).  F32 output: 0.299 R +
 * 0.587 G + 0.114 B on the sample scale, then norm (mean[0], std[0]) if given.
 * Type pairs as for the resizes.
 */
kr_status kr_rgb_to_gray(const void *src, int h, int w, kr_dtype src_t, void *dst, kr_dtype dst_t,
                         const kr_normalize *norm, void *stream);

/*
 * Bilinear affine warp of one image (Sec. II-A geometric transforms).
 * m: HOST pointer to the row-major 2x3 matrix [[a, b, c], [d, e, f]].  It
 * maps source to destination unless flags contains KR_WARP_INVERSE_MAP.  A
 * forward matrix is inverted on the host by kr_invert_affine().
 * Every destination pixel is written: taps outside the source follow border.
 * Returns KR_ERR_SINGULAR_MATRIX for a non-finite matrix or, for a forward
 * matrix, |det| <= 1e-12 * max(|a|, |b|, |d|, |e|)^2.
 */
kr_status kr_warp_affine(const void *src, int src_h, int src_w, int c, kr_dtype src_t,
                         void *dst, int dst_h, int dst_w, kr_dtype dst_t,
                         const double m[6], int flags,
                         kr_border border, float border_value, const kr_normalize *norm,
                         void *stream);

/*
 * Bilinear perspective warp of one image (a homography; Sec. II-A geometric
 * transforms beyond the affine case).  m: HOST pointer to the row-major 3x3
 * matrix, source to destination unless flags contains KR_WARP_INVERSE_MAP
 * (then it is the inverse map [[A, B, C], [D, E, F], [G, H, I]]; a forward
 * matrix is inverted by kr_invert_homography).  Destination pixel (x, y):
 * w = fma(G, x, fma(H, y, I)), xs = fma(A, x, fma(B, y, C)) / w,
 * ys = fma(D, x, fma(E, y, F)) / w in binary64 (correctly rounded
 * quotients); a quotient that is not a number reads as -2; then the clamp,
 * taps, weights, borders and outputs of kr_warp_affine.  Returns
 * KR_ERR_SINGULAR_MATRIX for a non-finite matrix or, for a forward matrix,
 * det = 0 or |det| <= 1e-12 * max|m_ij|^3.
 */
kr_status kr_warp_perspective(const void *src, int src_h, int src_w, int c, kr_dtype src_t,
                              void *dst, int dst_h, int dst_w, kr_dtype dst_t,
                              const double m[9], int flags,
                              kr_border border, float border_value, const kr_normalize *norm,
                              void *stream);

/*
 * Inverse of the 3x3 homography m (host arrays, row-major) by the adjugate:
 * cofactors c_ij as differences of two rounded products (c00 = m4 m8 - m5 m7,
 * c01 = m5 m6 - m3 m8, c02 = m3 m7 - m4 m6, c10 = m2 m7 - m1 m8,
 * c11 = m0 m8 - m2 m6, c12 = m1 m6 - m0 m7, c20 = m1 m5 - m2 m4,
 * c21 = m2 m3 - m0 m5, c22 = m0 m4 - m1 m3), det = (m0 c00 + m1 c01) + m2 c02,
 * inv[3 r + k] = c_kr / det.  Same singularity rule as kr_warp_perspective.
 */
kr_status kr_invert_homography(const double m[9], double inv[9]);

/*
 * Source views (zero-copy crops and slices of a larger image, Sec. II-B.3):
 * the same operators reading a source whose rows are src_pitch BYTES apart
 * instead of src_w * c elements.  src points at the view's first pixel; pixel
 * (x, y) of the view starts at src + y * src_pitch + x * c * elem_size.
 *  - src_pitch = 0 means contiguous and is the plain entry point (src then
 *    16-byte aligned as usual);
 *  - otherwise src_pitch must be a whole number of pixels (c * elem_size
 *    bytes) and at least one row (src_w * c * elem_size), and src must lie a
 *    whole number of pixels past a 16-byte boundary: any pixel-aligned view
 *    into a 16-byte-aligned buffer qualifies (KR_ERR_INVALID_ARGUMENT else);
 *  - the view may span at most 2^31 - 32 pixels of its buffer, counted from
 *    the 16-byte boundary at or below src;
 *  - bytes read: the view's pixels, the bytes between its rows that the
 *    kernels' 16-byte row loads cover, and at most the aligned dwords that
 *    hold its first and last bytes; nothing before the dword holding the
 *    first byte or after the dword holding the last one;
 *  - dst is written exactly as by the plain entry point; it must not overlap
 *    the source's span (first to last byte, pitch included).
 * The output equals the plain entry point's on a contiguous copy of the view,
 * bit for bit.
 */
kr_status kr_resize_bilinear_view(const void *src, int src_h, int src_w, size_t src_pitch, int c, kr_dtype src_t,
                                  void *dst, int dst_h, int dst_w, kr_dtype dst_t,
                                  kr_border border, float border_value, const kr_normalize *norm, void *stream);
kr_status kr_warp_affine_view(const void *src, int src_h, int src_w, size_t src_pitch, int c, kr_dtype src_t,
                              void *dst, int dst_h, int dst_w, kr_dtype dst_t,
                              const double m[6], int flags,
                              kr_border border, float border_value, const kr_normalize *norm, void *stream);
kr_status kr_warp_perspective_view(const void *src, int src_h, int src_w, size_t src_pitch, int c, kr_dtype src_t,
                                   void *dst, int dst_h, int dst_w, kr_dtype dst_t,
                                   const double m[9], int flags,
                                   kr_border border, float border_value, const kr_normalize *norm, void *stream);
kr_status kr_resize_nearest_view(const void *src, int src_h, int src_w, size_t src_pitch, int c, kr_dtype src_t,
                                 void *dst, int dst_h, int dst_w, kr_dtype dst_t,
                                 const kr_normalize *norm, void *stream);
/* Flip and RGB -> gray of a source view; the destination (h x w) is contiguous. */
kr_status kr_flip_view(const void *src, int h, int w, size_t src_pitch, int c, kr_dtype t,
                       void *dst, int flip_x, int flip_y, void *stream);
kr_status kr_rgb_to_gray_view(const void *src, int h, int w, size_t src_pitch, kr_dtype src_t,
                              void *dst, kr_dtype dst_t, const kr_normalize *norm, void *stream);

/*
 * Resize / affine warp fused with RGB -> gray (ITU-R BT.601 luma): the
 * source is an RGB u8 image (src_pitch bytes between rows, 0 = contiguous;
 * the rules of kr_resize_bilinear_view), dst one channel of dst_h x dst_w,
 * u8 or f32 (KR_ERR_UNSUPPORTED otherwise).  The result equals the operator
 * (kr_resize_bilinear / kr_warp_affine with u8 source and dst_t output,
 * without normalisation) followed by kr_rgb_to_gray, bit for bit, in one
 * pass: u8 interpolates each channel to u8 (11-bit weights), then takes the
 * 14-bit gray weights with their rounding; f32 combines the 0..255 channel
 * values in binary32.  norm (f32 only) normalises the gray with mean[0] and
 * std[0]; border_value is a u8 sample in [0, 255] for either output type.
 * The paper benchmarks resizing and RGB -> gray as operators (Sec. III) and
 * converts captured frames to gray (Sec. IV-B).
 */
kr_status kr_resize_bilinear_gray(const void *src, int src_h, int src_w, size_t src_pitch, void *dst, int dst_h,
                                  int dst_w, kr_dtype dst_t, kr_border border, float border_value,
                                  const kr_normalize *norm, void *stream);
kr_status kr_warp_affine_gray(const void *src, int src_h, int src_w, size_t src_pitch, void *dst, int dst_h,
                              int dst_w, kr_dtype dst_t, const double m[6], int flags, kr_border border,
                              float border_value, const kr_normalize *norm, void *stream);

/* One image of a batch.  op: 0 = resize, 1 = warp.  m and flags are read for
 * warps only (same meaning as in kr_warp_affine).  src_pitch: bytes between
 * source rows, 0 for a contiguous source, else a view with the rules of
 * kr_resize_bilinear_view. */
typedef struct {
    int op;
    const void *src;
    int src_h, src_w;
    void *dst;
    int dst_h, dst_w;
    double m[6];
    int flags;
    size_t src_pitch;
} kr_batch_item;

#define KR_OP_RESIZE 0
#define KR_OP_WARP 1

/* Device workspace bytes kr_resize_batch needs for n items. */
size_t kr_resize_batch_workspace_size(int n);

/*
 * Many resizes and warps of uneven sizes in one launch per operation (all
 * resizes in one, all warps in another) over a work-list of output tiles
 * spanning every image (the batched form of the operators above).
 * items: HOST array of n items, all with c channels and types (src_t, dst_t);
 * border, border_value and norm apply to every item.  workspace: DEVICE
 * buffer of at least kr_resize_batch_workspace_size(n) bytes, owned by the
 * caller and not touched by other work until the batch completes.  Each
 * item's output is bit-identical to the single-image call on the same item.
 * Destinations must not overlap each other or any source.  Batched launches
 * take u8 sources with 1-4 channels (KR_ERR_UNSUPPORTED otherwise).
 */
kr_status kr_resize_batch(const kr_batch_item *items, int n, int c, kr_dtype src_t, kr_dtype dst_t,
                          kr_border border, float border_value, const kr_normalize *norm,
                          void *workspace, size_t workspace_bytes, void *stream);

/*
 * Destination layouts of the batched forms: interleaved HWC (as everywhere
 * else) or planar CHW (channel c of pixel (x, y) at c * dst_h * dst_w +
 * y * dst_w + x; a batch of equal-size outputs packed back to back is then an
 * NCHW tensor, the layout models consume).
 */
#define KR_LAYOUT_HWC 0
#define KR_LAYOUT_CHW 1

/* kr_resize_batch with an explicit destination layout (KR_LAYOUT_*);
 * KR_ERR_INVALID_ARGUMENT for another value.  The destination of each item
 * still spans dst_h * dst_w * c samples. */
kr_status kr_resize_batch_ex(const kr_batch_item *items, int n, int c, kr_dtype src_t, kr_dtype dst_t,
                             kr_border border, float border_value, const kr_normalize *norm, int dst_layout,
                             void *workspace, size_t workspace_bytes, void *stream);

/*
 * kr_resize_batch_ex for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same validation, kernels and outputs (bit-identical to
 * kr_resize_batch_ex on the same items), with the work-list written to a
 * device scratch array of the library's own instead of a caller workspace.
 *  - The scratch is KR_NOALLOC_SCRATCH_BYTES (1 MiB) per GPU, held from the
 *    library's load until the process ends; a batch may have at most
 *    KR_NOALLOC_MAX_ITEMS items (KR_ERR_WORKSPACE_TOO_SMALL beyond that,
 *    nothing enqueued).
 *  - The call allocates no device memory (no hipMalloc, hipFree or
 *    allocating library routine); it uploads the work-list with one
 *    hipMemcpyAsync from host memory on stream, then launches.
 *  - Every call on one GPU shares that GPU's scratch, which keeps the last
 *    call's work-list: calls on one GPU must be ordered (issued on one stream,
 *    or synchronised); calls that overlap on one GPU race and may read each
 *    other's work-lists.
 *  - The scratch of a device is looked up (hipGetSymbolAddress) on the first
 *    call with that device current; KR_ERR_HIP if that fails.
 */
#define KR_NOALLOC_SCRATCH_BYTES (1u << 20)
#define KR_NOALLOC_MAX_ITEMS 4096
kr_status kr_resize_batch_noalloc(const kr_batch_item *items, int n, int c, kr_dtype src_t, kr_dtype dst_t,
                                  kr_border border, float border_value, const kr_normalize *norm, int dst_layout,
                                  void *stream);

/*
 * A reusable batch: kr_batch_plan_create validates the items, builds the
 * work-list once (it allocates and fills its own device memory, synchronously)
 * and captures the batch's launches into a HIP graph (kernel nodes only).
 * kr_batch_plan_launch replays that graph on stream.  Replays of one plan are
 * ordered: a replay on another stream starts after the previous replay has
 * completed.  Source and destination buffers named by the items must stay
 * valid while the plan is used.
 * kr_batch_plan_destroy waits for the plan's own replays (no other work of
 * the device) and frees it; NULL is ignored.
 */
typedef struct kr_batch_plan kr_batch_plan;
kr_status kr_batch_plan_create(const kr_batch_item *items, int n, int c, kr_dtype src_t,
                               kr_dtype dst_t, kr_border border, float border_value,
                               const kr_normalize *norm, kr_batch_plan **plan);
/* kr_batch_plan_create with an explicit destination layout (KR_LAYOUT_*). */
kr_status kr_batch_plan_create_ex(const kr_batch_item *items, int n, int c, kr_dtype src_t,
                                  kr_dtype dst_t, kr_border border, float border_value,
                                  const kr_normalize *norm, int dst_layout, kr_batch_plan **plan);
kr_status kr_batch_plan_launch(kr_batch_plan *plan, void *stream);
void kr_batch_plan_destroy(kr_batch_plan *plan);

/*
 * Inverse of the 2x3 affine map m (host arrays, row-major) by the fixed
 * formula: det = a*e - b*d (two rounded products, one rounded difference);
 * A = e/det, B = -b/det, D = -d/det, E = a/det; C = -(A*c + B*f),
 * F = -(D*c + E*f).  Same singularity rule as kr_warp_affine.
 */
kr_status kr_invert_affine(const double m[6], double inv[6]);

/*
 * Request server: continuous batching of resize / warp requests on one GPU.
 *
 * Requests wait in a FIFO queue.  Whenever one of `slots` in-flight batch
 * slots (one HIP stream each) is free, queued requests are admitted in
 * arrival order into a new batch while their outputs fit in the output arena
 * (budget_bytes of device memory, allocated once by kr_server_create) and the
 * batch holds fewer than max_batch requests; the batch is launched at once
 * (a work-list launch as in kr_resize_batch) and batches of different slots
 * run concurrently.  Every output is bit-identical to the single-image call.
 * Outputs stay in the arena until kr_server_release().  Sources are caller
 * owned device images that must stay valid until their request completes.
 * A server is driven by one host thread at a time (calls on one server must
 * not overlap); different servers are independent.  Supported: u8 sources
 * with 1-4 channels, u8 or f32 outputs.
 */
typedef struct kr_server kr_server;

typedef struct {
    size_t budget_bytes; /* output arena size (>= 256) */
    int slots;           /* batches in flight, 1..16 */
    int max_batch;       /* requests per batch, 1..4096 */
} kr_server_config;

/* One request; op 0 = resize, 1 = warp (m, flags as in kr_warp_affine). */
typedef struct {
    int op;
    const void *src;
    int src_h, src_w;
    int dst_h, dst_w;
    double m[6];
    int flags;
} kr_request;

typedef struct {
    uint64_t id;      /* as returned by kr_server_submit */
    void *dst;        /* device pointer to the output (dst_h x dst_w x c) in the arena */
    size_t dst_bytes;
    double t_done;    /* server clock (seconds) when the completion was observed */
} kr_completion;

kr_status kr_server_create(const kr_server_config *cfg, int c, kr_dtype src_t, kr_dtype dst_t, kr_border border,
                           float border_value, const kr_normalize *norm, kr_server **server);
/* Seconds since the server was created (the clock of t_done). */
double kr_server_now(const kr_server *server);
/* Queue one request.  KR_ERR_OUT_OF_BUDGET if its output can never fit. */
kr_status kr_server_submit(kr_server *server, const kr_request *req, uint64_t *id);
/* Make progress (harvest finished batches, admit and launch new ones) and
 * return up to max_out completions (*n_out of them). */
kr_status kr_server_poll(kr_server *server, kr_completion *out, int max_out, int *n_out);
/* Free a completed request's output block. */
kr_status kr_server_release(kr_server *server, uint64_t id);
kr_status kr_server_stats(const kr_server *server, size_t *arena_used, size_t *queued, int *busy_slots);
/*
 * Replay a request trace on the host clock: request i is submitted when
 * arrival_s[i] seconds (ascending) have passed since the call started; every
 * output is released as soon as it completes.  latency_s[i] = completion
 * observed - arrival_s[i].  Needs an idle server with nothing unreleased.
 */
kr_status kr_server_run_trace(kr_server *server, const kr_request *reqs, const double *arrival_s, int n,
                              double *latency_s);
/* Waits for in-flight work, then frees everything; NULL is ignored. */
void kr_server_destroy(kr_server *server);

/*
 * Autotuner: picks the tile shape and pixels-per-thread of the u8-source
 * kernels by timing every compiled configuration on the caller's own workload
 * (the project-written tuner of the batched path).  The winner is recorded in
 * a process-wide table keyed by (operation, channels, output type, single
 * image or batch, half-octave class of source pixels per output pixel,
 * factor-4 class of output pixels); later launches of the same class use it.
 * Every configuration computes bit-identical results, so tuning changes
 * speed only.  The table is loaded from the text file named by the
 * environment variable KR_AUTOTUNE_CACHE on first use, if set.
 *
 * kr_autotune_image: same arguments as kr_resize_bilinear (op 0) or
 * kr_warp_affine (op 1), plus reps timed launches per configuration (1..1000).
 * It launches on stream, synchronises it, and leaves the correct output in
 * dst.  report: NULL, or a host buffer receiving a one-line summary.
 * scrub: NULL (launches timed back to back: a source that stays in the
 * caches) or a DEVICE buffer of scrub_bytes (16-byte aligned, >= 32, best
 * larger than the 256 MB last-level cache) overlapping no other argument,
 * whose contents the tuner overwrites before each launch so that the source
 * is read from HBM and the previous output is written back, as in a stream
 * of distinct images; the time of the overwrites alone is subtracted.
 * Only u8 sources with 3 or 4 channels have configurations
 * (KR_ERR_UNSUPPORTED otherwise; one- and two-channel sources run fixed
 * configurations).
 * kr_autotune_batch: same arguments as kr_resize_batch plus reps, scrub and
 * report; tunes the resize and the warp launch of the batch separately.
 * kr_autotune_save: writes the table as text into buf (truncated to len
 * bytes, NUL-terminated) and returns the bytes the full text needs.
 * kr_autotune_load: merges a text table (as written by kr_autotune_save).
 * Its first entry line is "key <arch> <hash>", the build key of the library
 * that measured it (kr_build_key); a table with another key is stale
 * (another GPU architecture, or kernels edited since) and is ignored
 * (KR_ERR_UNSUPPORTED, table unchanged).  A missing key, a malformed line or
 * an unknown configuration rejects the whole text (KR_ERR_INVALID_ARGUMENT,
 * table unchanged).  The KR_AUTOTUNE_CACHE file follows the same rules (a
 * rejected file is reported on stderr and ignored).
 * kr_build_key: "<arch> <hash>", static text: the GPU architecture the
 * library was compiled for and a hash of its kernel sources.
 * kr_autotune_clear: empties the table (launches return to the defaults).
 */
kr_status kr_autotune_image(int op, const void *src, int src_h, int src_w, int c, kr_dtype src_t, void *dst,
                            int dst_h, int dst_w, kr_dtype dst_t, const double m[6], int flags, kr_border border,
                            float border_value, const kr_normalize *norm, int reps, void *scrub,
                            size_t scrub_bytes, void *stream, char *report, size_t report_len);
kr_status kr_autotune_batch(const kr_batch_item *items, int n, int c, kr_dtype src_t, kr_dtype dst_t,
                            kr_border border, float border_value, const kr_normalize *norm, void *workspace,
                            size_t workspace_bytes, int reps, void *scrub, size_t scrub_bytes, void *stream,
                            char *report, size_t report_len);
size_t kr_autotune_save(char *buf, size_t len);
kr_status kr_autotune_load(const char *text);
const char *kr_build_key(void);
void kr_autotune_clear(void);

/* Static text for a status code. */
const char *kr_status_string(kr_status s);

/* Message describing the last failed call on this thread ("" if none). */
const char *kr_last_error(void);

/*
 * Plain device-to-device copy of `bytes` bytes with 16-byte vector loads and
 * stores: the HBM-bandwidth ceiling probe the resampling kernels are measured
 * against.  dst and src must be 16-byte aligned and must not overlap.
 */
kr_status kr_hbm_copy(void *dst, const void *src, size_t bytes, void *stream);

/*
 * Traffic-mix bandwidth probe: reads src_bytes from src and writes dst_bytes
 * to dst with 16-byte vector loads and stores, so a kernel's HBM traffic (for
 * example 1 byte read per 4 written, for an RGB u8 -> f32 warp) can be timed
 * without its arithmetic.  Output chunk i (16 bytes) is the XOR of the input
 * chunks mapped to it: chunks i*k .. i*k + k - 1 when src_bytes = k *
 * dst_bytes, chunk i / k when dst_bytes = k * src_bytes, so every input byte is
 * read (k neighbouring threads share a chunk in the second case) and every
 * output byte written once.
 *   dst, src    device pointers, 16-byte aligned, not overlapping;
 *   dst_bytes,  multiples of 16, > 0, whose ratio (either way round) is a
 *   src_bytes   power of two, with at most 256 input chunks per output chunk.
 * Errors: KR_ERR_INVALID_ARGUMENT (nothing launched); KR_ERR_HIP.
 */
kr_status kr_hbm_stream(void *dst, size_t dst_bytes, const void *src, size_t src_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* KR_H */
