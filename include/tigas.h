/*
 * tigas.h -- C ABI of the MI355X (gfx950) forward 3D Gaussian Splatting
 * rasterizer behind the TIGAS rendering backend (arXiv 2605.08699).
 *
 * The paper's backend (Section 4.1 and Section 5.1) keeps parsed Gaussian
 * scenes resident in GPU memory and renders, per stateless client request
 * (Section 4.2), one frame from a 6DoF pose, pinhole intrinsics and an ABR
 * resolution rung with a tile-based rasterizer.  This library is that
 * rasterizer: a resident-scene loader and a render call, plus the batched
 * (many views, one launch sequence) and serving (request loop) forms; around
 * it, the backend's JPEG payload encoder (on the GPU), the adaptive client's
 * latency ABR controller and the scene registry that parses PLY models and
 * loads, shares and unloads them (host code).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns a tigas_status; TIGAS_OK is 0, errors are negative.
 *   A failing call writes a message retrievable with tigas_last_error() on
 *   the same thread and leaves its outputs unspecified.  No C++ exception
 *   crosses the boundary.
 * - "device" pointers are HIP device addresses valid on the context's
 *   device; "host" pointers are ordinary process memory.
 * - A pose is (R, t): R is the camera-to-world rotation (row-major 3x3,
 *   columns are the camera axes in world coordinates; x right, y down,
 *   z forward), t the camera centre.  The world-to-camera transform is
 *   [R^T, -R^T t] (Section 5.1, Rendering Engine).
 * - Intrinsics are given for the full (width, height) frame.  A render at
 *   resolution scale s produces out_w = floor(width*s + 0.5) by
 *   out_h = floor(height*s + 0.5) pixels with fx, cx multiplied by
 *   out_w/width and fy, cy by out_h/height (the principal point is
 *   re-centred with the frame, Section 5.1), each rounded to FP32.
 * - Frames are row-major HWC, row 0 at the top, RGB interleaved; RGB8 is
 *   floor(clamp(c, 0, 1) * 255 + 0.5), RGBF32 is the unclamped composite.
 * - Degenerate Gaussians (non-finite attributes, zero quaternion, centre at
 *   or in front of the z = 0.2 near plane) are dropped, not reported as
 *   errors; a scene with no Gaussians renders the background.
 */
#ifndef TIGAS_H
#define TIGAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TIGAS_OK = 0,
    TIGAS_E_INVALID = -1, /* null pointer, out-of-range argument, non-finite pose */
    TIGAS_E_OOM = -2,     /* device allocation failed */
    TIGAS_E_DEVICE = -3,  /* a HIP runtime call failed (message names it) */
    TIGAS_E_BUFFER = -4,  /* caller's output buffer too small (sizes still filled in) */
    TIGAS_E_BUDGET = -5   /* serving: request larger than the whole memory budget */
} tigas_status;

/* Storage precision of the resident Gaussian attributes.  Centres are always
 * FP32; with F16/BF16 the log-scales, quaternion, opacity logit and SH
 * coefficients are stored rounded to nearest-even and decoded to FP32 before
 * any arithmetic. */
typedef enum { TIGAS_ATTR_F32 = 0, TIGAS_ATTR_F16 = 1, TIGAS_ATTR_BF16 = 2 } tigas_attr;

typedef enum { TIGAS_OUT_RGB8 = 0, TIGAS_OUT_RGBF32 = 1 } tigas_format;

typedef struct tigas_context tigas_context;
typedef struct tigas_scene tigas_scene;

/* Scene attributes as parsed from a 3DGS PLY (Section 5.1, PLY Model and
 * Primitives): n centres [n][3], log-scales [n][3] (exponentiated), quaternions
 * [n][4] as (w, x, y, z) (normalised by the renderer), opacity logits [n]
 * (passed through a sigmoid) and SH coefficients [n][16][3] (coefficient-major;
 * entries above sh_degree are ignored).  All arrays are FP32, host memory when
 * is_device == 0, device memory of the context's device otherwise.  The
 * library copies them into its own resident layout; the caller keeps
 * ownership. */
typedef struct {
    int64_t n;
    int sh_degree; /* 0..3 */
    const float* means;
    const float* log_scales;
    const float* quats_wxyz;
    const float* opacity_logits;
    const float* sh;
    int is_device;
    tigas_attr storage;
} tigas_scene_desc;

typedef struct {
    float R[9]; /* camera -> world, row-major */
    float t[3]; /* camera centre in world coordinates */
} tigas_pose;

typedef struct {
    float fx, fy, cx, cy; /* pixels, for the full (width, height) frame */
} tigas_intrinsics;

/* Per-request quality knobs.  Zero-initialised means: full resolution,
 * SH degree 0 (the colour of the DC term only, the paper's default in
 * Section 5.1), RGB8, black background, autotuned tile/batch. */
typedef struct {
    float res_scale;  /* ABR rung, (0, 1]; 0 means 1 */
    int sh_degree;    /* 0 .. the scene's degree; < 0: the scene's degree; above it: E_INVALID */
    tigas_format fmt;
    float bg[3];
    int tile_w, tile_h; /* 8x8, 16x16, 16x32 or 32x16; 0x0 = autotuned for the workload's shape */
    int batch_depth;    /* Gaussians staged per wavefront batch: 64, 128 or 256; 0 = autotuned (64 with an explicit tile) */
    int pixels_per_lane; /* blend pixels per lane, 1 or 2 (tiles 16 or more tall); 0 = autotuned (1 with an
                            explicit tile).  Frames are identical for every choice of these three fields. */
} tigas_quality;

/* Output frame.  data: device pointer when is_device, host otherwise;
 * capacity in bytes.  out_w/out_h are written by the render call. */
typedef struct {
    void* data;
    size_t capacity;
    int is_device;
    int out_w, out_h;
} tigas_frame;

/* Counters of the last render on a context (read after it completed). */
typedef struct {
    int64_t n;          /* Gaussians in the scene(s) rendered */
    int64_t visible;    /* Gaussians that touched at least one tile */
    int64_t duplicates; /* D: (Gaussian, tile) pairs sorted */
    int64_t fallbacks;  /* 2D covariances inverted on the FP64 path */
    int64_t tiles;
    int64_t sort_passes;
    int64_t rerenders;  /* workspace regrowths after an overflowing first attempt */
    int32_t tile_w, tile_h, batch_depth, pixels_per_lane; /* configuration used (requested or autotuned) */
} tigas_stats;

/* Creates a context on HIP device `device`: a stream, workspaces and the
 * tuning cache (the autotuner's choices per workload shape; persisted in the
 * file named by the environment variable TIGAS_TUNE_CACHE when set).  *out
 * is owned by the caller; free with tigas_context_destroy.
 * Environment read here: TIGAS_GRAPHS=0 (no graph capture),
 * TIGAS_BLEND_CULL=0 (the blend keeps every list entry whose pixel box meets
 * a wave's block, instead of also dropping those whose exponent stays below
 * the skip threshold on the whole block; frames are identical either way). */
tigas_status tigas_context_create(int device, tigas_context** out);
void tigas_context_destroy(tigas_context* ctx);

/* Loads a scene into resident device memory (Section 4.1: persistent VRAM
 * residency).  The scene is immutable and may be rendered by any number of
 * concurrent calls.  E_INVALID for n < 0, null arrays with n > 0, a degree
 * outside 0..3; E_OOM when device memory is exhausted. */
tigas_status tigas_scene_load(tigas_context* ctx, const tigas_scene_desc* desc, tigas_scene** out);
void tigas_scene_free(tigas_scene* scene);
/* Bytes of device memory the scene holds. */
size_t tigas_scene_bytes(const tigas_scene* scene);

/* Renders one frame (Section 5.1, Rendering Engine): preprocess, duplicate
 * with (tile | depth) keys, radix sort, tile ranges, front-to-back blend.
 * hip_stream: a hipStream_t of the context's device or NULL for the context
 * stream.  The call returns once the frame is complete in `out`.  E_BUFFER
 * when out->capacity < out_w*out_h*3*(1 or 4) bytes (out_w and out_h are
 * still written); E_INVALID for null or non-finite arguments and for a
 * q->sh_degree above the scene's degree. */
tigas_status tigas_render(tigas_scene* scene, const tigas_pose* pose, const tigas_intrinsics* intr,
                          int width, int height, const tigas_quality* q, tigas_frame* out, void* hip_stream);

/* The same frame without waiting for it: the frame is launched on the stream
 * (after everything already queued there) and *ticket names it.  At most two
 * frames per stream are in flight: submitting a third first completes the
 * oldest.  `out` must be device memory (out->is_device) that stays valid until
 * the frame is waited for; stage and kernel timing must be off.  Frames on
 * one stream still execute one after the other, so the host prepares and
 * launches a frame while the previous one renders.  E_INVALID for a host
 * output or timing on; the other errors as tigas_render. */
tigas_status tigas_render_submit(tigas_scene* scene, const tigas_pose* pose, const tigas_intrinsics* intr,
                                 int width, int height, const tigas_quality* q, tigas_frame* out, void* hip_stream,
                                 int64_t* ticket);
/* Waits for a submitted frame and collects it (once): its statistics
 * (may be NULL) and its GPU time in milliseconds, from events recorded on
 * the stream just before and after its launch sequence (may be NULL).  A
 * frame whose duplicates overflowed is rendered again here (its GPU time is
 * that of the first attempt).  E_INVALID for an unknown or collected ticket;
 * the frame's own error otherwise. */
tigas_status tigas_render_wait(tigas_context* ctx, int64_t ticket, tigas_stats* stats, float* gpu_ms);

/* ---------------------------------------------------------------------------
 * Allocation-free render, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  It renders the same frame as tigas_render with the same tile
 * configuration, but every buffer of its launch sequence lies in one static
 * device array of TIGAS_NOALLOC_SCRATCH_BYTES per device (set up when a
 * context is created on the device, held until the process ends); the call
 * allocates nothing, neither device nor pinned host memory.
 *
 * The launch sequence is enqueued on hip_stream (NULL: the context stream)
 * and the call returns without waiting; the frame is complete when the
 * stream has passed it, and `scene` must stay loaded until then.  Only
 * kernels are enqueued (no memset or copy), so the call may be captured.
 * out must be device memory (out->is_device); out_w/out_h are written.
 * Tiles: q's tile_w/tile_h/batch_depth/pixels_per_lane, or 16x16, depth 64,
 * one pixel per lane when zero (no autotuner).
 * counters: device-accessible memory (device, or pinned host) that receives
 * the frame's counters when it completes; may be NULL.  When the frame has
 * more (Gaussian, tile) pairs than the array holds, nothing is composited
 * (the frame is the background) and counters->overflow is 1: the caller
 * renders it with tigas_render instead.
 * Limits: the scene's records (n rounded up to 256) take 92 bytes each and
 * every (Gaussian, tile) pair 24 bytes, out of the 64 MiB; a scene whose
 * records leave fewer pair slots than records is refused with E_INVALID.
 * Every call on one device shares that device's array and leaves its
 * contents there: calls that overlap on one device (other streams, other
 * threads) race and must be serialised by the caller.
 * Errors as tigas_render, plus E_INVALID for a host frame.
 * ------------------------------------------------------------------------- */
#define TIGAS_NOALLOC_SCRATCH_BYTES (64u << 20)

typedef struct {
    uint32_t duplicates; /* D: (Gaussian, tile) pairs (saturates at 2^32-1) */
    uint32_t visible;    /* Gaussians that touched a tile */
    uint32_t fallbacks;  /* 2D covariances inverted on the FP64 path */
    uint32_t overflow;   /* 1: more pairs than the scratch array holds; the frame is the background */
    uint32_t reserved[2];
} tigas_frame_counters;

tigas_status tigas_render_noalloc(tigas_scene* scene, const tigas_pose* pose, const tigas_intrinsics* intr,
                                  int width, int height, const tigas_quality* q, tigas_frame* out,
                                  tigas_frame_counters* counters, void* hip_stream);

/* Renders n_views views, each with its own scene, pose, intrinsics, size and
 * quality q[i] (rung, SH degree, format, background; q may be NULL for
 * defaults; the tile size and batch depth of q[0] apply to all views), with one
 * launch sequence: one preprocess over all (view, Gaussian) pairs, one sort
 * over global tile ids, one blend launch over every tile of every view.
 * Captured into a HIP graph and replayed when the view shapes repeat.
 * Frames are identical to n_views separate tigas_render calls. */
tigas_status tigas_render_batch(tigas_scene* const* scenes, const tigas_pose* poses,
                                const tigas_intrinsics* intrs, const int* widths, const int* heights,
                                const tigas_quality* q, int n_views, tigas_frame* outs, void* hip_stream);

tigas_status tigas_last_stats(tigas_context* ctx, tigas_stats* out);

/* Stage timing with HIP events recorded on the rendering stream around each
 * stage of every render on this context (preprocess, block scan, duplicate,
 * radix sort, tile ranges, blend); while it is on, launch sequences run
 * uncaptured (events between the launches).  tigas_profile_stages switches it on or
 * off and resets the accumulated milliseconds; tigas_stage_times reads them
 * (sums over `frames` renders). */
typedef struct {
    double preprocess, scan, duplicate, sort, ranges, blend; /* milliseconds */
    int64_t frames;
} tigas_stage_ms;

tigas_status tigas_profile_stages(tigas_context* ctx, int enable);
/* Launch sequences are captured into HIP graphs per workload shape and
 * replayed (default on; environment TIGAS_GRAPHS=0 turns it off at context
 * creation).  This switches it for the context. */
tigas_status tigas_set_graphs(tigas_context* ctx, int enable);
/* Single-view renders place the tile digit of the (tile | depth) keys by
 * counting (per-block tile histograms of the depth-ordered Gaussians, then
 * each entry written straight to its sorted position) when the view's tile
 * grid has at most 8192 tiles; otherwise, and when this is switched off
 * (environment TIGAS_TILE_BIN=0 at context creation), by radix passes over the
 * emitted duplicates.  The sorted lists are identical either way. */
tigas_status tigas_set_tile_binning(tigas_context* ctx, int enable);
/* Tighter tile culling: a (Gaussian, tile) entry of the tile lists is
 * emitted only when the Gaussian's exponent can reach the skip threshold at
 * one of the tile's pixel centres (the exact maximum of the concave quadratic
 * over the tile's pixel rectangle, with the blend's rounding margin), not for
 * every tile of its bounding rectangle.  Fewer entries to sort and stage;
 * frames are identical (a dropped entry is one every pixel of its tile would
 * skip).  Off by default (environment TIGAS_TILE_CULL=1 at context creation
 * turns it on); while on, single views use the radix tile passes, since the
 * counting placement needs whole rectangles. */
tigas_status tigas_set_tile_culling(tigas_context* ctx, int enable);
/* Depth order of the visible Gaussians (the depth digits of the radix sort,
 * Sections 4.1 and 5.1): passes = 3 (the default) sorts the FP32 depth bits
 * less the frame's smallest visible depth key in three passes of 9-bit
 * digits when those keys span less than 2^27 (depths within about 16
 * octaves) and every view has at most 256 x 256 tiles; a frame whose keys
 * span more is detected on the GPU, rendered again with four passes, and the
 * context keeps four passes from then on (counted in tigas_stats.rerenders).
 * passes = 4 always takes four 8-bit passes of the whole key (environment
 * TIGAS_DEPTH_PASSES=4 at context creation).  The order, and so every frame,
 * is identical either way.  E_INVALID for another value. */
tigas_status tigas_set_depth_passes(tigas_context* ctx, int passes);
tigas_status tigas_stage_times(tigas_context* ctx, tigas_stage_ms* out);

/* Kernel timing with HIP events recorded on the rendering stream around every
 * kernel launch of every render on this context; while it is on, launch
 * sequences run uncaptured.  tigas_profile_kernels switches it on or off and
 * clears the totals; tigas_kernel_times copies up to `cap` entries (kernel
 * instantiation name, launches, summed milliseconds) into the caller's
 * array, sorted by name, and sets *count to the number of kernels timed
 * (which may exceed cap).  TIGAS_E_INVALID for null pointers. */
typedef struct {
    char name[120];
    int64_t launches;
    double total_ms;
} tigas_kernel_time;

tigas_status tigas_profile_kernels(tigas_context* ctx, int enable);
tigas_status tigas_kernel_times(tigas_context* ctx, tigas_kernel_time* out, int cap, int* count);

/* Renders like tigas_render with a blend kernel that also counts the work it
 * does: *evaluations = (pixel, Gaussian) pairs whose alpha was evaluated
 * before the pixel terminated, *contributions = pairs composited. */
tigas_status tigas_count_blend_work(tigas_scene* scene, const tigas_pose* pose, const tigas_intrinsics* intr,
                                    int width, int height, const tigas_quality* q, tigas_frame* out,
                                    int64_t* evaluations, int64_t* contributions);

/* ---------------------------------------------------------------------------
 * Serving form.  Many clients send per-frame requests (pose, intrinsics, ABR
 * rung) for resident scenes (Sections 4.2 and 5.1: stateless per-frame
 * requests, one shared resident model per scene, every request an isolated
 * render task).  The server admits requests by a device-memory budget and
 * renders them with continuous batching: whenever one of its slots (a stream
 * with its own workspace) is idle, all pending requests that fit the slot's
 * share of the budget (oldest first, up to max_batch) are rendered there as
 * one launch sequence, while requests arriving meanwhile wait for the next
 * idle slot; batches on different slots overlap on the device.  Frames are
 * identical to rendering each request alone.
 * ------------------------------------------------------------------------- */
typedef struct tigas_server tigas_server;

typedef struct {
    int slots;         /* concurrent batches (streams, default priority); 0 = 2, at most 8 */
    int max_batch;     /* requests per batch; 0 = 64 */
    size_t hbm_budget; /* workspace bytes across all slots (resident scenes excluded), reserved at
                          creation; 0 = unlimited (workspaces grow on demand) */
    int supersede;     /* 1: a client's newer request replaces its request still waiting (latest pose wins) */
    int tile_w, tile_h, batch_depth; /* 0 = 16x32 tiles, depth 64 */
    int pixels_per_lane;             /* 1 or 2 (tiles 16 or more tall); 0 = 1 */
    int64_t max_batch_pixels; /* output pixels per batch (bounds a batch's duration); 0 = no cap */
} tigas_server_config;

/* One request.  The output frame must stay valid until its completion is
 * reported; `arrival_s` is used only by tigas_server_replay.  With
 * jpeg_quality 1..100 the frame (RGB8, device memory) is also encoded as the
 * per-request payload (tigas_jpeg_encode's format) into the device buffer
 * jpeg_out of jpeg_capacity bytes; 0 = no JPEG. */
typedef struct {
    tigas_scene* scene;
    tigas_pose pose;
    tigas_intrinsics intr;
    int width, height;
    tigas_quality q; /* rung, SH degree, format, background (tile fields ignored) */
    tigas_frame out;
    int client;
    double arrival_s;
    int jpeg_quality;
    void* jpeg_out;
    size_t jpeg_capacity;
} tigas_request;

/* status: 0 rendered, 1 superseded (not rendered), < 0 a tigas_status error.
 * Times in seconds on the server clock (replay: relative to its start). */
typedef struct {
    int64_t id;
    int client;
    int status;
    double arrival_s, dispatch_s, done_s; /* done: frame and payload complete */
    int batch_size;
    int64_t jpeg_bytes; /* stream length (above jpeg_capacity: only a prefix was written); 0 without JPEG */
} tigas_completion;

typedef struct {
    int64_t admitted, deferred, superseded, rendered, failed, batches, max_batch_seen, pending;
} tigas_server_stats;

/* Starts the dispatcher and slot threads.  E_INVALID for bad configuration. */
tigas_status tigas_server_create(tigas_context* ctx, const tigas_server_config* cfg, tigas_server** out);
/* Waits for every submitted request, then stops the threads and frees the
 * slot workspaces. */
void tigas_server_destroy(tigas_server* server);
/* Queues a request arriving now.  E_BUDGET when the request alone needs more
 * workspace than a slot's share of the budget; E_INVALID for bad requests. */
tigas_status tigas_server_submit(tigas_server* server, const tigas_request* req, int64_t* id);
/* Moves up to max completions (in completion order) into out; *n = count. */
tigas_status tigas_server_poll(tigas_server* server, tigas_completion* out, int max, int* n);
/* Blocks until every submitted request has completed. */
tigas_status tigas_server_drain(tigas_server* server);
/* Open-loop replay: submits reqs[i] at time reqs[i].arrival_s after the call
 * starts (from the calling thread), waits for all of them and writes the
 * completion of reqs[i] to out[i]. */
tigas_status tigas_server_replay(tigas_server* server, const tigas_request* reqs, int n, tigas_completion* out);
tigas_status tigas_server_get_stats(tigas_server* server, tigas_server_stats* out);

/* Thread-local message of the last failing call on this thread ("" if none);
 * valid until the next call on this thread. */
const char* tigas_last_error(void);

/* ---------------------------------------------------------------------------
 * Inspection of the intermediate stages of one render, for parity tests.
 * Renders like tigas_render and copies to caller-provided HOST arrays
 * (any pointer may be NULL to skip it):
 *   rec      [n][12] f32: u_hi, v_hi, u_lo, v_lo (pixel centre = u_hi + u_lo),
 *            A, B, C, L (exponent coefficients: alpha = 2^(A dx^2 + B dx dy +
 *            C dy^2 + L) before the 0.99 clamp), r, g, b, opacity
 *   bbox     [n][4] i32 inclusive pixel box x0, y0, x1, y1 (x1 < x0: empty)
 *   zkey     [n] u32 FP32 depth-key bits;  touched [n] u32 tiles overlapped
 *   keys     [cap_dup] u64 duplicate keys in emission order, vals [cap_dup] u32
 *   skeys    [cap_dup] u64 sorted keys, svals [cap_dup] u32 sorted values
 *   ranges   [tiles][2] u32 [start, end) per tile, (0, 0) for an empty tile
 * *n_dup receives D; arrays sized below D are not written (E_BUFFER).
 * ------------------------------------------------------------------------- */
typedef struct {
    float* rec;
    int32_t* bbox;
    uint32_t* zkey;
    uint32_t* touched;
    uint64_t* keys;
    uint32_t* vals;
    uint64_t* skeys;
    uint32_t* svals;
    uint32_t* ranges;
    int64_t cap_dup;
    int64_t cap_tiles;
    int64_t n_dup;
    int64_t n_tiles;
} tigas_debug_out;

tigas_status tigas_render_debug(tigas_scene* scene, const tigas_pose* pose, const tigas_intrinsics* intr,
                                int width, int height, const tigas_quality* q, tigas_frame* out,
                                tigas_debug_out* dbg);

/* Baseline JPEG of an RGB8 frame in device memory: the per-frame payload of
 * the paper's backend (Section 5.1: frames leave as 8-bit JPEG; Sections 4.2
 * and 5.2: one stateless JPEG per request), at a quality factor of its
 * bitrate ladder (Table 1: 10, 35, 65, 90).  Format:
 * JFIF, YCbCr 4:4:4, the Annex K quantisation tables of ITU-T T.81 scaled by
 * quality (5000/q percent below 50, else 200 - 2q, clamped to 1..255) and its
 * Annex K Huffman tables, restart intervals of 40 MCUs (8x8 pixel blocks).
 *   rgb: device pointer, `height` rows of 3 * `width` bytes, top row first (the
 *        RGB8 layout tigas_render writes); width and height 1..65535;
 *   quality: 1..100;
 *   out: device buffer of `capacity` bytes (tigas_jpeg_max_bytes bounds the
 *        stream); *out_len (host) receives the stream length.  A stream longer
 *        than `capacity` returns TIGAS_E_BUFFER with *out_len set and only a
 *        prefix written;
 *   hip_stream: NULL = the context stream.  The call returns when the stream
 *        has finished (the length is read back).  Scratch buffers belong to
 *        the stream's workspace; calls on one stream run one after another.
 * Errors: TIGAS_E_INVALID for null pointers or out-of-range sizes/quality. */
tigas_status tigas_jpeg_encode(tigas_context* ctx, const void* rgb, int width, int height, int quality,
                               void* out, size_t capacity, size_t* out_len, void* hip_stream);
/* Upper bound on the stream length of a width x height frame (0 for
 * non-positive sizes). */
size_t tigas_jpeg_max_bytes(int width, int height);

/* Latency ABR controller of the adaptive client (Section 5.3, Throughput
 * Monitoring and ABR Controller): per completed request the client reports
 * the payload size and its download time; the controller keeps an
 * exponential moving average (factor alpha) of the throughput over the last
 * `history` requests and picks the next request's level of the bitrate
 * ladder.  With T_l = expected_bytes[l] / (average in KB/s * 1024): up one
 * level when T_{l+1} <= t_target_s, down one when T_l > t_margin_s, each only
 * after its condition held on `hold` consecutive requests, except a downgrade
 * during rapid panning, which is immediate.  Levels are numbered by rising
 * quality (0 = the smallest rung).  Host-only; no GPU work.  A controller
 * serves one client: calls on one controller must not overlap. */
typedef struct {
    int n_levels;              /* 1..8 */
    double expected_bytes[8];  /* expected payload per level, rising */
    double t_target_s;         /* upgrade target */
    double t_margin_s;         /* downgrade margin, above the target */
    double alpha;              /* moving-average factor, 0 < alpha <= 1 */
    int history;               /* requests in the average, 1..64 */
    int hold;                  /* consecutive requests before a change, >= 1 */
    int start_level;
} tigas_abr_config;
typedef struct tigas_abr tigas_abr;

/* Defaults: the four rungs of Table 1 with the middles of its size ranges
 * (7, 20, 55, 240 KB), 100 ms target, 150 ms margin, alpha 0.3, history 5,
 * hold 3, start at level 0. */
void tigas_abr_default_config(tigas_abr_config* cfg);
/* E_INVALID for out-of-range fields (cfg NULL = the defaults). */
tigas_status tigas_abr_create(const tigas_abr_config* cfg, tigas_abr** out);
void tigas_abr_destroy(tigas_abr* abr);
/* One completed request: payload bytes and download seconds (both > 0);
 * *level receives the level of the next request. */
tigas_status tigas_abr_observe(tigas_abr* abr, double bytes, double seconds, int rapid_pan, int* level);
/* The current throughput average in KB/s (0 before the first request). */
tigas_status tigas_abr_rate(const tigas_abr* abr, double* kbytes_per_s);

/* ---- Scene registry (Section 4.1, GPU Backend; Section 5.1, PLY Model and
 * Primitives and Dynamic Multi-Model Runtime) ----
 *
 * A registry scans a root directory once, at creation, for models: every
 * sub-folder holding a 3DGS PLY file (point_cloud.ply in the folder, else
 * point_cloud/iteration_<k>/point_cloud.ply with the highest k, else the
 * first *.ply in the folder by name) and every *.ply directly under the root.
 * A model's id is its folder's name (or the file's name without ".ply"); its
 * preview image is preview.{png,jpg,jpeg,webp} in the folder (or
 * <id>.{png,...} beside a root-level file).  Folders and files without a
 * readable 3DGS PLY header are not registered.
 *
 * Models are loaded on first access (acquire or load), stay resident while
 * clients hold references, and are unloaded once unreferenced and idle for at
 * least idle_timeout_s, by a sweep: tigas_registry_evict_idle, or a thread
 * of the registry every sweep_period_s.  Every function of one registry may be
 * called from any thread at any time, except destroy, which must not overlap
 * any other call on the registry.
 *
 * PLY layout read (the 3DGS training output; ascii, binary_little_endian or
 * binary_big_endian, any scalar property types): element "vertex", one per
 * Gaussian, with x y z, f_dc_0..2, f_rest_0..K-1 (K = 0, 9, 24 or 45 gives SH
 * degree 0..3; channel-major: f_rest_{c*(K/3) + k - 1} is coefficient k of
 * colour channel c), opacity (logit), scale_0..2 (log-scales) and rot_0..3
 * (w, x, y, z).  Other vertex properties and other elements are skipped;
 * vertex list properties are an error.  Values are converted to FP32 with
 * round-to-nearest. */
typedef struct tigas_registry tigas_registry;

typedef struct {
    double idle_timeout_s; /* unload after this long unreferenced; < 0: never by a sweep.  Default 300 */
    double sweep_period_s; /* > 0: a registry thread sweeps this often; 0: sweeps only on request.  Default 0 */
    tigas_attr storage;    /* resident precision of loaded models.  Default F32 */
} tigas_registry_config;

typedef struct {
    const char* id;           /* strings owned by the registry, valid until destroy */
    const char* ply_path;
    const char* preview_path; /* "" when there is none */
    int64_t n;                /* Gaussians (from the header; refreshed at each load) */
    int sh_degree;
    int loaded;               /* resident now */
    int refs;                 /* references held */
    int64_t loads;            /* times loaded since the registry was created */
    size_t device_bytes;      /* resident bytes, 0 when not loaded */
    double idle_s;            /* seconds since the last acquire, load or release (loaded models) */
} tigas_model_info;

/* Reads the header of a 3DGS PLY file: vertex count and SH degree.  Host
 * only.  E_INVALID for a missing or malformed file. */
tigas_status tigas_ply_info(const char* path, int64_t* n, int* sh_degree);
/* Reads a 3DGS PLY file into host arrays in the tigas_scene_desc layout
 * (means [n][3], log_scales [n][3], quats_wxyz [n][4], opacity_logits [n],
 * sh [n][16][3] with the coefficients above the file's degree set to 0).  n
 * must be the file's vertex count.  Host only; the caller owns the arrays.
 * E_INVALID for a malformed or truncated file (arrays then unspecified). */
tigas_status tigas_ply_read(const char* path, int64_t n, float* means, float* log_scales, float* quats_wxyz,
                            float* opacity_logits, float* sh);

void tigas_registry_default_config(tigas_registry_config* cfg);
/* Creates a registry of the models under root (cfg null: defaults).  ctx is
 * the context models load into; null gives a discovery-only registry (info
 * works, acquire and load fail with E_INVALID).  *out is owned by the
 * caller; tigas_registry_destroy before the context. */
tigas_status tigas_registry_create(tigas_context* ctx, const char* root, const tigas_registry_config* cfg,
                                   tigas_registry** out);
/* Stops the sweeping thread and frees every resident model, referenced or
 * not: scenes acquired from the registry are invalid afterwards. */
void tigas_registry_destroy(tigas_registry* reg);
/* Models registered (ordered by id). */
int64_t tigas_registry_count(const tigas_registry* reg);
tigas_status tigas_registry_info(tigas_registry* reg, int64_t index, tigas_model_info* info);
/* Returns model `id` resident, loading it first if it is not (a concurrent
 * first access waits for the one load), and takes a reference: the scene
 * stays valid until the matching tigas_registry_release.  Release only after
 * the renders of the scene have completed (serving: after their completion
 * was polled).  E_INVALID for an unknown id or a malformed file; E_OOM. */
tigas_status tigas_registry_acquire(tigas_registry* reg, const char* id, tigas_scene** out);
/* Makes model `id` resident without taking a reference (explicit loading);
 * it is then evictable once idle. */
tigas_status tigas_registry_load(tigas_registry* reg, const char* id);
/* Drops one reference taken by acquire.  E_INVALID for a scene that is not a
 * resident model of the registry or has no reference left. */
tigas_status tigas_registry_release(tigas_registry* reg, tigas_scene* scene);
/* One sweep: unloads every resident model that has no reference and was idle
 * for at least idle_timeout_s; *evicted (may be null) = models unloaded.  A
 * model is freed after the device has finished all queued work. */
tigas_status tigas_registry_evict_idle(tigas_registry* reg, int* evicted);

/* Self-test of the wave64 DPP prefix scan used by the scan and sort kernels:
 * inclusive scan of n u32 host values in groups of 64 lanes, result to host. */
tigas_status tigas_selftest_wave_scan(const uint32_t* in, uint32_t* out, int n);

#ifdef __cplusplus
}
#endif
#endif /* TIGAS_H */
