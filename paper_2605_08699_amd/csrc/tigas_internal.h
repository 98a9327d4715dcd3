// Internal structures shared by the HIP kernels and the host side of libtigas.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tigas {

constexpr int K1_THREADS = 256;       // one Gaussian per thread in preprocess / duplicate
constexpr int SORT_THREADS = 256;     // 4 wave64 per sort workgroup
constexpr int SORT_CHUNK = 2048;      // keys ranked per workgroup step (4 waves x 8 rounds x 64)
constexpr int SORT_MAX_BLOCKS = 4096; // workgroups per sort pass (at most)
// Chunked scans of per-block counts: one count per thread, so that many short
// workgroups (on many compute units) read in parallel the counts that the
// previous kernel's workgroups on every XCD just wrote.
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 1;
constexpr int SCAN_CHUNK = SCAN_THREADS * SCAN_ITEMS;  // counts per workgroup of the chunked scans
constexpr int MAX_SORT_PASSES = 8;
// Binned tile digit (single view): Gaussians per histogram block (eight
// rounds of 256), work per emission workgroup (entries, with each round of
// 256 Gaussians also counting BIN_ROUND_COST), groups of blocks for the
// prefix, cells of the (tiles_x + 1) x (tiles_y + 1) difference grid, tiles.
constexpr int BIN_BLOCK = 2048;
constexpr int BIN_PAIRS = 8192;
constexpr int BIN_ROUND_COST = 2048;  // fixed steps of a round, in entries
constexpr int BIN_GROUPS = 32;
constexpr int BIN_GRID_MAX = 8448;
constexpr int BIN_TILES_MAX = 8192;

// Resident scene (device pointers).  Layout by storage precision:
//   mean:  f32 planes [3][n] (x, y, z)
//   F32:   attr float4 [2][n]: (qw, qx, qy, qz), (ls0, ls1, ls2, logit)
//          sh   float4 [12][n]: 48 floats per Gaussian, coefficient-major (k*3 + ch)
//   F16/BF16: attr uint4 [n]: 8 halves (qw, qx, qy, qz, ls0, ls1, ls2, logit)
//          sh   uint4 [6][n]: 48 halves per Gaussian, coefficient-major
struct SceneView {
    int64_t n;
    int storage;  // 0 f32, 1 f16, 2 bf16
    int sh_degree;
    const float* mean;
    const void* attr;
    const void* sh;  // per Gaussian: sh_stride contiguous 16-byte words (4 floats or 8 halves)
    int sh_stride;
};

// Per-view camera and tiling parameters, computed on the host in FP64 and
// rounded once to FP32.
struct ViewParams {
    float V[9];        // world -> camera rotation R^T, row-major
    float cam[3];      // camera centre t
    float tz_key;      // float((-R^T t)_z): constant term of the FP32 depth key
    float fx, fy, cx, cy;
    float lim_x, lim_y;  // Jacobian clamp: 1.3 x the half-FoV tangents
    int width, height;
    int tile_w, tile_h, tiles_x, tiles_y;
    uint32_t tile_base;  // first global tile id of this view
    int sh_degree;
    int fmt;             // 0 RGB8, 1 RGBF32
    float bg[3];
    uint64_t out_ptr;    // device address of this view's frame
    SceneView scene;     // the scene this view renders
};

struct Counters {
    uint32_t D;         // duplicates (clamped to 2^32-1)
    uint32_t visible;
    uint32_t fallbacks;
    uint32_t overflow;  // D exceeded the duplicate capacity: nothing was emitted
    uint32_t fb_list;   // append cursor of the FP64-fallback list (cleared once counted)
    uint32_t fb_listed; // entries in the FP64-fallback list this frame
};

// Preprocess outputs, one slot per record (record = view-local index of a
// Gaussian, padded per view to a multiple of 256).
// One projected Gaussian (record), 64 bytes: all that the blend gathers for
// a list entry lies in one 64-byte segment.
struct alignas(64) Rec {
    float4 r0;   // u_hi, v_hi, u_lo, v_lo
    float4 r1;   // A, B, C, L: alpha = 2^(A dx^2 + B dx dy + C dy^2 + L)
    float4 r2;   // r, g, b, opacity
    uint2 bbox;  // inclusive pixel box: x0 | y0 << 16, x1 | y1 << 16
    uint2 pad;
};
static_assert(sizeof(Rec) == 64, "record is one 64-byte segment");

struct PreOut {
    Rec* rec;           // records (written only for Gaussians that touch a tile)
    uint2* rect;        // per record: tile rectangle tx0 | ty0 << 16, nx | ny << 16 (0 when no tile;
                        // a record is visible when nx ny > 0)
    uint2* srect;       // the visible records' tile rectangles in depth order (last depth pass)
    uint32_t* zkey;     // FP32 depth-key bits
    uint32_t* blk_sum;  // per 256-record block: tiles touched
    uint32_t* blk_vis;  // per block: records that touch a tile
    uint32_t* blk_fb;   // per block: FP64 fallbacks
    uint32_t* blk_view; // per block: view index
    uint32_t* chunk_vis;            // per SCAN_CHUNK block counts: visible records,
    unsigned long long* chunk_dup;  // duplicates,
    uint32_t* chunk_fb;             // FP64 fallbacks,
    uint32_t* chunk_dups;           // and (later) depth-ordered duplicate counts
    uint2* fb_list;     // (record, Gaussian) pairs whose conic is recomputed in FP64
    uint32_t fb_cap;
    Counters* cnt;
};

// Double-buffered (key, value, extra) words of a radix sort.
struct SortBuffers {
    uint32_t* key[2];
    uint32_t* val[2];
    uint32_t* ext[2];
    uint32_t* hist;    // [512][segments] digit counts per segment (then each digit's offsets)
    uint32_t* dtot;    // [512] per-digit totals
    uint32_t* zr;      // 2 words: smallest and largest visible depth key (three-pass depth sort)
    uint32_t* segmm;   // [segments][2]: each segment's smallest and largest key
};

// Arrays cleared (as u32 words) by the first kernel after preprocess.
struct ZeroList {
    static constexpr int N = 4;
    uint32_t* p[N];
    uint32_t n[N];
};

struct SortPass {
    int shift;
    int bits;   // <= 8, or 9 for the passes of the three-pass depth sort
    int adapt;  // -1: a fixed digit of the key; 0..2: pass of the three-pass depth sort
};

// ---- launchers (kernels.hip) ----
void launch_preprocess(const SceneView& s, const ViewParams* views_dev, const ViewParams* views_host, int nviews,
                       uint32_t rec_base, uint32_t n_pad, uint32_t view_base, const PreOut& o, hipStream_t st);
// One view's parameters stored to device memory by a kernel (argument by value).
void launch_store_view(const ViewParams& v, ViewParams* dst, hipStream_t st);
// p[0 .. n) = value, by a kernel (no memset node in captured sequences).
void launch_fill_u32(uint32_t* p, uint32_t n, uint32_t value, hipStream_t st);
void launch_scan_visible(const PreOut& o, int nblk, uint32_t* blk_off, Counters* cnt, uint32_t cap,
                         const ZeroList& zl, hipStream_t st);
// Visible records as (depth key, record) pairs; with ext, also each one's
// tile rectangle packed into one word (views of at most 256 x 256 tiles).
// The same launch recomputes, in FP64, the conic of every Gaussian
// preprocess listed as near-singular (before anything reads it).
void launch_compact(const PreOut& o, int nblk, const uint32_t* blk_off, uint32_t* key, uint32_t* val, uint32_t* ext,
                    const ViewParams* views_dev, hipStream_t st);
// The depth-ordered tile rectangles come packed (sorted_packed, carried by the
// depth passes) or, when that is null, as two words (sorted_rect).
void launch_duplicate(const PreOut& o, int nblk, const uint32_t* sorted_rec, const uint2* sorted_rect,
                      const uint32_t* sorted_packed,
                      uint32_t* blk_sum2, uint32_t* blk_off2, const Counters* cnt, uint32_t cap,
                      const ViewParams* views_dev, uint32_t* tile_out, uint32_t* val_out, uint32_t* depth_out,
                      hipStream_t st);
// Duplicates with tighter tile culling (packed rectangles only): per
// (Gaussian, tile of its rectangle), kept when the Gaussian can reach the
// skip threshold at one of the tile's pixels; the kept entries in emission
// order (blk_cnt, blk_off: per-256-Gaussian kept counts and their scan), and
// the kept count stored as the frame's D.
void launch_duplicate_culled(const PreOut& o, int nblk, const uint32_t* sorted_rec, const uint32_t* sorted_packed,
                             uint32_t* blk_cnt, uint32_t* blk_off, Counters* cnt, const ViewParams* views_dev,
                             int tile_w, int tile_h, uint32_t* tile_out, uint32_t* val_out, uint32_t* depth_out,
                             hipStream_t st);
// Runs LSD passes over the count selected by `which` (0 duplicates, 1 visible)
// starting in buffer `start`; returns the buffer index holding the result.
// With `rect_src`, the last pass also writes rect_src[value] to rect_dst in
// sorted order.
int launch_sort(const SortBuffers& b, const SortPass* passes, int npasses, int which, uint32_t cap, int nblocks,
                int start, bool extra, Counters* cnt, const uint2* rect_src,
                uint2* rect_dst, hipStream_t st);
// Tile ranges of the sorted list.  host_cnt: pinned host memory (or device
// memory) that receives a copy of the counters.
void launch_ranges(const uint32_t* tile_sorted, const Counters* cnt, uint32_t cap, uint2* ranges, Counters* host_cnt,
                   const PreOut& o, const ViewParams* views_dev, hipStream_t st);
// The blend's dense-first dispatch order of n_tiles tiles (longest lists
// first) from their ranges: order receives a permutation of 0 .. n_tiles-1.
void launch_tile_order(const uint2* ranges, uint32_t n_tiles, uint32_t* order, hipStream_t st);
// Tile placement by counting (single view, packed rectangles, a tile grid
// that fits BIN_GRID_MAX / BIN_TILES_MAX): from the depth-ordered records and
// packed rectangles, writes each (Gaussian, tile) entry's record id to its
// sorted position in val_out (with tile_out/depth_out, also its tile id and
// depth word), the tile ranges and the counters to host_cnt.  hist: ceil(nrec / BIN_BLOCK) x tiles words; gsum:
// (BIN_GROUPS + 2) x tiles words (group rows, tile totals, tile starts) and
// bin_emit_groups(cap, nrec) more (each emission workgroup's first round);
// round_cnt / round_off: nrec / 256 + 1 words; cap: the entry capacity.
// order (may be null): receives the blend's dense-first dispatch order.
bool bin_fits(int tiles_x, int tiles_y);
uint32_t bin_emit_groups(uint32_t cap, uint32_t nrec);
void launch_bin(const uint32_t* sorted_rec, const uint32_t* sorted_packed, const Counters* cnt, uint32_t nrec,
                uint32_t cap, int tiles_x, int tiles_y, uint32_t* hist, uint32_t* gsum, uint32_t* round_cnt,
                uint32_t* round_off, uint2* ranges, Counters* host_cnt, const PreOut& o, const ViewParams* views_dev,
                uint32_t* val_out, uint32_t* tile_out, uint32_t* depth_out, uint32_t* order, hipStream_t st);
// Baseline JPEG of an RGB8 frame: one workgroup per restart interval of
// JPEG_SEG_MCUS MCUs; the header is written by the host.
constexpr int JPEG_THREADS = 128;
constexpr int JPEG_SEG_MCUS = 40;  // 120 blocks: one thread each
struct JpegArgs {
    const uint8_t* rgb;  // H x W x 3, row-major
    int width, height, w8, h8;
    int64_t n_mcu;  // w8 h8
    int nseg;       // restart intervals
    float dct[64];        // M[k][n] = c(k)/2 cos((2n+1) k pi/16), FP32
    float rq_luma[64];    // 1/Q, row-major
    float rq_chroma[64];
    const uint32_t* huff;  // [4][256] length << 16 | code: DC luma, AC luma, DC chroma, AC chroma
    uint32_t* bits;        // [nseg][seg_words] entropy-coded bits of each interval (all zero between calls)
    uint32_t seg_words;
    uint32_t* seg_bits;  // [nseg] bits of each interval
    uint32_t* seg_len;   // [nseg] output bytes of each interval (stuffing and marker included)
    uint8_t* out;
    uint64_t capacity;
    uint64_t header_len;
    uint64_t* out_len;  // total length (written by the last interval)
};
void launch_jpeg(const JpegArgs& a, hipStream_t st);
void launch_blend(const ViewParams* views_dev, int nviews, uint32_t n_tiles, const uint2* ranges,
                  const uint32_t* vals, const PreOut& o, uint32_t nrec, int tile_w, int tile_h, int batch_depth,
                  int ppl, unsigned long long* work, uint32_t* queue, int persistent_blocks, bool cull,
                  const uint32_t* order, hipStream_t st);
// order (one workgroup per tile, without queue): the tiles' dispatch order,
// or null for the XCD-chunked order.
// With `queue` (8 counters cleared per frame) the blend runs as a persistent
// kernel of persistent_blocks workgroups pulling tiles from work queues.
// ppl: pixels per lane (1, or 2 for tiles at least 16 tall).  cull: drop,
// per wave, the entries whose exponent stays below the skip threshold on the
// wave's whole pixel block (they would be skipped at every pixel anyway).
int blend_persistent_occupancy(int tile_w, int tile_h, int batch_depth, int ppl);
void launch_wave_scan_selftest(const uint32_t* in, uint32_t* out, int n, hipStream_t st);

// Per-launch timing for profiling: while a timer is installed for the calling
// host thread, every kernel launch is bracketed by two events on its stream
// (never used for captured launches).
struct KernelTimer {
    virtual void before(const void* kernel, hipStream_t st) = 0;  // kernel: its host-side handle
    virtual void after(hipStream_t st) = 0;
    virtual ~KernelTimer() = default;
};
extern thread_local KernelTimer* g_kernel_timer;

// Sets the message tigas_last_error() returns on the calling thread.
void set_last_error(const char* msg);

}  // namespace tigas
