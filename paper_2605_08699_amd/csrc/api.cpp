// Host side of libtigas: the C ABI declared in include/tigas.h.
//
// Owns contexts (device, stream, workspaces), resident scenes and the launch
// sequence of a render.  Counts that depend on the data (visible Gaussians,
// duplicates D) stay on the device: kernels read them from device memory, so a
// render is a fixed sequence of launches with no host round trip inside it.
// The duplicate buffers are sized from the previous frame with headroom; if a
// frame needs more, its duplicate kernel emits nothing, the overflow flag is
// seen after the frame and the frame is rendered again with larger buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <condition_variable>
#include <deque>
#include <thread>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <cxxabi.h>
#include <stdexcept>
#include <string>
#include <system_error>
#include <vector>

#include "../../include/tigas.h"
#include "tigas_internal.h"

using namespace tigas;

thread_local KernelTimer* tigas::g_kernel_timer = nullptr;

namespace {

thread_local std::string g_err;

}  // namespace

void tigas::set_last_error(const char* msg) { g_err = msg ? msg : ""; }

namespace {

struct Error : std::runtime_error {
    tigas_status st;
    Error(tigas_status s, const std::string& m) : std::runtime_error(m), st(s) {}
};

[[noreturn]] void fail(tigas_status s, const std::string& m) { throw Error(s, m); }

void hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return;
    if (e == hipErrorOutOfMemory) fail(TIGAS_E_OOM, std::string(what) + ": out of device memory");
    fail(TIGAS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPCHK(x) hip_check((x), #x)

template <typename F>
tigas_status guard(F&& f) {
    try {
        g_err.clear();
        f();
        return TIGAS_OK;
    } catch (const Error& e) {
        g_err = e.what();
        return e.st;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return TIGAS_E_OOM;
    } catch (const std::exception& e) {
        g_err = e.what();
        return TIGAS_E_DEVICE;
    }
}

// Device buffer that grows (never shrinks) on demand.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    // returns true when the buffer was (re)allocated
    bool ensure(size_t need) {
        if (need <= bytes) return false;
        if (p) HIPCHK(hipFree(p));
        p = nullptr;
        bytes = 0;
        size_t want = std::max<size_t>(need, 256);
        HIPCHK(hipMalloc(&p, want));
        bytes = want;
        return true;
    }
    template <typename T>
    T* as() const {
        return reinterpret_cast<T*>(p);
    }
};

struct HostPinned {
    void* p = nullptr;
    size_t bytes = 0;
    ~HostPinned() {
        if (p) (void)hipHostFree(p);
    }
    // coherent: fine-grained, so device stores reach host memory directly
    void ensure(size_t need, bool coherent = false) {
        if (need <= bytes) return;
        if (p) HIPCHK(hipHostFree(p));
        p = nullptr;
        bytes = 0;
        HIPCHK(hipHostMalloc(&p, std::max<size_t>(need, 256), coherent ? hipHostMallocCoherent : hipHostMallocDefault));
        bytes = std::max<size_t>(need, 256);
    }
    template <typename T>
    T* as() const {
        return reinterpret_cast<T*>(p);
    }
};

uint32_t round_up(uint64_t x, uint64_t m) { return (uint32_t)((x + m - 1) / m * m); }

int ceil_log2(uint64_t x) {
    int b = 0;
    while ((1ull << b) < x) ++b;
    return b;
}

// ---------------------------------------------------------------- halves
uint16_t f32_to_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                           // nearest even
    return (uint16_t)(u >> 16);
}

uint16_t f32_to_f16(float f) {
    uint32_t x;
    std::memcpy(&x, &f, 4);
    const uint32_t sign = (x >> 16) & 0x8000u;
    uint32_t absx = x & 0x7fffffffu;
    if (absx >= 0x7f800000u) return (uint16_t)(sign | 0x7c00u | (absx > 0x7f800000u ? 0x200u : 0u));
    if (absx >= 0x477ff000u) return (uint16_t)(sign | 0x7c00u);  // rounds to infinity
    if (absx < 0x38800000u) {                                     // subnormal half or zero
        if (absx < 0x33000000u) return (uint16_t)sign;            // below half of the smallest subnormal
        const int e = (int)(absx >> 23);
        const uint32_t mant = (absx & 0x7fffffu) | 0x800000u;
        const int shift = 126 - e;  // so that the result counts units of 2^-24
        uint32_t q = mant >> (shift);
        const uint32_t rem = mant & ((1u << shift) - 1u);
        const uint32_t half = 1u << (shift - 1);
        if (rem > half || (rem == half && (q & 1u))) ++q;
        return (uint16_t)(sign | q);
    }
    uint32_t r = absx - 0x38000000u;  // rebias exponent 127 -> 15
    const uint32_t rem = r & 0x1fffu;
    uint32_t q = r >> 13;
    if (rem > 0x1000u || (rem == 0x1000u && (q & 1u))) ++q;
    return (uint16_t)(sign | q);
}

}  // namespace

static_assert(sizeof(tigas_frame_counters) == sizeof(Counters), "public counters mirror the device counters");
static_assert(offsetof(tigas_frame_counters, duplicates) == offsetof(Counters, D) &&
                  offsetof(tigas_frame_counters, visible) == offsetof(Counters, visible) &&
                  offsetof(tigas_frame_counters, fallbacks) == offsetof(Counters, fallbacks) &&
                  offsetof(tigas_frame_counters, overflow) == offsetof(Counters, overflow),
              "public counters mirror the device counters");

// Scratch array of the allocation-free render (see render_noalloc): one copy
// per device, held until the process ends.
static __device__ __align__(256) unsigned char scratch[TIGAS_NOALLOC_SCRATCH_BYTES];

// ------------------------------------------------------------- objects

namespace {

struct TileCfg {
    int tw, th, bd, ppl;  // tile width/height, staged entries per wave batch, pixels per lane
};

const TileCfg kTileCandidates[] = {{8, 8, 64, 1},    {8, 8, 128, 1},   {16, 16, 64, 1},  {16, 16, 128, 1},
                                   {16, 16, 64, 2},  {16, 16, 128, 2}, {16, 32, 64, 1},  {16, 32, 128, 1},
                                   {16, 32, 64, 2},  {16, 32, 128, 2}, {32, 16, 64, 1},  {32, 16, 128, 1},
                                   {32, 16, 64, 2}};

// A group of views of one scene inside a launch sequence.
struct Group {
    tigas_scene* scene;
    int first_view, nviews;
    uint32_t rec_base, n_pad;
};

struct Plan {
    std::vector<ViewParams> views;
    std::vector<Group> groups;
    uint32_t nrec = 0, n_tiles = 0;
    TileCfg tc{16, 16, 64, 1};
    bool persistent = false;  // blend as a persistent kernel over a tile work queue
    bool allow_graph = true;  // capture/replay (off for one-off shapes such as serving batches)
};

// Per-frame host-visible state.  A workspace has two: a frame can be prepared
// and launched while the previous one still runs on the stream, each slot's
// launch sequence reading its own view parameters and writing its own counters.
struct FrameSlot {
    DevBuf views;
    HostPinned host_views, host_counters;
    uint32_t view_cap = 0;
    hipEvent_t t0 = nullptr, t1 = nullptr;  // start / end of an asynchronous frame on the stream
    bool pending = false;                    // launched asynchronously and not yet finished
    int64_t ticket = -1;
    Plan plan;
    int cur = 0;
};

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    uint64_t gen = 0;
    int cur = 0;
};

}  // namespace

// Events around every launch of one frame (kernel profiling); the pool is
// reused frame after frame.
struct EventTimer final : KernelTimer {
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<std::pair<const void*, size_t>> recs;  // kernel handle, index of its start event
    hipEvent_t next() {
        if (used == pool.size()) {
            hipEvent_t e = nullptr;
            HIPCHK(hipEventCreate(&e));
            pool.push_back(e);
        }
        return pool[used++];
    }
    void before(const void* kernel, hipStream_t st) override {
        recs.emplace_back(kernel, used);
        HIPCHK(hipEventRecord(next(), st));
    }
    void after(hipStream_t st) override { HIPCHK(hipEventRecord(next(), st)); }
    void reset() {
        used = 0;
        recs.clear();
    }
    ~EventTimer() override {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

// Demangled name of a kernel from its host-side handle, as profilers print it.
std::string kernel_name(const void* kernel, hipStream_t st) {
    static std::mutex mu;
    static std::map<const void*, std::string> names;
    std::lock_guard<std::mutex> lk(mu);
    auto it = names.find(kernel);
    if (it != names.end()) return it->second;
    const char* m = hipKernelNameRefByPtr(kernel, st);
    std::string name = m ? m : "?";
    int status = 0;
    char* d = m ? abi::__cxa_demangle(m, nullptr, nullptr, &status) : nullptr;
    if (d && status == 0) name = d;
    std::free(d);
    names[kernel] = name;
    return name;
}

// Installs a timer for the calling thread's launches for one scope.
struct TimerScope {
    KernelTimer* prev;
    explicit TimerScope(KernelTimer* t) : prev(g_kernel_timer) { g_kernel_timer = t; }
    ~TimerScope() { g_kernel_timer = prev; }
};

// Device memory of one launch sequence as plain pointers (a workspace's
// buffers, or any other memory laid out the same way).
struct FrameMem {
    hipStream_t stream = nullptr;
    ViewParams* views = nullptr;      // device view parameters of the plan
    const void* views_src = nullptr;  // pinned host copy read by a copy (graphs re-read it on replay);
                                      // null: a single view uploaded as a kernel argument
    PreOut pre{};
    Counters* cnt = nullptr;
    Counters* cnt_out = nullptr;  // receives the final counters (pinned host memory or device memory)
    uint32_t* key[2] = {nullptr, nullptr};
    uint32_t* val[2] = {nullptr, nullptr};
    uint32_t* ext[2] = {nullptr, nullptr};
    uint32_t* hist = nullptr;      // digit counts per sort segment
    uint32_t* hist_tot = nullptr;  // per-digit totals
    uint32_t* zr = nullptr;        // three-pass depth sort: key range and per-segment ranges
    uint32_t* segmm = nullptr;     //   (null: the four-pass depth sort only)
    uint32_t* queue = nullptr;
    uint2* ranges = nullptr;
    uint32_t* order = nullptr;     // the blend's dispatch order of the tiles
    uint32_t* bin_hist = nullptr;  // binned tile digit: block histograms, group starts
    uint32_t* bin_gsum = nullptr;
    uint32_t* blk_off = nullptr;
    uint32_t* blk_sum2 = nullptr;
    uint32_t* blk_off2 = nullptr;
    uint32_t dup_cap = 0;
    hipEvent_t* ev = nullptr;  // 7 stage-boundary events (stage timing only)
    uint32_t* dbg_key = nullptr;
    uint32_t* dbg_val = nullptr;
    uint32_t* dbg_ext = nullptr;
};

struct Workspace {
    hipStream_t stream = nullptr;
    std::mutex mu;  // one launch sequence at a time per workspace
    // per record
    DevBuf recs, rect, srect, zkey;
    DevBuf blk_sum, blk_vis, blk_fb, blk_view, blk_off, blk_sum2, blk_off2;
    DevBuf fb_list;  // near-singular Gaussians for the FP64 conic kernel
    DevBuf chunk_vis, chunk_dup, chunk_fb, chunk_dups;  // totals per chunk of block counts
    DevBuf counters;
    // per duplicate (also holds the visible Gaussians during the depth passes)
    DevBuf key[2], val[2], ext[2];
    DevBuf hist, queue, sortrange;
    // emission-order copies for the inspection entry point
    DevBuf dbg_key, dbg_val, dbg_ext;
    // per tile / per view
    DevBuf ranges;
    DevBuf bin_hist, bin_gsum;
    DevBuf frame_staging;
    static constexpr int NSLOT = 2;
    FrameSlot slot[NSLOT];
    int active = 0;      // slot used by the launch being prepared
    int next_async = 0;  // slot for the next asynchronous frame
    FrameSlot& fs() { return slot[active]; }
    DevBuf work;            // blend work counters (evaluations, contributions)
    // JPEG encoder: per-interval bit buffers (all zero between calls),
    // per-interval bit counts and output lengths, code tables, length
    DevBuf jpeg_bits, jpeg_seg_bits, jpeg_seg_len, jpeg_huff, jpeg_len;
    HostPinned jpeg_len_host;
    hipEvent_t ev[7] = {};  // stage boundaries when stage timing is on
    EventTimer ktimer;      // per-launch events when kernel timing is on
    uint32_t rec_cap = 0, dup_cap = 0, tile_cap = 0;
    uint32_t last_D = 0;
    uint64_t gen = 1;  // bumped whenever a buffer is reallocated (captured graphs hold its pointers)
    std::map<std::string, GraphEntry> graphs;

    FrameMem mem() {
        FrameMem m;
        m.stream = stream;
        m.views = fs().views.as<ViewParams>();
        m.views_src = fs().host_views.p;
        m.pre = pre();
        m.cnt = counters.as<Counters>();
        m.cnt_out = fs().host_counters.as<Counters>();
        for (int i = 0; i < 2; ++i) {
            m.key[i] = key[i].as<uint32_t>();
            m.val[i] = val[i].as<uint32_t>();
            m.ext[i] = ext[i].as<uint32_t>();
        }
        m.hist = hist.as<uint32_t>();
        m.hist_tot = m.hist + (size_t)512 * SORT_MAX_BLOCKS;
        m.zr = sortrange.as<uint32_t>();
        m.segmm = m.zr + 2;
        m.queue = queue.as<uint32_t>();
        m.ranges = ranges.as<uint2>();
        m.order = reinterpret_cast<uint32_t*>(m.ranges + tile_cap);  // after the ranges, in the same buffer
        m.bin_hist = bin_hist.as<uint32_t>();
        m.bin_gsum = bin_gsum.as<uint32_t>();
        m.blk_off = blk_off.as<uint32_t>();
        m.blk_sum2 = blk_sum2.as<uint32_t>();
        m.blk_off2 = blk_off2.as<uint32_t>();
        m.dup_cap = dup_cap;
        m.ev = ev[0] ? ev : nullptr;
        m.dbg_key = dbg_key.as<uint32_t>();
        m.dbg_val = dbg_val.as<uint32_t>();
        m.dbg_ext = dbg_ext.as<uint32_t>();
        return m;
    }
    PreOut pre() const {
        PreOut o;
        o.rec = recs.as<Rec>();
        o.rect = rect.as<uint2>();
        o.srect = srect.as<uint2>();
        o.zkey = zkey.as<uint32_t>();
        o.blk_sum = blk_sum.as<uint32_t>();
        o.blk_vis = blk_vis.as<uint32_t>();
        o.blk_fb = blk_fb.as<uint32_t>();
        o.blk_view = blk_view.as<uint32_t>();
        o.fb_list = fb_list.as<uint2>();
        o.chunk_vis = chunk_vis.as<uint32_t>();
        o.chunk_dup = chunk_dup.as<unsigned long long>();
        o.chunk_fb = chunk_fb.as<uint32_t>();
        o.chunk_dups = chunk_dups.as<uint32_t>();
        o.fb_cap = rec_cap;
        o.cnt = counters.as<Counters>();
        return o;
    }
    void grow(DevBuf& b, size_t bytes) {
        if (b.ensure(bytes)) ++gen;
    }
    void ensure_records(uint32_t nrec) {
        if (nrec <= rec_cap && recs.p) return;
        const size_t r = std::max<uint32_t>(nrec, 256);
        grow(recs, r * sizeof(Rec));
        grow(rect, r * 8);
        grow(srect, r * 8);
        grow(zkey, r * 4);
        const size_t nb = r / K1_THREADS + 1;
        for (DevBuf* b : {&blk_sum, &blk_vis, &blk_fb, &blk_view, &blk_off, &blk_sum2, &blk_off2}) grow(*b, nb * 4);
        grow(fb_list, r * 8);
        const size_t nch = nb / SCAN_CHUNK + 2;
        for (DevBuf* b : {&chunk_vis, &chunk_fb, &chunk_dups}) grow(*b, nch * 4);
        grow(chunk_dup, nch * 8);
        rec_cap = (uint32_t)r;
    }
    void ensure_dups(uint32_t cap) {
        if (cap <= dup_cap && key[0].p) return;
        cap = std::max<uint32_t>(std::max(cap, dup_cap), 1u << 16);
        for (int i = 0; i < 2; ++i) {
            grow(key[i], (size_t)cap * 4);
            grow(val[i], (size_t)cap * 4);
            grow(ext[i], (size_t)cap * 4);
        }
        grow(hist, ((size_t)512 * SORT_MAX_BLOCKS + 512) * 4);  // counts per (digit, segment), then digit totals
        grow(sortrange, (size_t)(2 + 2 * SORT_MAX_BLOCKS) * 4);
        grow(queue, 8 * 4);                                  // blend band queues
        dup_cap = cap;
    }
    void ensure_tiles(uint32_t n) {
        if (n <= tile_cap && ranges.p) return;
        grow(ranges, (size_t)std::max<uint32_t>(n, 1) * 12);  // ranges, then the dispatch order
        tile_cap = std::max<uint32_t>(n, 1);
    }
    void ensure_views(int n) {
        FrameSlot& f = fs();
        if ((uint32_t)n <= f.view_cap && f.views.p) return;
        grow(f.views, sizeof(ViewParams) * (size_t)n);
        if (f.host_views.bytes < sizeof(ViewParams) * (size_t)n) {
            f.host_views.ensure(sizeof(ViewParams) * (size_t)n);
            ++gen;
        }
        f.view_cap = (uint32_t)n;
    }
    void ensure_events() {
        if (ev[0]) return;
        for (auto& e : ev) HIPCHK(hipEventCreate(&e));
        ++gen;
    }
    void drop_graphs() {
        for (auto& kv : graphs)
            if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        graphs.clear();
    }
    ~Workspace() {
        for (FrameSlot& f : slot)
            for (hipEvent_t e : {f.t0, f.t1})
                if (e) (void)hipEventDestroy(e);
        drop_graphs();
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

struct tigas_context {
    int device = 0;
    int cus = 256;
    hipStream_t stream = nullptr;
    std::mutex mu;
    std::map<hipStream_t, std::unique_ptr<Workspace>> ws;
    tigas_stats last{};
    std::mutex stats_mu;
    std::atomic<bool> profile{false};
    std::atomic<bool> profile_kernels{false};
    std::map<std::string, std::pair<int64_t, double>> kernel_ms;  // name -> (launches, total ms)
    std::atomic<bool> use_graphs{true};
    std::atomic<bool> blend_cull{true};     // blend: per-block threshold culling
    std::atomic<bool> tile_bin{true};       // single view: tile digit placed by counting
    std::atomic<bool> tile_cull{false};     // duplicates only for tiles each Gaussian can reach
    std::atomic<bool> depth4{false};        // four-pass depth sort (requested, or after a frame too deep for three)
    double stage_ms[6] = {0, 0, 0, 0, 0, 0};
    int64_t stage_frames = 0;
    std::mutex tune_mu;
    std::map<std::string, TileCfg> tuned;  // shape -> best tile / batch depth
    std::string tune_file;
    // asynchronous frames: ticket -> (workspace, slot) while in flight, then its outcome
    struct AsyncDone {
        tigas_status status = TIGAS_OK;
        std::string error;
        tigas_stats stats{};
        float gpu_ms = 0.f;
    };
    std::mutex async_mu;
    std::map<int64_t, std::pair<Workspace*, int>> async_pending;
    std::map<int64_t, AsyncDone> async_done;
    int64_t ticket_seq = 0;

    Workspace& workspace(hipStream_t s) {
        std::lock_guard<std::mutex> lk(mu);
        auto& p = ws[s];
        if (!p) {
            p.reset(new Workspace());
            p->stream = s;
            for (FrameSlot& f : p->slot) f.host_counters.ensure(sizeof(Counters), /*coherent=*/true);
            if (p->counters.ensure(sizeof(Counters))) HIPCHK(hipMemset(p->counters.p, 0, sizeof(Counters)));
        }
        return *p;
    }
};

struct tigas_scene {
    tigas_context* ctx = nullptr;
    uint64_t uid = 0;  // unique over the process: a captured graph holds this scene's device pointers
    SceneView view{};
    DevBuf mean, attr, sh;
    size_t bytes = 0;
    std::atomic<int> refs{0};
};

namespace {

struct SceneRef {  // keeps a scene referenced while a render uses it
    tigas_scene* s;
    explicit SceneRef(tigas_scene* s_) : s(s_) { s->refs.fetch_add(1); }
    ~SceneRef() { s->refs.fetch_sub(1); }
};

bool finite3(const float* p, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// fn(i0, i1) over [0, n) split among up to 16 host threads (one thread for
// small n or when no thread can be started).
template <typename F>
void parallel_for(int64_t n, F&& fn) {
    const int64_t hw = std::max<int64_t>(1, (int64_t)std::thread::hardware_concurrency());
    const int64_t nt = std::min<int64_t>({16, hw, (n + 65535) / 65536});
    if (nt <= 1) {
        if (n > 0) fn((int64_t)0, n);
        return;
    }
    const int64_t per = (n + nt - 1) / nt;
    std::vector<std::thread> pool;
    pool.reserve((size_t)nt);
    int64_t started = 0;
    try {
        for (int64_t t = 0; t < nt; ++t) {
            const int64_t i0 = t * per, i1 = std::min(n, i0 + per);
            if (i0 < i1) pool.emplace_back([&fn, i0, i1] { fn(i0, i1); });
            started = i1;
        }
    } catch (const std::system_error&) {
    }
    if (started < n) fn(started, n);
    for (std::thread& th : pool) th.join();
}

// Tile configuration requested by q: {0, 0} asks for the autotuner.
bool tile_requested(const tigas_quality* q) { return q && (q->tile_w != 0 || q->tile_h != 0); }

TileCfg tile_cfg(const tigas_quality* q) {
    int tw = q ? q->tile_w : 0, th = q ? q->tile_h : 0, bd = q ? q->batch_depth : 0;
    if (tw == 0 && th == 0) {
        tw = 16;
        th = 16;
    }
    const bool okt = (tw == 8 && th == 8) || (tw == 16 && th == 16) || (tw == 16 && th == 32) || (tw == 32 && th == 16);
    if (!okt) fail(TIGAS_E_INVALID, "tile must be 8x8, 16x16, 16x32 or 32x16");
    if (bd == 0) bd = 64;
    if (bd != 64 && bd != 128 && bd != 256) fail(TIGAS_E_INVALID, "batch_depth must be 64, 128 or 256");
    int ppl = q ? q->pixels_per_lane : 0;
    if (ppl == 0) ppl = 1;
    if (ppl != 1 && ppl != 2) fail(TIGAS_E_INVALID, "pixels_per_lane must be 1 or 2");
    if (th < 16) ppl = 1;
    return {tw, th, bd, ppl};
}

// Camera of one view: V = R^T, the FP32 key constant, rung-scaled intrinsics
// (computed in FP64, rounded once to FP32) and the Jacobian clamp.
ViewParams make_view(const tigas_scene* sc, const tigas_pose* pose, const tigas_intrinsics* intr, int width,
                     int height, const tigas_quality* q) {
    if (!pose || !intr) fail(TIGAS_E_INVALID, "pose and intrinsics are required");
    if (!finite3(pose->R, 9) || !finite3(pose->t, 3)) fail(TIGAS_E_INVALID, "pose is not finite");
    if (!(intr->fx > 0.f) || !(intr->fy > 0.f) || !std::isfinite(intr->fx) || !std::isfinite(intr->fy) ||
        !std::isfinite(intr->cx) || !std::isfinite(intr->cy))
        fail(TIGAS_E_INVALID, "intrinsics must be finite with fx, fy > 0");
    if (width < 1 || height < 1 || width > 16384 || height > 16384)
        fail(TIGAS_E_INVALID, "width and height must be in 1..16384");
    const float s = (q && q->res_scale != 0.f) ? q->res_scale : 1.0f;
    if (!(s > 0.f && s <= 1.f)) fail(TIGAS_E_INVALID, "res_scale must be in (0, 1]");
    const int ow = (int)std::floor((double)width * (double)s + 0.5);
    const int oh = (int)std::floor((double)height * (double)s + 0.5);
    if (ow < 1 || oh < 1) fail(TIGAS_E_INVALID, "res_scale gives an empty frame");
    ViewParams v{};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) v.V[i * 3 + j] = pose->R[j * 3 + i];
    for (int i = 0; i < 3; ++i) v.cam[i] = pose->t[i];
    const double tz = -((double)v.V[6] * pose->t[0] + (double)v.V[7] * pose->t[1] + (double)v.V[8] * pose->t[2]);
    v.tz_key = (float)tz;
    const double rx = (double)ow / width, ry = (double)oh / height;
    v.fx = (float)((double)intr->fx * rx);
    v.fy = (float)((double)intr->fy * ry);
    v.cx = (float)((double)intr->cx * rx);
    v.cy = (float)((double)intr->cy * ry);
    v.lim_x = (float)(1.3 * std::max((double)v.cx, (double)ow - v.cx) / v.fx);
    v.lim_y = (float)(1.3 * std::max((double)v.cy, (double)oh - v.cy) / v.fy);
    v.width = ow;
    v.height = oh;
    int deg = q ? q->sh_degree : -1;
    if (deg > sc->view.sh_degree) fail(TIGAS_E_INVALID, "sh_degree above the scene's degree");
    if (deg < 0) deg = sc->view.sh_degree;
    v.sh_degree = deg;
    v.fmt = q ? (int)q->fmt : 0;
    if (v.fmt != 0 && v.fmt != 1) fail(TIGAS_E_INVALID, "unknown frame format");
    for (int i = 0; i < 3; ++i) v.bg[i] = q ? q->bg[i] : 0.f;
    if (!finite3(v.bg, 3)) fail(TIGAS_E_INVALID, "background is not finite");
    v.scene = sc->view;
    return v;
}

size_t frame_bytes(const ViewParams& v) { return (size_t)v.width * v.height * 3 * (v.fmt == 1 ? 4 : 1); }

// Depth digits of the (tile | depth) key: positive FP32 bit patterns, bit 31 clear.
const SortPass kDepthPasses[4] = {{0, 8, -1}, {8, 8, -1}, {16, 8, -1}, {24, 7, -1}};
// Three passes of 9-bit digits of the key less the frame's smallest key, for
// frames whose visible keys span less than 2^27 (depths within about 16
// octaves); a wider frame is flagged by the first pass's scan, skipped by the
// later passes and rendered again with kDepthPasses.
const SortPass kDepthPasses3[3] = {{0, 9, 0}, {9, 9, 1}, {18, 9, 2}};

// The fewest passes of at most 8 bits, with the bits spread evenly over them
// (e.g. 12 bits as 6 + 6): fewer digits per pass give longer runs of equal
// digits per chunk, so the scatter writes whole cache lines more often.
std::vector<SortPass> tile_passes(uint32_t n_tiles) {
    std::vector<SortPass> p;
    const int tb = ceil_log2(n_tiles);
    const int np = (tb + 7) / 8;
    int sh = 0;
    for (int i = 0; i < np; ++i) {
        const int b = (tb - sh + (np - i) - 1) / (np - i);
        p.push_back({sh, b, -1});
        sh += b;
    }
    return p;
}

// Workgroups of a sort pass: one per 4096 keys, at most 1024 up to 16M keys
// (more only lengthen the scans there) and up to SORT_MAX_BLOCKS beyond, so
// that a batch's hundred million duplicates do not queue 60 chunks per
// workgroup.
int sort_blocks(uint64_t n) {
    const uint64_t cap = n <= (16ull << 20) ? 1024 : SORT_MAX_BLOCKS;
    return (int)std::min<uint64_t>(cap, std::max<uint64_t>(1, n / 4096));
}

// Tile layout of a plan for a tile configuration (tile ids are global:
// view tile offset + row-major local id).
void set_tiles(Plan& plan, const TileCfg& tc) {
    plan.tc = tc;
    plan.n_tiles = 0;
    for (ViewParams& v : plan.views) {
        v.tile_w = tc.tw;
        v.tile_h = tc.th;
        v.tiles_x = (v.width + tc.tw - 1) / tc.tw;
        v.tiles_y = (v.height + tc.th - 1) / tc.th;
        v.tile_base = plan.n_tiles;
        plan.n_tiles += (uint32_t)(v.tiles_x * v.tiles_y);
    }
}

// Everything about a plan that a captured graph depends on, except the view
// parameters themselves (copied from pinned memory by the graph each replay).
// Key of a plan's shape.  with_tiles (a captured graph's key): also the
// tile configuration and the identity of each scene, whose device pointers
// the graph holds (a scene loaded after another was freed may reuse its host
// address, never its uid).  Without: only sizes (the autotuner's key).
std::string shape_key(const Plan& plan, bool with_tiles) {
    std::string k;
    char buf[160];
    for (const Group& g : plan.groups) {
        std::snprintf(buf, sizeof buf, "g%llu:%lld:%d:%d:%d:%d:%u:%u;",
                      with_tiles ? (unsigned long long)g.scene->uid : 0ull, (long long)g.scene->view.n,
                      g.scene->view.storage, g.scene->view.sh_degree, g.first_view, g.nviews, g.rec_base, g.n_pad);
        k += buf;
    }
    for (const ViewParams& v : plan.views) {
        std::snprintf(buf, sizeof buf, "v%dx%d:%d;", v.width, v.height, v.sh_degree);
        k += buf;
    }
    if (with_tiles) {
        std::snprintf(buf, sizeof buf, "t%dx%d:%d:%d:%d", plan.tc.tw, plan.tc.th, plan.tc.bd, plan.tc.ppl,
                      (int)plan.persistent);
        k += buf;
    }
    return k;
}

// Buffers of the binned tile digit for a single-view plan (they depend on the
// duplicate capacity too: call again after it grows).
void ensure_bin(Workspace& ws, const Plan& plan) {
    if (plan.views.size() != 1 || !bin_fits(plan.views[0].tiles_x, plan.views[0].tiles_y)) return;
    const size_t nbc = std::max<size_t>(1, (plan.nrec + BIN_BLOCK - 1) / BIN_BLOCK);
    ws.grow(ws.bin_hist, nbc * plan.n_tiles * 4);
    ws.grow(ws.bin_gsum, ((size_t)(BIN_GROUPS + 2) * plan.n_tiles + BIN_TILES_MAX / 256 + nbc +
                          bin_emit_groups(ws.dup_cap, plan.nrec)) * 4);
}

void prepare(Workspace& ws, const Plan& plan, bool debug) {
    if (ws.counters.ensure(sizeof(Counters))) {
        // the FP64-list count is cleared by each frame after use; start at zero
        HIPCHK(hipMemset(ws.counters.p, 0, sizeof(Counters)));
        ++ws.gen;
    }
    ws.ensure_views((int)plan.views.size());
    ws.ensure_records(plan.nrec);
    ws.ensure_tiles(plan.n_tiles);
    // never below 4x the record count: the depth passes keep the visible
    // Gaussians in the same buffers
    uint64_t est = std::max<uint64_t>((uint64_t)ws.last_D + ws.last_D / 4, (uint64_t)plan.nrec * 4);
    est = std::max<uint64_t>(est, 1u << 20);
    ws.ensure_dups((uint32_t)std::min<uint64_t>(est, 0xfff00000ull));
    ensure_bin(ws, plan);
    if (debug) {
        const size_t bytes = (size_t)ws.dup_cap * 4;
        ws.dbg_key.ensure(bytes);
        ws.dbg_val.ensure(bytes);
        ws.dbg_ext.ensure(bytes);
    }
}

// Enqueue the whole launch sequence of a plan on ws.stream (no allocation, no
// host synchronisation: capturable).  Returns the index of the sort buffer
// that holds the sorted lists.
//   preprocess -> scan visible -> compact -> depth passes (visible Gaussians)
//   -> duplicate in depth order -> tile passes (duplicates) -> ranges -> blend
// Per-context switches that change the launch sequence (not its results).
struct LaunchOptions {
    bool cull = true;         // blend: per-block threshold culling of list entries
    bool bin = true;          // single view: tile digit placed by counting (else radix passes over the duplicates)
    bool cull_tiles = false;  // duplicates only for tiles the Gaussian can reach (radix passes then)
    bool depth3 = true;       // three-pass depth sort (when the rectangles pack and the buffers are there)
};

// Whether every view's tile rectangles fit the packed one-word form.
bool packed_rects(const Plan& plan) {
    bool packed = true;
    for (const ViewParams& v : plan.views) packed = packed && v.tiles_x <= 256 && v.tiles_y <= 256;
    return packed;
}

// Whether the plan's tile digit is placed by counting.
bool use_bin(const Plan& plan, const LaunchOptions& opt) {
    return opt.bin && !(opt.cull_tiles && packed_rects(plan)) && plan.views.size() == 1 &&
           plan.views[0].tiles_x <= 256 && plan.views[0].tiles_y <= 256 &&
           bin_fits(plan.views[0].tiles_x, plan.views[0].tiles_y);
}

int enqueue(const FrameMem& m, const Plan& plan, bool debug, bool prof, unsigned long long* work, int pblocks,
            const LaunchOptions& opt) {
    hipStream_t st = m.stream;
    auto mark = [&](int i) {
        if (prof) HIPCHK(hipEventRecord(m.ev[i], st));
    };
    const int nv = (int)plan.views.size();
    if (m.views_src) {
        HIPCHK(hipMemcpyAsync(m.views, m.views_src, sizeof(ViewParams) * nv, hipMemcpyHostToDevice, st));
    } else {
        if (nv != 1) fail(TIGAS_E_INVALID, "kernel-argument view upload takes one view");
        launch_store_view(plan.views[0], m.views, st);
    }
    const PreOut& o = m.pre;
    const ViewParams* vdev = m.views;
    mark(0);
    for (const Group& g : plan.groups) {
        if (g.n_pad == 0) continue;
        launch_preprocess(g.scene->view, vdev + g.first_view, plan.views.data() + g.first_view, g.nviews,
                          g.rec_base, g.n_pad, (uint32_t)g.first_view, o, st);
    }
    mark(1);
    const int nblk = (int)(plan.nrec / K1_THREADS);
    Counters* cnt = m.cnt;
    ZeroList zl{};
    zl.p[0] = m.queue;
    zl.n[0] = 8;
    zl.p[1] = reinterpret_cast<uint32_t*>(m.ranges);
    zl.n[1] = 2 * plan.n_tiles;
    launch_scan_visible(o, nblk, m.blk_off, cnt, m.dup_cap, zl, st);
    mark(2);
    SortBuffers sb;
    for (int i = 0; i < 2; ++i) {
        sb.key[i] = m.key[i];
        sb.val[i] = m.val[i];
        sb.ext[i] = m.ext[i];
    }
    sb.hist = m.hist;
    sb.dtot = m.hist_tot;
    sb.zr = m.zr;
    sb.segmm = m.segmm;
    // depth digits, on the visible Gaussians (record order in, depth order
    // out); the tile rectangles travel packed with them when every view has
    // at most 256 x 256 tiles, else the last pass gathers them.  Three 9-bit
    // passes when the rectangles pack (a frame whose keys turn out to span
    // too much is flagged and redone with four), else four 8-bit passes.
    const bool packed = packed_rects(plan);
    const bool depth3 = opt.depth3 && packed && m.zr;
    launch_compact(o, nblk, m.blk_off, sb.key[0], sb.val[0], packed ? sb.ext[0] : nullptr, vdev, st);
    const int cv = launch_sort(sb, depth3 ? kDepthPasses3 : kDepthPasses, depth3 ? 3 : 4, /*which=*/1, m.dup_cap,
                               sort_blocks(plan.nrec), 0, packed, cnt, packed ? nullptr : o.rect,
                               packed ? nullptr : o.srect, st);
    const int cd = cv ^ 1;
    const bool bin = use_bin(plan, opt);
    if (!bin && opt.cull_tiles && packed) {
        // duplicates in depth order, only for the tiles each Gaussian can reach
        launch_duplicate_culled(o, nblk, sb.val[cv], sb.ext[cv], m.blk_sum2, m.blk_off2, cnt, vdev, plan.tc.tw,
                                plan.tc.th, sb.key[cd], sb.val[cd], debug ? sb.ext[cd] : nullptr, st);
    } else if (!bin || debug) {
        // duplicates in depth order (kept for inspection only when binning)
        launch_duplicate(o, nblk, sb.val[cv], o.srect, packed ? sb.ext[cv] : nullptr, m.blk_sum2, m.blk_off2, cnt,
                         m.dup_cap, vdev, sb.key[cd], sb.val[cd], debug ? sb.ext[cd] : nullptr, st);
    }
    mark(3);
    if (debug) {
        const size_t bytes = (size_t)m.dup_cap * 4;
        HIPCHK(hipMemcpyAsync(m.dbg_key, sb.key[cd], bytes, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(m.dbg_val, sb.val[cd], bytes, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(m.dbg_ext, sb.ext[cd], bytes, hipMemcpyDeviceToDevice, st));
    }
    int cur = cd;
    if (bin) {
        // tile digit by counting, straight from the depth-ordered Gaussians
        const ViewParams& v = plan.views[0];
        launch_bin(sb.val[cv], sb.ext[cv], cnt, plan.nrec, m.dup_cap, v.tiles_x, v.tiles_y, m.bin_hist, m.bin_gsum,
                   m.blk_sum2, m.blk_off2, m.ranges, m.cnt_out, o, vdev, sb.val[cd], debug ? sb.key[cd] : nullptr,
                   debug ? sb.ext[cd] : nullptr, m.order, st);
        mark(4);
        mark(5);
    } else {
        // tile digits, on the duplicates
        const std::vector<SortPass> tp = tile_passes(plan.n_tiles);
        cur = launch_sort(sb, tp.data(), (int)tp.size(), /*which=*/0, m.dup_cap, sort_blocks(m.dup_cap), cd, debug,
                          cnt, nullptr, nullptr, st);
        mark(4);
        launch_ranges(sb.key[cur], cnt, m.dup_cap, m.ranges, m.cnt_out, o, vdev, st);
        if (!plan.persistent) launch_tile_order(m.ranges, plan.n_tiles, m.order, st);
        mark(5);
    }
    launch_blend(vdev, nv, plan.n_tiles, m.ranges, sb.val[cur], o, plan.nrec, plan.tc.tw, plan.tc.th, plan.tc.bd,
                 plan.tc.ppl, work, plan.persistent ? m.queue : nullptr, pblocks, opt.cull,
                 plan.persistent ? nullptr : m.order, st);
    mark(6);
    HIPCHK(hipGetLastError());
    return cur;
}

bool plan_binned(tigas_context* ctx, const Plan& plan) {
    LaunchOptions opt;
    opt.bin = ctx->tile_bin.load();
    opt.cull_tiles = ctx->tile_cull.load();
    return use_bin(plan, opt);
}

// Depth passes of the context's frames of this plan (after a frame settled).
int depth_passes(tigas_context* ctx, const Plan& plan) {
    return !ctx->depth4.load() && packed_rects(plan) ? 3 : 4;
}

// Launch the plan once: from a captured graph when allowed (captured on the
// first use of its shape, re-captured after any workspace reallocation), else
// eagerly.  Returns the sort buffer index.
int launch_plan(tigas_context* ctx, Workspace& ws, const Plan& plan, bool debug, bool prof,
                unsigned long long* work) {
    std::memcpy(ws.fs().host_views.p, plan.views.data(), sizeof(ViewParams) * plan.views.size());
    if (prof) ws.ensure_events();
    const int pblocks =
        plan.persistent ? ctx->cus * blend_persistent_occupancy(plan.tc.tw, plan.tc.th, plan.tc.bd, plan.tc.ppl) : 0;
    // stage timing needs events between the launches: that runs uncaptured
    LaunchOptions opt;
    opt.cull = ctx->blend_cull.load();
    opt.bin = ctx->tile_bin.load();
    opt.cull_tiles = ctx->tile_cull.load();
    opt.depth3 = !ctx->depth4.load();
    const bool kprof = ctx->profile_kernels.load();
    const bool graph = ctx->use_graphs.load() && plan.allow_graph && !debug && !work && !prof && !kprof;
    if (kprof) {
        ws.ktimer.reset();
        TimerScope ts(&ws.ktimer);
        return enqueue(ws.mem(), plan, debug, prof, work, pblocks, opt);
    }
    if (!graph) return enqueue(ws.mem(), plan, debug, prof, work, pblocks, opt);
    const std::string key = shape_key(plan, true) + (opt.cull ? "c1" : "c0") + (opt.bin ? "b1" : "b0") + (opt.cull_tiles ? "t1" : "t0") +
                            (opt.depth3 ? "d3" : "d4") + (ws.active ? "f1" : "f0");
    GraphEntry& g = ws.graphs[key];
    if (!g.exec || g.gen != ws.gen) {
        if (g.exec) HIPCHK(hipGraphExecDestroy(g.exec));
        g.exec = nullptr;
        if (ws.graphs.size() > 64) {  // bound the cache
            ws.drop_graphs();
            return launch_plan(ctx, ws, plan, debug, prof, work);
        }
        hipGraph_t graph_t = nullptr;
        HIPCHK(hipStreamBeginCapture(ws.stream, hipStreamCaptureModeThreadLocal));
        int cur = 0;
        try {
            cur = enqueue(ws.mem(), plan, debug, prof, work, pblocks, opt);
        } catch (...) {
            (void)hipStreamEndCapture(ws.stream, &graph_t);
            if (graph_t) (void)hipGraphDestroy(graph_t);
            throw;
        }
        HIPCHK(hipStreamEndCapture(ws.stream, &graph_t));
        const hipError_t e = hipGraphInstantiate(&g.exec, graph_t, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph_t);
        HIPCHK(e);
        g.gen = ws.gen;
        g.cur = cur;
    }
    HIPCHK(hipGraphLaunch(g.exec, ws.stream));
    return g.cur;
}

// Waits for the stream: polls for up to ~2 ms (a frame's completion is then
// seen within a microsecond or two instead of after a blocking wake-up), then
// blocks.
void wait_stream(hipStream_t st) {
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const hipError_t e = hipStreamQuery(st);
        if (e == hipSuccess) return;
        if (e != hipErrorNotReady) HIPCHK(e);
        if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(2000)) break;
    }
    HIPCHK(hipStreamSynchronize(st));
}

// After a launch of `plan` from the active slot has completed: a frame whose
// duplicates overflowed the buffers (it then emitted nothing) is rendered
// again (synchronously) with larger buffers; returns the counters of the
// final attempt.
Counters settle_frame(tigas_context* ctx, Workspace& ws, const Plan& plan, bool debug, bool prof,
                      unsigned long long* work, int& cur, int& rerenders) {
    Counters c;
    std::memcpy(&c, ws.fs().host_counters.p, sizeof(c));
    rerenders = 0;
    if (c.overflow) {
        // bit 1: the visible depth keys span too much for the three-pass
        // sort: four passes from now on; bit 0: more duplicates than the
        // buffers hold: grow them
        if (c.overflow & 2u) ctx->depth4.store(true);
        if (c.overflow & 1u) {
            const uint64_t want = (uint64_t)c.D + c.D / 4 + 1024;
            if (want > 0xfff00000ull) fail(TIGAS_E_OOM, "duplicate count exceeds the 32-bit index range");
            ws.ensure_dups((uint32_t)want);
            ensure_bin(ws, plan);
        }
        if (debug) prepare(ws, plan, debug);
        if (work) HIPCHK(hipMemsetAsync(work, 0, 16, ws.stream));
        cur = launch_plan(ctx, ws, plan, debug, prof, work);
        wait_stream(ws.stream);
        std::memcpy(&c, ws.fs().host_counters.p, sizeof(c));
        if (c.overflow) fail(TIGAS_E_DEVICE, "duplicate buffer overflow after regrowth or four-pass depth sort");
        rerenders += 1;
    }
    ws.last_D = c.D;
    return c;
}

tigas_stats frame_stats(const Plan& plan, const Counters& c, int rerenders, bool binned, int depth_passes) {
    tigas_stats st{};
    st.visible = c.visible;
    st.duplicates = c.D;
    st.fallbacks = c.fallbacks;
    st.tiles = plan.n_tiles;
    st.sort_passes = depth_passes + (binned ? 1 : (int64_t)tile_passes(plan.n_tiles).size());
    st.rerenders = rerenders;
    st.tile_w = plan.tc.tw;
    st.tile_h = plan.tc.th;
    st.batch_depth = plan.tc.bd;
    st.pixels_per_lane = plan.tc.ppl;
    int64_t n = 0;
    for (const Group& g : plan.groups) n += g.scene->view.n * g.nviews;
    st.n = n;
    return st;
}

// Stage and kernel timings of the finished launch, and the context's stats.
// Adds the per-launch event times of the workspace's kernel timer to the
// context's per-kernel totals (the stream has completed).
void record_kernel_times(tigas_context* ctx, Workspace& ws) {
    for (const auto& r : ws.ktimer.recs) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ws.ktimer.pool[r.second], ws.ktimer.pool[r.second + 1]));
        auto& e = ctx->kernel_ms[kernel_name(r.first, ws.stream)];
        e.first += 1;
        e.second += ms;
    }
    ws.ktimer.reset();
}

void record_stats(tigas_context* ctx, Workspace& ws, const tigas_stats& st, bool prof) {
    std::lock_guard<std::mutex> lk(ctx->stats_mu);
    if (prof) {
        for (int i = 0; i < 6; ++i) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, ws.ev[i], ws.ev[i + 1]));
            ctx->stage_ms[i] += ms;
        }
        ctx->stage_frames += 1;
    }
    if (ctx->profile_kernels.load()) record_kernel_times(ctx, ws);
    ctx->last = st;
}

// Waits for an event: polls for up to ~2 ms, then blocks.
void wait_event(hipEvent_t ev) {
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const hipError_t e = hipEventQuery(ev);
        if (e == hipSuccess) return;
        if (e != hipErrorNotReady) HIPCHK(e);
        if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(2000)) break;
    }
    HIPCHK(hipEventSynchronize(ev));
}

// Completes the asynchronous frame of slot si (caller holds ws.mu): waits for
// it, redoes it if it overflowed, records its outcome under its ticket.
void finish_async(tigas_context* ctx, Workspace& ws, int si) {
    FrameSlot& f = ws.slot[si];
    if (!f.pending) return;
    f.pending = false;
    tigas_context::AsyncDone d;
    try {
        wait_event(f.t1);
        HIPCHK(hipEventElapsedTime(&d.gpu_ms, f.t0, f.t1));
        ws.active = si;
        int cur = f.cur, rerenders = 0;
        const Counters c = settle_frame(ctx, ws, f.plan, false, false, nullptr, cur, rerenders);
        d.stats = frame_stats(f.plan, c, rerenders, plan_binned(ctx, f.plan), depth_passes(ctx, f.plan));
        record_stats(ctx, ws, d.stats, false);
    } catch (const Error& e) {
        d.status = e.st;
        d.error = e.what();
    } catch (const std::exception& e) {
        d.status = TIGAS_E_DEVICE;
        d.error = e.what();
    }
    std::lock_guard<std::mutex> lk(ctx->async_mu);
    ctx->async_pending.erase(f.ticket);
    ctx->async_done[f.ticket] = d;
}

// Completes every asynchronous frame of the workspace, oldest first.
void finish_all_async(tigas_context* ctx, Workspace& ws) {
    int order[Workspace::NSLOT];
    for (int i = 0; i < Workspace::NSLOT; ++i) order[i] = i;
    std::sort(order, order + Workspace::NSLOT, [&](int a, int b) { return ws.slot[a].ticket < ws.slot[b].ticket; });
    for (int i : order) finish_async(ctx, ws, i);
}

// Runs the plan to completion (synchronous) from slot 0, after any
// asynchronous frames of the workspace.
int run_plan(tigas_context* ctx, Workspace& ws, const Plan& plan, bool debug, unsigned long long* work = nullptr) {
    finish_all_async(ctx, ws);
    ws.active = 0;
    prepare(ws, plan, debug);
    const bool prof = ctx->profile.load();
    int cur = launch_plan(ctx, ws, plan, debug, prof, work);
    wait_stream(ws.stream);
    int rerenders = 0;
    const Counters c = settle_frame(ctx, ws, plan, debug, prof, work, cur, rerenders);
    record_stats(ctx, ws, frame_stats(plan, c, rerenders, plan_binned(ctx, plan), depth_passes(ctx, plan)), prof);
    return cur;
}

// ------------------------------------------------------------- autotuner

void load_tune_file(tigas_context* ctx) {
    if (ctx->tune_file.empty()) return;
    FILE* f = std::fopen(ctx->tune_file.c_str(), "r");
    if (!f) return;
    char line[4096];
    while (std::fgets(line, sizeof line, f)) {
        int tw, th, bd, ppl;
        char key[4000];
        if (std::sscanf(line, "%d %d %d %d %3999s", &tw, &th, &bd, &ppl, key) == 5) ctx->tuned[key] = {tw, th, bd, ppl};
    }
    std::fclose(f);
}

void save_tune_file(tigas_context* ctx) {
    if (ctx->tune_file.empty()) return;
    const std::string tmp = ctx->tune_file + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    for (const auto& kv : ctx->tuned)
        std::fprintf(f, "%d %d %d %d %s\n", kv.second.tw, kv.second.th, kv.second.bd, kv.second.ppl, kv.first.c_str());
    std::fclose(f);
    std::rename(tmp.c_str(), ctx->tune_file.c_str());
}

// Picks the tile shape and batch depth for the plan's shape: each candidate
// is rendered (graph captured, two warm-ups) and timed by the median of seven
// replays; the fastest is cached per shape (and in the file named by TIGAS_TUNE_CACHE).
// Frames are identical for every candidate, so tuning changes only speed.
TileCfg autotune(tigas_context* ctx, Workspace& ws, Plan& plan) {
    const std::string key = shape_key(plan, false) + (plan.persistent ? "|P" : "|G");
    {
        std::lock_guard<std::mutex> lk(ctx->tune_mu);
        auto it = ctx->tuned.find(key);
        if (it != ctx->tuned.end()) return it->second;
    }
    const bool prof = ctx->profile.exchange(false);
    TileCfg best = kTileCandidates[2];
    double best_ms = 1e30;
    for (const TileCfg& tc : kTileCandidates) {
        set_tiles(plan, tc);
        run_plan(ctx, ws, plan, false);  // capture + warm
        run_plan(ctx, ws, plan, false);
        double ts[7];
        for (double& t : ts) {
            const auto t0 = std::chrono::steady_clock::now();
            run_plan(ctx, ws, plan, false);
            t = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        std::sort(ts, ts + 7);
        if (ts[3] < best_ms) {  // median: one slow or lucky replay does not decide
            best_ms = ts[3];
            best = tc;
        }
    }
    ctx->profile.store(prof);
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    ctx->tuned[key] = best;
    save_tune_file(ctx);
    return best;
}

hipStream_t pick_stream(tigas_context* ctx, void* s) { return s ? (hipStream_t)s : ctx->stream; }

// Host frames are rendered into a device staging buffer and copied out.
void bind_outputs(Workspace& ws, Plan& plan, tigas_frame* outs, std::vector<size_t>& stage_off) {
    size_t staging = 0;
    stage_off.assign(plan.views.size(), 0);
    for (size_t i = 0; i < plan.views.size(); ++i) {
        const ViewParams& v = plan.views[i];
        outs[i].out_w = v.width;
        outs[i].out_h = v.height;
        const size_t need = frame_bytes(v);
        if (!outs[i].data || outs[i].capacity < need) fail(TIGAS_E_BUFFER, "output frame buffer too small");
        if (!outs[i].is_device) {
            stage_off[i] = staging;
            staging += (need + 255) / 256 * 256;
        }
    }
    if (staging) ws.frame_staging.ensure(staging);  // not referenced by kernels: no graph invalidation needed
    for (size_t i = 0; i < plan.views.size(); ++i)
        plan.views[i].out_ptr = outs[i].is_device ? (uint64_t)(uintptr_t)outs[i].data
                                                  : (uint64_t)(uintptr_t)ws.frame_staging.p + stage_off[i];
}

void copy_host_outputs(Workspace& ws, const Plan& plan, tigas_frame* outs, const std::vector<size_t>& stage_off) {
    bool any = false;
    for (size_t i = 0; i < plan.views.size(); ++i)
        if (!outs[i].is_device) {
            HIPCHK(hipMemcpyAsync(outs[i].data, (char*)ws.frame_staging.p + stage_off[i], frame_bytes(plan.views[i]),
                                  hipMemcpyDeviceToHost, ws.stream));
            any = true;
        }
    if (any) HIPCHK(hipStreamSynchronize(ws.stream));
}

void debug_copy(Workspace& ws, const Plan& plan, int cur, int64_t n, uint32_t n_pad, tigas_debug_out* dbg);

// Renders the views of `plan` (already holding view parameters and groups)
// into `outs`: tile configuration from q or the autotuner.
void render_views(tigas_context* ctx, Workspace& ws, Plan& plan, const tigas_quality* q, tigas_frame* outs,
                  tigas_debug_out* dbg, int64_t* work_out) {
    std::lock_guard<std::mutex> lk(ws.mu);
    std::vector<size_t> stage_off;
    bind_outputs(ws, plan, outs, stage_off);
    // explicit tile shape: as requested; otherwise the autotuned shape for
    // this workload (16x16 for the inspection and counting entry points)
    TileCfg tc = tile_cfg(q);
    if (!tile_requested(q) && !dbg && !work_out) {
        const TileCfg req = tc;
        tc = autotune(ctx, ws, plan);
        if (q && q->batch_depth != 0) tc.bd = req.bd;
        if (q && q->pixels_per_lane != 0 && tc.th >= 16) tc.ppl = req.ppl;
    }
    set_tiles(plan, tc);
    unsigned long long* work = nullptr;
    if (work_out) {
        ws.work.ensure(16);
        work = ws.work.as<unsigned long long>();
        HIPCHK(hipMemsetAsync(work, 0, 16, ws.stream));
    }
    const int cur = run_plan(ctx, ws, plan, dbg != nullptr, work);
    if (work_out) {
        unsigned long long w[2];
        HIPCHK(hipMemcpy(w, work, 16, hipMemcpyDeviceToHost));
        work_out[0] = (int64_t)w[0];
        work_out[1] = (int64_t)w[1];
    }
    copy_host_outputs(ws, plan, outs, stage_off);
    if (dbg) debug_copy(ws, plan, cur, plan.groups[0].scene->view.n, plan.groups[0].n_pad, dbg);
}

void render_one(tigas_scene* scene, const tigas_pose* pose, const tigas_intrinsics* intr, int width, int height,
                const tigas_quality* q, tigas_frame* out, void* hip_stream, tigas_debug_out* dbg,
                int64_t* work_out = nullptr) {
    if (!scene || !out) fail(TIGAS_E_INVALID, "scene and frame are required");
    tigas_context* ctx = scene->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    SceneRef ref(scene);
    Plan plan;
    plan.views.push_back(make_view(scene, pose, intr, width, height, q));
    const uint32_t n_pad = round_up((uint64_t)scene->view.n, K1_THREADS);
    plan.groups.push_back({scene, 0, 1, 0, n_pad});
    plan.nrec = n_pad;
    Workspace& ws = ctx->workspace(pick_stream(ctx, hip_stream));
    render_views(ctx, ws, plan, q, out, dbg, work_out);
}

// Launches one frame without waiting for it (see tigas_render_submit).
void render_submit(tigas_scene* scene, const tigas_pose* pose, const tigas_intrinsics* intr, int width, int height,
                   const tigas_quality* q, tigas_frame* out, void* hip_stream, int64_t* ticket) {
    if (!scene || !out || !ticket) fail(TIGAS_E_INVALID, "scene, frame and ticket are required");
    if (!out->is_device) fail(TIGAS_E_INVALID, "an asynchronous frame needs a device output buffer");
    tigas_context* ctx = scene->ctx;
    if (ctx->profile.load() || ctx->profile_kernels.load())
        fail(TIGAS_E_INVALID, "stage and kernel timing need synchronous frames");
    HIPCHK(hipSetDevice(ctx->device));
    Plan plan;
    plan.views.push_back(make_view(scene, pose, intr, width, height, q));
    const uint32_t n_pad = round_up((uint64_t)scene->view.n, K1_THREADS);
    plan.groups.push_back({scene, 0, 1, 0, n_pad});
    plan.nrec = n_pad;
    Workspace& ws = ctx->workspace(pick_stream(ctx, hip_stream));
    std::lock_guard<std::mutex> lk(ws.mu);
    std::vector<size_t> stage_off;
    bind_outputs(ws, plan, out, stage_off);
    TileCfg tc = tile_cfg(q);
    if (!tile_requested(q)) {
        const TileCfg req = tc;
        tc = autotune(ctx, ws, plan);  // renders synchronously (after earlier frames) the first time only
        if (q && q->batch_depth != 0) tc.bd = req.bd;
        if (q && q->pixels_per_lane != 0 && tc.th >= 16) tc.ppl = req.ppl;
    }
    set_tiles(plan, tc);
    const int si = ws.next_async;
    FrameSlot& f = ws.slot[si];
    if (f.pending) finish_async(ctx, ws, si);  // two frames in flight at most
    ws.next_async = (si + 1) % Workspace::NSLOT;
    ws.active = si;
    prepare(ws, plan, false);
    if (!f.t0) HIPCHK(hipEventCreate(&f.t0));
    if (!f.t1) HIPCHK(hipEventCreate(&f.t1));
    HIPCHK(hipEventRecord(f.t0, ws.stream));
    f.cur = launch_plan(ctx, ws, plan, false, false, nullptr);
    HIPCHK(hipEventRecord(f.t1, ws.stream));
    f.plan = plan;
    f.pending = true;
    std::lock_guard<std::mutex> lk2(ctx->async_mu);
    f.ticket = ++ctx->ticket_seq;
    ctx->async_pending[f.ticket] = {&ws, si};
    *ticket = f.ticket;
}

void render_wait(tigas_context* ctx, int64_t ticket, tigas_stats* stats, float* gpu_ms) {
    Workspace* ws = nullptr;
    int si = 0;
    {
        std::lock_guard<std::mutex> lk(ctx->async_mu);
        auto it = ctx->async_pending.find(ticket);
        if (it != ctx->async_pending.end()) {
            ws = it->second.first;
            si = it->second.second;
        } else if (!ctx->async_done.count(ticket)) {
            fail(TIGAS_E_INVALID, "unknown or already collected ticket");
        }
    }
    if (ws) {
        std::lock_guard<std::mutex> lk(ws->mu);
        if (ws->slot[si].pending && ws->slot[si].ticket == ticket) finish_async(ctx, *ws, si);
    }
    tigas_context::AsyncDone d;
    {
        std::lock_guard<std::mutex> lk(ctx->async_mu);
        auto it = ctx->async_done.find(ticket);
        if (it == ctx->async_done.end()) fail(TIGAS_E_INVALID, "unknown or already collected ticket");
        d = it->second;
        ctx->async_done.erase(it);
    }
    if (d.status != TIGAS_OK) fail(d.status, d.error);
    if (stats) *stats = d.stats;
    if (gpu_ms) *gpu_ms = d.gpu_ms;
}

// ------------------------------------------------ allocation-free render
// Every buffer of the launch sequence is carved out of `scratch`, one static
// device array per device.  Host code never uses the array's name as an
// address (it names a host-side stand-in): its device address comes from
// hipGetSymbolAddress, taken once per device when a context is created there.

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};
std::string g_scratch_err[kScratchDevices];

void* scratch_address(int device) {
    if (device < 0 || device >= kScratchDevices) fail(TIGAS_E_INVALID, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device])
        fail(TIGAS_E_DEVICE, "scratch array of this device is not set up: " +
                                 (g_scratch_err[device].empty() ? std::string("no context was created on it")
                                                                : g_scratch_err[device]));
    return g_scratch_ptr[device];
}

// Bump allocator over the scratch array (256-byte aligned pieces).
struct Carver {
    char* base;
    size_t cap, off = 0;
    template <typename T>
    T* take(size_t bytes) {
        off = (off + 255) / 256 * 256;
        T* p = reinterpret_cast<T*>(base + off);
        off += std::max<size_t>(bytes, 4);
        return p;
    }
};

// Lays out a single-view launch sequence of nrec records and n_tiles tiles
// in the scratch array; the duplicate buffers take what is left.
FrameMem carve_scratch(void* scratch_dev, uint32_t nrec, uint32_t n_tiles, Counters* cnt_out, hipStream_t st) {
    Carver c{static_cast<char*>(scratch_dev), (size_t)TIGAS_NOALLOC_SCRATCH_BYTES};
    FrameMem m;
    m.stream = st;
    m.views = c.take<ViewParams>(sizeof(ViewParams));
    m.views_src = nullptr;  // the view is stored by a kernel
    m.cnt = c.take<Counters>(sizeof(Counters));
    m.cnt_out = cnt_out ? cnt_out : c.take<Counters>(sizeof(Counters));
    m.queue = c.take<uint32_t>(8 * 4);
    PreOut& o = m.pre;
    o.rec = c.take<Rec>((size_t)nrec * sizeof(Rec));
    o.rect = c.take<uint2>((size_t)nrec * 8);
    o.srect = c.take<uint2>((size_t)nrec * 8);
    o.zkey = c.take<uint32_t>((size_t)nrec * 4);
    o.fb_list = c.take<uint2>((size_t)nrec * 8);
    o.fb_cap = nrec;
    const size_t nb = (size_t)nrec / K1_THREADS + 1;
    o.blk_sum = c.take<uint32_t>(nb * 4);
    o.blk_vis = c.take<uint32_t>(nb * 4);
    o.blk_fb = c.take<uint32_t>(nb * 4);
    o.blk_view = c.take<uint32_t>(nb * 4);
    m.blk_off = c.take<uint32_t>(nb * 4);
    m.blk_sum2 = c.take<uint32_t>(nb * 4);
    m.blk_off2 = c.take<uint32_t>(nb * 4);
    const size_t nch = nb / SCAN_CHUNK + 2;
    o.chunk_vis = c.take<uint32_t>(nch * 4);
    o.chunk_fb = c.take<uint32_t>(nch * 4);
    o.chunk_dups = c.take<uint32_t>(nch * 4);
    o.chunk_dup = c.take<unsigned long long>(nch * 8);
    o.cnt = m.cnt;
    m.ranges = c.take<uint2>((size_t)std::max<uint32_t>(n_tiles, 1) * 8);
    m.order = c.take<uint32_t>((size_t)std::max<uint32_t>(n_tiles, 1) * 4);
    m.bin_hist = c.take<uint32_t>(((size_t)nrec + BIN_BLOCK - 1) / BIN_BLOCK * n_tiles * 4);
    // the first-round table sized for the largest duplicate capacity below
    m.bin_gsum = c.take<uint32_t>(((size_t)(BIN_GROUPS + 2) * n_tiles + BIN_TILES_MAX / 256 +
                                   ((size_t)nrec + BIN_BLOCK - 1) / BIN_BLOCK + 1 + bin_emit_groups(16u << 20, nrec)) * 4);
    // sort passes over at most 16M keys use at most 1024 segments
    m.hist = c.take<uint32_t>((size_t)256 * 1024 * 4);
    m.hist_tot = c.take<uint32_t>((size_t)512 * 4);
    // six duplicate arrays of dup_cap words (keys, values, extra; two each)
    const size_t left = c.cap > c.off + 6 * 256 ? c.cap - c.off - 6 * 256 : 0;
    const uint64_t dup_cap = std::min<uint64_t>(left / 24 / 256 * 256, 16u << 20);
    if (dup_cap < std::max<uint64_t>(nrec, 1))
        fail(TIGAS_E_INVALID, "scene too large for the allocation-free render: its records and the duplicate "
                              "buffers need more than the " + std::to_string(TIGAS_NOALLOC_SCRATCH_BYTES >> 20) +
                                  " MiB scratch array");
    for (int i = 0; i < 2; ++i) {
        m.key[i] = c.take<uint32_t>(dup_cap * 4);
        m.val[i] = c.take<uint32_t>(dup_cap * 4);
        m.ext[i] = c.take<uint32_t>(dup_cap * 4);
    }
    if (c.off > c.cap) fail(TIGAS_E_DEVICE, "scratch layout exceeds the array");
    m.dup_cap = (uint32_t)dup_cap;
    return m;
}

void render_noalloc(tigas_scene* scene, const tigas_pose* pose, const tigas_intrinsics* intr, int width, int height,
                    const tigas_quality* q, tigas_frame* out, tigas_frame_counters* counters, void* hip_stream) {
    if (!scene || !out) fail(TIGAS_E_INVALID, "scene and frame are required");
    if (!out->is_device) fail(TIGAS_E_INVALID, "the allocation-free render writes a device frame only");
    tigas_context* ctx = scene->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    void* scratch_dev = scratch_address(ctx->device);
    SceneRef ref(scene);
    Plan plan;
    plan.views.push_back(make_view(scene, pose, intr, width, height, q));
    const uint32_t n_pad = round_up((uint64_t)scene->view.n, K1_THREADS);
    plan.groups.push_back({scene, 0, 1, 0, n_pad});
    plan.nrec = n_pad;
    ViewParams& v = plan.views[0];
    out->out_w = v.width;
    out->out_h = v.height;
    if (!out->data || out->capacity < frame_bytes(v)) fail(TIGAS_E_BUFFER, "output frame buffer too small");
    v.out_ptr = (uint64_t)(uintptr_t)out->data;
    set_tiles(plan, tile_cfg(q));  // as requested, else 16x16 tiles: no autotuner here
    const hipStream_t st = pick_stream(ctx, hip_stream);
    const FrameMem m =
        carve_scratch(scratch_dev, plan.nrec, plan.n_tiles, reinterpret_cast<Counters*>(counters), st);
    // the previous call's counters stay in the array: start this frame from zero
    launch_fill_u32(reinterpret_cast<uint32_t*>(m.cnt), sizeof(Counters) / 4, 0u, st);
    LaunchOptions opt;
    opt.cull = ctx->blend_cull.load();
    opt.bin = ctx->tile_bin.load();
    opt.cull_tiles = ctx->tile_cull.load();
    (void)enqueue(m, plan, false, false, nullptr, 0, opt);
}

void debug_copy(Workspace& ws, const Plan& plan, int cur, int64_t n, uint32_t n_pad, tigas_debug_out* dbg) {
    Counters c;
    std::memcpy(&c, ws.fs().host_counters.p, sizeof(c));
    dbg->n_dup = c.D;
    dbg->n_tiles = plan.n_tiles;
    hipStream_t st = ws.stream;
    if (dbg->rec) {
        std::vector<Rec> a(n_pad);
        HIPCHK(hipMemcpyAsync(a.data(), ws.recs.p, sizeof(Rec) * (size_t)n_pad, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int64_t i = 0; i < n; ++i) {
            float* r = dbg->rec + 12 * i;
            const float4 x = a[i].r0, y = a[i].r1, z = a[i].r2;
            r[0] = x.x; r[1] = x.y; r[2] = x.z; r[3] = x.w;
            r[4] = y.x; r[5] = y.y; r[6] = y.z; r[7] = y.w;
            r[8] = z.x; r[9] = z.y; r[10] = z.z; r[11] = z.w;
        }
    }
    // tiles touched per record, from the tile rectangles
    std::vector<uint2> rect(n_pad);
    if (n_pad) HIPCHK(hipMemcpyAsync(rect.data(), ws.rect.p, 8 * (size_t)n_pad, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<uint32_t> touched(n_pad);
    for (uint32_t i = 0; i < n_pad; ++i) touched[i] = (rect[i].y & 0xffffu) * (rect[i].y >> 16);
    if (dbg->touched && n) std::memcpy(dbg->touched, touched.data(), 4 * (size_t)n);
    if (dbg->zkey && n) HIPCHK(hipMemcpyAsync(dbg->zkey, ws.zkey.p, 4 * (size_t)n, hipMemcpyDeviceToHost, st));
    if (dbg->bbox) {
        std::vector<Rec> rr(n_pad);
        if (n_pad) HIPCHK(hipMemcpyAsync(rr.data(), ws.recs.p, sizeof(Rec) * (size_t)n_pad, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        std::vector<uint2> bb(n_pad);
        for (uint32_t i = 0; i < n_pad; ++i) bb[i] = rr[i].bbox;
        for (int64_t i = 0; i < n; ++i) {
            int32_t* r = dbg->bbox + 4 * i;
            if (touched[i]) {
                r[0] = (int32_t)(bb[i].x & 0xffffu);
                r[1] = (int32_t)(bb[i].x >> 16);
                r[2] = (int32_t)(bb[i].y & 0xffffu);
                r[3] = (int32_t)(bb[i].y >> 16);
            } else {
                r[0] = 0; r[1] = 0; r[2] = -1; r[3] = -1;
            }
        }
    }
    const bool fits = (int64_t)c.D <= dbg->cap_dup;
    if ((dbg->keys || dbg->vals || dbg->skeys || dbg->svals) && !fits)
        fail(TIGAS_E_BUFFER, "debug duplicate arrays smaller than D");
    std::vector<uint32_t> lo(c.D), hi(c.D);
    if (c.D && (dbg->keys || dbg->vals)) {
        // entries as emitted (Gaussians in depth order), saved before the tile passes
        HIPCHK(hipMemcpyAsync(hi.data(), ws.dbg_key.p, 4 * (size_t)c.D, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(lo.data(), ws.dbg_ext.p, 4 * (size_t)c.D, hipMemcpyDeviceToHost, st));
        if (dbg->vals) HIPCHK(hipMemcpyAsync(dbg->vals, ws.dbg_val.p, 4 * (size_t)c.D, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (dbg->keys)
            for (uint32_t i = 0; i < c.D; ++i) dbg->keys[i] = ((uint64_t)hi[i] << 32) | lo[i];
    }
    if (c.D && (dbg->skeys || dbg->svals)) {
        HIPCHK(hipMemcpyAsync(hi.data(), ws.key[cur].p, 4 * (size_t)c.D, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(lo.data(), ws.ext[cur].p, 4 * (size_t)c.D, hipMemcpyDeviceToHost, st));
        if (dbg->svals) HIPCHK(hipMemcpyAsync(dbg->svals, ws.val[cur].p, 4 * (size_t)c.D, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (dbg->skeys)
            for (uint32_t i = 0; i < c.D; ++i) dbg->skeys[i] = ((uint64_t)hi[i] << 32) | lo[i];
    }
    if (dbg->ranges) {
        if (dbg->cap_tiles < (int64_t)plan.n_tiles) fail(TIGAS_E_BUFFER, "debug ranges array too small");
        HIPCHK(hipMemcpyAsync(dbg->ranges, ws.ranges.p, 8 * (size_t)plan.n_tiles, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
}

}  // namespace


// ================================================================ serving

// One JPEG of an RGB8 device frame (the result: the stream length).
struct JpegJob {
    const uint8_t* rgb;
    int width, height, quality;
    uint8_t* out;
    size_t capacity;
    uint64_t bytes;
};
void check_jpeg_args(int width, int height, int quality);
// Encodes the jobs one after another on `st` with the workspace's scratch
// buffers, then waits for the stream and fills in the lengths.
void jpeg_encode_jobs(tigas_context* ctx, Workspace& ws, hipStream_t st, JpegJob* jobs, int n);

struct tigas_server {
    tigas_context* ctx = nullptr;
    tigas_server_config cfg{};
    std::chrono::steady_clock::time_point t0;

    struct Req {
        int64_t id;
        tigas_request r;
        double arrival, dispatch = 0, done = 0;
        size_t need = 0;
        int64_t jpeg_bytes = 0;
    };
    struct Slot {
        hipStream_t stream = nullptr;
        std::thread th;
        std::vector<Req> batch;
        bool busy = false;
    };

    std::mutex mu;
    std::condition_variable cv_sched, cv_slot, cv_done;
    std::deque<Req> pending;
    std::vector<std::unique_ptr<Slot>> slots;
    std::vector<tigas_completion> completed;
    std::thread dispatcher;
    bool stop = false;
    int64_t next_id = 0, submitted = 0, finished = 0;
    tigas_server_stats st{};
    // largest duplicates-per-record seen, to size admission estimates
    double dup_per_rec = 4.0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

uint32_t request_records(const tigas_request& r) { return round_up((uint64_t)r.scene->view.n, K1_THREADS); }

// Device bytes a request adds to a batch's workspace: per record the
// preprocess outputs (64 B) and block arrays, per expected duplicate the
// double-buffered key / value / extra words (24 B), plus a staging frame
// for host outputs.
double request_pixels(const tigas_request& r) {
    const double s = r.q.res_scale != 0.f ? r.q.res_scale : 1.0;
    return std::floor(r.width * s + 0.5) * std::floor(r.height * s + 0.5);
}

// Workspace bytes per record: the 64-byte record, its tile rectangle (index
// order and depth order), depth key, FP64-list entry.
constexpr size_t kBytesPerRecord = sizeof(Rec) + 8 + 8 + 4 + 8;

size_t request_need(const tigas_server* sv, const tigas_request& r) {
    const double rec = (double)request_records(r);
    const double dup = std::max(4.0, sv->dup_per_rec) * 1.25 * rec;
    size_t frame = 0;
    if (!r.out.is_device) {
        const float s = r.q.res_scale != 0.f ? r.q.res_scale : 1.f;
        frame = (size_t)((double)r.width * s + 1) * (size_t)((double)r.height * s + 1) * 3 *
                (r.q.fmt == TIGAS_OUT_RGBF32 ? 4 : 1);
    }
    return (size_t)(rec * (double)kBytesPerRecord + dup * 24.0) + frame;
}

void server_render(tigas_server* sv, tigas_server::Slot& slot) {
    std::vector<tigas_server::Req>& b = slot.batch;
    // views of one scene next to each other: one preprocess launch per scene
    std::stable_sort(b.begin(), b.end(), [](const tigas_server::Req& x, const tigas_server::Req& y) {
        return (uintptr_t)x.r.scene < (uintptr_t)y.r.scene;
    });
    tigas_context* ctx = sv->ctx;
    Plan plan;
    plan.persistent = true;
    plan.allow_graph = false;
    std::vector<tigas_frame> outs;
    std::vector<std::unique_ptr<SceneRef>> refs;
    for (const auto& q : b) {
        plan.views.push_back(make_view(q.r.scene, &q.r.pose, &q.r.intr, q.r.width, q.r.height, &q.r.q));
        outs.push_back(q.r.out);
    }
    for (size_t i = 0; i < b.size();) {
        size_t j = i;
        while (j < b.size() && b[j].r.scene == b[i].r.scene) ++j;
        const uint32_t n_pad = request_records(b[i].r);
        plan.groups.push_back({b[i].r.scene, (int)i, (int)(j - i), plan.nrec, n_pad});
        refs.emplace_back(new SceneRef(b[i].r.scene));
        plan.nrec += n_pad * (uint32_t)(j - i);
        i = j;
    }
    tigas_quality q{};
    q.tile_w = sv->cfg.tile_w;
    q.tile_h = sv->cfg.tile_h;
    q.batch_depth = sv->cfg.batch_depth;
    q.pixels_per_lane = sv->cfg.pixels_per_lane;
    Workspace& ws = ctx->workspace(slot.stream);
    render_views(ctx, ws, plan, &q, outs.data(), nullptr, nullptr);
    // the payload: a JPEG of each frame that asks for one, on the same stream
    std::vector<JpegJob> jobs;
    std::vector<size_t> job_req;
    for (size_t i = 0; i < b.size(); ++i) {
        const tigas_request& r = b[i].r;
        if (r.jpeg_quality <= 0) continue;
        const tigas_frame& f = outs[i];  // out_w / out_h filled in by the render
        jobs.push_back({(const uint8_t*)f.data, f.out_w, f.out_h, r.jpeg_quality, (uint8_t*)r.jpeg_out,
                        r.jpeg_capacity, 0});
        job_req.push_back(i);
    }
    if (!jobs.empty()) {
        std::lock_guard<std::mutex> wl(ws.mu);
        jpeg_encode_jobs(ctx, ws, slot.stream, jobs.data(), (int)jobs.size());
        for (size_t k = 0; k < jobs.size(); ++k) b[job_req[k]].jpeg_bytes = (int64_t)jobs[k].bytes;
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    const double dpr = (double)ws.last_D / std::max<double>(1.0, (double)plan.nrec);
    sv->dup_per_rec = std::max(sv->dup_per_rec, dpr);
}

void slot_main(tigas_server* sv, tigas_server::Slot* slot) {
    (void)hipSetDevice(sv->ctx->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        sv->cv_slot.wait(lk, [&] { return sv->stop || slot->busy; });
        if (!slot->busy && sv->stop) return;
        const double t_disp = sv->now();
        for (auto& r : slot->batch) r.dispatch = t_disp;
        lk.unlock();
        int status = 0;
        std::string err;
        try {
            server_render(sv, *slot);
        } catch (const Error& e) {
            status = e.st;
            err = e.what();
        } catch (const std::exception& e) {
            status = TIGAS_E_DEVICE;
            err = e.what();
        }
        const double t_done = sv->now();
        lk.lock();
        for (auto& r : slot->batch) {
            tigas_completion c{};
            c.id = r.id;
            c.client = r.r.client;
            c.status = status;
            c.arrival_s = r.arrival;
            c.dispatch_s = r.dispatch;
            c.done_s = t_done;
            c.batch_size = (int)slot->batch.size();
            c.jpeg_bytes = r.jpeg_bytes;
            sv->completed.push_back(c);
        }
        sv->finished += (int64_t)slot->batch.size();
        sv->st.batches += 1;
        sv->st.rendered += (int64_t)slot->batch.size();
        if (status != 0) sv->st.failed += (int64_t)slot->batch.size();
        slot->batch.clear();
        slot->busy = false;
        sv->cv_sched.notify_all();
        sv->cv_done.notify_all();
    }
}

// Continuous batching: whenever a slot is idle and requests are pending, the
// pending requests (oldest first) that fit the slot's share of the memory
// budget (and the batch limit) are dispatched to it as one launch sequence.
// Requests arriving meanwhile wait for the next idle slot; slots run on their
// own streams, so batches overlap on the device.
void dispatcher_main(tigas_server* sv) {
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        tigas_server::Slot* idle = nullptr;
        sv->cv_sched.wait(lk, [&] {
            if (sv->stop) return true;
            if (sv->pending.empty()) return false;
            for (auto& s : sv->slots)
                if (!s->busy) {
                    idle = s.get();
                    return true;
                }
            return false;
        });
        if (sv->stop) return;
        const size_t budget = sv->cfg.hbm_budget ? sv->cfg.hbm_budget / sv->slots.size() : SIZE_MAX;
        const double px_cap = sv->cfg.max_batch_pixels > 0 ? (double)sv->cfg.max_batch_pixels : 1e300;
        size_t used = 0;
        double px = 0.0;
        std::deque<tigas_server::Req> keep;
        while (!sv->pending.empty()) {
            tigas_server::Req r = std::move(sv->pending.front());
            sv->pending.pop_front();
            r.need = request_need(sv, r.r);
            const double rpx = request_pixels(r.r);
            // the first request of a batch is always taken (its need fits the
            // share: checked at submit), later ones while budget and caps allow
            const bool first = idle->batch.empty();
            if ((int)idle->batch.size() < sv->cfg.max_batch && used + r.need <= budget && (first || px + rpx <= px_cap)) {
                used += r.need;
                px += rpx;
                idle->batch.push_back(std::move(r));
            } else {
                if (used + r.need > budget) sv->st.deferred += 1;
                keep.push_back(std::move(r));
            }
        }
        sv->pending.swap(keep);
        if (idle->batch.empty()) {
            // the oldest request alone exceeds what is left: it was admitted at
            // submit (fits the whole share), so take it by itself
            idle->batch.push_back(std::move(sv->pending.front()));
            sv->pending.pop_front();
        }
        sv->st.admitted += (int64_t)idle->batch.size();
        sv->st.max_batch_seen = std::max<int64_t>(sv->st.max_batch_seen, (int64_t)idle->batch.size());
        idle->busy = true;
        sv->cv_slot.notify_all();
    }
}

void validate_request(tigas_server* sv, const tigas_request* r) {
    if (!r || !r->scene) fail(TIGAS_E_INVALID, "request without a scene");
    if (r->scene->ctx != sv->ctx) fail(TIGAS_E_INVALID, "scene belongs to another context");
    (void)make_view(r->scene, &r->pose, &r->intr, r->width, r->height, &r->q);
    if (!r->out.data) fail(TIGAS_E_INVALID, "request without an output frame");
    if (r->jpeg_quality != 0) {
        if (!r->out.is_device || r->q.fmt != TIGAS_OUT_RGB8)
            fail(TIGAS_E_INVALID, "a JPEG needs an RGB8 frame in device memory");
        if (!r->jpeg_out || r->jpeg_capacity == 0) fail(TIGAS_E_INVALID, "request without a JPEG buffer");
        const float s = r->q.res_scale != 0.f ? r->q.res_scale : 1.f;
        check_jpeg_args((int)std::lround(r->width * (double)s), (int)std::lround(r->height * (double)s), r->jpeg_quality);
    }
    if (sv->cfg.hbm_budget && request_need(sv, *r) > sv->cfg.hbm_budget / sv->slots.size())
        fail(TIGAS_E_BUDGET, "request needs more workspace than a slot's share of the memory budget");
}

int64_t submit_locked(tigas_server* sv, const tigas_request* r, double arrival) {
    tigas_server::Req q;
    q.id = sv->next_id++;
    q.r = *r;
    q.arrival = arrival;
    if (sv->cfg.supersede) {
        // latest pose wins: a newer request replaces the client's waiting one
        for (auto it = sv->pending.begin(); it != sv->pending.end(); ++it)
            if (it->r.client == r->client) {
                tigas_completion c{};
                c.id = it->id;
                c.client = it->r.client;
                c.status = 1;
                c.arrival_s = it->arrival;
                c.dispatch_s = arrival;
                c.done_s = arrival;
                sv->completed.push_back(c);
                sv->finished += 1;
                sv->st.superseded += 1;
                sv->pending.erase(it);
                break;
            }
    }
    sv->pending.push_back(std::move(q));
    sv->submitted += 1;
    sv->cv_sched.notify_all();
    return sv->next_id - 1;
}

}  // namespace

// ================================================================== C ABI

namespace {

// ITU-T T.81 Annex K: quantisation tables (Tables K.1, K.2, row-major) and
// Huffman tables (K.3 to K.6: code counts per length 1..16, then symbols).
const uint8_t kQLuma[64] = {16, 11, 10, 16, 24,  40,  51,  61,  12, 12, 14, 19, 26,  58,  60,  55,
                            14, 13, 16, 24, 40,  57,  69,  56,  14, 17, 22, 29, 51,  87,  80,  62,
                            18, 22, 37, 56, 68,  109, 103, 77,  24, 35, 55, 64, 81,  104, 113, 92,
                            49, 64, 78, 87, 103, 121, 120, 101, 72, 92, 95, 98, 112, 100, 103, 99};
const uint8_t kQChroma[64] = {17, 18, 24, 47, 99, 99, 99, 99, 18, 21, 26, 66, 99, 99, 99, 99,
                              24, 26, 56, 99, 99, 99, 99, 99, 47, 66, 99, 99, 99, 99, 99, 99,
                              99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99,
                              99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99};
struct HuffSpec {
    uint8_t counts[16];
    uint8_t syms[162];
};
const HuffSpec kHuff[4] = {
    // DC luminance
    {{0, 1, 5, 1, 1, 1, 1, 1, 1, 0, 0, 0, 0, 0, 0, 0}, {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11}},
    // AC luminance
    {{0, 2, 1, 3, 3, 2, 4, 3, 5, 5, 4, 4, 0, 0, 1, 0x7d},
     {0x01, 0x02, 0x03, 0x00, 0x04, 0x11, 0x05, 0x12, 0x21, 0x31, 0x41, 0x06, 0x13, 0x51, 0x61, 0x07, 0x22, 0x71,
      0x14, 0x32, 0x81, 0x91, 0xa1, 0x08, 0x23, 0x42, 0xb1, 0xc1, 0x15, 0x52, 0xd1, 0xf0, 0x24, 0x33, 0x62, 0x72,
      0x82, 0x09, 0x0a, 0x16, 0x17, 0x18, 0x19, 0x1a, 0x25, 0x26, 0x27, 0x28, 0x29, 0x2a, 0x34, 0x35, 0x36, 0x37,
      0x38, 0x39, 0x3a, 0x43, 0x44, 0x45, 0x46, 0x47, 0x48, 0x49, 0x4a, 0x53, 0x54, 0x55, 0x56, 0x57, 0x58, 0x59,
      0x5a, 0x63, 0x64, 0x65, 0x66, 0x67, 0x68, 0x69, 0x6a, 0x73, 0x74, 0x75, 0x76, 0x77, 0x78, 0x79, 0x7a, 0x83,
      0x84, 0x85, 0x86, 0x87, 0x88, 0x89, 0x8a, 0x92, 0x93, 0x94, 0x95, 0x96, 0x97, 0x98, 0x99, 0x9a, 0xa2, 0xa3,
      0xa4, 0xa5, 0xa6, 0xa7, 0xa8, 0xa9, 0xaa, 0xb2, 0xb3, 0xb4, 0xb5, 0xb6, 0xb7, 0xb8, 0xb9, 0xba, 0xc2, 0xc3,
      0xc4, 0xc5, 0xc6, 0xc7, 0xc8, 0xc9, 0xca, 0xd2, 0xd3, 0xd4, 0xd5, 0xd6, 0xd7, 0xd8, 0xd9, 0xda, 0xe1, 0xe2,
      0xe3, 0xe4, 0xe5, 0xe6, 0xe7, 0xe8, 0xe9, 0xea, 0xf1, 0xf2, 0xf3, 0xf4, 0xf5, 0xf6, 0xf7, 0xf8, 0xf9, 0xfa}},
    // DC chrominance
    {{0, 3, 1, 1, 1, 1, 1, 1, 1, 1, 1, 0, 0, 0, 0, 0}, {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11}},
    // AC chrominance
    {{0, 2, 1, 2, 4, 4, 3, 4, 7, 5, 4, 4, 0, 1, 2, 0x77},
     {0x00, 0x01, 0x02, 0x03, 0x11, 0x04, 0x05, 0x21, 0x31, 0x06, 0x12, 0x41, 0x51, 0x07, 0x61, 0x71, 0x13, 0x22,
      0x32, 0x81, 0x08, 0x14, 0x42, 0x91, 0xa1, 0xb1, 0xc1, 0x09, 0x23, 0x33, 0x52, 0xf0, 0x15, 0x62, 0x72, 0xd1,
      0x0a, 0x16, 0x24, 0x34, 0xe1, 0x25, 0xf1, 0x17, 0x18, 0x19, 0x1a, 0x26, 0x27, 0x28, 0x29, 0x2a, 0x35, 0x36,
      0x37, 0x38, 0x39, 0x3a, 0x43, 0x44, 0x45, 0x46, 0x47, 0x48, 0x49, 0x4a, 0x53, 0x54, 0x55, 0x56, 0x57, 0x58,
      0x59, 0x5a, 0x63, 0x64, 0x65, 0x66, 0x67, 0x68, 0x69, 0x6a, 0x73, 0x74, 0x75, 0x76, 0x77, 0x78, 0x79, 0x7a,
      0x82, 0x83, 0x84, 0x85, 0x86, 0x87, 0x88, 0x89, 0x8a, 0x92, 0x93, 0x94, 0x95, 0x96, 0x97, 0x98, 0x99, 0x9a,
      0xa2, 0xa3, 0xa4, 0xa5, 0xa6, 0xa7, 0xa8, 0xa9, 0xaa, 0xb2, 0xb3, 0xb4, 0xb5, 0xb6, 0xb7, 0xb8, 0xb9, 0xba,
      0xc2, 0xc3, 0xc4, 0xc5, 0xc6, 0xc7, 0xc8, 0xc9, 0xca, 0xd2, 0xd3, 0xd4, 0xd5, 0xd6, 0xd7, 0xd8, 0xd9, 0xda,
      0xe2, 0xe3, 0xe4, 0xe5, 0xe6, 0xe7, 0xe8, 0xe9, 0xea, 0xf2, 0xf3, 0xf4, 0xf5, 0xf6, 0xf7, 0xf8, 0xf9, 0xfa}},
};

int huff_count(const HuffSpec& h) {
    int n = 0;
    for (uint8_t c : h.counts) n += c;
    return n;
}

// Quality scaling of a base table: 5000/q below 50, else 200 - 2q percent,
// rounded, within 1..255 (8-bit tables).
void scaled_qtable(const uint8_t* base, int quality, uint8_t* out) {
    const long s = quality < 50 ? 5000 / quality : 200 - 2 * quality;
    for (int i = 0; i < 64; ++i) out[i] = (uint8_t)std::min(255L, std::max(1L, ((long)base[i] * s + 50) / 100));
}

// Row-major index of each zig-zag scan position.
void zigzag_order(int* zz) {
    int i = 0;
    for (int d = 0; d < 15; ++d)
        for (int j = std::min(d, 7); j >= std::max(0, d - 7); --j) {
            const int row = (d & 1) ? d - j : j;
            zz[i++] = row * 8 + (d - row);
        }
}

// Canonical codes (Annex C) of a table, as length << 16 | code per symbol.
void huff_codes(const HuffSpec& h, uint32_t* out) {
    std::fill(out, out + 256, 0u);
    uint32_t code = 0;
    int k = 0;
    for (int len = 1; len <= 16; ++len) {
        for (int i = 0; i < h.counts[len - 1]; ++i, ++k) out[h.syms[k]] = ((uint32_t)len << 16) | code++;
        code <<= 1;
    }
}

// SOI, JFIF APP0, DQT, SOF0 (4:4:4), DHT, DRI (JPEG_SEG_MCUS MCUs), SOS.
std::vector<uint8_t> jpeg_header(int W, int H, const uint8_t* ql, const uint8_t* qc) {
    std::vector<uint8_t> h;
    auto b = [&](unsigned v) { h.push_back((uint8_t)v); };
    auto w16 = [&](unsigned v) {
        b(v >> 8);
        b(v & 0xff);
    };
    int zz[64];
    zigzag_order(zz);
    w16(0xFFD8);
    w16(0xFFE0);
    w16(16);
    const uint8_t jfif[14] = {'J', 'F', 'I', 'F', 0, 1, 1, 0, 0, 1, 0, 1, 0, 0};  // version 1.01, no density units
    for (uint8_t v : jfif) b(v);
    w16(0xFFDB);
    w16(2 + 2 * 65);
    b(0);
    for (int i = 0; i < 64; ++i) b(ql[zz[i]]);
    b(1);
    for (int i = 0; i < 64; ++i) b(qc[zz[i]]);
    w16(0xFFC0);
    w16(17);
    b(8);
    w16((unsigned)H);
    w16((unsigned)W);
    b(3);
    for (int c = 0; c < 3; ++c) {
        b(c + 1);
        b(0x11);
        b(c ? 1 : 0);
    }
    int len = 2;
    for (const HuffSpec& t : kHuff) len += 17 + huff_count(t);
    w16(0xFFC4);
    w16((unsigned)len);
    const unsigned cls_id[4] = {0x00, 0x10, 0x01, 0x11};
    for (int t = 0; t < 4; ++t) {
        b(cls_id[t]);
        for (uint8_t c : kHuff[t].counts) b(c);
        for (int i = 0; i < huff_count(kHuff[t]); ++i) b(kHuff[t].syms[i]);
    }
    w16(0xFFDD);
    w16(4);
    w16((unsigned)JPEG_SEG_MCUS);
    w16(0xFFDA);
    w16(12);
    b(3);
    for (int c = 0; c < 3; ++c) {
        b(c + 1);
        b(c ? 0x11 : 0x00);
    }
    b(0);
    b(63);
    b(0);
    return h;
}

// Bound on the entropy-coded bits of one block: DC 11 + 11, 63 AC symbols of
// at most 16 + 10 bits.
constexpr uint32_t kBlockMaxBits = 22 + 63 * 26;

}  // namespace

void check_jpeg_args(int width, int height, int quality) {
    if (width < 1 || width > 65535 || height < 1 || height > 65535)
        fail(TIGAS_E_INVALID, "jpeg: width and height must be 1..65535");
    if (quality < 1 || quality > 100) fail(TIGAS_E_INVALID, "jpeg: quality must be 1..100");
}

void jpeg_encode_jobs(tigas_context* ctx, Workspace& ws, hipStream_t st, JpegJob* jobs, int n) {
    if (n <= 0) return;
    const uint32_t seg_words = (uint32_t)((3 * JPEG_SEG_MCUS * (size_t)kBlockMaxBits + 31) / 32 + 1);
    int max_seg = 1;
    for (int i = 0; i < n; ++i) {
        const int64_t n_mcu = (int64_t)((jobs[i].width + 7) / 8) * ((jobs[i].height + 7) / 8);
        max_seg = std::max(max_seg, (int)((n_mcu + JPEG_SEG_MCUS - 1) / JPEG_SEG_MCUS));
    }
    if (ws.jpeg_bits.ensure((size_t)max_seg * seg_words * 4)) HIPCHK(hipMemset(ws.jpeg_bits.p, 0, ws.jpeg_bits.bytes));
    ws.jpeg_seg_bits.ensure((size_t)max_seg * 4);
    ws.jpeg_seg_len.ensure((size_t)max_seg * 4);
    ws.jpeg_huff.ensure(4 * 256 * 4);
    ws.jpeg_len.ensure((size_t)n * 8);
    ws.jpeg_len_host.ensure((size_t)n * 8);
    uint32_t codes[4 * 256];
    for (int t = 0; t < 4; ++t) huff_codes(kHuff[t], codes + 256 * t);
    HIPCHK(hipMemcpyAsync(ws.jpeg_huff.p, codes, sizeof codes, hipMemcpyHostToDevice, st));
    float dct[64];
    for (int k = 0; k < 8; ++k)
        for (int m = 0; m < 8; ++m) {  // rounded once from FP64
            const double ck = k == 0 ? std::sqrt(0.5) : 1.0;
            dct[k * 8 + m] = (float)(0.5 * ck * std::cos((2 * m + 1) * k * 3.14159265358979323846 / 16.0));
        }
    const bool kprof = ctx->profile_kernels.load();
    if (kprof) ws.ktimer.reset();
    TimerScope ts(kprof ? &ws.ktimer : nullptr);
    std::vector<std::vector<uint8_t>> hdrs(n);  // alive until the stream has finished
    for (int i = 0; i < n; ++i) {
        const JpegJob& j = jobs[i];
        JpegArgs a{};
        a.rgb = j.rgb;
        a.width = j.width;
        a.height = j.height;
        a.w8 = (j.width + 7) / 8;
        a.h8 = (j.height + 7) / 8;
        a.n_mcu = (int64_t)a.w8 * a.h8;
        a.nseg = (int)((a.n_mcu + JPEG_SEG_MCUS - 1) / JPEG_SEG_MCUS);
        a.seg_words = seg_words;
        uint8_t ql[64], qc[64];
        scaled_qtable(kQLuma, j.quality, ql);
        scaled_qtable(kQChroma, j.quality, qc);
        for (int k = 0; k < 64; ++k) {
            a.rq_luma[k] = 1.0f / (float)ql[k];
            a.rq_chroma[k] = 1.0f / (float)qc[k];
            a.dct[k] = dct[k];
        }
        hdrs[i] = jpeg_header(j.width, j.height, ql, qc);
        HIPCHK(hipMemcpyAsync(j.out, hdrs[i].data(), std::min(hdrs[i].size(), j.capacity), hipMemcpyHostToDevice, st));
        a.huff = ws.jpeg_huff.as<uint32_t>();
        a.bits = ws.jpeg_bits.as<uint32_t>();
        a.seg_bits = ws.jpeg_seg_bits.as<uint32_t>();
        a.seg_len = ws.jpeg_seg_len.as<uint32_t>();
        a.out = j.out;
        a.capacity = j.capacity;
        a.header_len = hdrs[i].size();
        a.out_len = ws.jpeg_len.as<uint64_t>() + i;
        launch_jpeg(a, st);  // jobs run one after another on the stream and share the scratch buffers
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(ws.jpeg_len_host.p, ws.jpeg_len.p, (size_t)n * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (kprof) record_kernel_times(ctx, ws);
    for (int i = 0; i < n; ++i) std::memcpy(&jobs[i].bytes, (const uint8_t*)ws.jpeg_len_host.p + 8 * i, 8);
}

// Latency ABR controller state (tigas_abr_*): the throughput samples of the
// window in arrival order, the average, the level and the hold counter.
struct tigas_abr {
    tigas_abr_config cfg{};
    std::deque<double> samples;  // KB/s, oldest first
    double rate_kbps = 0.0;
    int level = 0;
    int direction = 0;  // +1 / -1: the condition of the last requests
    int streak = 0;

    double expected_time(int l) const { return cfg.expected_bytes[l] / (rate_kbps * 1024.0); }
    int observe(double bytes, double seconds, bool rapid_pan) {
        samples.push_back(bytes / seconds / 1024.0);
        while ((int)samples.size() > cfg.history) samples.pop_front();
        double e = samples.front();  // the window's oldest sample, then the newer ones
        for (size_t i = 1; i < samples.size(); ++i) e = cfg.alpha * samples[i] + (1.0 - cfg.alpha) * e;
        rate_kbps = e;
        int want = 0;
        if (level + 1 < cfg.n_levels && expected_time(level + 1) <= cfg.t_target_s) want = 1;
        else if (level > 0 && expected_time(level) > cfg.t_margin_s) want = -1;
        if (want == -1 && rapid_pan) {  // panning: downgrade at once
            --level;
            direction = streak = 0;
            return level;
        }
        if (want != 0 && want == direction) {
            ++streak;
        } else {
            direction = want;
            streak = want ? 1 : 0;
        }
        if (want != 0 && streak >= cfg.hold) {
            level += want;
            direction = streak = 0;
        }
        return level;
    }
};

extern "C" {

const char* tigas_last_error(void) { return g_err.c_str(); }

tigas_status tigas_context_create(int device, tigas_context** out) {
    return guard([&] {
        if (!out) fail(TIGAS_E_INVALID, "out is null");
        int n = 0;
        HIPCHK(hipGetDeviceCount(&n));
        if (device < 0 || device >= n) fail(TIGAS_E_INVALID, "no such HIP device");
        HIPCHK(hipSetDevice(device));
        std::unique_ptr<tigas_context> c(new tigas_context());
        c->device = device;
        hipDeviceProp_t prop;
        HIPCHK(hipGetDeviceProperties(&prop, device));
        c->cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
        if (device < kScratchDevices) {  // device address of this device's scratch array, once per device
            std::lock_guard<std::mutex> lk(g_scratch_mu);
            if (!g_scratch_ptr[device]) {
                void* ptr = nullptr;
                const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
                if (e == hipSuccess && ptr) {
                    g_scratch_ptr[device] = ptr;
                } else {  // only the allocation-free render needs it: it reports this error
                    (void)hipGetLastError();
                    g_scratch_err[device] = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
                }
            }
        }
        HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        if (const char* f = std::getenv("TIGAS_TUNE_CACHE")) c->tune_file = f;
        if (const char* g = std::getenv("TIGAS_GRAPHS")) c->use_graphs.store(std::atoi(g) != 0);
        if (const char* g = std::getenv("TIGAS_BLEND_CULL")) c->blend_cull.store(std::atoi(g) != 0);
        if (const char* g = std::getenv("TIGAS_TILE_BIN")) c->tile_bin.store(std::atoi(g) != 0);
        if (const char* g = std::getenv("TIGAS_TILE_CULL")) c->tile_cull.store(std::atoi(g) != 0);
        if (const char* g = std::getenv("TIGAS_DEPTH_PASSES")) c->depth4.store(std::atoi(g) == 4);
        load_tune_file(c.get());
        *out = c.release();
    });
}

void tigas_context_destroy(tigas_context* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->ws.clear();
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

tigas_status tigas_scene_load(tigas_context* ctx, const tigas_scene_desc* d, tigas_scene** out) {
    return guard([&] {
        if (!ctx || !d || !out) fail(TIGAS_E_INVALID, "null argument");
        if (d->n < 0 || d->n > (int64_t)0x7f000000) fail(TIGAS_E_INVALID, "n out of range");
        if (d->sh_degree < 0 || d->sh_degree > 3) fail(TIGAS_E_INVALID, "sh_degree must be 0..3");
        if (d->storage < TIGAS_ATTR_F32 || d->storage > TIGAS_ATTR_BF16) fail(TIGAS_E_INVALID, "unknown storage");
        const int64_t n = d->n;
        if (n > 0 && (!d->means || !d->log_scales || !d->quats_wxyz || !d->opacity_logits || !d->sh))
            fail(TIGAS_E_INVALID, "attribute array is null");
        HIPCHK(hipSetDevice(ctx->device));
        // device inputs come to the host first; host inputs are read in place
        std::vector<float> mv, lsv, qv, opv, shv;
        auto fetch = [&](std::vector<float>& dst, const float* src, size_t cnt) -> const float* {
            if (!d->is_device || cnt == 0) return src;
            dst.resize(cnt);
            HIPCHK(hipMemcpy(dst.data(), src, cnt * 4, hipMemcpyDeviceToHost));
            return dst.data();
        };
        const float* m = fetch(mv, d->means, (size_t)n * 3);
        const float* ls = fetch(lsv, d->log_scales, (size_t)n * 3);
        const float* q = fetch(qv, d->quats_wxyz, (size_t)n * 4);
        const float* op = fetch(opv, d->opacity_logits, (size_t)n);
        const float* sh = fetch(shv, d->sh, (size_t)n * 48);
        std::unique_ptr<tigas_scene> s(new tigas_scene());
        static std::atomic<uint64_t> next_uid{0};
        s->uid = ++next_uid;
        s->ctx = ctx;
        const int deg = d->sh_degree;
        const int ncoef = 3 * (deg + 1) * (deg + 1);
        const size_t nn = (size_t)std::max<int64_t>(n, 1);
        // centres: FP32 planes
        std::vector<float> mp(3 * nn);
        parallel_for(n, [&](int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i)
                for (int c = 0; c < 3; ++c) mp[c * n + i] = m[3 * i + c];
        });
        s->mean.ensure(mp.size() * 4);
        HIPCHK(hipMemcpy(s->mean.p, mp.data(), (size_t)n * 12, hipMemcpyHostToDevice));
        if (d->storage == TIGAS_ATTR_F32) {
            std::vector<float> a(8 * nn);
            parallel_for(n, [&](int64_t i0, int64_t i1) {
                for (int64_t i = i0; i < i1; ++i) {
                    for (int c = 0; c < 4; ++c) a[4 * i + c] = q[4 * i + c];
                    for (int c = 0; c < 3; ++c) a[4 * n + 4 * i + c] = ls[3 * i + c];
                    a[4 * n + 4 * i + 3] = op[i];
                }
            });
            // SH: the np 16-byte words of a Gaussian are contiguous, so a
            // culled Gaussian's coefficients are never fetched
            const int np = (ncoef + 3) / 4;
            std::vector<float> shp((size_t)np * 4 * nn, 0.f);
            parallel_for(n, [&](int64_t i0, int64_t i1) {
                for (int64_t i = i0; i < i1; ++i)
                    for (int k = 0; k < ncoef; ++k) shp[(size_t)i * np * 4 + k] = sh[48 * i + k];
            });
            s->view.sh_stride = np;
            s->attr.ensure(a.size() * 4);
            s->sh.ensure(shp.size() * 4);
            HIPCHK(hipMemcpy(s->attr.p, a.data(), (size_t)n * 32, hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(s->sh.p, shp.data(), (size_t)np * n * 16, hipMemcpyHostToDevice));
            s->bytes = (size_t)n * (12 + 32 + (size_t)np * 16);
        } else {
            auto cvt = [&](float f) { return d->storage == TIGAS_ATTR_BF16 ? f32_to_bf16(f) : f32_to_f16(f); };
            std::vector<uint16_t> a(8 * nn);
            parallel_for(n, [&](int64_t i0, int64_t i1) {
                for (int64_t i = i0; i < i1; ++i) {
                    for (int c = 0; c < 4; ++c) a[8 * i + c] = cvt(q[4 * i + c]);
                    for (int c = 0; c < 3; ++c) a[8 * i + 4 + c] = cvt(ls[3 * i + c]);
                    a[8 * i + 7] = cvt(op[i]);
                }
            });
            const int np = (ncoef + 7) / 8;
            std::vector<uint16_t> shp((size_t)np * 8 * nn, 0);
            parallel_for(n, [&](int64_t i0, int64_t i1) {
                for (int64_t i = i0; i < i1; ++i)
                    for (int k = 0; k < ncoef; ++k) shp[(size_t)i * np * 8 + k] = cvt(sh[48 * i + k]);
            });
            s->view.sh_stride = np;
            s->attr.ensure(a.size() * 2);
            s->sh.ensure(shp.size() * 2);
            HIPCHK(hipMemcpy(s->attr.p, a.data(), (size_t)n * 16, hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(s->sh.p, shp.data(), (size_t)np * n * 16, hipMemcpyHostToDevice));
            s->bytes = (size_t)n * (12 + 16 + (size_t)np * 16);
        }
        s->view.n = n;
        s->view.storage = (int)d->storage;
        s->view.sh_degree = deg;
        s->view.mean = s->mean.as<float>();
        s->view.attr = s->attr.p;
        s->view.sh = s->sh.p;
        *out = s.release();
    });
}

void tigas_scene_free(tigas_scene* s) {
    if (!s) return;
    (void)hipSetDevice(s->ctx->device);
    (void)hipDeviceSynchronize();
    delete s;
}

size_t tigas_scene_bytes(const tigas_scene* s) { return s ? s->bytes : 0; }

tigas_status tigas_render(tigas_scene* scene, const tigas_pose* pose, const tigas_intrinsics* intr, int width,
                          int height, const tigas_quality* q, tigas_frame* out, void* hip_stream) {
    return guard([&] { render_one(scene, pose, intr, width, height, q, out, hip_stream, nullptr); });
}

tigas_status tigas_render_noalloc(tigas_scene* scene, const tigas_pose* pose, const tigas_intrinsics* intr,
                                  int width, int height, const tigas_quality* q, tigas_frame* out,
                                  tigas_frame_counters* counters, void* hip_stream) {
    return guard([&] { render_noalloc(scene, pose, intr, width, height, q, out, counters, hip_stream); });
}

tigas_status tigas_render_debug(tigas_scene* scene, const tigas_pose* pose, const tigas_intrinsics* intr, int width,
                                int height, const tigas_quality* q, tigas_frame* out, tigas_debug_out* dbg) {
    return guard([&] {
        if (!dbg) fail(TIGAS_E_INVALID, "debug output is null");
        render_one(scene, pose, intr, width, height, q, out, nullptr, dbg);
    });
}

tigas_status tigas_render_batch(tigas_scene* const* scenes, const tigas_pose* poses, const tigas_intrinsics* intrs,
                                const int* widths, const int* heights, const tigas_quality* q, int n_views,
                                tigas_frame* outs, void* hip_stream) {
    return guard([&] {
        if (n_views < 1 || !scenes || !poses || !intrs || !widths || !heights || !outs)
            fail(TIGAS_E_INVALID, "null argument or no views");
        tigas_context* ctx = scenes[0] ? scenes[0]->ctx : nullptr;
        if (!ctx) fail(TIGAS_E_INVALID, "null scene");
        HIPCHK(hipSetDevice(ctx->device));
        Plan plan;
        plan.persistent = true;
        std::vector<std::unique_ptr<SceneRef>> refs;
        for (int i = 0; i < n_views; ++i) {
            if (!scenes[i] || scenes[i]->ctx != ctx) fail(TIGAS_E_INVALID, "scenes must share one context");
            plan.views.push_back(make_view(scenes[i], &poses[i], &intrs[i], widths[i], heights[i], q ? &q[i] : nullptr));
        }
        // consecutive views of one scene share one preprocess launch
        for (int i = 0; i < n_views;) {
            int j = i;
            while (j < n_views && scenes[j] == scenes[i]) ++j;
            const uint32_t n_pad = round_up((uint64_t)scenes[i]->view.n, K1_THREADS);
            plan.groups.push_back({scenes[i], i, j - i, plan.nrec, n_pad});
            refs.emplace_back(new SceneRef(scenes[i]));
            plan.nrec += n_pad * (uint32_t)(j - i);
            i = j;
        }
        Workspace& ws = ctx->workspace(pick_stream(ctx, hip_stream));
        render_views(ctx, ws, plan, q, outs, nullptr, nullptr);
    });
}

tigas_status tigas_last_stats(tigas_context* ctx, tigas_stats* out) {
    return guard([&] {
        if (!ctx || !out) fail(TIGAS_E_INVALID, "null argument");
        std::lock_guard<std::mutex> lk(ctx->stats_mu);
        *out = ctx->last;
    });
}

tigas_status tigas_profile_stages(tigas_context* ctx, int enable) {
    return guard([&] {
        if (!ctx) fail(TIGAS_E_INVALID, "null context");
        std::lock_guard<std::mutex> lk(ctx->stats_mu);
        for (double& x : ctx->stage_ms) x = 0.0;
        ctx->stage_frames = 0;
        ctx->profile.store(enable != 0);
    });
}

tigas_status tigas_profile_kernels(tigas_context* ctx, int enable) {
    return guard([&] {
        if (!ctx) fail(TIGAS_E_INVALID, "null context");
        std::lock_guard<std::mutex> lk(ctx->stats_mu);
        ctx->kernel_ms.clear();
        ctx->profile_kernels.store(enable != 0);
    });
}

tigas_status tigas_kernel_times(tigas_context* ctx, tigas_kernel_time* out, int cap, int* count) {
    return guard([&] {
        if (!ctx || !count || cap < 0 || (cap > 0 && !out)) fail(TIGAS_E_INVALID, "null argument");
        std::lock_guard<std::mutex> lk(ctx->stats_mu);
        int i = 0;
        for (const auto& kv : ctx->kernel_ms) {
            if (i < cap) {
                std::snprintf(out[i].name, sizeof out[i].name, "%s", kv.first.c_str());
                out[i].launches = kv.second.first;
                out[i].total_ms = kv.second.second;
            }
            ++i;
        }
        *count = i;
    });
}

tigas_status tigas_stage_times(tigas_context* ctx, tigas_stage_ms* out) {
    return guard([&] {
        if (!ctx || !out) fail(TIGAS_E_INVALID, "null argument");
        std::lock_guard<std::mutex> lk(ctx->stats_mu);
        out->preprocess = ctx->stage_ms[0];
        out->scan = ctx->stage_ms[1];
        out->duplicate = ctx->stage_ms[2];
        out->sort = ctx->stage_ms[3];
        out->ranges = ctx->stage_ms[4];
        out->blend = ctx->stage_ms[5];
        out->frames = ctx->stage_frames;
    });
}

tigas_status tigas_render_submit(tigas_scene* scene, const tigas_pose* pose, const tigas_intrinsics* intr, int width,
                                 int height, const tigas_quality* q, tigas_frame* out, void* hip_stream,
                                 int64_t* ticket) {
    return guard([&] { render_submit(scene, pose, intr, width, height, q, out, hip_stream, ticket); });
}

tigas_status tigas_render_wait(tigas_context* ctx, int64_t ticket, tigas_stats* stats, float* gpu_ms) {
    return guard([&] {
        if (!ctx) fail(TIGAS_E_INVALID, "null context");
        render_wait(ctx, ticket, stats, gpu_ms);
    });
}

tigas_status tigas_set_graphs(tigas_context* ctx, int enable) {
    return guard([&] {
        if (!ctx) fail(TIGAS_E_INVALID, "null context");
        ctx->use_graphs.store(enable != 0);
    });
}

tigas_status tigas_set_tile_binning(tigas_context* ctx, int enable) {
    return guard([&] {
        if (!ctx) fail(TIGAS_E_INVALID, "null context");
        ctx->tile_bin.store(enable != 0);
    });
}

tigas_status tigas_set_tile_culling(tigas_context* ctx, int enable) {
    return guard([&] {
        if (!ctx) fail(TIGAS_E_INVALID, "null context");
        ctx->tile_cull.store(enable != 0);
    });
}

tigas_status tigas_set_depth_passes(tigas_context* ctx, int passes) {
    return guard([&] {
        if (!ctx) fail(TIGAS_E_INVALID, "null context");
        if (passes != 3 && passes != 4) fail(TIGAS_E_INVALID, "depth passes must be 3 or 4");
        ctx->depth4.store(passes == 4);
    });
}


tigas_status tigas_count_blend_work(tigas_scene* scene, const tigas_pose* pose, const tigas_intrinsics* intr,
                                    int width, int height, const tigas_quality* q, tigas_frame* out,
                                    int64_t* evaluations, int64_t* contributions) {
    return guard([&] {
        if (!evaluations || !contributions) fail(TIGAS_E_INVALID, "null counter output");
        int64_t w[2] = {0, 0};
        render_one(scene, pose, intr, width, height, q, out, nullptr, nullptr, w);
        *evaluations = w[0];
        *contributions = w[1];
    });
}

size_t tigas_jpeg_max_bytes(int width, int height) {
    if (width < 1 || height < 1) return 0;
    const size_t n_mcu = (((size_t)width + 7) / 8) * (((size_t)height + 7) / 8);
    const size_t nseg = (n_mcu + JPEG_SEG_MCUS - 1) / JPEG_SEG_MCUS;
    const size_t seg = (3 * JPEG_SEG_MCUS * (size_t)kBlockMaxBits + 7) / 8;
    return 1024 + nseg * (2 * seg + 2);  // every byte stuffed at worst, plus the marker
}

tigas_status tigas_jpeg_encode(tigas_context* ctx, const void* rgb, int width, int height, int quality, void* out,
                               size_t capacity, size_t* out_len, void* hip_stream) {
    return guard([&] {
        if (!ctx || !rgb || !out || !out_len) fail(TIGAS_E_INVALID, "null argument");
        check_jpeg_args(width, height, quality);
        HIPCHK(hipSetDevice(ctx->device));
        hipStream_t st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
        Workspace& ws = ctx->workspace(st);
        std::lock_guard<std::mutex> lk(ws.mu);
        JpegJob job{(const uint8_t*)rgb, width, height, quality, (uint8_t*)out, capacity, 0};
        jpeg_encode_jobs(ctx, ws, st, &job, 1);
        *out_len = (size_t)job.bytes;
        if (job.bytes > capacity) fail(TIGAS_E_BUFFER, "jpeg: output buffer smaller than the stream");
    });
}

void tigas_abr_default_config(tigas_abr_config* cfg) {
    if (!cfg) return;
    *cfg = tigas_abr_config{};
    cfg->n_levels = 4;
    const double kb[4] = {7, 20, 55, 240};  // Table 1: middles of the size ranges
    for (int i = 0; i < 4; ++i) cfg->expected_bytes[i] = kb[i] * 1024.0;
    cfg->t_target_s = 0.100;
    cfg->t_margin_s = 0.150;
    cfg->alpha = 0.3;
    cfg->history = 5;
    cfg->hold = 3;
    cfg->start_level = 0;
}

tigas_status tigas_abr_create(const tigas_abr_config* cfg, tigas_abr** out) {
    return guard([&] {
        if (!out) fail(TIGAS_E_INVALID, "null output");
        tigas_abr_config c;
        if (cfg) c = *cfg;
        else tigas_abr_default_config(&c);
        if (c.n_levels < 1 || c.n_levels > 8) fail(TIGAS_E_INVALID, "abr: n_levels must be 1..8");
        for (int i = 0; i < c.n_levels; ++i)
            if (!(c.expected_bytes[i] > 0) || (i > 0 && !(c.expected_bytes[i] > c.expected_bytes[i - 1])))
                fail(TIGAS_E_INVALID, "abr: expected sizes must be positive and rising");
        if (!(c.t_target_s > 0) || !(c.t_margin_s > c.t_target_s))
            fail(TIGAS_E_INVALID, "abr: need 0 < t_target < t_margin");
        if (!(c.alpha > 0 && c.alpha <= 1)) fail(TIGAS_E_INVALID, "abr: alpha must be in (0, 1]");
        if (c.history < 1 || c.history > 64 || c.hold < 1) fail(TIGAS_E_INVALID, "abr: history 1..64, hold >= 1");
        if (c.start_level < 0 || c.start_level >= c.n_levels) fail(TIGAS_E_INVALID, "abr: bad start level");
        tigas_abr* a = new tigas_abr;
        a->cfg = c;
        a->level = c.start_level;
        *out = a;
    });
}

void tigas_abr_destroy(tigas_abr* abr) { delete abr; }

tigas_status tigas_abr_observe(tigas_abr* abr, double bytes, double seconds, int rapid_pan, int* level) {
    return guard([&] {
        if (!abr || !level) fail(TIGAS_E_INVALID, "null argument");
        if (!(bytes > 0) || !(seconds > 0) || !std::isfinite(bytes) || !std::isfinite(seconds))
            fail(TIGAS_E_INVALID, "abr: bytes and seconds must be positive");
        *level = abr->observe(bytes, seconds, rapid_pan != 0);
    });
}

tigas_status tigas_abr_rate(const tigas_abr* abr, double* kbytes_per_s) {
    return guard([&] {
        if (!abr || !kbytes_per_s) fail(TIGAS_E_INVALID, "null argument");
        *kbytes_per_s = abr->rate_kbps;
    });
}

tigas_status tigas_selftest_wave_scan(const uint32_t* in, uint32_t* out, int n) {
    return guard([&] {
        if (!in || !out || n < 0) fail(TIGAS_E_INVALID, "bad arguments");
        if (n == 0) return;
        void *din = nullptr, *dout = nullptr;
        HIPCHK(hipMalloc(&din, (size_t)n * 4));
        HIPCHK(hipMalloc(&dout, (size_t)n * 4));
        HIPCHK(hipMemcpy(din, in, (size_t)n * 4, hipMemcpyHostToDevice));
        launch_wave_scan_selftest((const uint32_t*)din, (uint32_t*)dout, n, nullptr);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpy(out, dout, (size_t)n * 4, hipMemcpyDeviceToHost));
        HIPCHK(hipFree(din));
        HIPCHK(hipFree(dout));
    });
}


tigas_status tigas_server_create(tigas_context* ctx, const tigas_server_config* cfg, tigas_server** out) {
    return guard([&] {
        if (!ctx || !out) fail(TIGAS_E_INVALID, "null argument");
        HIPCHK(hipSetDevice(ctx->device));
        std::unique_ptr<tigas_server> sv(new tigas_server());
        sv->ctx = ctx;
        if (cfg) sv->cfg = *cfg;
        if (sv->cfg.slots <= 0) sv->cfg.slots = 2;
        if (sv->cfg.slots > 8) fail(TIGAS_E_INVALID, "at most 8 slots");
        if (sv->cfg.max_batch <= 0) sv->cfg.max_batch = 64;
        if (sv->cfg.tile_w == 0 && sv->cfg.tile_h == 0) {
            sv->cfg.tile_w = 16;
            sv->cfg.tile_h = 32;
        }
        tigas_quality q{};
        q.tile_w = sv->cfg.tile_w;
        q.tile_h = sv->cfg.tile_h;
        q.batch_depth = sv->cfg.batch_depth;
        const TileCfg tc = tile_cfg(&q);
        sv->cfg.batch_depth = tc.bd;
        // one pixel per lane: the faster blend for the mixed batches of the serving load
        if (sv->cfg.pixels_per_lane == 0) sv->cfg.pixels_per_lane = 1;
        sv->t0 = std::chrono::steady_clock::now();
        for (int i = 0; i < sv->cfg.slots; ++i) {
            std::unique_ptr<tigas_server::Slot> sl(new tigas_server::Slot());
            HIPCHK(hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking));
            sv->slots.push_back(std::move(sl));
        }
        if (sv->cfg.hbm_budget) {
            // reserve each slot's workspace for its whole share up front, so
            // serving never reallocates (a reallocation waits for the device)
            const size_t share = sv->cfg.hbm_budget / sv->slots.size();
            const uint64_t recs = share / (kBytesPerRecord + 5 * 24 + 1);
            for (auto& sl : sv->slots) {
                Workspace& ws = ctx->workspace(sl->stream);
                std::lock_guard<std::mutex> lk(ws.mu);
                ws.counters.ensure(sizeof(Counters));
                ws.ensure_records((uint32_t)std::min<uint64_t>(recs, 0x7f000000ull));
                ws.ensure_dups((uint32_t)std::min<uint64_t>(recs * 5, 0xfff00000ull));
                ws.ensure_views(sv->cfg.max_batch);
                ws.ensure_tiles((uint32_t)std::min<uint64_t>((uint64_t)sv->cfg.max_batch * 16384, 1u << 26));
            }
        }
        for (auto& sl : sv->slots) sl->th = std::thread(slot_main, sv.get(), sl.get());
        sv->dispatcher = std::thread(dispatcher_main, sv.get());
        *out = sv.release();
    });
}

void tigas_server_destroy(tigas_server* sv) {
    if (!sv) return;
    {
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->cv_done.wait(lk, [&] { return sv->finished >= sv->submitted; });
        sv->stop = true;
        sv->cv_sched.notify_all();
        sv->cv_slot.notify_all();
    }
    if (sv->dispatcher.joinable()) sv->dispatcher.join();
    for (auto& sl : sv->slots)
        if (sl->th.joinable()) sl->th.join();
    (void)hipSetDevice(sv->ctx->device);
    for (auto& sl : sv->slots) {
        {
            std::lock_guard<std::mutex> lk(sv->ctx->mu);
            sv->ctx->ws.erase(sl->stream);
        }
        (void)hipStreamDestroy(sl->stream);
    }
    delete sv;
}

tigas_status tigas_server_submit(tigas_server* sv, const tigas_request* r, int64_t* id) {
    return guard([&] {
        if (!sv) fail(TIGAS_E_INVALID, "null server");
        validate_request(sv, r);
        std::lock_guard<std::mutex> lk(sv->mu);
        const int64_t i = submit_locked(sv, r, sv->now());
        if (id) *id = i;
    });
}

tigas_status tigas_server_poll(tigas_server* sv, tigas_completion* out, int max, int* n) {
    return guard([&] {
        if (!sv || !n || (max > 0 && !out)) fail(TIGAS_E_INVALID, "null argument");
        std::lock_guard<std::mutex> lk(sv->mu);
        const int k = std::min<int>(max, (int)sv->completed.size());
        for (int i = 0; i < k; ++i) out[i] = sv->completed[i];
        sv->completed.erase(sv->completed.begin(), sv->completed.begin() + k);
        *n = k;
    });
}

tigas_status tigas_server_drain(tigas_server* sv) {
    return guard([&] {
        if (!sv) fail(TIGAS_E_INVALID, "null server");
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->cv_done.wait(lk, [&] { return sv->finished >= sv->submitted; });
    });
}

tigas_status tigas_server_replay(tigas_server* sv, const tigas_request* reqs, int n, tigas_completion* out) {
    return guard([&] {
        if (!sv || (n > 0 && (!reqs || !out))) fail(TIGAS_E_INVALID, "null argument");
        for (int i = 0; i < n; ++i) validate_request(sv, &reqs[i]);
        std::vector<int64_t> ids(n);
        const double base = sv->now();
        for (int i = 0; i < n; ++i) {
            const double t = base + reqs[i].arrival_s;
            // open loop: wait for the arrival time (sleep, then spin the last 200 us)
            for (;;) {
                const double left = t - sv->now();
                if (left <= 0) break;
                if (left > 3e-4) std::this_thread::sleep_for(std::chrono::duration<double>(left - 2e-4));
            }
            std::lock_guard<std::mutex> lk(sv->mu);
            ids[i] = submit_locked(sv, &reqs[i], t);
        }
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->cv_done.wait(lk, [&] { return sv->finished >= sv->submitted; });
        std::map<int64_t, tigas_completion> byid;
        for (const auto& c : sv->completed) byid[c.id] = c;
        std::vector<tigas_completion> rest;
        for (int i = 0; i < n; ++i) {
            auto it = byid.find(ids[i]);
            out[i] = it != byid.end() ? it->second : tigas_completion{};
            if (it != byid.end()) {
                out[i].arrival_s -= base;
                out[i].dispatch_s -= base;
                out[i].done_s -= base;
                byid.erase(it);
            }
        }
        for (const auto& kv : byid) rest.push_back(kv.second);
        sv->completed.swap(rest);
    });
}

tigas_status tigas_server_get_stats(tigas_server* sv, tigas_server_stats* out) {
    return guard([&] {
        if (!sv || !out) fail(TIGAS_E_INVALID, "null argument");
        std::lock_guard<std::mutex> lk(sv->mu);
        *out = sv->st;
        out->pending = (int64_t)sv->pending.size();
    });
}

}  // extern "C"
