// registry.cpp -- the scene registry of the backend (Section 4.1, GPU
// Backend; Section 5.1, PLY Model and Primitives and Dynamic Multi-Model
// Runtime): discovery of the model folders under a root directory, parsing of
// a model's PLY file into the resident attribute layout, loading on first
// access, reference counts held while clients render a model, and unloading
// of models that stayed unreferenced for longer than an inactivity timeout.
// Host code only; the device work is the scene load of the rasterizer.
//
// PLY layout of a 3DGS model (the format written by the original 3DGS
// training code, Kerbl et al. 2023): one "vertex" element per Gaussian with
// the properties x y z (centre), f_dc_0..2 (SH degree-0 coefficient per
// colour channel), f_rest_0..K-1 (the higher coefficients, channel-major:
// f_rest_{c*(K/3) + k-1} is coefficient k of channel c), opacity (logit),
// scale_0..2 (log-scales) and rot_0..3 (quaternion w, x, y, z).  K is 0, 9,
// 24 or 45 for SH degree 0..3.  Other properties (normals) and elements are
// skipped.

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <filesystem>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "../../include/tigas.h"
#include "tigas_internal.h"

namespace fs = std::filesystem;

namespace {

struct RegError : std::runtime_error {
    tigas_status st;
    RegError(tigas_status s, const std::string& m) : std::runtime_error(m), st(s) {}
};
[[noreturn]] void rfail(tigas_status s, const std::string& m) { throw RegError(s, m); }

// a library call made from here failed and already left its own message
struct Passthrough {
    tigas_status st;
};

template <typename F>
tigas_status rguard(F&& f) {
    try {
        tigas::set_last_error("");
        f();
        return TIGAS_OK;
    } catch (const Passthrough& p) {
        return p.st;
    } catch (const RegError& e) {
        tigas::set_last_error(e.what());
        return e.st;
    } catch (const std::bad_alloc&) {
        tigas::set_last_error("host allocation failed");
        return TIGAS_E_OOM;
    } catch (const std::exception& e) {  // filesystem errors
        tigas::set_last_error(e.what());
        return TIGAS_E_INVALID;
    }
}

// ---------------------------------------------------------------- PLY ----

enum class PType { I8, U8, I16, U16, I32, U32, F32, F64 };

int ptype_size(PType t) {
    switch (t) {
        case PType::I8: case PType::U8: return 1;
        case PType::I16: case PType::U16: return 2;
        case PType::I32: case PType::U32: case PType::F32: return 4;
        default: return 8;
    }
}

bool parse_ptype(const std::string& s, PType* t) {
    static const std::pair<const char*, PType> names[] = {
        {"char", PType::I8},     {"int8", PType::I8},     {"uchar", PType::U8},   {"uint8", PType::U8},
        {"short", PType::I16},   {"int16", PType::I16},   {"ushort", PType::U16}, {"uint16", PType::U16},
        {"int", PType::I32},     {"int32", PType::I32},   {"uint", PType::U32},   {"uint32", PType::U32},
        {"float", PType::F32},   {"float32", PType::F32}, {"double", PType::F64}, {"float64", PType::F64}};
    for (const auto& n : names)
        if (s == n.first) {
            *t = n.second;
            return true;
        }
    return false;
}

enum class PlyFormat { Ascii, BinLE, BinBE };

struct PlyProp {
    std::string name;
    PType type = PType::F32;
    bool list = false;
    PType count_type = PType::U8;
    size_t offset = 0;  // within a record (elements without lists)
};

struct PlyElem {
    std::string name;
    int64_t count = 0;
    std::vector<PlyProp> props;
    size_t stride = 0;
    bool has_list = false;
};

struct PlyHeader {
    PlyFormat fmt = PlyFormat::BinLE;
    std::vector<PlyElem> elems;
};

// Properties of the vertex element that the scene layout takes, as indices
// into the element's property list.
struct VertexMap {
    int elem = -1;
    int64_t n = 0;
    int deg = 0;
    int xyz[3], dc[3], scale[3], rot[4], opacity;
    std::vector<int> rest;  // f_rest_0 .. f_rest_{K-1}
};

std::vector<std::string> split(const std::string& s) {
    std::vector<std::string> t;
    size_t i = 0;
    while (i < s.size()) {
        while (i < s.size() && (s[i] == ' ' || s[i] == '\t')) ++i;
        size_t j = i;
        while (j < s.size() && s[j] != ' ' && s[j] != '\t') ++j;
        if (j > i) t.push_back(s.substr(i, j - i));
        i = j;
    }
    return t;
}

struct File {
    FILE* f = nullptr;
    explicit File(const std::string& path) : f(std::fopen(path.c_str(), "rb")) {
        if (!f) rfail(TIGAS_E_INVALID, path + ": cannot open");
    }
    ~File() {
        if (f) std::fclose(f);
    }
};

PlyHeader read_header(FILE* f, const std::string& path) {
    constexpr size_t kMaxLine = 4096, kMaxHeader = 1 << 20;
    size_t total = 0;
    auto line = [&](std::string& s) {
        s.clear();
        for (;;) {
            const int c = std::fgetc(f);
            if (c == EOF) return false;
            if (++total > kMaxHeader) rfail(TIGAS_E_INVALID, path + ": PLY header too long");
            if (c == '\n') break;
            if (s.size() >= kMaxLine) rfail(TIGAS_E_INVALID, path + ": PLY header line too long");
            s.push_back((char)c);
        }
        if (!s.empty() && s.back() == '\r') s.pop_back();
        return true;
    };
    std::string s;
    if (!line(s) || s != "ply") rfail(TIGAS_E_INVALID, path + ": not a PLY file");
    PlyHeader h;
    bool have_format = false;
    for (;;) {
        if (!line(s)) rfail(TIGAS_E_INVALID, path + ": PLY header has no end_header");
        const std::vector<std::string> t = split(s);
        if (t.empty() || t[0] == "comment" || t[0] == "obj_info") continue;
        if (t[0] == "end_header") break;
        if (t[0] == "format") {
            if (t.size() != 3 || t[2] != "1.0") rfail(TIGAS_E_INVALID, path + ": unsupported PLY format line");
            if (t[1] == "ascii") h.fmt = PlyFormat::Ascii;
            else if (t[1] == "binary_little_endian") h.fmt = PlyFormat::BinLE;
            else if (t[1] == "binary_big_endian") h.fmt = PlyFormat::BinBE;
            else rfail(TIGAS_E_INVALID, path + ": unknown PLY format " + t[1]);
            have_format = true;
        } else if (t[0] == "element") {
            if (t.size() != 3) rfail(TIGAS_E_INVALID, path + ": bad element line");
            char* end = nullptr;
            const long long c = std::strtoll(t[2].c_str(), &end, 10);
            if (*end || c < 0) rfail(TIGAS_E_INVALID, path + ": bad element count");
            PlyElem e;
            e.name = t[1];
            e.count = c;
            h.elems.push_back(e);
        } else if (t[0] == "property") {
            if (h.elems.empty()) rfail(TIGAS_E_INVALID, path + ": property before any element");
            PlyProp p;
            if (t.size() == 5 && t[1] == "list") {
                if (!parse_ptype(t[2], &p.count_type) || !parse_ptype(t[3], &p.type))
                    rfail(TIGAS_E_INVALID, path + ": unknown property type");
                p.list = true;
                p.name = t[4];
            } else if (t.size() == 3) {
                if (!parse_ptype(t[1], &p.type)) rfail(TIGAS_E_INVALID, path + ": unknown property type " + t[1]);
                p.name = t[2];
            } else {
                rfail(TIGAS_E_INVALID, path + ": bad property line");
            }
            PlyElem& e = h.elems.back();
            for (const PlyProp& q : e.props)
                if (q.name == p.name) rfail(TIGAS_E_INVALID, path + ": duplicate property " + p.name);
            p.offset = e.stride;
            e.stride += p.list ? 0 : (size_t)ptype_size(p.type);
            e.has_list = e.has_list || p.list;
            e.props.push_back(p);
        } else {
            rfail(TIGAS_E_INVALID, path + ": unknown PLY header keyword " + t[0]);
        }
    }
    if (!have_format) rfail(TIGAS_E_INVALID, path + ": PLY header has no format line");
    return h;
}

VertexMap map_vertex(const PlyHeader& h, const std::string& path) {
    VertexMap m;
    for (size_t i = 0; i < h.elems.size(); ++i)
        if (h.elems[i].name == "vertex") {
            m.elem = (int)i;
            break;
        }
    if (m.elem < 0) rfail(TIGAS_E_INVALID, path + ": no vertex element");
    const PlyElem& e = h.elems[(size_t)m.elem];
    if (e.has_list) rfail(TIGAS_E_INVALID, path + ": list property in the vertex element");
    if (e.count > (int64_t)0x7f000000) rfail(TIGAS_E_INVALID, path + ": too many vertices");
    m.n = e.count;
    auto find = [&](const std::string& name) {
        for (size_t i = 0; i < e.props.size(); ++i)
            if (e.props[i].name == name) return (int)i;
        rfail(TIGAS_E_INVALID, path + ": vertex property " + name + " missing");
    };
    static const char* xyz[3] = {"x", "y", "z"};
    for (int c = 0; c < 3; ++c) {
        m.xyz[c] = find(xyz[c]);
        m.dc[c] = find("f_dc_" + std::to_string(c));
        m.scale[c] = find("scale_" + std::to_string(c));
    }
    for (int c = 0; c < 4; ++c) m.rot[c] = find("rot_" + std::to_string(c));
    m.opacity = find("opacity");
    int k = 0;
    for (const PlyProp& p : e.props)
        if (p.name.compare(0, 7, "f_rest_") == 0) ++k;
    m.deg = k == 0 ? 0 : k == 9 ? 1 : k == 24 ? 2 : k == 45 ? 3 : -1;
    if (m.deg < 0) rfail(TIGAS_E_INVALID, path + ": " + std::to_string(k) + " f_rest properties (0, 9, 24 or 45 expected)");
    for (int j = 0; j < k; ++j) m.rest.push_back(find("f_rest_" + std::to_string(j)));
    return m;
}

double decode(const unsigned char* p, PType t, bool swap) {
    unsigned char b[8];
    const int n = ptype_size(t);
    for (int i = 0; i < n; ++i) b[i] = swap ? p[n - 1 - i] : p[i];
    switch (t) {
        case PType::I8: { int8_t v; std::memcpy(&v, b, 1); return v; }
        case PType::U8: return b[0];
        case PType::I16: { int16_t v; std::memcpy(&v, b, 2); return v; }
        case PType::U16: { uint16_t v; std::memcpy(&v, b, 2); return v; }
        case PType::I32: { int32_t v; std::memcpy(&v, b, 4); return v; }
        case PType::U32: { uint32_t v; std::memcpy(&v, b, 4); return v; }
        case PType::F32: { float v; std::memcpy(&v, b, 4); return v; }
        default: { double v; std::memcpy(&v, b, 8); return v; }
    }
}

// Whitespace-separated tokens of an ASCII body.
struct Tokens {
    FILE* f;
    const std::string& path;
    std::string tok;
    const std::string& next() {
        tok.clear();
        int c;
        do c = std::fgetc(f);
        while (c == ' ' || c == '\t' || c == '\n' || c == '\r');
        while (c != EOF && c != ' ' && c != '\t' && c != '\n' && c != '\r') {
            tok.push_back((char)c);
            c = std::fgetc(f);
        }
        if (tok.empty()) rfail(TIGAS_E_INVALID, path + ": file ends before the last element");
        return tok;
    }
    double number() {
        const std::string& s = next();
        char* end = nullptr;
        const double v = std::strtod(s.c_str(), &end);
        if (*end) rfail(TIGAS_E_INVALID, path + ": bad number " + s);
        return v;
    }
};

// Destination of the scene attributes: host arrays in the layout of
// tigas_scene_desc.
struct SceneArrays {
    float *means, *log_scales, *quats, *opacity, *sh;
};

// Writes the attributes of vertex i from its property values.
template <typename Get>
void store_vertex(const VertexMap& m, int64_t i, Get&& get, const SceneArrays& out) {
    for (int c = 0; c < 3; ++c) {
        out.means[i * 3 + c] = (float)get(m.xyz[c]);
        out.log_scales[i * 3 + c] = (float)get(m.scale[c]);
    }
    for (int c = 0; c < 4; ++c) out.quats[i * 4 + c] = (float)get(m.rot[c]);
    out.opacity[i] = (float)get(m.opacity);
    float* sh = out.sh + i * 48;
    std::fill(sh, sh + 48, 0.0f);
    for (int c = 0; c < 3; ++c) sh[c] = (float)get(m.dc[c]);
    const int per = (int)m.rest.size() / 3;  // coefficients above degree 0, per channel
    for (int c = 0; c < 3; ++c)
        for (int k = 1; k <= per; ++k) sh[k * 3 + c] = (float)get(m.rest[(size_t)(c * per + k - 1)]);
}

void read_body(FILE* f, const PlyHeader& h, const VertexMap& m, const std::string& path, const SceneArrays& out) {
    const bool swap = h.fmt == PlyFormat::BinBE;
    if (h.fmt == PlyFormat::Ascii) {
        Tokens tk{f, path, {}};
        for (int ei = 0; ei < m.elem; ++ei) {  // elements before the vertices
            const PlyElem& e = h.elems[(size_t)ei];
            for (int64_t r = 0; r < e.count; ++r)
                for (const PlyProp& p : e.props) {
                    const double c = p.list ? tk.number() : 1.0;
                    if (c < 0 || c != (double)(int64_t)c) rfail(TIGAS_E_INVALID, path + ": bad list length");
                    for (int64_t j = 0; j < (int64_t)c; ++j) tk.next();
                }
        }
        const PlyElem& e = h.elems[(size_t)m.elem];
        std::vector<double> vals(e.props.size());
        for (int64_t i = 0; i < m.n; ++i) {
            for (size_t j = 0; j < vals.size(); ++j) vals[j] = tk.number();
            store_vertex(m, i, [&](int j) { return vals[(size_t)j]; }, out);
        }
        return;
    }
    for (int ei = 0; ei < m.elem; ++ei) {
        const PlyElem& e = h.elems[(size_t)ei];
        if (!e.has_list) {
            if (e.count && std::fseek(f, (long)(e.stride * (size_t)e.count), SEEK_CUR) != 0)
                rfail(TIGAS_E_INVALID, path + ": file ends before the vertices");
            continue;
        }
        unsigned char b[8];
        for (int64_t r = 0; r < e.count; ++r)
            for (const PlyProp& p : e.props) {
                int64_t items = 1;
                if (p.list) {
                    const int cs = ptype_size(p.count_type);
                    if (std::fread(b, 1, (size_t)cs, f) != (size_t)cs)
                        rfail(TIGAS_E_INVALID, path + ": file ends before the vertices");
                    const double c = decode(b, p.count_type, swap);
                    if (c < 0) rfail(TIGAS_E_INVALID, path + ": bad list length");
                    items = (int64_t)c;
                }
                if (items && std::fseek(f, (long)(items * ptype_size(p.type)), SEEK_CUR) != 0)
                    rfail(TIGAS_E_INVALID, path + ": file ends before the vertices");
            }
    }
    const PlyElem& e = h.elems[(size_t)m.elem];
    const size_t stride = e.stride;
    // FP32 properties in the host's byte order are copied as they are
    std::vector<char> plain(e.props.size());
    for (size_t j = 0; j < e.props.size(); ++j) plain[j] = e.props[j].type == PType::F32 && !swap;
    // records are read in chunks and decoded by up to 16 host threads
    constexpr int64_t kChunk = 1 << 20, kPerThread = 1 << 15;
    const int64_t hw = std::max<int64_t>(1, (int64_t)std::thread::hardware_concurrency());
    std::vector<unsigned char> buf((size_t)std::min<int64_t>(std::max<int64_t>(m.n, 1), kChunk) * stride);
    for (int64_t i0 = 0; i0 < m.n; i0 += kChunk) {
        const int64_t cnt = std::min(kChunk, m.n - i0);
        if (std::fread(buf.data(), stride, (size_t)cnt, f) != (size_t)cnt)
            rfail(TIGAS_E_INVALID, path + ": file ends before the last vertex");
        auto decode_range = [&](int64_t r0, int64_t r1) {
            for (int64_t r = r0; r < r1; ++r) {
                const unsigned char* rec = buf.data() + (size_t)r * stride;
                store_vertex(m, i0 + r,
                             [&](int j) -> double {
                                 const PlyProp& p = e.props[(size_t)j];
                                 if (plain[(size_t)j]) {
                                     float v;
                                     std::memcpy(&v, rec + p.offset, 4);
                                     return v;
                                 }
                                 return decode(rec + p.offset, p.type, swap);
                             },
                             out);
            }
        };
        const int64_t nt = std::min<int64_t>({16, hw, (cnt + kPerThread - 1) / kPerThread});
        if (nt <= 1) {
            decode_range(0, cnt);
            continue;
        }
        std::vector<std::thread> pool;
        pool.reserve((size_t)nt);
        const int64_t per = (cnt + nt - 1) / nt;
        int64_t started = 0;  // records handed to threads
        try {
            for (int64_t t = 0; t < nt; ++t) {
                const int64_t r0 = t * per, r1 = std::min(cnt, r0 + per);
                if (r0 < r1) pool.emplace_back(decode_range, r0, r1);
                started = r1;
            }
        } catch (const std::system_error&) {
            // no more threads: this one decodes the rest
        }
        if (started < cnt) decode_range(started, cnt);
        for (std::thread& th : pool) th.join();
    }
}

// Header of a model file: vertex count and SH degree.
void ply_info(const std::string& path, int64_t* n, int* deg) {
    File f(path);
    const PlyHeader h = read_header(f.f, path);
    const VertexMap m = map_vertex(h, path);
    *n = m.n;
    *deg = m.deg;
}

void ply_read(const std::string& path, int64_t n, const SceneArrays& out, int* deg) {
    File f(path);
    const PlyHeader h = read_header(f.f, path);
    const VertexMap m = map_vertex(h, path);
    if (m.n != n) rfail(TIGAS_E_INVALID, path + ": holds " + std::to_string(m.n) + " vertices, not " + std::to_string(n));
    read_body(f.f, h, m, path, out);
    if (deg) *deg = m.deg;
}

// -------------------------------------------------------------- models ----

using Clock = std::chrono::steady_clock;

enum class State { Unloaded, Loading, Loaded };

struct Model {
    std::string id, ply, preview;
    int64_t n = 0;
    int deg = 0;
    tigas_scene* scene = nullptr;
    State state = State::Unloaded;
    int refs = 0;
    int64_t loads = 0;
    Clock::time_point last_use{};
};

// The PLY file of a model folder: point_cloud.ply in it, else the one of the
// highest point_cloud/iteration_<k>/ (the layout of 3DGS training outputs),
// else the first *.ply directly in it by name.
std::string model_ply(const fs::path& dir) {
    std::error_code ec;
    if (fs::is_regular_file(dir / "point_cloud.ply", ec)) return (dir / "point_cloud.ply").string();
    long best = -1;
    std::string best_path;
    if (fs::is_directory(dir / "point_cloud", ec))
        for (const auto& it : fs::directory_iterator(dir / "point_cloud", ec)) {
            const std::string name = it.path().filename().string();
            if (name.compare(0, 10, "iteration_") != 0) continue;
            char* end = nullptr;
            const long k = std::strtol(name.c_str() + 10, &end, 10);
            if (*end || name.size() == 10) continue;
            const fs::path p = it.path() / "point_cloud.ply";
            if (k > best && fs::is_regular_file(p, ec)) {
                best = k;
                best_path = p.string();
            }
        }
    if (best >= 0) return best_path;
    std::vector<std::string> plys;
    for (const auto& it : fs::directory_iterator(dir, ec))
        if (it.path().extension() == ".ply" && fs::is_regular_file(it.path(), ec)) plys.push_back(it.path().string());
    std::sort(plys.begin(), plys.end());
    return plys.empty() ? std::string() : plys[0];
}

std::string preview_image(const fs::path& dir, const std::string& stem) {
    std::error_code ec;
    for (const char* ext : {".png", ".jpg", ".jpeg", ".webp"}) {
        const fs::path p = dir / (stem + ext);
        if (fs::is_regular_file(p, ec)) return p.string();
    }
    return std::string();
}

}  // namespace

struct tigas_registry {
    tigas_context* ctx = nullptr;
    tigas_registry_config cfg{};
    std::vector<Model> models;  // fixed at creation, sorted by id
    std::mutex mu;
    std::condition_variable cv;  // loads finishing, shutdown
    bool stop = false;
    std::thread sweeper;

    Model& find(const char* id) {
        if (!id) rfail(TIGAS_E_INVALID, "model id is null");
        for (Model& m : models)
            if (m.id == id) return m;
        rfail(TIGAS_E_INVALID, std::string("no model with id ") + id);
    }

    // Loads m (unloaded, marked Loading by the caller) outside the lock; the
    // file's vertex count and degree as read now come back in n and deg.
    tigas_scene* load(const Model& m, int64_t& n, int& deg) {
        ply_info(m.ply, &n, &deg);
        std::vector<float> means((size_t)n * 3), ls((size_t)n * 3), q((size_t)n * 4), op((size_t)n), sh((size_t)n * 48);
        ply_read(m.ply, n, SceneArrays{means.data(), ls.data(), q.data(), op.data(), sh.data()}, &deg);
        tigas_scene_desc d{};
        d.n = n;
        d.sh_degree = deg;
        d.means = means.data();
        d.log_scales = ls.data();
        d.quats_wxyz = q.data();
        d.opacity_logits = op.data();
        d.sh = sh.data();
        d.is_device = 0;
        d.storage = cfg.storage;
        tigas_scene* s = nullptr;
        const tigas_status st = tigas_scene_load(ctx, &d, &s);
        if (st != TIGAS_OK) throw Passthrough{st};
        return s;
    }

    // Makes m resident (loading it if needed); with `ref` takes a reference.
    tigas_scene* get(Model& m, bool ref) {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return m.state != State::Loading; });
        if (m.state == State::Unloaded) {
            m.state = State::Loading;
            lk.unlock();
            tigas_scene* s = nullptr;
            int64_t n = 0;
            int deg = 0;
            try {
                s = load(m, n, deg);
            } catch (...) {
                lk.lock();
                m.state = State::Unloaded;
                cv.notify_all();
                throw;
            }
            lk.lock();
            m.scene = s;
            m.state = State::Loaded;
            m.n = n;
            m.deg = deg;
            ++m.loads;
            cv.notify_all();
        }
        if (ref) ++m.refs;
        m.last_use = Clock::now();
        return m.scene;
    }

    // Unloads the resident models without references that were last used at
    // least the idle timeout ago (none when the timeout is negative).
    int evict() {
        std::vector<tigas_scene*> drop;
        {
            std::lock_guard<std::mutex> lk(mu);
            const Clock::time_point now = Clock::now();
            for (Model& m : models) {
                if (m.state != State::Loaded || m.refs != 0) continue;
                const double idle = std::chrono::duration<double>(now - m.last_use).count();
                if (cfg.idle_timeout_s < 0.0 || idle < cfg.idle_timeout_s) continue;
                drop.push_back(m.scene);
                m.scene = nullptr;
                m.state = State::Unloaded;
            }
        }
        for (tigas_scene* s : drop) tigas_scene_free(s);
        return (int)drop.size();
    }

    void sweep_loop() {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            const auto until = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                                  std::chrono::duration<double>(cfg.sweep_period_s));
            if (cv.wait_until(lk, until, [&] { return stop; })) return;
            lk.unlock();
            evict();
            lk.lock();
        }
    }
};

extern "C" {

tigas_status tigas_ply_info(const char* path, int64_t* n, int* sh_degree) {
    return rguard([&] {
        if (!path || !n || !sh_degree) rfail(TIGAS_E_INVALID, "null argument");
        ply_info(path, n, sh_degree);
    });
}

tigas_status tigas_ply_read(const char* path, int64_t n, float* means, float* log_scales, float* quats_wxyz,
                            float* opacity_logits, float* sh) {
    return rguard([&] {
        if (!path) rfail(TIGAS_E_INVALID, "path is null");
        if (n < 0) rfail(TIGAS_E_INVALID, "n < 0");
        if (n > 0 && (!means || !log_scales || !quats_wxyz || !opacity_logits || !sh))
            rfail(TIGAS_E_INVALID, "output array is null");
        ply_read(path, n, SceneArrays{means, log_scales, quats_wxyz, opacity_logits, sh}, nullptr);
    });
}

void tigas_registry_default_config(tigas_registry_config* cfg) {
    if (!cfg) return;
    cfg->idle_timeout_s = 300.0;
    cfg->sweep_period_s = 0.0;
    cfg->storage = TIGAS_ATTR_F32;
}

tigas_status tigas_registry_create(tigas_context* ctx, const char* root, const tigas_registry_config* cfg,
                                   tigas_registry** out) {
    return rguard([&] {
        if (!root || !out) rfail(TIGAS_E_INVALID, "null argument");
        *out = nullptr;
        std::unique_ptr<tigas_registry> r(new tigas_registry());
        r->ctx = ctx;
        tigas_registry_default_config(&r->cfg);
        if (cfg) r->cfg = *cfg;
        if (r->cfg.storage < TIGAS_ATTR_F32 || r->cfg.storage > TIGAS_ATTR_BF16) rfail(TIGAS_E_INVALID, "unknown storage");
        if (!(r->cfg.sweep_period_s >= 0.0) || r->cfg.sweep_period_s > 1e6 || r->cfg.idle_timeout_s != r->cfg.idle_timeout_s)
            rfail(TIGAS_E_INVALID, "sweep period must be in [0, 1e6] s and the idle timeout a number");
        const fs::path dir(root);
        if (!fs::is_directory(dir)) rfail(TIGAS_E_INVALID, std::string(root) + ": not a directory");
        std::map<std::string, Model> found;
        std::vector<fs::path> entries;
        for (const auto& it : fs::directory_iterator(dir)) entries.push_back(it.path());
        std::sort(entries.begin(), entries.end());
        // folders first, then PLY files directly under the root; the first
        // entry with a given id wins
        for (int pass = 0; pass < 2; ++pass)
            for (const fs::path& p : entries) {
                std::error_code ec;
                Model m;
                if (pass == 0 && fs::is_directory(p, ec)) {
                    m.id = p.filename().string();
                    m.ply = model_ply(p);
                    m.preview = preview_image(p, "preview");
                } else if (pass == 1 && p.extension() == ".ply" && fs::is_regular_file(p, ec)) {
                    m.id = p.stem().string();
                    m.ply = p.string();
                    m.preview = preview_image(dir, m.id);
                } else {
                    continue;
                }
                if (m.ply.empty() || m.id.empty() || found.count(m.id)) continue;
                try {
                    ply_info(m.ply, &m.n, &m.deg);
                } catch (const RegError&) {
                    continue;  // no readable 3DGS header: not a model
                }
                found.emplace(m.id, m);
            }
        for (auto& kv : found) r->models.push_back(kv.second);
        if (r->cfg.sweep_period_s > 0.0) {
            tigas_registry* rp = r.get();
            r->sweeper = std::thread([rp] { rp->sweep_loop(); });
        }
        *out = r.release();
    });
}

void tigas_registry_destroy(tigas_registry* r) {
    if (!r) return;
    {
        std::lock_guard<std::mutex> lk(r->mu);
        r->stop = true;
    }
    r->cv.notify_all();
    if (r->sweeper.joinable()) r->sweeper.join();
    for (Model& m : r->models)
        if (m.scene) tigas_scene_free(m.scene);
    delete r;
}

int64_t tigas_registry_count(const tigas_registry* r) { return r ? (int64_t)r->models.size() : 0; }

tigas_status tigas_registry_info(tigas_registry* r, int64_t index, tigas_model_info* info) {
    return rguard([&] {
        if (!r || !info) rfail(TIGAS_E_INVALID, "null argument");
        if (index < 0 || index >= (int64_t)r->models.size()) rfail(TIGAS_E_INVALID, "model index out of range");
        std::lock_guard<std::mutex> lk(r->mu);
        const Model& m = r->models[(size_t)index];
        info->id = m.id.c_str();
        info->ply_path = m.ply.c_str();
        info->preview_path = m.preview.c_str();
        info->n = m.n;
        info->sh_degree = m.deg;
        info->loaded = m.state == State::Loaded ? 1 : 0;
        info->refs = m.refs;
        info->loads = m.loads;
        info->device_bytes = m.state == State::Loaded ? tigas_scene_bytes(m.scene) : 0;
        info->idle_s = m.state == State::Loaded ? std::chrono::duration<double>(Clock::now() - m.last_use).count() : 0.0;
    });
}

tigas_status tigas_registry_acquire(tigas_registry* r, const char* id, tigas_scene** out) {
    return rguard([&] {
        if (!r || !out) rfail(TIGAS_E_INVALID, "null argument");
        *out = nullptr;
        if (!r->ctx) rfail(TIGAS_E_INVALID, "registry has no context (discovery only)");
        *out = r->get(r->find(id), true);
    });
}

tigas_status tigas_registry_load(tigas_registry* r, const char* id) {
    return rguard([&] {
        if (!r) rfail(TIGAS_E_INVALID, "null argument");
        if (!r->ctx) rfail(TIGAS_E_INVALID, "registry has no context (discovery only)");
        r->get(r->find(id), false);
    });
}

tigas_status tigas_registry_release(tigas_registry* r, tigas_scene* scene) {
    return rguard([&] {
        if (!r || !scene) rfail(TIGAS_E_INVALID, "null argument");
        std::lock_guard<std::mutex> lk(r->mu);
        for (Model& m : r->models)
            if (m.state == State::Loaded && m.scene == scene) {
                if (m.refs == 0) rfail(TIGAS_E_INVALID, "scene released more often than acquired");
                --m.refs;
                m.last_use = Clock::now();
                return;
            }
        rfail(TIGAS_E_INVALID, "scene is not a resident model of this registry");
    });
}

tigas_status tigas_registry_evict_idle(tigas_registry* r, int* evicted) {
    return rguard([&] {
        if (!r) rfail(TIGAS_E_INVALID, "null argument");
        const int k = r->evict();
        if (evicted) *evicted = k;
    });
}

}  // extern "C"
