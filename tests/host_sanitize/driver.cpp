// Host-only driver for the sanitizer build of libtigas: runs the PLY reader
// over every file named on the command line (valid, truncated, malformed or
// randomly corrupted), a discovery-only scene registry over a directory, and
// latency-ABR controllers over seeded random observations.  No GPU call is
// made.  Prints one line per file; the sanitizers abort on any error they
// find.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "../../include/tigas.h"

int main(int argc, char** argv) {
    if (argc < 2) {
        std::fprintf(stderr, "usage: driver REGISTRY_ROOT [PLY ...]\n");
        return 2;
    }
    int ok = 0, rejected = 0;
    for (int i = 2; i < argc; ++i) {
        int64_t n = 0;
        int deg = 0;
        if (tigas_ply_info(argv[i], &n, &deg) != TIGAS_OK) {
            ++rejected;
            std::printf("info rejected %s: %s\n", argv[i], tigas_last_error());
            continue;
        }
        if (n > (int64_t)1 << 22) {  // a corrupted count: do not allocate for it
            ++rejected;
            continue;
        }
        const size_t m = (size_t)(n > 0 ? n : 1);
        std::vector<float> means(m * 3), ls(m * 3), q(m * 4), op(m), sh(m * 48);
        const tigas_status s = tigas_ply_read(argv[i], n, means.data(), ls.data(), q.data(), op.data(), sh.data());
        if (s == TIGAS_OK) ++ok; else ++rejected;
        std::printf("read %s: n=%lld deg=%d status=%d\n", argv[i], (long long)n, deg, (int)s);
    }
    // discovery-only registry (no context): scan, list, destroy
    tigas_registry_config rc;
    tigas_registry_default_config(&rc);
    tigas_registry* reg = nullptr;
    if (tigas_registry_create(nullptr, argv[1], &rc, &reg) == TIGAS_OK) {
        const int64_t cnt = tigas_registry_count(reg);
        for (int64_t k = 0; k < cnt; ++k) {
            tigas_model_info mi;
            if (tigas_registry_info(reg, k, &mi) == TIGAS_OK) std::printf("model %s n=%lld\n", mi.id, (long long)mi.n);
        }
        tigas_scene* sc = nullptr;
        if (cnt > 0) {
            tigas_model_info mi;
            tigas_registry_info(reg, 0, &mi);
            std::printf("acquire without a context: status %d\n", (int)tigas_registry_acquire(reg, mi.id, &sc));
        }
        tigas_registry_destroy(reg);
    }
    // latency-ABR controllers over random observations, and invalid configurations
    std::mt19937_64 rng(7);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    for (int c = 0; c < 64; ++c) {
        tigas_abr_config cfg;
        tigas_abr_default_config(&cfg);
        cfg.history = 1 + (int)(u(rng) * 64);
        cfg.hold = 1 + (int)(u(rng) * 5);
        cfg.n_levels = 1 + (int)(u(rng) * 8);
        for (int l = 0; l < 8; ++l) cfg.expected_bytes[l] = 1000.0 * (l + 1) * (1.0 + u(rng));
        tigas_abr* abr = nullptr;
        if (tigas_abr_create(&cfg, &abr) != TIGAS_OK) continue;
        int level = 0;
        for (int r = 0; r < 500; ++r)
            tigas_abr_observe(abr, 1.0 + u(rng) * 3e5, 1e-4 + u(rng) * 0.5, u(rng) < 0.1, &level);
        double rate = 0.0;
        tigas_abr_rate(abr, &rate);
        tigas_abr_destroy(abr);
    }
    tigas_abr_config bad;
    tigas_abr_default_config(&bad);
    bad.n_levels = 9;
    tigas_abr* none = nullptr;
    std::printf("invalid ABR config: status %d\n", (int)tigas_abr_create(&bad, &none));
    std::printf("files read %d, rejected %d\n", ok, rejected);
    return 0;
}
