// Host-only checks of the library's bookkeeping under the address and undefined-behaviour
// sanitizers: the server arena's first-fit allocator, and the C ABI's argument checks and
// workspace sizing (paths that return before any device call).  Exit status 0 = every check
// passed; a sanitizer report aborts with a nonzero status.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "arena_alloc.h"
#include "qlra.h"

static int failures = 0;
#define CHECK(cond)                                                          \
    do {                                                                     \
        if (!(cond)) {                                                       \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            failures++;                                                      \
        }                                                                    \
    } while (0)

static void arena_tests() {
    using qlra_impl::ArenaAlloc;
    // first fit, 256-byte granules, exhaustion
    ArenaAlloc a(4096);
    size_t o1, o2, o3, o4;
    CHECK(a.alloc(1, &o1) && o1 == 0);
    CHECK(a.alloc(300, &o2) && o2 == 256);
    CHECK(a.alloc(1024, &o3) && o3 == 768);
    CHECK(a.used() == 256 + 512 + 1024);
    CHECK(!a.alloc(4096, &o4));
    // a freed hole is reused first; neighbours merge back into one range
    a.release(o2, 300);
    CHECK(a.alloc(200, &o4) && o4 == 256);
    a.release(o4, 200);
    a.release(o1, 1);
    a.release(o3, 1024);
    CHECK(a.used() == 0);
    CHECK(a.alloc(4096, &o4) && o4 == 0);
    a.release(o4, 4096);
    // random traffic against a byte map of ownership
    std::mt19937_64 rng(7);
    const size_t cap = 1 << 20;
    ArenaAlloc b(cap);
    std::vector<int> owner(cap / 256, -1);
    std::vector<std::pair<size_t, size_t>> live;
    for (int it = 0; it < 20000; it++) {
        if (!live.empty() && (rng() % 3 == 0)) {
            const size_t i = rng() % live.size();
            const size_t off = live[i].first, bytes = live[i].second;
            for (size_t g = off / 256; g < (off + bytes + 255) / 256; g++) owner[g] = -1;
            b.release(off, bytes);
            live[i] = live.back();
            live.pop_back();
        } else {
            const size_t bytes = 1 + rng() % 40000;
            size_t off = 0;
            if (b.alloc(bytes, &off)) {
                CHECK(off % 256 == 0 && off + bytes <= cap);
                for (size_t g = off / 256; g < (off + bytes + 255) / 256; g++) {
                    CHECK(owner[g] == -1);
                    owner[g] = it;
                }
                live.emplace_back(off, bytes);
            }
        }
    }
    size_t used = 0;
    for (auto& l : live) used += (l.second + 255) & ~size_t(255);
    CHECK(b.used() == used);
    for (auto& l : live) b.release(l.first, l.second);
    CHECK(b.used() == 0);
    size_t o5;
    CHECK(b.alloc(cap, &o5) && o5 == 0);
}

static void abi_tests() {
    size_t bytes = 0;
    qlra_opts_t o;
    std::memset(&o, 0, sizeof(o));
    o.estimate_passes = 1;
    // sizes for the configurations and odd shapes, every scheme, precision and orientation
    const int64_t shapes[][2] = {{256, 256}, {2048, 2048}, {1024, 1536}, {16384, 16384}, {97, 61}, {1, 1}, {9, 1}};
    for (auto& s : shapes)
        for (int scheme = 0; scheme < 2; scheme++)
            for (int prec = 0; prec <= 4; prec++)
                for (int tr = 0; tr < 2; tr++)
                    for (int v = 2; v <= 8; v += 3) {
                        o.pass_precision = prec;
                        o.transpose = tr;
                        const int k = s[0] >= 128 && s[1] >= 128 ? 64 : 1, p = s[0] >= 128 && s[1] >= 128 ? 16 : 0;
                        CHECK(qlra_workspace_size(s[0], s[1], k, p, v, scheme, &o, &bytes) == QLRA_OK && bytes > 0);
                    }
    // argument errors (Sec. 4: k + p <= min(m, n); Alg. 2 / Alg. 4: v >= 2)
    CHECK(qlra_workspace_size(10, 8, 0, 2, 2, 0, nullptr, &bytes) == QLRA_E_ARG);
    CHECK(qlra_workspace_size(10, 8, 3, -1, 2, 0, nullptr, &bytes) == QLRA_E_ARG);
    CHECK(qlra_workspace_size(10, 8, 3, 2, 1, 0, nullptr, &bytes) == QLRA_E_ARG);
    CHECK(qlra_workspace_size(10, 8, 7, 2, 2, 0, nullptr, &bytes) == QLRA_E_ARG);
    CHECK(qlra_workspace_size(10, 8, 3, 2, 2, 5, nullptr, &bytes) == QLRA_E_ARG);
    CHECK(qlra_workspace_size(10, 8, 3, 2, 2, 0, nullptr, nullptr) == QLRA_E_ARG);
    o.pass_precision = 9;
    CHECK(qlra_workspace_size(100, 80, 3, 2, 2, 0, &o, &bytes) == QLRA_E_UNSUPPORTED);
    o.pass_precision = 0;
    // qlra(): argument and workspace errors return before any device call
    float dummy[16];
    double dd[16];
    CHECK(qlra(dummy, 100, 80, 80, 8000, 3, 2, 3, 0, 1, nullptr, dummy, 3, 300, dd, dummy, 3, 240, dd) == QLRA_E_ARG);
    CHECK(qlra(nullptr, 100, 80, 80, 8000, 3, 2, 3, 0, 1, &o, dummy, 3, 300, dd, dummy, 3, 240, dd) == QLRA_E_ARG);
    CHECK(qlra(dummy, 100, 80, 70, 8000, 3, 2, 3, 0, 1, &o, dummy, 3, 300, dd, dummy, 3, 240, dd) == QLRA_E_ARG);
    CHECK(qlra(dummy, 100, 80, 80, 8000, 3, 2, 3, 0, 1, &o, dummy, 2, 300, dd, dummy, 3, 240, dd) == QLRA_E_ARG);
    CHECK(qlra(dummy, 100, 80, 80, 8000, 3, 2, 3, 0, 1, &o, dummy, 3, 300, nullptr, dummy, 3, 240, dd) == QLRA_E_ARG);
    o.workspace = nullptr;
    o.workspace_bytes = 0;
    CHECK(qlra(dummy, 100, 80, 80, 8000, 3, 2, 3, 0, 1, &o, dummy, 3, 300, dd, dummy, 3, 240, dd) == QLRA_E_WORKSPACE);
    o.workspace = dummy;                                  // too small
    o.workspace_bytes = sizeof(dummy);
    CHECK(qlra(dummy, 100, 80, 80, 8000, 3, 2, 3, 0, 1, &o, dummy, 3, 300, dd, dummy, 3, 240, dd) == QLRA_E_WORKSPACE);
    // the other entry points' sizing and argument checks
    CHECK(qlra_cholqr_workspace_size(100, 20, &bytes) == QLRA_OK && bytes > 0);
    CHECK(qlra_cholqr_workspace_size(10, 20, &bytes) == QLRA_E_ARG);
    CHECK(qlra_qgemm_workspace_size(0, 300, 200, 60, &bytes) == QLRA_OK);
    CHECK(qlra_qgemm_workspace_size(1, 16384, 16384, 640, &bytes) == QLRA_OK);
    CHECK(qlra_qgemm_lp_workspace_size(0, QLRA_BF16, 300, 200, 160, &bytes) == QLRA_OK);
    CHECK(qlra_qgemm_split_workspace_size(1, QLRA_BF16, 300, 200, 640, &bytes) == QLRA_OK);
    CHECK(qlra_qsvd_workspace_size(97, &bytes) == QLRA_OK && bytes > 0);
    CHECK(qlra_complete_workspace_size(256, 256, 30, 10, 2, 0, 0.6, nullptr, &bytes) == QLRA_OK && bytes > 0);
    CHECK(qlra_complete_workspace_size(256, 256, 30, 10, 2, 0, 4.0, nullptr, &bytes) == QLRA_E_UNSUPPORTED);
    size_t lo = 0, lot = 0;
    CHECK(qlra_lowp_copy_bytes(129, 67, &lo, &lot) == QLRA_OK && lo > 0 && lot > 0);
    qlra_server_t* sv = nullptr;
    qlra_server_opts_t so;
    std::memset(&so, 0, sizeof(so));
    CHECK(qlra_server_create(&so, &sv) == QLRA_E_ARG && sv == nullptr);
    CHECK(qlra_server_create(nullptr, &sv) == QLRA_E_ARG);
    for (int st = -1; st <= 7; st++) CHECK(qlra_strerror(st) != nullptr);
}

int main() {
    arena_tests();
    abi_tests();
    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("host sanitizer checks passed\n");
    return 0;
}
