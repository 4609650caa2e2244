// Host-side checks of librmrcm run under AddressSanitizer and
// UndefinedBehaviorSanitizer (the library's host code instrumented, its
// kernels as built): argument validation, the geometry and level tables of
// many decompositions (through the memory plan, which builds every table
// and counts every array without a device), the weight-file parser on
// malformed files, and the status codes.  Without a GPU every call that
// passes validation stops at the device query with RMRCM_EDEVICE.
// Prints one line per failed expectation; exit status = number of failures.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rmrcm.h"

static int failures = 0, checks = 0;

static void expect(bool ok, const std::string& what) {
    ++checks;
    if (!ok) {
        ++failures;
        std::printf("FAIL %s\n", what.c_str());
    }
}

static rmrcm_params geometry(int nx, int ny, int bx, int by, int seg, int precision) {
    rmrcm_params p;
    rmrcm_default_params(&p);
    p.nx = nx, p.ny = ny, p.sub_nx = bx, p.sub_ny = by, p.seg = seg, p.precision = precision;
    return p;
}

static void plan_sweep() {
    const int sizes[] = {8, 16, 24, 32, 64, 96, 128, 256, 1024};
    const int subs[] = {4, 6, 8, 12, 16, 32, 64};
    const int segs[] = {1, 2, 3, 4, 8};
    int valid = 0;
    for (int nx : sizes)
        for (int ny : {nx, nx / 2 > 0 ? nx / 2 : 1, 2 * nx})
            for (int bx : subs)
                for (int by : {bx, 2 * bx})
                    for (int seg : segs)
                        for (int prec : {0, 1, 3}) {
                            rmrcm_params p = geometry(nx, ny, bx, by, seg, prec);
                            uint64_t b = 7;
                            const int r = rmrcm_plan_bytes(&p, &b);
                            const std::string tag = "plan " + std::to_string(nx) + "x" + std::to_string(ny) +
                                                    " sub " + std::to_string(bx) + "x" + std::to_string(by) +
                                                    " seg " + std::to_string(seg) + " prec " +
                                                    std::to_string(prec);
                            expect(r == RMRCM_OK || r == RMRCM_EINVAL || r == RMRCM_ENOTSUP, tag + " status");
                            expect(r == RMRCM_OK ? b > 0 : b == 0, tag + " bytes");
                            valid += r == RMRCM_OK;
                        }
    // one large decomposition: 8192^2 cells, 32^2 subdomains, 16 levels
    {
        rmrcm_params p = geometry(8192, 8192, 32, 32, 8, 0);
        uint64_t b = 0;
        expect(rmrcm_plan_bytes(&p, &b) == RMRCM_OK && b > ((uint64_t)25 << 30), "plan 8192^2");
    }
    expect(valid > 100, "plan sweep has valid geometries");
    std::printf("plan sweep: %d valid geometries\n", valid);
    rmrcm_params p = geometry(64, 64, 16, 16, 4, RMRCM_MIXED_LEARNED);
    uint64_t b = 0;
    expect(rmrcm_plan_bytes(&p, &b) == RMRCM_EINVAL, "learned without weights");
    expect(rmrcm_plan_bytes(nullptr, &b) == RMRCM_EINVAL, "plan null params");
    p = geometry(64, 64, 16, 16, 4, 0);
    expect(rmrcm_plan_bytes(&p, nullptr) == RMRCM_EINVAL, "plan null out");
    p.alpha = std::nan("");
    expect(rmrcm_plan_bytes(&p, &b) == RMRCM_EINVAL, "plan alpha nan");
}

static void setup_validation(bool have_gpu) {
    const int n = 64;
    std::vector<double> K(n * n, 1.0);
    std::vector<int8_t> t(4 * n, RMRCM_BC_NEUMANN);
    for (int j = 0; j < n; ++j) t[j] = t[n + j] = RMRCM_BC_DIRICHLET;
    rmrcm_params p = geometry(n, n, 16, 16, 4, 0);
    rmrcm_ctx* c = nullptr;
    expect(rmrcm_setup(&p, K.data(), t.data(), nullptr) == RMRCM_EINVAL, "setup null out");
    expect(rmrcm_setup(&p, nullptr, t.data(), &c) == RMRCM_EINVAL, "setup null perm");
    expect(rmrcm_setup(&p, K.data(), nullptr, &c) == RMRCM_EINVAL, "setup null bc");
    uint64_t need = 0;
    expect(rmrcm_plan_bytes(&p, &need) == RMRCM_OK, "plan");
    p.mem_cap = need - 1;
    expect(rmrcm_setup(&p, K.data(), t.data(), &c) == RMRCM_ENOMEM && !c, "setup over the cap");
    p.mem_cap = 0;
    if (have_gpu) return;   // below: every call reaches the device query
    t[5] = 7;
    expect(rmrcm_setup(&p, K.data(), t.data(), &c) == RMRCM_EDEVICE, "device query first");
    t[5] = RMRCM_BC_DIRICHLET;
    expect(rmrcm_setup(&p, K.data(), t.data(), &c) == RMRCM_EDEVICE && !c, "setup without a device");
    std::vector<double> src(n * n, 0.0), bv(4 * n, 0.0), pr(n * n), fl(4 * n * n);
    expect(rmrcm_step_noalloc(&p, K.data(), t.data(), src.data(), bv.data(), pr.data(), fl.data(), nullptr) ==
               RMRCM_EDEVICE,
           "noalloc without a device");
    rmrcm_params m = p;
    m.precision = RMRCM_MIXED;
    expect(rmrcm_step_noalloc(&m, K.data(), t.data(), src.data(), bv.data(), pr.data(), fl.data(), nullptr) ==
               RMRCM_ENOTSUP,
           "noalloc mixed");
    expect(rmrcm_step_noalloc(&p, nullptr, t.data(), src.data(), bv.data(), pr.data(), fl.data(), nullptr) ==
               RMRCM_EINVAL,
           "noalloc null perm");
}

static void context_nulls() {
    char buf[64];
    int64_t a = 0, b = 0;
    expect(rmrcm_get_stats(nullptr, buf, sizeof buf) == RMRCM_EINVAL, "stats null");
    expect(rmrcm_counts(nullptr, &a, &b) == RMRCM_EINVAL, "counts null");
    expect(rmrcm_set_stream(nullptr, nullptr) == RMRCM_EINVAL, "stream null");
    expect(rmrcm_set_refinement(nullptr, 1e-12, 3) == RMRCM_EINVAL, "refinement null");
    expect(rmrcm_solve(nullptr, nullptr, nullptr, nullptr, nullptr) == RMRCM_EINVAL, "solve null");
    expect(rmrcm_sync(nullptr) == RMRCM_EINVAL, "sync null");
    rmrcm_destroy(nullptr);
    rmrcm_batch_destroy(nullptr);
    rmrcm_cnn_destroy(nullptr);
    rmrcm_batch* bt = nullptr;
    expect(rmrcm_batch_create(0, nullptr, nullptr, nullptr, 0, &bt) == RMRCM_EINVAL, "batch of none");
}

static void weight_files(const std::string& dir, bool have_gpu) {
    auto write = [&](const std::string& name, const std::vector<char>& bytes) {
        const std::string path = dir + "/" + name;
        FILE* f = std::fopen(path.c_str(), "wb");
        if (f) {
            if (!bytes.empty()) std::fwrite(bytes.data(), 1, bytes.size(), f);
            std::fclose(f);
        }
        return path;
    };
    auto header = [](int32_t S, int32_t C, int32_t L, int32_t R, int64_t np) {
        std::vector<char> v(8 + 16 + 8);
        std::memcpy(v.data(), "RMRCMCNN", 8);
        const int32_t h[4] = {S, C, L, R};
        std::memcpy(v.data() + 8, h, 16);
        std::memcpy(v.data() + 24, &np, 8);
        return v;
    };
    rmrcm_cnn* net = nullptr;
    expect(rmrcm_cnn_load((dir + "/missing.bin").c_str(), 8, 0, &net) == RMRCM_EINVAL, "no file");
    expect(rmrcm_cnn_load(write("empty.bin", {}).c_str(), 8, 0, &net) == RMRCM_EINVAL, "empty file");
    std::vector<char> bad = header(16, 16, 5, 16, 10);
    bad[0] = 'X';
    expect(rmrcm_cnn_load(write("magic.bin", bad).c_str(), 8, 0, &net) == RMRCM_EINVAL, "bad magic");
    for (int64_t np : {(int64_t)-1, (int64_t)0, (int64_t)1 << 40}) {
        expect(rmrcm_cnn_load(write("np.bin", header(16, 16, 5, 16, np)).c_str(), 8, 0, &net) == RMRCM_EINVAL,
               "absurd parameter count " + std::to_string(np));
    }
    std::vector<char> trunc = header(16, 16, 5, 16, 1000);
    trunc.resize(trunc.size() + 999 * 4);
    expect(rmrcm_cnn_load(write("trunc.bin", trunc).c_str(), 8, 0, &net) == RMRCM_EINVAL, "truncated");
    for (auto h : {header(7, 16, 5, 16, 4), header(16, 0, 5, 16, 4), header(16, 16, 1, 16, 4),
                   header(16, 16, 5, 99, 4), header(-16, 16, 5, 16, 4)}) {
        h.resize(h.size() + 16, 0);
        expect(rmrcm_cnn_load(write("shape.bin", h).c_str(), 8, 0, &net) == RMRCM_EINVAL, "bad shape");
    }
    std::vector<char> ok = header(16, 16, 5, 16, 4);
    ok.resize(ok.size() + 16, 0);
    if (!have_gpu)
        expect(rmrcm_cnn_load(write("ok.bin", ok).c_str(), 8, 0, &net) == RMRCM_EDEVICE, "load without a device");
    expect(!net, "no network returned");
}

static void status_strings() {
    for (int s = -9; s <= 1; ++s) {
        const char* m = rmrcm_strerror(s);
        expect(m && std::strlen(m) > 0, "strerror " + std::to_string(s));
    }
}

int main(int argc, char** argv) {
    const std::string dir = argc > 1 ? argv[1] : ".";
    const bool have_gpu = argc > 2 && std::strcmp(argv[2], "gpu") == 0;
    status_strings();
    plan_sweep();
    setup_validation(have_gpu);
    context_nulls();
    weight_files(dir, have_gpu);
    std::printf("%d checks, %d failures\n", checks, failures);
    return failures;
}
