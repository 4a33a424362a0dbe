// Drives the host side of libspmvc's C ABI under AddressSanitizer and
// UndefinedBehaviorSanitizer (api.cpp and tune.cpp are built instrumented):
// every entry point with the arguments its host-side checks reject, which
// return before any device work, plus the status strings, the thread-local
// error message and the allocator hooks.  Exit status 0 when every call
// returns the documented status (test infrastructure).
#include <cstdio>
#include <cstring>

#include "../../include/spmvc.h"

#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                                        \
        }                                                                    \
    } while (0)

static void *fake_alloc(size_t, void *, void *) { return nullptr; }
static void fake_free(void *, void *, void *) {}

int main() {
    for (int s = -9; s <= 1; ++s) CHECK(spmvc_status_string(s) != nullptr && std::strlen(spmvc_status_string(s)) > 0);
    CHECK(std::strcmp(spmvc_status_string(0), "ok") == 0);
    spmvc_matrix M = nullptr;
    int64_t rp[2] = {0, 0};
    CHECK(spmv_compress(-1, 4, 0, rp, nullptr, nullptr, nullptr, nullptr, &M) == SPMVC_EINVAL);
    CHECK(std::strlen(spmvc_last_error()) > 0);
    CHECK(spmv_compress(4, 4, 0, nullptr, nullptr, nullptr, nullptr, nullptr, &M) == SPMVC_EINVAL);
    CHECK(spmv_compress(4, 4, 0, rp, nullptr, nullptr, nullptr, nullptr, nullptr) == SPMVC_EINVAL);
    CHECK(spmv_compress(int64_t(1) << 31, 4, 0, rp, nullptr, nullptr, nullptr, nullptr, &M) == SPMVC_EINVAL);
    CHECK(spmv_compress(4, 4, 3, rp, nullptr, nullptr, nullptr, nullptr, &M) == SPMVC_EINVAL);
    int32_t col[1] = {0};
    double val[1] = {1.0};
    CHECK(spmv_compress(1, 0, 1, rp, col, val, nullptr, nullptr, &M) == SPMVC_ERANGE);
    spmvc_compress_opts o{};
    for (int bad = 0; bad < 5; ++bad) {
        o = spmvc_compress_opts{SPMVC_FMT_DIT, 15, 65535, 2, 1};
        if (bad == 0) o.fmt = 9;
        if (bad == 1) o.k_max = 16;
        if (bad == 2) o.p_max = 0;
        if (bad == 3) o.min_pattern_rows = 0;
        if (bad == 4) o.fmt = -1;
        CHECK(spmv_compress(1, 1, 1, rp, col, val, &o, nullptr, &M) == SPMVC_EINVAL);
    }
    CHECK(M == nullptr);
    double x[4] = {}, y[4] = {};
    CHECK(spmv(nullptr, SPMVC_F64, x, y, nullptr) == SPMVC_EINVAL);
    CHECK(spmv_block(nullptr, SPMVC_F64, 2, x, 2, y, 2, nullptr) == SPMVC_EINVAL);
    spmvc_cg_stat st[4];
    const double *bs[1] = {x};
    double *xs[1] = {y};
    spmvc_matrix hs[1] = {nullptr};
    CHECK(cg_solve(nullptr, 1, 1, bs, xs, nullptr, st, nullptr) == SPMVC_EINVAL);
    CHECK(cg_solve(hs, 0, 1, bs, xs, nullptr, st, nullptr) == SPMVC_EINVAL);
    CHECK(cg_solve(hs, 1, 0, bs, xs, nullptr, st, nullptr) == SPMVC_EINVAL);
    CHECK(cg_solve(hs, 1, 17, bs, xs, nullptr, st, nullptr) == SPMVC_EINVAL);
    CHECK(cg_solve(hs, 1, 1, bs, xs, nullptr, st, nullptr) == SPMVC_EINVAL);  // null handle inside
    spmvc_cg_opts co{1e-10, 10000, 0, 1e-5, 20, 16, 2};
    co.rtol = 0.0;
    CHECK(cg_solve(hs, 1, 1, bs, xs, &co, st, nullptr) == SPMVC_EINVAL);
    co.rtol = 1e-10;
    co.mode = 3;
    CHECK(cg_solve(hs, 1, 1, bs, xs, &co, st, nullptr) == SPMVC_EINVAL);
    CHECK(cg_solve_noalloc(nullptr, x, y, nullptr, st, nullptr) == SPMVC_EINVAL);
    CHECK(cg_solve_mg(nullptr, nullptr, 1, x, y, nullptr, st, nullptr) == SPMVC_EINVAL);
    CHECK(cg_solve_mg(hs, nullptr, 0, x, y, nullptr, st, nullptr) == SPMVC_EINVAL);
    CHECK(cg_solve_mg(hs, nullptr, 17, x, y, nullptr, st, nullptr) == SPMVC_EINVAL);
    CHECK(cg_solve_mg(hs, nullptr, 2, x, y, nullptr, st, nullptr) == SPMVC_EINVAL);
    CHECK(spmv_symgs(nullptr, x, y, 1, nullptr) == SPMVC_EINVAL);
    int32_t nc = 0;
    CHECK(spmv_colors(nullptr, &nc, nullptr, nullptr) == SPMVC_EINVAL);
    CHECK(spmv_decompress(nullptr, rp, col, val, nullptr) == SPMVC_EINVAL);
    spmvc_info info;
    CHECK(spmv_info(nullptr, &info) == SPMVC_EINVAL);
    int64_t bytes = 0;
    CHECK(spmv_get_array(nullptr, SPMVC_ARR_IDS, nullptr, &bytes, nullptr) == SPMVC_EINVAL);
    CHECK(spmv_set_config(nullptr, 512, 1) == SPMVC_EINVAL);
    CHECK(spmv_set_block_mode(nullptr, 1) == SPMVC_EINVAL);
    int32_t br = 0, bl = 0;
    double bu = 0.0;
    CHECK(spmv_tune(nullptr, SPMVC_F64, 1, nullptr, &br, &bl, &bu) == SPMVC_EINVAL);
    CHECK(spmvc_batched_config(nullptr, nullptr, nullptr) == SPMVC_EINVAL);
    int32_t form = 0, chunk = 0;
    CHECK(spmvc_batched_config(&form, &chunk, &bu) == SPMVC_OK && form == -1);
    CHECK(spmvc_set_allocator(fake_alloc, nullptr, nullptr) == SPMVC_EINVAL);
    CHECK(spmvc_set_allocator(nullptr, fake_free, nullptr) == SPMVC_EINVAL);
    CHECK(spmvc_set_allocator(fake_alloc, fake_free, nullptr) == SPMVC_OK);
    CHECK(spmvc_set_allocator(nullptr, nullptr, nullptr) == SPMVC_OK);
    CHECK(spmv_rcm(-1, rp, col, nullptr, nullptr) == SPMVC_EINVAL);
    CHECK(spmv_rcm(int64_t(1) << 31, rp, col, col, nullptr) == SPMVC_EINVAL);
    CHECK(spmv_permute(4, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == SPMVC_EINVAL);
    spmv_free(nullptr);
    std::puts("ABI sanitizer driver: ok");
    return 0;
}
