// The C ABI of libspmvc: argument checks, error reporting, handle lifetime.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>

#include <mutex>

#include "internal.h"

namespace spmvc {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

spmvc_status fail(spmvc_status st, const std::string &msg) {
    set_error(msg);
    return st;
}

namespace {

template <class F> spmvc_status guarded(F &&f) {
    try {
        g_last_error.clear();
        return f();
    } catch (const Error &e) {
        return fail(e.st, e.msg);
    } catch (const std::bad_alloc &) {
        return fail(SPMVC_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(SPMVC_EHIP, e.what());
    } catch (...) {
        return fail(SPMVC_EHIP, "unknown error");
    }
}

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
    return na && nb && pa < pb + nb && pb < pa + na;
}

bool f32_ready(const spmvc_matrix_s *M) {
    return M->f32_shadow || (M->raw_elems == 0 && M->n_esc_nnz == 0);
}

// XCDs the hardware spreads consecutive blocks over (gfx94x / gfx95x: eight).
int xcd_count() {
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 1;
    const std::string arch = prop.gcnArchName;
    return (arch.rfind("gfx94", 0) == 0 || arch.rfind("gfx95", 0) == 0) ? 8 : 1;
}

int cu_count() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
        return 256;
    return n;
}

}  // namespace

void prepare_handle(spmvc_matrix_s *M) {
    M->n_xcd = xcd_count();
    M->n_cu = cu_count();
    if (M->fmt != SPMVC_FMT_DIT && M->fmt != SPMVC_FMT_BMASK) return;
    for (int dt : {SPMVC_F64, SPMVC_F32}) {
        for (int rows : {M->rows_per_block[dt], 1024, 512, 256}) {
            build_lds_plan(M, dt, rows);
            if (M->plan[dt].n_win > 0) {
                M->rows_per_block[dt] = rows;
                break;
            }
        }
    }
}

}  // namespace spmvc

using namespace spmvc;

namespace spmvc {
namespace {
std::mutex g_alloc_mu;
Allocator g_alloc;
}  // namespace
Allocator current_allocator() {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_alloc;
}
}  // namespace spmvc

extern "C" {

const char *spmvc_status_string(int32_t st) {
    switch (st) {
    case SPMVC_OK: return "ok";
    case SPMVC_EINVAL: return "invalid argument";
    case SPMVC_ENOMEM: return "out of device memory";
    case SPMVC_EUNSORTED: return "CSR columns not strictly ascending within a row";
    case SPMVC_ERANGE: return "CSR row pointer or column index out of range";
    case SPMVC_EHIP: return "HIP runtime error";
    case SPMVC_ENOTSPD: return "CG breakdown (matrix not SPD)";
    case SPMVC_ENOCONV: return "CG did not converge";
    case SPMVC_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

const char *spmvc_last_error(void) { return g_last_error.c_str(); }

spmvc_status spmvc_set_allocator(void *(*alloc_fn)(size_t, void *, void *), void (*free_fn)(void *, void *, void *),
                                 void *ctx) {
    return guarded([&]() -> spmvc_status {
        if ((alloc_fn == nullptr) != (free_fn == nullptr))
            return fail(SPMVC_EINVAL, "alloc and free must both be set or both be NULL");
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        g_alloc.alloc = reinterpret_cast<void *(*)(size_t, hipStream_t, void *)>(alloc_fn);
        g_alloc.free = reinterpret_cast<void (*)(void *, hipStream_t, void *)>(free_fn);
        g_alloc.ctx = alloc_fn ? ctx : nullptr;
        return SPMVC_OK;
    });
}

spmvc_status spmv_compress(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *row_ptr,
                           const int32_t *col_idx, const double *vals, const spmvc_compress_opts *opts,
                           void *stream, spmvc_matrix *out) {
    return guarded([&]() -> spmvc_status {
        if (!out) return fail(SPMVC_EINVAL, "out is null");
        *out = nullptr;
        if (n_rows < 0 || n_cols < 0 || nnz < 0) return fail(SPMVC_EINVAL, "negative size");
        if (n_rows >= (1ll << 31) || n_cols >= (1ll << 31) || nnz >= (1ll << 31))
            return fail(SPMVC_EINVAL, "n_rows, n_cols and nnz must be < 2^31");
        if (!row_ptr) return fail(SPMVC_EINVAL, "row_ptr is null");
        if (nnz > 0 && (!col_idx || !vals)) return fail(SPMVC_EINVAL, "col_idx / vals is null");
        if (nnz > 0 && n_cols == 0) return fail(SPMVC_ERANGE, "entries in a matrix with no columns");
        spmvc_compress_opts o{SPMVC_FMT_DIT, 15, 65535, 2, 1};
        if (opts) o = *opts;
        if (o.fmt < SPMVC_FMT_ELL || o.fmt > SPMVC_FMT_BMASK) return fail(SPMVC_EINVAL, "unknown format");
        const bool autofmt = o.fmt == SPMVC_FMT_AUTO;
        if (autofmt) o.fmt = SPMVC_FMT_DIT;
        if (o.k_max < 0 || o.k_max > kMaxK) return fail(SPMVC_EINVAL, "k_max must be in 0..15");
        if (o.p_max < 1 || o.p_max > 0x7FFFFFFE) return fail(SPMVC_EINVAL, "p_max must be in 1..2^31-2");
        if (o.min_pattern_rows < 1) return fail(SPMVC_EINVAL, "min_pattern_rows must be >= 1");
        auto *M = new spmvc_matrix_s();
        M->n_rows = n_rows;
        M->n_cols = n_cols;
        M->nnz = nnz;
        try {
            compress(M, row_ptr, col_idx, vals, o, static_cast<hipStream_t>(stream));
            if (autofmt && M->n_rows > 0) {
                // AUTO: DIT unless its stream is not smaller than ELL's (12 bytes per
                // slot of the longest pattern, escape rows as CSR)
                int64_t maxlen = 0;
                for (int q = 0; q < M->P; ++q) maxlen = std::max<int64_t>(maxlen, M->h_pat_len[q]);
                const int64_t ell = 12 * maxlen * M->n_pad + 12 * M->n_esc_nnz + 16 * M->n_esc;
                if (stream_bytes(M, SPMVC_F64) >= ell) {
                    auto *E = new spmvc_matrix_s();
                    E->n_rows = n_rows;
                    E->n_cols = n_cols;
                    E->nnz = nnz;
                    o.fmt = SPMVC_FMT_ELL;
                    try {
                        compress(E, row_ptr, col_idx, vals, o, static_cast<hipStream_t>(stream));
                    } catch (...) {
                        delete E;
                        throw;
                    }
                    delete M;
                    M = E;
                }
            }
            prepare_handle(M);
        } catch (...) {
            delete M;
            throw;
        }
        *out = M;
        return SPMVC_OK;
    });
}

spmvc_status spmv(spmvc_matrix A, int32_t dt, const void *x, void *y, void *stream) {
    return guarded([&]() -> spmvc_status {
        if (!A) return fail(SPMVC_EINVAL, "matrix handle is null");
        if (dt != SPMVC_F64 && dt != SPMVC_F32) return fail(SPMVC_EINVAL, "dtype must be F64 or F32");
        if ((A->n_cols > 0 && !x) || (A->n_rows > 0 && !y)) return fail(SPMVC_EINVAL, "x / y is null");
        const size_t es = dt == SPMVC_F64 ? 8 : 4;
        if (overlap(x, es * A->n_cols, y, es * A->n_rows)) return fail(SPMVC_EINVAL, "x and y overlap");
        if (dt == SPMVC_F32 && !f32_ready(A)) return fail(SPMVC_EUNSUPPORTED, "FP32 spmv needs f32_shadow at compress time");
        launch_spmv(A, dt, x, y, static_cast<hipStream_t>(stream));
        return SPMVC_OK;
    });
}

spmvc_status spmv_block(spmvc_matrix A, int32_t dt, int32_t nrhs, const void *X, int64_t ldx, void *Y, int64_t ldy,
                        void *stream) {
    return guarded([&]() -> spmvc_status {
        if (!A) return fail(SPMVC_EINVAL, "matrix handle is null");
        if (dt != SPMVC_F64 && dt != SPMVC_F32) return fail(SPMVC_EINVAL, "dtype must be F64 or F32");
        if (nrhs < 1 || nrhs > 16) return fail(SPMVC_EINVAL, "nrhs must be in 1..16");
        if (ldx < nrhs || ldy < nrhs) return fail(SPMVC_EINVAL, "ldx and ldy must be >= nrhs");
        if ((A->n_cols > 0 && !X) || (A->n_rows > 0 && !Y)) return fail(SPMVC_EINVAL, "X / Y is null");
        const size_t es = dt == SPMVC_F64 ? 8 : 4;
        if (overlap(X, es * A->n_cols * ldx, Y, es * A->n_rows * ldy)) return fail(SPMVC_EINVAL, "X and Y overlap");
        if (dt == SPMVC_F32 && !f32_ready(A)) return fail(SPMVC_EUNSUPPORTED, "FP32 spmv needs f32_shadow at compress time");
        launch_spmv_block(A, dt, nrhs, X, ldx, Y, ldy, static_cast<hipStream_t>(stream));
        return SPMVC_OK;
    });
}

spmvc_status cg_solve(const spmvc_matrix *A, int32_t n_sys, int32_t nrhs, const double *const *b, double *const *x,
                      const spmvc_cg_opts *opts, spmvc_cg_stat *stat, void *stream) {
    return guarded([&]() -> spmvc_status {
        if (!A || !b || !x || !stat) return fail(SPMVC_EINVAL, "null argument");
        if (n_sys < 1) return fail(SPMVC_EINVAL, "n_sys must be >= 1");
        if (nrhs < 1 || nrhs > 16) return fail(SPMVC_EINVAL, "nrhs must be in 1..16");
        spmvc_cg_opts o{1e-10, 10000, 0, 1e-5, 20, 16, 2};
        if (opts) o = *opts;
        if (!(o.rtol > 0.0) || o.max_iter < 1 || o.check_every < 1 || o.mode < 0 || o.mode > 3 ||
            o.batched < 0 || o.batched > 2)
            return fail(SPMVC_EINVAL, "invalid cg options");
        if ((o.mode == 1 || o.mode == 3) && (n_sys != 1 || nrhs != 1))
            return fail(SPMVC_EUNSUPPORTED, "mixed-precision modes take one system with one right-hand side");
        if (o.mode == 2 && (n_sys != 1 || nrhs != 1))
            return fail(SPMVC_EUNSUPPORTED, "preconditioned mode takes one system with one right-hand side");
        if ((o.mode == 1 || o.mode == 3) && (!(o.inner_rtol > 0.0) || o.max_outer < 0))
            return fail(SPMVC_EINVAL, "invalid inner options");
        for (int s = 0; s < n_sys; ++s) {
            if (!A[s]) return fail(SPMVC_EINVAL, "matrix handle is null");
            if (A[s]->n_rows != A[s]->n_cols) return fail(SPMVC_EINVAL, "CG needs square matrices");
            if (A[s]->n_rows > 0 && (!b[s] || !x[s])) return fail(SPMVC_EINVAL, "b / x is null");
            if (overlap(b[s], 8 * A[s]->n_rows * nrhs, x[s], 8 * A[s]->n_rows * nrhs))
                return fail(SPMVC_EINVAL, "b and x overlap");
            if ((o.mode == 1 || o.mode == 3) && !f32_ready(A[s]))
                return fail(SPMVC_EUNSUPPORTED, "mixed modes need f32_shadow");
        }
        for (int i = 0; i < n_sys * nrhs; ++i) stat[i] = spmvc_cg_stat{};
        const spmvc_status st = cg_solve_impl(A, n_sys, nrhs, b, x, o, stat, static_cast<hipStream_t>(stream));
        if (st != SPMVC_OK) set_error(spmvc_status_string(st));
        return st;
    });
}

spmvc_status cg_solve_noalloc(spmvc_matrix A, const double *b, double *x, const spmvc_cg_opts *opts,
                              spmvc_cg_stat *stat, void *stream) {
    return guarded([&]() -> spmvc_status {
        if (!A || !stat) return fail(SPMVC_EINVAL, "null argument");
        spmvc_cg_opts o{1e-10, 10000, 0, 1e-5, 20, 16, 0};
        if (opts) o = *opts;
        if (!(o.rtol > 0.0) || o.max_iter < 1 || o.check_every < 1) return fail(SPMVC_EINVAL, "invalid cg options");
        if (o.mode != 0) return fail(SPMVC_EINVAL, "cg_solve_noalloc runs FP64 CG (mode 0) only");
        if (A->n_rows != A->n_cols) return fail(SPMVC_EINVAL, "CG needs square matrices");
        if (A->n_rows > cg_noalloc_max_rows())
            return fail(SPMVC_EINVAL, "cg_solve_noalloc: " + std::to_string(A->n_rows) +
                                          " rows exceed the scratch limit of " + std::to_string(cg_noalloc_max_rows()));
        if (A->n_rows > 0 && (!b || !x)) return fail(SPMVC_EINVAL, "b / x is null");
        if (overlap(b, 8 * A->n_rows, x, 8 * A->n_rows)) return fail(SPMVC_EINVAL, "b and x overlap");
        *stat = spmvc_cg_stat{};
        if (A->n_rows == 0) return SPMVC_OK;
        const spmvc_status st = cg_solve_noalloc_impl(A, b, x, o, *stat, static_cast<hipStream_t>(stream));
        if (st != SPMVC_OK) set_error(spmvc_status_string(st));
        return st;
    });
}

spmvc_status cg_solve_mg(const spmvc_matrix *levels, const int32_t *const *f2c, int32_t n_levels, const double *b,
                         double *x, const spmvc_cg_opts *opts, spmvc_cg_stat *stat, void *stream) {
    return guarded([&]() -> spmvc_status {
        if (!levels || !stat) return fail(SPMVC_EINVAL, "null argument");
        if (n_levels < 1 || n_levels > 16) return fail(SPMVC_EINVAL, "n_levels must be in 1..16");
        if (n_levels > 1 && !f2c) return fail(SPMVC_EINVAL, "f2c is null");
        spmvc_cg_opts o{1e-10, 10000, 0, 1e-5, 20, 16, 2};
        if (opts) o = *opts;
        if (!(o.rtol > 0.0) || o.max_iter < 1 || o.check_every < 1) return fail(SPMVC_EINVAL, "invalid cg options");
        for (int l = 0; l < n_levels; ++l) {
            const spmvc_matrix_s *A = levels[l];
            if (!A) return fail(SPMVC_EINVAL, "matrix handle is null");
            if (A->n_rows != A->n_cols) return fail(SPMVC_EINVAL, "CG needs square matrices");
            if (l > 0) {
                if (A->n_rows < 1 || A->n_rows > levels[l - 1]->n_rows)
                    return fail(SPMVC_EINVAL, "a coarse level must be non-empty and no larger than the level above");
                if (!f2c[l - 1]) return fail(SPMVC_EINVAL, "f2c entry is null");
            }
        }
        const int64_t n = levels[0]->n_rows;
        if (n > 0 && (!b || !x)) return fail(SPMVC_EINVAL, "b / x is null");
        if (overlap(b, 8 * n, x, 8 * n)) return fail(SPMVC_EINVAL, "b and x overlap");
        stat[0] = spmvc_cg_stat{};
        const spmvc_status st = cg_solve_mg_impl(levels, f2c, n_levels, b, x, o, stat, static_cast<hipStream_t>(stream));
        if (st != SPMVC_OK) set_error(spmvc_status_string(st));
        return st;
    });
}

spmvc_status spmv_rcm(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, int32_t *perm, void *stream) {
    return guarded([&]() -> spmvc_status {
        if (n < 0 || n > INT32_MAX) return fail(SPMVC_EINVAL, "n must be in 0..2^31-1");
        if (!row_ptr || (n > 0 && !perm)) return fail(SPMVC_EINVAL, "null argument");
        rcm_order(n, row_ptr, col_idx, perm, static_cast<hipStream_t>(stream));
        return SPMVC_OK;
    });
}

spmvc_status spmv_permute(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const double *vals,
                          const int32_t *perm, int64_t *out_row_ptr, int32_t *out_col_idx, double *out_vals,
                          void *stream) {
    return guarded([&]() -> spmvc_status {
        if (n < 0 || n > INT32_MAX) return fail(SPMVC_EINVAL, "n must be in 0..2^31-1");
        if (!row_ptr || !out_row_ptr || (n > 0 && !perm)) return fail(SPMVC_EINVAL, "null argument");
        permute_csr(n, row_ptr, col_idx, vals, perm, out_row_ptr, out_col_idx, out_vals,
                    static_cast<hipStream_t>(stream));
        return SPMVC_OK;
    });
}

spmvc_status spmv_decompress(spmvc_matrix A, int64_t *row_ptr, int32_t *col_idx, double *vals, void *stream) {
    return guarded([&]() -> spmvc_status {
        if (!A || !row_ptr) return fail(SPMVC_EINVAL, "null argument");
        if (A->nnz > 0 && (!col_idx || !vals)) return fail(SPMVC_EINVAL, "col_idx / vals is null");
        decompress(A, row_ptr, col_idx, vals, static_cast<hipStream_t>(stream));
        return SPMVC_OK;
    });
}

spmvc_status spmv_symgs(spmvc_matrix A, const double *b, double *x, int32_t sweeps, void *stream) {
    return guarded([&]() -> spmvc_status {
        if (!A) return fail(SPMVC_EINVAL, "matrix handle is null");
        if (sweeps < 0) return fail(SPMVC_EINVAL, "sweeps must be >= 0");
        if (A->n_rows > 0 && (!b || !x)) return fail(SPMVC_EINVAL, "b / x is null");
        if (overlap(b, 8 * A->n_rows, x, 8 * A->n_rows)) return fail(SPMVC_EINVAL, "b and x overlap");
        const hipStream_t s = static_cast<hipStream_t>(stream);
        build_coloring(A, s);
        launch_symgs(A, b, x, sweeps, s);
        return SPMVC_OK;
    });
}

spmvc_status spmvc_batched_config(int32_t *form, int32_t *chunk, double *us_per_spmv) {
    return guarded([&]() -> spmvc_status {
        if (!form || !chunk || !us_per_spmv) return fail(SPMVC_EINVAL, "null argument");
        batched_last_tune(form, chunk, us_per_spmv);
        return SPMVC_OK;
    });
}

spmvc_status spmv_colors(spmvc_matrix A, int32_t *n_colors, int32_t *color, void *stream) {
    return guarded([&]() -> spmvc_status {
        if (!A || !n_colors) return fail(SPMVC_EINVAL, "null argument");
        const hipStream_t s = static_cast<hipStream_t>(stream);
        build_coloring(A, s);
        *n_colors = A->gs_n_colors;
        if (color && A->n_rows > 0) {
            SPMVC_HIP(hipMemcpyAsync(color, A->gs_color.p, sizeof(int32_t) * A->n_rows, hipMemcpyDeviceToDevice, s));
            SPMVC_HIP(hipStreamSynchronize(s));
        }
        return SPMVC_OK;
    });
}

spmvc_status spmv_info(spmvc_matrix A, spmvc_info *info) {
    return guarded([&]() -> spmvc_status {
        if (!A || !info) return fail(SPMVC_EINVAL, "null argument");
        spmvc_info r{};
        r.fmt = A->fold ? SPMVC_FMT_DITV : A->fmt;
        r.K = A->K;
        r.P = A->P;
        r.id_bytes = A->id_bytes;
        r.width = A->width;
        r.max_raw = A->max_raw;
        r.n_rows = A->n_rows;
        r.n_cols = A->n_cols;
        r.nnz = A->nnz;
        r.n_escape_rows = A->n_esc;
        r.n_escape_nnz = A->n_esc_nnz;
        r.n_raw = A->n_raw;
        r.bytes_stream = stream_bytes(A, SPMVC_F64);
        // ELL of the same matrix: width = longest row, 12 bytes per slot over padded rows
        int64_t maxlen = A->width;  // BMASK: the longest row
        if (A->fmt == SPMVC_FMT_DIT) {
            maxlen = 0;
            for (int q = 0; q < A->P; ++q) maxlen = std::max<int64_t>(maxlen, A->h_pat_len[q]);
        }
        r.bytes_ell = 12 * maxlen * A->n_pad + 12 * A->n_esc_nnz + 16 * A->n_esc;
        const int64_t k4 = 4 * static_cast<int64_t>(A->K);
        if (A->fmt == SPMVC_FMT_ELL)
            r.bytes_paper = 12 * A->nnz;
        else if (A->fmt == SPMVC_FMT_DT)
            r.bytes_paper = 4 * (A->nnz - A->n_esc_nnz) + k4 * (A->n_rows - A->n_esc) + 12 * A->n_esc_nnz +
                            8 * A->n_raw;
        else if (A->fmt == SPMVC_FMT_BMASK)  // the masks at their own width, values as stored
            r.bytes_paper = stream_bytes(A, SPMVC_F64);
        else if (!A->fold)
            r.bytes_paper = (4 + k4) * (A->n_rows - A->n_esc) + 12 * A->n_esc_nnz + 8 * A->n_raw;
        else  // DITV: the 4-byte ID alone
            r.bytes_paper = 4 * (A->n_rows - A->n_esc) + 12 * A->n_esc_nnz + 8 * A->n_raw;
        const bool planned = A->fmt == SPMVC_FMT_DIT || A->fmt == SPMVC_FMT_BMASK;
        r.lds_windows = (planned && A->lds_mode[SPMVC_F64] >= 1) ? A->plan[SPMVC_F64].n_win : 0;
        r.rows_per_block = planned ? A->plan[SPMVC_F64].rows : kBlock;
        if (A->fmt == SPMVC_FMT_BMASK) {
            r.P = A->bm_nd;
            r.id_bytes = A->bm_bytes;
        }
        for (int c = 0; c < A->K; ++c) r.V[c] = A->V[c];
        r.kernel = kernel_kind(A, SPMVC_F64);
        r.kernel_f32 = kernel_kind(A, SPMVC_F32);
        r.rows_per_block_f32 = planned ? A->plan[SPMVC_F32].rows : kBlock;
        r.block_split = A->plan[SPMVC_F64].bw && A->plan[SPMVC_F64].bw_split ? 1 : 0;
        *info = r;
        return SPMVC_OK;
    });
}

spmvc_status spmv_get_array(spmvc_matrix A, int32_t which, void *dst, int64_t *bytes, void *stream) {
    return guarded([&]() -> spmvc_status {
        if (!A || !bytes) return fail(SPMVC_EINVAL, "null argument");
        const DevBuf *b = nullptr;
        switch (which) {
        case SPMVC_ARR_ELL_VAL: b = &A->ell_val; break;
        case SPMVC_ARR_ELL_COL: b = &A->ell_col; break;
        case SPMVC_ARR_DT_S: b = &A->dt_S; break;
        case SPMVC_ARR_IDS: b = &A->ids; break;
        case SPMVC_ARR_T: b = &A->T; break;
        case SPMVC_ARR_PAT_OFF: b = &A->pat_off; break;
        case SPMVC_ARR_PAT_LEN: b = &A->pat_len; break;
        case SPMVC_ARR_PAT_T: b = &A->pat_T; break;
        case SPMVC_ARR_RAW: b = &A->raw; break;
        case SPMVC_ARR_RAW_SLICE: b = &A->raw_slice; break;
        case SPMVC_ARR_ESC_ROWS: b = &A->esc_rows; break;
        case SPMVC_ARR_ESC_PTR: b = &A->esc_ptr; break;
        case SPMVC_ARR_ESC_COL: b = &A->esc_col; break;
        case SPMVC_ARR_ESC_VAL: b = &A->esc_val; break;
        case SPMVC_ARR_V: b = &A->V_dev; break;
        case SPMVC_ARR_BM_D: b = &A->bm_d; break;
        case SPMVC_ARR_BM_MASK: b = &A->bm_mask; break;
        case SPMVC_ARR_BM_VMASK: b = &A->bm_vmask; break;
        default: return fail(SPMVC_EINVAL, "unknown array id");
        }
        *bytes = static_cast<int64_t>(b->bytes);
        if (dst && b->bytes) {
            hipStream_t s = static_cast<hipStream_t>(stream);
            SPMVC_HIP(hipMemcpyAsync(dst, b->p, b->bytes, hipMemcpyDeviceToDevice, s));
            SPMVC_HIP(hipStreamSynchronize(s));
        }
        return SPMVC_OK;
    });
}

spmvc_status spmv_set_block_mode(spmvc_matrix A, int32_t mode) {
    return guarded([&]() -> spmvc_status {
        if (!A) return fail(SPMVC_EINVAL, "matrix handle is null");
        if (mode < 0 || mode > 3) return fail(SPMVC_EINVAL, "block mode must be 0, 1, 2 or 3");
        A->block_mode[SPMVC_F64] = mode;
        A->block_mode[SPMVC_F32] = mode;
        return SPMVC_OK;
    });
}

spmvc_status spmv_set_config(spmvc_matrix A, int32_t rows_per_block, int32_t lds) {
    return guarded([&]() -> spmvc_status {
        if (!A) return fail(SPMVC_EINVAL, "matrix handle is null");
        if (rows_per_block != 0 && (rows_per_block < 256 || rows_per_block > 4096 || rows_per_block % 256))
            return fail(SPMVC_EINVAL, "rows_per_block must be a multiple of 256 in 256..4096");
        if (lds < -1 || lds > 2) return fail(SPMVC_EINVAL, "lds must be -1, 0, 1 or 2");
        for (int dt : {SPMVC_F64, SPMVC_F32}) {
            if (lds >= 0) A->lds_mode[dt] = lds;
            if (rows_per_block) {
                A->rows_per_block[dt] = rows_per_block;
                build_lds_plan(A, dt, rows_per_block);
            }
        }
        return SPMVC_OK;
    });
}

spmvc_status spmv_color_order(spmvc_matrix A, spmvc_matrix *B, int32_t *perm, void *stream) {
    return guarded([&]() -> spmvc_status {
        if (!A || !B) return fail(SPMVC_EINVAL, "null argument");
        *B = nullptr;
        if (A->n_rows != A->n_cols) return fail(SPMVC_EINVAL, "the color order needs a square matrix");
        *B = color_order_copy(A, perm, static_cast<hipStream_t>(stream));
        return SPMVC_OK;
    });
}

spmvc_status spmvc_check_violations(int64_t *count, int32_t *checked) {
    return guarded([&]() -> spmvc_status {
        if (!count || !checked) return fail(SPMVC_EINVAL, "null argument");
#ifdef SPMVC_CHECK
        *checked = 1;
#else
        *checked = 0;
#endif
        SPMVC_HIP(hipDeviceSynchronize());
        *count = static_cast<int64_t>(check_violations_spmv() + check_violations_batched() + check_violations_symgs());
        return SPMVC_OK;
    });
}

spmvc_status spmvc_check_probe(int64_t i, int64_t n, void *stream) {
    return guarded([&]() -> spmvc_status {
        if (!check_probe(i, n, static_cast<hipStream_t>(stream)))
            return fail(SPMVC_EUNSUPPORTED, "not a bounds-checked build");
        return SPMVC_OK;
    });
}

void spmv_free(spmvc_matrix A) { delete A; }

}  // extern "C"
