// Symmetric Gauss-Seidel over the compressed matrix, in multicolor order.
//
// SymGS is the other kernel of the HPCG iteration the paper accelerates
// (Section III, Table I: SymGS beside SpMV); it walks the same rows as the
// SpMV.  A sweep updates x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii forward
// through the rows and then backward.  On the GPU the rows are taken color by
// color: rows of one color share no entry (a proper coloring of the pattern
// of A + A^T), so one launch updates all of them; a sweep is the colors
// forward, then backward.
//
// The coloring is greedy in row order: each row takes the smallest color no
// lower-numbered neighbour holds (on a 27-point stencil: the 8 parity
// classes).  It is built once per handle on first use, on the host from the
// decompressed CSR -- an O(nnz) set-up step like the LDS plans -- and kept
// on the device as the rows of each color, ascending.
//
// k_symgs_color: one thread per row of the color; the row is decoded from
// the handle's own format (ELL, DT, DIT/DITV, raw values, escape rows) and
// x is gathered straight from global memory, since the rows of a color are
// spread over the whole grid.  k_symgs_dit: the same for DIT/DITV stencil-like
// matrices, with all of a row's gathers in flight at once.
#include <algorithm>
#include <vector>

#include "check.h"
#include "internal.h"

namespace spmvc {
namespace {

constexpr int kGsThreads = 256;
constexpr int kGsTblInts = 2048;  // pattern-offset words staged in LDS (8 KB)

struct GsArgs {
    int64_t n_rows, n_pad;
    int32_t fmt, K, width, id_bytes;
    const void *ids;
    const uint8_t *T;
    const uint8_t *pat_T;  // DITV: T of each pattern
    const int32_t *pat_off;
    const uint8_t *pat_len;
    const int32_t *cols;   // ELL columns or DT's S
    const double *ell_val;
    const double *raw;
    const int64_t *raw_slice;
    const int64_t *esc_rows, *esc_ptr;
    const int32_t *esc_col;
    const double *esc_val;
    int64_t n_esc;
    int32_t P;
    double V[kMaxK];
    // BMASK: displacement list, per-row masks (4 or 8 bytes)
    const int32_t *bm_d;
    const void *bm_mask, *bm_vmask;
    int32_t bm_bytes;
};

__device__ __forceinline__ uint32_t gs_id(const GsArgs &a, int64_t row) {
    if (a.id_bytes == 1) return static_cast<const uint8_t *>(a.ids)[row];
    if (a.id_bytes == 2) return static_cast<const uint16_t *>(a.ids)[row];
    return static_cast<const uint32_t *>(a.ids)[row];
}

// Calls f(value, column) for every entry of `row`.
template <class F> __device__ __forceinline__ void gs_visit(const GsArgs &a, int64_t row, F f) {
    if (a.fmt == SPMVC_FMT_BMASK) {  // set bits ascending = columns ascending; no escape rows
        auto mask_at = [&](const void *m) -> uint64_t {
            return a.bm_bytes == 4 ? static_cast<const uint32_t *>(m)[row] : static_cast<const uint64_t *>(m)[row];
        };
        uint64_t m = mask_at(a.bm_mask);
        const uint64_t vm = a.K == 2 ? mask_at(a.bm_vmask) : 0;
        const int64_t rb = a.raw ? a.raw_slice[row / kSlice] + (row % kSlice) : 0;
        for (int64_t j = 0; m; ++j) {
            const int k = __builtin_ctzll(m);
            m &= m - 1;
            f(a.raw ? a.raw[rb + j * kSlice] : a.V[(vm >> k) & 1], row + a.bm_d[k]);
        }
        return;
    }
    bool escape = false;
    uint32_t id = 0;
    if (a.fmt == SPMVC_FMT_DIT) {
        id = gs_id(a, row);
        escape = id == (a.id_bytes == 1 ? 0xFFu : (a.id_bytes == 2 ? 0xFFFFu : 0xFFFFFFFFu));
    } else {
        escape = a.cols[row] == kEscapeColumn;
    }
    if (escape) {  // plain CSR row: find it among the (ascending) escape rows
        int64_t lo = 0, hi = a.n_esc;
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) / 2;
            if (a.esc_rows[mid] <= row) lo = mid; else hi = mid;
        }
        for (int64_t k = a.esc_ptr[lo]; k < a.esc_ptr[lo + 1]; ++k) f(a.esc_val[k], static_cast<int64_t>(a.esc_col[k]));
        return;
    }
    if (a.fmt == SPMVC_FMT_ELL) {
        for (int k = 0; k < a.width; ++k) {
            const int64_t o = static_cast<int64_t>(k) * a.n_pad + row;
            const int32_t c = a.cols[o];
            if (c >= 0) f(a.ell_val[o], static_cast<int64_t>(c));
        }
        return;
    }
    // DT and DIT: canonical order, the value of position k from T, raw values after the coded ones
    const bool dit = a.fmt == SPMVC_FMT_DIT;
    const int32_t *pat = dit ? a.pat_off + static_cast<int64_t>(id) * a.width : nullptr;
    const int len = dit ? static_cast<int>(a.pat_len[id]) : a.width;
    auto column = [&](int k) -> int64_t {
        return dit ? row + pat[k] : static_cast<int64_t>(a.cols[static_cast<int64_t>(k) * a.n_pad + row]);
    };
    auto t_end = [&](int c) -> int {
        return a.pat_T ? a.pat_T[static_cast<int64_t>(id) * a.K + c] : a.T[static_cast<int64_t>(c) * a.n_pad + row];
    };
    int k = 0;
    for (int c = 0; c < a.K; ++c) {
        const int te = t_end(c);
        for (; k < te; ++k) f(a.V[c], column(k));
    }
    if (a.raw) {
        const int64_t rb = a.raw_slice[row / kSlice] + (row % kSlice) - static_cast<int64_t>(k) * kSlice;
        for (; k < len; ++k) {
            const int64_t j = column(k);
            if (!dit && j < 0) break;  // DT padding
            f(a.raw[rb + static_cast<int64_t>(k) * kSlice], j);
        }
    }
}

// Workgroups go to the 8 XCDs round-robin (block b on XCD b mod 8).  The
// logical block index below gives each XCD one contiguous run of the color's
// rows, which lie in a contiguous part of the grid, so the x lines that
// neighbouring blocks share are fetched into one XCD's L2 rather than several.
// A bijection of [0, gridDim.x): XCD k holds blocks k, k + 8, ..., and its run
// starts after the runs of XCDs 0..k-1.
__device__ inline int64_t xcd_block() {
    const unsigned nb = gridDim.x, bid = blockIdx.x;
    const unsigned xcd = bid % 8u, slot = bid / 8u, q = nb / 8u, r = nb % 8u;
    return static_cast<int64_t>(xcd) * q + (xcd < r ? xcd : r) + slot;
}

// The rows rows[0..n) of one color -- or, for a color-ordered matrix (rows
// null), the contiguous rows r0 .. r0 + n: x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii.
__global__ __launch_bounds__(kGsThreads) void k_symgs_color(GsArgs a, const int32_t *__restrict__ rows, int64_t r0,
                                                            int64_t n, const double *__restrict__ b, double *x,
                                                            const int *skip) {
    if (skip && *skip) return;
    const int64_t t = xcd_block() * kGsThreads + threadIdx.x;
    if (t >= n) return;
    const int64_t i = rows ? rows[t] : r0 + t;
    double s = 0.0, d = 0.0;
    gs_visit(a, i, [&](double v, int64_t j) {
        if (j == i)
            d = v;
        else
            s = fma(v, x[in_bounds<int64_t>(j, a.n_rows)], s);
    });
    x[i] = (b[i] - s) / d;
}

// The DIT form for a value table of at most two entries, no raw values and
// patterns of at most MAXW entries (the stencil case), without branches on
// the row's length: every lane issues its MAXW gathers at once (entries past
// the row's length read x_i and take weight 0), then the FMAs.  The generic
// loop above waits for each pattern offset and each gather in turn.
//
// A color launch is short (one eighth of the rows), so its time is its chain
// of dependent loads.  Everything that does not depend on the row's pattern
// is issued first, together: the row's pattern word and index, b_i, (TBL) the
// whole pattern table, which is then staged in LDS so that the offsets come
// from LDS rather than from a second global round trip, and last the done
// flag.  The chain is then: those loads, a barrier, the offsets, the gathers.
template <int MAXW, bool TBL>
__global__ __launch_bounds__(kGsThreads) void k_symgs_dit(GsArgs a, const int32_t *__restrict__ rows, int64_t r0,
                                                          const uint32_t *__restrict__ meta, int64_t n,
                                                          const double *__restrict__ b, double *x, const int *skip) {
    constexpr int kQ = kGsTblInts / kGsThreads;  // table words per thread
    __shared__ int32_t s_off[TBL ? kGsTblInts : 1];
    __shared__ uint8_t s_len[TBL ? kGsTblInts : 1];
    const int64_t t = xcd_block() * kGsThreads + threadIdx.x;
    const bool live = t < n;
    int64_t i = 0;
    uint32_t mw = 0;
    double bi = 0.0;
    if (live) {
        mw = meta[t];
        i = rows ? rows[t] : r0 + t;
        bi = b[i];
    }
    const int tn = a.P * a.width;
    int32_t tv[kQ];
    uint8_t lv[kQ];
    if constexpr (TBL) {
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const int k = q * kGsThreads + static_cast<int>(threadIdx.x);
            tv[q] = k < tn ? a.pat_off[k] : 0;
            lv[q] = k < a.P ? a.pat_len[k] : 0;
        }
    }
    // the flag last, so that waiting for it does not hold back the loads above
    const int done = skip ? *skip : 0;
    if constexpr (TBL) {
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const int k = q * kGsThreads + static_cast<int>(threadIdx.x);
            if (k < tn) s_off[k] = tv[q];
            if (k < a.P) s_len[k] = lv[q];
        }
        __syncthreads();
    }
    if (done || !live) return;
    const uint32_t id = mw & 0xFFFFFFu;
    double s = 0.0, d = 0.0;
    if (id == 0xFFFFFFu) {  // escape row
        gs_visit(a, i, [&](double v, int64_t j) {
            if (j == i)
                d = v;
            else
                s = fma(v, x[in_bounds<int64_t>(j, a.n_rows)], s);
        });
    } else {
        const int64_t pb = static_cast<int64_t>(id) * a.width;
        const int len = TBL ? s_len[in_bounds<int>(static_cast<int>(id), a.P)] : a.pat_len[id];
        const int t0 = a.K >= 2 ? static_cast<int>(mw >> 24) : len;
        int32_t off[MAXW];
#pragma unroll
        for (int k = 0; k < MAXW; ++k) {
            if (k >= a.width)
                off[k] = 0;
            else if constexpr (TBL)
                off[k] = s_off[in_bounds<int64_t>(pb + k, static_cast<int64_t>(tn))];
            else
                off[k] = a.pat_off[pb + k];
        }
        double xv[MAXW];
#pragma unroll
        for (int k = 0; k < MAXW; ++k) xv[k] = x[in_bounds<int64_t>(i + (k < len ? off[k] : 0), a.n_rows)];
#pragma unroll
        for (int k = 0; k < MAXW; ++k) {
            const double v = k < len ? (k < t0 ? a.V[0] : a.V[1]) : 0.0;
            const bool diag = k < len && off[k] == 0;
            d = diag ? v : d;
            s = diag ? s : fma(v, xv[k], s);
        }
    }
    x[i] = (bi - s) / d;
}

// meta[t] = (T_i[0] << 24) | ID of row rows[t] (ID 0xFFFFFF: escape row).
__global__ void k_gs_meta(GsArgs a, const int32_t *__restrict__ rows, int64_t n, uint32_t *meta) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kGsThreads + threadIdx.x;
    if (t >= n) return;
    const int64_t i = rows ? rows[t] : t;
    const uint32_t id = gs_id(a, i);
    const uint32_t esc = a.id_bytes == 1 ? 0xFFu : (a.id_bytes == 2 ? 0xFFFFu : 0xFFFFFFFFu);
    if (id == esc) {
        meta[t] = 0xFFFFFFu;
        return;
    }
    uint32_t t0 = 0;
    if (a.K >= 2) t0 = a.pat_T ? a.pat_T[static_cast<int64_t>(id) * a.K] : a.T[i];
    meta[t] = (t0 << 24) | id;
}

GsArgs gs_args(const spmvc_matrix_s *M) {
    GsArgs a{};
    a.n_rows = M->n_rows;
    a.n_pad = M->n_pad;
    a.fmt = M->fmt;
    a.K = M->K;
    a.width = M->width;
    a.id_bytes = M->id_bytes;
    a.ids = M->ids.p;
    a.T = M->T.as<uint8_t>();
    a.pat_T = M->fold ? M->pat_T.as<uint8_t>() : nullptr;
    a.pat_off = M->pat_off.as<int32_t>();
    a.pat_len = M->pat_len.as<uint8_t>();
    a.cols = M->fmt == SPMVC_FMT_ELL ? M->ell_col.as<int32_t>() : M->dt_S.as<int32_t>();
    a.ell_val = M->ell_val.as<double>();
    a.raw = M->raw_elems > 0 ? M->raw.as<double>() : nullptr;
    a.raw_slice = M->raw_slice.as<int64_t>();
    a.esc_rows = M->esc_rows.as<int64_t>();
    a.esc_ptr = M->esc_ptr.as<int64_t>();
    a.esc_col = M->esc_col.as<int32_t>();
    a.esc_val = M->esc_val.as<double>();
    a.n_esc = M->n_esc;
    a.P = static_cast<int32_t>(M->P);
    for (int c = 0; c < kMaxK; ++c) a.V[c] = M->V[c];
    a.bm_d = M->bm_d.as<int32_t>();
    a.bm_mask = M->bm_mask.p;
    a.bm_vmask = M->bm_vmask.p;
    a.bm_bytes = M->bm_bytes;
    return a;
}

// The branch-free DIT kernel applies: DIT/DITV, at most two table values, no
// raw values, patterns of at most 27 entries, IDs below 2^24.
bool gs_dit27(const spmvc_matrix_s *M) {
    return M->fmt == SPMVC_FMT_DIT && M->raw_elems == 0 && M->K <= 2 && M->width <= 27 && M->P > 0 &&
           M->P < 0xFFFFFF;
}

// Every row holds a non-zero diagonal entry (the last entry in column i
// decides, as in the decompressed CSR); otherwise *bad = 1.
__global__ void k_diag_check(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                             const double *__restrict__ val, int64_t n, int *bad) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool ok = false;
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
        if (col[k] == i) ok = val[k] != 0.0;
    if (!ok) *bad = 1;
}

// Greedy colors in row order over the pattern of A + A^T: each row takes the
// smallest color that no lower-numbered neighbour holds.  The neighbours
// j < i through A^T are the rows j < i that hold column i; instead of building
// A^T, each row, once colored, marks its color in a 64-bit mask of every
// higher-numbered column it holds, so that row i finds the colors of both
// kinds of neighbours in its own row and its mask.  Returns false (colors
// unset) when some row would need a 65th color.
bool greedy_colors_masks(int64_t n, const std::vector<int64_t> &rp, const std::vector<int32_t> &col,
                         std::vector<int32_t> &color, int32_t &n_colors) {
    std::vector<uint64_t> taken(n, 0);
    n_colors = 0;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t m = taken[i];
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            if (col[k] < i) m |= 1ull << color[col[k]];
        if (m == ~0ull) return false;
        const int32_t c = __builtin_ctzll(~m);
        color[i] = c;
        n_colors = std::max(n_colors, c + 1);
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            if (col[k] > i) taken[col[k]] |= 1ull << c;
    }
    return true;
}

// The same for any number of colors, through A^T's pattern.
void greedy_colors_any(int64_t n, const std::vector<int64_t> &rp, const std::vector<int32_t> &col,
                       std::vector<int32_t> &color, int32_t &n_colors) {
    const int64_t nnz = rp[n];
    std::vector<int64_t> tp(n + 1, 0);  // for each row, the rows that hold it as a column
    for (int64_t k = 0; k < nnz; ++k) ++tp[col[k] + 1];
    for (int64_t i = 0; i < n; ++i) tp[i + 1] += tp[i];
    std::vector<int32_t> tr(nnz);
    {
        std::vector<int64_t> fill(tp.begin(), tp.end() - 1);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t k = rp[i]; k < rp[i + 1]; ++k) tr[fill[col[k]]++] = static_cast<int32_t>(i);
    }
    std::vector<int64_t> mark(32, -1);
    n_colors = 0;
    for (int64_t i = 0; i < n; ++i) {
        auto take = [&](int64_t j) {
            if (j < i) {
                const int32_t c = color[j];
                if (c >= static_cast<int32_t>(mark.size())) mark.resize(2 * c + 2, -1);
                mark[c] = i;
            }
        };
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) take(col[k]);
        for (int64_t k = tp[i]; k < tp[i + 1]; ++k) take(tr[k]);
        int32_t c = 0;
        while (c < static_cast<int32_t>(mark.size()) && mark[c] == i) ++c;
        color[i] = c;
        n_colors = std::max(n_colors, c + 1);
    }
}

}  // namespace

// Greedy row-order coloring of the pattern of A + A^T, built once per handle;
// also checks (on the device) that every row holds a non-zero diagonal entry.
// The greedy pass is a sequential recurrence over the rows (each row's color
// depends on its lower-numbered neighbours' colors), so it runs on the host
// over the decompressed pattern; only row pointers and columns come back.
void build_coloring(spmvc_matrix_s *M, hipStream_t s) {
    if (M->gs_ready) return;
    if (M->n_rows != M->n_cols) throw Error{SPMVC_EINVAL, "Gauss-Seidel needs a square matrix"};
    const int64_t n = M->n_rows, nnz = M->nnz;
    std::vector<int64_t> rp(n + 1, 0);
    std::vector<int32_t> col(nnz);
    if (n > 0) {
        DevBuf drp, dcol, dval, dbad;
        drp.alloc(sizeof(int64_t) * (n + 1));
        dcol.alloc(sizeof(int32_t) * std::max<int64_t>(nnz, 1));
        dval.alloc(sizeof(double) * std::max<int64_t>(nnz, 1));
        dbad.alloc(sizeof(int));
        decompress(M, drp.as<int64_t>(), dcol.as<int32_t>(), dval.as<double>(), s);
        SPMVC_HIP(hipMemsetAsync(dbad.p, 0, sizeof(int), s));
        k_diag_check<<<grid_for(n, 256, 0x7fffffff), 256, 0, s>>>(drp.as<int64_t>(), dcol.as<int32_t>(),
                                                                  dval.as<double>(), n, dbad.as<int>());
        SPMVC_CHECK_LAUNCH();
        int bad = 0;
        SPMVC_HIP(hipMemcpyAsync(&bad, dbad.p, sizeof(int), hipMemcpyDeviceToHost, s));
        SPMVC_HIP(hipMemcpyAsync(rp.data(), drp.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, s));
        if (nnz > 0)
            SPMVC_HIP(hipMemcpyAsync(col.data(), dcol.p, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, s));
        SPMVC_HIP(hipStreamSynchronize(s));
        if (bad) throw Error{SPMVC_EINVAL, "Gauss-Seidel needs a non-zero diagonal entry in every row"};
    }
    std::vector<int32_t> color(n, 0);
    int32_t n_colors = 0;
    if (!greedy_colors_masks(n, rp, col, color, n_colors)) greedy_colors_any(n, rp, col, color, n_colors);
    // rows of each color, ascending
    M->gs_off.assign(n_colors + 1, 0);
    for (int64_t i = 0; i < n; ++i) ++M->gs_off[color[i] + 1];
    for (int c = 0; c < n_colors; ++c) M->gs_off[c + 1] += M->gs_off[c];
    std::vector<int32_t> rows(n);
    {
        std::vector<int64_t> fill(M->gs_off.begin(), M->gs_off.end() - 1);
        for (int64_t i = 0; i < n; ++i) rows[fill[color[i]]++] = static_cast<int32_t>(i);
    }
    M->gs_rows.alloc(sizeof(int32_t) * std::max<int64_t>(n, 1));
    M->gs_color.alloc(sizeof(int32_t) * std::max<int64_t>(n, 1));
    if (n > 0) {
        SPMVC_HIP(hipMemcpyAsync(M->gs_rows.p, rows.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
        SPMVC_HIP(hipMemcpyAsync(M->gs_color.p, color.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
        SPMVC_HIP(hipStreamSynchronize(s));
    }
    M->gs_n_colors = n_colors;
    if (gs_dit27(M) && n > 0) {
        M->gs_meta.alloc(sizeof(uint32_t) * n);
        k_gs_meta<<<grid_for(n, kGsThreads, 0x7fffffff), kGsThreads, 0, s>>>(gs_args(M), M->gs_rows.as<int32_t>(), n,
                                                                            M->gs_meta.as<uint32_t>());
        SPMVC_CHECK_LAUNCH();
        SPMVC_HIP(hipStreamSynchronize(s));
    }
    M->gs_ready = 1;
}

void launch_symgs(const spmvc_matrix_s *M, const double *b, double *x, int sweeps, hipStream_t s, const int *skip,
                  bool reverse) {
    const GsArgs a = gs_args(M);
    const int C = M->gs_n_colors;
    const int32_t *rows = M->gs_contig ? nullptr : M->gs_rows.as<int32_t>();
    const bool dit27 = gs_dit27(M);
    // the pattern table fits the LDS staging area
    const bool tbl = M->P * static_cast<int64_t>(M->width) <= kGsTblInts && M->P <= kGsTblInts;
    int last = -1;  // color of the previous launch
    for (int sw = 0; sw < sweeps; ++sw)
        for (int q = 0; q < 2 * C; ++q) {
            const int cq = q < C ? q : 2 * C - 1 - q;  // colors forward, then backward
            const int c = reverse ? C - 1 - cq : cq;      // or backward, then forward
            // Updating one color twice in a row repeats the same arithmetic on
            // unchanged neighbours (a color's rows read only other colors), so
            // the turn at the end of each half-sweep is launched once.
            if (c == last) continue;
            last = c;
            const int64_t r0 = M->gs_off[c], cnt = M->gs_off[c + 1] - r0;
            if (cnt == 0) continue;
            const unsigned g = grid_for(cnt, kGsThreads, 0x7fffffff);
            const int32_t *rc = rows ? rows + r0 : nullptr;
            if (dit27 && tbl)
                k_symgs_dit<27, true><<<g, kGsThreads, 0, s>>>(a, rc, r0, M->gs_meta.as<uint32_t>() + r0, cnt, b, x,
                                                               skip);
            else if (dit27)
                k_symgs_dit<27, false><<<g, kGsThreads, 0, s>>>(a, rc, r0, M->gs_meta.as<uint32_t>() + r0, cnt, b, x,
                                                                skip);
            else
                k_symgs_color<<<g, kGsThreads, 0, s>>>(a, rc, r0, cnt, b, x, skip);
            SPMVC_CHECK_LAUNCH();
        }
}

namespace {

// color[i] for the rows of color c: the ranges gs_off[c] .. gs_off[c+1]
__global__ void k_range_colors(const int64_t *off, int n_colors, int64_t n, int32_t *color) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = 0;
    while (c + 1 < n_colors && off[c + 1] <= i) ++c;
    color[i] = c;
}

// B = P A P^T with P = M's rows color by color, compressed with M's options,
// its coloring the ranges of M's colors.
std::unique_ptr<spmvc_matrix_s> make_color_twin(spmvc_matrix_s *M, hipStream_t s) {
    build_coloring(M, s);
    const int64_t n = M->n_rows, nnz = M->nnz;
    DevBuf rp, col, val, prp, pcol, pval;
    rp.alloc(sizeof(int64_t) * (n + 1));
    col.alloc(sizeof(int32_t) * std::max<int64_t>(nnz, 1));
    val.alloc(sizeof(double) * std::max<int64_t>(nnz, 1));
    prp.alloc(sizeof(int64_t) * (n + 1));
    pcol.alloc(sizeof(int32_t) * std::max<int64_t>(nnz, 1));
    pval.alloc(sizeof(double) * std::max<int64_t>(nnz, 1));
    decompress(M, rp.as<int64_t>(), col.as<int32_t>(), val.as<double>(), s);
    permute_csr(n, rp.as<int64_t>(), col.as<int32_t>(), val.as<double>(), M->gs_rows.as<int32_t>(),
                prp.as<int64_t>(), pcol.as<int32_t>(), pval.as<double>(), s);
    rp.release();
    col.release();
    val.release();
    std::unique_ptr<spmvc_matrix_s> T(new spmvc_matrix_s());
    T->n_rows = n;
    T->n_cols = n;
    T->nnz = nnz;
    compress(T.get(), prp.as<int64_t>(), pcol.as<int32_t>(), pval.as<double>(), M->copts, s);
    prepare_handle(T.get());
    // the induced coloring: color c is the contiguous range of M's color c
    T->gs_off = M->gs_off;
    T->gs_n_colors = M->gs_n_colors;
    T->gs_contig = 1;
    if (n > 0) {
        DevBuf off;
        off.alloc(sizeof(int64_t) * T->gs_off.size());
        SPMVC_HIP(hipMemcpyAsync(off.p, T->gs_off.data(), off.bytes, hipMemcpyHostToDevice, s));
        T->gs_color.alloc(sizeof(int32_t) * n);
        k_range_colors<<<grid_for(n, kGsThreads, 0x7fffffff), kGsThreads, 0, s>>>(
            off.as<int64_t>(), T->gs_n_colors, n, T->gs_color.as<int32_t>());
        SPMVC_CHECK_LAUNCH();
        if (gs_dit27(T.get())) {
            T->gs_meta.alloc(sizeof(uint32_t) * n);
            k_gs_meta<<<grid_for(n, kGsThreads, 0x7fffffff), kGsThreads, 0, s>>>(gs_args(T.get()), nullptr, n,
                                                                                T->gs_meta.as<uint32_t>());
            SPMVC_CHECK_LAUNCH();
        }
        SPMVC_HIP(hipStreamSynchronize(s));
    }
    T->gs_ready = 1;
    return T;
}

}  // namespace

spmvc_matrix_s *color_order_copy(spmvc_matrix_s *M, int32_t *perm, hipStream_t s) {
    std::unique_ptr<spmvc_matrix_s> T = make_color_twin(M, s);
    if (perm && M->n_rows > 0) {
        SPMVC_HIP(hipMemcpyAsync(perm, M->gs_rows.p, sizeof(int32_t) * M->n_rows, hipMemcpyDeviceToDevice, s));
        SPMVC_HIP(hipStreamSynchronize(s));
    }
    return T.release();
}

// bounds violations the kernels of this file recorded (checked builds)
SPMVC_CHECK_READER(check_violations_symgs)

}  // namespace spmvc
