// SpMV kernels: y = A x (Eq. 1) over the ELL, DT and DIT encodings.
//
// Layout (all streams column-major over rows, so a wavefront's 64 lanes read 64
// consecutive rows of one slot with one coalesced load):
//   ELL  col/val [width][n_pad]            (Section IV-B baseline, 12 B per slot)
//   DT   S [width][n_pad], T u8 [K][n_pad]  (value table + sorted columns, Fig. 1)
//   DIT  ID [n_pad], T u8 [K][n_pad]        (pattern ID + terminal indices)
// One lane owns one row.  A row's entries are consumed in the canonical order
// of Section V: first all entries of V[0] (positions < T[0]), then V[1], ...,
// then the raw FP64 entries; the value of a run is a wave-uniform scalar, so
// the decode costs one compare per entry.
//
// DIT with LDS staging: for a block of R consecutive rows [r0, r0+R) every
// displacement d of the pattern table reads x[r0+d .. r0+R-1+d].  The sorted
// set of displacements is cut into a few dense windows (for the 27-point stencil:
// one per z-plane), each window is loaded into LDS once with coalesced loads,
// and the pattern table is re-expressed as LDS element indices (uint16).  The
// gather x[row + d] -- the indirect access the paper names as its bottleneck --
// becomes an LDS read.
//
// Escape rows (plain CSR) are served by extra blocks appended to the same grid;
// the main blocks skip them (ID == all-ones, or column -2 in slot 0).
#include <algorithm>
#include <set>

#include "internal.h"

namespace spmvc {
namespace {

struct SpmvArgs {
    int64_t n_rows, n_cols, n_pad;
    int32_t K, width, P, raw_present;
    const void *ids;
    const uint8_t *T;
    const int32_t *pat_off;
    const uint8_t *pat_len;
    const int32_t *cols; // ELL col or DT S
    const double *ell_val;
    const void *raw;     // f64 or f32 by kernel dtype
    const int64_t *raw_slice;
    const int64_t *esc_rows, *esc_ptr;
    const int32_t *esc_col;
    const void *esc_val; // f64 or f32 by kernel dtype
    int64_t n_esc;
    unsigned n_main_blocks;
    const int *skip; // optional: when *skip != 0 the launch does nothing (solver done)
    double V[kMaxK];
    float V32[kMaxK];
    // LDS plan (DIT)
    int32_t rows, n_win, lds_total;
    int64_t win_lo[kMaxWindows];
    int32_t win_len[kMaxWindows];
    int32_t win_base[kMaxWindows];
    const uint16_t *tab; // [P][width+1]: len, then LDS indices
    int32_t tab_elems;
};

template <class Real> __device__ __forceinline__ Real vtab(const SpmvArgs &a, int c);
template <> __device__ __forceinline__ double vtab<double>(const SpmvArgs &a, int c) { return a.V[c]; }
template <> __device__ __forceinline__ float vtab<float>(const SpmvArgs &a, int c) { return a.V32[c]; }

template <class T> __device__ __forceinline__ T ldg_stream(const T *p) {
    return __builtin_nontemporal_load(p);
}

// One escape row per thread: plain CSR, columns ascending.
template <class Real, int NR>
__device__ __forceinline__ void escape_row(const SpmvArgs &a, int64_t e, int nrhs, const Real *__restrict__ x,
                                           int64_t ldx, Real *__restrict__ y, int64_t ldy) {
    if (e >= a.n_esc) return;
    const int64_t row = a.esc_rows[e];
    const Real *ev = static_cast<const Real *>(a.esc_val);
    Real acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = Real(0);
    for (int64_t k = a.esc_ptr[e]; k < a.esc_ptr[e + 1]; ++k) {
        const Real v = ev[k];
        const Real *xp = x + static_cast<int64_t>(a.esc_col[k]) * ldx;
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if (NR == 1 || r < nrhs) acc[r] = fma(v, xp[r], acc[r]);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if (NR == 1 || r < nrhs) y[row * ldy + r] = acc[r];
}

template <class IdT> __device__ __forceinline__ constexpr IdT esc_id() { return static_cast<IdT>(~static_cast<IdT>(0)); }

// ---- direct-gather kernel: every format, 1..16 right-hand sides --------------------
// FMT: SPMVC_FMT_ELL / DT / DIT.  NR: compile-time RHS capacity (runtime nrhs <= NR).
template <int FMT, class Real, class IdT, bool RAW, int NR>
__global__ __launch_bounds__(kBlock) void k_spmv_direct(SpmvArgs a, int nrhs, const Real *__restrict__ x,
                                                         int64_t ldx, Real *__restrict__ y, int64_t ldy) {
    if (a.skip && *a.skip) return;
    if (blockIdx.x >= a.n_main_blocks) {
        escape_row<Real, NR>(a, static_cast<int64_t>(blockIdx.x - a.n_main_blocks) * kBlock + threadIdx.x, nrhs, x,
                             ldx, y, ldy);
        return;
    }
    const int64_t row = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (row >= a.n_rows) return;
    Real acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = Real(0);

    auto apply = [&](Real v, int64_t j) {
        const Real *xp = x + j * ldx;
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if (NR == 1 || r < nrhs) acc[r] = fma(v, xp[r], acc[r]);
    };

    if constexpr (FMT == SPMVC_FMT_ELL) {
        if (a.cols[row] == kEscapeColumn) return;
        for (int k = 0; k < a.width; ++k) {
            const int64_t o = static_cast<int64_t>(k) * a.n_pad + row;
            const int32_t c = ldg_stream(a.cols + o);
            if (c < 0) break;
            apply(static_cast<Real>(ldg_stream(a.ell_val + o)), c);
        }
    } else {
        const int32_t *pat = nullptr;
        int len = 0;
        if constexpr (FMT == SPMVC_FMT_DIT) {
            const IdT id = static_cast<const IdT *>(a.ids)[row];
            if (id == esc_id<IdT>()) return;
            pat = a.pat_off + static_cast<int64_t>(id) * a.width;
            len = a.pat_len[id];
        } else {
            if (a.cols[row] == kEscapeColumn) return;
            len = a.width;
        }
        auto column = [&](int k) -> int64_t {
            if constexpr (FMT == SPMVC_FMT_DIT)
                return row + pat[k];
            else
                return ldg_stream(a.cols + static_cast<int64_t>(k) * a.n_pad + row);
        };
        int k = 0;
        for (int c = 0; c < a.K; ++c) {
            const int tend = a.T[static_cast<int64_t>(c) * a.n_pad + row];
            const Real v = vtab<Real>(a, c);
            for (; k < tend; ++k) apply(v, column(k));
        }
        if constexpr (RAW) {
            const Real *raw = static_cast<const Real *>(a.raw);
            const int64_t rb = a.raw_slice[row / kSlice] + (row % kSlice) - static_cast<int64_t>(k) * kSlice;
            for (; k < len; ++k) {
                const int64_t j = column(k);
                if (FMT == SPMVC_FMT_DT && j < 0) break;
                apply(ldg_stream(raw + rb + static_cast<int64_t>(k) * kSlice), j);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if (NR == 1 || r < nrhs) y[row * ldy + r] = acc[r];
}

// ---- DIT with x windows staged in LDS (single right-hand side) ----------------------
template <class Real, class IdT, bool RAW, bool TAB_LDS>
__global__ __launch_bounds__(kBlock) void k_dit_lds(SpmvArgs a, const Real *__restrict__ x, Real *__restrict__ y) {
    if (a.skip && *a.skip) return;
    if (blockIdx.x >= a.n_main_blocks) {
        escape_row<Real, 1>(a, static_cast<int64_t>(blockIdx.x - a.n_main_blocks) * kBlock + threadIdx.x, 1, x, 1, y, 1);
        return;
    }
    extern __shared__ __align__(16) unsigned char smem[];
    Real *xs = reinterpret_cast<Real *>(smem);
    uint16_t *tab_s = reinterpret_cast<uint16_t *>(smem + sizeof(Real) * a.lds_total);
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * a.rows;
    for (int w = 0; w < a.n_win; ++w) {
        const int64_t g0 = r0 + a.win_lo[w];
        Real *dst = xs + a.win_base[w];
        const int n = a.win_len[w];
        for (int e = threadIdx.x; e < n; e += kBlock) {
            const int64_t g = g0 + e;
            dst[e] = (g >= 0 && g < a.n_cols) ? x[g] : Real(0);
        }
    }
    if constexpr (TAB_LDS) {
        for (int e = threadIdx.x; e < a.tab_elems; e += kBlock) tab_s[e] = a.tab[e];
    }
    __syncthreads();
    const uint16_t *tab = TAB_LDS ? tab_s : a.tab;
    const int tw = a.width + 1;
    for (int rel = threadIdx.x; rel < a.rows; rel += kBlock) {
        const int64_t row = r0 + rel;
        if (row >= a.n_rows) break;
        const IdT id = static_cast<const IdT *>(a.ids)[row];
        if (id == esc_id<IdT>()) continue;
        const uint16_t *t = tab + static_cast<int64_t>(id) * tw + 1;
        const Real *xr = xs + rel;
        Real acc = Real(0);
        int k = 0;
        for (int c = 0; c < a.K; ++c) {
            const int tend = a.T[static_cast<int64_t>(c) * a.n_pad + row];
            const Real v = vtab<Real>(a, c);
            for (; k < tend; ++k) acc = fma(v, xr[t[k]], acc);
        }
        if constexpr (RAW) {
            const int len = t[-1];
            const Real *raw = static_cast<const Real *>(a.raw);
            const int64_t rb = a.raw_slice[row / kSlice] + (row % kSlice) - static_cast<int64_t>(k) * kSlice;
            for (; k < len; ++k) acc = fma(ldg_stream(raw + rb + static_cast<int64_t>(k) * kSlice), xr[t[k]], acc);
        }
        y[row] = acc;
    }
}

template <class Real> SpmvArgs make_args(const spmvc_matrix_s *M, const int *skip) {
    SpmvArgs a{};
    a.skip = skip;
    a.n_rows = M->n_rows;
    a.n_cols = M->n_cols;
    a.n_pad = M->n_pad;
    a.K = M->K;
    a.width = M->width;
    a.P = M->P;
    a.raw_present = M->raw_elems > 0;
    a.ids = M->ids.p;
    a.T = M->T.as<uint8_t>();
    a.pat_off = M->pat_off.as<int32_t>();
    a.pat_len = M->pat_len.as<uint8_t>();
    a.cols = M->fmt == SPMVC_FMT_ELL ? M->ell_col.as<int32_t>() : M->dt_S.as<int32_t>();
    a.ell_val = M->ell_val.as<double>();
    const bool f32 = std::is_same<Real, float>::value;
    a.raw = f32 ? M->raw32.p : M->raw.p;
    a.raw_slice = M->raw_slice.as<int64_t>();
    a.esc_rows = M->esc_rows.as<int64_t>();
    a.esc_ptr = M->esc_ptr.as<int64_t>();
    a.esc_col = M->esc_col.as<int32_t>();
    a.esc_val = f32 ? M->esc_val32.p : M->esc_val.p;
    a.n_esc = M->n_esc;
    for (int c = 0; c < kMaxK; ++c) {
        a.V[c] = M->V[c];
        a.V32[c] = M->V32[c];
    }
    return a;
}

unsigned escape_blocks(const spmvc_matrix_s *M) {
    return static_cast<unsigned>((M->n_esc + kBlock - 1) / kBlock);
}

template <class Real, int NR>
void launch_direct_nr(const spmvc_matrix_s *M, SpmvArgs a, int nrhs, const void *x, int64_t ldx, void *y,
                      int64_t ldy, hipStream_t s) {
    a.n_main_blocks = static_cast<unsigned>(M->n_pad / kBlock + (M->n_pad % kBlock ? 1 : 0));
    const unsigned grid = a.n_main_blocks + escape_blocks(M);
    if (grid == 0) return;
    const Real *xp = static_cast<const Real *>(x);
    Real *yp = static_cast<Real *>(y);
    const bool raw = M->raw_elems > 0;
    if (M->fmt == SPMVC_FMT_ELL) {
        k_spmv_direct<SPMVC_FMT_ELL, Real, uint8_t, false, NR><<<grid, kBlock, 0, s>>>(a, nrhs, xp, ldx, yp, ldy);
    } else if (M->fmt == SPMVC_FMT_DT) {
        if (raw)
            k_spmv_direct<SPMVC_FMT_DT, Real, uint8_t, true, NR><<<grid, kBlock, 0, s>>>(a, nrhs, xp, ldx, yp, ldy);
        else
            k_spmv_direct<SPMVC_FMT_DT, Real, uint8_t, false, NR><<<grid, kBlock, 0, s>>>(a, nrhs, xp, ldx, yp, ldy);
    } else {
#define SPMVC_DIT_DIRECT(IDT)                                                                                 \
    if (raw)                                                                                                  \
        k_spmv_direct<SPMVC_FMT_DIT, Real, IDT, true, NR><<<grid, kBlock, 0, s>>>(a, nrhs, xp, ldx, yp, ldy);  \
    else                                                                                                      \
        k_spmv_direct<SPMVC_FMT_DIT, Real, IDT, false, NR><<<grid, kBlock, 0, s>>>(a, nrhs, xp, ldx, yp, ldy);
        if (M->id_bytes == 1) {
            SPMVC_DIT_DIRECT(uint8_t)
        } else if (M->id_bytes == 2) {
            SPMVC_DIT_DIRECT(uint16_t)
        } else {
            SPMVC_DIT_DIRECT(uint32_t)
        }
#undef SPMVC_DIT_DIRECT
    }
    SPMVC_CHECK_LAUNCH();
}

template <class Real>
void launch_lds(const spmvc_matrix_s *M, SpmvArgs a, const void *x, void *y, hipStream_t s) {
    const LdsPlan &p = M->plan;
    a.rows = p.rows;
    a.n_win = p.n_win;
    a.lds_total = p.total;
    for (int w = 0; w < p.n_win; ++w) {
        a.win_lo[w] = p.lo[w];
        a.win_len[w] = p.len[w];
        a.win_base[w] = p.base[w];
    }
    a.tab = p.tab.as<uint16_t>();
    a.tab_elems = M->P * (M->width + 1);
    a.n_main_blocks = static_cast<unsigned>((M->n_rows + p.rows - 1) / p.rows);
    const unsigned grid = a.n_main_blocks + escape_blocks(M);
    size_t shmem = sizeof(Real) * static_cast<size_t>(p.total);
    if (p.tab_in_lds) shmem += sizeof(uint16_t) * static_cast<size_t>(a.tab_elems) + 16;
    const Real *xp = static_cast<const Real *>(x);
    Real *yp = static_cast<Real *>(y);
    const bool raw = M->raw_elems > 0;
#define SPMVC_LDS(IDT)                                                                                \
    if (raw) {                                                                                        \
        if (p.tab_in_lds)                                                                             \
            k_dit_lds<Real, IDT, true, true><<<grid, kBlock, shmem, s>>>(a, xp, yp);                 \
        else                                                                                          \
            k_dit_lds<Real, IDT, true, false><<<grid, kBlock, shmem, s>>>(a, xp, yp);                \
    } else {                                                                                          \
        if (p.tab_in_lds)                                                                             \
            k_dit_lds<Real, IDT, false, true><<<grid, kBlock, shmem, s>>>(a, xp, yp);                \
        else                                                                                          \
            k_dit_lds<Real, IDT, false, false><<<grid, kBlock, shmem, s>>>(a, xp, yp);               \
    }
    if (M->id_bytes == 1) {
        SPMVC_LDS(uint8_t)
    } else if (M->id_bytes == 2) {
        SPMVC_LDS(uint16_t)
    } else {
        SPMVC_LDS(uint32_t)
    }
#undef SPMVC_LDS
    SPMVC_CHECK_LAUNCH();
}

template <class Real>
void launch_block_t(const spmvc_matrix_s *M, int nrhs, const void *X, int64_t ldx, void *Y, int64_t ldy,
                    hipStream_t s, const int *skip) {
    SpmvArgs a = make_args<Real>(M, skip);
    if (nrhs == 1)
        launch_direct_nr<Real, 1>(M, a, 1, X, ldx, Y, ldy, s);
    else if (nrhs <= 4)
        launch_direct_nr<Real, 4>(M, a, nrhs, X, ldx, Y, ldy, s);
    else if (nrhs <= 8)
        launch_direct_nr<Real, 8>(M, a, nrhs, X, ldx, Y, ldy, s);
    else
        launch_direct_nr<Real, 16>(M, a, nrhs, X, ldx, Y, ldy, s);
}

template <class Real>
void launch_spmv_t(const spmvc_matrix_s *M, const void *x, void *y, hipStream_t s, const int *skip) {
    if (M->n_rows == 0) return;
    if (M->fmt == SPMVC_FMT_DIT && M->lds_mode == 1 && M->plan.n_win > 0 && M->P > 0) {
        launch_lds<Real>(M, make_args<Real>(M, skip), x, y, s);
        return;
    }
    launch_block_t<Real>(M, 1, x, 1, y, 1, s, skip);
}

}  // namespace

// Cut the displacement set into dense windows for `rows` rows per block.
void build_lds_plan(spmvc_matrix_s *M, int rows) {
    LdsPlan &p = M->plan;
    p.tab.release();
    p.rows = rows;
    p.n_win = 0;
    p.total = 0;
    p.tab_in_lds = false;
    if (M->fmt != SPMVC_FMT_DIT || M->P == 0 || M->width == 0) return;
    const int W = M->width;
    std::set<int64_t> ds;
    for (int q = 0; q < M->P; ++q)
        for (int k = 0; k < M->h_pat_len[q]; ++k) ds.insert(M->h_pat_off[static_cast<size_t>(q) * W + k]);
    if (ds.empty()) return;
    // Two windows merge when the gap between them is below `rows`: a separate
    // window costs `rows` more LDS elements than the gap it skips.
    std::vector<std::pair<int64_t, int64_t>> win;
    for (int64_t d : ds) {
        if (!win.empty() && d - win.back().second <= rows)
            win.back().second = d;
        else
            win.push_back({d, d});
    }
    if (static_cast<int>(win.size()) > kMaxWindows) return;
    int64_t total = 0;
    int64_t lo[kMaxWindows], base[kMaxWindows], len[kMaxWindows];
    for (size_t w = 0; w < win.size(); ++w) {
        lo[w] = win[w].first;
        len[w] = rows + win[w].second - win[w].first;
        base[w] = total;
        total += len[w];
    }
    if (total * static_cast<int64_t>(sizeof(double)) > kLdsBudgetBytes || total > 65535) return;
    const int64_t tab_bytes = static_cast<int64_t>(M->P) * (W + 1) * static_cast<int64_t>(sizeof(uint16_t));
    std::vector<uint16_t> tab(static_cast<size_t>(M->P) * (W + 1), 0);
    for (int q = 0; q < M->P; ++q) {
        const int L = M->h_pat_len[q];
        tab[static_cast<size_t>(q) * (W + 1)] = static_cast<uint16_t>(L);
        for (int k = 0; k < L; ++k) {
            const int64_t d = M->h_pat_off[static_cast<size_t>(q) * W + k];
            size_t w = 0;
            while (!(d >= win[w].first && d <= win[w].second)) ++w;
            tab[static_cast<size_t>(q) * (W + 1) + 1 + k] = static_cast<uint16_t>(base[w] + d - lo[w]);
        }
    }
    p.tab.alloc(sizeof(uint16_t) * tab.size());
    SPMVC_HIP(hipMemcpy(p.tab.p, tab.data(), p.tab.bytes, hipMemcpyHostToDevice));
    p.tab_in_lds = tab_bytes <= 16 * 1024 && total * 8 + tab_bytes + 16 <= kLdsBudgetBytes;
    for (size_t w = 0; w < win.size(); ++w) {
        p.lo[w] = lo[w];
        p.len[w] = static_cast<int32_t>(len[w]);
        p.base[w] = static_cast<int32_t>(base[w]);
    }
    p.total = static_cast<int32_t>(total);
    p.n_win = static_cast<int>(win.size());
}

void launch_spmv(const spmvc_matrix_s *M, int dt, const void *x, void *y, hipStream_t s, const int *skip) {
    if (dt == SPMVC_F64)
        launch_spmv_t<double>(M, x, y, s, skip);
    else
        launch_spmv_t<float>(M, x, y, s, skip);
}

void launch_spmv_block(const spmvc_matrix_s *M, int dt, int nrhs, const void *X, int64_t ldx, void *Y,
                       int64_t ldy, hipStream_t s, const int *skip) {
    if (M->n_rows == 0) return;
    if (dt == SPMVC_F64)
        launch_block_t<double>(M, nrhs, X, ldx, Y, ldy, s, skip);
    else
        launch_block_t<float>(M, nrhs, X, ldx, Y, ldy, s, skip);
}

// Bytes of the matrix encoding one spmv of dtype dt reads (vectors excluded).
int64_t stream_bytes(const spmvc_matrix_s *M, int dt) {
    const int64_t vb = dt == SPMVC_F64 ? 8 : 4;
    int64_t b = 0;
    const int64_t slots = static_cast<int64_t>(M->width) * M->n_pad;
    if (M->fmt == SPMVC_FMT_ELL) {
        b += slots * (4 + 8);
    } else {
        b += static_cast<int64_t>(M->K) * M->n_pad;            // T
        b += M->raw_elems * vb;                               // raw values
        if (M->raw_elems) b += 8 * (M->n_pad / kSlice + 1);   // slice pointers
        if (M->fmt == SPMVC_FMT_DT)
            b += slots * 4;                                   // S
        else
            b += static_cast<int64_t>(M->id_bytes) * M->n_pad + static_cast<int64_t>(M->P) * (M->width + 1) * 2;
    }
    b += M->n_esc_nnz * (4 + vb) + M->n_esc * 16;
    return b;
}

}  // namespace spmvc
