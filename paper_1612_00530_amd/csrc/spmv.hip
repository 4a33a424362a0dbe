// SpMV kernels: y = A x (Eq. 1) over the ELL, DT, DIT and DITV encodings.
//
// Layout (all streams column-major over rows, so a wavefront's 64 lanes read 64
// consecutive rows of one slot with one coalesced load):
//   ELL  col/val [width][n_pad]            (Section IV-B baseline, 12 B per slot)
//   DT   S [width][n_pad], T u8 [K][n_pad]  (value table + sorted columns, Fig. 1)
//   DIT  ID [n_pad], T u8 [K][n_pad]        (pattern ID + terminal indices)
//   DITV ID [n_pad]                         (values registered in the table too:
//                                            T per pattern, pat_T [P][K]; row_T)
// In the single-vector kernels one lane owns one row.  A row's entries are
// consumed in the canonical order of Section V: first all entries of V[0]
// (positions < T[0]), then V[1], ..., then the raw FP64 entries.
//
// DIT with LDS staging: for a block of R consecutive rows [r0, r0+R) every
// displacement d of the pattern table reads x[r0+d .. r0+R-1+d].  The sorted
// set of displacements is cut into a few dense windows (for the 27-point stencil:
// one per z-plane), each window is loaded into LDS once with coalesced loads,
// and the pattern table is re-expressed as LDS offsets (uint16).  The gather
// x[row + d] -- the indirect access the paper names as its bottleneck --
// becomes an LDS read.
//
// The register kernel (k_dit_reg) holds a row's whole pattern (at most 31
// entries, 64 bytes of LDS offsets) in registers, so its LDS reads are
// independent and issue back to back.  Per entry it costs one add (offset +
// row), one LDS read and one add (one FMA where the value must be selected per
// lane).  Entries past a row's length (rows shorter than the table width) read
// zeros (exact when every table value is finite): in FP64 they carry the
// offset 0xFFFF and the kernel reads min(row + offset, Z), Z a single zero
// element after the windows -- one more VALU operation per entry instead of a
// zero window of one element per row, a fifth of the block's LDS, so that more
// blocks are resident; FP32 (and the marching form) keep the zero window.  With
// every value raw, a row's values are read up to its 64-row slice's width
// (zero padding).
// k_dit_march is its plane-marching form: a block walks one row tile through
// consecutive planes and stages one new window per step.
//
// Several right-hand sides (row-interleaved blocks): k_dit_block_win holds
// whole rows of one window at a time in LDS; k_dit_reg_pairs the windows of
// one right-hand-side pair; k_spmv_lanes gathers through the caches with a
// group of lanes per row.
//
// Escape rows (plain CSR) are served by extra blocks appended to the same grid
// (or a launch of their own); the main blocks skip them (ID == all-ones, or
// column -2 in slot 0).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <set>

#include "check.h"
#include "internal.h"
#include "lds_window.h"
#include "reduce.h"

namespace spmvc {
namespace {

struct SpmvArgs {
    int64_t n_rows, n_cols, n_pad;
    int32_t K, width, P, raw_present, id_bytes;
    const void *ids;
    const uint8_t *T;
    const uint8_t *pat_T;  // DITV: T of each pattern [P][K] (the rows keep none), else null
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
    double *dot;     // optional: per-block partial of x.y (x at the row, y the result), FP64
    double V[kMaxK];
    float V32[kMaxK];
    // LDS plan (DIT)
    int32_t rows, n_win, lds_total;
    int64_t win_lo[kMaxWindows];
    int32_t win_len[kMaxWindows];
    int32_t win_base[kMaxWindows];
    const uint16_t *tab; // [P][width+1]: len, then LDS element indices
    int32_t tab_elems;
    int32_t zero_base, zero_len;   // zeros after the windows: one element (FP64 register kernel) or
                                   // one per row (the other register-table kernels)
    const uint16_t *reg_tab;       // [P][kRegTw]: len, then LDS byte offsets
    int32_t lds_x_bytes;           // bytes of the windows (+ zero window), 16-byte multiple
    int32_t n_xcd;                 // XCDs the blocks are spread over (tile mapping)
    int32_t async_lds;             // x is 16-byte aligned: stage windows with direct LDS loads
    int32_t bw_split;              // window-phased block SpMV: records split into value runs
    // plane-marching kernel (k_dit_march)
    int64_t m_S;                   // row distance between consecutive windows (one plane)
    int64_t m_nz;                  // planes: ceil(n_rows / m_S)
    int64_t m_lo0;                 // start of window 0 relative to the tile's first row
    int32_t m_np;                  // row tiles per plane
    int32_t m_C;                   // planes per block
    int32_t m_L;                   // elements per window buffer
    int32_t m_NB;                  // window buffers in the ring (windows + 1)
    int32_t m_NW;                  // windows a tile reads
    // neighbour-bitmask format: displacement list, masks, LDS offsets
    const int32_t *bm_d;
    const void *bm_mask, *bm_vmask;
    int32_t bm_nd;
    int32_t bm_off[64];            // element offset of D[k] in the windows (LDS kernel)
    int32_t self_off;              // register kernel: byte offset (from the row's slot) of the
                                   // row's own x in the windows, -1 when no window holds it
};

template <class Real> __device__ __forceinline__ Real vtab(const SpmvArgs &a, int c);
template <> __device__ __forceinline__ double vtab<double>(const SpmvArgs &a, int c) { return a.V[c]; }
template <> __device__ __forceinline__ float vtab<float>(const SpmvArgs &a, int c) { return a.V32[c]; }

// T_i[c] of a non-escape row: its own byte of the T stream, or -- values
// registered in the pattern table (DITV) -- its pattern's.
__device__ __forceinline__ int row_T(const SpmvArgs &a, int c, int64_t row, uint32_t id) {
    return a.pat_T ? a.pat_T[static_cast<int64_t>(id) * a.K + c] : a.T[static_cast<int64_t>(c) * a.n_pad + row];
}

template <class T> __device__ __forceinline__ T ldg_stream(const T *p) {
    return __builtin_nontemporal_load(p);
}

// Writes the block's partial of x.y when the launch asks for it (all threads call).
__device__ __forceinline__ void emit_dot(const SpmvArgs &a, double part) {
    if (!a.dot) return;
    const double b = block_sum<kBlock>(part);
    if (threadIdx.x == 0) a.dot[blockIdx.x] = b;
}

// The same with the wavefront sums in the caller's LDS (a buffer it is done with).
__device__ __forceinline__ void emit_dot(const SpmvArgs &a, double part, double *sh) {
    if (!a.dot) return;
    const double b = block_sum<kBlock>(part, sh);
    if (threadIdx.x == 0) a.dot[blockIdx.x] = b;
}

// One escape row per thread: plain CSR, columns ascending.  Returns x_row * y_row
// (first right-hand side) for the optional dot product.
template <class Real, int NR>
__device__ __forceinline__ double escape_row(const SpmvArgs &a, int64_t e, int nrhs, const Real *__restrict__ x,
                                             int64_t ldx, Real *__restrict__ y, int64_t ldy) {
    if (e >= a.n_esc) return 0.0;
    const int64_t row = a.esc_rows[e];
    const Real *ev = static_cast<const Real *>(a.esc_val);
    Real acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = Real(0);
    for (int64_t k = a.esc_ptr[e]; k < a.esc_ptr[e + 1]; ++k) {
        const Real v = ev[k];
        const Real *xp = x + in_bounds<int64_t>(a.esc_col[k], a.n_cols) * ldx;
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if (NR == 1 || r < nrhs) acc[r] = fma(v, xp[r], acc[r]);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if (NR == 1 || r < nrhs) y[row * ldy + r] = acc[r];
    return a.dot ? static_cast<double>(x[row * ldx]) * static_cast<double>(acc[0]) : 0.0;
}

template <class IdT> __device__ __forceinline__ constexpr IdT esc_id() { return static_cast<IdT>(~static_cast<IdT>(0)); }

// Row tile of block `bid` among `nb` tiles.  Blocks are dispatched round-robin
// over the XCDs (bid % n_xcd); each XCD is given a contiguous run of tiles so
// that neighbouring tiles, whose x windows overlap, share that XCD's L2.
__device__ __forceinline__ int64_t xcd_tile(unsigned bid, unsigned nb, int n_xcd) {
    if (n_xcd <= 1 || nb < static_cast<unsigned>(n_xcd)) return bid;
    const unsigned q = nb / n_xcd, r = nb % n_xcd;
    const unsigned xcd = bid % n_xcd, j = bid / n_xcd;
    return static_cast<int64_t>(xcd) * q + min(xcd, r) + j;
}

template <int FMT, class Real, class IdT, bool RAW, int NR>
__device__ __forceinline__ double direct_row(const SpmvArgs &a, int64_t row, int nrhs, const Real *__restrict__ x,
                                             int64_t ldx, Real *__restrict__ y, int64_t ldy);

// ---- direct-gather kernel: every format, 1..16 right-hand sides --------------------
// FMT: SPMVC_FMT_ELL / DT / DIT.  NR: compile-time RHS capacity (runtime nrhs <= NR).
template <int FMT, class Real, class IdT, bool RAW, int NR>
__global__ __launch_bounds__(kBlock) void k_spmv_direct(SpmvArgs a, int nrhs, const Real *__restrict__ x,
                                                         int64_t ldx, Real *__restrict__ y, int64_t ldy) {
    if (a.skip && *a.skip) return;
    if (blockIdx.x >= a.n_main_blocks) {
        emit_dot(a, escape_row<Real, NR>(a, static_cast<int64_t>(blockIdx.x - a.n_main_blocks) * kBlock + threadIdx.x,
                                         nrhs, x, ldx, y, ldy));
        return;
    }
    const int64_t row = xcd_tile(blockIdx.x, a.n_main_blocks, a.n_xcd) * kBlock + threadIdx.x;
    double dotc = 0.0;
    if (row < a.n_rows) dotc = direct_row<FMT, Real, IdT, RAW, NR>(a, row, nrhs, x, ldx, y, ldy);
    emit_dot(a, dotc);
}

// One row of the direct kernel; returns x_row * y_row (first right-hand side).
template <int FMT, class Real, class IdT, bool RAW, int NR>
__device__ __forceinline__ double direct_row(const SpmvArgs &a, int64_t row, int nrhs, const Real *__restrict__ x,
                                             int64_t ldx, Real *__restrict__ y, int64_t ldy) {
    Real acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = Real(0);

    auto apply = [&](Real v, int64_t j) {
        const Real *xp = x + in_bounds<int64_t>(j, a.n_cols) * ldx;
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if (NR == 1 || r < nrhs) acc[r] = fma(v, xp[r], acc[r]);
    };

    if constexpr (FMT == SPMVC_FMT_ELL) {
        if (a.cols[row] == kEscapeColumn) return 0.0;
        // Slots are read four at a time with no data-dependent exit, so the
        // column and value loads of a group are all in flight together.
        int k = 0;
        for (; k + 4 <= a.width; k += 4) {
            int32_t c[4];
            double v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t o = static_cast<int64_t>(k + j) * a.n_pad + row;
                c[j] = ldg_stream(a.cols + o);
                v[j] = ldg_stream(a.ell_val + o);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (c[j] >= 0) apply(static_cast<Real>(v[j]), c[j]);
        }
        for (; k < a.width; ++k) {
            const int64_t o = static_cast<int64_t>(k) * a.n_pad + row;
            const int32_t c = ldg_stream(a.cols + o);
            if (c >= 0) apply(static_cast<Real>(ldg_stream(a.ell_val + o)), c);
        }
    } else if constexpr (FMT == SPMVC_FMT_BMASK) {
        // set bits of the row's mask in ascending order = its columns ascending;
        // IdT is the mask type
        IdT m = static_cast<const IdT *>(a.bm_mask)[row];
        const IdT vm = a.K == 2 ? static_cast<const IdT *>(a.bm_vmask)[row] : IdT(0);
        const Real *raw = static_cast<const Real *>(a.raw);
        const int64_t rb = RAW ? a.raw_slice[row / kSlice] + (row % kSlice) : 0;
        for (int j = 0; m; ++j) {
            const int k = static_cast<int>(__builtin_ctzll(static_cast<uint64_t>(m)));
            m &= m - 1;
            const Real v = RAW ? ldg_stream(raw + rb + static_cast<int64_t>(j) * kSlice)
                               : vtab<Real>(a, a.K == 2 ? static_cast<int>((vm >> k) & 1) : 0);
            apply(v, row + a.bm_d[k]);
        }
    } else {
        const int32_t *pat = nullptr;
        int len = 0;
        uint32_t pid = 0;
        if constexpr (FMT == SPMVC_FMT_DIT) {
            const IdT id = static_cast<const IdT *>(a.ids)[row];
            pid = id;
            if (id == esc_id<IdT>()) return 0.0;
            pat = a.pat_off + static_cast<int64_t>(id) * a.width;
            len = a.pat_len[id];
        } else {
            if (a.cols[row] == kEscapeColumn) return 0.0;
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
            const int tend = row_T(a, c, row, pid);
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
    return a.dot ? static_cast<double>(x[row * ldx]) * static_cast<double>(acc[0]) : 0.0;
}

// Load the block's x windows (and a zero window, if any) into LDS.  Each window is a
// contiguous range of x.  Interior windows are copied with direct
// global-to-LDS loads (16 bytes per lane, no register round trip), so every
// load of the block is in flight at once; windows that reach past either end
// of x (first and last blocks), or an x that is not 16-byte aligned, take the
// register path with clamped indices (a window slot outside [0, n_cols) is
// never read by a stored entry).  Window starts and lengths are multiples of
// four elements, so each 16-byte chunk lies wholly inside its window.
// Issues the copies of the block's x windows for rows [r0, r0 + rows) into xs.
// Direct loads are left in flight (the caller waits for them); the register
// path (edge windows, unaligned x) has completed its LDS stores on return.
template <class Real>
__device__ __forceinline__ void stage_windows_async(const SpmvArgs &a, const Real *__restrict__ x, Real *xs,
                                                    int64_t r0) {
    constexpr int PER = 16 / sizeof(Real);  // elements per lane per direct load
    constexpr int CH = 64 * PER;            // elements per wavefront per direct load
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int w = 0; w < a.n_win; ++w) {
        const int64_t g0 = r0 + a.win_lo[w];
        const int n = a.win_len[w];
        Real *dst = xs + a.win_base[w];
        if (a.async_lds && g0 >= 0 && g0 + n <= a.n_cols) {
            const int nch = (n + CH - 1) / CH;
            for (int c = wave; c < nch; c += kBlock / 64) {
                const int e = c * CH + lane * PER;
                if (e < n) lds_load16(x + g0 + e, dst + c * CH);
            }
        } else {
            const int64_t last = a.n_cols - 1;
            for (int e = threadIdx.x; e < n; e += kBlock) {
                int64_t g = g0 + e;
                g = g < 0 ? 0 : (g > last ? last : g);
                dst[e] = x[g];
            }
        }
    }
}

template <class Real>
__device__ __forceinline__ void stage_windows(const SpmvArgs &a, const Real *__restrict__ x, Real *xs, int64_t r0) {
    stage_windows_async<Real>(a, x, xs, r0);
    for (int e = threadIdx.x; e < a.zero_len; e += kBlock) xs[a.zero_base + e] = Real(0);
    __builtin_amdgcn_s_waitcnt(0);  // direct loads have landed in LDS
}

// ---- DIT, LDS windows, generic walk (any K, raw values, any pattern length) --------
template <class Real, class IdT, bool RAW, bool TAB_LDS>
__global__ __launch_bounds__(kBlock) void k_dit_lds(SpmvArgs a, const Real *__restrict__ x, Real *__restrict__ y) {
    if (a.skip && *a.skip) return;
    if (blockIdx.x >= a.n_main_blocks) {
        emit_dot(a, escape_row<Real, 1>(a, static_cast<int64_t>(blockIdx.x - a.n_main_blocks) * kBlock + threadIdx.x,
                                        1, x, 1, y, 1));
        return;
    }
    extern __shared__ __align__(16) unsigned char smem[];
    Real *xs = reinterpret_cast<Real *>(smem);
    uint16_t *tab_s = reinterpret_cast<uint16_t *>(smem + sizeof(Real) * a.lds_total);
    const int64_t r0 = xcd_tile(blockIdx.x, a.n_main_blocks, a.n_xcd) * a.rows;
    stage_windows<Real>(a, x, xs, r0);
    if constexpr (TAB_LDS) {
        for (int e = threadIdx.x; e < a.tab_elems; e += kBlock) tab_s[e] = a.tab[e];
    }
    __syncthreads();
    const uint16_t *tab = TAB_LDS ? tab_s : a.tab;
    const int tw = a.width + 1;
    double dotc = 0.0;
    for (int rel = threadIdx.x; rel < a.rows; rel += kBlock) {
        const int64_t row = r0 + rel;
        if (row >= a.n_rows) break;
        const IdT id = static_cast<const IdT *>(a.ids)[row];
        if (id == esc_id<IdT>()) continue;
        const uint16_t *t = tab + static_cast<int64_t>(id) * tw + 1;
        Real acc = Real(0);
        int k = 0;
        for (int c = 0; c < a.K; ++c) {
            const int tend = row_T(a, c, row, id);
            const Real v = vtab<Real>(a, c);
            for (; k < tend; ++k) acc = fma(v, xs[in_bounds<int>(rel + t[k], a.lds_total)], acc);
        }
        if constexpr (RAW) {
            const int len = t[-1];
            const Real *raw = static_cast<const Real *>(a.raw);
            const int64_t rb = a.raw_slice[row / kSlice] + (row % kSlice) - static_cast<int64_t>(k) * kSlice;
            for (; k < len; ++k)
                acc = fma(ldg_stream(raw + rb + static_cast<int64_t>(k) * kSlice),
                          xs[in_bounds<int>(rel + t[k], a.lds_total)], acc);
        }
        y[row] = acc;
        if (a.dot) dotc += static_cast<double>(x[row]) * static_cast<double>(acc);
    }
    emit_dot(a, dotc);
}

// ---- DIT, LDS windows, pattern held in registers (patterns of <= 32 entries) -------
// KK = 1 or 2: value table of KK entries, no raw values, short rows padded with
// zero-window entries.  The table lists each pattern's entries in *reverse*
// canonical order, so a row's V[1] entries (positions >= T[0]) come first: the
// first m = len - T[0] entries take V[1], the rest V[0].  When every active
// lane of a wavefront has the same m (two ballots decide), the row is
// V[1] * (sum of its first m x values) + V[0] * (sum of the rest): values are
// scalar operands and there are two multiplies per row instead of one per
// entry.  Otherwise each entry selects its value per lane.  For the 27-point
// stencil every row has m = 1.  KK = 0: no value table, every value raw
// (canonical order), read up to the width of the row's 64-row raw slice.  RPT rows per thread (rows per block =
// 256 * RPT); each thread's row IDs and T are loaded before the windows are
// staged, so their latency overlaps the staging.  MAXW: entries per row.
__device__ __forceinline__ uint32_t load_id(const void *ids, int id_bytes, int64_t row) {
    if (id_bytes == 1) return static_cast<const uint8_t *>(ids)[row];
    if (id_bytes == 2) return static_cast<const uint16_t *>(ids)[row];
    return static_cast<const uint32_t *>(ids)[row];
}

// A value known to be the same in every lane, kept in scalar registers (so it
// can feed an FMA as a scalar operand instead of costing a per-lane select).
__device__ __forceinline__ double uniform(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane(static_cast<int>(b));
    const int hi = __builtin_amdgcn_readfirstlane(static_cast<int>(b >> 32));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float uniform(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Sum of xat(k) for k in [LO, HI).  Every read is issued first; the adds run
// in groups of four, each group starting from its last element, so one wait
// for that element's read covers the whole group (reads complete in order);
// the group sums are added pairwise.
template <int LO, int HI, class F> __device__ __forceinline__ auto sum_entries(F xat) -> decltype(xat(0)) {
    using R = decltype(xat(0));
    constexpr int N = HI - LO, G = 4, NG = (N + G - 1) / G;
    R xv[N];
#pragma unroll
    for (int k = 0; k < N; ++k) xv[k] = xat(LO + k);
    R g[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q) {
        const int a = q * G, b = (a + G < N) ? a + G : N;
        R t = xv[b - 1];
#pragma unroll
        for (int k = b - 2; k >= a; --k) t += xv[k];
        g[q] = t;
    }
#pragma unroll
    for (int w = 1; w < NG; w *= 2)
#pragma unroll
        for (int q = 0; q + w < NG; q += 2 * w) g[q] += g[q + w];
    return g[0];
}

// Row metadata of one tile (IDs, T[0], and with EARLY_X x at the row) for the
// RPT rows of this thread.
template <class Real, int KK, int RPT, bool EARLY_X = true>
__device__ __forceinline__ void load_tile_meta(const SpmvArgs &a, const Real *__restrict__ x, int64_t r0,
                                               uint32_t (&idv)[RPT], int (&t0v)[RPT], Real (&xrow)[RPT]) {
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int64_t row = r0 + threadIdx.x + j * kBlock;
        const int64_t rc = row < a.n_rows ? row : a.n_rows - 1;
        idv[j] = load_id(a.ids, a.id_bytes, rc);
        t0v[j] = (KK >= 1 && !a.pat_T) ? static_cast<int>(a.T[rc]) : 0;  // DITV: from the pattern row
        if constexpr (EARLY_X) xrow[j] = a.dot ? x[rc] : Real(0);
    }
}

// The rows of one tile, x windows already in LDS at `buf` (byte base of the
// windows), pattern rows at `tab`.  Adds the tile's x.y to dotc:
// with EARLY_X the row's x comes from xrow (loaded with the metadata),
// otherwise it is read when needed -- from the windows at self_off when one
// holds it, else from x -- so that no register holds it through the tile.
template <class Real, int KK, int RPT, int MAXW, bool EARLY_X = true, bool ZEL = false>
__device__ __forceinline__ void reg_tile(const SpmvArgs &a, const unsigned char *buf, const uint4 *tab, int64_t r0,
                                         int rel_end, const uint32_t (&idv)[RPT], const int (&t0v)[RPT],
                                         const Real (&xrow)[RPT], Real v0, Real v1, Real *__restrict__ y,
                                         double &dotc, const Real *__restrict__ x = nullptr) {
    const uint32_t esc = a.id_bytes == 1 ? 0xFFu : (a.id_bytes == 2 ? 0xFFFFu : 0xFFFFFFFFu);
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int rel = threadIdx.x + j * kBlock;
        const int64_t row = r0 + rel;
        const bool active = rel < rel_end && row < a.n_rows && idv[j] != esc;
        const uint4 *tp = tab + static_cast<int64_t>(active ? idv[j] : 0u) * (kRegTw * 2 / 16);
        uint32_t w[16];
#pragma unroll
        for (int q = 0; q < (MAXW + 8) / 8; ++q) {
            const uint4 u = tp[q];
            w[4 * q + 0] = u.x;
            w[4 * q + 1] = u.y;
            w[4 * q + 2] = u.z;
            w[4 * q + 3] = u.w;
        }
        // word 0 of the pattern row: length, and for DITV the pattern's T_i[0]
        const int len = static_cast<int>(w[0] & 0xFFu);
        const int t0 = a.pat_T ? static_cast<int>((w[0] >> 8) & 0xFFu) : t0v[j];
        const int m = KK == 2 ? len - t0 : 0;  // leading entries that take V[1]
        // Is the split the same in every active lane?  Reference: the lowest
        // active lane's m (two ballots and one lane read, all scalar results).
        int ms = 0;
        bool uni = true;
        if constexpr (KK == 2) {
            const uint64_t act = __ballot(active);
            if (act == 0) continue;  // no active lane: uniform exit
            ms = __builtin_amdgcn_readlane(m, static_cast<int>(__builtin_ctzll(act)));
            uni = __ballot(active && m != ms) == 0;
        }
        if (!active) continue;
        const uint32_t relb = static_cast<uint32_t>(rel) * sizeof(Real);
        // ZEL: LDS addresses of the buffer, of this row's slot and of the zero element
        typedef const __attribute__((address_space(3))) unsigned char lds_byte;
        const uint32_t bufa = static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_byte *)buf));
        const uint32_t rowa = bufa + relb, zeroa = bufa + static_cast<uint32_t>(a.zero_base) * sizeof(Real);
        Real acc = Real(0);
        auto xat = [&](int k) -> Real {
            const uint32_t word = w[(k + 1) >> 1];
            const uint32_t off = ((k + 1) & 1) ? (word >> 16) : (word & 0xFFFFu);
            if constexpr (ZEL) {
                // entries past the row's length (offset 0xFFFF) read the zero element.
                // The minimum is taken of LDS addresses (row start with the buffer's
                // base already added), so an entry costs an add and a minimum.
                const uint32_t ad = min(rowa + off, zeroa);
                (void)in_bounds<uint32_t>(ad - bufa, a.lds_x_bytes);
                return *(const __attribute__((address_space(3))) Real *)(static_cast<uintptr_t>(ad));
            } else {
                // entries past the length point at the row's slot in a zero window
                return *reinterpret_cast<const Real *>(buf + in_bounds<uint32_t>(relb + off, a.lds_x_bytes));
            }
        };
        if constexpr (KK == 0) {
            // Raw values up to the width of the row's 64-row slice (the same for
            // every lane of the wave; the slice's padding is zero): these loads
            // do not wait for the pattern row.  Entries past the row's length
            // read zeros, so they add 0 * 0.
            const Real *raw = static_cast<const Real *>(a.raw);
            const int64_t s0 = a.raw_slice[row / kSlice];
            const int sw = static_cast<int>((a.raw_slice[row / kSlice + 1] - s0) / kSlice);
            const Real *rp = raw + s0 + (row % kSlice);
            Real rv[MAXW];
#pragma unroll
            for (int k = 0; k < MAXW; ++k) rv[k] = k < sw ? ldg_stream(rp + static_cast<int64_t>(k) * kSlice) : Real(0);
#pragma unroll
            for (int k = 0; k < MAXW; ++k) acc = fma(rv[k], xat(k), acc);
        } else if (KK == 1 || uni) {
            // every lane of the wave splits at the same position: one sum per
            // value, scaled once (scalar values); the common splits are compiled
            // with the split position fixed
            if (ms == 0) {
                acc = v0 * sum_entries<0, MAXW>(xat);
            } else if (ms == 1) {
                acc = fma(v0, sum_entries<1, MAXW>(xat), v1 * xat(0));
            } else if (ms == 2) {
                acc = fma(v0, sum_entries<2, MAXW>(xat), v1 * (xat(1) + xat(0)));
            } else {
#pragma unroll
                for (int k = 0; k < MAXW; ++k) acc = fma(uniform(k < ms ? v1 : v0), xat(k), acc);
            }
        } else {
#pragma unroll
            for (int k = 0; k < MAXW; ++k) acc = fma(k < m ? v1 : v0, xat(k), acc);
        }
        y[row] = acc;
        if (a.dot) {
            Real xr;
            if constexpr (EARLY_X)
                xr = xrow[j];
            else
                xr = a.self_off >= 0
                         ? *reinterpret_cast<const Real *>(
                               buf + in_bounds<uint32_t>(relb + static_cast<uint32_t>(a.self_off), a.lds_x_bytes))
                         : x[row];
            dotc += static_cast<double>(xr) * static_cast<double>(acc);
        }
    }
}

template <class Real, int KK> __device__ __forceinline__ void value_pair(const SpmvArgs &a, Real &v0, Real &v1) {
    if constexpr (sizeof(Real) == 8) {
        v0 = a.V[0];
        v1 = a.V[KK >= 2 ? 1 : 0];
    } else {
        v0 = a.V32[0];
        v1 = a.V32[KK >= 2 ? 1 : 0];
    }
}

// With one or two rows per thread an FP64 block of the 27-point stencil takes
// about 19 KB of LDS (three plane windows, the zero element, the table), so
// eight blocks fit a CU by LDS; asking for seven waves per SIMD keeps registers
// from spilling (at most 72 VGPRs instead of 80).  With three rows per thread
// (768 rows, 25 KB) six blocks fit, six waves per SIMD: at 104^3 the whole
// grid is then resident at once.  With raw values (KK = 0) a row also holds its values in registers:
// six waves (80 VGPRs) keep those from spilling.
template <class Real, int KK, bool TAB_LDS, int RPT, int MAXW>
__global__ __launch_bounds__(kBlock, (KK == 0 && RPT <= 3) ? 6 : (RPT <= 2 ? 7 : (RPT == 3 ? 6 : 1))) void k_dit_reg(SpmvArgs a,
                                                                                      const Real *__restrict__ x,
                                                                                      Real *__restrict__ y) {
    // only dynamic LDS (the dot product's wavefront sums reuse the windows), so
    // that LDS addresses are the buffer offsets themselves
    extern __shared__ __align__(16) unsigned char smem[];
    if (a.skip && *a.skip) return;
    if (blockIdx.x >= a.n_main_blocks) {
        emit_dot(a,
                 escape_row<Real, 1>(a, static_cast<int64_t>(blockIdx.x - a.n_main_blocks) * kBlock + threadIdx.x, 1,
                                     x, 1, y, 1),
                 reinterpret_cast<double *>(smem));
        return;
    }
    Real *xs = reinterpret_cast<Real *>(smem);
    const int64_t r0 = xcd_tile(blockIdx.x, a.n_main_blocks, a.n_xcd) * (kBlock * RPT);
    double dotc = 0.0;
    uint32_t idv[RPT];
    int t0v[RPT];
    Real xrow[RPT];  // unused: the row's x is read after the staging (reg_tile, EARLY_X false)
    load_tile_meta<Real, KK, RPT, false>(a, x, r0, idv, t0v, xrow);
    stage_windows<Real>(a, x, xs, r0);
    uint4 *tab_s = reinterpret_cast<uint4 *>(smem + a.lds_x_bytes);
    if constexpr (TAB_LDS) {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.reg_tab);
        const int n16 = a.P * (kRegTw * 2 / 16);
        for (int e = threadIdx.x; e < n16; e += kBlock) tab_s[e] = src[e];
    }
    __syncthreads();
    const uint4 *tab = TAB_LDS ? tab_s : reinterpret_cast<const uint4 *>(a.reg_tab);
    Real v0, v1;
    value_pair<Real, KK>(a, v0, v1);
    reg_tile<Real, KK, RPT, MAXW, false, sizeof(Real) == 8>(a, smem, tab, r0, kBlock * RPT, idv, t0v, xrow, v0, v1, y,
                                                           dotc, x);
    emit_dot(a, dotc, reinterpret_cast<double *>(smem));
}

// ---- DIT, plane-marching register kernel ------------------------------------------
// For matrices whose x windows are NW equal windows spaced one plane (m_S rows)
// apart -- the 27-point stencil: planes z-1, z, z+1.  A block owns one row
// tile (rows p0 .. p0 + R of a plane) in m_C consecutive planes.  Window w of
// the tile in plane z is plane slot q = z + w, so the tile in plane z + 1
// needs only one slot the tile in plane z did not: the block keeps NW + 1 window
// buffers in LDS as a ring (slot q in buffer q mod NB) and, while it computes
// plane z, copies slot z + NW into the free buffer.  Each plane step thus
// stages one window instead of NW, and the block's setup (arguments, table,
// first windows) is paid once per m_C tiles.  The pattern table is held in LDS
// once per ring phase (z mod NB), with each entry's byte offset resolved for
// that phase, so the inner loop is the register kernel's (reg_tile).
template <class Real, int KK, bool TAB_LDS, int RPT, int MAXW>
__global__ __launch_bounds__(kBlock) void k_dit_march(SpmvArgs a, const Real *__restrict__ x, Real *__restrict__ y) {
    extern __shared__ __align__(16) unsigned char smem[];  // only dynamic LDS, as in k_dit_reg
    if (a.skip && *a.skip) return;
    if (blockIdx.x >= a.n_main_blocks) {
        emit_dot(a,
                 escape_row<Real, 1>(a, static_cast<int64_t>(blockIdx.x - a.n_main_blocks) * kBlock + threadIdx.x, 1,
                                     x, 1, y, 1),
                 reinterpret_cast<double *>(smem));
        return;
    }
    constexpr int kRows = kBlock * RPT;
    Real *xs = reinterpret_cast<Real *>(smem);
    const int64_t ord = xcd_tile(blockIdx.x, a.n_main_blocks, a.n_xcd);
    const int64_t pt = ord % a.m_np, zc = ord / a.m_np;
    const int64_t p0 = pt * kRows;
    const int rel_end = static_cast<int>(a.m_S - p0 < kRows ? a.m_S - p0 : kRows);
    const int64_t z_beg = zc * a.m_C;
    const int64_t z_end = z_beg + a.m_C < a.m_nz ? z_beg + a.m_C : a.m_nz;
    const int L = a.m_L, NB = a.m_NB;
    // zero window (if any) and the per-phase pattern tables
    for (int e = threadIdx.x; e < a.zero_len; e += kBlock) xs[a.zero_base + e] = Real(0);
    const int tab_u4 = a.P * (kRegTw * 2 / 16);  // uint4 per phase
    const uint4 *tab_all = reinterpret_cast<const uint4 *>(a.reg_tab);
    if constexpr (TAB_LDS) {
        uint4 *tab_s = reinterpret_cast<uint4 *>(smem + a.lds_x_bytes);
        for (int e = threadIdx.x; e < tab_u4 * NB; e += kBlock) tab_s[e] = tab_all[e];
        tab_all = tab_s;
    }
    // copy plane slot q (rows q*S + p0 + lo0 .. + L) into its ring buffer
    auto stage_slot = [&](int64_t q) {
        constexpr int PER = 16 / sizeof(Real);
        constexpr int CH = 64 * PER;
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        const int64_t g0 = q * a.m_S + p0 + a.m_lo0;
        Real *dst = xs + static_cast<int64_t>(q % NB) * L;
        if (a.async_lds && g0 >= 0 && g0 + L <= a.n_cols) {
            const int nch = (L + CH - 1) / CH;
            for (int c = wave; c < nch; c += kBlock / 64) {
                const int e = c * CH + lane * PER;
                if (e < L) lds_load16(x + g0 + e, dst + c * CH);
            }
        } else {
            const int64_t last = a.n_cols - 1;
            for (int e = threadIdx.x; e < L; e += kBlock) {
                int64_t g = g0 + e;
                g = g < 0 ? 0 : (g > last ? last : g);
                dst[e] = x[g];
            }
        }
    };
    Real v0, v1;
    value_pair<Real, KK>(a, v0, v1);
    double dotc = 0.0;
    // next step's metadata as the raw aligned words that hold it (read after the wait)
    uint32_t idw[RPT], t0w[RPT];
    Real xn[RPT];
    auto load_raw_meta = [&](int64_t r0) {
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int64_t row = r0 + threadIdx.x + j * kBlock;
            const int64_t rc = row < a.n_rows ? row : a.n_rows - 1;
            const int64_t ib = rc * a.id_bytes;
            idw[j] = *reinterpret_cast<const uint32_t *>(static_cast<const uint8_t *>(a.ids) + (ib & ~int64_t(3)));
            t0w[j] = (KK >= 1 && !a.pat_T) ? *reinterpret_cast<const uint32_t *>(a.T + (rc & ~int64_t(3))) : 0u;
            xn[j] = a.dot ? x[rc] : Real(0);
        }
    };
    if (z_beg < z_end) {
        load_raw_meta(z_beg * a.m_S + p0);
        for (int w = 0; w < a.m_NW; ++w) stage_slot(z_beg + w);
    }
    const uint32_t id_mask = a.id_bytes == 4 ? 0xFFFFFFFFu : ((1u << (8 * a.id_bytes)) - 1u);
    for (int64_t z = z_beg; z < z_end; ++z) {
        // plane z's windows and metadata have landed (every wave's copies), and
        // every wave is done with the buffer of slot z - 1
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        const int64_t r0 = z * a.m_S + p0;
        uint32_t idv[RPT];
        int t0v[RPT];
        Real xrow[RPT];
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int64_t row = r0 + threadIdx.x + j * kBlock;
            const int64_t rc = row < a.n_rows ? row : a.n_rows - 1;
            idv[j] = (idw[j] >> (8 * ((rc * a.id_bytes) & 3))) & id_mask;
            t0v[j] = static_cast<int>((t0w[j] >> (8 * (rc & 3))) & 0xFFu);
            xrow[j] = xn[j];
        }
        if (z + 1 < z_end) {
            load_raw_meta(r0 + a.m_S);
            stage_slot(z + a.m_NW);
        }
        const uint4 *tab = tab_all + static_cast<int64_t>(z % NB) * tab_u4;
        reg_tile<Real, KK, RPT, MAXW>(a, smem, tab, r0, rel_end, idv, t0v, xrow, v0, v1, y, dotc);
    }
    // the last plane stages nothing further: no copy into LDS is in flight here
    emit_dot(a, dotc, reinterpret_cast<double *>(smem));
}

// The value of the first active lane, as a wavefront-uniform (scalar) value.
template <class T> __device__ __forceinline__ T first_lane(T v) {
    if constexpr (sizeof(T) == 8) {
        const uint64_t u = static_cast<uint64_t>(v);
        const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u));
        const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u >> 32));
        return static_cast<T>((static_cast<uint64_t>(hi) << 32) | lo);
    } else {
        return static_cast<T>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v)));
    }
}

// ---- BMASK: neighbour bitmask over the displacement list, x windows in LDS --------
// Every row shares one displacement list D, so entry k of any row reads its x
// element at the same offset from the row's own slot in the LDS windows
// (bm_off[k], uniform across the wavefront).  With a value table the loop runs
// over k: where every lane of a wavefront has the full mask and the same V[1]
// mask (the interior of a stencil), the entries are summed without any
// per-lane test, all LDS reads in flight; otherwise each entry is taken under
// its lane's mask bit.  With no table (KK = 0) the values come in column order
// from the row's raw slice (the slice width is uniform per wavefront, 16-byte
// loads of consecutive rows), eight at a time, and the column of the j-th value
// is the j-th set bit of the mask, its offset read from a copy of bm_off in LDS.
template <class Real, class MaskT, int KK, int RPT, int NDM>
__global__ __launch_bounds__(kBlock) void k_bmask_lds(SpmvArgs a, const Real *__restrict__ x, Real *__restrict__ y) {
    if (a.skip && *a.skip) return;
    extern __shared__ __align__(16) unsigned char smem[];
    Real *xs = reinterpret_cast<Real *>(smem);
    int32_t *offs = reinterpret_cast<int32_t *>(smem + ((static_cast<size_t>(a.lds_total) * sizeof(Real) + 15) & ~size_t(15)));
    const int64_t r0 = xcd_tile(blockIdx.x, a.n_main_blocks, a.n_xcd) * (kBlock * RPT);
    const MaskT *mk = static_cast<const MaskT *>(a.bm_mask);
    const MaskT *vmk = static_cast<const MaskT *>(a.bm_vmask);
    MaskT mv[RPT], vv[RPT];
    Real xrow[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int64_t row = r0 + threadIdx.x + j * kBlock;
        const int64_t rc = row < a.n_rows ? row : a.n_rows - 1;
        mv[j] = row < a.n_rows ? mk[rc] : MaskT(0);
        vv[j] = KK == 2 ? vmk[rc] : MaskT(0);
        xrow[j] = a.dot ? x[rc] : Real(0);
    }
    stage_windows_async<Real>(a, x, xs, r0);
    if (KK == 0 && threadIdx.x < static_cast<unsigned>(a.bm_nd)) offs[threadIdx.x] = a.bm_off[threadIdx.x];
    __builtin_amdgcn_s_waitcnt(0);  // direct loads have landed in LDS
    __syncthreads();
    Real v0, v1;
    if constexpr (KK >= 1) value_pair<Real, KK>(a, v0, v1);
    const int nd = a.bm_nd;
    const MaskT full = nd >= static_cast<int>(8 * sizeof(MaskT)) ? ~MaskT(0) : ((MaskT(1) << nd) - 1);
    double dotc = 0.0;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int rel = threadIdx.x + j * kBlock;
        const int64_t row = r0 + rel;
        MaskT m = mv[j];
        Real acc = Real(0);
        if constexpr (KK == 0) {
            const Real *raw = static_cast<const Real *>(a.raw);
            const int64_t sl = (row < a.n_rows ? row : a.n_rows - 1) / kSlice;
            const int64_t s0 = a.raw_slice[sl];
            const int sw = static_cast<int>((a.raw_slice[sl + 1] - s0) / kSlice);
            const Real *rp = raw + s0 + (row % kSlice);
            for (int j0 = 0; j0 < sw; j0 += 8) {
                Real rv[8];
                int kk[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const bool on = j0 + u < sw && m != 0;
                    kk[u] = on ? static_cast<int>(__builtin_ctzll(static_cast<uint64_t>(m))) : -1;
                    if (on) m &= m - 1;
                    rv[u] = on ? ldg_stream(rp + static_cast<int64_t>(j0 + u) * kSlice) : Real(0);
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (kk[u] >= 0) acc = fma(rv[u], xs[in_bounds<int>(rel + offs[kk[u]], a.lds_total)], acc);
            }
        } else {
            // uniform wavefront: full masks and one V[1] mask
            const MaskT vm = vv[j];
            const MaskT vm0 = first_lane(vm);
            const bool uni = __ballot(m != full || vm != vm0) == 0;
            Real s0 = Real(0), s1 = Real(0);
            if (uni) {
                Real xv[NDM];
#pragma unroll
                for (int k = 0; k < NDM; ++k) xv[k] = k < nd ? xs[in_bounds<int>(rel + a.bm_off[k], a.lds_total)] : Real(0);
#pragma unroll
                for (int k = 0; k < NDM; ++k) {
                    if (KK == 2 && ((vm0 >> k) & 1))
                        s1 += xv[k];
                    else
                        s0 += xv[k];
                }
            } else {
#pragma unroll
                for (int k = 0; k < NDM; ++k) {
                    if (k < nd && ((m >> k) & 1)) {
                        const Real xk = xs[in_bounds<int>(rel + a.bm_off[k], a.lds_total)];
                        if (KK == 2 && ((vm >> k) & 1))
                            s1 += xk;
                        else
                            s0 += xk;
                    }
                }
            }
            acc = KK == 2 ? fma(v1, s1, v0 * s0) : v0 * s0;
        }
        if (row < a.n_rows) {
            y[row] = acc;
            if (a.dot) dotc += static_cast<double>(xrow[j]) * static_cast<double>(acc);
        }
    }
    emit_dot(a, dotc);
}

// ---- block SpMV: a group of LPR lanes per row -------------------------------------
// Y = A X for nrhs row-interleaved right-hand sides.  A row is served by LPR
// lanes, each taking VEC adjacent right-hand sides (VEC = 2: one 8- or
// 16-byte load per gather), so the gathers of a row's lanes are one
// contiguous run of X and every decoded entry serves all right-hand sides.
// The lanes of a row read the same stream bytes (the loads coincide); rows
// of a wavefront are consecutive, so those reads stay coalesced.
template <class Real, int VEC> struct LaneVec;
template <class Real> struct LaneVec<Real, 1> {
    Real v[1];
    __device__ __forceinline__ static LaneVec load(const Real *p) { return LaneVec{{*p}}; }
};
template <> struct LaneVec<double, 2> {
    double v[2];
    __device__ __forceinline__ static LaneVec load(const double *p) {
        const double2 t = *reinterpret_cast<const double2 *>(p);
        return LaneVec{{t.x, t.y}};
    }
};
template <> struct LaneVec<float, 2> {
    float v[2];
    __device__ __forceinline__ static LaneVec load(const float *p) {
        const float2 t = *reinterpret_cast<const float2 *>(p);
        return LaneVec{{t.x, t.y}};
    }
};

template <int FMT, class Real, class IdT, bool RAW, int LPR, int VEC>
__global__ __launch_bounds__(kBlock) void k_spmv_lanes(SpmvArgs a, int nrhs, const Real *__restrict__ x,
                                                        int64_t ldx, Real *__restrict__ y, int64_t ldy) {
    if (a.skip && *a.skip) return;
    if (blockIdx.x >= a.n_main_blocks) {
        escape_row<Real, 16>(a, static_cast<int64_t>(blockIdx.x - a.n_main_blocks) * kBlock + threadIdx.x, nrhs, x,
                             ldx, y, ldy);
        return;
    }
    constexpr int RPB = kBlock / LPR;  // rows per block
    const int64_t row = xcd_tile(blockIdx.x, a.n_main_blocks, a.n_xcd) * RPB + threadIdx.x / LPR;
    if (row >= a.n_rows) return;
    const int r = (threadIdx.x % LPR) * VEC;
    const bool lane_on = r < nrhs;
    const Real *xr = x + (lane_on ? r : 0);
    Real acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = Real(0);
    auto apply = [&](Real val, int64_t j) {
        const LaneVec<Real, VEC> xv = LaneVec<Real, VEC>::load(xr + in_bounds<int64_t>(j, a.n_cols) * ldx);
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[v] = fma(val, xv.v[v], acc[v]);
    };
    if constexpr (FMT == SPMVC_FMT_ELL) {
        if (a.cols[row] == kEscapeColumn) return;
        for (int k = 0; k < a.width; ++k) {
            const int64_t o = static_cast<int64_t>(k) * a.n_pad + row;
            const int32_t c = a.cols[o];
            if (c >= 0) apply(static_cast<Real>(a.ell_val[o]), c);
        }
    } else if constexpr (FMT == SPMVC_FMT_BMASK) {
        // set bits of the row's mask in ascending order = its columns ascending;
        // IdT is the mask type
        IdT m = static_cast<const IdT *>(a.bm_mask)[row];
        const IdT vm = a.K == 2 ? static_cast<const IdT *>(a.bm_vmask)[row] : IdT(0);
        const Real *raw = static_cast<const Real *>(a.raw);
        const int64_t rb = RAW ? a.raw_slice[row / kSlice] + (row % kSlice) : 0;
        for (int j = 0; m; ++j) {
            const int k = static_cast<int>(__builtin_ctzll(static_cast<uint64_t>(m)));
            m &= m - 1;
            const Real v = RAW ? ldg_stream(raw + rb + static_cast<int64_t>(j) * kSlice)
                               : vtab<Real>(a, a.K == 2 ? static_cast<int>((vm >> k) & 1) : 0);
            apply(v, row + a.bm_d[k]);
        }
    } else {
        const int32_t *pat = nullptr;
        int len = 0;
        uint32_t pid = 0;
        if constexpr (FMT == SPMVC_FMT_DIT) {
            const IdT id = static_cast<const IdT *>(a.ids)[row];
            pid = id;
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
                return a.cols[static_cast<int64_t>(k) * a.n_pad + row];
        };
        int k = 0;
        for (int c = 0; c < a.K; ++c) {
            const int tend = row_T(a, c, row, pid);
            const Real v = vtab<Real>(a, c);
            for (; k < tend; ++k) apply(v, column(k));
        }
        if constexpr (RAW) {
            const Real *raw = static_cast<const Real *>(a.raw);
            const int64_t rb = a.raw_slice[row / kSlice] + (row % kSlice) - static_cast<int64_t>(k) * kSlice;
            for (; k < len; ++k) {
                const int64_t j = column(k);
                if (FMT == SPMVC_FMT_DT && j < 0) break;
                apply(raw[rb + static_cast<int64_t>(k) * kSlice], j);
            }
        }
    }
    if (lane_on) {
#pragma unroll
        for (int v = 0; v < VEC; ++v)
            if (VEC == 1 || r + v < nrhs) y[row * ldy + r + v] = acc[v];
    }
}

// ---- block SpMV, right-hand sides in pairs, x windows in LDS ------------------------
// The register kernel with 16-byte elements: a block owns a row tile and one
// pair (2p, 2p + 1) of FP64 right-hand sides; its x windows hold that pair of
// every row (16 bytes), copied with direct loads from the row-interleaved
// block (one row per lane, rows ldx apart).  Every entry is then one 16-byte
// LDS read and two adds.  Values from a table of K = 1 or 2 entries.
struct D2 {
    double x, y;
};
__device__ __forceinline__ D2 &operator+=(D2 &a, D2 b) {
    a.x += b.x;
    a.y += b.y;
    return a;
}
__device__ __forceinline__ D2 operator*(double v, D2 a) { return D2{v * a.x, v * a.y}; }
__device__ __forceinline__ D2 fma(double v, D2 a, D2 c) { return D2{::fma(v, a.x, c.x), ::fma(v, a.y, c.y)}; }

template <int KK, int RPT, int MAXW>
__global__ __launch_bounds__(kBlock) void k_dit_reg_pairs(SpmvArgs a, const double *__restrict__ X, int64_t ldx,
                                                           double *__restrict__ Y, int64_t ldy) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t pr = blockIdx.y;  // right-hand-side pair
    const double *xp = X + 2 * pr;
    if (blockIdx.x >= a.n_main_blocks) {  // escape rows: one lane per row, this pair, from global memory
        escape_row<double, 2>(a, static_cast<int64_t>(blockIdx.x - a.n_main_blocks) * kBlock + threadIdx.x, 2, xp, ldx,
                              Y + 2 * pr, ldy);
        return;
    }
    D2 *xs = reinterpret_cast<D2 *>(smem);
    const int64_t r0 = xcd_tile(blockIdx.x, a.n_main_blocks, a.n_xcd) * (kBlock * RPT);
    const uint32_t esc = a.id_bytes == 1 ? 0xFFu : (a.id_bytes == 2 ? 0xFFFFu : 0xFFFFFFFFu);
    uint32_t idv[RPT];
    int t0v[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int64_t row = r0 + threadIdx.x + j * kBlock;
        const int64_t rc = row < a.n_rows ? row : a.n_rows - 1;
        idv[j] = load_id(a.ids, a.id_bytes, rc);
        t0v[j] = a.pat_T ? 0 : static_cast<int>(a.T[rc]);  // DITV: from the pattern row
    }
    // windows: element e of window w is the pair of row r0 + lo[w] + e
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int w = 0; w < a.n_win; ++w) {
        const int64_t g0 = r0 + a.win_lo[w];
        const int n = a.win_len[w];
        D2 *dst = xs + a.win_base[w];
        if (a.async_lds && g0 >= 0 && g0 + n <= a.n_cols) {
            for (int c = wave; c * 64 < n; c += kBlock / 64) {
                const int e = c * 64 + lane;
                if (e < n) lds_load16(xp + (g0 + e) * ldx, dst + c * 64);
            }
        } else {
            const int64_t last = a.n_cols - 1;
            for (int e = threadIdx.x; e < n; e += kBlock) {
                int64_t g = g0 + e;
                g = g < 0 ? 0 : (g > last ? last : g);
                dst[e] = D2{xp[g * ldx], xp[g * ldx + 1]};
            }
        }
    }
    for (int e = threadIdx.x; e < a.zero_len; e += kBlock) xs[a.zero_base + e] = D2{0.0, 0.0};
    uint4 *tab_s = reinterpret_cast<uint4 *>(smem + a.lds_x_bytes);
    const int n16 = a.P * (kRegTw * 2 / 16);
    for (int e = threadIdx.x; e < n16; e += kBlock) tab_s[e] = reinterpret_cast<const uint4 *>(a.reg_tab)[e];
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const double v0 = a.V[0], v1 = a.V[KK >= 2 ? 1 : 0];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int rel = threadIdx.x + j * kBlock;
        const int64_t row = r0 + rel;
        const bool active = row < a.n_rows && idv[j] != esc;
        const uint4 *tp = tab_s + static_cast<int64_t>(active ? idv[j] : 0u) * (kRegTw * 2 / 16);
        uint32_t wv[16];
#pragma unroll
        for (int q = 0; q < (MAXW + 8) / 8; ++q) {
            const uint4 u = tp[q];
            wv[4 * q + 0] = u.x;
            wv[4 * q + 1] = u.y;
            wv[4 * q + 2] = u.z;
            wv[4 * q + 3] = u.w;
        }
        const int len = static_cast<int>(wv[0] & 0xFFu);
        const int m = KK == 2 ? len - (a.pat_T ? static_cast<int>((wv[0] >> 8) & 0xFFu) : t0v[j]) : 0;
        int ms = 0;
        bool uni = true;
        if constexpr (KK == 2) {
            const uint64_t act = __ballot(active);
            if (act == 0) continue;
            ms = __builtin_amdgcn_readlane(m, static_cast<int>(__builtin_ctzll(act)));
            uni = __ballot(active && m != ms) == 0;
        }
        if (!active) continue;
        const uint32_t relb = static_cast<uint32_t>(rel) * 16u;
        auto xat = [&](int k) -> D2 {
            const uint32_t word = wv[(k + 1) >> 1];
            const uint32_t off = ((k + 1) & 1) ? (word >> 16) : (word & 0xFFFFu);
            const double2 t = *reinterpret_cast<const double2 *>(smem + in_bounds<uint32_t>(relb + off, a.lds_x_bytes));
            return D2{t.x, t.y};
        };
        D2 acc{0.0, 0.0};
        if (KK == 1 || (uni && ms == 0)) {
            acc = v0 * sum_entries<0, MAXW>(xat);
        } else if (uni && ms == 1) {
            acc = fma(v0, sum_entries<1, MAXW>(xat), v1 * xat(0));
        } else {
#pragma unroll
            for (int k = 0; k < MAXW; ++k) acc = fma(k < m ? v1 : v0, xat(k), acc);
        }
        double *yr = Y + row * ldy + 2 * pr;
        *reinterpret_cast<double2 *>(yr) = double2{acc.x, acc.y};
    }
}

// ---- block SpMV, whole right-hand-side rows in LDS, one window at a time ----------
// Four entries of a row's (pattern, window) record against the x window: four
// 16-byte x reads in flight, then four weighted FMAs (value V[0] for
// canonical index < t0, else V[1]).
template <int NRB>
__device__ __forceinline__ void win_group(uint4 e, const unsigned char *xrow, uint32_t lim, int t0, double v0,
                                          double v1, double &a0, double &a1) {
    const uint32_t ent[4] = {e.x, e.y, e.z, e.w};
    double2 xv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        xv[j] = *reinterpret_cast<const double2 *>(xrow + in_bounds<uint32_t>(ent[j] & 0xFFFFu, lim) * NRB);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double wgt = static_cast<int>(ent[j] >> 16) < t0 ? v0 : v1;
        a0 = ::fma(wgt, xv[j].x, a0);
        a1 = ::fma(wgt, xv[j].y, a1);
    }
}

// The products of one row's entries that fall in the current x window, for
// this lane's pair of right-hand sides: `rec` is the row's (pattern, window)
// record (count, then the entries from word 4), `xrow` the lane's element
// pair in window row 0, NRB the bytes of a window row.  One 16-byte table
// read per four entries; the last cnt mod 4 entries one at a time.
template <int NRB>
__device__ __forceinline__ void win_row(const uint4 *rec, const unsigned char *xrow, uint32_t lim, int t0, double v0,
                                        double v1, double &a0, double &a1) {
    const int cnt = static_cast<int>(rec[0].x);
    int k0 = 0;
    for (; k0 + 4 <= cnt; k0 += 4) win_group<NRB>(rec[1 + (k0 >> 2)], xrow, lim, t0, v0, v1, a0, a1);
    const uint32_t *recw = reinterpret_cast<const uint32_t *>(rec) + 4;
    for (; k0 < cnt; ++k0) {
        const uint32_t e = recw[k0];
        const double2 xv = *reinterpret_cast<const double2 *>(xrow + in_bounds<uint32_t>(e & 0xFFFFu, lim) * NRB);
        const double wgt = static_cast<int>(e >> 16) < t0 ? v0 : v1;
        a0 = ::fma(wgt, xv.x, a0);
        a1 = ::fma(wgt, xv.y, a1);
    }
}

// nrhs = Q * LPR FP64 right-hand sides, row-interleaved and unpadded.  A block
// owns kWinRows rows; for each x window in turn it copies the window's rows
// of the block (all nrhs values of a row: 8 * nrhs bytes, a contiguous range
// of memory) into LDS, then every row adds the products of its entries that
// fall in that window (win_row).  Only one window is held at a time, so whole
// rows fit.  A group of LPR lanes serves a row, each lane Q consecutive
// right-hand sides (16-byte LDS reads): Q = 2, or Q = 4 with split records,
// where each record read and loop set-up then serves twice the right-hand
// sides (the record handling, not the sums, is most of the kernel's VALU work).
template <int LPR, int Q = 2>
__global__ __launch_bounds__(kBlock) void k_dit_block_win(SpmvArgs a, const double *__restrict__ X,
                                                           double *__restrict__ Y) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NR = Q * LPR;          // right-hand sides
    constexpr int PASSES = kWinRows / (kBlock / LPR);
    if (blockIdx.x >= a.n_main_blocks) {  // escape rows: one lane per row, all right-hand sides, from global memory
        escape_row<double, NR>(a, static_cast<int64_t>(blockIdx.x - a.n_main_blocks) * kBlock + threadIdx.x, NR, X, NR,
                               Y, NR);
        return;
    }
    const int NW = a.n_win;
    double *xs = reinterpret_cast<double *>(smem);
    const uint4 *tab_s = reinterpret_cast<const uint4 *>(smem + a.lds_x_bytes);
    const int64_t r0 = xcd_tile(blockIdx.x, a.n_main_blocks, a.n_xcd) * kWinRows;
    const uint32_t esc = a.id_bytes == 1 ? 0xFFu : (a.id_bytes == 2 ? 0xFFFFu : 0xFFFFFFFFu);
    const int lr = threadIdx.x / LPR;           // row within a pass
    const int rp = (threadIdx.x % LPR) * Q;     // this lane's first right-hand side
    uint32_t idv[PASSES];
    int t0v[PASSES];
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps) {
        const int64_t row = r0 + ps * (kBlock / LPR) + lr;
        const int64_t rc = row < a.n_rows ? row : a.n_rows - 1;
        idv[ps] = load_id(a.ids, a.id_bytes, rc);
        t0v[ps] = a.K < 2 ? 255 : (idv[ps] == esc ? 0 : row_T(a, 0, rc, idv[ps]));
    }
    {
        const int n16 = a.P * NW * (kWinSt / 4);
        const uint4 *src = reinterpret_cast<const uint4 *>(a.reg_tab);
        uint4 *dst = reinterpret_cast<uint4 *>(smem + a.lds_x_bytes);
        for (int e = threadIdx.x; e < n16; e += kBlock) dst[e] = src[e];
    }
    const double v0 = a.V[0], v1 = a.V[a.K >= 2 ? 1 : 0];
    double acc[PASSES][Q];
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps)
#pragma unroll
        for (int q = 0; q < Q; ++q) acc[ps][q] = 0.0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int w = 0; w < NW; ++w) {
        if (w > 0) __syncthreads();  // every row is done with the previous window
        const int64_t g0 = r0 + a.win_lo[w];
        const int n = a.win_len[w];
        if (a.async_lds && g0 >= 0 && g0 + n <= a.n_cols) {
            // rows g0 .. g0 + n: n * NR doubles, contiguous; 16 bytes per lane
            const double *src = X + g0 * NR;
            const int nchunk = n * NR / 2;
            for (int c = wave * 64; c < nchunk; c += kBlock) {
                const int e = c + lane;
                if (e < nchunk) lds_load16(src + 2 * e, xs + 2 * c);
            }
        } else {
            const int64_t last = a.n_cols - 1;
            for (int e = threadIdx.x; e < n * NR; e += kBlock) {
                int64_t g = g0 + e / NR;
                g = g < 0 ? 0 : (g > last ? last : g);
                xs[e] = X[g * NR + e % NR];
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) {
            const int rel = ps * (kBlock / LPR) + lr;
            const int64_t row = r0 + rel;
            if (row >= a.n_rows || idv[ps] == esc) continue;
            const uint4 *rec = tab_s + (static_cast<int64_t>(idv[ps]) * NW + w) * (kWinSt / 4);
            const unsigned char *xrow = reinterpret_cast<const unsigned char *>(xs + rel * NR + rp);
            const uint32_t lim = static_cast<uint32_t>(a.win_len[w] - rel);  // window rows from this row on
            if constexpr (Q == 4) {  // launched only with split records
                win_row_split<NR * 8, Q>(reinterpret_cast<const uint32_t *>(rec), xrow, lim, v0, v1, acc[ps]);
            } else {
                if (a.bw_split)
                    win_row_split<NR * 8, Q>(reinterpret_cast<const uint32_t *>(rec), xrow, lim, v0, v1, acc[ps]);
                else
                    win_row<NR * 8>(rec, xrow, lim, t0v[ps], v0, v1, acc[ps][0], acc[ps][1]);
            }
        }
    }
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps) {
        const int64_t row = r0 + ps * (kBlock / LPR) + lr;
        if (row >= a.n_rows || idv[ps] == esc) continue;
#pragma unroll
        for (int h = 0; h < Q / 2; ++h)
            *reinterpret_cast<double2 *>(Y + row * NR + rp + 2 * h) = double2{acc[ps][2 * h], acc[ps][2 * h + 1]};
    }
}

template <class Real> SpmvArgs make_args(const spmvc_matrix_s *M, const int *skip, double *dot) {
    SpmvArgs a{};
    a.skip = skip;
    a.dot = dot;
    a.self_off = -1;
    a.n_rows = M->n_rows;
    a.n_cols = M->n_cols;
    a.n_pad = M->n_pad;
    a.K = M->K;
    a.width = M->width;
    a.P = M->P;
    a.raw_present = M->raw_elems > 0;
    a.id_bytes = M->id_bytes;
    a.ids = M->ids.p;
    a.T = M->T.as<uint8_t>();
    a.pat_T = M->fold ? M->pat_T.as<uint8_t>() : nullptr;
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
    a.n_xcd = M->n_xcd;
    a.bm_d = M->bm_d.as<int32_t>();
    a.bm_mask = M->bm_mask.p;
    a.bm_vmask = M->bm_vmask.p;
    a.bm_nd = M->bm_nd;
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
    } else if (M->fmt == SPMVC_FMT_BMASK) {
        if (M->bm_bytes == 4) {
            if (raw)
                k_spmv_direct<SPMVC_FMT_BMASK, Real, uint32_t, true, NR><<<grid, kBlock, 0, s>>>(a, nrhs, xp, ldx, yp, ldy);
            else
                k_spmv_direct<SPMVC_FMT_BMASK, Real, uint32_t, false, NR><<<grid, kBlock, 0, s>>>(a, nrhs, xp, ldx, yp, ldy);
        } else {
            if (raw)
                k_spmv_direct<SPMVC_FMT_BMASK, Real, uint64_t, true, NR><<<grid, kBlock, 0, s>>>(a, nrhs, xp, ldx, yp, ldy);
            else
                k_spmv_direct<SPMVC_FMT_BMASK, Real, uint64_t, false, NR><<<grid, kBlock, 0, s>>>(a, nrhs, xp, ldx, yp, ldy);
        }
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

// Which register-kernel variant fits the matrix: 0 = none, else KK + 1.
int reg_variant(const spmvc_matrix_s *M, int dt) {
    const LdsPlan &p = M->plan[dt];
    if (!p.reg) return 0;
    if (M->K == 0 && M->raw_elems > 0) return 1;                       // KK = 0
    if ((M->K == 1 || M->K == 2) && M->raw_elems == 0 && p.v_finite) return M->K + 1;
    return 0;
}

// Returns the number of blocks launched (one dot partial each).
template <class Real>
unsigned launch_lds(const spmvc_matrix_s *M, SpmvArgs a, const void *x, void *y, hipStream_t s) {
    constexpr int dt = sizeof(Real) == 8 ? SPMVC_F64 : SPMVC_F32;
    const LdsPlan &p = M->plan[dt];
    a.rows = p.rows;
    a.n_win = p.n_win;
    a.lds_total = p.total;
    for (int w = 0; w < p.n_win; ++w) {
        a.win_lo[w] = p.lo[w];
        a.win_len[w] = p.len[w];
        a.win_base[w] = p.base[w];
    }
    a.n_main_blocks = static_cast<unsigned>((M->n_rows + p.rows - 1) / p.rows);
    a.async_lds = (reinterpret_cast<uintptr_t>(x) % 16) == 0;
    const unsigned grid = a.n_main_blocks + escape_blocks(M);
    const Real *xp = static_cast<const Real *>(x);
    Real *yp = static_cast<Real *>(y);
    const int rv = reg_variant(M, dt);
    if (rv > 0) {
        const bool f64 = sizeof(Real) == 8;
        a.zero_base = p.zero_base;
        a.zero_len = f64 ? 1 : p.rows;  // FP64: one zero element; FP32: a zero window
        a.reg_tab = f64 ? p.reg_tab64.as<uint16_t>() : p.reg_tab32.as<uint16_t>();
        const int x_bytes = static_cast<int>(sizeof(Real)) * (p.zero_base + a.zero_len);
        a.lds_x_bytes = (x_bytes + 15) & ~15;
        const int rpt = p.rows / kBlock;
        const bool w27 = M->width <= 27;  // the 27-point stencil: no padded step
        // With the dot product (CG), each block leaves a partial that every block
        // of the next kernel sums: past kDotMaxTiles register tiles that sum
        // costs more than the register form saves, and the marching form of the
        // same plan (fewer, longer-lived blocks) is taken instead.
        const bool many_partials = a.dot && M->lds_mode[dt] == 1 && a.n_main_blocks > kDotMaxTiles;
        if ((M->lds_mode[dt] == 2 || many_partials) && p.march) {
            a.m_S = p.m_S;
            a.m_nz = p.m_nz;
            a.m_lo0 = p.m_lo0;
            a.m_np = p.m_np;
            a.m_C = p.m_C;
            a.m_L = p.m_L;
            a.m_NB = p.m_NB;
            a.m_NW = p.m_NW;
            a.zero_base = p.m_zero_base;
            a.zero_len = p.rows;
            a.reg_tab = f64 ? p.m_tab64.as<uint16_t>() : p.m_tab32.as<uint16_t>();
            const int mx_bytes = static_cast<int>(sizeof(Real)) * (p.m_zero_base + p.rows);
            a.lds_x_bytes = (mx_bytes + 15) & ~15;
            const size_t msh = a.lds_x_bytes + (p.m_tab_lds ? static_cast<size_t>(p.m_NB) * M->P * kRegTw * 2 : 0);
            const int64_t nzc = (p.m_nz + p.m_C - 1) / p.m_C;
            a.n_main_blocks = static_cast<unsigned>(p.m_np * nzc);
            const unsigned mgrid = a.n_main_blocks + escape_blocks(M);
#define SPMVC_MARCH_W(KK, TL, R)                                                               \
    if (w27)                                                                                   \
        k_dit_march<Real, KK, TL, R, 27><<<mgrid, kBlock, msh, s>>>(a, xp, yp);                \
    else                                                                                       \
        k_dit_march<Real, KK, TL, R, kRegW><<<mgrid, kBlock, msh, s>>>(a, xp, yp);
#define SPMVC_MARCH_R(KK, TL)    \
    if (rpt == 1) {              \
        SPMVC_MARCH_W(KK, TL, 1) \
    } else if (rpt == 2) {       \
        SPMVC_MARCH_W(KK, TL, 2) \
    } else {                     \
        SPMVC_MARCH_W(KK, TL, 4) \
    }
            if (rv == 1) {
                if (p.m_tab_lds) {
                    SPMVC_MARCH_R(0, true)
                } else {
                    SPMVC_MARCH_R(0, false)
                }
            } else if (rv == 2) {
                if (p.m_tab_lds) {
                    SPMVC_MARCH_R(1, true)
                } else {
                    SPMVC_MARCH_R(1, false)
                }
            } else {
                if (p.m_tab_lds) {
                    SPMVC_MARCH_R(2, true)
                } else {
                    SPMVC_MARCH_R(2, false)
                }
            }
#undef SPMVC_MARCH_R
#undef SPMVC_MARCH_W
            SPMVC_CHECK_LAUNCH();
            return mgrid;
        }
        size_t shmem = a.lds_x_bytes;
        if (p.reg_tab_in_lds) shmem += static_cast<size_t>(M->P) * kRegTw * 2;
        // the window that holds every row of the block (displacement 0), if any
        a.self_off = -1;
        for (int w = 0; w < p.n_win; ++w)
            if (p.lo[w] <= 0 && p.lo[w] + p.len[w] >= p.rows) {
                a.self_off = static_cast<int32_t>((p.base[w] - p.lo[w]) * static_cast<int64_t>(sizeof(Real)));
                break;
            }
#define SPMVC_REG_W(KK, TL, R)                                                                                  \
    if (w27)                                                                                                    \
        k_dit_reg<Real, KK, TL, R, 27><<<grid, kBlock, shmem, s>>>(a, xp, yp);                                  \
    else                                                                                                        \
        k_dit_reg<Real, KK, TL, R, kRegW><<<grid, kBlock, shmem, s>>>(a, xp, yp);
#define SPMVC_REG_R(KK, TL)      \
    if (rpt == 1) {              \
        SPMVC_REG_W(KK, TL, 1)   \
    } else if (rpt == 2) {       \
        SPMVC_REG_W(KK, TL, 2)   \
    } else if (rpt == 3) {       \
        SPMVC_REG_W(KK, TL, 3)   \
    } else if (rpt == 4) {       \
        SPMVC_REG_W(KK, TL, 4)   \
    } else {                     \
        SPMVC_REG_W(KK, TL, 8)   \
    }
#define SPMVC_REG_T(KK)          \
    if (p.reg_tab_in_lds) {      \
        SPMVC_REG_R(KK, true)    \
    } else {                     \
        SPMVC_REG_R(KK, false)   \
    }
        if (rv == 1) {
            SPMVC_REG_T(0)
        } else if (rv == 2) {
            SPMVC_REG_T(1)
        } else {
            SPMVC_REG_T(2)
        }
#undef SPMVC_REG_T
#undef SPMVC_REG_R
#undef SPMVC_REG_W
        SPMVC_CHECK_LAUNCH();
        return grid;
    }
    a.zero_len = 0;
    a.tab = p.tab.as<uint16_t>();
    a.tab_elems = M->P * (M->width + 1);
    size_t shmem = sizeof(Real) * static_cast<size_t>(p.total);
    if (p.tab_in_lds) shmem += sizeof(uint16_t) * static_cast<size_t>(a.tab_elems) + 16;
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
    return grid;
}

// Window-phased block SpMV (k_dit_block_win): FP64, 2, 4 or 8 right-hand
// sides, unpadded row-interleaved blocks; false when it does not apply.
bool launch_block_win(const spmvc_matrix_s *M, SpmvArgs a, int nrhs, const void *X, int64_t ldx, void *Y,
                      int64_t ldy, hipStream_t s) {
    const LdsPlan &p = M->plan[SPMVC_F64];
    if (M->fmt != SPMVC_FMT_DIT || !p.bw || M->P == 0) return false;
    if (!(nrhs == 2 || nrhs == 4 || nrhs == 8) || ldx != nrhs || ldy != nrhs) return false;
    if (reinterpret_cast<uintptr_t>(X) % 16 || reinterpret_cast<uintptr_t>(Y) % 16) return false;
    const int64_t xb = static_cast<int64_t>(p.bw_maxlen) * nrhs * 8;
    const int64_t tb = static_cast<int64_t>(M->P) * p.bw_nw * kWinSt * 4;
    if (xb + tb > kLdsBudgetBytes) return false;
    a.n_win = p.bw_nw;
    for (int w = 0; w < p.bw_nw; ++w) {
        a.win_lo[w] = p.bw_lo[w];
        a.win_len[w] = p.bw_len[w];
    }
    a.async_lds = 1;
    a.bw_split = p.bw_split ? 1 : 0;
    a.lds_x_bytes = static_cast<int32_t>(xb);
    a.reg_tab = reinterpret_cast<const uint16_t *>(p.bw_tab.p);
    const size_t shmem = static_cast<size_t>(xb + tb);
    // the row tiles, then the escape rows' blocks (same launch)
    a.n_main_blocks = static_cast<unsigned>((M->n_rows + kWinRows - 1) / kWinRows);
    const unsigned grid = a.n_main_blocks + escape_blocks(M);
    const double *xp = static_cast<const double *>(X);
    double *yp = static_cast<double *>(Y);
    // with split records a lane takes four right-hand sides (nrhs 4 and 8)
    if (nrhs == 2)
        k_dit_block_win<1><<<grid, kBlock, shmem, s>>>(a, xp, yp);
    else if (nrhs == 4 && p.bw_split)
        k_dit_block_win<1, 4><<<grid, kBlock, shmem, s>>>(a, xp, yp);
    else if (nrhs == 4)
        k_dit_block_win<2><<<grid, kBlock, shmem, s>>>(a, xp, yp);
    else if (p.bw_split)
        k_dit_block_win<2, 4><<<grid, kBlock, shmem, s>>>(a, xp, yp);
    else
        k_dit_block_win<4><<<grid, kBlock, shmem, s>>>(a, xp, yp);
    SPMVC_CHECK_LAUNCH();
    return true;
}

// Block SpMV of FP64 right-hand-side pairs with LDS windows (k_dit_reg_pairs);
// false when it does not apply (format, value table, alignment, LDS size).
bool launch_pairs(const spmvc_matrix_s *M, SpmvArgs a, int nrhs, const void *X, int64_t ldx, void *Y, int64_t ldy,
                  hipStream_t s) {
    const LdsPlan &p = M->plan[SPMVC_F64];
    if (M->fmt != SPMVC_FMT_DIT || !p.reg128 || p.n_win == 0 || M->P == 0 || M->lds_mode[SPMVC_F64] == 0) return false;
    if (!(M->K == 1 || M->K == 2) || M->raw_elems > 0 || !p.v_finite) return false;
    if (nrhs % 2 || ldx % 2 || ldy % 2 || reinterpret_cast<uintptr_t>(X) % 16 || reinterpret_cast<uintptr_t>(Y) % 16)
        return false;
    const int rpt = p.rows / kBlock;
    if (rpt != 1 && rpt != 2 && rpt != 4) return false;  // instances for 1, 2 and 4 rows per thread
    a.rows = p.rows;
    a.n_win = p.n_win;
    for (int w = 0; w < p.n_win; ++w) {
        a.win_lo[w] = p.lo[w];
        a.win_len[w] = p.len[w];
        a.win_base[w] = p.base[w];
    }
    a.async_lds = 1;
    a.zero_base = p.zero_base;
    a.zero_len = p.rows;
    a.reg_tab = p.reg_tab128.as<uint16_t>();
    a.lds_x_bytes = 16 * (p.zero_base + p.rows);
    const size_t shmem = a.lds_x_bytes + static_cast<size_t>(M->P) * kRegTw * 2;
    // the row tiles, then the escape rows' blocks (same launch), for each pair
    a.n_main_blocks = static_cast<unsigned>((M->n_rows + p.rows - 1) / p.rows);
    const dim3 grid(a.n_main_blocks + escape_blocks(M), static_cast<unsigned>(nrhs / 2));
    const double *xp = static_cast<const double *>(X);
    double *yp = static_cast<double *>(Y);
    const bool w27 = M->width <= 27;
#define SPMVC_PAIRS_W(KK, R)                                                                         \
    if (w27)                                                                                         \
        k_dit_reg_pairs<KK, R, 27><<<grid, kBlock, shmem, s>>>(a, xp, ldx, yp, ldy);                 \
    else                                                                                             \
        k_dit_reg_pairs<KK, R, kRegW><<<grid, kBlock, shmem, s>>>(a, xp, ldx, yp, ldy);
#define SPMVC_PAIRS_R(KK)        \
    if (rpt == 1) {              \
        SPMVC_PAIRS_W(KK, 1)     \
    } else if (rpt == 2) {       \
        SPMVC_PAIRS_W(KK, 2)     \
    } else {                     \
        SPMVC_PAIRS_W(KK, 4)     \
    }
    if (M->K == 1) {
        SPMVC_PAIRS_R(1)
    } else {
        SPMVC_PAIRS_R(2)
    }
#undef SPMVC_PAIRS_R
#undef SPMVC_PAIRS_W
    SPMVC_CHECK_LAUNCH();
    return true;
}

template <class Real, int LPR, int VEC>
void launch_lanes_l(const spmvc_matrix_s *M, SpmvArgs a, int nrhs, const Real *xp, int64_t ldx, Real *yp,
                    int64_t ldy, hipStream_t s) {
    constexpr int RPB = kBlock / LPR;
    a.n_main_blocks = static_cast<unsigned>((M->n_rows + RPB - 1) / RPB);
    const unsigned grid = a.n_main_blocks + escape_blocks(M);
    const bool raw = M->raw_elems > 0;
#define SPMVC_LANES(FMT, IDT)                                                                                  \
    if (raw)                                                                                                   \
        k_spmv_lanes<FMT, Real, IDT, true, LPR, VEC><<<grid, kBlock, 0, s>>>(a, nrhs, xp, ldx, yp, ldy);        \
    else                                                                                                       \
        k_spmv_lanes<FMT, Real, IDT, false, LPR, VEC><<<grid, kBlock, 0, s>>>(a, nrhs, xp, ldx, yp, ldy);
    if (M->fmt == SPMVC_FMT_ELL) {
        k_spmv_lanes<SPMVC_FMT_ELL, Real, uint8_t, false, LPR, VEC><<<grid, kBlock, 0, s>>>(a, nrhs, xp, ldx, yp, ldy);
    } else if (M->fmt == SPMVC_FMT_DT) {
        SPMVC_LANES(SPMVC_FMT_DT, uint8_t)
    } else if (M->id_bytes == 1) {
        SPMVC_LANES(SPMVC_FMT_DIT, uint8_t)
    } else if (M->id_bytes == 2) {
        SPMVC_LANES(SPMVC_FMT_DIT, uint16_t)
    } else {
        SPMVC_LANES(SPMVC_FMT_DIT, uint32_t)
    }
#undef SPMVC_LANES
    SPMVC_CHECK_LAUNCH();
}

// Several right-hand sides: a lane group per row (LPR lanes of VEC right-hand
// sides each; VEC = 2 when the blocks are 16-/8-byte aligned for pairs).
template <class Real>
void launch_lanes(const spmvc_matrix_s *M, SpmvArgs a, int nrhs, const void *X, int64_t ldx, void *Y,
                  int64_t ldy, hipStream_t s) {
    const Real *xp = static_cast<const Real *>(X);
    Real *yp = static_cast<Real *>(Y);
    const uintptr_t al = 2 * sizeof(Real);
    const bool pairs = nrhs % 2 == 0 && ldx % 2 == 0 && ldy % 2 == 0 && reinterpret_cast<uintptr_t>(X) % al == 0 &&
                       reinterpret_cast<uintptr_t>(Y) % al == 0;
    const int lanes = pairs ? nrhs / 2 : nrhs;
    if (pairs) {
        if (lanes <= 1)
            launch_lanes_l<Real, 1, 2>(M, a, nrhs, xp, ldx, yp, ldy, s);
        else if (lanes <= 2)
            launch_lanes_l<Real, 2, 2>(M, a, nrhs, xp, ldx, yp, ldy, s);
        else if (lanes <= 4)
            launch_lanes_l<Real, 4, 2>(M, a, nrhs, xp, ldx, yp, ldy, s);
        else
            launch_lanes_l<Real, 8, 2>(M, a, nrhs, xp, ldx, yp, ldy, s);
    } else {
        if (lanes <= 2)
            launch_lanes_l<Real, 2, 1>(M, a, nrhs, xp, ldx, yp, ldy, s);
        else if (lanes <= 4)
            launch_lanes_l<Real, 4, 1>(M, a, nrhs, xp, ldx, yp, ldy, s);
        else if (lanes <= 8)
            launch_lanes_l<Real, 8, 1>(M, a, nrhs, xp, ldx, yp, ldy, s);
        else
            launch_lanes_l<Real, 16, 1>(M, a, nrhs, xp, ldx, yp, ldy, s);
    }
}

template <class Real>
void launch_block_t(const spmvc_matrix_s *M, int nrhs, const void *X, int64_t ldx, void *Y, int64_t ldy,
                    hipStream_t s, const int *skip, double *dot = nullptr) {
    SpmvArgs a = make_args<Real>(M, skip, dot);
    constexpr int dt = sizeof(Real) == 8 ? SPMVC_F64 : SPMVC_F32;
    if constexpr (dt == SPMVC_F64) {
        if (nrhs > 1 && !dot && M->block_mode[dt] == 3 && launch_block_win(M, a, nrhs, X, ldx, Y, ldy, s)) return;
        if (nrhs > 1 && !dot && M->block_mode[dt] == 2 && launch_pairs(M, a, nrhs, X, ldx, Y, ldy, s)) return;
    }
    if (nrhs > 1 && !dot && M->block_mode[dt] && M->fmt != SPMVC_FMT_BMASK) {
        launch_lanes<Real>(M, a, nrhs, X, ldx, Y, ldy, s);
        return;
    }
    if (nrhs == 1)
        launch_direct_nr<Real, 1>(M, a, 1, X, ldx, Y, ldy, s);
    else if (nrhs <= 4)
        launch_direct_nr<Real, 4>(M, a, nrhs, X, ldx, Y, ldy, s);
    else if (nrhs <= 8)
        launch_direct_nr<Real, 8>(M, a, nrhs, X, ldx, Y, ldy, s);
    else
        launch_direct_nr<Real, 16>(M, a, nrhs, X, ldx, Y, ldy, s);
}

// BMASK with x windows in LDS (k_bmask_lds); returns the number of blocks.
template <class Real>
unsigned launch_bmask_lds(const spmvc_matrix_s *M, SpmvArgs a, const void *x, void *y, hipStream_t s) {
    constexpr int dt = sizeof(Real) == 8 ? SPMVC_F64 : SPMVC_F32;
    const LdsPlan &p = M->plan[dt];
    a.rows = p.rows;
    a.n_win = p.n_win;
    a.lds_total = p.total;
    for (int w = 0; w < p.n_win; ++w) {
        a.win_lo[w] = p.lo[w];
        a.win_len[w] = p.len[w];
        a.win_base[w] = p.base[w];
    }
    for (int k = 0; k < 64; ++k) a.bm_off[k] = k < M->bm_nd ? p.bm_off[k] : 0;
    a.zero_len = 0;
    a.n_main_blocks = static_cast<unsigned>((M->n_rows + p.rows - 1) / p.rows);
    a.async_lds = (reinterpret_cast<uintptr_t>(x) % 16) == 0;
    const unsigned grid = a.n_main_blocks;
    const size_t shmem = ((sizeof(Real) * static_cast<size_t>(p.total) + 15) & ~size_t(15)) + sizeof(int32_t) * 64;
    const Real *xp = static_cast<const Real *>(x);
    Real *yp = static_cast<Real *>(y);
    const int rpt = p.rows / kBlock;
    const int kk = M->raw_elems > 0 ? 0 : M->K;  // 0: values raw; 1, 2: table
#define SPMVC_BM_R(MT, KK, NDM)                                                              \
    if (rpt == 1)                                                                            \
        k_bmask_lds<Real, MT, KK, 1, NDM><<<grid, kBlock, shmem, s>>>(a, xp, yp);            \
    else if (rpt == 2)                                                                       \
        k_bmask_lds<Real, MT, KK, 2, NDM><<<grid, kBlock, shmem, s>>>(a, xp, yp);            \
    else                                                                                     \
        k_bmask_lds<Real, MT, KK, 4, NDM><<<grid, kBlock, shmem, s>>>(a, xp, yp);
#define SPMVC_BM_K(MT, NDM)     \
    if (kk == 0) {              \
        SPMVC_BM_R(MT, 0, NDM)  \
    } else if (kk == 1) {       \
        SPMVC_BM_R(MT, 1, NDM)  \
    } else {                    \
        SPMVC_BM_R(MT, 2, NDM)  \
    }
    if (M->bm_bytes == 4) {
        if (M->bm_nd <= 27) {
            SPMVC_BM_K(uint32_t, 27)
        } else {
            SPMVC_BM_K(uint32_t, 32)
        }
    } else {
        SPMVC_BM_K(uint64_t, 64)
    }
#undef SPMVC_BM_K
#undef SPMVC_BM_R
    SPMVC_CHECK_LAUNCH();
    return grid;
}

bool uses_lds(const spmvc_matrix_s *M, int dt) {
    if (M->fmt == SPMVC_FMT_BMASK) return M->lds_mode[dt] >= 1 && M->plan[dt].n_win > 0;
    return M->fmt == SPMVC_FMT_DIT && M->lds_mode[dt] >= 1 && M->plan[dt].n_win > 0 && M->P > 0;
}

// Returns the number of blocks launched (one dot partial each).
template <class Real>
unsigned launch_spmv_t(const spmvc_matrix_s *M, const void *x, void *y, hipStream_t s, const int *skip,
                       double *dot = nullptr) {
    if (M->n_rows == 0) return 0;
    constexpr int dt = sizeof(Real) == 8 ? SPMVC_F64 : SPMVC_F32;
    if (uses_lds(M, dt)) {
        if (M->fmt == SPMVC_FMT_BMASK) return launch_bmask_lds<Real>(M, make_args<Real>(M, skip, dot), x, y, s);
        return launch_lds<Real>(M, make_args<Real>(M, skip, dot), x, y, s);
    }
    launch_block_t<Real>(M, 1, x, 1, y, 1, s, skip, dot);
    return static_cast<unsigned>((M->n_pad + kBlock - 1) / kBlock + escape_blocks(M));
}

}  // namespace

// Word 0 of a register-kernel pattern row: the length in the low byte and,
// for DITV, the pattern's T_i[0] in the high byte (the kernels take the split
// from there; DIT rows read theirs from the T stream).
static uint16_t reg_row_head(const spmvc_matrix_s *M, int q) {
    const int L = M->h_pat_len[q];
    const int t0 = (M->fold && M->K >= 1) ? M->h_pat_T[static_cast<size_t>(q) * M->K] : 0;
    return static_cast<uint16_t>(L | (t0 << 8));
}

// Plane-marching form of the register-kernel plan: applies when the windows
// are equally spaced (by S rows, a multiple of 4) and equally long, so that
// window w of the tile in plane z is window w - 1 of the tile in plane z + 1.
// The ring holds NB = windows + 1 buffers; table phase ph resolves window w
// of a tile to buffer (ph + w) mod NB.  Planes per block (m_C) are chosen so
// that the grid about fills the device once.
static void build_march_plan(spmvc_matrix_s *M, LdsPlan &p, const std::vector<std::pair<int64_t, int64_t>> &win,
                      const int64_t *lo, const int64_t *len, int rows) {
    if (!p.reg || p.n_win < 2 || !(rows == 256 || rows == 512 || rows == 1024)) return;
    const int NW = p.n_win, NB = NW + 1;
    const int64_t S = lo[1] - lo[0];
    if (S <= 0 || S % 4 != 0) return;
    for (int w = 1; w < NW; ++w)
        if (lo[w] - lo[w - 1] != S || len[w] != len[0]) return;
    const int64_t L = len[0];
    const int64_t x_elems = NB * L + rows;  // ring + zero window
    const int64_t x_bytes64 = ((x_elems * 8) + 15) & ~int64_t(15);
    if (rows > 1024) return;  // row tiles of 256, 512 or 1024
    const int64_t tab_bytes = static_cast<int64_t>(NB) * M->P * kRegTw * 2;
    const bool tab_lds = tab_bytes <= 16 * 1024 && x_bytes64 + tab_bytes <= kLdsBudgetBytes;
    if (x_bytes64 > kLdsBudgetBytes || x_elems * 8 > 65535) return;
    const int W = M->width;
    auto window_of = [&](int64_t d) {
        int w = 0;
        while (!(d >= win[w].first && d <= win[w].second)) ++w;
        return w;
    };
    for (int es : {8, 4}) {
        std::vector<uint16_t> rt(static_cast<size_t>(NB) * M->P * kRegTw, 0);
        for (int ph = 0; ph < NB; ++ph)
            for (int q = 0; q < M->P; ++q) {
                const int Lq = M->h_pat_len[q];
                uint16_t *r = rt.data() + (static_cast<size_t>(ph) * M->P + q) * kRegTw;
                r[0] = reg_row_head(M, q);
                const bool rev = M->K >= 1;
                for (int k = 0; k < kRegW; ++k) {
                    uint16_t off = static_cast<uint16_t>(NB * L * es);  // past the length: the zero window
                    if (k < Lq) {
                        const int64_t d = M->h_pat_off[static_cast<size_t>(q) * W + (rev ? Lq - 1 - k : k)];
                        const int w = window_of(d);
                        off = static_cast<uint16_t>((((ph + w) % NB) * L + (d - lo[w])) * es);
                    }
                    r[1 + k] = off;
                }
            }
        DevBuf &dst = es == 8 ? p.m_tab64 : p.m_tab32;
        dst.alloc(sizeof(uint16_t) * rt.size());
        SPMVC_HIP(hipMemcpy(dst.p, rt.data(), dst.bytes, hipMemcpyHostToDevice));
    }
    p.m_S = S;
    p.m_nz = (M->n_rows + S - 1) / S;
    p.m_lo0 = lo[0];
    p.m_np = static_cast<int32_t>((S + rows - 1) / rows);
    p.m_L = static_cast<int32_t>(L);
    p.m_NB = NB;
    p.m_NW = NW;
    p.m_zero_base = static_cast<int32_t>(NB * L);
    // blocks resident at once: LDS of 160 KB per CU, at most 6 per CU
    p.m_tab_lds = tab_lds;
    const int64_t block_lds = x_bytes64 + (tab_lds ? tab_bytes : 0);
    const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(6, (160 * 1024) / block_lds));
    const int64_t resident = per_cu * M->n_cu;
    const int64_t steps = static_cast<int64_t>(p.m_np) * p.m_nz;
    p.m_C = static_cast<int32_t>(std::max<int64_t>(1, (steps + resident - 1) / resident));
    p.march = true;
}

// Window-phased block SpMV plan: displacement windows for row tiles of
// kWinRows; per pattern and window the entry count and entries
// (canonical index << 16 | element offset in the window).  Applies to DIT
// matrices with a value table of 1 or 2 entries and no raw values, when no
// pattern has more than kWinMaxPw entries in one window.
// T_i[0] of every row using pattern q, when they all agree (DIT with two
// table values): the range over the rows, taken once per handle.
// With at most kT0LdsMax patterns each block first reduces its rows in LDS
// and then adds one global min and max per pattern it holds (a few patterns
// and millions of rows would otherwise serialize millions of global atomics
// on a handful of addresses); with more patterns the rows go to global memory
// directly.  The grid strides over the rows.
constexpr int kT0LdsMax = 4096;
__global__ void k_pattern_t0_range(int64_t n_rows, const void *ids, int id_bytes, const uint8_t *T, int P, int *tmin,
                                   int *tmax) {
    __shared__ int smin[kT0LdsMax], smax[kT0LdsMax];
    const bool local = P <= kT0LdsMax;
    if (local) {
        for (int q = threadIdx.x; q < P; q += blockDim.x) {
            smin[q] = 1 << 30;
            smax[q] = -1;
        }
        __syncthreads();
    }
    const uint32_t esc = id_bytes == 1 ? 0xFFu : (id_bytes == 2 ? 0xFFFFu : 0xFFFFFFFFu);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n_rows; i += stride) {
        const uint32_t id = load_id(ids, id_bytes, i);
        if (id == esc || id >= static_cast<uint32_t>(P)) continue;
        const int t = T[i];
        if (local) {
            atomicMin(&smin[id], t);
            atomicMax(&smax[id], t);
        } else {
            atomicMin(&tmin[id], t);
            atomicMax(&tmax[id], t);
        }
    }
    if (local) {
        __syncthreads();
        for (int q = threadIdx.x; q < P; q += blockDim.x)
            if (smax[q] >= 0) {
                atomicMin(&tmin[q], smin[q]);
                atomicMax(&tmax[q], smax[q]);
            }
    }
}

static void pattern_t0(spmvc_matrix_s *M) {
    if (M->pat_t0_ready) return;
    M->h_pat_t0.assign(static_cast<size_t>(M->P), -1);
    if (M->fold) {
        for (int q = 0; q < M->P; ++q) M->h_pat_t0[q] = M->h_pat_T[static_cast<size_t>(q) * M->K];
    } else if (M->P > 0 && M->n_rows > 0) {
        DevBuf tmin, tmax;
        tmin.alloc(sizeof(int) * M->P);
        tmax.alloc(sizeof(int) * M->P);
        std::vector<int> hmin(M->P, 1 << 30), hmax(M->P, -1);
        SPMVC_HIP(hipMemcpy(tmin.p, hmin.data(), tmin.bytes, hipMemcpyHostToDevice));
        SPMVC_HIP(hipMemcpy(tmax.p, hmax.data(), tmax.bytes, hipMemcpyHostToDevice));
        const unsigned g = static_cast<unsigned>(std::min<int64_t>((M->n_rows + kBlock - 1) / kBlock, 1024));
        k_pattern_t0_range<<<g, kBlock>>>(M->n_rows, M->ids.p, M->id_bytes, M->T.as<uint8_t>(), M->P, tmin.as<int>(),
                                          tmax.as<int>());
        SPMVC_CHECK_LAUNCH();
        SPMVC_HIP(hipMemcpy(hmin.data(), tmin.p, tmin.bytes, hipMemcpyDeviceToHost));
        SPMVC_HIP(hipMemcpy(hmax.data(), tmax.p, tmax.bytes, hipMemcpyDeviceToHost));
        for (int q = 0; q < M->P; ++q) M->h_pat_t0[q] = hmin[q] == hmax[q] ? hmin[q] : -1;
    }
    M->pat_t0_ready = true;
}

// Plan of the window-phased block SpMV (k_dit_block_win, and per system the
// batched k_bspmv_win): windows for kWinRows-row tiles and, per (pattern,
// window), a record of the entries of the pattern in that window.  When every
// row of each pattern shares its split between the V[0] and V[1] runs (one
// table value; DITV, whose T is the pattern's; DIT where the rows agree, as
// on a stencil), the record is split into the two runs (word 0: V[0] count,
// word 1: V[1] count, word 2: slot where the V[1] run starts, 4-aligned;
// entries are window element indices) and the kernels sum each run and scale
// it once.  Otherwise the record lists the entries in canonical order (word
// 0: count; entries (canonical index << 16) | window element) and each entry
// takes its weight by comparing its index with the row's T_i[0].
static void build_block_window_plan(spmvc_matrix_s *M, LdsPlan &p, const std::set<int64_t> &ds) {
    if (!(M->K == 1 || M->K == 2) || M->raw_elems > 0 || ds.empty()) return;
    // windows for kWinRows-row tiles: clusters closer than a tile merge
    std::vector<std::pair<int64_t, int64_t>> win;
    for (int64_t d : ds) {
        if (!win.empty() && d - win.back().second <= kWinRows)
            win.back().second = d;
        else
            win.push_back({d, d});
    }
    if (static_cast<int>(win.size()) > kMaxWindows) return;
    const int NW = static_cast<int>(win.size());
    int64_t lo[kMaxWindows], len[kMaxWindows];
    int64_t maxlen = 0;
    for (int w = 0; w < NW; ++w) {
        lo[w] = win[w].first - (((win[w].first % 4) + 4) % 4);
        len[w] = (kWinRows + win[w].second - lo[w] + 3) / 4 * 4;
        if (len[w] > 65535) return;
        maxlen = std::max(maxlen, len[w]);
    }
    const int W = M->width;
    const int stride = kWinSt;
    auto window_of = [&](int64_t d) {
        int w = 0;
        while (!(d >= win[w].first && d <= win[w].second)) ++w;
        return w;
    };
    std::vector<uint32_t> tab(static_cast<size_t>(M->P) * NW * stride, 0);
    for (int q = 0; q < M->P; ++q) {
        const int L = M->h_pat_len[q];
        for (int k = 0; k < L; ++k) {
            const int64_t d = M->h_pat_off[static_cast<size_t>(q) * W + k];
            const int w = window_of(d);
            uint32_t *t = tab.data() + (static_cast<size_t>(q) * NW + w) * stride;
            if (t[0] >= static_cast<uint32_t>(kWinMaxPw)) return;  // too many entries in one window
            t[4 + t[0]] = (static_cast<uint32_t>(k) << 16) | static_cast<uint32_t>(d - lo[w]);
            ++t[0];
        }
    }
    // the split form, where every pattern's rows share T_i[0] and the two
    // runs fit a record with the V[1] run moved to a 4-aligned slot
    p.bw_split = false;
    if (M->K == 2) pattern_t0(M);
    bool split = true;
    for (int q = 0; q < M->P && split; ++q) split = M->K == 1 || M->h_pat_t0[q] >= 0;
    std::vector<uint32_t> stab(static_cast<size_t>(M->P) * NW * stride, 0);
    for (int q = 0; q < M->P && split; ++q) {
        const int L = M->h_pat_len[q];
        const int t0 = M->K == 1 ? L : M->h_pat_t0[q];
        for (int w = 0; w < NW && split; ++w) {
            const uint32_t *g = tab.data() + (static_cast<size_t>(q) * NW + w) * stride;
            uint32_t *t = stab.data() + (static_cast<size_t>(q) * NW + w) * stride;
            uint32_t c0 = 0, c1 = 0;
            for (uint32_t e = 0; e < g[0]; ++e)
                ((static_cast<int>(g[4 + e] >> 16) < t0) ? c0 : c1) += 1;
            const uint32_t o1 = (c0 + 3) / 4 * 4;
            if (o1 + c1 > static_cast<uint32_t>(kWinMaxPw)) {
                split = false;
                break;
            }
            t[0] = c0;
            t[1] = c1;
            t[2] = o1;
            uint32_t j0 = 0, j1 = 0;
            for (uint32_t e = 0; e < g[0]; ++e) {
                const uint32_t elem = g[4 + e] & 0xFFFFu;
                if (static_cast<int>(g[4 + e] >> 16) < t0)
                    t[4 + j0++] = elem;
                else
                    t[4 + o1 + j1++] = elem;
            }
        }
    }
    if (split) {
        tab.swap(stab);
        p.bw_split = true;
    }
    p.bw_tab.alloc(sizeof(uint32_t) * tab.size());
    SPMVC_HIP(hipMemcpy(p.bw_tab.p, tab.data(), p.bw_tab.bytes, hipMemcpyHostToDevice));
    p.bw_nw = NW;
    p.bw_maxlen = static_cast<int32_t>(maxlen);
    for (int w = 0; w < NW; ++w) {
        p.bw_lo[w] = lo[w];
        p.bw_len[w] = static_cast<int32_t>(len[w]);
    }
    p.bw = true;
}

// Cut the displacement set into dense windows for `rows` rows per block and
// express the pattern table in LDS offsets (the plan of dtype dt).  All LDS
// use stays within kLdsBudgetBytes for FP64 elements (FP32 uses half of the x
// part).
void build_lds_plan(spmvc_matrix_s *M, int dt, int rows) {
    LdsPlan &p = M->plan[dt];
    p.tab.release();
    p.reg_tab64.release();
    p.reg_tab32.release();
    p.rows = rows;
    p.n_win = 0;
    p.total = 0;
    p.tab_in_lds = false;
    p.reg = false;
    p.reg_tab_in_lds = false;
    p.reg128 = false;
    p.reg_tab128.release();
    p.bw = false;
    p.bw_tab.release();
    p.march = false;
    p.m_tab64.release();
    p.m_tab32.release();
    const bool bmask = M->fmt == SPMVC_FMT_BMASK;
    if (bmask ? M->bm_nd == 0 : (M->fmt != SPMVC_FMT_DIT || M->P == 0 || M->width == 0)) return;
    const int W = M->width;
    std::set<int64_t> ds;
    if (bmask)
        ds.insert(M->h_bm_d.begin(), M->h_bm_d.end());
    else
        for (int q = 0; q < M->P; ++q)
            for (int k = 0; k < M->h_pat_len[q]; ++k) ds.insert(M->h_pat_off[static_cast<size_t>(q) * W + k]);
    if (ds.empty()) return;
    if (!bmask) build_block_window_plan(M, p, ds);  // independent of `rows`
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
        // start at a multiple of 4 elements (rows is a multiple of 256, so every
        // block's window start is 16-byte aligned), length a multiple of 4
        lo[w] = win[w].first - (((win[w].first % 4) + 4) % 4);
        len[w] = (rows + win[w].second - lo[w] + 3) / 4 * 4;
        base[w] = total;
        total += len[w];
    }
    if (total * static_cast<int64_t>(sizeof(double)) > kLdsBudgetBytes || total > 65535) return;
    auto lds_index = [&](int64_t d) -> int64_t {
        size_t w = 0;
        while (!(d >= win[w].first && d <= win[w].second)) ++w;
        return base[w] + d - lo[w];  // lo[w] <= win[w].first
    };
    if (bmask) {
        // the element offset of every displacement; no pattern tables.  The
        // kernel takes 1, 2 or 4 rows per thread.
        if (rows != kBlock && rows != 2 * kBlock && rows != 4 * kBlock) return;
        for (int k = 0; k < 64; ++k) p.bm_off[k] = 0;
        for (int k = 0; k < M->bm_nd; ++k) p.bm_off[k] = static_cast<int32_t>(lds_index(M->h_bm_d[k]));
        for (size_t w = 0; w < win.size(); ++w) {
            p.lo[w] = lo[w];
            p.len[w] = static_cast<int32_t>(len[w]);
            p.base[w] = static_cast<int32_t>(base[w]);
        }
        p.total = static_cast<int32_t>(total);
        p.n_win = static_cast<int>(win.size());
        return;
    }
    // walk-kernel table: [len, element index...]
    const int64_t tab_bytes = static_cast<int64_t>(M->P) * (W + 1) * static_cast<int64_t>(sizeof(uint16_t));
    std::vector<uint16_t> tab(static_cast<size_t>(M->P) * (W + 1), 0);
    for (int q = 0; q < M->P; ++q) {
        const int L = M->h_pat_len[q];
        tab[static_cast<size_t>(q) * (W + 1)] = static_cast<uint16_t>(L);
        for (int k = 0; k < L; ++k)
            tab[static_cast<size_t>(q) * (W + 1) + 1 + k] =
                static_cast<uint16_t>(lds_index(M->h_pat_off[static_cast<size_t>(q) * W + k]));
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

    // register-kernel table: [len, byte offset...] of the x windows; entries past
    // the length read zeros after the windows: FP64 one zero element (the
    // kernel clamps their offset 0xFFFF to it: one more VALU operation per
    // entry, a fifth less LDS per block), FP32 a zero window of one element per
    // row (the FP32 kernel spends its time on VALU, not on LDS capacity).  The
    // values must be finite (per dtype: a value finite in FP64 can be infinite
    // in FP32, and an infinite table value times 0 would give NaN)
    p.v_finite = true;
    for (int c = 0; c < M->K; ++c)
        p.v_finite = p.v_finite && (dt == SPMVC_F32 ? std::isfinite(M->V32[c]) : std::isfinite(M->V[c]));
    p.v_same_lo = true;
    for (int c = 0; c < M->K; ++c) {
        uint64_t b0, bc;
        std::memcpy(&b0, &M->V[0], 8);
        std::memcpy(&bc, &M->V[c], 8);
        p.v_same_lo = p.v_same_lo && (static_cast<uint32_t>(b0) == static_cast<uint32_t>(bc));
    }
    const int64_t x_elems = total + 1;  // FP64: the windows and the zero element
    const int64_t x_bytes64 = ((x_elems * 8) + 15) & ~int64_t(15);
    const int64_t x_bytes32 = (total + rows) * 4;  // FP32: the windows and the zero window
    const bool rows_ok = rows == 256 || rows == 512 || rows == 768 || rows == 1024 || rows == 2048;
    if (rows_ok && W <= kRegW && x_bytes64 <= kLdsBudgetBytes && x_elems * 8 <= 65535 && x_bytes32 <= 65535) {
        const int64_t reg_tab_bytes = static_cast<int64_t>(M->P) * kRegTw * 2;
        p.zero_base = static_cast<int32_t>(total);
        for (int es : {8, 4}) {
            std::vector<uint16_t> rt(static_cast<size_t>(M->P) * kRegTw, 0);
            for (int q = 0; q < M->P; ++q) {
                const int L = M->h_pat_len[q];
                uint16_t *r = rt.data() + static_cast<size_t>(q) * kRegTw;
                r[0] = reg_row_head(M, q);
                // dictionary kernels take the entries in reverse canonical order
                const bool rev = M->K >= 1;
                for (int k = 0; k < kRegW; ++k) {
                    // entries past the length: FP64 0xFFFF, which the kernel clamps to
                    // the zero element; FP32 the row's slot in the zero window
                    const int src = rev ? L - 1 - k : k;
                    r[1 + k] = k < L ? static_cast<uint16_t>(
                                           lds_index(M->h_pat_off[static_cast<size_t>(q) * W + src]) * es)
                                     : (es == 8 ? uint16_t(0xFFFF) : static_cast<uint16_t>(total * es));
                }
            }
            DevBuf &dst = es == 8 ? p.reg_tab64 : p.reg_tab32;
            dst.alloc(sizeof(uint16_t) * rt.size());
            SPMVC_HIP(hipMemcpy(dst.p, rt.data(), dst.bytes, hipMemcpyHostToDevice));
        }
        p.reg_tab_in_lds = reg_tab_bytes <= 16 * 1024 && x_bytes64 + reg_tab_bytes <= kLdsBudgetBytes;
        p.reg = true;
        // the same windows as 16-byte elements (pairs of FP64 right-hand sides)
        const int64_t x_elems128 = total + rows;  // windows + zero window
        const int64_t x_bytes128 = x_elems128 * 16;
        if (x_bytes128 + reg_tab_bytes <= kLdsBudgetBytes && x_elems128 * 16 <= 65535 && M->K >= 1) {
            std::vector<uint16_t> rt(static_cast<size_t>(M->P) * kRegTw, 0);
            for (int q = 0; q < M->P; ++q) {
                const int L = M->h_pat_len[q];
                uint16_t *r = rt.data() + static_cast<size_t>(q) * kRegTw;
                r[0] = reg_row_head(M, q);
                for (int k = 0; k < kRegW; ++k) {
                    const int64_t e = k < L ? lds_index(M->h_pat_off[static_cast<size_t>(q) * W + (L - 1 - k)]) : total;
                    r[1 + k] = static_cast<uint16_t>(e * 16);
                }
            }
            p.reg_tab128.alloc(sizeof(uint16_t) * rt.size());
            SPMVC_HIP(hipMemcpy(p.reg_tab128.p, rt.data(), p.reg_tab128.bytes, hipMemcpyHostToDevice));
            p.reg128 = true;
        }
    }
    build_march_plan(M, p, win, lo, len, rows);
}

int kernel_kind(const spmvc_matrix_s *M, int dt) {
    if (!uses_lds(M, dt)) return 0;
    if (M->fmt == SPMVC_FMT_BMASK) return 4;
    if (reg_variant(M, dt) == 0) return 1;
    return M->lds_mode[dt] == 2 && M->plan[dt].march ? 3 : 2;
}

void launch_spmv(const spmvc_matrix_s *M, int dt, const void *x, void *y, hipStream_t s, const int *skip) {
    if (dt == SPMVC_F64)
        launch_spmv_t<double>(M, x, y, s, skip);
    else
        launch_spmv_t<float>(M, x, y, s, skip);
}

// Blocks of the single-vector launch (main + escape), one dot partial each:
// the larger of the two dtypes' counts.
int64_t spmv_dot_blocks(const spmvc_matrix_s *M) {
    if (M->n_rows == 0) return 0;
    int64_t main = 0;
    for (int dt : {SPMVC_F64, SPMVC_F32}) {
        const LdsPlan &p = M->plan[dt];
        int64_t m = uses_lds(M, dt) ? (M->n_rows + p.rows - 1) / p.rows : (M->n_pad + kBlock - 1) / kBlock;
        if (uses_lds(M, dt) && p.march) m = std::max<int64_t>(m, p.m_np * ((p.m_nz + p.m_C - 1) / p.m_C));
        main = std::max(main, m);
    }
    return main + escape_blocks(M);
}

unsigned launch_spmv_dot(const spmvc_matrix_s *M, int dt, const void *x, void *y, hipStream_t s, const int *skip,
                         double *dot) {
    if (M->n_rows == 0) return 0;
    if (dt == SPMVC_F64) return launch_spmv_t<double>(M, x, y, s, skip, dot);
    return launch_spmv_t<float>(M, x, y, s, skip, dot);
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
    } else if (M->fmt == SPMVC_FMT_BMASK) {
        b += static_cast<int64_t>(M->bm_bytes) * M->n_pad * (M->K == 2 ? 2 : 1);  // masks
        b += M->raw_elems * vb;                                                  // values
        if (M->raw_elems) b += 8 * (M->n_pad / kSlice + 1);                      // slice pointers
        b += 4 * static_cast<int64_t>(M->bm_nd);                                 // D
    } else {
        if (!M->fold) b += static_cast<int64_t>(M->K) * M->n_pad;  // T (DITV: in the pattern table)
        b += M->raw_elems * vb;                               // raw values
        if (M->raw_elems) b += 8 * (M->n_pad / kSlice + 1);   // slice pointers
        if (M->fmt == SPMVC_FMT_DT)
            b += slots * 4;                                   // S
        else
            b += static_cast<int64_t>(M->id_bytes) * M->n_pad + static_cast<int64_t>(M->P) * (M->width + 1) * 2 +
                 (M->fold ? static_cast<int64_t>(M->P) * M->K : 0);
    }
    b += M->n_esc_nnz * (4 + vb) + M->n_esc * 16;
    return b;
}

// bounds violations the kernels of this file recorded (checked builds)
SPMVC_CHECK_READER(check_violations_spmv)

namespace {
__global__ void k_check_probe(int64_t i, int64_t n) {
    if (blockIdx.x == 0 && threadIdx.x == 0) (void)in_bounds<int64_t>(i, n);
}
}  // namespace

bool check_probe(int64_t i, int64_t n, hipStream_t s) {
#ifdef SPMVC_CHECK
    k_check_probe<<<1, 64, 0, s>>>(i, n);
    SPMVC_CHECK_LAUNCH();
    SPMVC_HIP(hipStreamSynchronize(s));
    return true;
#else
    (void)i;
    (void)n;
    (void)s;
    return false;
#endif
}

}  // namespace spmvc
