// Internal declarations of libspmvc (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/spmvc.h"

namespace spmvc {

constexpr int kMaxK = 15;           // value-table capacity
constexpr int kMaxPatternLen = 255; // T and positions are one byte
constexpr int kSlice = 64;          // rows per raw-value slice (one wavefront)
constexpr int kMaxWindows = 8;      // x windows staged in LDS per block
constexpr int kLdsBudgetBytes = 64 * 1024;
// Register tiles above which an SpMV with the dot product (CG) takes the
// marching form of its plan, where it has one (each block leaves a partial that
// every block of the next kernel sums): measured at 192^3, FP64 CG 36.2 ms with
// 13,824 register tiles of 512 rows, 35.2 ms with the marching form's 1,009
// blocks; at 104^3 the 1,465 tiles of 768 rows are the faster choice.  The
// autotuner avoids configurations past it that have no marching form.
constexpr int64_t kDotMaxTiles = 8192;
constexpr int kBlock = 256;         // threads per block of the SpMV kernels
constexpr int32_t kEscapeColumn = -2; // ELL/DT slot-0 marker of an escape row (padding is -1)

// ---- errors -------------------------------------------------------------------------
void set_error(const std::string &msg);
spmvc_status fail(spmvc_status st, const std::string &msg);

struct Error {
    spmvc_status st;
    std::string msg;
};

#define SPMVC_HIP(call)                                                                     \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            throw ::spmvc::Error{e_ == hipErrorOutOfMemory ? SPMVC_ENOMEM : SPMVC_EHIP,     \
                                 std::string(#call) + ": " + hipGetErrorString(e_)};        \
    } while (0)

#define SPMVC_CHECK_LAUNCH() SPMVC_HIP(hipGetLastError())

// ---- device buffers ------------------------------------------------------------------
// Device memory comes from the allocator set with spmvc_set_allocator, else
// hipMalloc / hipFree.  Each buffer keeps the allocator that gave it its
// memory and returns it there, so changing the allocator never mixes them.
struct Allocator {
    void *(*alloc)(size_t, hipStream_t, void *) = nullptr;
    void (*free)(void *, hipStream_t, void *) = nullptr;
    void *ctx = nullptr;
};
Allocator current_allocator();  // api.cpp

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    Allocator owner;  // where p came from (hipMalloc when owner.alloc is null)
    void alloc(size_t n) {
        release();
        if (n == 0) return;
        owner = current_allocator();
        if (owner.alloc) {
            p = owner.alloc(n, nullptr, owner.ctx);
            if (!p) throw Error{SPMVC_ENOMEM, "the allocator set with spmvc_set_allocator returned NULL"};
        } else {
            SPMVC_HIP(hipMalloc(&p, n));
        }
        bytes = n;
    }
    void release() {
        if (p) {
            if (owner.alloc)
                owner.free(p, nullptr, owner.ctx);
            else
                (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
};

// ---- LDS staging plan of the DIT kernel for one rows-per-block value ------------------
struct LdsPlan {
    int rows = 0;                 // rows per block this plan was built for
    int n_win = 0;                // 0 = plan not usable (direct gather)
    int64_t lo[kMaxWindows] = {}; // window w holds x[r0+lo[w] .. r0+rows-1+hi[w]]
    int32_t len[kMaxWindows] = {};
    int32_t base[kMaxWindows] = {}; // element offset of window w in LDS
    int32_t total = 0;            // LDS elements of the x windows
    bool tab_in_lds = false;      // table small enough to copy into LDS per block
    DevBuf tab;                   // uint16 [P][width+1]: length, then LDS element index per entry
    // register kernel (patterns of at most kRegW entries): rows of kRegTw uint16 =
    // length, then the LDS *byte* offset of each entry; entries past the length
    // point at a window of `rows` zeros, so every row runs the same kRegW steps.
    bool reg = false;
    int32_t zero_base = 0;        // element offset of the zero window (after the x windows)
    bool reg_tab_in_lds = false;
    DevBuf reg_tab64, reg_tab32;  // byte offsets for FP64 and FP32 elements
    bool reg128 = false;          // the windows also fit as 16-byte elements (block SpMV,
    DevBuf reg_tab128;            //   pairs of FP64 right-hand sides): offsets for those
    // window-phased block SpMV (whole right-hand-side rows in LDS, one window
    // at a time, row tiles of kWinRows): windows, and per pattern and window
    // a kWinSt-word record: the count and the entries
    // ((canonical index << 16) | element in window)
    bool bw = false;
    bool bw_split = false;        // records split into value runs (see build_block_window_plan)
    int32_t bw_nw = 0, bw_maxlen = 0;
    int64_t bw_lo[kMaxWindows] = {};
    int32_t bw_len[kMaxWindows] = {};
    DevBuf bw_tab;
    bool v_finite = false;        // every value-table entry finite (v * 0 == 0)
    bool v_same_lo = false;       // value-table entries share their low 32 bits
    // plane-marching form of the register kernel: windows equally spaced by
    // m_S rows, a ring of m_NB = windows + 1 buffers of m_L elements, one
    // table per ring phase (m_NB tables of P rows of kRegTw uint16)
    bool march = false;
    bool m_tab_lds = false;       // the phase tables are copied into LDS
    int64_t m_S = 0, m_nz = 0, m_lo0 = 0;
    int32_t m_np = 0, m_C = 1, m_L = 0, m_NB = 0, m_NW = 0, m_zero_base = 0;
    DevBuf m_tab64, m_tab32;
    // neighbour-bitmask format: LDS element offset of each displacement D[k]
    // relative to the row's own position in its block
    int32_t bm_off[64] = {};
};

constexpr int kRegW = 31;   // longest pattern the register kernel takes
constexpr int kWinRows = 256;   // row tile of the window-phased block SpMV
constexpr int kWinMaxPw = 32;   // most entries of one pattern in one window (window-phased)
// uint32 words per (pattern, window) record of the window-phased table: the
// count, three unused words, then up to kWinMaxPw entries, zero-padded, so
// the entries can be read four at a time with 16-byte loads
constexpr int kWinSt = 4 + kWinMaxPw;
constexpr int kRegTw = 32;  // uint16 per register-table row (64 bytes, 16-byte aligned)

}  // namespace spmvc

// The opaque handle.
struct spmvc_matrix_s {
    int64_t n_rows = 0, n_cols = 0, nnz = 0, n_pad = 0;
    int32_t fmt = SPMVC_FMT_DIT;  // ELL, DT, DIT or BMASK (DITV is DIT with fold set)
    int32_t fold = 0;             // DITV: T_i registered per pattern (pat_T), no per-row T
    int32_t K = 0, P = 0, id_bytes = 1, width = 0, max_raw = 0;
    int32_t f32_shadow = 1;
    double V[spmvc::kMaxK] = {};
    float V32[spmvc::kMaxK] = {};
    int64_t n_esc = 0, n_esc_nnz = 0, n_raw = 0, raw_elems = 0;
    // device arrays
    spmvc::DevBuf ell_val, ell_col, dt_S, ids, T, pat_off, pat_len, pat_T, raw, raw32, raw_slice,
        esc_rows, esc_ptr, esc_col, esc_val, esc_val32, V_dev;
    // neighbour-bitmask format (BMASK): the ascending displacement list D and,
    // per row, a mask over D (bm_bytes = 4 when |D| <= 32, else 8) and, with
    // two table values, a mask of the entries holding V[1]
    int32_t bm_nd = 0, bm_bytes = 4;
    spmvc::DevBuf bm_d, bm_mask, bm_vmask;
    std::vector<int32_t> h_bm_d;
    // host copies of the (small) pattern table, for LDS plans
    std::vector<int32_t> h_pat_off; // [P][width]
    std::vector<uint8_t> h_pat_len; // [P]
    std::vector<uint8_t> h_pat_T;   // [P][K], DITV only
    // per pattern, the T_i[0] every row using it shares, or -1 when its rows
    // differ (DIT with two table values; computed on first use)
    std::vector<int32_t> h_pat_t0;
    bool pat_t0_ready = false;
    // kernel configuration
    int32_t rows_per_block[2] = {512, 512};  // per dtype (index SPMVC_F64 / SPMVC_F32)
    int32_t lds_mode[2] = {1, 1};          // per dtype: 1 = stage in LDS when a plan fits,
                                           // 2 = as 1, plane-marching where it applies
    spmvc::LdsPlan plan[2];                // per dtype
    int32_t block_mode[2] = {3, 3};        // per dtype, several right-hand sides: 3 = whole rows
                                           // of the block in LDS one window at a time, 2 = x windows
                                           // of right-hand-side pairs in LDS (3 and 2 where they
                                           // apply, else 1); 1 = a lane group per row; 0 = one lane
                                           // per row (all rhs)
    spmvc_compress_opts copts{};          // the options the handle was compressed with
    // multicolor Gauss-Seidel (symgs.hip): greedy coloring, built on first use
    int32_t gs_ready = 0, gs_n_colors = 0;
    int32_t gs_contig = 0;                // the rows of each color are one contiguous range
                                          // (a color-ordered twin): no row lists

    std::vector<int64_t> gs_off;          // rows of color c: gs_rows[gs_off[c] .. gs_off[c+1])
    spmvc::DevBuf gs_rows, gs_color;      // int32 [n]: rows by color (ascending); color of each row
    spmvc::DevBuf gs_meta;                // DIT: uint32 [n] per entry of gs_rows: (T_i[0] << 24) | pattern ID
    int32_t block_rows = 256;   // spmv_block: rows per block
    int32_t n_xcd = 8;          // XCDs of the device (block-to-tile mapping)
    int32_t n_cu = 256;         // compute units of the device (grid sizing)
};

namespace spmvc {

// api.cpp: kernel plans and device properties of a freshly compressed handle
void prepare_handle(spmvc_matrix_s *M);

// compress.hip
void compress(spmvc_matrix_s *M, const int64_t *row_ptr, const int32_t *col, const double *val,
              const spmvc_compress_opts &o, hipStream_t s);
void decompress(const spmvc_matrix_s *M, int64_t *row_ptr, int32_t *col, double *val,
                hipStream_t s);

// spmv.hip
void build_lds_plan(spmvc_matrix_s *M, int dt, int rows);
// `skip` (device int, may be null): when *skip != 0 the kernels return at once.
void launch_spmv(const spmvc_matrix_s *M, int dt, const void *x, void *y, hipStream_t s,
                 const int *skip = nullptr);
void launch_spmv_block(const spmvc_matrix_s *M, int dt, int nrhs, const void *X, int64_t ldx,
                       void *Y, int64_t ldy, hipStream_t s, const int *skip = nullptr);
int64_t stream_bytes(const spmvc_matrix_s *M, int dt);
// y = A x that also writes one partial of x.y per block into dot (FP64); returns
// the number of partials (= spmv_dot_blocks(M)).  Used by CG for p.Ap.
unsigned launch_spmv_dot(const spmvc_matrix_s *M, int dt, const void *x, void *y, hipStream_t s,
                         const int *skip, double *dot);
int64_t spmv_dot_blocks(const spmvc_matrix_s *M);

// reorder.hip (blocking; throw Error on a bad matrix or permutation)
void rcm_order(int64_t n, const int64_t *rp, const int32_t *col, int32_t *perm, hipStream_t s);
void permute_csr(int64_t n, const int64_t *rp, const int32_t *col, const double *val, const int32_t *perm,
                 int64_t *out_rp, int32_t *out_col, double *out_val, hipStream_t s);

// cg.hip
spmvc_status cg_solve_mg_impl(spmvc_matrix const *levels, const int32_t *const *f2c, int n_levels, const double *b,
                              double *x, const spmvc_cg_opts &o, spmvc_cg_stat *stat, hipStream_t s);
spmvc_status cg_solve_impl(const spmvc_matrix *A, int n_sys, int nrhs, const double *const *b,
                           double *const *x, const spmvc_cg_opts &o, spmvc_cg_stat *stat,
                           hipStream_t s);
// FP64 CG of one system with every buffer in the library's static scratch
// region (no allocation); blocking; throws Error beyond the region's limits.
spmvc_status cg_solve_noalloc_impl(const spmvc_matrix_s *M, const double *b, double *x,
                                   const spmvc_cg_opts &o, spmvc_cg_stat &stat, hipStream_t s);
int64_t cg_noalloc_max_rows();

// batched.hip
// Kernel one spmv of dtype dt launches: 0 direct gather, 1 DIT LDS walk, 2 DIT register,
// 3 DIT register, plane-marching.
int kernel_kind(const spmvc_matrix_s *M, int dt);
bool batched_supported(const spmvc_matrix *A, int n_sys);
void batched_note_fallback();
void batched_last_tune(int32_t *form, int32_t *chunk, double *us);
spmvc_status cg_solve_batched(const spmvc_matrix *A, int n_sys, int nrhs, const double *const *b,
                              double *const *x, const spmvc_cg_opts &o, spmvc_cg_stat *stat,
                              hipStream_t s, bool use_graph);

// symgs.hip
void build_coloring(spmvc_matrix_s *M, hipStream_t s);  // blocking; throws Error on a bad matrix
// A new handle (owned by the caller, blocking) holding B = P A P^T, P listing
// M's rows color by color (each color's rows ascending: M->gs_rows),
// compressed with M's options, with the coloring induced from M's (color c =
// rows gs_off[c] .. gs_off[c+1] of B): a sweep on B computes the same updates
// as a sweep on M, in its own numbering.  perm (device int32 [n], may be
// null) receives P's row list.
spmvc_matrix_s *color_order_copy(spmvc_matrix_s *M, int32_t *perm, hipStream_t s);
// `skip` (device int, may be null): when *skip != 0 the sweep's kernels return at once.
void launch_symgs(const spmvc_matrix_s *M, const double *b, double *x, int sweeps, hipStream_t s,
                  const int *skip = nullptr, bool reverse = false);

// Bounds violations recorded by the kernels of spmv.hip, batched.hip and
// symgs.hip since the last read (always 0 unless built with -DSPMVC_CHECK).
unsigned long long check_violations_spmv();
unsigned long long check_violations_batched();
unsigned long long check_violations_symgs();
// Checked builds: one kernel passes index i against [0, n) through the kernels'
// bounds check (so a test can see a violation recorded); false otherwise.
bool check_probe(int64_t i, int64_t n, hipStream_t s);

// scan.hip: exclusive prefix sum of n int64 values (in may equal out); returns the total.
int64_t exclusive_scan(const int64_t *in, int64_t *out, int64_t n, hipStream_t s);

inline unsigned grid_for(int64_t work, int block, unsigned cap = 1u << 20) {
    int64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return static_cast<unsigned>(g);
}

}  // namespace spmvc
