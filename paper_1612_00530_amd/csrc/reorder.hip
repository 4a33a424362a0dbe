// Reverse Cuthill-McKee reordering and the symmetric permutation B = P A P^T.
//
// Section V (after Table II) traces the gap between measured and theoretical
// SpMV speed to x being read through large column offsets, and proposes
// reordering the matrix and the vector.  Reverse Cuthill-McKee numbers the
// vertices breadth first so that each row's neighbours get nearby numbers.
//
// Numbering rules (they make the result unique): the graph is the pattern of
// A without the diagonal (A must be structurally symmetric); deg(v) is the
// number of off-diagonal entries of row v; each component starts at the
// unnumbered vertex of least (deg, index); within a breadth-first level the
// vertices are ordered by the least number among their neighbours in the
// level before, then (deg, index) -- the order in which Cuthill-McKee's queue
// appends them.  The sequence is then reversed.
//
// Level-synchronous on the GPU: per level, one launch finds each next-level
// vertex's least parent (atomicMin), one counts each parent's children, a scan
// places them, and one launch writes every parent's children in (deg, index)
// order.  Isolated vertices (deg 0) come first in index order, in one pass.
// Each further component costs one O(n) search for its start vertex.
#include <climits>

#include "internal.h"

namespace spmvc {
namespace {

constexpr int kR = 256;
constexpr int kBadRange = 1, kBadOrder = 2, kBadSym = 4;
// One thread orders a row's entries (or a vertex's children) by counting, in
// O(len^2): rows longer than this are refused rather than left to run for
// minutes in one thread.
constexpr int64_t kMaxRowLen = 1024;

unsigned rblocks(int64_t n) { return grid_for(std::max<int64_t>(n, 1), kR, 8192); }

// row_ptr monotone from 0 to nnz, columns in [0, n) and strictly ascending;
// flags[1] = longest row
__global__ __launch_bounds__(kR) void k_ro_validate(int64_t n, int64_t nnz, const int64_t *rp, const int32_t *col,
                                                   int *flags) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kR + threadIdx.x;
    if (g == 0 && (rp[0] != 0 || rp[n] != nnz)) atomicOr(flags, kBadRange);
    for (int64_t i = g; i < n; i += static_cast<int64_t>(gridDim.x) * kR) {
        const int64_t a = rp[i], b = rp[i + 1];
        if (a < 0 || b < a || b > nnz) {
            atomicOr(flags, kBadRange);
            continue;
        }
        atomicMax(&flags[1], static_cast<int>(b - a > INT_MAX ? INT_MAX : b - a));
        int64_t prev = -1;
        for (int64_t k = a; k < b; ++k) {
            const int64_t c = col[k];
            if (c < 0 || c >= n) {
                atomicOr(flags, kBadRange);
                break;
            }
            if (c <= prev) {
                atomicOr(flags, kBadOrder);
                break;
            }
            prev = c;
        }
    }
}

// every off-diagonal (i, j) has its mirror (j, i); run only on a validated matrix
__global__ __launch_bounds__(kR) void k_ro_symmetric(int64_t n, const int64_t *rp, const int32_t *col, int *flags) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kR + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kR) {
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int32_t j = col[k];
            if (j == i) continue;
            int64_t lo = rp[j], hi = rp[j + 1];  // binary search for i in row j
            while (lo < hi) {
                const int64_t mid = (lo + hi) / 2;
                if (col[mid] < i)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            if (lo == rp[j + 1] || col[lo] != i) {
                atomicOr(flags, kBadSym);
                return;
            }
        }
    }
}

// deg = off-diagonal count; num = -1 (unnumbered); key = INT_MAX (no parent yet);
// iso = 1 for isolated vertices
__global__ __launch_bounds__(kR) void k_ro_init(int64_t n, const int64_t *rp, const int32_t *col, int32_t *deg,
                                               int32_t *num, int32_t *key, int64_t *iso) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kR + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kR) {
        int32_t d = 0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) d += col[k] != i;
        deg[i] = d;
        num[i] = -1;
        key[i] = INT_MAX;
        iso[i] = d == 0;
    }
}

// isolated vertices numbered in index order (pos: exclusive scan of iso)
__global__ __launch_bounds__(kR) void k_ro_isolated(int64_t n, const int64_t *iso, const int64_t *pos, int32_t *num,
                                                   int32_t *order) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kR + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kR)
        if (iso[i]) {
            num[i] = static_cast<int32_t>(pos[i]);
            order[pos[i]] = static_cast<int32_t>(i);
        }
}

// least (deg, index) over unnumbered vertices, packed in one 64-bit key
__global__ __launch_bounds__(kR) void k_ro_start(int64_t n, const int32_t *deg, const int32_t *num,
                                                unsigned long long *best) {
    unsigned long long b = ~0ull;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kR + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kR)
        if (num[i] < 0) {
            const unsigned long long k = (static_cast<unsigned long long>(deg[i]) << 32) | static_cast<uint32_t>(i);
            b = k < b ? k : b;
        }
    if (b != ~0ull) atomicMin(best, b);
}

__global__ void k_ro_seed(const unsigned long long *best, int32_t label, int32_t *num, int32_t *order) {
    if (*best == ~0ull) return;  // no unnumbered vertex (cannot happen while labeled < n)
    const int32_t v = static_cast<int32_t>(*best & 0xffffffffull);
    num[v] = label;
    order[label] = v;
}

// for the parents order[base .. base + m): key[u] = least parent number of each
// unnumbered neighbour u
__global__ __launch_bounds__(kR) void k_ro_discover(int64_t base, int64_t m, const int32_t *order, const int64_t *rp,
                                                   const int32_t *col, const int32_t *num, int32_t *key) {
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * kR + threadIdx.x; t < m;
         t += static_cast<int64_t>(gridDim.x) * kR) {
        const int32_t p = order[base + t];
        const int32_t lab = static_cast<int32_t>(base + t);
        for (int64_t k = rp[p]; k < rp[p + 1]; ++k) {
            const int32_t u = col[k];
            if (u != p && num[u] < 0) atomicMin(&key[u], lab);
        }
    }
}

// children of each parent: its neighbours whose least parent it is.  Numbered
// vertices never hold a key in [base, base + m): theirs predate this level.
__global__ __launch_bounds__(kR) void k_ro_count(int64_t base, int64_t m, const int32_t *order, const int64_t *rp,
                                                const int32_t *col, const int32_t *key, int64_t *cnt) {
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * kR + threadIdx.x; t < m;
         t += static_cast<int64_t>(gridDim.x) * kR) {
        const int32_t p = order[base + t];
        const int32_t lab = static_cast<int32_t>(base + t);
        int64_t c = 0;
        for (int64_t k = rp[p]; k < rp[p + 1]; ++k) c += col[k] != p && key[col[k]] == lab;
        cnt[t] = c;
    }
}

// each parent numbers its children next + off[t] + (rank by (deg, index))
__global__ __launch_bounds__(kR) void k_ro_emit(int64_t base, int64_t m, int64_t next, const int64_t *off,
                                               const int32_t *deg, const int64_t *rp, const int32_t *col,
                                               const int32_t *key, int32_t *num, int32_t *order) {
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * kR + threadIdx.x; t < m;
         t += static_cast<int64_t>(gridDim.x) * kR) {
        const int32_t p = order[base + t];
        const int32_t lab = static_cast<int32_t>(base + t);
        const int64_t a = rp[p], b = rp[p + 1];
        for (int64_t k = a; k < b; ++k) {
            const int32_t u = col[k];
            if (u == p || key[u] != lab) continue;
            const int32_t du = deg[u];
            int64_t r = 0;
            for (int64_t k2 = a; k2 < b; ++k2) {
                const int32_t w = col[k2];
                if (w == p || key[w] != lab) continue;
                r += deg[w] < du || (deg[w] == du && w < u);
            }
            const int64_t pos = next + off[t] + r;
            num[u] = static_cast<int32_t>(pos);
            order[pos] = u;
        }
    }
}

__global__ __launch_bounds__(kR) void k_ro_reverse(int64_t n, const int32_t *order, int32_t *perm) {
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * kR + threadIdx.x; k < n;
         k += static_cast<int64_t>(gridDim.x) * kR)
        perm[k] = order[n - 1 - k];
}

// ---- B = P A P^T ----------------------------------------------------------------------

// bad unless perm is a permutation of [0, n); rank = inverse of perm
__global__ __launch_bounds__(kR) void k_pm_rank(int64_t n, const int32_t *perm, int32_t *rank, int *hits, int *bad) {
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * kR + threadIdx.x; k < n;
         k += static_cast<int64_t>(gridDim.x) * kR) {
        const int64_t o = perm[k];
        if (o < 0 || o >= n || atomicAdd(&hits[o], 1) != 0) {
            atomicOr(bad, 1);
            continue;
        }
        rank[o] = static_cast<int32_t>(k);
    }
}

__global__ __launch_bounds__(kR) void k_pm_len(int64_t n, const int32_t *perm, const int64_t *rp, int64_t *len) {
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * kR + threadIdx.x; k < n;
         k += static_cast<int64_t>(gridDim.x) * kR) {
        const int64_t o = perm[k];
        len[k] = rp[o + 1] - rp[o];
    }
}

// row k of B = row perm[k] of A, columns renamed by rank and put in ascending
// order (each entry's place = number of renamed columns below it; columns of a
// row are distinct)
__global__ __launch_bounds__(kR) void k_pm_rows(int64_t n, const int32_t *perm, const int32_t *rank, const int64_t *rp,
                                               const int32_t *col, const double *val, const int64_t *out_rp,
                                               int32_t *out_col, double *out_val) {
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * kR + threadIdx.x; k < n;
         k += static_cast<int64_t>(gridDim.x) * kR) {
        const int64_t o = perm[k], a = rp[o], b = rp[o + 1], dst = out_rp[k];
        for (int64_t e = a; e < b; ++e) {
            const int32_t c = rank[col[e]];
            int64_t r = 0;
            for (int64_t e2 = a; e2 < b; ++e2) r += rank[col[e2]] < c;
            out_col[dst + r] = c;
            out_val[dst + r] = val[e];
        }
    }
}

// row_ptr[n] read back, then the CSR checks of the reordering calls
int64_t validate_csr(int64_t n, const int64_t *rp, const int32_t *col, bool symmetric, hipStream_t s) {
    int64_t nnz = 0;
    SPMVC_HIP(hipMemcpyAsync(&nnz, rp + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPMVC_HIP(hipStreamSynchronize(s));
    if (nnz < 0) throw Error{SPMVC_ERANGE, "row_ptr[n] is negative"};
    if (nnz > 0 && !col) throw Error{SPMVC_EINVAL, "col_idx is null"};
    DevBuf flags;
    flags.alloc(2 * sizeof(int));
    SPMVC_HIP(hipMemsetAsync(flags.p, 0, 2 * sizeof(int), s));
    k_ro_validate<<<rblocks(n), kR, 0, s>>>(n, nnz, rp, col, flags.as<int>());
    SPMVC_CHECK_LAUNCH();
    int fl[2] = {0, 0};
    SPMVC_HIP(hipMemcpyAsync(fl, flags.p, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    SPMVC_HIP(hipStreamSynchronize(s));
    int f = fl[0];
    if (f & kBadRange) throw Error{SPMVC_ERANGE, "row_ptr not monotone / not ending at nnz, or a column out of range"};
    if (f & kBadOrder) throw Error{SPMVC_EUNSORTED, "column indices must be strictly ascending within each row"};
    if (fl[1] > kMaxRowLen) throw Error{SPMVC_EUNSUPPORTED, "reordering takes rows of at most 1024 entries"};
    if (symmetric) {
        k_ro_symmetric<<<rblocks(n), kR, 0, s>>>(n, rp, col, flags.as<int>());
        SPMVC_CHECK_LAUNCH();
        SPMVC_HIP(hipMemcpyAsync(&f, flags.p, sizeof(int), hipMemcpyDeviceToHost, s));
        SPMVC_HIP(hipStreamSynchronize(s));
        if (f & kBadSym) throw Error{SPMVC_EINVAL, "reordering needs a structurally symmetric matrix"};
    }
    return nnz;
}

}  // namespace

void rcm_order(int64_t n, const int64_t *rp, const int32_t *col, int32_t *perm, hipStream_t s) {
    if (n == 0) return;
    validate_csr(n, rp, col, true, s);
    DevBuf deg, num, key, order, a64, b64, best;
    deg.alloc(sizeof(int32_t) * n);
    num.alloc(sizeof(int32_t) * n);
    key.alloc(sizeof(int32_t) * n);
    order.alloc(sizeof(int32_t) * n);
    a64.alloc(sizeof(int64_t) * n);  // isolated flags, then children counts
    b64.alloc(sizeof(int64_t) * n);  // their exclusive scans
    best.alloc(sizeof(unsigned long long));
    int32_t *pdeg = deg.as<int32_t>(), *pnum = num.as<int32_t>(), *pkey = key.as<int32_t>(),
            *pord = order.as<int32_t>();
    k_ro_init<<<rblocks(n), kR, 0, s>>>(n, rp, col, pdeg, pnum, pkey, a64.as<int64_t>());
    SPMVC_CHECK_LAUNCH();
    int64_t labeled = exclusive_scan(a64.as<int64_t>(), b64.as<int64_t>(), n, s);
    k_ro_isolated<<<rblocks(n), kR, 0, s>>>(n, a64.as<int64_t>(), b64.as<int64_t>(), pnum, pord);
    SPMVC_CHECK_LAUNCH();
    while (labeled < n) {
        SPMVC_HIP(hipMemsetAsync(best.p, 0xff, sizeof(unsigned long long), s));
        k_ro_start<<<rblocks(n), kR, 0, s>>>(n, pdeg, pnum, best.as<unsigned long long>());
        k_ro_seed<<<1, 1, 0, s>>>(best.as<unsigned long long>(), static_cast<int32_t>(labeled), pnum, pord);
        SPMVC_CHECK_LAUNCH();
        int64_t base = labeled, m = 1;
        labeled += 1;
        while (m > 0) {
            k_ro_discover<<<rblocks(m), kR, 0, s>>>(base, m, pord, rp, col, pnum, pkey);
            k_ro_count<<<rblocks(m), kR, 0, s>>>(base, m, pord, rp, col, pkey, a64.as<int64_t>());
            SPMVC_CHECK_LAUNCH();
            const int64_t total = exclusive_scan(a64.as<int64_t>(), b64.as<int64_t>(), m, s);  // synchronises
            if (total > n - labeled) throw Error{SPMVC_EINVAL, "reordering numbered a vertex twice (inconsistent pattern)"};
            if (total > 0) {
                k_ro_emit<<<rblocks(m), kR, 0, s>>>(base, m, labeled, b64.as<int64_t>(), pdeg, rp, col, pkey, pnum,
                                                    pord);
                SPMVC_CHECK_LAUNCH();
            }
            base = labeled;
            m = total;
            labeled += total;
        }
    }
    k_ro_reverse<<<rblocks(n), kR, 0, s>>>(n, pord, perm);
    SPMVC_CHECK_LAUNCH();
    SPMVC_HIP(hipStreamSynchronize(s));
}

void permute_csr(int64_t n, const int64_t *rp, const int32_t *col, const double *val, const int32_t *perm,
                 int64_t *out_rp, int32_t *out_col, double *out_val, hipStream_t s) {
    const int64_t nnz = validate_csr(n, rp, col, false, s);
    if (nnz > 0 && (!val || !out_col || !out_val)) throw Error{SPMVC_EINVAL, "vals / out_col_idx / out_vals is null"};
    if (n > 0) {
        DevBuf rank, hits, bad, len;
        rank.alloc(sizeof(int32_t) * n);
        hits.alloc(sizeof(int) * n);
        bad.alloc(sizeof(int));
        len.alloc(sizeof(int64_t) * n);
        SPMVC_HIP(hipMemsetAsync(hits.p, 0, sizeof(int) * n, s));
        SPMVC_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
        k_pm_rank<<<rblocks(n), kR, 0, s>>>(n, perm, rank.as<int32_t>(), hits.as<int>(), bad.as<int>());
        SPMVC_CHECK_LAUNCH();
        int f = 0;
        SPMVC_HIP(hipMemcpyAsync(&f, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
        SPMVC_HIP(hipStreamSynchronize(s));
        if (f) throw Error{SPMVC_EINVAL, "perm is not a permutation of 0..n-1"};
        k_pm_len<<<rblocks(n), kR, 0, s>>>(n, perm, rp, len.as<int64_t>());
        SPMVC_CHECK_LAUNCH();
        exclusive_scan(len.as<int64_t>(), out_rp, n, s);
        k_pm_rows<<<rblocks(n), kR, 0, s>>>(n, perm, rank.as<int32_t>(), rp, col, val, out_rp, out_col, out_val);
        SPMVC_CHECK_LAUNCH();
    }
    SPMVC_HIP(hipMemcpyAsync(out_rp + n, &nnz, sizeof(int64_t), hipMemcpyHostToDevice, s));
    SPMVC_HIP(hipStreamSynchronize(s));
}

}  // namespace spmvc
