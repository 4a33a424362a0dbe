// GPU compressor and decompressor for the ELL, DT, DIT and DITV formats.
//
// The steps follow Section V: (1) scan all values and build the ascending
// value table V; (2) sort each row's entries by value, ties by column (the
// sorted column list S_i); (3) record each value's run end (terminal indices
// T_i); (4) turn columns into displacements from the diagonal; (5) register
// each row's displacement sequence in a pattern table and store its type ID;
// (6, DITV) register T_i with the sequence as well, so the row keeps only the
// ID and each pattern its T.
//
// Everything that touches per-entry or per-row data runs in the kernels
// below.  The host only sizes and allocates, reads back a handful of scalars,
// and -- only when more than p_max patterns qualify -- ranks the qualifying
// patterns' (count, first row) pairs to pick the p_max most frequent.
//
// Determinism: counts are exact (hash tables keyed by the full 64-bit value
// pattern / sequence hash, verified); V is ordered by IEEE totalOrder; pattern
// IDs are ranks of the patterns' first rows; nothing depends on the order in
// which blocks run.
#include <algorithm>
#include <cstdlib>

#include "internal.h"

namespace spmvc {
namespace {

constexpr uint64_t kEmpty = ~0ull;
constexpr int kFlagRange = 1, kFlagUnsorted = 2, kFlagCollision = 4, kFlagOverflow = 8,
              kFlagCandOverflow = 16, kFlagBmValueSentinel = 32;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t total_order_key(uint64_t b) {
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ uint64_t load_relaxed(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct VTab {
    uint64_t b[kMaxK];
    int K;
};

__device__ __forceinline__ int code_of(uint64_t bits, const VTab &v) {
    for (int c = 0; c < v.K; ++c)
        if (bits == v.b[c]) return c;
    return v.K;
}

__device__ __forceinline__ uint64_t bits_of(const double *val, int64_t k) {
    return __double_as_longlong(val[k]);
}

// ---- step 0: CSR validation ----------------------------------------------------------
__global__ void k_validate(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *rp,
                           const int32_t *col, int *flags) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g == 0 && (rp[0] != 0 || rp[n_rows] != nnz)) atomicOr(flags, kFlagRange);
    for (int64_t i = g; i < n_rows; i += stride) {
        const int64_t a = rp[i], b = rp[i + 1];
        if (a < 0 || b < a || b > nnz) {
            atomicOr(flags, kFlagRange);
            continue;
        }
        int64_t prev = -1;
        for (int64_t k = a; k < b; ++k) {
            const int64_t c = col[k];
            if (c < 0 || c >= n_cols) {
                atomicOr(flags, kFlagRange);
                break;
            }
            if (c <= prev) {
                atomicOr(flags, kFlagUnsorted);
                break;
            }
            prev = c;
        }
    }
}

// ---- exact counting of 64-bit keys: block-local LDS table, then a global table -------
struct GTable {
    uint64_t *keys;
    uint32_t *cnt;
    int64_t *minidx; // may be null
    uint64_t mask;   // capacity - 1
    int *fill;       // occupied slots
    int fill_limit;
    int *flags;
};

// Bounded insert: a key that finds no slot within kMaxProbe steps, or would
// push the fill past fill_limit, raises kFlagOverflow instead (the host then
// recounts with more partitions), so no insert can run long.
constexpr uint64_t kMaxProbe = 1024;

__device__ void g_insert(const GTable &t, uint64_t key, uint32_t c, int64_t idx) {
    uint64_t s = mix64(key) & t.mask;
    const uint64_t limit = t.mask < kMaxProbe ? t.mask + 1 : kMaxProbe;
    for (uint64_t probe = 0; probe < limit; ++probe) {
        uint64_t k = load_relaxed(&t.keys[s]);
        if (k == kEmpty) {
            if (__hip_atomic_load(t.fill, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= t.fill_limit) {
                atomicOr(t.flags, kFlagOverflow);
                return;
            }
            const uint64_t old = atomicCAS(reinterpret_cast<unsigned long long *>(&t.keys[s]),
                                           static_cast<unsigned long long>(kEmpty),
                                           static_cast<unsigned long long>(key));
            if (old == kEmpty) {
                if (atomicAdd(t.fill, 1) >= t.fill_limit) atomicOr(t.flags, kFlagOverflow);
                k = key;
            } else {
                k = old;
            }
        }
        if (k == key) {
            atomicAdd(&t.cnt[s], c);
            if (t.minidx) atomicMin(reinterpret_cast<long long *>(&t.minidx[s]), static_cast<long long>(idx));
            return;
        }
        s = (s + 1) & t.mask;
    }
    atomicOr(t.flags, kFlagOverflow);
}

constexpr int kLocalSlots = 512;
constexpr int kAggThreads = 256;
constexpr int kAggChunk = 8192;

// keys[i] for i in [0, n); kEmpty keys are skipped (counted in *sentinel when given).
// With n_parts > 1 only keys whose hash falls in partition `part` are counted.
__global__ __launch_bounds__(kAggThreads) void k_aggregate(const uint64_t *keys, int64_t n,
                                                           GTable t, int n_parts, int part,
                                                           unsigned long long *sentinel) {
    __shared__ uint64_t lkey[kLocalSlots];
    __shared__ uint32_t lcnt[kLocalSlots];
    __shared__ int64_t lmin[kLocalSlots];
    for (int s = threadIdx.x; s < kLocalSlots; s += blockDim.x) {
        lkey[s] = kEmpty;
        lcnt[s] = 0;
        lmin[s] = INT64_MAX;
    }
    __syncthreads();
    const int64_t chunks = (n + kAggChunk - 1) / kAggChunk;
    for (int64_t ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
        const int64_t end = min(n, (ch + 1) * kAggChunk);
        for (int64_t i = ch * kAggChunk + threadIdx.x; i < end; i += blockDim.x) {
            const uint64_t key = keys[i];
            if (key == kEmpty) {
                if (sentinel && part == 0) atomicAdd(sentinel, 1ull);
                continue;
            }
            const uint64_t h = mix64(key);
            if (n_parts > 1 && static_cast<int>((h >> 40) % static_cast<uint64_t>(n_parts)) != part)
                continue;
            uint32_t s = static_cast<uint32_t>(h) & (kLocalSlots - 1);
            bool done = false;
            for (int p = 0; p < 8 && !done; ++p) {
                uint64_t k = __hip_atomic_load(&lkey[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (k == kEmpty) {
                    const uint64_t old = atomicCAS(reinterpret_cast<unsigned long long *>(&lkey[s]),
                                                   static_cast<unsigned long long>(kEmpty),
                                                   static_cast<unsigned long long>(key));
                    k = (old == kEmpty) ? key : old;
                }
                if (k == key) {
                    atomicAdd(&lcnt[s], 1u);
                    if (t.minidx) atomicMin(reinterpret_cast<long long *>(&lmin[s]), static_cast<long long>(i));
                    done = true;
                } else {
                    s = (s + 1) & (kLocalSlots - 1);
                }
            }
            if (!done) g_insert(t, key, 1u, i);
        }
    }
    __syncthreads();
    for (int s = threadIdx.x; s < kLocalSlots; s += blockDim.x)
        if (lkey[s] != kEmpty && lcnt[s] > 0) g_insert(t, lkey[s], lcnt[s], lmin[s]);
}

__global__ void k_fill_u64(uint64_t *p, uint64_t v, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_i64(int64_t *p, int64_t v, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Move every table entry with 8*count > n_rows into the candidate list, then clear it.
__global__ void k_extract_candidates(GTable t, int64_t cap, int64_t n_rows, uint64_t *cand_key,
                                     uint32_t *cand_cnt, int *cand_n, int cand_cap) {
    const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= cap) return;
    const uint64_t k = t.keys[s];
    if (k != kEmpty && 8ll * static_cast<int64_t>(t.cnt[s]) > n_rows) {
        const int j = atomicAdd(cand_n, 1);
        if (j < cand_cap) {
            cand_key[j] = k;
            cand_cnt[j] = t.cnt[s];
        } else {
            atomicOr(t.flags, kFlagCandOverflow);
        }
    }
    t.keys[s] = kEmpty;
    t.cnt[s] = 0;
}

// Pick the k_max most frequent candidates (ties: totalOrder), output sorted by totalOrder.
__global__ void k_select_dictionary(const uint64_t *cand_key, const uint32_t *cand_cnt,
                                    const int *cand_n_ptr, const unsigned long long *sentinel,
                                    int64_t n_rows, int k_max, uint64_t *v_out, int *k_out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int n = *cand_n_ptr;
    const unsigned long long sent = *sentinel;
    uint64_t chosen[kMaxK];
    int K = 0;
    for (; K < k_max; ++K) {
        bool found = false;
        uint64_t best_key = 0, best_tok = 0;
        unsigned long long best_cnt = 0;
        for (int j = 0; j <= n; ++j) {
            uint64_t key;
            unsigned long long c;
            if (j < n) {
                key = cand_key[j];
                c = cand_cnt[j];
            } else {
                if (!(8ull * sent > static_cast<unsigned long long>(n_rows))) continue;
                key = kEmpty;
                c = sent;
            }
            bool taken = false;
            for (int q = 0; q < K; ++q) taken |= (chosen[q] == key);
            if (taken) continue;
            const uint64_t tok = total_order_key(key);
            if (!found || c > best_cnt || (c == best_cnt && tok < best_tok)) {
                found = true;
                best_key = key;
                best_cnt = c;
                best_tok = tok;
            }
        }
        if (!found) break;
        chosen[K] = best_key;
    }
    // insertion sort by totalOrder
    for (int a = 1; a < K; ++a) {
        const uint64_t v = chosen[a];
        int b = a - 1;
        while (b >= 0 && total_order_key(chosen[b]) > total_order_key(v)) {
            chosen[b + 1] = chosen[b];
            --b;
        }
        chosen[b + 1] = v;
    }
    for (int c = 0; c < K; ++c) v_out[c] = chosen[c];
    *k_out = K;
}

// ---- steps 2-4: canonical order, T_i, displacement-sequence hash ----------------------
__device__ __forceinline__ uint64_t seq_hash_step(uint64_t h, int32_t d) {
    return (h ^ static_cast<uint32_t>(d)) * 0x100000001B3ull;
}

__device__ __forceinline__ uint64_t seq_hash_final(uint64_t h, int64_t len, int bits) {
    uint64_t r = mix64(h ^ (static_cast<uint64_t>(len) * 0x9E3779B97F4A7C15ull));
    if (bits < 64) r &= (1ull << bits) - 1;
    return r == kEmpty ? kEmpty - 1 : r;
}

struct RowArgs {
    int64_t n_rows, n_pad;
    const int64_t *rp;
    const int32_t *col;
    const double *val;
    VTab v;
    int fold;  // DITV: a pattern is (displacement sequence, T_i)
    // pattern hash: seed (a hash collision between two different sequences
    // makes the compressor hash again with the next seed) and width in bits
    // (64; narrower only to exercise that retry in tests)
    uint64_t hash_seed = 0;
    int hash_bits = 64;
};

__global__ void k_canon(RowArgs a, uint8_t *T, int32_t *nraw, uint64_t *hash, uint8_t *is_long) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n_rows) return;
    const int64_t b0 = a.rp[i], b1 = a.rp[i + 1];
    const int64_t len = b1 - b0;
    if (len > kMaxPatternLen) {
        is_long[i] = 1;
        for (int c = 0; c < a.v.K; ++c) T[c * a.n_pad + i] = 0;
        nraw[i] = 0;
        hash[i] = kEmpty;
        return;
    }
    is_long[i] = 0;
    uint64_t h = 0xCBF29CE484222325ull ^ mix64(a.hash_seed);
    int pos = 0;
    for (int c = 0; c <= a.v.K; ++c) {
        for (int64_t k = b0; k < b1; ++k) {
            if (code_of(bits_of(a.val, k), a.v) != c) continue;
            h = seq_hash_step(h, static_cast<int32_t>(static_cast<int64_t>(a.col[k]) - i));
            ++pos;
        }
        if (c < a.v.K) T[c * a.n_pad + i] = static_cast<uint8_t>(pos);
    }
    const int coded = a.v.K ? T[(a.v.K - 1) * a.n_pad + i] : 0;
    nraw[i] = static_cast<int32_t>(len) - coded;
    if (a.fold)  // the registered key includes T_i (with V fixed: the values)
        for (int c = 0; c < a.v.K; ++c) h = seq_hash_step(h, 0x40000000 + T[c * a.n_pad + i]);
    hash[i] = seq_hash_final(h, len, a.hash_bits);
}

// Cursor over one row's entries in canonical (code, column) order.
struct Cursor {
    int64_t b0, b1, k;
    int c;
};

__device__ __forceinline__ bool cursor_next(Cursor &cu, const RowArgs &a, int32_t &col_out,
                                            int &code_out) {
    while (cu.c <= a.v.K) {
        while (cu.k < cu.b1) {
            const int64_t k = cu.k++;
            if (code_of(bits_of(a.val, k), a.v) == cu.c) {
                col_out = a.col[k];
                code_out = cu.c;
                return true;
            }
        }
        ++cu.c;
        cu.k = cu.b0;
    }
    return false;
}

__device__ __forceinline__ Cursor cursor_begin(const RowArgs &a, int64_t i) {
    Cursor c;
    c.b0 = a.rp[i];
    c.b1 = a.rp[i + 1];
    c.k = c.b0;
    c.c = 0;
    return c;
}

__device__ __forceinline__ int64_t table_find(const GTable &t, uint64_t key) {
    uint64_t s = mix64(key) & t.mask;
    for (uint64_t probe = 0; probe <= t.mask; ++probe) {
        const uint64_t k = t.keys[s];
        if (k == key) return static_cast<int64_t>(s);
        if (k == kEmpty) return -1;
        s = (s + 1) & t.mask;
    }
    return -1;
}

// Each row finds its sequence's slot and checks that it equals the first row's sequence.
__global__ void k_pattern_lookup(RowArgs a, GTable t, const uint64_t *hash, const uint8_t *is_long,
                                 int64_t *rowslot) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n_rows) return;
    if (is_long[i]) {
        rowslot[i] = -1;
        return;
    }
    const int64_t s = table_find(t, hash[i]);
    if (s < 0) {
        atomicOr(t.flags, kFlagCollision);
        rowslot[i] = -1;
        return;
    }
    rowslot[i] = s;
    const int64_t rep = t.minidx[s];
    if (rep == i) return;
    if (rep < 0 || rep >= a.n_rows || (a.rp[rep + 1] - a.rp[rep]) != (a.rp[i + 1] - a.rp[i])) {
        atomicOr(t.flags, kFlagCollision);
        return;
    }
    Cursor x = cursor_begin(a, i), y = cursor_begin(a, rep);
    int32_t cx, cy;
    int kx, ky;
    while (true) {
        const bool hx = cursor_next(x, a, cx, kx);
        const bool hy = cursor_next(y, a, cy, ky);
        if (hx != hy) {
            atomicOr(t.flags, kFlagCollision);
            return;
        }
        if (!hx) break;
        if (static_cast<int64_t>(cx) - i != static_cast<int64_t>(cy) - rep || (a.fold && kx != ky)) {
            atomicOr(t.flags, kFlagCollision);
            return;
        }
    }
}

__global__ void k_mark_keep(GTable t, int64_t cap, int min_rows, uint8_t *keep, int *n_keep) {
    const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= cap) return;
    const bool k = t.keys[s] != kEmpty && static_cast<int>(t.cnt[s]) >= min_rows;
    keep[s] = k ? 1 : 0;
    if (k) atomicAdd(n_keep, 1);
}

__global__ void k_list_keep(const uint8_t *keep, int64_t cap, int64_t *list, int *n) {
    const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= cap) return;
    if (keep[s]) list[atomicAdd(n, 1)] = s;
}

__global__ void k_set_keep(uint8_t *keep, const int64_t *slots, int n) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) keep[slots[j]] = 1;
}

// is_rep[i] = 1 when row i is the first row of a kept pattern.
__global__ void k_rep_flags(int64_t n_rows, const int64_t *rowslot, const int64_t *minidx,
                            const uint8_t *keep, int64_t *is_rep) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_rows) return;
    const int64_t s = rowslot[i];
    is_rep[i] = (s >= 0 && keep[s] && minidx[s] == i) ? 1 : 0;
}

// After the scan, pid[i] is the ID of the pattern first used by row i (valid when rep).
__global__ void k_slot_ids(const int64_t *rowslot, const int64_t *minidx, const uint8_t *keep,
                           const int64_t *pid, int64_t n_rows, int64_t *slot_id, const int64_t *rp,
                           int *width) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_rows) return;
    const int64_t s = rowslot[i];
    if (s >= 0 && keep[s] && minidx[s] == i) {
        slot_id[s] = pid[i];
        atomicMax(width, static_cast<int>(rp[i + 1] - rp[i]));
    }
}

template <class IdT>
__global__ void k_write_ids(const int64_t *rowslot, const uint8_t *keep, const int64_t *slot_id,
                            int64_t n_rows, int64_t n_pad, IdT *ids, uint8_t *esc) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    if (i >= n_rows) {
        ids[i] = static_cast<IdT>(~static_cast<IdT>(0));
        return;
    }
    const int64_t s = rowslot[i];
    const bool kept = s >= 0 && keep[s];
    ids[i] = kept ? static_cast<IdT>(slot_id[s]) : static_cast<IdT>(~static_cast<IdT>(0));
    esc[i] = kept ? 0 : 1;
}

// Pattern table row p = canonical displacement sequence of the pattern's first row.
__global__ void k_write_patterns(RowArgs a, const int64_t *rowslot, const int64_t *minidx,
                                 const uint8_t *keep, const int64_t *slot_id, int width,
                                 int32_t *pat_off, uint8_t *pat_len, const uint8_t *T, uint8_t *pat_T) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n_rows) return;
    const int64_t s = rowslot[i];
    if (!(s >= 0 && keep[s] && minidx[s] == i)) return;
    const int64_t p = slot_id[s];
    Cursor cu = cursor_begin(a, i);
    int32_t c;
    int code;
    int k = 0;
    while (cursor_next(cu, a, c, code)) {
        pat_off[p * width + k] = static_cast<int32_t>(static_cast<int64_t>(c) - i);
        ++k;
    }
    pat_len[p] = static_cast<uint8_t>(k);
    if (pat_T)
        for (int cc = 0; cc < a.v.K; ++cc) pat_T[p * a.v.K + cc] = T[cc * a.n_pad + i];
}

// Escape rows (long rows for ELL/DT; plus unkept patterns for DIT).
__global__ void k_escape_flags(int64_t n_rows, const int64_t *rp, const uint8_t *esc,
                               int64_t *eflag, int64_t *elen) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_rows) return;
    const bool e = esc[i] != 0;
    eflag[i] = e ? 1 : 0;
    elen[i] = e ? (rp[i + 1] - rp[i]) : 0;
}

__global__ void k_escape_fill(RowArgs a, const uint8_t *esc, const int64_t *eidx, const int64_t *eoff,
                              int64_t n_esc, int64_t n_esc_nnz, int64_t *esc_rows, int64_t *esc_ptr,
                              int32_t *esc_col, double *esc_val, float *esc_val32) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i == 0) esc_ptr[n_esc] = n_esc_nnz;
    if (i >= a.n_rows || !esc[i]) return;
    const int64_t e = eidx[i], o = eoff[i];
    esc_rows[e] = i;
    esc_ptr[e] = o;
    for (int64_t k = a.rp[i]; k < a.rp[i + 1]; ++k) {
        esc_col[o + k - a.rp[i]] = a.col[k];
        esc_val[o + k - a.rp[i]] = a.val[k];
        if (esc_val32) esc_val32[o + k - a.rp[i]] = static_cast<float>(a.val[k]);
    }
}

// T of escape rows is zero; max length of non-escape rows (ELL/DT width).
__global__ void k_fix_escape_T(int64_t n_rows, int64_t n_pad, int K, const uint8_t *esc, uint8_t *T,
                               int32_t *nraw, const int64_t *rp, int *width) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_rows) return;
    if (esc[i]) {
        for (int c = 0; c < K; ++c) T[c * n_pad + i] = 0;
        nraw[i] = 0;
    } else if (width) {
        atomicMax(width, static_cast<int>(rp[i + 1] - rp[i]));
    }
}

// Raw values are stored in slices of 64 rows, column-major inside a slice.
__global__ void k_slice_widths(int64_t n_rows, int64_t n_slices, const int32_t *nraw,
                               int64_t *slice_elems, int *max_raw, unsigned long long *n_raw) {
    const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= n_slices) return;
    int w = 0;
    long long tot = 0;
    for (int l = 0; l < kSlice; ++l) {
        const int64_t i = s * kSlice + l;
        if (i >= n_rows) break;
        w = max(w, nraw[i]);
        tot += nraw[i];
    }
    slice_elems[s] = static_cast<int64_t>(w) * kSlice;
    if (w) atomicMax(max_raw, w);
    if (tot) atomicAdd(n_raw, static_cast<unsigned long long>(tot));
}

__global__ void k_raw_fill(RowArgs a, const uint8_t *esc, const int32_t *nraw, const int64_t *slice,
                           double *raw, float *raw32) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n_rows || esc[i] || nraw[i] == 0) return;
    const int64_t base = slice[i / kSlice] + (i % kSlice);
    int k = 0;
    for (int64_t e = a.rp[i]; e < a.rp[i + 1]; ++e) {
        const double v = a.val[e];
        if (code_of(__double_as_longlong(v), a.v) != a.v.K) continue;
        raw[base + static_cast<int64_t>(k) * kSlice] = v;
        if (raw32) raw32[base + static_cast<int64_t>(k) * kSlice] = static_cast<float>(v);
        ++k;
    }
}

// DT: S_i in canonical order, column-major [width][n_pad].
__global__ void k_dt_fill(RowArgs a, const uint8_t *esc, int width, int32_t *S) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n_rows) return;
    if (esc[i]) {
        S[i] = kEscapeColumn;  // slot 0 marks rows served by the escape path
        return;
    }
    Cursor cu = cursor_begin(a, i);
    int32_t c;
    int code;
    int k = 0;
    while (cursor_next(cu, a, c, code) && k < width) {
        S[static_cast<int64_t>(k) * a.n_pad + i] = c;
        ++k;
    }
}

// ELL: columns and values in stored order, column-major [width][n_pad].
__global__ void k_ell_fill(RowArgs a, const uint8_t *esc, int width, int32_t *ecol, double *evals) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n_rows) return;
    if (esc[i]) {
        ecol[i] = kEscapeColumn;  // slot 0 marks rows served by the escape path
        return;
    }
    int k = 0;
    for (int64_t e = a.rp[i]; e < a.rp[i + 1] && k < width; ++e, ++k) {
        ecol[static_cast<int64_t>(k) * a.n_pad + i] = a.col[e];
        evals[static_cast<int64_t>(k) * a.n_pad + i] = a.val[e];
    }
}

__global__ void k_long_flags(int64_t n_rows, const int64_t *rp, uint8_t *esc) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_rows) return;
    esc[i] = (rp[i + 1] - rp[i]) > kMaxPatternLen ? 1 : 0;
}

// ---- decompression ------------------------------------------------------------------
// ---- neighbour-bitmask format (BMASK) -------------------------------------------------
// The pattern table reduced to one list: D = every displacement col - row of
// the matrix, ascending; a row stores a bitmask over D.  Distinct keys (the
// displacements, and the values to decide the value table) are gathered in a
// small open-addressing set; a key is looked up before any atomic, so the
// few insertions are the only contended operations.
constexpr int kBmSetCap = 1024;    // slots of the displacement set (power of two)
constexpr int kBmMaxDisp = 64;     // displacements a 64-bit mask holds
constexpr int kBmValCap = 16;      // slots of the value set

__device__ __forceinline__ void small_set_insert(unsigned long long *set, int cap, uint64_t key, int *count) {
    uint64_t s = mix64(key) & static_cast<uint64_t>(cap - 1);
    for (int probe = 0; probe < cap; ++probe) {
        const unsigned long long v = __atomic_load_n(&set[s], __ATOMIC_RELAXED);
        if (v == key) return;
        if (v == kEmpty) {
            const unsigned long long old = atomicCAS(&set[s], kEmpty, static_cast<unsigned long long>(key));
            if (old == kEmpty) {
                atomicAdd(count, 1);
                return;
            }
            if (old == key) return;
        }
        s = (s + 1) & static_cast<uint64_t>(cap - 1);
    }
}

// Every entry's displacement (stored as d + 2^32, never the empty key) into
// the set; rows stop once more than kBmMaxDisp keys are known.
__global__ void k_bm_disp(int64_t n_rows, const int64_t *rp, const int32_t *col, unsigned long long *set, int *count) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_rows) return;
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
        if (__atomic_load_n(count, __ATOMIC_RELAXED) > kBmMaxDisp) return;
        const int64_t d = static_cast<int64_t>(col[k]) - i;
        small_set_insert(set, kBmSetCap, static_cast<uint64_t>(d + (int64_t(1) << 32)), count);
    }
}

// The distinct values (bit patterns), up to three of them (the empty key's own
// bit pattern, a NaN, is reported by a flag instead).
__global__ void k_bm_values(int64_t nnz, const uint64_t *bits, unsigned long long *set, int *count, int *flags) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < nnz; k += stride) {
        if (__atomic_load_n(count, __ATOMIC_RELAXED) > 2) return;
        const uint64_t b = bits[k];
        if (b == kEmpty)
            atomicOr(flags, kFlagBmValueSentinel);
        else
            small_set_insert(set, kBmValCap, b, count);
    }
}

// Row i: its mask over D (bit k for the entry at column i + D[k]) and, with
// two table values, the mask of its V[1] entries; raw count (all entries when
// there is no table); longest row.
template <class MaskT>
__global__ void k_bm_rows(RowArgs a, const int32_t *D, int nd, MaskT *mask, MaskT *vmask, int32_t *nraw,
                          int *width) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n_rows) return;
    MaskT m = 0, vm = 0;
    for (int64_t k = a.rp[i]; k < a.rp[i + 1]; ++k) {
        const int64_t d = static_cast<int64_t>(a.col[k]) - i;
        int lo = 0, hi = nd - 1;  // D is ascending and holds d
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (D[mid] < d)
                lo = mid + 1;
            else
                hi = mid;
        }
        const MaskT bit = static_cast<MaskT>(1) << lo;
        m |= bit;
        if (a.v.K == 2 && code_of(bits_of(a.val, k), a.v) == 1) vm |= bit;
    }
    mask[i] = m;
    if (vmask) vmask[i] = vm;
    const int len = static_cast<int>(a.rp[i + 1] - a.rp[i]);
    nraw[i] = a.v.K == 0 ? len : 0;
    atomicMax(width, len);
}

struct DecArgs {
    int64_t n_rows, n_pad;
    int fmt, K, width, id_bytes;
    const double *V;
    const uint8_t *T;
    const uint8_t *pat_T;  // DITV: T of each pattern [P][K]; T is then unused
    const void *ids;
    const int32_t *pat_off;
    const uint8_t *pat_len;
    const int32_t *S;
    const int32_t *ell_col;
    const double *ell_val;
    const double *raw;
    const int64_t *raw_slice;
    const int64_t *esc_rows, *esc_ptr;
    const int32_t *esc_col;
    const double *esc_val;
    const int64_t *esc_of_row; // [n_rows], -1 when not an escape row
    // BMASK
    const int32_t *bm_d;
    const void *bm_mask, *bm_vmask;
    int32_t bm_bytes;
};

__device__ __forceinline__ uint64_t dec_mask(const void *m, int bytes, int64_t i) {
    return bytes == 4 ? static_cast<const uint32_t *>(m)[i] : static_cast<const uint64_t *>(m)[i];
}

__device__ __forceinline__ uint32_t dec_id(const DecArgs &a, int64_t i) {
    if (a.id_bytes == 1) return static_cast<const uint8_t *>(a.ids)[i];
    if (a.id_bytes == 2) return static_cast<const uint16_t *>(a.ids)[i];
    return static_cast<const uint32_t *>(a.ids)[i];
}

__device__ __forceinline__ uint32_t esc_marker(int id_bytes) {
    return id_bytes == 1 ? 0xFFu : (id_bytes == 2 ? 0xFFFFu : 0xFFFFFFFFu);
}

__device__ int64_t dec_len(const DecArgs &a, int64_t i) {
    const int64_t e = a.esc_of_row[i];
    if (e >= 0) return a.esc_ptr[e + 1] - a.esc_ptr[e];
    if (a.fmt == SPMVC_FMT_BMASK) return __popcll(dec_mask(a.bm_mask, a.bm_bytes, i));
    if (a.fmt == SPMVC_FMT_DIT) {
        const uint32_t id = dec_id(a, i);
        return id == esc_marker(a.id_bytes) ? 0 : a.pat_len[id];
    }
    const int32_t *cols = a.fmt == SPMVC_FMT_DT ? a.S : a.ell_col;
    int64_t n = 0;
    for (int k = 0; k < a.width; ++k)
        if (cols[static_cast<int64_t>(k) * a.n_pad + i] >= 0) ++n;
    return n;
}

__global__ void k_dec_len(DecArgs a, int64_t *len) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < a.n_rows) len[i] = dec_len(a, i);
}

__global__ void k_esc_of_row(int64_t n_esc, const int64_t *esc_rows, int64_t *esc_of_row) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e < n_esc) esc_of_row[esc_rows[e]] = e;
}

__global__ void k_dec_fill(DecArgs a, const int64_t *out_rp, int32_t *out_col, double *out_val) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n_rows) return;
    const int64_t o = out_rp[i];
    const int64_t n = out_rp[i + 1] - o;
    const int64_t e = a.esc_of_row[i];
    if (e >= 0) {
        for (int64_t k = 0; k < n; ++k) {
            out_col[o + k] = a.esc_col[a.esc_ptr[e] + k];
            out_val[o + k] = a.esc_val[a.esc_ptr[e] + k];
        }
        return;
    }
    if (a.fmt == SPMVC_FMT_ELL) {
        int64_t j = 0;
        for (int k = 0; k < a.width && j < n; ++k) {
            const int32_t c = a.ell_col[static_cast<int64_t>(k) * a.n_pad + i];
            if (c < 0) continue;
            out_col[o + j] = c;
            out_val[o + j] = a.ell_val[static_cast<int64_t>(k) * a.n_pad + i];
            ++j;
        }
        return;
    }
    if (a.fmt == SPMVC_FMT_BMASK) {  // set bits in ascending order = columns ascending
        uint64_t m = dec_mask(a.bm_mask, a.bm_bytes, i);
        const uint64_t vm = a.K == 2 ? dec_mask(a.bm_vmask, a.bm_bytes, i) : 0;
        const int64_t slice_base = a.K == 0 ? a.raw_slice[i / kSlice] + (i % kSlice) : 0;
        for (int64_t j = 0; m; ++j) {
            const int k = __builtin_ctzll(m);
            m &= m - 1;
            out_col[o + j] = static_cast<int32_t>(i + a.bm_d[k]);
            out_val[o + j] = a.K == 0 ? a.raw[slice_base + j * kSlice] : a.V[(vm >> k) & 1];
        }
        return;
    }
    // DT / DIT: canonical order, then sort by column (insertion sort, <= 255 entries)
    const uint32_t id = a.fmt == SPMVC_FMT_DIT ? dec_id(a, i) : 0;
    const int64_t slice_base = a.raw_slice ? a.raw_slice[i / kSlice] + (i % kSlice) : 0;
    // T_i: the row's own (DT, DIT) or its pattern's (DITV)
    const uint8_t *Ti = a.pat_T ? a.pat_T + static_cast<int64_t>(id) * a.K : a.T + i;
    const int64_t ts = a.pat_T ? 1 : a.n_pad;
    const int coded_end = a.K ? Ti[(a.K - 1) * ts] : 0;
    int c = 0;
    for (int64_t k = 0; k < n; ++k) {
        while (c < a.K && k >= Ti[c * ts]) ++c;
        int32_t colk;
        if (a.fmt == SPMVC_FMT_DIT)
            colk = static_cast<int32_t>(i + a.pat_off[static_cast<int64_t>(id) * a.width + k]);
        else
            colk = a.S[k * a.n_pad + i];
        const double v = (c < a.K) ? a.V[c] : a.raw[slice_base + (k - coded_end) * kSlice];
        // insert (colk, v) into the sorted prefix
        int64_t j = k - 1;
        while (j >= 0 && out_col[o + j] > colk) {
            out_col[o + j + 1] = out_col[o + j];
            out_val[o + j + 1] = out_val[o + j];
            --j;
        }
        out_col[o + j + 1] = colk;
        out_val[o + j + 1] = v;
    }
}

int64_t next_pow2(int64_t v) {
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

template <class T> T read_scalar(const void *dev, hipStream_t s) {
    T v{};
    SPMVC_HIP(hipMemcpyAsync(&v, dev, sizeof(T), hipMemcpyDeviceToHost, s));
    SPMVC_HIP(hipStreamSynchronize(s));
    return v;
}

constexpr int kT = 256;

}  // namespace

// ---------------------------------------------------------------------------------------
void compress(spmvc_matrix_s *M, const int64_t *rp, const int32_t *col, const double *val,
              const spmvc_compress_opts &o_in, hipStream_t s) {
    const int64_t n = M->n_rows, nnz = M->nnz;
    M->n_pad = ((n + kSlice - 1) / kSlice) * kSlice;
    const int64_t n_pad = M->n_pad;
    // DITV is DIT whose pattern key also holds T_i; the row's T is dropped at the end
    spmvc_compress_opts o = o_in;
    M->copts = o_in;
    M->fold = o.fmt == SPMVC_FMT_DITV ? 1 : 0;
    if (M->fold) o.fmt = SPMVC_FMT_DIT;
    M->fmt = o.fmt;
    M->f32_shadow = o.f32_shadow ? 1 : 0;

    DevBuf flags_b;
    flags_b.alloc(64);
    SPMVC_HIP(hipMemsetAsync(flags_b.p, 0, 64, s));
    int *flags = flags_b.as<int>();

    // step 0: validate the CSR before anything reads through it
    if (n > 0 || nnz > 0) {
        k_validate<<<grid_for(n, kT, 4096), kT, 0, s>>>(n, M->n_cols, nnz, rp, col, flags);
        SPMVC_CHECK_LAUNCH();
        const int f = read_scalar<int>(flags, s);
        if (f & kFlagRange) throw Error{SPMVC_ERANGE, "row_ptr not monotone / not ending at nnz, or a column index is out of range"};
        if (f & kFlagUnsorted) throw Error{SPMVC_EUNSORTED, "column indices must be strictly ascending within each row"};
    }
    if (n == 0) {
        M->K = 0;
        M->P = 0;
        if (M->fold) {
            M->pat_T.alloc(16);
            SPMVC_HIP(hipMemsetAsync(M->pat_T.p, 0, 16, s));
            SPMVC_HIP(hipStreamSynchronize(s));
        }
        return;
    }

    // step 1: value table V (not needed for ELL)
    VTab vt{};
    vt.K = 0;
    if (o.fmt == SPMVC_FMT_BMASK && o.k_max > 0 && nnz > 0) {
        // the table holds the matrix's values when there are at most two (and
        // k_max allows them), ascending in totalOrder; else every value is raw
        DevBuf vset, vcnt;
        vset.alloc(sizeof(unsigned long long) * kBmValCap);
        vcnt.alloc(sizeof(int));
        k_fill_u64<<<1, kBmValCap, 0, s>>>(vset.as<uint64_t>(), kEmpty, kBmValCap);
        SPMVC_HIP(hipMemsetAsync(vcnt.p, 0, sizeof(int), s));
        SPMVC_HIP(hipMemsetAsync(flags, 0, sizeof(int), s));
        k_bm_values<<<grid_for(nnz, kT, 4096), kT, 0, s>>>(nnz, reinterpret_cast<const uint64_t *>(val),
                                                          vset.as<unsigned long long>(), vcnt.as<int>(), flags);
        SPMVC_CHECK_LAUNCH();
        std::vector<uint64_t> hv(kBmValCap);
        SPMVC_HIP(hipMemcpyAsync(hv.data(), vset.p, vset.bytes, hipMemcpyDeviceToHost, s));
        const int f = read_scalar<int>(flags, s);
        std::vector<uint64_t> distinct;
        for (uint64_t b : hv)
            if (b != kEmpty) distinct.push_back(b);
        if (f & kFlagBmValueSentinel) distinct.push_back(kEmpty);
        if (static_cast<int>(distinct.size()) <= std::min(o.k_max, 2)) {
            auto tok = [](uint64_t b) { return (b >> 63) ? ~b : (b | (1ull << 63)); };  // totalOrder key
            std::sort(distinct.begin(), distinct.end(), [&](uint64_t x, uint64_t y) { return tok(x) < tok(y); });
            vt.K = static_cast<int>(distinct.size());
            for (int c = 0; c < vt.K; ++c) vt.b[c] = distinct[c];
        }
    } else if (o.fmt != SPMVC_FMT_ELL && o.k_max > 0 && nnz > 0) {
        const int64_t cap = std::min<int64_t>(next_pow2(std::max<int64_t>(2 * nnz, 1024)), 1ll << 24);
        DevBuf keys, cnt, fill, cand_key, cand_cnt, cand_n, sent, vout, kout;
        keys.alloc(sizeof(uint64_t) * cap);
        cnt.alloc(sizeof(uint32_t) * cap);
        fill.alloc(sizeof(int));
        const int cand_cap = static_cast<int>(std::min<int64_t>(8 * nnz / n + 64, 1 << 22));
        cand_key.alloc(sizeof(uint64_t) * cand_cap);
        cand_cnt.alloc(sizeof(uint32_t) * cand_cap);
        cand_n.alloc(sizeof(int));
        sent.alloc(sizeof(unsigned long long));
        vout.alloc(sizeof(uint64_t) * kMaxK);
        kout.alloc(sizeof(int));
        GTable t{keys.as<uint64_t>(), cnt.as<uint32_t>(), nullptr, static_cast<uint64_t>(cap - 1),
                 fill.as<int>(), static_cast<int>(cap / 2), flags};
        int n_parts = 1;
        while (true) {
            k_fill_u64<<<grid_for(cap, kT, 0x7fffffff), kT, 0, s>>>(keys.as<uint64_t>(), kEmpty, cap);
            SPMVC_HIP(hipMemsetAsync(cnt.p, 0, cnt.bytes, s));
            SPMVC_HIP(hipMemsetAsync(cand_n.p, 0, sizeof(int), s));
            SPMVC_HIP(hipMemsetAsync(sent.p, 0, sizeof(unsigned long long), s));
            SPMVC_HIP(hipMemsetAsync(flags, 0, sizeof(int), s));
            bool overflow = false;
            for (int part = 0; part < n_parts && !overflow; ++part) {
                SPMVC_HIP(hipMemsetAsync(fill.p, 0, sizeof(int), s));
                k_aggregate<<<grid_for(nnz, kAggChunk, 2048), kAggThreads, 0, s>>>(
                    reinterpret_cast<const uint64_t *>(val), nnz, t, n_parts, part,
                    sent.as<unsigned long long>());
                SPMVC_CHECK_LAUNCH();
                k_extract_candidates<<<grid_for(cap, kT, 0x7fffffff), kT, 0, s>>>(
                    t, cap, n, cand_key.as<uint64_t>(), cand_cnt.as<uint32_t>(), cand_n.as<int>(), cand_cap);
                SPMVC_CHECK_LAUNCH();
                const int f = read_scalar<int>(flags, s);
                if (f & kFlagCandOverflow) throw Error{SPMVC_EUNSUPPORTED, "value-table candidate list overflow"};
                overflow = (f & kFlagOverflow) != 0;
            }
            if (!overflow) break;
            if (n_parts >= 4096) throw Error{SPMVC_EUNSUPPORTED, "too many distinct values to count"};
            n_parts *= 8;
        }
        k_select_dictionary<<<1, 64, 0, s>>>(cand_key.as<uint64_t>(), cand_cnt.as<uint32_t>(),
                                              cand_n.as<int>(), sent.as<unsigned long long>(), n,
                                              std::min(o.k_max, kMaxK), vout.as<uint64_t>(), kout.as<int>());
        SPMVC_CHECK_LAUNCH();
        uint64_t vb[kMaxK] = {};
        int K = 0;
        SPMVC_HIP(hipMemcpyAsync(vb, vout.p, sizeof(vb), hipMemcpyDeviceToHost, s));
        SPMVC_HIP(hipMemcpyAsync(&K, kout.p, sizeof(int), hipMemcpyDeviceToHost, s));
        SPMVC_HIP(hipStreamSynchronize(s));
        vt.K = K;
        for (int c = 0; c < K; ++c) vt.b[c] = vb[c];
    }
    M->K = vt.K;
    for (int c = 0; c < vt.K; ++c) {
        std::memcpy(&M->V[c], &vt.b[c], sizeof(double));
        M->V32[c] = static_cast<float>(M->V[c]);
    }
    if (M->K > 0) {
        M->V_dev.alloc(sizeof(double) * kMaxK + sizeof(float) * kMaxK);
        SPMVC_HIP(hipMemcpyAsync(M->V_dev.p, M->V, sizeof(double) * kMaxK, hipMemcpyHostToDevice, s));
        SPMVC_HIP(hipMemcpyAsync(static_cast<char *>(M->V_dev.p) + sizeof(double) * kMaxK, M->V32,
                                 sizeof(float) * kMaxK, hipMemcpyHostToDevice, s));
    }

    RowArgs ra{n, n_pad, rp, col, val, vt, M->fold};
    const unsigned gr = grid_for(n, kT, 0x7fffffff);

    DevBuf esc_b;
    esc_b.alloc(n_pad);
    SPMVC_HIP(hipMemsetAsync(esc_b.p, 0, n_pad, s));
    uint8_t *esc = esc_b.as<uint8_t>();
    DevBuf nraw_b;
    nraw_b.alloc(sizeof(int32_t) * n_pad);
    SPMVC_HIP(hipMemsetAsync(nraw_b.p, 0, nraw_b.bytes, s));

    if (o.fmt == SPMVC_FMT_ELL) {
        k_long_flags<<<gr, kT, 0, s>>>(n, rp, esc);
        SPMVC_CHECK_LAUNCH();
    } else if (o.fmt == SPMVC_FMT_BMASK) {
        // the displacement list D, then every row's masks
        DevBuf dset, dcnt;
        dset.alloc(sizeof(unsigned long long) * kBmSetCap);
        dcnt.alloc(sizeof(int));
        k_fill_u64<<<grid_for(kBmSetCap, kT, 64), kT, 0, s>>>(dset.as<uint64_t>(), kEmpty, kBmSetCap);
        SPMVC_HIP(hipMemsetAsync(dcnt.p, 0, sizeof(int), s));
        k_bm_disp<<<gr, kT, 0, s>>>(n, rp, col, dset.as<unsigned long long>(), dcnt.as<int>());
        SPMVC_CHECK_LAUNCH();
        const int cnt = read_scalar<int>(dcnt.p, s);
        if (cnt > kBmMaxDisp)
            throw Error{SPMVC_EUNSUPPORTED, "the matrix has more than 64 distinct displacements (col - row); "
                                            "the bitmask format holds at most 64"};
        std::vector<uint64_t> hs(kBmSetCap);
        SPMVC_HIP(hipMemcpyAsync(hs.data(), dset.p, dset.bytes, hipMemcpyDeviceToHost, s));
        SPMVC_HIP(hipStreamSynchronize(s));
        M->h_bm_d.clear();
        for (uint64_t k : hs)
            if (k != kEmpty) M->h_bm_d.push_back(static_cast<int32_t>(static_cast<int64_t>(k) - (int64_t(1) << 32)));
        std::sort(M->h_bm_d.begin(), M->h_bm_d.end());
        M->bm_nd = static_cast<int32_t>(M->h_bm_d.size());
        M->bm_bytes = M->bm_nd <= 32 ? 4 : 8;
        M->bm_d.alloc(sizeof(int32_t) * M->bm_nd);
        if (M->bm_nd > 0)
            SPMVC_HIP(hipMemcpyAsync(M->bm_d.p, M->h_bm_d.data(), sizeof(int32_t) * M->bm_nd, hipMemcpyHostToDevice, s));
        M->bm_mask.alloc(static_cast<size_t>(M->bm_bytes) * n_pad);
        SPMVC_HIP(hipMemsetAsync(M->bm_mask.p, 0, M->bm_mask.bytes, s));
        if (vt.K == 2) {
            M->bm_vmask.alloc(static_cast<size_t>(M->bm_bytes) * n_pad);
            SPMVC_HIP(hipMemsetAsync(M->bm_vmask.p, 0, M->bm_vmask.bytes, s));
        }
        DevBuf wmax;
        wmax.alloc(sizeof(int));
        SPMVC_HIP(hipMemsetAsync(wmax.p, 0, sizeof(int), s));
        if (M->bm_bytes == 4)
            k_bm_rows<uint32_t><<<gr, kT, 0, s>>>(ra, M->bm_d.as<int32_t>(), M->bm_nd, M->bm_mask.as<uint32_t>(),
                                                  M->bm_vmask.as<uint32_t>(), nraw_b.as<int32_t>(), wmax.as<int>());
        else
            k_bm_rows<uint64_t><<<gr, kT, 0, s>>>(ra, M->bm_d.as<int32_t>(), M->bm_nd, M->bm_mask.as<uint64_t>(),
                                                  M->bm_vmask.as<uint64_t>(), nraw_b.as<int32_t>(), wmax.as<int>());
        SPMVC_CHECK_LAUNCH();
        M->width = std::max(read_scalar<int>(wmax.p, s), 1);
    } else {
        // steps 2-4: canonical order, T_i, sequence hash
        M->T.alloc(static_cast<size_t>(std::max(vt.K, 1)) * n_pad);
        SPMVC_HIP(hipMemsetAsync(M->T.p, 0, M->T.bytes, s));
        DevBuf hash_b;
        hash_b.alloc(sizeof(uint64_t) * n_pad);
        k_canon<<<gr, kT, 0, s>>>(ra, M->T.as<uint8_t>(), nraw_b.as<int32_t>(), hash_b.as<uint64_t>(), esc);
        SPMVC_CHECK_LAUNCH();
        if (o.fmt == SPMVC_FMT_DIT) {
            // step 5: pattern table
            const int64_t pcap = next_pow2(std::max<int64_t>(2 * n, 1024));
            DevBuf pkeys, pcnt, pmin, pfill, keep, nkeep, rowslot, isrep, slot_id, wbuf;
            pkeys.alloc(sizeof(uint64_t) * pcap);
            pcnt.alloc(sizeof(uint32_t) * pcap);
            pmin.alloc(sizeof(int64_t) * pcap);
            pfill.alloc(sizeof(int));
            rowslot.alloc(sizeof(int64_t) * n);
            keep.alloc(pcap);
            nkeep.alloc(sizeof(int));
            // SPMVC_TEST_WEAK_PATTERN_HASH=1 narrows the first attempt's hash to
            // 4 bits (collisions certain), to exercise the retry with a new seed
            const char *weak = std::getenv("SPMVC_TEST_WEAK_PATTERN_HASH");
            const bool weak_first = weak && weak[0] == '1';
            constexpr int kHashAttempts = 4;
            for (int attempt = 0;; ++attempt) {  // (loop body not indented)
            if (attempt > 0 || weak_first) {  // hash the sequences again
                ra.hash_seed = static_cast<uint64_t>(attempt);
                ra.hash_bits = (attempt == 0 && weak_first) ? 4 : 64;
                k_canon<<<gr, kT, 0, s>>>(ra, M->T.as<uint8_t>(), nraw_b.as<int32_t>(), hash_b.as<uint64_t>(), esc);
                SPMVC_CHECK_LAUNCH();
            }
            k_fill_u64<<<grid_for(pcap, kT, 0x7fffffff), kT, 0, s>>>(pkeys.as<uint64_t>(), kEmpty, pcap);
            k_fill_i64<<<grid_for(pcap, kT, 0x7fffffff), kT, 0, s>>>(pmin.as<int64_t>(), INT64_MAX, pcap);
            SPMVC_HIP(hipMemsetAsync(pcnt.p, 0, pcnt.bytes, s));
            SPMVC_HIP(hipMemsetAsync(pfill.p, 0, sizeof(int), s));
            SPMVC_HIP(hipMemsetAsync(flags, 0, sizeof(int), s));
            GTable pt{pkeys.as<uint64_t>(), pcnt.as<uint32_t>(), pmin.as<int64_t>(),
                      static_cast<uint64_t>(pcap - 1), pfill.as<int>(), static_cast<int>(pcap - 1), flags};
            k_aggregate<<<grid_for(n, kAggChunk, 2048), kAggThreads, 0, s>>>(hash_b.as<uint64_t>(), n, pt,
                                                                            1, 0, nullptr);
            SPMVC_CHECK_LAUNCH();
            k_pattern_lookup<<<gr, kT, 0, s>>>(ra, pt, hash_b.as<uint64_t>(), esc, rowslot.as<int64_t>());
            SPMVC_CHECK_LAUNCH();
            SPMVC_HIP(hipMemsetAsync(nkeep.p, 0, sizeof(int), s));
            k_mark_keep<<<grid_for(pcap, kT, 0x7fffffff), kT, 0, s>>>(pt, pcap, std::max(o.min_pattern_rows, 1),
                                                                    keep.as<uint8_t>(), nkeep.as<int>());
            SPMVC_CHECK_LAUNCH();
            const int f = read_scalar<int>(flags, s);
            if (f & kFlagOverflow) throw Error{SPMVC_EUNSUPPORTED, "pattern hash table overflow"};
            if (!(f & kFlagCollision)) break;
            if (attempt + 1 == kHashAttempts)
                throw Error{SPMVC_EUNSUPPORTED, "pattern-hash collisions between different displacement sequences "
                                                "with every hash seed tried"};
            }
            int n_keep = read_scalar<int>(nkeep.p, s);
            if (n_keep > o.p_max) {
                // rank the qualifying patterns by (count desc, first row asc), keep p_max
                DevBuf list, ln;
                list.alloc(sizeof(int64_t) * n_keep);
                ln.alloc(sizeof(int));
                SPMVC_HIP(hipMemsetAsync(ln.p, 0, sizeof(int), s));
                k_list_keep<<<grid_for(pcap, kT, 0x7fffffff), kT, 0, s>>>(keep.as<uint8_t>(), pcap,
                                                                        list.as<int64_t>(), ln.as<int>());
                SPMVC_CHECK_LAUNCH();
                std::vector<int64_t> slots(n_keep);
                std::vector<uint32_t> hc(pcap);
                std::vector<int64_t> hm(pcap);
                SPMVC_HIP(hipMemcpyAsync(slots.data(), list.p, sizeof(int64_t) * n_keep, hipMemcpyDeviceToHost, s));
                SPMVC_HIP(hipMemcpyAsync(hc.data(), pcnt.p, sizeof(uint32_t) * pcap, hipMemcpyDeviceToHost, s));
                SPMVC_HIP(hipMemcpyAsync(hm.data(), pmin.p, sizeof(int64_t) * pcap, hipMemcpyDeviceToHost, s));
                SPMVC_HIP(hipStreamSynchronize(s));
                std::sort(slots.begin(), slots.end(), [&](int64_t a, int64_t b) {
                    if (hc[a] != hc[b]) return hc[a] > hc[b];
                    return hm[a] < hm[b];
                });
                slots.resize(o.p_max);
                n_keep = o.p_max;
                SPMVC_HIP(hipMemsetAsync(keep.p, 0, pcap, s));
                SPMVC_HIP(hipMemcpyAsync(list.p, slots.data(), sizeof(int64_t) * n_keep, hipMemcpyHostToDevice, s));
                k_set_keep<<<grid_for(n_keep, kT, 0x7fffffff), kT, 0, s>>>(keep.as<uint8_t>(), list.as<int64_t>(), n_keep);
                SPMVC_CHECK_LAUNCH();
                SPMVC_HIP(hipStreamSynchronize(s));
            }
            isrep.alloc(sizeof(int64_t) * n);
            k_rep_flags<<<gr, kT, 0, s>>>(n, rowslot.as<int64_t>(), pmin.as<int64_t>(), keep.as<uint8_t>(),
                                          isrep.as<int64_t>());
            SPMVC_CHECK_LAUNCH();
            const int64_t P = exclusive_scan(isrep.as<int64_t>(), isrep.as<int64_t>(), n, s);
            M->P = static_cast<int32_t>(P);
            if (M->fold) {
                // never null for DITV (the kernels tell DITV by it), large enough for
                // pattern 0's K bytes even when every row escapes
                M->pat_T.alloc(static_cast<size_t>(std::max<int64_t>(P, 1)) * std::max(vt.K, 1));
                SPMVC_HIP(hipMemsetAsync(M->pat_T.p, 0, M->pat_T.bytes, s));
            }
            M->id_bytes = P <= 255 ? 1 : (P <= 65535 ? 2 : 4);
            slot_id.alloc(sizeof(int64_t) * pcap);
            wbuf.alloc(sizeof(int));
            SPMVC_HIP(hipMemsetAsync(wbuf.p, 0, sizeof(int), s));
            k_slot_ids<<<gr, kT, 0, s>>>(rowslot.as<int64_t>(), pmin.as<int64_t>(), keep.as<uint8_t>(),
                                         isrep.as<int64_t>(), n, slot_id.as<int64_t>(), rp, wbuf.as<int>());
            SPMVC_CHECK_LAUNCH();
            M->ids.alloc(static_cast<size_t>(M->id_bytes) * n_pad);
            const unsigned grp = grid_for(n_pad, kT, 0x7fffffff);
            if (M->id_bytes == 1)
                k_write_ids<uint8_t><<<grp, kT, 0, s>>>(rowslot.as<int64_t>(), keep.as<uint8_t>(), slot_id.as<int64_t>(),
                                                        n, n_pad, M->ids.as<uint8_t>(), esc);
            else if (M->id_bytes == 2)
                k_write_ids<uint16_t><<<grp, kT, 0, s>>>(rowslot.as<int64_t>(), keep.as<uint8_t>(), slot_id.as<int64_t>(),
                                                         n, n_pad, M->ids.as<uint16_t>(), esc);
            else
                k_write_ids<uint32_t><<<grp, kT, 0, s>>>(rowslot.as<int64_t>(), keep.as<uint8_t>(), slot_id.as<int64_t>(),
                                                         n, n_pad, M->ids.as<uint32_t>(), esc);
            SPMVC_CHECK_LAUNCH();
            M->width = read_scalar<int>(wbuf.p, s);
            if (P > 0) {
                const int w = std::max(M->width, 1);
                M->pat_off.alloc(sizeof(int32_t) * static_cast<size_t>(P) * w);
                M->pat_len.alloc(static_cast<size_t>(P));
                SPMVC_HIP(hipMemsetAsync(M->pat_off.p, 0, M->pat_off.bytes, s));
                k_write_patterns<<<gr, kT, 0, s>>>(ra, rowslot.as<int64_t>(), pmin.as<int64_t>(), keep.as<uint8_t>(),
                                                   slot_id.as<int64_t>(), w, M->pat_off.as<int32_t>(),
                                                   M->pat_len.as<uint8_t>(), M->T.as<uint8_t>(),
                                                   vt.K > 0 ? M->pat_T.as<uint8_t>() : nullptr);
                SPMVC_CHECK_LAUNCH();
                if (M->fold && vt.K > 0) {
                    M->h_pat_T.resize(static_cast<size_t>(P) * vt.K);
                    SPMVC_HIP(hipMemcpyAsync(M->h_pat_T.data(), M->pat_T.p, M->h_pat_T.size(), hipMemcpyDeviceToHost, s));
                }
                M->h_pat_off.resize(static_cast<size_t>(P) * w);
                M->h_pat_len.resize(static_cast<size_t>(P));
                SPMVC_HIP(hipMemcpyAsync(M->h_pat_off.data(), M->pat_off.p, M->pat_off.bytes, hipMemcpyDeviceToHost, s));
                SPMVC_HIP(hipMemcpyAsync(M->h_pat_len.data(), M->pat_len.p, M->pat_len.bytes, hipMemcpyDeviceToHost, s));
                SPMVC_HIP(hipStreamSynchronize(s));
            }
        }
    }

    // escape rows: zero their T; width of ELL/DT = longest non-escape row
    DevBuf wb;
    wb.alloc(sizeof(int));
    SPMVC_HIP(hipMemsetAsync(wb.p, 0, sizeof(int), s));
    k_fix_escape_T<<<gr, kT, 0, s>>>(n, n_pad, vt.K, esc, M->T.as<uint8_t>(), nraw_b.as<int32_t>(), rp,
                                     (o.fmt == SPMVC_FMT_DIT || o.fmt == SPMVC_FMT_BMASK) ? nullptr : wb.as<int>());
    SPMVC_CHECK_LAUNCH();
    if (o.fmt != SPMVC_FMT_DIT && o.fmt != SPMVC_FMT_BMASK) M->width = std::max(read_scalar<int>(wb.p, s), 1);

    {
        DevBuf eflag, elen;
        eflag.alloc(sizeof(int64_t) * n);
        elen.alloc(sizeof(int64_t) * n);
        k_escape_flags<<<gr, kT, 0, s>>>(n, rp, esc, eflag.as<int64_t>(), elen.as<int64_t>());
        SPMVC_CHECK_LAUNCH();
        M->n_esc = exclusive_scan(eflag.as<int64_t>(), eflag.as<int64_t>(), n, s);
        M->n_esc_nnz = exclusive_scan(elen.as<int64_t>(), elen.as<int64_t>(), n, s);
        M->esc_ptr.alloc(sizeof(int64_t) * (M->n_esc + 1));
        if (M->n_esc > 0) {
            M->esc_rows.alloc(sizeof(int64_t) * M->n_esc);
            M->esc_col.alloc(sizeof(int32_t) * std::max<int64_t>(M->n_esc_nnz, 1));
            M->esc_val.alloc(sizeof(double) * std::max<int64_t>(M->n_esc_nnz, 1));
            if (M->f32_shadow) M->esc_val32.alloc(sizeof(float) * std::max<int64_t>(M->n_esc_nnz, 1));
        }
        k_escape_fill<<<gr, kT, 0, s>>>(ra, esc, eflag.as<int64_t>(), elen.as<int64_t>(), M->n_esc, M->n_esc_nnz,
                                        M->esc_rows.as<int64_t>(), M->esc_ptr.as<int64_t>(), M->esc_col.as<int32_t>(),
                                        M->esc_val.as<double>(), M->esc_val32.as<float>());
        SPMVC_CHECK_LAUNCH();
    }

    if (o.fmt != SPMVC_FMT_ELL) {
        // raw values, sliced by 64 rows
        const int64_t n_slices = n_pad / kSlice;
        M->raw_slice.alloc(sizeof(int64_t) * (n_slices + 1));
        DevBuf mr, nr;
        mr.alloc(sizeof(int));
        nr.alloc(sizeof(unsigned long long));
        SPMVC_HIP(hipMemsetAsync(mr.p, 0, sizeof(int), s));
        SPMVC_HIP(hipMemsetAsync(nr.p, 0, sizeof(unsigned long long), s));
        k_slice_widths<<<grid_for(n_slices, kT, 0x7fffffff), kT, 0, s>>>(n, n_slices, nraw_b.as<int32_t>(),
                                                                        M->raw_slice.as<int64_t>(), mr.as<int>(),
                                                                        nr.as<unsigned long long>());
        SPMVC_CHECK_LAUNCH();
        M->raw_elems = exclusive_scan(M->raw_slice.as<int64_t>(), M->raw_slice.as<int64_t>(), n_slices, s);
        SPMVC_HIP(hipMemcpyAsync(M->raw_slice.as<int64_t>() + n_slices, &M->raw_elems, sizeof(int64_t),
                                 hipMemcpyHostToDevice, s));
        M->max_raw = read_scalar<int>(mr.p, s);
        M->n_raw = static_cast<int64_t>(read_scalar<unsigned long long>(nr.p, s));
        if (M->raw_elems > 0) {
            M->raw.alloc(sizeof(double) * M->raw_elems);
            SPMVC_HIP(hipMemsetAsync(M->raw.p, 0, M->raw.bytes, s));
            if (M->f32_shadow) {
                M->raw32.alloc(sizeof(float) * M->raw_elems);
                SPMVC_HIP(hipMemsetAsync(M->raw32.p, 0, M->raw32.bytes, s));
            }
            k_raw_fill<<<gr, kT, 0, s>>>(ra, esc, nraw_b.as<int32_t>(), M->raw_slice.as<int64_t>(),
                                         M->raw.as<double>(), M->raw32.as<float>());
            SPMVC_CHECK_LAUNCH();
        }
    }
    if (o.fmt == SPMVC_FMT_DT) {
        M->dt_S.alloc(sizeof(int32_t) * static_cast<size_t>(M->width) * n_pad);
        SPMVC_HIP(hipMemsetAsync(M->dt_S.p, 0xFF, M->dt_S.bytes, s));
        k_dt_fill<<<gr, kT, 0, s>>>(ra, esc, M->width, M->dt_S.as<int32_t>());
        SPMVC_CHECK_LAUNCH();
    }
    if (o.fmt == SPMVC_FMT_ELL) {
        M->ell_col.alloc(sizeof(int32_t) * static_cast<size_t>(M->width) * n_pad);
        M->ell_val.alloc(sizeof(double) * static_cast<size_t>(M->width) * n_pad);
        SPMVC_HIP(hipMemsetAsync(M->ell_col.p, 0xFF, M->ell_col.bytes, s));
        SPMVC_HIP(hipMemsetAsync(M->ell_val.p, 0, M->ell_val.bytes, s));
        k_ell_fill<<<gr, kT, 0, s>>>(ra, esc, M->width, M->ell_col.as<int32_t>(), M->ell_val.as<double>());
        SPMVC_CHECK_LAUNCH();
    }
    SPMVC_HIP(hipStreamSynchronize(s));
    if (M->fold) M->T.release();  // DITV rows keep no T: every kernel reads the pattern's
}

void decompress(const spmvc_matrix_s *M, int64_t *rp, int32_t *col, double *val, hipStream_t s) {
    const int64_t n = M->n_rows;
    if (n == 0) {
        SPMVC_HIP(hipMemsetAsync(rp, 0, sizeof(int64_t), s));
        SPMVC_HIP(hipStreamSynchronize(s));
        return;
    }
    DevBuf esc_of_row;
    esc_of_row.alloc(sizeof(int64_t) * n);
    k_fill_i64<<<grid_for(n, kT, 0x7fffffff), kT, 0, s>>>(esc_of_row.as<int64_t>(), -1, n);
    if (M->n_esc > 0)
        k_esc_of_row<<<grid_for(M->n_esc, kT, 0x7fffffff), kT, 0, s>>>(M->n_esc, M->esc_rows.as<int64_t>(),
                                                                      esc_of_row.as<int64_t>());
    SPMVC_CHECK_LAUNCH();
    DecArgs a{};
    a.n_rows = n;
    a.n_pad = M->n_pad;
    a.fmt = M->fmt;
    a.K = M->K;
    a.width = M->width;
    a.id_bytes = M->id_bytes;
    a.V = M->V_dev.as<double>();
    a.T = M->T.as<uint8_t>();
    a.pat_T = M->fold ? M->pat_T.as<uint8_t>() : nullptr;
    a.ids = M->ids.p;
    a.pat_off = M->pat_off.as<int32_t>();
    a.pat_len = M->pat_len.as<uint8_t>();
    a.S = M->dt_S.as<int32_t>();
    a.ell_col = M->ell_col.as<int32_t>();
    a.ell_val = M->ell_val.as<double>();
    a.raw = M->raw.as<double>();
    a.raw_slice = M->raw_slice.as<int64_t>();
    a.esc_rows = M->esc_rows.as<int64_t>();
    a.esc_ptr = M->esc_ptr.as<int64_t>();
    a.esc_col = M->esc_col.as<int32_t>();
    a.esc_val = M->esc_val.as<double>();
    a.esc_of_row = esc_of_row.as<int64_t>();
    a.bm_d = M->bm_d.as<int32_t>();
    a.bm_mask = M->bm_mask.p;
    a.bm_vmask = M->bm_vmask.p;
    a.bm_bytes = M->bm_bytes;
    DevBuf lens;
    lens.alloc(sizeof(int64_t) * (n + 1));
    k_dec_len<<<grid_for(n, kT, 0x7fffffff), kT, 0, s>>>(a, lens.as<int64_t>());
    SPMVC_CHECK_LAUNCH();
    const int64_t total = exclusive_scan(lens.as<int64_t>(), lens.as<int64_t>(), n, s);
    if (total != M->nnz) throw Error{SPMVC_EHIP, "decompressed entry count differs from nnz"};
    SPMVC_HIP(hipMemcpyAsync(lens.as<int64_t>() + n, &total, sizeof(int64_t), hipMemcpyHostToDevice, s));
    SPMVC_HIP(hipMemcpyAsync(rp, lens.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice, s));
    k_dec_fill<<<grid_for(n, kT, 0x7fffffff), kT, 0, s>>>(a, lens.as<int64_t>(), col, val);
    SPMVC_CHECK_LAUNCH();
    SPMVC_HIP(hipStreamSynchronize(s));
}

}  // namespace spmvc
