// Batched conjugate gradients: many independent systems, each with several
// right-hand sides, advanced together.
//
// Every launch covers all systems: the row tiles of all systems form one grid
// (tile -> system through a table), so a batch of uneven systems costs the
// same number of launches as one system.  Each (system, rhs) pair runs its own
// textbook CG (the CG part of Table I) with its own scalars and stops at its
// own tolerance; a finished pair is frozen and a system whose pairs are all
// finished drops out of the tile loops.
//
// One iteration is five launches:
//   bspmv      Q = A_s P for the active systems and per-tile partials of p.q
//              for every rhs: for 2, 4 or 8 right-hand sides whole rows of each
//              x window in turn are staged in LDS (k_bspmv_win); otherwise a
//              group of lanes per row gathers through the caches, one lane per
//              right-hand side (or pair) of the row-interleaved block (k_bspmv);
//   fin_alpha  one block per system: sigma = sum of its tiles' partials (fixed
//              order), alpha = rho / sigma, breakdown test;
//   update     R -= alpha Q for the pairs taking a step; partials of r.r;
//   fin_beta   one block per system: rho', convergence, beta, pair/system flags;
//   pupdate    X += alpha P for the pairs that took the step (P is read once),
//              and P = R + beta P for those still running.
// All reductions are fixed-order, so results repeat exactly.  Iterations are
// recorded once into a hipGraph and the graph is replayed; the host reads one
// counter (active pairs) per replay.  No memset is recorded in the graph.
#include <algorithm>
#include <cmath>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <vector>

#include "check.h"
#include "internal.h"
#include "lds_window.h"
#include "reduce.h"

namespace spmvc {
namespace {

constexpr int kT = 256;     // threads per block = rows per tile
constexpr int kMaxRestarts = 4;  // restarts from the true residual per solve (see k_brestart_fin)

struct SysDesc {
    int64_t row0, n;   // first global row, rows
    int64_t n_pad;
    int64_t tile0;     // first tile
    int32_t ntiles, K, width, id_bytes, P;
    const void *ids;
    const uint8_t *T;
    const uint8_t *pat_T;  // DITV: T of each pattern [P][K] (no per-row T), else null
    const int32_t *pat_off;
    const uint8_t *pat_len;
    const int64_t *esc_rows, *esc_ptr;
    const int32_t *esc_col;
    const double *esc_val;
    int64_t n_esc;
    double V[2];
    // window-phased SpMV: the system's x windows for 256-row tiles and its
    // per-(pattern, window) entry lists (see the FP64 plan of the handle)
    int32_t bw_nw, bw_split;  // bw_split: records split into value runs
    int64_t bw_lo[kMaxWindows];
    int32_t bw_len[kMaxWindows];
    const uint32_t *bw_tab;
};

struct Batch {
    const SysDesc *sys;
    const int32_t *tile_sys;
    int32_t n_sys, nrhs, n_tiles;
    int64_t n_total;
    // row-interleaved [n_total][nrhs]
    const double *B;
    double *X, *R, *P, *Q;
    double *part;    // [n_tiles][nrhs]
    // per pair (s*nrhs + r)
    double *rho;     // [2][pairs]
    double *rho0, *alpha, *beta, *relres;
    int32_t *iters, *status, *done;
    int32_t *step;        // the pair took this iteration's step (set with alpha)
    int32_t *sys_active;  // [n_sys]
    int32_t *sys_step;    // [n_sys]: some pair of the system took this iteration's step
    int32_t *n_active;    // [1]: pairs still running
    double rtol;
    int32_t max_iter;
    int32_t max_width;  // longest pattern of any system
    int32_t tab_lds;    // every system's pattern table fits the LDS copy of the SpMV
    int32_t tab_ints;   // largest pattern table (P * width entries)
    int32_t win_x_bytes;  // window-phased SpMV: LDS bytes of the largest window (0: not used)
    int32_t win_tab_bytes; // ... and of the largest entry-list table
    int32_t all_split;     // every system's records are split into value runs (four rhs per lane)
    int32_t n_xcd;      // XCDs the blocks are dispatched over (tile mapping of the SpMV)
    // SpMV configuration (tuned per batch shape): 0 = window-phased (where it
    // applies), 1 = lane groups with two right-hand sides per lane (16-byte
    // gathers, even nrhs), 2 = lane groups with one per lane; tiles per XCD chunk
    int32_t spmv_form;
    int32_t chunk;
};

__device__ __forceinline__ uint32_t load_id(const void *ids, int id_bytes, int64_t row) {
    if (id_bytes == 1) return static_cast<const uint8_t *>(ids)[row];
    if (id_bytes == 2) return static_cast<const uint16_t *>(ids)[row];
    return static_cast<const uint32_t *>(ids)[row];
}

// Lane layout.  A tile is 256 rows of one system, handled by one block of 256
// threads.  Thread t serves right-hand side r = t % LPR (LPR = nrhs rounded up
// to a power of two) of rows t / LPR, t / LPR + 256/LPR, ... -- so the LPR
// lanes of a row read that row's nrhs contiguous values of a row-interleaved
// block (coalesced), the matrix entry is decoded once per lane group, and each
// thread keeps one rhs for the per-rhs partial sums.

// Sum over the threads of the block that share t % LPR; result valid in
// threads r < LPR (r = the rhs).
template <int LPR> __device__ __forceinline__ double rhs_sum(double v) {
    __shared__ double sh[kT / 64][LPR];
#pragma unroll
    for (int off = LPR; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) < LPR) sh[threadIdx.x >> 6][threadIdx.x & 63] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x < LPR)
#pragma unroll
        for (int w = 0; w < kT / 64; ++w) s += sh[w][threadIdx.x];
    return s;
}


// Sum over a row's pattern entries with value V[0] (k < t0) and with V[1]
// (t0 <= k < len) of x at the entries' columns.  All MAXW pattern offsets are
// read first and all MAXW loads issued before any add, so a row's gathers are
// in flight together; entries past len read the row's own element and add 0.
// VEC consecutive doubles (one lane's right-hand sides), as one load.
template <int VEC> struct VecT;
template <> struct VecT<1> {
    double v[1];
    __device__ __forceinline__ static VecT load(const double *p) { return VecT{{*p}}; }
};
template <> struct VecT<2> {
    double v[2];
    __device__ __forceinline__ static VecT load(const double *p) {
        const double2 t = *reinterpret_cast<const double2 *>(p);
        return VecT{{t.x, t.y}};
    }
};

template <int MAXW, int VEC>
__device__ __forceinline__ void gather_row(const int32_t *__restrict__ pat, int len, int t0, const double *pr,
                                           int64_t lrow, int64_t n, int nr, double (&s0)[VEC], double (&s1)[VEC]) {
    int32_t off[MAXW];
#pragma unroll
    for (int k = 0; k < MAXW; ++k) off[k] = k < len ? pat[k] : 0;
    VecT<VEC> xv[MAXW];
#pragma unroll
    for (int k = 0; k < MAXW; ++k) xv[k] = VecT<VEC>::load(pr + in_bounds<int64_t>(lrow + off[k], n) * nr);
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        s0[v] = 0.0;
        s1[v] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < MAXW; ++k)
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            s0[v] += k < t0 ? xv[k].v[v] : 0.0;
            s1[v] += (k >= t0 && k < len) ? xv[k].v[v] : 0.0;
        }
}

// Q = A_s P for the tile's rows; per-tile partials of p.q for each rhs.
// Rows with at most MAXW entries take the unrolled gather; longer ones a loop.
// Blocks are dispatched round-robin over the XCDs.  Tiles are handed out in
// chunks of `chunk` consecutive tiles (tuned: 8, 32 or 128), chunk k to XCD
// k % n_xcd: the rows a tile gathers from (adjacent lines and planes of its
// grid) mostly lie in its own chunk and hit that XCD's L2, while every
// system's chunks stay spread over all XCDs, so the work stays balanced as
// systems finish.  Tiles past the last whole round of chunks keep their own
// index.

// T_i[c] of a non-escape row of system d: its own T byte, or for DITV its pattern's.
__device__ __forceinline__ int sys_T(const SysDesc &d, int c, int64_t lrow, uint32_t id) {
    return d.pat_T ? d.pat_T[static_cast<int64_t>(id) * d.K + c] : d.T[static_cast<int64_t>(c) * d.n_pad + lrow];
}

__device__ __forceinline__ int chunk_tile(unsigned bid, unsigned nb, int n_xcd, int chunk) {
    const unsigned ch = static_cast<unsigned>(chunk);
    const unsigned round = ch * n_xcd;
    const unsigned full = nb / round * round;
    if (n_xcd <= 1 || bid >= full) return static_cast<int>(bid);
    const unsigned x = bid % n_xcd, j = bid / n_xcd;
    return static_cast<int>(((j / ch) * n_xcd + x) * ch + j % ch);
}

// VEC = 2 when nrhs is even: each lane takes two adjacent right-hand sides
// with 16-byte loads, halving the gather instructions per row.
template <int LPR, int MAXW, int VEC>
__global__ __launch_bounds__(kT) void k_bspmv(Batch b, const double *__restrict__ Pin, double *__restrict__ Qout,
                                              double *part, int with_dot) {
    extern __shared__ int32_t pat_s[];
    const int tile = chunk_tile(blockIdx.x, gridDim.x, b.n_xcd, b.chunk);
    const int s = b.tile_sys[tile];
    if (!b.sys_active[s]) return;  // uniform per block
    const SysDesc &d = b.sys[s];
    const int nr = b.nrhs;
    const int r = (threadIdx.x % LPR) * VEC;  // this lane's first rhs
    const bool lane_on = r < nr;
    const int rc = lane_on ? r : 0;  // idle lanes mirror rhs 0 and store nothing
    const uint32_t esc = d.id_bytes == 1 ? 0xFFu : (d.id_bytes == 2 ? 0xFFFFu : 0xFFFFFFFFu);
    // metadata of all of this thread's rows first: independent loads, in flight together
    const int64_t lbase = static_cast<int64_t>(tile - d.tile0) * kT + threadIdx.x / LPR;
    uint32_t idv[LPR];
    int lenv[LPR], t0v[LPR];
#pragma unroll
    for (int pass = 0; pass < LPR; ++pass) {
        int64_t lrow = lbase + pass * (kT / LPR);
        lrow = lrow < d.n ? lrow : d.n - 1;
        idv[pass] = load_id(d.ids, d.id_bytes, lrow);
        const uint32_t idc = idv[pass] == esc ? 0u : idv[pass];  // escape rows: any valid pattern
        lenv[pass] = d.K > 0 ? sys_T(d, d.K - 1, lrow, idc) : 0;
        t0v[pass] = d.K > 1 ? sys_T(d, 0, lrow, idc) : lenv[pass];
    }
    // the system's pattern table, copied to LDS once per block
    const int32_t *ptab = d.pat_off;
    if (b.tab_lds) {
        const int ne = d.P * d.width;
        for (int e = threadIdx.x; e < ne; e += kT) pat_s[e] = d.pat_off[e];
        __syncthreads();
        ptab = pat_s;
    }
    const double *pr = Pin + d.row0 * nr + rc;
    double dotc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) dotc[v] = 0.0;
#pragma unroll
    for (int pass = 0; pass < LPR; ++pass) {
        const int64_t lrow = lbase + pass * (kT / LPR);
        if (lrow >= d.n) break;
        const int64_t grow = d.row0 + lrow;
        const uint32_t id = idv[pass];
        double acc[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[v] = 0.0;
        if (id != esc) {
            if (d.K > 0) {
                const int32_t *pat = ptab + static_cast<int64_t>(id) * d.width;
                // exclusive run ends: entries [0, t0) take V[0], [t0, len) V[1]
                const int len = lenv[pass], t0 = t0v[pass];
                double s0[VEC], s1[VEC];
                if (len <= MAXW) {
                    gather_row<MAXW, VEC>(pat, len, t0, pr, lrow, d.n, nr, s0, s1);
                } else {
#pragma unroll
                    for (int v = 0; v < VEC; ++v) {
                        s0[v] = 0.0;
                        s1[v] = 0.0;
                    }
                    for (int k = 0; k < len; ++k) {
                        const VecT<VEC> xv = VecT<VEC>::load(pr + in_bounds<int64_t>(lrow + pat[k], d.n) * nr);
#pragma unroll
                        for (int v = 0; v < VEC; ++v) {
                            if (k < t0)
                                s0[v] += xv.v[v];
                            else
                                s1[v] += xv.v[v];
                        }
                    }
                }
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    acc[v] = d.V[0] * s0[v];
                    if (d.K > 1) acc[v] = fma(d.V[1], s1[v], acc[v]);
                }
            }
        } else {
            // escape row: position in the (ascending) escape-row list by bisection
            int64_t lo = 0, hi = d.n_esc;
            while (hi - lo > 1) {
                const int64_t mid = (lo + hi) / 2;
                if (d.esc_rows[mid] <= lrow) lo = mid; else hi = mid;
            }
            for (int64_t e = d.esc_ptr[lo]; e < d.esc_ptr[lo + 1]; ++e) {
                const VecT<VEC> xv = VecT<VEC>::load(pr + in_bounds<int64_t>(d.esc_col[e], d.n) * nr);
#pragma unroll
                for (int v = 0; v < VEC; ++v) acc[v] = fma(d.esc_val[e], xv.v[v], acc[v]);
            }
        }
        if (lane_on) {
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                Qout[grow * nr + r + v] = acc[v];
                if (with_dot) dotc[v] += Pin[grow * nr + r + v] * acc[v];
            }
        }
    }
    if (!with_dot) return;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        const double t = rhs_sum<LPR>(dotc[v]);
        const int rr = static_cast<int>(threadIdx.x) * VEC + v;
        if (threadIdx.x < LPR && rr < nr) part[static_cast<int64_t>(tile) * nr + rr] = t;
    }
}

// Four entries of a row's (pattern, window) record against the x window: four
// 16-byte x reads in flight, then four weighted FMAs (value V[0] for
// canonical index < t0, else V[1]).
template <int NRB>
__device__ __forceinline__ void bwin_group(uint4 e, const unsigned char *xrow, uint32_t lim, int t0, double v0,
                                           double v1, double &a0, double &a1) {
    const uint32_t ent[4] = {e.x, e.y, e.z, e.w};
    double2 xv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        xv[j] = *reinterpret_cast<const double2 *>(xrow + in_bounds<uint32_t>(ent[j] & 0xFFFFu, lim) * NRB);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double wgt = static_cast<int>(ent[j] >> 16) < t0 ? v0 : v1;
        a0 = fma(wgt, xv[j].x, a0);
        a1 = fma(wgt, xv[j].y, a1);
    }
}

// Window-phased form of k_bspmv for nrhs = Q * LPR (2, 4 or 8): the tile's
// rows of one x window at a time -- whole rows of the row-interleaved block,
// a contiguous range -- are copied into LDS, and every row adds the products
// of its entries that fall in that window (per pattern and window a record of
// the count and the entries, read four entries at a time, the last cnt mod 4
// one by one).  LPR lanes per row, each taking Q consecutive right-hand sides:
// Q = 2, or Q = 4 when every system's records are split into value runs (a
// record then serves twice the right-hand sides per read and loop set-up).
// Without split records each product is weighted by its value-table entry as
// it is added.
template <int LPR, int Q = 2>
__global__ __launch_bounds__(kT) void k_bspmv_win(Batch b, const double *__restrict__ Pin,
                                                  double *__restrict__ Qout, double *part, int with_dot) {
    extern __shared__ __align__(16) unsigned char wsm[];
    constexpr int NR = Q * LPR;
    constexpr int PASSES = kT / (kT / LPR);  // = LPR
    const int tile = chunk_tile(blockIdx.x, gridDim.x, b.n_xcd, b.chunk);
    const int s = b.tile_sys[tile];
    if (!b.sys_active[s]) return;  // uniform per block
    const SysDesc &d = b.sys[s];
    double *xs = reinterpret_cast<double *>(wsm);
    const uint4 *tab_s = reinterpret_cast<const uint4 *>(wsm + b.win_x_bytes);
    const int NW = d.bw_nw;
    const int64_t r0 = static_cast<int64_t>(tile - d.tile0) * kT;  // system-local first row
    const uint32_t esc = d.id_bytes == 1 ? 0xFFu : (d.id_bytes == 2 ? 0xFFFFu : 0xFFFFFFFFu);
    const int lr = threadIdx.x / LPR;
    const int rp = (threadIdx.x % LPR) * Q;
    const bool lane_on = rp < b.nrhs;
    uint32_t idv[PASSES];
    int t0v[PASSES];
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps) {
        int64_t lrow = r0 + ps * (kT / LPR) + lr;
        lrow = lrow < d.n ? lrow : d.n - 1;
        idv[ps] = load_id(d.ids, d.id_bytes, lrow);
        t0v[ps] = d.K < 2 ? 255 : sys_T(d, 0, lrow, idv[ps] == esc ? 0u : idv[ps]);
    }
    {
        const int n16 = d.P * NW * (kWinSt / 4);
        const uint4 *src = reinterpret_cast<const uint4 *>(d.bw_tab);
        uint4 *dst = reinterpret_cast<uint4 *>(wsm + b.win_x_bytes);
        for (int e = threadIdx.x; e < n16; e += kT) dst[e] = src[e];
    }
    const double v0 = d.V[0], v1 = d.K >= 2 ? d.V[1] : d.V[0];
    double acc[PASSES][Q];
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps)
#pragma unroll
        for (int q = 0; q < Q; ++q) acc[ps][q] = 0.0;
    const double *sysP = Pin + d.row0 * NR;  // the system's rows
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int w = 0; w < NW; ++w) {
        if (w > 0) __syncthreads();  // every row is done with the previous window
        const int64_t g0 = r0 + d.bw_lo[w];
        const int n = d.bw_len[w];
        if (g0 >= 0 && g0 + n <= d.n) {
            const double *src = sysP + g0 * NR;
            const int nchunk = n * NR / 2;
            for (int c = wave * 64; c < nchunk; c += kT) {
                const int e = c + lane;
                if (e < nchunk) lds_load16(src + 2 * e, xs + 2 * c);
            }
        } else {
            const int64_t last = d.n - 1;
            for (int e = threadIdx.x; e < n * NR; e += kT) {
                int64_t g = g0 + e / NR;
                g = g < 0 ? 0 : (g > last ? last : g);
                xs[e] = sysP[g * NR + e % NR];
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) {
            const int rel = ps * (kT / LPR) + lr;
            if (r0 + rel >= d.n || idv[ps] == esc) continue;
            const uint4 *rec = tab_s + (static_cast<int64_t>(idv[ps]) * NW + w) * (kWinSt / 4);
            const unsigned char *xrow = reinterpret_cast<const unsigned char *>(xs + rel * NR + rp);
            const uint32_t lim = static_cast<uint32_t>(d.bw_len[w] - rel);  // window rows from this row on
            if (Q == 4 || d.bw_split) {  // Q = 4 is launched only with split records
                win_row_split<NR * 8, Q>(reinterpret_cast<const uint32_t *>(rec), xrow, lim, v0, v1, acc[ps]);
                continue;
            }
            if constexpr (Q != 2) continue;
            const int cnt = static_cast<int>(rec[0].x);
            int k0 = 0;
            for (; k0 + 4 <= cnt; k0 += 4)
                bwin_group<NR * 8>(rec[1 + (k0 >> 2)], xrow, lim, t0v[ps], v0, v1, acc[ps][0], acc[ps][1]);
            // the last cnt mod 4 entries one at a time (no padded work)
            const uint32_t *recw = reinterpret_cast<const uint32_t *>(rec) + 4;
            for (; k0 < cnt; ++k0) {
                const uint32_t e = recw[k0];
                const double2 xv =
                    *reinterpret_cast<const double2 *>(xrow + in_bounds<uint32_t>(e & 0xFFFFu, lim) * (NR * 8));
                const double wgt = static_cast<int>(e >> 16) < t0v[ps] ? v0 : v1;
                acc[ps][0] = fma(wgt, xv.x, acc[ps][0]);
                acc[ps][1] = fma(wgt, xv.y, acc[ps][1]);
            }
        }
    }
    double dotc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) dotc[q] = 0.0;
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps) {
        const int64_t lrow = r0 + ps * (kT / LPR) + lr;
        if (lrow >= d.n) continue;
        double qv[Q];
        if (idv[ps] != esc) {
#pragma unroll
            for (int q = 0; q < Q; ++q) qv[q] = acc[ps][q];
        } else {
            // escape row: plain CSR gathers from global memory
            int64_t lo = 0, hi = d.n_esc;
            while (hi - lo > 1) {
                const int64_t mid = (lo + hi) / 2;
                if (d.esc_rows[mid] <= lrow) lo = mid; else hi = mid;
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) qv[q] = 0.0;
            for (int64_t e = d.esc_ptr[lo]; e < d.esc_ptr[lo + 1]; ++e) {
                const double *xe = sysP + in_bounds<int64_t>(d.esc_col[e], d.n) * NR + rp;
#pragma unroll
                for (int h = 0; h < Q / 2; ++h) {
                    const double2 xv = *reinterpret_cast<const double2 *>(xe + 2 * h);
                    qv[2 * h] = fma(d.esc_val[e], xv.x, qv[2 * h]);
                    qv[2 * h + 1] = fma(d.esc_val[e], xv.y, qv[2 * h + 1]);
                }
            }
        }
        if (lane_on) {
            const int64_t gi = (d.row0 + lrow) * NR + rp;
#pragma unroll
            for (int h = 0; h < Q / 2; ++h) {
                *reinterpret_cast<double2 *>(Qout + gi + 2 * h) = double2{qv[2 * h], qv[2 * h + 1]};
                if (with_dot) {
                    const double2 pv = *reinterpret_cast<const double2 *>(Pin + gi + 2 * h);
                    dotc[2 * h] += pv.x * qv[2 * h];
                    dotc[2 * h + 1] += pv.y * qv[2 * h + 1];
                }
            }
        }
    }
    if (!with_dot) return;
#pragma unroll
    for (int v = 0; v < Q; ++v) {
        const double t = rhs_sum<LPR>(dotc[v]);
        const int rr = static_cast<int>(threadIdx.x) * Q + v;
        if (threadIdx.x < LPR && rr < b.nrhs) part[static_cast<int64_t>(tile) * b.nrhs + rr] = t;
    }
}

// Sum of the tiles' partials of system s for rhs r (fixed order), in every thread.
// Sums of the system's tile partials for every right-hand side, in a fixed
// order (out[r], valid in every thread).  A tile's partials of all right-hand
// sides are adjacent, so each step issues all of them at once; one pass over
// the tiles serves every right-hand side.
__device__ __forceinline__ void sys_sums(const Batch &b, const SysDesc &d, double (&out)[16]) {
    double acc[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0;
    for (int t = threadIdx.x; t < d.ntiles; t += kT) {
        const double *p = b.part + (d.tile0 + t) * b.nrhs;
#pragma unroll
        for (int r = 0; r < 16; ++r)
            if (r < b.nrhs) acc[r] += p[r];
    }
#pragma unroll
    for (int r = 0; r < 16; ++r)
        if (r < b.nrhs) out[r] = block_sum<kT>(acc[r]);
}

// Element loop of a tile: f(global element index, rhs) for the tile's rows.
#define SPMVC_TILE_ELEMS(BODY)                                                                      \
    {                                                                                               \
        const int r = threadIdx.x % LPR;                                                            \
        if (r < nr)                                                                                 \
            for (int pass = 0; pass < LPR; ++pass) {                                                \
                const int64_t lrow =                                                                \
                    static_cast<int64_t>(tile - d.tile0) * kT + pass * (kT / LPR) + threadIdx.x / LPR; \
                if (lrow >= d.n) break;                                                             \
                const int64_t g = (d.row0 + lrow) * nr + r;                                         \
                BODY                                                                                \
            }                                                                                       \
    }

// Two-phase form for the update kernels: BODY runs for every row slot of the
// thread (ok: the row exists; g is clamped to a valid element otherwise), so
// a first loop can issue all loads and a second do the stores: the loads are
// then all in flight together (the vectors are not marked non-aliasing, so a
// store would otherwise order every later load behind it).
#define SPMVC_TILE_SLOTS(BODY)                                                                   \
    {                                                                                            \
        const int64_t lb_ = static_cast<int64_t>(tile - d.tile0) * kT + threadIdx.x / LPR;       \
        _Pragma("unroll") for (int pass = 0; pass < LPR; ++pass) {                               \
            const int64_t lrow = lb_ + pass * (kT / LPR);                                        \
            const bool ok = lrow < d.n;                                                          \
            const int64_t g = (d.row0 + (ok ? lrow : 0)) * nr + rr_;                             \
            BODY                                                                                 \
        }                                                                                        \
    }

// X = 0, R = B, P = B; partials of b.b
template <int LPR> __global__ __launch_bounds__(kT) void k_bstart(Batch b) {
    const int tile = blockIdx.x;
    const int s = b.tile_sys[tile];
    const SysDesc &d = b.sys[s];
    const int nr = b.nrhs;
    double acc = 0.0;
    SPMVC_TILE_ELEMS(const double v = b.B[g]; b.X[g] = 0.0; b.R[g] = v; b.P[g] = v; acc += v * v;)
    const double t = rhs_sum<LPR>(acc);
    if (static_cast<int>(threadIdx.x) < nr) b.part[static_cast<int64_t>(tile) * nr + threadIdx.x] = t;
}

__global__ __launch_bounds__(kT) void k_bstart_fin(Batch b) {
    const int s = blockIdx.x;
    const SysDesc &d = b.sys[s];
    int active = 0;
    double sums[16];
    sys_sums(b, d, sums);
    for (int r = 0; r < b.nrhs; ++r) {
        const double rr = sums[r];
        if (threadIdx.x == 0) {
            const int q = s * b.nrhs + r;
            b.rho[q] = rr;
            b.rho[b.n_sys * b.nrhs + q] = 0.0;
            b.rho0[q] = rr;
            b.iters[q] = 0;
            // a right-hand side that is not finite (NaN or inf in b) stops its pair at once
            const bool bad = !(rr == rr) || rr > 1.7e308;
            b.relres[q] = rr > 0.0 ? 1.0 : 0.0;
            b.status[q] = bad ? SPMVC_EINVAL : SPMVC_OK;
            b.done[q] = rr > 0.0 && !bad ? 0 : 1;
            if (rr > 0.0 && !bad) {
                ++active;
                atomicAdd(b.n_active, 1);
            }
        }
    }
    if (threadIdx.x == 0) b.sys_active[s] = active > 0 ? 1 : 0;
}

// alpha per pair (breakdown stops the pair).  rho is double-buffered by the
// parity of the pair's own iteration count, so the kernels take no iteration
// index and one recorded graph serves every replay.
__global__ __launch_bounds__(kT) void k_bfin_alpha(Batch b) {
    const int s = blockIdx.x;
    if (!b.sys_active[s]) {
        if (threadIdx.x == 0) b.sys_step[s] = 0;
        return;
    }
    const SysDesc &d = b.sys[s];
    int any = 0;
    double sums[16];
    sys_sums(b, d, sums);
    for (int r = 0; r < b.nrhs; ++r) {
        const double sigma = sums[r];
        if (threadIdx.x == 0) {
            const int q = s * b.nrhs + r;
            b.step[q] = 0;
            if (b.done[q]) continue;
            if (!(sigma > 0.0) || !isfinite(sigma)) {
                b.done[q] = 1;
                b.status[q] = SPMVC_ENOTSPD;
                b.iters[q] += 1;
                b.alpha[q] = 0.0;
                atomicSub(b.n_active, 1);
            } else {
                b.alpha[q] = b.rho[(b.iters[q] & 1) * b.n_sys * b.nrhs + q] / sigma;
                b.step[q] = 1;
                any = 1;
            }
        }
    }
    if (threadIdx.x == 0) b.sys_step[s] = any;
}

// R -= alpha Q for the pairs taking a step; partials of r.r (X advances in the
// p-update, which reads P anyway)
template <int LPR> __global__ __launch_bounds__(kT) void k_bupdate(Batch b) {
    const int tile = blockIdx.x;
    const int s = b.tile_sys[tile];
    if (!b.sys_step[s]) return;
    const SysDesc &d = b.sys[s];
    const int nr = b.nrhs;
    const int rr_ = threadIdx.x % LPR;
    const int q = s * nr + (rr_ < nr ? rr_ : 0);
    const bool run = rr_ < nr && b.step[q];
    const double a = run ? b.alpha[q] : 0.0;
    double acc = 0.0;
    if (run) {
        double rv[LPR], qv[LPR];
        SPMVC_TILE_SLOTS(rv[pass] = b.R[g]; qv[pass] = b.Q[g];)
        SPMVC_TILE_SLOTS(if (ok) {
            const double t = rv[pass] - a * qv[pass];
            b.R[g] = t;
            acc += t * t;
        })
    }
    const double t = rhs_sum<LPR>(acc);
    if (static_cast<int>(threadIdx.x) < nr) b.part[static_cast<int64_t>(tile) * nr + threadIdx.x] = t;
}

// rho', convergence, beta
__global__ __launch_bounds__(kT) void k_bfin_beta(Batch b) {
    const int s = blockIdx.x;
    if (!b.sys_active[s]) return;
    const SysDesc &d = b.sys[s];
    const int np = b.n_sys * b.nrhs;
    int still = 0;
    double sums[16];
    sys_sums(b, d, sums);
    for (int r = 0; r < b.nrhs; ++r) {
        const double rho_new = sums[r];
        if (threadIdx.x == 0) {
            const int q = s * b.nrhs + r;
            if (b.done[q]) continue;
            const int it = b.iters[q];
            const int par = it & 1;
            const double rho = b.rho[par * np + q];
            b.iters[q] = it + 1;
            b.relres[q] = sqrt(rho_new) / sqrt(b.rho0[q]);
            b.rho[(par ^ 1) * np + q] = rho_new;
            b.beta[q] = rho_new / rho;
            int st = -1;
            if (sqrt(rho_new) <= b.rtol * sqrt(b.rho0[q]))
                st = SPMVC_OK;
            else if (!isfinite(rho_new))
                st = SPMVC_ENOTSPD;
            else if (it + 1 >= b.max_iter)
                st = SPMVC_ENOCONV;
            if (st != -1) {
                b.done[q] = 1;  // finished this step: pupdate skips it
                b.status[q] = st;
                atomicSub(b.n_active, 1);
            } else {
                ++still;
            }
        }
    }
    if (threadIdx.x == 0 && still == 0) {
        bool any = false;
        for (int r = 0; r < b.nrhs; ++r) any |= (b.done[s * b.nrhs + r] == 0);
        if (!any) b.sys_active[s] = 0;
    }
}

// X += alpha P for the pairs that took this iteration's step, then
// P = R + beta P for those still running
template <int LPR> __global__ __launch_bounds__(kT) void k_bpupdate(Batch b) {
    const int tile = blockIdx.x;
    const int s = b.tile_sys[tile];
    if (!b.sys_step[s]) return;
    const SysDesc &d = b.sys[s];
    const int nr = b.nrhs;
    const int rr_ = threadIdx.x % LPR;
    const int q = s * nr + (rr_ < nr ? rr_ : 0);
    if (rr_ >= nr || !b.step[q]) return;
    const double alpha = b.alpha[q];
    double xv[LPR], pv[LPR];
    if (b.done[q]) {
        SPMVC_TILE_SLOTS(xv[pass] = b.X[g]; pv[pass] = b.P[g];)
        SPMVC_TILE_SLOTS(if (ok) b.X[g] = xv[pass] + alpha * pv[pass];)
        return;
    }
    const double beta = b.beta[q];
    double rv[LPR];
    SPMVC_TILE_SLOTS(xv[pass] = b.X[g]; pv[pass] = b.P[g]; rv[pass] = b.R[g];)
    SPMVC_TILE_SLOTS(if (ok) {
        b.X[g] = xv[pass] + alpha * pv[pass];
        b.P[g] = rv[pass] + beta * pv[pass];
    })
}

// partials of (b - Ax).(b - Ax) per rhs, with Ax in Q (all systems)
template <int LPR> __global__ __launch_bounds__(kT) void k_bresid(Batch b) {
    const int tile = blockIdx.x;
    const int s = b.tile_sys[tile];
    const SysDesc &d = b.sys[s];
    const int nr = b.nrhs;
    double acc = 0.0;
    SPMVC_TILE_ELEMS(const double v = b.B[g] - b.Q[g]; acc += v * v;)
    const double t = rhs_sum<LPR>(acc);
    if (static_cast<int>(threadIdx.x) < nr) b.part[static_cast<int64_t>(tile) * nr + threadIdx.x] = t;
}

__global__ __launch_bounds__(kT) void k_bresid_fin(Batch b, double *out) {
    const int s = blockIdx.x;
    const SysDesc &d = b.sys[s];
    double sums[16];
    sys_sums(b, d, sums);
    for (int r = 0; r < b.nrhs; ++r) {
        const double rr = sums[r];
        if (threadIdx.x == 0) out[s * b.nrhs + r] = rr;
    }
}

// After the true residuals (rr, per pair; Q = A X): a pair that stopped with
// SPMVC_OK on its recursive residual while its true one misses the tolerance
// restarts from the true residual -- flagged in `step`, running again with
// rho = rr of its current iteration parity (rho0, the ||b||^2 of the stopping
// test, is kept).  A system runs again when one of its pairs does.
__global__ __launch_bounds__(kT) void k_brestart_fin(Batch b, const double *rr) {
    const int s = blockIdx.x;
    if (threadIdx.x != 0) return;
    const int np = b.n_sys * b.nrhs;
    int any = 0;
    for (int r = 0; r < b.nrhs; ++r) {
        const int q = s * b.nrhs + r;
        const bool again = b.done[q] && b.status[q] == SPMVC_OK && b.iters[q] < b.max_iter &&
                           sqrt(rr[q]) > b.rtol * sqrt(b.rho0[q]);
        b.step[q] = again ? 1 : 0;
        if (again) {
            b.done[q] = 0;
            b.rho[(b.iters[q] & 1) * np + q] = rr[q];
            b.relres[q] = sqrt(rr[q]) / sqrt(b.rho0[q]);
            atomicAdd(b.n_active, 1);
            any = 1;
        }
    }
    b.sys_active[s] = any;
}

// R = B - Q (Q = A X) and P = R for the restarting pairs
template <int LPR> __global__ __launch_bounds__(kT) void k_brestart(Batch b) {
    const int tile = blockIdx.x;
    const int s = b.tile_sys[tile];
    if (!b.sys_active[s]) return;
    const SysDesc &d = b.sys[s];
    const int nr = b.nrhs;
    const int rr_ = threadIdx.x % LPR;
    const int q = s * nr + (rr_ < nr ? rr_ : 0);
    if (rr_ >= nr || !b.step[q]) return;
    SPMVC_TILE_SLOTS(if (ok) {
        const double t = b.B[g] - b.Q[g];
        b.R[g] = t;
        b.P[g] = t;
    })
}

__global__ void k_set_all(int32_t *p, int32_t v, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Launch a tile kernel with LPR = nrhs rounded up to a power of two.
#define SPMVC_LPR_LAUNCH(KERNEL, GRID, STREAM, ...)                                  \
    do {                                                                             \
        if (b.nrhs <= 1)                                                             \
            KERNEL<1><<<GRID, kT, 0, STREAM>>>(__VA_ARGS__);                         \
        else if (b.nrhs <= 2)                                                        \
            KERNEL<2><<<GRID, kT, 0, STREAM>>>(__VA_ARGS__);                         \
        else if (b.nrhs <= 4)                                                        \
            KERNEL<4><<<GRID, kT, 0, STREAM>>>(__VA_ARGS__);                         \
        else if (b.nrhs <= 8)                                                        \
            KERNEL<8><<<GRID, kT, 0, STREAM>>>(__VA_ARGS__);                         \
        else                                                                         \
            KERNEL<16><<<GRID, kT, 0, STREAM>>>(__VA_ARGS__);                        \
    } while (0)

// The same for k_bspmv (width W, VEC right-hand sides per lane, LDS bytes SH);
// LPR = ceil(nrhs / VEC) rounded up to a power of two.
#define SPMVC_BSPMV_LAUNCH(W, VEC, GRID, SH, STREAM, ...)                            \
    do {                                                                             \
        const int lanes_ = (b.nrhs + VEC - 1) / VEC;                                 \
        if (lanes_ <= 1)                                                             \
            k_bspmv<1, W, VEC><<<GRID, kT, SH, STREAM>>>(__VA_ARGS__);               \
        else if (lanes_ <= 2)                                                        \
            k_bspmv<2, W, VEC><<<GRID, kT, SH, STREAM>>>(__VA_ARGS__);               \
        else if (lanes_ <= 4)                                                        \
            k_bspmv<4, W, VEC><<<GRID, kT, SH, STREAM>>>(__VA_ARGS__);               \
        else if (lanes_ <= 8)                                                        \
            k_bspmv<8, W, VEC><<<GRID, kT, SH, STREAM>>>(__VA_ARGS__);               \
        else                                                                         \
            k_bspmv<16, W, VEC><<<GRID, kT, SH, STREAM>>>(__VA_ARGS__);              \
    } while (0)

constexpr int kTabLdsInts = 4096;  // pattern tables up to 16 KB are copied to LDS

void launch_bspmv(const Batch &b, const double *Pin, double *Qout, int with_dot, hipStream_t s) {
    const unsigned g = static_cast<unsigned>(b.n_tiles);
    if (b.spmv_form == 0 && b.win_x_bytes > 0) {
        const size_t wsh = static_cast<size_t>(b.win_x_bytes) + static_cast<size_t>(b.win_tab_bytes);
        // four right-hand sides per lane when every system's records are split
        if (b.nrhs == 2)
            k_bspmv_win<1><<<g, kT, wsh, s>>>(b, Pin, Qout, b.part, with_dot);
        else if (b.nrhs == 4 && b.all_split)
            k_bspmv_win<1, 4><<<g, kT, wsh, s>>>(b, Pin, Qout, b.part, with_dot);
        else if (b.nrhs == 4)
            k_bspmv_win<2><<<g, kT, wsh, s>>>(b, Pin, Qout, b.part, with_dot);
        else if (b.all_split)
            k_bspmv_win<2, 4><<<g, kT, wsh, s>>>(b, Pin, Qout, b.part, with_dot);
        else
            k_bspmv_win<4><<<g, kT, wsh, s>>>(b, Pin, Qout, b.part, with_dot);
        return;
    }
    const size_t sh = b.tab_lds ? sizeof(int32_t) * static_cast<size_t>(b.tab_ints) : 0;
    // two right-hand sides per lane when every row's block starts 16-byte aligned
    const bool pairs = b.nrhs % 2 == 0 && b.spmv_form != 2;
    if (b.max_width <= 28) {
        if (pairs)
            SPMVC_BSPMV_LAUNCH(28, 2, g, sh, s, b, Pin, Qout, b.part, with_dot);
        else
            SPMVC_BSPMV_LAUNCH(28, 1, g, sh, s, b, Pin, Qout, b.part, with_dot);
    } else {
        if (pairs)
            SPMVC_BSPMV_LAUNCH(32, 2, g, sh, s, b, Pin, Qout, b.part, with_dot);
        else
            SPMVC_BSPMV_LAUNCH(32, 1, g, sh, s, b, Pin, Qout, b.part, with_dot);
    }
}

// Tuned SpMV configurations, per batch shape (systems, rows, tiles, nrhs,
// longest pattern, first and last system's rows); the last one chosen.
struct BatchTune {
    int32_t form, chunk;
    double us;
};
std::mutex g_tune_mu;
std::map<std::vector<int64_t>, BatchTune> g_tune_cache;
BatchTune g_last_tune{-1, 0, 0.0};

// Times each candidate SpMV configuration on the batch (P already holds the
// right-hand sides; Q is scratch; no partials written) and keeps the fastest:
// forms {window-phased, lane-group pairs, lane-group singles} that apply x
// chunks {8, 32, 128}.  The choice is cached per batch shape, so repeated
// solves of one batch take the same summation order.
BatchTune tune_bspmv(Batch &b, const std::vector<int64_t> &key, hipStream_t s) {
    // SPMVC_BATCHED_SPMV="form,chunk" fixes the configuration (tests, experiments)
    if (const char *env = std::getenv("SPMVC_BATCHED_SPMV")) {
        int f = -1, ch = 0;
        if (std::sscanf(env, "%d,%d", &f, &ch) == 2 && f >= 0 && f <= 2 && ch >= 1 && ch <= 4096) {
            if (f == 0 && b.win_x_bytes == 0) f = b.nrhs % 2 == 0 ? 1 : 2;
            if (f == 1 && b.nrhs % 2 != 0) f = 2;
            return {f, ch, 0.0};
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) return it->second;
    }
    std::vector<int> forms;
    if (b.win_x_bytes > 0) forms.push_back(0);
    if (b.nrhs % 2 == 0) forms.push_back(1);
    forms.push_back(2);
    hipEvent_t e0, e1;
    SPMVC_HIP(hipEventCreate(&e0));
    SPMVC_HIP(hipEventCreate(&e1));
    BatchTune best{forms[0], 32, 1e300};
    for (int f : forms)
        for (int ch : {8, 32, 128}) {
            b.spmv_form = f;
            b.chunk = ch;
            launch_bspmv(b, b.P, b.Q, 0, s);  // warm
            SPMVC_HIP(hipEventRecord(e0, s));
            constexpr int kReps = 3;
            for (int r = 0; r < kReps; ++r) launch_bspmv(b, b.P, b.Q, 0, s);
            SPMVC_HIP(hipEventRecord(e1, s));
            SPMVC_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            SPMVC_HIP(hipEventElapsedTime(&ms, e0, e1));
            const double us = 1000.0 * ms / kReps;
            if (us < best.us) best = {f, ch, us};
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
    return best;
}

void record_iteration(const Batch &b, hipStream_t s) {
    const unsigned g = static_cast<unsigned>(b.n_tiles), ns = static_cast<unsigned>(b.n_sys);
    launch_bspmv(b, b.P, b.Q, 1, s);
    k_bfin_alpha<<<ns, kT, 0, s>>>(b);
    SPMVC_LPR_LAUNCH(k_bupdate, g, s, b);
    k_bfin_beta<<<ns, kT, 0, s>>>(b);
    SPMVC_LPR_LAUNCH(k_bpupdate, g, s, b);
}

}  // namespace

// The SpMV configuration the last batched solve used (form, chunk, microseconds per launch).
void batched_last_tune(int32_t *form, int32_t *chunk, double *us) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    *form = g_last_tune.form;
    *chunk = g_last_tune.chunk;
    *us = g_last_tune.us;
}

// A solve that asked for batched kernels took the one-after-another path
// instead (form -2 in spmvc_batched_config).
void batched_note_fallback() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_last_tune = BatchTune{-2, 0, 0.0};
}

// Is the batched solver able to take these matrices (DIT, value table <= 2, no raw values)?
bool batched_supported(const spmvc_matrix *A, int n_sys) {
    for (int s = 0; s < n_sys; ++s) {
        const spmvc_matrix_s *M = A[s];
        if (M->fmt != SPMVC_FMT_DIT || M->K > 2 || M->raw_elems > 0 || M->n_rows != M->n_cols) return false;
    }
    return true;
}

spmvc_status cg_solve_batched(const spmvc_matrix *A, int n_sys, int nrhs, const double *const *bvec,
                              double *const *xvec, const spmvc_cg_opts &o, spmvc_cg_stat *stat, hipStream_t st,
                              bool use_graph) {
    // layout: all systems stacked, row-interleaved [n_total][nrhs]
    std::vector<SysDesc> sd(n_sys);
    std::vector<int32_t> tile_sys;
    int64_t row0 = 0, tile0 = 0;
    for (int s = 0; s < n_sys; ++s) {
        const spmvc_matrix_s *M = A[s];
        SysDesc &d = sd[s];
        d.row0 = row0;
        d.n = M->n_rows;
        d.n_pad = M->n_pad;
        d.tile0 = tile0;
        d.ntiles = static_cast<int32_t>((M->n_rows + kT - 1) / kT);
        d.K = M->K;
        d.width = M->width;
        d.P = M->P;
        d.id_bytes = M->id_bytes;
        d.ids = M->ids.p;
        d.T = M->T.as<uint8_t>();
        d.pat_T = M->fold ? M->pat_T.as<uint8_t>() : nullptr;
        d.pat_off = M->pat_off.as<int32_t>();
        d.pat_len = M->pat_len.as<uint8_t>();
        d.esc_rows = M->esc_rows.as<int64_t>();
        d.esc_ptr = M->esc_ptr.as<int64_t>();
        d.esc_col = M->esc_col.as<int32_t>();
        d.esc_val = M->esc_val.as<double>();
        d.n_esc = M->n_esc;
        d.V[0] = M->V[0];
        d.V[1] = M->V[1];
        const LdsPlan &pl = M->plan[SPMVC_F64];
        d.bw_nw = pl.bw ? pl.bw_nw : 0;
        d.bw_split = pl.bw && pl.bw_split ? 1 : 0;
        for (int w = 0; w < kMaxWindows; ++w) {
            d.bw_lo[w] = pl.bw_lo[w];
            d.bw_len[w] = pl.bw_len[w];
        }
        d.bw_tab = pl.bw ? pl.bw_tab.as<uint32_t>() : nullptr;
        for (int t = 0; t < d.ntiles; ++t) tile_sys.push_back(s);
        row0 += M->n_rows;
        tile0 += d.ntiles;
    }
    const int64_t n_total = row0;
    const int n_tiles = static_cast<int>(tile0);
    const int np = n_sys * nrhs;
    if (n_total == 0) {  // every system empty: nothing to solve
        for (int q = 0; q < np; ++q) stat[q] = spmvc_cg_stat{0, 0, SPMVC_OK, 0, 0.0, 0.0};
        return SPMVC_OK;
    }
    DevBuf dsys, dtile, B, X, R, P, Q, part, rho, rho0, alpha, beta, relres, iters, status, done, step, sact, sstep,
        nact, rr;
    dsys.alloc(sizeof(SysDesc) * n_sys);
    dtile.alloc(sizeof(int32_t) * std::max(n_tiles, 1));
    const size_t vb = sizeof(double) * static_cast<size_t>(std::max<int64_t>(n_total, 1)) * nrhs;
    B.alloc(vb);
    X.alloc(vb);
    R.alloc(vb);
    P.alloc(vb);
    Q.alloc(vb);
    part.alloc(sizeof(double) * static_cast<size_t>(std::max(n_tiles, 1)) * nrhs);
    rho.alloc(sizeof(double) * 2 * np);
    rho0.alloc(sizeof(double) * np);
    alpha.alloc(sizeof(double) * np);
    beta.alloc(sizeof(double) * np);
    relres.alloc(sizeof(double) * np);
    rr.alloc(sizeof(double) * np * 2);
    iters.alloc(sizeof(int32_t) * np);
    status.alloc(sizeof(int32_t) * np);
    done.alloc(sizeof(int32_t) * np);
    sact.alloc(sizeof(int32_t) * n_sys);
    step.alloc(sizeof(int32_t) * np);
    sstep.alloc(sizeof(int32_t) * n_sys);
    nact.alloc(sizeof(int32_t));
    SPMVC_HIP(hipMemcpyAsync(dsys.p, sd.data(), dsys.bytes, hipMemcpyHostToDevice, st));
    SPMVC_HIP(hipMemcpyAsync(dtile.p, tile_sys.data(), sizeof(int32_t) * n_tiles, hipMemcpyHostToDevice, st));
    for (int s = 0; s < n_sys; ++s)
        SPMVC_HIP(hipMemcpyAsync(B.as<double>() + sd[s].row0 * nrhs, bvec[s], sizeof(double) * sd[s].n * nrhs,
                                 hipMemcpyDeviceToDevice, st));
    SPMVC_HIP(hipMemsetAsync(nact.p, 0, sizeof(int32_t), st));

    Batch b{};
    b.sys = dsys.as<SysDesc>();
    b.tile_sys = dtile.as<int32_t>();
    b.n_sys = n_sys;
    b.nrhs = nrhs;
    b.n_tiles = n_tiles;
    b.n_total = n_total;
    b.n_xcd = n_sys > 0 ? A[0]->n_xcd : 1;
    b.max_width = 0;
    b.tab_ints = 0;
    for (int q = 0; q < n_sys; ++q) {
        b.max_width = std::max(b.max_width, sd[q].width);
        b.tab_ints = std::max(b.tab_ints, sd[q].P * sd[q].width);
    }
    b.tab_lds = b.tab_ints > 0 && b.tab_ints <= kTabLdsInts;
    // window-phased SpMV when every system has its window plan (or no pattern
    // at all: then every row is an escape row, taken from global memory), nrhs
    // is 2, 4 or 8 and the largest window and table fit the LDS budget
    b.win_x_bytes = 0;
    b.win_tab_bytes = 0;
    b.all_split = 1;
    bool win_ok = nrhs == 2 || nrhs == 4 || nrhs == 8;
    for (int q = 0; q < n_sys && win_ok; ++q) {
        const LdsPlan &pl = A[q]->plan[SPMVC_F64];
        if (!pl.bw && A[q]->P == 0) continue;
        if (!pl.bw) {
            win_ok = false;
            break;
        }
        if (!pl.bw_split) b.all_split = 0;
        b.win_x_bytes = std::max<int32_t>(b.win_x_bytes, pl.bw_maxlen * nrhs * 8);
        b.win_tab_bytes = std::max<int32_t>(b.win_tab_bytes, A[q]->P * pl.bw_nw * kWinSt * 4);
    }
    if (!win_ok || b.win_x_bytes + b.win_tab_bytes > kLdsBudgetBytes) b.win_x_bytes = 0;
    b.B = B.as<double>();
    b.X = X.as<double>();
    b.R = R.as<double>();
    b.P = P.as<double>();
    b.Q = Q.as<double>();
    b.part = part.as<double>();
    b.rho = rho.as<double>();
    b.rho0 = rho0.as<double>();
    b.alpha = alpha.as<double>();
    b.beta = beta.as<double>();
    b.relres = relres.as<double>();
    b.iters = iters.as<int32_t>();
    b.status = status.as<int32_t>();
    b.done = done.as<int32_t>();
    b.sys_active = sact.as<int32_t>();
    b.step = step.as<int32_t>();
    b.sys_step = sstep.as<int32_t>();
    b.n_active = nact.as<int32_t>();
    b.rtol = o.rtol;
    b.max_iter = o.max_iter;

    b.spmv_form = b.win_x_bytes > 0 ? 0 : (nrhs % 2 == 0 ? 1 : 2);
    b.chunk = 32;
    SPMVC_LPR_LAUNCH(k_bstart, static_cast<unsigned>(n_tiles), st, b);
    k_bstart_fin<<<static_cast<unsigned>(n_sys), kT, 0, st>>>(b);
    SPMVC_CHECK_LAUNCH();
    {
        // the SpMV configuration for this batch shape (P = the right-hand sides now)
        const std::vector<int64_t> key{n_sys, n_total, n_tiles, nrhs, b.max_width, sd.front().n, sd.back().n,
                                       b.win_x_bytes};
        const BatchTune t = tune_bspmv(b, key, st);
        b.spmv_form = t.form;
        b.chunk = t.chunk;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_last_tune = t;
    }

    int32_t *h_active = nullptr;
    SPMVC_HIP(hipHostMalloc(reinterpret_cast<void **>(&h_active), sizeof(int32_t), hipHostMallocDefault));
    struct HostFree {
        int32_t *p;
        ~HostFree() { (void)hipHostFree(p); }
    } hf{h_active};
    auto active = [&]() {
        SPMVC_HIP(hipMemcpyAsync(h_active, nact.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        SPMVC_HIP(hipStreamSynchronize(st));
        return *h_active;
    };

    const int chunk = std::max(1, o.check_every);
    int it = 0;
    // iterations in groups of `chunk` until every pair has stopped
    hipGraphExec_t exec = nullptr;
    hipStream_t cs = st;
    struct GraphFree {
        hipGraphExec_t *e;
        hipStream_t *s;
        hipStream_t owner;
        ~GraphFree() {
            if (*e) (void)hipGraphExecDestroy(*e);
            if (*s != owner) (void)hipStreamDestroy(*s);
        }
    } gf{&exec, &cs, st};
    if (use_graph) {
        // `chunk` iterations recorded once, replayed
        SPMVC_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        SPMVC_HIP(hipStreamSynchronize(st));
        hipGraph_t graph = nullptr;
        SPMVC_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        for (int j = 0; j < chunk; ++j) record_iteration(b, cs);
        SPMVC_HIP(hipStreamEndCapture(cs, &graph));
        const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        SPMVC_HIP(ie);
    }
    auto run = [&]() {
        while (it < o.max_iter && active() > 0) {
            if (use_graph) {
                SPMVC_HIP(hipGraphLaunch(exec, cs));
                SPMVC_HIP(hipStreamSynchronize(cs));
            } else {
                for (int j = 0; j < chunk; ++j) record_iteration(b, st);
                SPMVC_CHECK_LAUNCH();
            }
            it += chunk;
        }
    };
    // true residuals ||b - A x||^2 per pair into rr (every system)
    auto true_residuals = [&]() {
        k_set_all<<<static_cast<unsigned>((n_sys + 255) / 256), 256, 0, st>>>(b.sys_active, 1, n_sys);
        launch_bspmv(b, b.X, b.Q, 0, st);
        SPMVC_LPR_LAUNCH(k_bresid, static_cast<unsigned>(n_tiles), st, b);
        k_bresid_fin<<<static_cast<unsigned>(n_sys), kT, 0, st>>>(b, rr.as<double>());
        SPMVC_CHECK_LAUNCH();
    };
    run();
    true_residuals();
    // pairs whose recursive residual met the tolerance but whose true one did
    // not restart from the true residual
    for (int k = 0; k < kMaxRestarts && active() == 0; ++k) {
        k_brestart_fin<<<static_cast<unsigned>(n_sys), kT, 0, st>>>(b, rr.as<double>());
        SPMVC_LPR_LAUNCH(k_brestart, static_cast<unsigned>(n_tiles), st, b);
        SPMVC_CHECK_LAUNCH();
        if (active() == 0) break;
        run();
        true_residuals();
    }
    std::vector<double> h_rr(np), h_rho0(np), h_rel(np);
    std::vector<int32_t> h_it(np), h_st(np), h_done(np);
    SPMVC_HIP(hipMemcpyAsync(h_rr.data(), rr.p, sizeof(double) * np, hipMemcpyDeviceToHost, st));
    SPMVC_HIP(hipMemcpyAsync(h_rho0.data(), rho0.p, sizeof(double) * np, hipMemcpyDeviceToHost, st));
    SPMVC_HIP(hipMemcpyAsync(h_rel.data(), relres.p, sizeof(double) * np, hipMemcpyDeviceToHost, st));
    SPMVC_HIP(hipMemcpyAsync(h_it.data(), iters.p, sizeof(int32_t) * np, hipMemcpyDeviceToHost, st));
    SPMVC_HIP(hipMemcpyAsync(h_st.data(), status.p, sizeof(int32_t) * np, hipMemcpyDeviceToHost, st));
    SPMVC_HIP(hipMemcpyAsync(h_done.data(), done.p, sizeof(int32_t) * np, hipMemcpyDeviceToHost, st));
    for (int s = 0; s < n_sys; ++s)
        SPMVC_HIP(hipMemcpyAsync(xvec[s], X.as<double>() + sd[s].row0 * nrhs, sizeof(double) * sd[s].n * nrhs,
                                 hipMemcpyDeviceToDevice, st));
    SPMVC_HIP(hipStreamSynchronize(st));
    spmvc_status first_bad = SPMVC_OK;
    for (int q = 0; q < np; ++q) {
        spmvc_cg_stat &c = stat[q];
        c.iters = h_it[q];
        c.outer_iters = 0;
        c.status = h_done[q] ? h_st[q] : SPMVC_ENOCONV;
        c.relres_recursive = h_rel[q];
        c.relres_true = h_rho0[q] > 0.0 ? std::sqrt(h_rr[q]) / std::sqrt(h_rho0[q]) : std::sqrt(h_rr[q]);
        if (c.status == SPMVC_OK && !(c.relres_true <= o.rtol)) c.status = SPMVC_ENOCONV;
        if (c.status != SPMVC_OK && first_bad == SPMVC_OK) first_bad = static_cast<spmvc_status>(c.status);
    }
    return first_bad;
}

// bounds violations the kernels of this file recorded (checked builds)
SPMVC_CHECK_READER(check_violations_batched)

}  // namespace spmvc
