// Conjugate gradients on the GPU: BLAS-1 kernels with deterministic grid
// reductions, the FP64 CG driver and the mixed-precision iterative-refinement
// driver.
//
// The CG part of the iteration in Table I (DotProduct, Waxpby, SpMV) in
// textbook Hestenes-Stiefel form from x0 = 0:
//   q = A p;  sigma = p.q;  alpha = rho / sigma;  x += alpha p;  r -= alpha q;
//   rho' = r.r;  stop when sqrt(rho') <= rtol sqrt(rho0);  p = r + (rho'/rho) p.
// All scalars live in device memory; the host reads them back once every
// `check_every` iterations.  Once a solve is finished every later kernel of
// the batch returns at entry (the `done` flag), so surplus launches cost only
// their launch overhead.
//
// Reductions without device-wide fences: every block reduces its elements in a
// fixed order (wavefront butterfly through lane permutes, then the waves in
// index order) and writes one partial; the *next* kernel reads all partials
// and every one of its blocks adds them in the same fixed order, so all blocks
// hold the identical scalar and no block waits for another.  (An agent-scope
// release per block -- the usual last-block-done pattern -- writes back the
// whole L2 of an XCD on this chip and costs more than the streaming itself.)
// The SpMV of the iteration writes the p.q partials itself, and x advances in
// the p-update kernel (which reads p anyway), so an iteration is three
// launches: SpMV + p.q, r-update + r.r, x- and p-update.  Scalars that
// persist across iterations are written by block 0 only, into slots other
// blocks of the same kernel do not read (rho is double-buffered by iteration
// parity; the iteration index comes from the host).  Results do not depend on
// block scheduling, so iteration counts repeat exactly from run to run.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <memory>
#include <mutex>

#include "internal.h"
#include "reduce.h"

namespace spmvc {
namespace {

constexpr int kRT = 512;                // threads per BLAS-1 block (8 waves)
constexpr unsigned kRMaxBlocks = 256;   // partials per reduction (fewer partials: cheaper consumer sums)

struct CgScal {
    double rho[2];    // r.r of the current iterate, by iteration parity
    double rho0, rtol, rel, sigma;
    int32_t iters, max_iter, done, status;
    int32_t go[2];    // the update step of the iteration (by parity) ran: the p-update must run
    double aux[4];
};

// Sum of partials[0..np) in a fixed order; identical in every block.  Each
// thread adds its partials i, i + NT, i + 2 NT, ... in that order, loading
// sixteen of them at a time (independent loads in flight, the last batch
// predicated): an SpMV can leave over ten thousand partials, and one
// dependent load per partial would make this sum a chain of cache round trips.
template <int NT> __device__ __forceinline__ double sum_partials(const double *partials, int np) {
    constexpr int B = 16;
    double s = 0.0;
    for (int i0 = threadIdx.x; i0 < np; i0 += B * NT) {
        double v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) v[u] = i0 + u * NT < np ? partials[i0 + u * NT] : 0.0;
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (i0 + u * NT < np) s += v[u];
    }
    return block_sum<NT>(s);
}

template <class Real> __device__ __forceinline__ double dd(Real v) { return static_cast<double>(v); }

// Grid-stride loop over [0, N) that handles four items per step, each a
// stride apart, so every thread has four independent loads of each stream in
// flight; the tail is handled one item at a time.
#define SPMVC_STREAM4N(N, BODY4, BODY1)                                                          \
    {                                                                                            \
        const int64_t stride_ = static_cast<int64_t>(gridDim.x) * kRT;                           \
        int64_t i = static_cast<int64_t>(blockIdx.x) * kRT + threadIdx.x;                        \
        for (; i + 3 * stride_ < (N); i += 4 * stride_) {                                        \
            BODY4                                                                                \
        }                                                                                        \
        for (; i < (N); i += stride_) {                                                          \
            BODY1                                                                                \
        }                                                                                        \
    }
#define SPMVC_STREAM4(BODY4, BODY1) SPMVC_STREAM4N(n, BODY4, BODY1)

// W consecutive elements moved as one access: 16-byte loads and stores double
// the bytes each wave has in flight over 8-byte (FP64) ones and quadruple them
// over 4-byte (FP32) ones, which is what the two CG update kernels need to
// approach the HBM rate with one 8-wave block per CU.
template <class Real, int W> struct Pack;
template <class Real> struct Pack<Real, 1> { using T = Real; };
template <> struct Pack<double, 2> { using T = double __attribute__((ext_vector_type(2))); };
template <> struct Pack<float, 4> { using T = float __attribute__((ext_vector_type(4))); };

__device__ __forceinline__ double sumsq(double v) { return v * v; }
__device__ __forceinline__ double sumsq(float v) { return static_cast<double>(v) * static_cast<double>(v); }
__device__ __forceinline__ double sumsq(Pack<double, 2>::T v) { return v.x * v.x + v.y * v.y; }
__device__ __forceinline__ double sumsq(Pack<float, 4>::T v) {
    return sumsq(v.x) + sumsq(v.y) + sumsq(v.z) + sumsq(v.w);
}

template <class Real> constexpr int pack_width() { return 16 / static_cast<int>(sizeof(Real)); }

inline bool aligned16(const void *a, const void *b, const void *c = nullptr) {
    return ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(c)) & 15) == 0;
}

// x = 0, r = rhs / norm, p = r; partials of r.r.  The division (in the
// precision of rhs, before any conversion) lets the mixed-precision driver
// hand the FP32 solve a right-hand side of unit norm whatever the scale of
// the FP64 residual; norm == 1 leaves rhs unchanged.
template <class Real, class RhsT>
__global__ __launch_bounds__(kRT) void k_cg_start(int64_t n, const RhsT *__restrict__ rhs, RhsT norm,
                                                  Real *__restrict__ x, Real *__restrict__ r, Real *__restrict__ p,
                                                  double *partials) {
    double acc = 0.0;
    const bool unit = norm == RhsT(1);
    SPMVC_STREAM4(
        Real v[4];
_Pragma("unroll") for (int u = 0; u < 4; ++u) {
            const RhsT w = rhs[i + u * stride_];
            v[u] = static_cast<Real>(unit ? w : w / norm);
        }
_Pragma("unroll") for (int u = 0; u < 4; ++u) {
            x[i + u * stride_] = Real(0); r[i + u * stride_] = v[u]; p[i + u * stride_] = v[u];
            acc += dd(v[u]) * dd(v[u]);
        }
        ,
        const Real v = static_cast<Real>(unit ? rhs[i] : rhs[i] / norm);
        x[i] = Real(0); r[i] = v; p[i] = v;
        acc += dd(v) * dd(v);
    )
    const double b = block_sum<kRT>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

// rho0 = rho[0] = sum of the partials; state reset (one block)
__device__ __forceinline__ void cg_start_fin(const double *partials, int np, CgScal *st, double rtol, int max_iter) {
    const double tot = sum_partials<kRT>(partials, np);
    if (threadIdx.x != 0) return;
    st->rho[0] = tot;
    st->rho[1] = 0.0;
    st->rho0 = tot;
    st->rtol = rtol;
    st->iters = 0;
    st->max_iter = max_iter;
    st->rel = tot > 0.0 ? 1.0 : 0.0;
    st->done = (tot == 0.0) ? 1 : 0;
    st->status = SPMVC_OK;
    st->go[0] = st->go[1] = 0;
    if (!(tot == tot) || tot > 1.7e308) {
        st->done = 1;
        st->status = SPMVC_EINVAL;
    }
}

__global__ __launch_bounds__(kRT) void k_cg_start_fin(const double *partials, int np, CgScal *st, double rtol,
                                                      int max_iter) {
    cg_start_fin(partials, np, st, rtol, max_iter);
}

// Restart of a finished solve whose recursive residual met the tolerance but
// whose true FP64 residual b - A x (already in r, squared norm rr) did not:
// p = r and the scalars of iteration `it` take rho = rr; rho0 (the ||b||^2 of
// the stopping test) is kept, so the solve continues towards the same target
// from the true residual.
__global__ __launch_bounds__(kRT) void k_cg_resume(int64_t n, const double *__restrict__ r, double *__restrict__ p,
                                                   CgScal *st, double rr, int it) {
    SPMVC_STREAM4(
_Pragma("unroll") for (int u = 0; u < 4; ++u) p[i + u * stride_] = r[i + u * stride_];
        ,
        p[i] = r[i];
    )
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rho[it & 1] = rr;
        st->rel = sqrt(rr) / sqrt(st->rho0);
        st->done = 0;
        st->status = SPMVC_OK;
        st->go[0] = st->go[1] = 0;
    }
}

// sigma = sum of the p.q partials of the SpMV; alpha = rho / sigma;
// r -= alpha q; partials of r.r.  A breakdown (sigma <= 0 or not finite) stops
// the solve.  Block 0 records sigma and whether the step ran (go), which the
// p-update reads: it must not read `done`, which its own block 0 may set.
// Each thread's first group of r and q is loaded before the scalars and the
// partial sums are read (it does not depend on alpha), so that the latency of
// those loads overlaps the latency of the sums; the elements and the order of
// the r.r sum are those of the plain grid-stride loop (SPMVC_STREAM4N).
template <class Real, int W>
__global__ __launch_bounds__(kRT) void k_cg_update(int64_t n, Real *__restrict__ r, const Real *__restrict__ q,
                                                   const double *sig_part, int n_sig, double *rr_part, CgScal *st,
                                                   int par, int it) {
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    using T = typename Pack<Real, W>::T;
    T *__restrict__ rw = reinterpret_cast<T *>(r);
    const T *__restrict__ qw = reinterpret_cast<const T *>(q);
    const int64_t nw = n / W;
    const int64_t stride_ = static_cast<int64_t>(gridDim.x) * kRT;
    int64_t i = static_cast<int64_t>(blockIdx.x) * kRT + threadIdx.x;
    T rv[4], qv[4];
    const bool first = i + 3 * stride_ < nw;
    if (first) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            rv[u] = rw[i + u * stride_];
            qv[u] = qw[i + u * stride_];
        }
    }
    if (st->done) {
        if (lead) st->go[par] = 0;
        return;
    }
    const double sigma = sum_partials<kRT>(sig_part, n_sig);
    if (!(sigma > 0.0) || !isfinite(sigma)) {
        if (lead) {
            st->sigma = sigma;
            st->done = 1;
            st->status = SPMVC_ENOTSPD;
            st->iters = it + 1;
            st->go[par] = 0;
        }
        return;
    }
    if (lead) {
        st->sigma = sigma;
        st->go[par] = 1;
    }
    const Real alpha = static_cast<Real>(st->rho[par] / sigma);
    double acc = 0.0;
    if (first) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const T ri = rv[u] - alpha * qv[u];
            rw[i + u * stride_] = ri;
            acc += sumsq(ri);
        }
        i += 4 * stride_;
    }
    for (; i + 3 * stride_ < nw; i += 4 * stride_) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            rv[u] = rw[i + u * stride_];
            qv[u] = qw[i + u * stride_];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const T ri = rv[u] - alpha * qv[u];
            rw[i + u * stride_] = ri;
            acc += sumsq(ri);
        }
    }
    for (; i < nw; i += stride_) {
        const T ri = rw[i] - alpha * qw[i];
        rw[i] = ri;
        acc += sumsq(ri);
    }
    if (W > 1 && blockIdx.x == 0) {  // the last n mod W elements
        const int64_t k = nw * W + threadIdx.x;
        if (k < n) {
            const Real ri = r[k] - alpha * q[k];
            r[k] = ri;
            acc += sumsq(ri);
        }
    }
    const double b = block_sum<kRT>(acc);
    if (threadIdx.x == 0) rr_part[blockIdx.x] = b;
}

// rho' = sum of the r.r partials; convergence test; x += alpha p (with the
// update step's alpha); unless the solve stops here, beta = rho'/rho and
// p = r + beta p.  x is updated here, not in k_cg_update, so p is read once.
// As in k_cg_update, each thread's first group of x, r and p is loaded before
// the scalars and the partial sums are read.
template <class Real, int W>
__global__ __launch_bounds__(kRT) void k_cg_pupdate(int64_t n, Real *__restrict__ x, const Real *__restrict__ r,
                                                    Real *__restrict__ p, const double *rr_part, int n_rr,
                                                    CgScal *st, int par, int it) {
    using T = typename Pack<Real, W>::T;
    T *__restrict__ xw = reinterpret_cast<T *>(x);
    const T *__restrict__ rw = reinterpret_cast<const T *>(r);
    T *__restrict__ pw = reinterpret_cast<T *>(p);
    const int64_t nw = n / W;
    const int64_t stride_ = static_cast<int64_t>(gridDim.x) * kRT;
    int64_t i = static_cast<int64_t>(blockIdx.x) * kRT + threadIdx.x;
    T xv[4], rv[4], pv[4];
    const bool first = i + 3 * stride_ < nw;
    if (first) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            xv[u] = xw[i + u * stride_];
            rv[u] = rw[i + u * stride_];
            pv[u] = pw[i + u * stride_];
        }
    }
    if (!st->go[par]) return;
    const double rho_new = sum_partials<kRT>(rr_part, n_rr);
    const double rho = st->rho[par];
    const bool conv = sqrt(rho_new) <= st->rtol * sqrt(st->rho0);
    const bool stop = conv || (it + 1 >= st->max_iter) || !isfinite(rho_new);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->iters = it + 1;
        st->rel = sqrt(rho_new) / sqrt(st->rho0);
        st->rho[par ^ 1] = rho_new;
        if (conv) {
            st->done = 1;
            st->status = SPMVC_OK;
        } else if (!isfinite(rho_new)) {
            st->done = 1;
            st->status = SPMVC_ENOTSPD;
        } else if (it + 1 >= st->max_iter) {
            st->done = 1;
            st->status = SPMVC_ENOCONV;
        }
    }
    const Real alpha = static_cast<Real>(rho / st->sigma);
    const int64_t tail = (W > 1 && blockIdx.x == 0) ? nw * W + threadIdx.x : n;  // the last n mod W elements
    if (stop) {
        if (first) {
#pragma unroll
            for (int u = 0; u < 4; ++u) xw[i + u * stride_] = xv[u] + alpha * pv[u];
            i += 4 * stride_;
        }
        for (; i + 3 * stride_ < nw; i += 4 * stride_) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                xv[u] = xw[i + u * stride_];
                pv[u] = pw[i + u * stride_];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) xw[i + u * stride_] = xv[u] + alpha * pv[u];
        }
        for (; i < nw; i += stride_) xw[i] = xw[i] + alpha * pw[i];
        if (tail < n) x[tail] = x[tail] + alpha * p[tail];
        return;
    }
    const Real beta = static_cast<Real>(rho_new / rho);
    if (first) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            xw[i + u * stride_] = xv[u] + alpha * pv[u];
            pw[i + u * stride_] = rv[u] + beta * pv[u];
        }
        i += 4 * stride_;
    }
    for (; i + 3 * stride_ < nw; i += 4 * stride_) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            xv[u] = xw[i + u * stride_];
            rv[u] = rw[i + u * stride_];
            pv[u] = pw[i + u * stride_];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            xw[i + u * stride_] = xv[u] + alpha * pv[u];
            pw[i + u * stride_] = rv[u] + beta * pv[u];
        }
    }
    for (; i < nw; i += stride_) {
        xw[i] = xw[i] + alpha * pw[i];
        pw[i] = rw[i] + beta * pw[i];
    }
    if (tail < n) {
        x[tail] = x[tail] + alpha * p[tail];
        p[tail] = r[tail] + beta * p[tail];
    }
}

// ---- preconditioned CG with one multicolor SymGS sweep as M^-1 (mode 2) -------------
// The iteration of Table I with SymGS as the whole preconditioner (no
// multigrid levels): z = M^-1 r is one symmetric Gauss-Seidel sweep on
// A z = r from z = 0.  rho[] holds r.z; the stopping test uses r.r.

// z = 0 (a fill kernel, no memset), unless the solve has stopped
__global__ __launch_bounds__(kRT) void k_pcg_zero(int64_t n, double *__restrict__ z, const CgScal *st) {
    if (st->done) return;
    SPMVC_STREAM4(
_Pragma("unroll") for (int u = 0; u < 4; ++u) z[i + u * stride_] = 0.0;
        ,
        z[i] = 0.0;
    )
}

// p = z; partials of r.z (start of the iteration)
__global__ __launch_bounds__(kRT) void k_pcg_init(int64_t n, const double *__restrict__ r, const double *__restrict__ z,
                                                  double *__restrict__ p, double *rz_part) {
    double acc = 0.0;
    SPMVC_STREAM4(
        double rv[4]; double zv[4];
_Pragma("unroll") for (int u = 0; u < 4; ++u) { rv[u] = r[i + u * stride_]; zv[u] = z[i + u * stride_]; }
_Pragma("unroll") for (int u = 0; u < 4; ++u) {
            p[i + u * stride_] = zv[u];
            acc += rv[u] * zv[u];
        }
        ,
        p[i] = z[i];
        acc += r[i] * z[i];
    )
    const double b = block_sum<kRT>(acc);
    if (threadIdx.x == 0) rz_part[blockIdx.x] = b;
}

// rho[slot] = r.z (one block)
__global__ __launch_bounds__(kRT) void k_pcg_init_fin(const double *rz_part, int np, CgScal *st, int slot) {
    const double tot = sum_partials<kRT>(rz_part, np);
    if (threadIdx.x == 0 && !st->done) st->rho[slot] = tot;
}

// Restart of a preconditioned solve from its true residual (see k_cg_resume):
// the solve is running again from iteration `it`; the preconditioner and
// k_pcg_init / k_pcg_init_fin (slot it & 1) follow.
__global__ void k_pcg_resume(CgScal *st, double rr) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rel = sqrt(rr) / sqrt(st->rho0);
        st->done = 0;
        st->status = SPMVC_OK;
        st->go[0] = st->go[1] = 0;
    }
}

// sigma = p.q (the SpMV's partials); alpha = rho / sigma; x += alpha p;
// r -= alpha q; partials of r.r.  Block 0 records sigma and go[par].
__global__ __launch_bounds__(kRT) void k_pcg_update(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                                    const double *__restrict__ p, const double *__restrict__ q,
                                                    const double *sig_part, int n_sig, double *rr_part, CgScal *st,
                                                    int par, int it) {
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (st->done) {
        if (lead) st->go[par] = 0;
        return;
    }
    const double sigma = sum_partials<kRT>(sig_part, n_sig);
    if (!(sigma > 0.0) || !isfinite(sigma)) {
        if (lead) {
            st->sigma = sigma;
            st->done = 1;
            st->status = SPMVC_ENOTSPD;
            st->iters = it + 1;
            st->go[par] = 0;
        }
        return;
    }
    if (lead) {
        st->sigma = sigma;
        st->go[par] = 1;
    }
    const double alpha = st->rho[par] / sigma;
    double acc = 0.0;
    SPMVC_STREAM4(
        double xv[4]; double rv[4]; double pv[4]; double qv[4];
_Pragma("unroll") for (int u = 0; u < 4; ++u) {
            xv[u] = x[i + u * stride_]; rv[u] = r[i + u * stride_];
            pv[u] = p[i + u * stride_]; qv[u] = q[i + u * stride_];
        }
_Pragma("unroll") for (int u = 0; u < 4; ++u) {
            x[i + u * stride_] = xv[u] + alpha * pv[u];
            const double ri = rv[u] - alpha * qv[u];
            r[i + u * stride_] = ri;
            acc += ri * ri;
        }
        ,
        x[i] = x[i] + alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        acc += ri * ri;
    )
    const double b = block_sum<kRT>(acc);
    if (threadIdx.x == 0) rr_part[blockIdx.x] = b;
}

// The stopping test on r.r; partials of r.z (z = M^-1 r of this iteration).
__global__ __launch_bounds__(kRT) void k_pcg_rz(int64_t n, const double *__restrict__ r, const double *__restrict__ z,
                                                const double *rr_part, int n_rr, double *rz_part, CgScal *st, int par,
                                                int it) {
    if (!st->go[par]) return;
    const double rr = sum_partials<kRT>(rr_part, n_rr);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->iters = it + 1;
        st->rel = sqrt(rr) / sqrt(st->rho0);
        if (sqrt(rr) <= st->rtol * sqrt(st->rho0)) {
            st->done = 1;
            st->status = SPMVC_OK;
        } else if (!isfinite(rr)) {
            st->done = 1;
            st->status = SPMVC_ENOTSPD;
        } else if (it + 1 >= st->max_iter) {
            st->done = 1;
            st->status = SPMVC_ENOCONV;
        }
    }
    double acc = 0.0;
    SPMVC_STREAM4(
        double rv[4]; double zv[4];
_Pragma("unroll") for (int u = 0; u < 4; ++u) { rv[u] = r[i + u * stride_]; zv[u] = z[i + u * stride_]; }
_Pragma("unroll") for (int u = 0; u < 4; ++u) acc += rv[u] * zv[u];
        ,
        acc += r[i] * z[i];
    )
    const double b = block_sum<kRT>(acc);
    if (threadIdx.x == 0) rz_part[blockIdx.x] = b;
}

// beta = rho' / rho (rho' = r.z); p = z + beta p.  `done` was settled by the
// previous kernel, so it can be read here.
__global__ __launch_bounds__(kRT) void k_pcg_p(int64_t n, const double *__restrict__ z, double *__restrict__ p,
                                               const double *rz_part, int n_rz, CgScal *st, int par) {
    if (!st->go[par] || st->done) return;
    const double rz = sum_partials<kRT>(rz_part, n_rz);
    if (blockIdx.x == 0 && threadIdx.x == 0) st->rho[par ^ 1] = rz;
    const double beta = rz / st->rho[par];
    SPMVC_STREAM4(
        double zv[4]; double pv[4];
_Pragma("unroll") for (int u = 0; u < 4; ++u) { zv[u] = z[i + u * stride_]; pv[u] = p[i + u * stride_]; }
_Pragma("unroll") for (int u = 0; u < 4; ++u) p[i + u * stride_] = zv[u] + beta * pv[u];
        ,
        p[i] = z[i] + beta * p[i];
    )
}

// partials of (b - ax).(b - ax), optionally storing r = b - ax; partials of b.b
__global__ __launch_bounds__(kRT) void k_residual(int64_t n, const double *__restrict__ b,
                                                  const double *__restrict__ ax, double *__restrict__ r,
                                                  double *rr_part, double *bb_part) {
    double acc = 0.0, accb = 0.0;
    SPMVC_STREAM4(
        double bv[4]; double av[4];
_Pragma("unroll") for (int u = 0; u < 4; ++u) { bv[u] = b[i + u * stride_]; av[u] = ax[i + u * stride_]; }
_Pragma("unroll") for (int u = 0; u < 4; ++u) {
            const double v = bv[u] - av[u];
            if (r) r[i + u * stride_] = v;
            acc += v * v;
            accb += bv[u] * bv[u];
        }
        ,
        const double v = b[i] - ax[i];
        if (r) r[i] = v;
        acc += v * v;
        accb += b[i] * b[i];
    )
    const double s1 = block_sum<kRT>(acc);
    const double s2 = block_sum<kRT>(accb);
    if (threadIdx.x == 0) {
        rr_part[blockIdx.x] = s1;
        bb_part[blockIdx.x] = s2;
    }
}

// aux[0] = sum of rr partials, aux[1] = sum of bb partials (one block)
__global__ __launch_bounds__(kRT) void k_residual_fin(const double *rr_part, const double *bb_part, int np,
                                                      CgScal *st) {
    const double a = sum_partials<kRT>(rr_part, np);
    const double b = sum_partials<kRT>(bb_part, np);
    if (threadIdx.x == 0) {
        st->aux[0] = a;
        st->aux[1] = b;
    }
}

// Scalars of the reliable-update solve that pass from one segment to the next
// on the device, so that the host can queue the FP64 replacement and the next
// segment without first reading the residual back.
struct RelState {
    double sn;       // the current segment's scale: ||b - A x|| at its start
    double beta;     // factor taking p into the units of sn (0: p = r)
    double seg_tol;  // the segment's tolerance, relative to its start
    double bnorm;    // ||b||
    int32_t fin;     // 0 while segments run; 1 converged, 2 out of iterations or replacements, 3 breakdown
};
constexpr int32_t kRelOk = 1, kRelNoConv = 2, kRelBreakdown = 3;

// the first segment's scalars, computed by the host from the first residual
__global__ void k_rel_first(RelState *rs, double sn, double seg_tol, double bnorm) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *rs = RelState{sn, 0.0, seg_tol, bnorm, 0};
}

// After a segment and the FP64 replacement r = b - A x (||r||^2 in aux[0]):
// the stopping tests, then the next segment's scale sn' = ||r||, the factor
// beta = sn' / (sn rho_k) that takes p into the new units (rho_k: the
// segment's r.r before its last step, in units of sn) and its tolerance,
// inner_rtol, raised so that the segment does not go past the final target
// (0.9 rtol / rel) and capped at 0.5.  On a stop, fin records why and the
// solve is marked done, so that the segment kernels queued behind do nothing.
// aux[2] = fin and aux[3] = the finished segment's recursive residual over
// ||b|| go back to the host with the scalars it reads next.
__global__ void k_rel_next(CgScal *st, RelState *rs, double rtol, double inner_rtol, int segs, int total,
                           int max_outer, int max_iter, double rho_k) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double rr = st->aux[0];
    const double rel = sqrt(rr) / rs->bnorm;
    const double sn_old = rs->sn;
    st->aux[3] = st->rel * sn_old / rs->bnorm;
    int32_t fin = 0;
    if (!isfinite(rel))
        fin = kRelBreakdown;
    else if (rel <= rtol)
        fin = kRelOk;
    else if (segs > max_outer || total >= max_iter)
        fin = kRelNoConv;
    rs->fin = fin;
    st->aux[2] = static_cast<double>(fin);
    if (fin) {
        st->done = 1;
        return;
    }
    const double sn = sqrt(rr);
    rs->beta = rho_k > 0.0 ? sn / (sn_old * rho_k) : 0.0;
    rs->sn = sn;
    rs->seg_tol = fmin(fmax(inner_rtol, 0.9 * rtol / rel), 0.5);
}

// Start of a reliable-update segment: r = r64 / s (the FP64 true residual in
// units of its norm s), p = r + beta p (beta = 0: p = r; otherwise p keeps the
// previous segment's direction, rescaled into the new units by beta), xl = 0;
// partials of r.r.  s and beta come from rs; nothing is done once the solve
// has stopped.
__global__ __launch_bounds__(kRT) void k_rel_start(int64_t n, const double *__restrict__ r64,
                                                   const RelState *rs, float *__restrict__ xl,
                                                   float *__restrict__ r, float *__restrict__ p,
                                                   double *partials) {
    if (rs->fin) return;
    const double s = rs->sn;
    const float beta = static_cast<float>(rs->beta);
    double acc = 0.0;
    const bool fresh = beta == 0.0f;
    SPMVC_STREAM4(
        float v[4]; float pv[4];
_Pragma("unroll") for (int u = 0; u < 4; ++u) {
            v[u] = static_cast<float>(r64[i + u * stride_] / s);
            pv[u] = fresh ? 0.0f : p[i + u * stride_];
        }
_Pragma("unroll") for (int u = 0; u < 4; ++u) {
            xl[i + u * stride_] = 0.0f; r[i + u * stride_] = v[u]; p[i + u * stride_] = v[u] + beta * pv[u];
            acc += dd(v[u]) * dd(v[u]);
        }
        ,
        const float v = static_cast<float>(r64[i] / s);
        p[i] = v + beta * (fresh ? 0.0f : p[i]);
        xl[i] = 0.0f; r[i] = v;
        acc += dd(v) * dd(v);
    )
    const double b = block_sum<kRT>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

// the segment's reset of the CG scalars with its tolerance from rs (one block)
__global__ __launch_bounds__(kRT) void k_rel_start_fin(const double *partials, int np, CgScal *st,
                                                       const RelState *rs, int max_iter) {
    if (rs->fin) return;
    cg_start_fin(partials, np, st, rs->seg_tol, max_iter);
}

// x += scale * (double) d
__global__ void k_add_f32(int64_t n, double *__restrict__ x, const float *__restrict__ d, double scale) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        x[i] += scale * static_cast<double>(d[i]);
}

// x += sn * (double) d with the segment's scale from rs
__global__ void k_add_rel(int64_t n, double *__restrict__ x, const float *__restrict__ d, const RelState *rs) {
    const double scale = rs->sn;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        x[i] += scale * static_cast<double>(d[i]);
}

// column r of a row-interleaved block <-> contiguous vector
__global__ void k_gather_col(int64_t n, const double *__restrict__ B, int ld, int r, double *__restrict__ v) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        v[i] = B[i * ld + r];
}

__global__ void k_scatter_col(int64_t n, const double *__restrict__ v, double *__restrict__ B, int ld, int r) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        B[i * ld + r] = v[i];
}

unsigned rgrid(int64_t n) {
    int64_t g = (n + kRT * 8 - 1) / (kRT * 8);
    return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(g, kRMaxBlocks)));
}

// scalars = 0 (a fill kernel rather than a memset node, so that the solver's
// work can also be recorded into a graph)
__global__ void k_zero_scal(CgScal *st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *st = CgScal{};
}

struct Pinned {
    CgScal *h = nullptr;  // three host copies: the synchronous read and the two pipelined slots
    Pinned() { SPMVC_HIP(hipHostMalloc(reinterpret_cast<void **>(&h), 3 * sizeof(CgScal), hipHostMallocDefault)); }
    ~Pinned() {
        if (h) (void)hipHostFree(h);
    }
    Pinned(const Pinned &) = delete;
    Pinned &operator=(const Pinned &) = delete;
};

// Scalars and reduction partials of one solve, on the device, plus the host
// copy the driver reads.  Either owned (allocated here) or carved from a
// caller's region (nothing allocated; the host copy is then pageable).
struct Solver {
    hipStream_t s;
    CgScal *dscal = nullptr;
    double *pa = nullptr, *pb = nullptr, *psig = nullptr;  // partials: kRMaxBlocks, kRMaxBlocks, SpMV blocks
    CgScal *h = nullptr;
    DevBuf scal, part_a, part_b, part_sig;
    std::unique_ptr<Pinned> pin;
    CgScal h_pageable{};
    hipEvent_t ev[2] = {nullptr, nullptr};  // pipelined status reads (owned solvers only)
    Solver(hipStream_t st, int64_t sig_blocks) : s(st) {
        scal.alloc(sizeof(CgScal));
        part_a.alloc(sizeof(double) * kRMaxBlocks);
        part_b.alloc(sizeof(double) * kRMaxBlocks);
        part_sig.alloc(sizeof(double) * std::max<int64_t>(sig_blocks, 1));
        pin.reset(new Pinned());
        for (hipEvent_t &e : ev) SPMVC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        bind(scal.as<CgScal>(), part_a.as<double>(), part_b.as<double>(), part_sig.as<double>(), pin->h);
    }
    ~Solver() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    Solver(const Solver &) = delete;
    Solver &operator=(const Solver &) = delete;
    // region: kSolverScalBytes of scalars, then 2 * kRMaxBlocks partials, then the SpMV partials
    Solver(hipStream_t st, char *region) : s(st) {
        double *parts = reinterpret_cast<double *>(region + kSolverScalBytes);
        bind(reinterpret_cast<CgScal *>(region), parts, parts + kRMaxBlocks, parts + 2 * kRMaxBlocks, &h_pageable);
    }
    static constexpr size_t kSolverScalBytes = 256;
    void bind(CgScal *d, double *a, double *b, double *sig, CgScal *host) {
        dscal = d;
        pa = a;
        pb = b;
        psig = sig;
        h = host;
        k_zero_scal<<<1, 64, 0, s>>>(dscal);
        SPMVC_CHECK_LAUNCH();
    }
    CgScal *st() { return dscal; }
    const CgScal &read() {
        SPMVC_HIP(hipMemcpyAsync(h, dscal, sizeof(CgScal), hipMemcpyDeviceToHost, s));
        SPMVC_HIP(hipStreamSynchronize(s));
        return *h;
    }
    // Enqueues chunks of at most `full` iterations (launch_chunk(n) queues up
    // to n and returns how many it queued, 0 when there is nothing left) until
    // the solve reports done.  The host reads the scalars after chunk k while
    // chunk k + 1 is already queued, so the device does not idle during the
    // read; iterations queued after the solve finished run as no-ops (every
    // kernel of an iteration returns at once when `done` is set, but each
    // launch still costs a few microseconds, and a preconditioned iteration is
    // dozens of launches).  So the residuals of the last two reads, continued
    // geometrically, predict how many iterations are still needed: when they
    // are fewer than the chunk in flight, the next chunk is queued only after
    // that chunk's status has been read, and when they end within the next
    // chunk, that chunk is cut to the prediction plus a margin.  Without
    // events (the allocation-free solver) each read waits for the stream.
    // Returns true with the scalars that showed the solve done in `out`;
    // false when launch_chunk() ran out first (nothing read since).  A chunk
    // queued past the end leaves these scalars as they were, so the caller
    // can go on enqueuing without another read.
    // A solve expected to take few iterations passes first > 0: the chunks
    // queued before any read is back then hold `first` iterations each.
    template <class F> bool iterate_chunks(int full, F &&launch_chunk, CgScal &out, int first = 0) {
        full = std::max(1, full);
        const int blind = first > 0 ? std::min(first, full) : full;
        if (!ev[0]) {
            while (true) {
                const CgScal &h = read();
                if (h.done) {
                    out = h;
                    return true;
                }
                if (!launch_chunk(full)) return false;
            }
        }
        auto post = [&](int slot) {
            SPMVC_HIP(hipMemcpyAsync(pin->h + 1 + slot, dscal, sizeof(CgScal), hipMemcpyDeviceToHost, s));
            SPMVC_HIP(hipEventRecord(ev[slot], s));
        };
        int len[2] = {0, 0};  // iterations of the chunk posted to each slot
        len[0] = launch_chunk(blind);
        if (!len[0]) return false;
        post(0);
        double rel_prev = -1.0, rel_last = -1.0, tol = 0.0;  // the last two reads
        int it_prev = 0, it_last = 0;
        // iterations still needed after the last read (infinite when unknown)
        auto need = [&]() -> double {
            if (!(rel_prev > 0.0 && rel_last > 0.0 && rel_last < rel_prev && it_last > it_prev && tol > 0.0))
                return HUGE_VAL;
            return std::log(tol / rel_last) / std::log(rel_last / rel_prev) * (it_last - it_prev);
        };
        // length of the next chunk when `ahead` iterations are queued past the last read
        auto next_len = [&](int ahead) -> int {
            if (rel_last < 0.0) return blind;  // nothing read yet
            const double left = need() - ahead;
            if (!(left < full)) return full;
            return std::min(full, std::max(1, static_cast<int>(std::ceil(1.25 * left)) + 1));
        };
        for (int slot = 0;; slot ^= 1) {
            const bool near_end = need() <= len[slot];
            int n = 0;
            if (!near_end) {
                n = launch_chunk(next_len(len[slot]));
                if (n) {
                    len[slot ^ 1] = n;
                    post(slot ^ 1);
                }
            }
            SPMVC_HIP(hipEventSynchronize(ev[slot]));
            const CgScal &h = pin->h[1 + slot];
            if (h.done) {
                out = h;
                return true;
            }
            rel_prev = rel_last;
            it_prev = it_last;
            rel_last = h.rel;
            it_last = h.iters;
            tol = h.rtol;
            if (near_end) {
                n = launch_chunk(next_len(0));
                if (n) {
                    len[slot ^ 1] = n;
                    post(slot ^ 1);
                }
            }
            if (!n) return false;
        }
    }
};
static_assert(sizeof(CgScal) <= Solver::kSolverScalBytes, "scalar block of the solver region");

// CG iterations it0, it0 + 1, ... on the state in (z, r, p) until the solve
// stops or max_iter; returns the final scalars.
template <class Real>
CgScal cg_iterate(const spmvc_matrix_s *M, Solver &sv, Real *z, Real *r, Real *p, Real *q, int it0, int max_iter,
                  int check_every, int first = 0) {
    const int64_t n = M->n_rows;
    const unsigned g = rgrid(n);
    const int dt = std::is_same<Real, double>::value ? SPMVC_F64 : SPMVC_F32;
    constexpr int VW = pack_width<Real>();
    const bool vec_u = aligned16(r, q), vec_p = aligned16(z, r, p);
    const int chunk = std::max(1, check_every);
    int it = it0;
    auto chunk_fn = [&](int want) -> int {
        int j = 0;
        for (; j < want && it < max_iter; ++j, ++it) {
            const int par = it & 1;
            const unsigned ns = launch_spmv_dot(M, dt, p, q, sv.s, &sv.st()->done, sv.psig);
            if (vec_u)
                k_cg_update<Real, VW><<<g, kRT, 0, sv.s>>>(n, r, q, sv.psig, static_cast<int>(ns),
                                                           sv.pb, sv.st(), par, it);
            else
                k_cg_update<Real, 1><<<g, kRT, 0, sv.s>>>(n, r, q, sv.psig, static_cast<int>(ns),
                                                          sv.pb, sv.st(), par, it);
            if (vec_p)
                k_cg_pupdate<Real, VW><<<g, kRT, 0, sv.s>>>(n, z, r, p, sv.pb, static_cast<int>(g),
                                                            sv.st(), par, it);
            else
                k_cg_pupdate<Real, 1><<<g, kRT, 0, sv.s>>>(n, z, r, p, sv.pb, static_cast<int>(g),
                                                           sv.st(), par, it);
        }
        SPMVC_CHECK_LAUNCH();
        return j;
    };
    CgScal out;
    if (!sv.iterate_chunks(chunk, chunk_fn, out, first)) out = sv.read();
    if (!out.done) {
        out.done = 1;
        out.status = SPMVC_ENOCONV;
    }
    return out;
}

// Runs CG on A z = rhs / rhs_norm (z overwritten) with vectors of type Real;
// returns the final scalars.
template <class Real, class RhsT>
CgScal run_cg(const spmvc_matrix_s *M, Solver &sv, const RhsT *rhs, RhsT rhs_norm, Real *z, Real *r, Real *p,
              Real *q, double rtol, int max_iter, int check_every) {
    const int64_t n = M->n_rows;
    const unsigned g = rgrid(n);
    k_cg_start<Real, RhsT><<<g, kRT, 0, sv.s>>>(n, rhs, rhs_norm, z, r, p, sv.pa);
    k_cg_start_fin<<<1, kRT, 0, sv.s>>>(sv.pa, static_cast<int>(g), sv.st(), rtol, max_iter);
    SPMVC_CHECK_LAUNCH();
    // a loose tolerance (the last refinement steps) is met in a few
    // iterations: start with short chunks rather than queue two full ones
    return cg_iterate<Real>(M, sv, z, r, p, q, 0, max_iter, check_every, rtol >= 0.1 ? 2 : 0);
}

// Queues ||b - A x||^2 -> aux[0] and ||b||^2 -> aux[1] in FP64 (tmp: n
// doubles; r receives b - Ax when not null).
void residual_enqueue(const spmvc_matrix_s *M, Solver &sv, const double *b, const double *x, double *tmp,
                      double *r) {
    const int64_t n = M->n_rows;
    const unsigned g = rgrid(n);
    launch_spmv(M, SPMVC_F64, x, tmp, sv.s);
    k_residual<<<g, kRT, 0, sv.s>>>(n, b, tmp, r, sv.pa, sv.pb);
    k_residual_fin<<<1, kRT, 0, sv.s>>>(sv.pa, sv.pb, static_cast<int>(g), sv.st());
    SPMVC_CHECK_LAUNCH();
}

// ||b - A x||^2 and ||b||^2 in FP64, read back
void residual(const spmvc_matrix_s *M, Solver &sv, const double *b, const double *x, double *tmp, double *r,
              double &rr, double &bb) {
    residual_enqueue(M, sv, b, x, tmp, r);
    const CgScal &h = sv.read();
    rr = h.aux[0];
    bb = h.aux[1];
}

double ratio(double rr, double bb) { return bb > 0.0 ? std::sqrt(rr) / std::sqrt(bb) : std::sqrt(rr); }

// A solve that stopped on its recursive residual is accepted only when its
// true FP64 residual ||b - A x|| / ||b|| meets the tolerance too; otherwise it
// restarts from the true residual (at most this many times) and, if still
// short when it stops again, reports SPMVC_ENOCONV.
constexpr int kMaxRestarts = 4;

// FP64 CG on A x = b with the solver state sv and work vectors r, p, q (n each).
spmvc_status solve_fp64_in(const spmvc_matrix_s *M, Solver &sv, const double *b, double *x, double *pr, double *pp,
                           double *pq, const spmvc_cg_opts &o, spmvc_cg_stat &stat) {
    const int64_t n = M->n_rows;
    const hipStream_t s = sv.s;
    CgScal h = run_cg<double, double>(M, sv, b, 1.0, x, pr, pp, pq, o.rtol, o.max_iter, o.check_every);
    double rr = 0.0, bb = 0.0;
    residual(M, sv, b, x, pq, pr, rr, bb);  // r = b - A x
    for (int k = 0; k < kMaxRestarts && h.status == SPMVC_OK && ratio(rr, bb) > o.rtol && h.iters < o.max_iter;
         ++k) {
        k_cg_resume<<<rgrid(n), kRT, 0, s>>>(n, pr, pp, sv.st(), rr, h.iters);
        SPMVC_CHECK_LAUNCH();
        h = cg_iterate<double>(M, sv, x, pr, pp, pq, h.iters, o.max_iter, o.check_every);
        residual(M, sv, b, x, pq, pr, rr, bb);
    }
    if (h.status == SPMVC_OK && ratio(rr, bb) > o.rtol) h.status = SPMVC_ENOCONV;
    stat.iters = h.iters;
    stat.outer_iters = 0;
    stat.status = h.status;
    stat.relres_recursive = h.rel;
    stat.relres_true = ratio(rr, bb);
    return static_cast<spmvc_status>(h.status);
}

spmvc_status solve_fp64(const spmvc_matrix_s *M, const double *b, double *x, const spmvc_cg_opts &o,
                        spmvc_cg_stat &stat, hipStream_t s) {
    const int64_t n = M->n_rows;
    Solver sv(s, spmv_dot_blocks(M));
    DevBuf r, p, q;
    r.alloc(sizeof(double) * std::max<int64_t>(n, 1));
    p.alloc(sizeof(double) * std::max<int64_t>(n, 1));
    q.alloc(sizeof(double) * std::max<int64_t>(n, 1));
    return solve_fp64_in(M, sv, b, x, r.as<double>(), p.as<double>(), q.as<double>(), o, stat);
}

// ---- the same FP64 CG without any allocation ----------------------------------------------
// For callers that cannot allocate device memory: every buffer of the solve
// lives in `scratch`, one fixed region per GPU that holds the solver scalars,
// the reduction partials and the vectors r, p, q.  Host code reaches it only
// through the address hipGetSymbolAddress gives on each device.
constexpr int64_t kNaMaxRows = int64_t(1) << 21;       // rows of the largest system (2,097,152)
constexpr int64_t kNaMaxSpmvBlocks = int64_t(1) << 16;  // p.q partials of one SpMV launch
constexpr size_t kNaSolverBytes = Solver::kSolverScalBytes + sizeof(double) * (2 * kRMaxBlocks + kNaMaxSpmvBlocks);
constexpr size_t kNaVecBytes = sizeof(double) * kNaMaxRows;
constexpr size_t kNaScratchBytes = kNaSolverBytes + 3 * kNaVecBytes;  // 48.5 MiB
static_assert(kNaSolverBytes % 256 == 0, "vectors start 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kNaScratchBytes];

constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;
char *g_na_ptr[kNaMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
char *scratch_on_current_device() {
    int dev = 0;
    SPMVC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNaMaxDevices) throw Error{SPMVC_EUNSUPPORTED, "device index beyond 63"};
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[dev]) {
        void *ptr = nullptr;
        SPMVC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_na_ptr[dev] = static_cast<char *>(ptr);
    }
    return g_na_ptr[dev];
}

}  // namespace

int64_t cg_noalloc_max_rows() { return kNaMaxRows; }

spmvc_status cg_solve_noalloc_impl(const spmvc_matrix_s *M, const double *b, double *x, const spmvc_cg_opts &o,
                                   spmvc_cg_stat &stat, hipStream_t s) {
    const int64_t n = M->n_rows;
    if (n > kNaMaxRows)
        throw Error{SPMVC_EINVAL, "cg_solve_noalloc: " + std::to_string(n) + " rows exceed the scratch limit of " +
                                      std::to_string(kNaMaxRows)};
    if (spmv_dot_blocks(M) > kNaMaxSpmvBlocks)
        throw Error{SPMVC_EINVAL, "cg_solve_noalloc: the SpMV configuration launches more than " +
                                      std::to_string(kNaMaxSpmvBlocks) + " blocks"};
    char *base = scratch_on_current_device();
    Solver sv(s, base);
    double *r = reinterpret_cast<double *>(base + kNaSolverBytes);
    double *p = reinterpret_cast<double *>(base + kNaSolverBytes + kNaVecBytes);
    double *q = reinterpret_cast<double *>(base + kNaSolverBytes + 2 * kNaVecBytes);
    const spmvc_status st = solve_fp64_in(M, sv, b, x, r, p, q, o, stat);
    SPMVC_HIP(hipStreamSynchronize(s));
    return st;
}

namespace {

// Preconditioned CG (mode 2): M^-1 r = one multicolor SymGS sweep from zero.
// prec(r, z, st, done) enqueues z = M^-1 r on s; every launch it makes
// returns at once once st->done is set.
template <class Prec>
spmvc_status solve_pcg(spmvc_matrix_s *M, const double *b, double *x, const spmvc_cg_opts &o, spmvc_cg_stat &stat,
                       hipStream_t s, Prec &&prec) {
    const int64_t n = M->n_rows;
    const int64_t nn = std::max<int64_t>(n, 1);
    Solver sv(s, spmv_dot_blocks(M));
    DevBuf r, z, p, q;
    r.alloc(sizeof(double) * nn);
    z.alloc(sizeof(double) * nn);
    p.alloc(sizeof(double) * nn);
    q.alloc(sizeof(double) * nn);
    const unsigned g = rgrid(n);
    double *pr = r.as<double>(), *pz = z.as<double>(), *pp = p.as<double>(), *pq = q.as<double>();
    const int *done = &sv.st()->done;
    // x = 0, r = b, rho0 = b.b; z = M^-1 r; p = z; rho = r.z
    k_cg_start<double, double><<<g, kRT, 0, s>>>(n, b, 1.0, x, pr, pp, sv.pa);
    k_cg_start_fin<<<1, kRT, 0, s>>>(sv.pa, static_cast<int>(g), sv.st(), o.rtol, o.max_iter);
    SPMVC_CHECK_LAUNCH();
    // z = M^-1 r, p = z, rho[it & 1] = r.z; then iterations it, it + 1, ... until the solve stops
    auto iterate = [&](int it) {
        prec(pr, pz, sv.st(), done);
        k_pcg_init<<<g, kRT, 0, s>>>(n, pr, pz, pp, sv.pa);
        k_pcg_init_fin<<<1, kRT, 0, s>>>(sv.pa, static_cast<int>(g), sv.st(), it & 1);
        SPMVC_CHECK_LAUNCH();
        // a preconditioned iteration is a sweep or a V-cycle, dozens of launches
        // and several plain iterations' time: the status is read four times as
        // often, which bounds the no-op iterations queued past convergence at
        // little cost (a read is one small copy)
        const int chunk = std::max(1, o.check_every / 4);
        auto chunk_fn = [&](int want) -> int {
            int j = 0;
            for (; j < want && it < o.max_iter; ++j, ++it) {
                const int par = it & 1;
                const unsigned ns = launch_spmv_dot(M, SPMVC_F64, pp, pq, s, done, sv.psig);
                k_pcg_update<<<g, kRT, 0, s>>>(n, x, pr, pp, pq, sv.psig, static_cast<int>(ns),
                                               sv.pb, sv.st(), par, it);
                prec(pr, pz, sv.st(), done);
                k_pcg_rz<<<g, kRT, 0, s>>>(n, pr, pz, sv.pb, static_cast<int>(g),
                                           sv.pa, sv.st(), par, it);
                k_pcg_p<<<g, kRT, 0, s>>>(n, pz, pp, sv.pa, static_cast<int>(g), sv.st(), par);
            }
            SPMVC_CHECK_LAUNCH();
            return j;
        };
        CgScal h;
        if (!sv.iterate_chunks(chunk, chunk_fn, h)) h = sv.read();
        if (!h.done) {
            h.done = 1;
            h.status = SPMVC_ENOCONV;
        }
        return h;
    };
    CgScal h = iterate(0);
    double rr = 0.0, bb = 0.0;
    residual(M, sv, b, x, pq, pr, rr, bb);  // r = b - A x
    for (int k = 0; k < kMaxRestarts && h.status == SPMVC_OK && ratio(rr, bb) > o.rtol && h.iters < o.max_iter;
         ++k) {
        k_pcg_resume<<<1, 64, 0, s>>>(sv.st(), rr);
        h = iterate(h.iters);
        residual(M, sv, b, x, pq, pr, rr, bb);
    }
    if (h.status == SPMVC_OK && ratio(rr, bb) > o.rtol) h.status = SPMVC_ENOCONV;
    stat.iters = h.iters;
    stat.outer_iters = 0;
    stat.status = h.status;
    stat.relres_recursive = h.rel;
    stat.relres_true = ratio(rr, bb);
    return static_cast<spmvc_status>(h.status);
}

// ---- multigrid V-cycle as M^-1 -------------------------------------------------------
// One V-cycle per iteration, in the order of Table I: on each level above the
// coarsest z = 0, SymGS, t = A z, restriction r_c = (r - t)[f2c], the next
// level, prolongation z[f2c] += z_c, SymGS; on the coarsest z = 0 and SymGS.
// The smoother visits the colors backward, then forward: the rows a sweep
// updates last keep zero residual, and in the forward order those are color
// 0, which on a grid hierarchy holds the injection points (the coarse levels
// would receive a zero residual).

// r_c[i] = r[f2c[i]] - t[f2c[i]]
__global__ __launch_bounds__(kRT) void k_mg_restrict(int64_t nc, const int32_t *__restrict__ f2c,
                                                     const double *__restrict__ r, const double *__restrict__ t,
                                                     double *__restrict__ rc, const CgScal *st) {
    if (st->done) return;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kRT) + threadIdx.x; i < nc;
         i += static_cast<int64_t>(gridDim.x) * kRT) {
        const int64_t j = f2c[i];
        rc[i] = r[j] - t[j];
    }
}

// z[f2c[i]] += z_c[i]  (f2c is injective, checked at set-up)
__global__ __launch_bounds__(kRT) void k_mg_prolong(int64_t nc, const int32_t *__restrict__ f2c,
                                                    const double *__restrict__ zc, double *__restrict__ z,
                                                    const CgScal *st) {
    if (st->done) return;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kRT) + threadIdx.x; i < nc;
         i += static_cast<int64_t>(gridDim.x) * kRT)
        z[f2c[i]] += zc[i];
}

// bad = 1 unless every f2c entry lies in [0, nf) and none repeats (hits: nf zeros)
__global__ __launch_bounds__(kRT) void k_mg_check(int64_t nc, const int32_t *__restrict__ f2c, int64_t nf,
                                                  int *hits, int *bad) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kRT) + threadIdx.x; i < nc;
         i += static_cast<int64_t>(gridDim.x) * kRT) {
        const int64_t j = f2c[i];
        if (j < 0 || j >= nf || atomicAdd(&hits[j], 1) != 0) atomicOr(bad, 1);
    }
}

struct MgLevel {
    spmvc_matrix_s *A = nullptr;
    const int32_t *f2c = nullptr;  // this level's rows -> rows of the level above (levels >= 1)
    DevBuf r, z;                   // right-hand side and correction (levels >= 1)
    DevBuf t;                      // A z (every level but the coarsest)
};

void vcycle(std::vector<MgLevel> &L, size_t l, const double *r, double *z, const CgScal *st, const int *done,
            hipStream_t s) {
    spmvc_matrix_s *A = L[l].A;
    const int64_t n = A->n_rows;
    k_pcg_zero<<<rgrid(n), kRT, 0, s>>>(n, z, st);
    SPMVC_CHECK_LAUNCH();
    launch_symgs(A, r, z, 1, s, done, true);
    if (l + 1 == L.size()) return;
    MgLevel &c = L[l + 1];
    const int64_t nc = c.A->n_rows;
    double *t = L[l].t.as<double>();
    launch_spmv(A, SPMVC_F64, z, t, s, done);
    k_mg_restrict<<<rgrid(nc), kRT, 0, s>>>(nc, c.f2c, r, t, c.r.as<double>(), st);
    SPMVC_CHECK_LAUNCH();
    vcycle(L, l + 1, c.r.as<double>(), c.z.as<double>(), st, done, s);
    k_mg_prolong<<<rgrid(nc), kRT, 0, s>>>(nc, c.f2c, c.z.as<double>(), z, st);
    SPMVC_CHECK_LAUNCH();
    launch_symgs(A, r, z, 1, s, done, true);
}

// Mixed precision: FP64 residual / update outside, FP32-SpMV CG inside.  The
// inner tolerance is inner_rtol, loosened for the last step to what the outer
// tolerance still needs (0.9 rtol ||b|| / ||r||), so no step over-solves.
spmvc_status solve_mixed(const spmvc_matrix_s *M, const double *b, double *x, const spmvc_cg_opts &o,
                         spmvc_cg_stat &stat, hipStream_t s) {
    const int64_t n = M->n_rows;
    const int64_t nn = std::max<int64_t>(n, 1);
    Solver sv(s, spmv_dot_blocks(M));
    DevBuf r64, q64, r32, p32, q32, d32;
    r64.alloc(sizeof(double) * nn);
    q64.alloc(sizeof(double) * nn);
    r32.alloc(sizeof(float) * nn);
    p32.alloc(sizeof(float) * nn);
    q32.alloc(sizeof(float) * nn);
    d32.alloc(sizeof(float) * nn);
    SPMVC_HIP(hipMemsetAsync(x, 0, sizeof(double) * nn, s));
    int inner_total = 0, outer = 0;
    spmvc_status st = SPMVC_ENOCONV;
    double rel = 1.0;
    while (outer <= o.max_outer) {
        double rr, bb;
        residual(M, sv, b, x, q64.as<double>(), r64.as<double>(), rr, bb);
        const double bnorm = std::sqrt(bb);
        if (bnorm == 0.0) {
            rel = 0.0;
            st = SPMVC_OK;
            break;
        }
        rel = std::sqrt(rr) / bnorm;
        if (rel <= o.rtol) {
            st = SPMVC_OK;
            break;
        }
        if (outer == o.max_outer || inner_total >= o.max_iter) break;
        ++outer;
        const double inner_tol = std::max(o.inner_rtol, 0.9 * o.rtol / rel);
        // the FP32 solve takes r / ||r|| (unit norm: no FP32 underflow or
        // overflow whatever the scale of b) and x advances by ||r|| d
        const double rnorm = std::sqrt(rr);
        const CgScal h = run_cg<float, double>(M, sv, r64.as<double>(), rnorm, d32.as<float>(), r32.as<float>(),
                                               p32.as<float>(), q32.as<float>(), std::min(inner_tol, 0.5),
                                               std::max(1, o.max_iter - inner_total), o.check_every);
        inner_total += h.iters;
        if (h.status == SPMVC_ENOTSPD || h.status == SPMVC_EINVAL) {
            st = static_cast<spmvc_status>(h.status);
            break;
        }
        k_add_f32<<<rgrid(n), kRT, 0, s>>>(n, x, d32.as<float>(), rnorm);
        SPMVC_CHECK_LAUNCH();
    }
    // every exit follows the residual of the current x (or leaves x as it
    // was then), so rel is already its true FP64 residual
    stat.iters = inner_total;
    stat.outer_iters = outer;
    stat.status = st;
    stat.relres_recursive = rel;
    stat.relres_true = rel;
    return st;
}

// Mixed precision with reliable updates (mode 3): one CG whose iterations
// all run in FP32 (SpMV over the FP32 shadow, FP32 vectors, FP64 dot
// products), with the FP64 residual put back in place of the recursive one
// whenever the latter has fallen by inner_rtol since the last replacement.  A
// segment solves A d = r / ||r|| in FP32 from d = 0; at its end x += ||r|| d in
// FP64, r = b - A x is recomputed in FP64, and the next segment starts from
// that residual but keeps the search direction p (rescaled to the new units,
// with beta = ||r_new||^2 / ||r_k||^2), so the Krylov space is not thrown away
// as at a refinement restart.  Stops when the true FP64 residual meets rtol.
// Between segments the scale, beta, the tolerance and the stopping tests are
// computed on the device (k_rel_next): the host reads the scalars once per
// segment, when the chunk reads show it done, and then queues the replacement
// and the next segment at once; the replacement's outcome is read on its own
// only after a segment that most likely reached the target, so that no
// iterations are queued past the stop.
spmvc_status solve_reliable(const spmvc_matrix_s *M, const double *b, double *x, const spmvc_cg_opts &o,
                            spmvc_cg_stat &stat, hipStream_t s) {
    const int64_t n = M->n_rows;
    const int64_t nn = std::max<int64_t>(n, 1);
    const unsigned g = rgrid(n);
    Solver sv(s, spmv_dot_blocks(M));
    DevBuf r64, q64, r32, p32, q32, xl32, rsb;
    r64.alloc(sizeof(double) * nn);
    q64.alloc(sizeof(double) * nn);
    r32.alloc(sizeof(float) * nn);
    p32.alloc(sizeof(float) * nn);
    q32.alloc(sizeof(float) * nn);
    xl32.alloc(sizeof(float) * nn);
    rsb.alloc(sizeof(RelState));
    RelState *rs = rsb.as<RelState>();
    SPMVC_HIP(hipMemsetAsync(x, 0, sizeof(double) * nn, s));
    double rr, bb;
    residual(M, sv, b, x, q64.as<double>(), r64.as<double>(), rr, bb);
    const double bnorm = std::sqrt(bb);
    int total = 0, segs = 0;
    if (!std::isfinite(bb) || !std::isfinite(rr)) {  // NaN or Inf in b
        stat = spmvc_cg_stat{};
        stat.status = SPMVC_EINVAL;
        stat.relres_true = stat.relres_recursive = std::numeric_limits<double>::quiet_NaN();
        return SPMVC_EINVAL;
    }
    double rel = bnorm > 0.0 ? std::sqrt(rr) / bnorm : 0.0, rel_rec = rel;
    spmvc_status st = SPMVC_ENOCONV;
    auto rel_status = [](double fin) {
        const int f = static_cast<int>(fin);
        return f == kRelOk ? SPMVC_OK : f == kRelBreakdown ? SPMVC_ENOTSPD : SPMVC_ENOCONV;
    };
    if (rel <= o.rtol) {
        st = SPMVC_OK;
    } else if (o.max_outer >= 0 && o.max_iter > 0) {
        k_rel_first<<<1, 64, 0, s>>>(rs, std::sqrt(rr), std::min(std::max(o.inner_rtol, 0.9 * o.rtol / rel), 0.5),
                                     bnorm);
        while (true) {
            k_rel_start<<<g, kRT, 0, s>>>(n, r64.as<double>(), rs, xl32.as<float>(), r32.as<float>(),
                                          p32.as<float>(), sv.pa);
            k_rel_start_fin<<<1, kRT, 0, s>>>(sv.pa, static_cast<int>(g), sv.st(), rs, o.max_iter - total);
            SPMVC_CHECK_LAUNCH();
            const CgScal h = cg_iterate<float>(M, sv, xl32.as<float>(), r32.as<float>(), p32.as<float>(),
                                               q32.as<float>(), 0, o.max_iter - total, o.check_every);
            if (segs > 0) {  // the values k_rel_next left after the last replacement
                rel = std::sqrt(h.aux[0]) / bnorm;
                rel_rec = h.aux[3];
            }
            if (h.aux[2] != 0.0) {  // k_rel_next stopped the solve; h still holds the last segment's scalars
                st = rel_status(h.aux[2]);
                break;
            }
            total += h.iters;
            ++segs;
            if (h.status == SPMVC_ENOTSPD || h.status == SPMVC_EINVAL) {
                st = static_cast<spmvc_status>(h.status);
                break;
            }
            k_add_rel<<<rgrid(n), kRT, 0, s>>>(n, x, xl32.as<float>(), rs);
            SPMVC_CHECK_LAUNCH();
            residual_enqueue(M, sv, b, x, q64.as<double>(), r64.as<double>());
            const double rho_k = h.iters > 0 ? h.rho[(h.iters - 1) & 1] : 0.0;
            k_rel_next<<<1, 64, 0, s>>>(sv.st(), rs, o.rtol, o.inner_rtol, segs, total, o.max_outer, o.max_iter,
                                        rho_k);
            SPMVC_CHECK_LAUNCH();
            // when the segment's recursive residual, times the true one at its
            // start (rel), comes within twice rtol, this is most likely the last
            // segment: read k_rel_next's decision now rather than queue
            // iterations that would run as no-ops
            if (rel * h.rel <= 2.0 * o.rtol) {
                const CgScal &c = sv.read();
                if (c.aux[2] != 0.0) {
                    rel = std::sqrt(c.aux[0]) / bnorm;
                    rel_rec = c.aux[3];
                    st = rel_status(c.aux[2]);
                    break;
                }
            }
        }
    }
    stat.iters = total;
    stat.outer_iters = segs;
    stat.status = st;
    stat.relres_recursive = rel_rec;
    stat.relres_true = rel;
    return st;
}

}  // namespace

spmvc_status cg_solve_mg_impl(spmvc_matrix const *levels, const int32_t *const *f2c, int n_levels, const double *b,
                              double *x, const spmvc_cg_opts &o, spmvc_cg_stat *stat, hipStream_t s) {
    std::vector<MgLevel> L(n_levels);
    for (int l = 0; l < n_levels; ++l) {
        L[l].A = const_cast<spmvc_matrix_s *>(levels[l]);
        build_coloring(L[l].A, s);  // throws for a missing or zero diagonal
    }
    {  // every injection map in range and injective
        DevBuf flag;
        flag.alloc(sizeof(int));
        SPMVC_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), s));
        for (int l = 1; l < n_levels; ++l) {
            const int64_t nf = L[l - 1].A->n_rows, nc = L[l].A->n_rows;
            DevBuf hits;
            hits.alloc(sizeof(int) * nf);
            SPMVC_HIP(hipMemsetAsync(hits.p, 0, sizeof(int) * nf, s));
            k_mg_check<<<rgrid(nc), kRT, 0, s>>>(nc, f2c[l - 1], nf, hits.as<int>(), flag.as<int>());
            SPMVC_CHECK_LAUNCH();
            SPMVC_HIP(hipStreamSynchronize(s));  // before hits is released
        }
        int bad = 0;
        SPMVC_HIP(hipMemcpyAsync(&bad, flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
        SPMVC_HIP(hipStreamSynchronize(s));
        if (bad) throw Error{SPMVC_EINVAL, "f2c entry out of range or repeated"};
    }
    for (int l = 0; l < n_levels; ++l) {
        const size_t bytes = sizeof(double) * L[l].A->n_rows;
        if (l > 0) {
            L[l].f2c = f2c[l - 1];
            L[l].r.alloc(bytes);
            L[l].z.alloc(bytes);
        }
        if (l + 1 < n_levels) L[l].t.alloc(bytes);
    }
    const spmvc_status st = solve_pcg(L[0].A, b, x, o, stat[0], s, [&](const double *r, double *z, const CgScal *sc,
                                                                       const int *done) { vcycle(L, 0, r, z, sc, done, s); });
    SPMVC_HIP(hipStreamSynchronize(s));
    return st;
}

spmvc_status cg_solve_impl(const spmvc_matrix *A, int n_sys, int nrhs, const double *const *b, double *const *x,
                           const spmvc_cg_opts &o, spmvc_cg_stat *stat, hipStream_t s) {
    spmvc_status first_bad = SPMVC_OK;
    if (o.mode == 1) {
        const spmvc_status st = solve_mixed(A[0], b[0], x[0], o, stat[0], s);
        SPMVC_HIP(hipStreamSynchronize(s));
        return st;
    }
    if (o.mode == 3) {
        const spmvc_status st = solve_reliable(A[0], b[0], x[0], o, stat[0], s);
        SPMVC_HIP(hipStreamSynchronize(s));
        return st;
    }
    if (o.mode == 2) {
        spmvc_matrix_s *M = const_cast<spmvc_matrix_s *>(A[0]);
        build_coloring(M, s);  // throws for a missing or zero diagonal
        const int64_t n = M->n_rows;
        const spmvc_status st =
            solve_pcg(M, b[0], x[0], o, stat[0], s, [&](const double *r, double *z, const CgScal *sc, const int *done) {
                k_pcg_zero<<<rgrid(n), kRT, 0, s>>>(n, z, sc);
                SPMVC_CHECK_LAUNCH();
                launch_symgs(M, r, z, 1, s, done);
            });
        SPMVC_HIP(hipStreamSynchronize(s));
        return st;
    }
    if ((n_sys > 1 || nrhs > 1) && o.batched != 0) {
        if (batched_supported(A, n_sys)) {
            const spmvc_status st = cg_solve_batched(A, n_sys, nrhs, b, x, o, stat, s, o.batched != 1);
            SPMVC_HIP(hipStreamSynchronize(s));
            return st;
        }
        batched_note_fallback();  // reported by spmvc_batched_config (form -2)
    }
    for (int sy = 0; sy < n_sys; ++sy) {
        const spmvc_matrix_s *M = A[sy];
        const int64_t n = M->n_rows;
        if (nrhs == 1) {
            const spmvc_status st = solve_fp64(M, b[sy], x[sy], o, stat[sy], s);
            if (st != SPMVC_OK && first_bad == SPMVC_OK) first_bad = st;
            continue;
        }
        DevBuf bv, xv;
        bv.alloc(sizeof(double) * std::max<int64_t>(n, 1));
        xv.alloc(sizeof(double) * std::max<int64_t>(n, 1));
        for (int r = 0; r < nrhs; ++r) {
            k_gather_col<<<rgrid(n), kRT, 0, s>>>(n, b[sy], nrhs, r, bv.as<double>());
            SPMVC_CHECK_LAUNCH();
            const spmvc_status st = solve_fp64(M, bv.as<double>(), xv.as<double>(), o, stat[sy * nrhs + r], s);
            k_scatter_col<<<rgrid(n), kRT, 0, s>>>(n, xv.as<double>(), x[sy], nrhs, r);
            SPMVC_CHECK_LAUNCH();
            if (st != SPMVC_OK && first_bad == SPMVC_OK) first_bad = st;
        }
    }
    SPMVC_HIP(hipStreamSynchronize(s));
    return first_bad;
}

}  // namespace spmvc
