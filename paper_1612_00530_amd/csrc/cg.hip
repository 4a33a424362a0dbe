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
// Reductions: every block reduces its elements in a fixed order (wavefront
// butterfly through lane permutes, then the waves in index order), writes one
// partial, and the last block to finish -- found with an acquire-release
// ticket -- adds the partials in index order.  The result does not depend on
// block scheduling, so iteration counts repeat exactly from run to run.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace spmvc {
namespace {

constexpr int kRT = 256;         // threads per reduction block
constexpr unsigned kRMaxBlocks = 2048;

struct CgScal {
    double rho, rho0, sigma, alpha, beta, rel, rtol, pad0;
    int32_t iters, max_iter, done, status;
    uint32_t ticket[4];
    double aux[4]; // aux[0]: result of standalone reductions
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the block; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kRT / 64; ++i) s += sh[i];
    __syncthreads();
    return s;
}

__device__ __forceinline__ double load_agent(const double *p) {
    const uint64_t b = __hip_atomic_load(reinterpret_cast<const uint64_t *>(p), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double(static_cast<long long>(b));
}

// Grid reduction; returns true in thread 0 of the last block, with *out = the sum.
__device__ bool grid_sum(double v, double *partials, uint32_t *ticket, double *out) {
    __shared__ double sh[kRT / 64];
    __shared__ int last;
    const double b = block_sum(v, sh);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = b;
        __threadfence();
        const uint32_t t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
    double s = 0.0;
    for (unsigned i = threadIdx.x; i < gridDim.x; i += kRT) s += load_agent(&partials[i]);
    const double tot = block_sum(s, sh);
    if (threadIdx.x == 0) {
        __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *out = tot;
        return true;
    }
    return false;
}

template <class Real> __device__ __forceinline__ double dd(Real v) { return static_cast<double>(v); }

// x = 0, r = rhs, p = rhs, rho = rho0 = r.r
template <class Real, class RhsT>
__global__ __launch_bounds__(kRT) void k_cg_start(int64_t n, const RhsT *__restrict__ rhs, Real *__restrict__ x,
                                                  Real *__restrict__ r, Real *__restrict__ p, double *partials,
                                                  CgScal *st, double rtol, int max_iter) {
    double acc = 0.0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kRT;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kRT + threadIdx.x; i < n; i += stride) {
        const Real v = static_cast<Real>(rhs[i]);
        x[i] = Real(0);
        r[i] = v;
        p[i] = v;
        acc += dd(v) * dd(v);
    }
    double tot;
    if (grid_sum(acc, partials, &st->ticket[0], &tot)) {
        st->rho = tot;
        st->rho0 = tot;
        st->rtol = rtol;
        st->iters = 0;
        st->max_iter = max_iter;
        st->rel = tot > 0.0 ? 1.0 : 0.0;
        st->done = (tot == 0.0) ? 1 : 0;
        st->status = SPMVC_OK;
        if (tot == 0.0) st->rel = 0.0;
        if (!(tot == tot) || tot > 1.7e308) {
            st->done = 1;
            st->status = SPMVC_EINVAL;
        }
    }
}

// sigma = p.q, alpha = rho / sigma (breakdown when sigma <= 0 or not finite)
template <class Real>
__global__ __launch_bounds__(kRT) void k_cg_alpha(int64_t n, const Real *__restrict__ p, const Real *__restrict__ q,
                                                  double *partials, CgScal *st) {
    if (st->done) return;
    double acc = 0.0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kRT;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kRT + threadIdx.x; i < n; i += stride)
        acc += dd(p[i]) * dd(q[i]);
    double sigma;
    if (grid_sum(acc, partials, &st->ticket[1], &sigma)) {
        st->sigma = sigma;
        if (!(sigma > 0.0) || !isfinite(sigma)) {
            st->done = 1;
            st->status = SPMVC_ENOTSPD;
            st->iters += 1;
        } else {
            st->alpha = st->rho / sigma;
        }
    }
}

// x += alpha p; r -= alpha q; rho' = r.r; convergence test; beta
template <class Real>
__global__ __launch_bounds__(kRT) void k_cg_update(int64_t n, Real *__restrict__ x, Real *__restrict__ r,
                                                   const Real *__restrict__ p, const Real *__restrict__ q,
                                                   double *partials, CgScal *st) {
    if (st->done) return;
    const Real alpha = static_cast<Real>(st->alpha);
    double acc = 0.0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kRT;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kRT + threadIdx.x; i < n; i += stride) {
        x[i] = x[i] + alpha * p[i];
        const Real ri = r[i] - alpha * q[i];
        r[i] = ri;
        acc += dd(ri) * dd(ri);
    }
    double rho_new;
    if (grid_sum(acc, partials, &st->ticket[2], &rho_new)) {
        st->iters += 1;
        st->rel = sqrt(rho_new) / sqrt(st->rho0);
        if (sqrt(rho_new) <= st->rtol * sqrt(st->rho0)) {
            st->done = 1;
            st->status = SPMVC_OK;
        } else if (st->iters >= st->max_iter) {
            st->done = 1;
            st->status = SPMVC_ENOCONV;
        } else if (!isfinite(rho_new)) {
            st->done = 1;
            st->status = SPMVC_ENOTSPD;
        }
        st->beta = rho_new / st->rho;
        st->rho = rho_new;
    }
}

// p = r + beta p
template <class Real>
__global__ __launch_bounds__(kRT) void k_cg_pupdate(int64_t n, const Real *__restrict__ r, Real *__restrict__ p,
                                                    const CgScal *st) {
    if (st->done) return;
    const Real beta = static_cast<Real>(st->beta);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kRT;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kRT + threadIdx.x; i < n; i += stride)
        p[i] = r[i] + beta * p[i];
}

// r = b - Ax (FP64) and aux[0] = r.r
__global__ __launch_bounds__(kRT) void k_residual(int64_t n, const double *__restrict__ b,
                                                  const double *__restrict__ ax, double *__restrict__ r,
                                                  double *partials, CgScal *st) {
    double acc = 0.0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kRT;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kRT + threadIdx.x; i < n; i += stride) {
        const double v = b[i] - ax[i];
        if (r) r[i] = v;
        acc += v * v;
    }
    double tot;
    if (grid_sum(acc, partials, &st->ticket[3], &tot)) st->aux[0] = tot;
}

// aux[1] = b.b
__global__ __launch_bounds__(kRT) void k_norm2(int64_t n, const double *__restrict__ b, double *partials,
                                               CgScal *st) {
    double acc = 0.0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kRT;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kRT + threadIdx.x; i < n; i += stride) acc += b[i] * b[i];
    double tot;
    if (grid_sum(acc, partials, &st->ticket[3], &tot)) st->aux[1] = tot;
}

// x += (double) d
__global__ void k_add_f32(int64_t n, double *__restrict__ x, const float *__restrict__ d) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        x[i] += static_cast<double>(d[i]);
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
    int64_t g = (n + kRT * 4 - 1) / (kRT * 4);
    return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(g, kRMaxBlocks)));
}

struct Pinned {
    CgScal *h = nullptr;
    Pinned() { SPMVC_HIP(hipHostMalloc(reinterpret_cast<void **>(&h), sizeof(CgScal), hipHostMallocDefault)); }
    ~Pinned() {
        if (h) (void)hipHostFree(h);
    }
};

struct Solver {
    hipStream_t s;
    DevBuf scal, partials;
    Pinned pin;
    explicit Solver(hipStream_t st) : s(st) {
        scal.alloc(sizeof(CgScal));
        SPMVC_HIP(hipMemsetAsync(scal.p, 0, sizeof(CgScal), s));
        partials.alloc(sizeof(double) * kRMaxBlocks);
    }
    CgScal *st() { return scal.as<CgScal>(); }
    const CgScal &read() {
        SPMVC_HIP(hipMemcpyAsync(pin.h, scal.p, sizeof(CgScal), hipMemcpyDeviceToHost, s));
        SPMVC_HIP(hipStreamSynchronize(s));
        return *pin.h;
    }
};

// Runs CG on A z = rhs (z overwritten) with vectors of type Real; returns the final scalars.
template <class Real, class RhsT>
CgScal run_cg(const spmvc_matrix_s *M, Solver &sv, const RhsT *rhs, Real *z, Real *r, Real *p, Real *q, double rtol,
              int max_iter, int check_every) {
    const int64_t n = M->n_rows;
    const unsigned g = rgrid(n);
    const int dt = std::is_same<Real, double>::value ? SPMVC_F64 : SPMVC_F32;
    k_cg_start<Real, RhsT><<<g, kRT, 0, sv.s>>>(n, rhs, z, r, p, sv.partials.as<double>(), sv.st(), rtol, max_iter);
    SPMVC_CHECK_LAUNCH();
    const int chunk = std::max(1, check_every);
    const int64_t max_chunks = static_cast<int64_t>(max_iter) / chunk + 2;
    for (int64_t c = 0; c < max_chunks; ++c) {
        if (sv.read().done) break;
        for (int j = 0; j < chunk; ++j) {
            launch_spmv(M, dt, p, q, sv.s, &sv.st()->done);
            k_cg_alpha<Real><<<g, kRT, 0, sv.s>>>(n, p, q, sv.partials.as<double>(), sv.st());
            k_cg_update<Real><<<g, kRT, 0, sv.s>>>(n, z, r, p, q, sv.partials.as<double>(), sv.st());
            k_cg_pupdate<Real><<<g, kRT, 0, sv.s>>>(n, r, p, sv.st());
        }
        SPMVC_CHECK_LAUNCH();
    }
    CgScal out = sv.read();
    if (!out.done) {
        out.done = 1;
        out.status = SPMVC_ENOCONV;
    }
    return out;
}

// ||b - A x|| / ||b|| in FP64 (tmp: n doubles)
double true_relres(const spmvc_matrix_s *M, Solver &sv, const double *b, const double *x, double *tmp) {
    const int64_t n = M->n_rows;
    const unsigned g = rgrid(n);
    launch_spmv(M, SPMVC_F64, x, tmp, sv.s);
    k_residual<<<g, kRT, 0, sv.s>>>(n, b, tmp, nullptr, sv.partials.as<double>(), sv.st());
    k_norm2<<<g, kRT, 0, sv.s>>>(n, b, sv.partials.as<double>(), sv.st());
    SPMVC_CHECK_LAUNCH();
    const CgScal &h = sv.read();
    return h.aux[1] > 0.0 ? std::sqrt(h.aux[0]) / std::sqrt(h.aux[1]) : std::sqrt(h.aux[0]);
}

spmvc_status solve_fp64(const spmvc_matrix_s *M, const double *b, double *x, const spmvc_cg_opts &o,
                        spmvc_cg_stat &stat, hipStream_t s) {
    const int64_t n = M->n_rows;
    Solver sv(s);
    DevBuf r, p, q;
    r.alloc(sizeof(double) * std::max<int64_t>(n, 1));
    p.alloc(sizeof(double) * std::max<int64_t>(n, 1));
    q.alloc(sizeof(double) * std::max<int64_t>(n, 1));
    const CgScal h = run_cg<double, double>(M, sv, b, x, r.as<double>(), p.as<double>(), q.as<double>(), o.rtol,
                                            o.max_iter, o.check_every);
    stat.iters = h.iters;
    stat.outer_iters = 0;
    stat.status = h.status;
    stat.relres_recursive = h.rel;
    stat.relres_true = true_relres(M, sv, b, x, q.as<double>());
    return static_cast<spmvc_status>(h.status);
}

// Mixed precision: FP64 residual / update outside, FP32-SpMV CG inside.
spmvc_status solve_mixed(const spmvc_matrix_s *M, const double *b, double *x, const spmvc_cg_opts &o,
                         spmvc_cg_stat &stat, hipStream_t s) {
    const int64_t n = M->n_rows;
    const int64_t nn = std::max<int64_t>(n, 1);
    Solver sv(s);
    DevBuf r64, q64, r32, p32, q32, d32;
    r64.alloc(sizeof(double) * nn);
    q64.alloc(sizeof(double) * nn);
    r32.alloc(sizeof(float) * nn);
    p32.alloc(sizeof(float) * nn);
    q32.alloc(sizeof(float) * nn);
    d32.alloc(sizeof(float) * nn);
    const unsigned g = rgrid(n);
    SPMVC_HIP(hipMemsetAsync(x, 0, sizeof(double) * nn, s));
    k_norm2<<<g, kRT, 0, s>>>(n, b, sv.partials.as<double>(), sv.st());
    SPMVC_CHECK_LAUNCH();
    const double bnorm = std::sqrt(sv.read().aux[1]);
    int inner_total = 0, outer = 0;
    spmvc_status st = SPMVC_ENOCONV;
    double rel = bnorm > 0 ? 1.0 : 0.0;
    if (bnorm == 0.0) st = SPMVC_OK;
    while (st != SPMVC_OK && outer <= o.max_outer) {
        launch_spmv(M, SPMVC_F64, x, q64.p, s);
        k_residual<<<g, kRT, 0, s>>>(n, b, q64.as<double>(), r64.as<double>(), sv.partials.as<double>(), sv.st());
        SPMVC_CHECK_LAUNCH();
        rel = std::sqrt(sv.read().aux[0]) / bnorm;
        if (rel <= o.rtol) {
            st = SPMVC_OK;
            break;
        }
        if (outer == o.max_outer || inner_total >= o.max_iter) break;
        ++outer;
        const CgScal h = run_cg<float, double>(M, sv, r64.as<double>(), d32.as<float>(), r32.as<float>(),
                                               p32.as<float>(), q32.as<float>(), o.inner_rtol,
                                               std::max(1, o.max_iter - inner_total), o.check_every);
        inner_total += h.iters;
        if (h.status == SPMVC_ENOTSPD || h.status == SPMVC_EINVAL) {
            st = static_cast<spmvc_status>(h.status);
            break;
        }
        k_add_f32<<<rgrid(n), kRT, 0, s>>>(n, x, d32.as<float>());
        SPMVC_CHECK_LAUNCH();
    }
    stat.iters = inner_total;
    stat.outer_iters = outer;
    stat.status = st;
    stat.relres_recursive = rel;
    stat.relres_true = true_relres(M, sv, b, x, q64.as<double>());
    return st;
}

}  // namespace

spmvc_status cg_solve_impl(const spmvc_matrix *A, int n_sys, int nrhs, const double *const *b, double *const *x,
                           const spmvc_cg_opts &o, spmvc_cg_stat *stat, hipStream_t s) {
    spmvc_status first_bad = SPMVC_OK;
    if (o.mode == 1) {
        const spmvc_status st = solve_mixed(A[0], b[0], x[0], o, stat[0], s);
        SPMVC_HIP(hipStreamSynchronize(s));
        return st;
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
