// Conjugate gradient on the normal equations Op^dagger Op x = b (Section 4 lists CG), in FP64 or
// in mixed precision with reliable updates (sloppy FP32 / FP16-storage iterations, FP64 solution,
// source and true residuals).
//
// Device side: per-site vector kernels (24 reals per site) fused as
//   dot:       <p, q>                                  -> per-block FP64 partial sums
//   update_xr: alpha = rho / <p,q>; x += alpha p; r -= alpha q; |r|^2 partials
//   update_p:  beta = |r_new|^2 / |r_old|^2; p = r + beta p
// Every block of update_xr / update_p first re-sums the partials of the previous kernel in the
// same fixed order, so alpha and beta never leave the device and are identical in all blocks;
// the |r|^2 partials are double-buffered by iteration parity. No atomics: results are bitwise
// reproducible run to run.
//
// Host side: launches the iteration, reads |r|^2 back once every `check_every` iterations, and
// performs a reliable update (x += x_hat, r = b - A x in FP64, r_hat = lo(r)) when the sloppy
// residual fell below delta times its maximum since the last update, or below the target.
// The solve stops only on an FP64 true residual <= tol |b|.
#include <chrono>
#include <math.h>
#include <string.h>

#include "device.h"
#include "launch.h"

namespace gridmi {

constexpr int kRedBlocks = 1024;   // maximum number of reduction partials
constexpr int kThreads = 256;

__device__ __forceinline__ double block_sum(double v, double *sm) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    return (sm[0] + sm[1]) + (sm[2] + sm[3]);
}

// Sum of n partials in a fixed order (identical result in every block).
__device__ __forceinline__ double sum_partials(const double *__restrict__ part, int n, double *sm) {
    double v = 0.0;
    for (int k = threadIdx.x; k < n; k += kThreads) v += part[k];
    return block_sum(v, sm);
}

template <class SA, class SB>
__global__ void __launch_bounds__(kThreads)
k_dot(const void *__restrict__ a, const float *__restrict__ as, const void *__restrict__ b, const float *__restrict__ bs,
      int n, double *__restrict__ part) {
    __shared__ double sm[4];
    double acc = 0.0;
    for (int site = blockIdx.x * kThreads + threadIdx.x; site < n; site += gridDim.x * kThreads) {
        Cx<typename SA::C> x[4][3];
        Cx<typename SB::C> y[4][3];
        SA::load(a, as, site, x);
        SB::load(b, bs, site, y);
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 12; ++k)
            s += double(x[k / 3][k % 3].r) * double(y[k / 3][k % 3].r) + double(x[k / 3][k % 3].i) * double(y[k / 3][k % 3].i);
        acc += s;
    }
    const double t = block_sum(acc, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// alpha = sum(rr_prev) / sum(pq); x += alpha p; r -= alpha q; rr_new = |r|^2 partials.
template <class SX, class SP, class SR, class SQ>
__global__ void __launch_bounds__(kThreads)
k_update_xr(void *__restrict__ x, const void *__restrict__ p, const float *__restrict__ ps, void *__restrict__ r,
            float *__restrict__ rs, const void *__restrict__ q, const float *__restrict__ qs, int n,
            const double *__restrict__ rr_prev, const double *__restrict__ pq_part, int np, double *__restrict__ rr_new,
            double *__restrict__ scal) {
    __shared__ double sm[4];
    const double rho = sum_partials(rr_prev, np, sm);
    const double pq = sum_partials(pq_part, np, sm);
    const double alpha = rho / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        scal[0] = alpha;
        scal[1] = pq;
        scal[2] = rho;
    }
    double acc = 0.0;
    for (int site = blockIdx.x * kThreads + threadIdx.x; site < n; site += gridDim.x * kThreads) {
        using CX = typename SX::C;
        using CR = typename SR::C;
        Cx<CX> xv[4][3];
        Cx<typename SP::C> pv[4][3];
        Cx<CR> rv[4][3];
        Cx<typename SQ::C> qv[4][3];
        SX::load(x, nullptr, site, xv);
        SP::load(p, ps, site, pv);
        SR::load(r, rs, site, rv);
        SQ::load(q, qs, site, qv);
        const CX ax = static_cast<CX>(alpha);
        const CR ar = static_cast<CR>(alpha);
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            Cx<CX> &xx = xv[k / 3][k % 3];
            Cx<CR> &rr = rv[k / 3][k % 3];
            xx.r += ax * static_cast<CX>(pv[k / 3][k % 3].r);
            xx.i += ax * static_cast<CX>(pv[k / 3][k % 3].i);
            rr.r -= ar * static_cast<CR>(qv[k / 3][k % 3].r);
            rr.i -= ar * static_cast<CR>(qv[k / 3][k % 3].i);
        }
        SX::store(x, nullptr, site, xv);
        SR::store(r, rs, site, rv);
        // the norm is taken of the stored (possibly FP16-coded) residual
        if (SR::kBytes == 52) SR::load(r, rs, site, rv);
#pragma unroll
        for (int k = 0; k < 12; ++k)
            s += double(rv[k / 3][k % 3].r) * double(rv[k / 3][k % 3].r) + double(rv[k / 3][k % 3].i) * double(rv[k / 3][k % 3].i);
        acc += s;
    }
    const double t = block_sum(acc, sm);
    if (threadIdx.x == 0) rr_new[blockIdx.x] = t;
}

// beta = sum(rr_new) / sum(rr_prev); p = r + beta p.
template <class SR, class SP>
__global__ void __launch_bounds__(kThreads)
k_update_p(const void *__restrict__ r, const float *__restrict__ rs, void *__restrict__ p, float *__restrict__ ps, int n,
           const double *__restrict__ rr_prev, const double *__restrict__ rr_new, int np, double *__restrict__ scal) {
    __shared__ double sm[4];
    const double rho = sum_partials(rr_prev, np, sm);
    const double rn = sum_partials(rr_new, np, sm);
    const double beta = rn / rho;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        scal[3] = beta;
        scal[4] = rn;
    }
    using CP = typename SP::C;
    const CP b = static_cast<CP>(beta);
    for (int site = blockIdx.x * kThreads + threadIdx.x; site < n; site += gridDim.x * kThreads) {
        Cx<typename SR::C> rv[4][3];
        Cx<CP> pv[4][3];
        SR::load(r, rs, site, rv);
        SP::load(p, ps, site, pv);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            pv[k / 3][k % 3].r = static_cast<CP>(rv[k / 3][k % 3].r) + b * pv[k / 3][k % 3].r;
            pv[k / 3][k % 3].i = static_cast<CP>(rv[k / 3][k % 3].i) + b * pv[k / 3][k % 3].i;
        }
        SP::store(p, ps, site, pv);
    }
}

// r = b - q (FP64) with |r|^2 partials; optionally also copy r into `lo` (and its norm partials).
template <class SL>
__global__ void __launch_bounds__(kThreads)
k_residual(const void *__restrict__ b, const void *__restrict__ q, void *__restrict__ r, int n, double *__restrict__ part,
           void *__restrict__ lo, float *__restrict__ los, void *__restrict__ lo2, float *__restrict__ lo2s,
           double *__restrict__ part_lo) {
    __shared__ double sm[4];
    double acc = 0.0, acc_lo = 0.0;
    for (int site = blockIdx.x * kThreads + threadIdx.x; site < n; site += gridDim.x * kThreads) {
        Cx<double> bv[4][3], qv[4][3];
        SpF64::load(b, nullptr, site, bv);
        SpF64::load(q, nullptr, site, qv);
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            bv[k / 3][k % 3] = csub(bv[k / 3][k % 3], qv[k / 3][k % 3]);
            s += bv[k / 3][k % 3].r * bv[k / 3][k % 3].r + bv[k / 3][k % 3].i * bv[k / 3][k % 3].i;
        }
        acc += s;
        SpF64::store(r, nullptr, site, bv);
        if (lo) {
            using CL = typename SL::C;
            Cx<CL> lv[4][3];
#pragma unroll
            for (int k = 0; k < 12; ++k) lv[k / 3][k % 3] = {static_cast<CL>(bv[k / 3][k % 3].r), static_cast<CL>(bv[k / 3][k % 3].i)};
            SL::store(lo, los, site, lv);
            if (lo2) SL::store(lo2, lo2s, site, lv);
            SL::load(lo, los, site, lv);
            double sl = 0.0;
#pragma unroll
            for (int k = 0; k < 12; ++k)
                sl += double(lv[k / 3][k % 3].r) * double(lv[k / 3][k % 3].r) + double(lv[k / 3][k % 3].i) * double(lv[k / 3][k % 3].i);
            acc_lo += sl;
        }
    }
    double t = block_sum(acc, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
    if (lo) {
        t = block_sum(acc_lo, sm);
        if (threadIdx.x == 0) part_lo[blockIdx.x] = t;
    }
}

// x += x_hat (FP32), x_hat = 0.
__global__ void __launch_bounds__(kThreads) k_accum_x(void *__restrict__ x, void *__restrict__ xh, int n) {
    for (int site = blockIdx.x * kThreads + threadIdx.x; site < n; site += gridDim.x * kThreads) {
        Cx<double> xv[4][3];
        Cx<float> hv[4][3];
        SpF64::load(x, nullptr, site, xv);
        SpF32::load(xh, nullptr, site, hv);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            xv[k / 3][k % 3].r += double(hv[k / 3][k % 3].r);
            xv[k / 3][k % 3].i += double(hv[k / 3][k % 3].i);
            hv[k / 3][k % 3] = {0.f, 0.f};
        }
        SpF64::store(x, nullptr, site, xv);
        SpF32::store(xh, nullptr, site, hv);
    }
}

// Final sum of partials into scal[slot] (one block).
__global__ void __launch_bounds__(kThreads) k_sum(const double *__restrict__ part, int np, double *__restrict__ scal, int slot) {
    __shared__ double sm[4];
    const double t = sum_partials(part, np, sm);
    if (threadIdx.x == 0) scal[slot] = t;
}

// --------------------------------------------------------------------------------------------
// Workspace layout
// --------------------------------------------------------------------------------------------

static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct CgLayout {
    size_t r, q, t;                       // FP64 vectors
    size_t p;                             // FP64 mode: search direction
    size_t xh;                            // mixed: FP32 x_hat
    size_t ph, rh, qh, th;                // mixed: sloppy vectors
    size_t phs, rhs, qhs, ths;            // mixed F16S: scales
    size_t ulo;                           // mixed: sloppy links
    size_t part;                          // partials: rr[2], pq, true, lo  (5 x kRedBlocks)
    size_t scal;                          // 16 doubles
    size_t total;
};

static CgLayout cg_layout(const GeomDev &g, int sloppy, int link_fmt) {
    CgLayout L;
    memset(&L, 0, sizeof(L));
    const size_t n = static_cast<size_t>(g.n5);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    L.r = take(n * 192);
    L.q = take(n * 192);
    L.t = take(n * 192);
    if (sloppy == GRID_F64) {
        L.p = take(n * 192);
    } else {
        const size_t sb = sloppy == GRID_F32 ? 96 : 48;
        L.xh = take(n * 96);
        L.ph = take(n * sb);
        L.rh = take(n * sb);
        L.qh = take(n * sb);
        L.th = take(n * sb);
        if (sloppy == GRID_F16S) {
            L.phs = take(n * 4);
            L.rhs = take(n * 4);
            L.qhs = take(n * 4);
            L.ths = take(n * 4);
        }
        const size_t rows = link_fmt == GRID_L12 ? 2 : 3;
        const size_t cb = sloppy == GRID_F32 ? 8 : 4;
        L.ulo = take(static_cast<size_t>(g.vol) * 4 * rows * 3 * cb);
    }
    L.part = take(5 * kRedBlocks * sizeof(double));
    L.scal = take(16 * sizeof(double));
    L.total = off;
    return L;
}

size_t cg_workspace_bytes(const GeomDev &g, int sloppy, int link_fmt) { return cg_layout(g, sloppy, link_fmt).total; }

// --------------------------------------------------------------------------------------------
// Driver
// --------------------------------------------------------------------------------------------

struct CgRun {
    const void *U;
    const void *b;
    void *x;
    GeomDev g;
    int kind;            // GRID_WILSON or GRID_DWF
    double diag, mf;
    double tol;
    int maxiter;
    int sloppy;
    int link_fmt;
    double delta;
    int check_every;
    char *ws;
    hipStream_t st;
};

#define HIPCHK(x)                               \
    do {                                        \
        hipError_t e_ = (x);                    \
        if (e_ != hipSuccess) return e_;        \
    } while (0)

static hipError_t apply_op(const CgRun &c, const void *U, int prec, int fmt, const void *in, const float *ins, void *out,
                           float *outs, int dag) {
    DhopArgs a;
    a.U = U;
    a.psi = in;
    a.psi_scale = ins;
    a.out = out;
    a.out_scale = outs;
    a.g = c.g;
    a.prec = prec;
    a.link_fmt = fmt;
    a.kind = c.kind;
    a.dag = dag;
    a.diag = c.diag;
    a.mf = c.mf;
    a.stream = c.st;
    return launch_dhop(a);
}

// Sum `part` into scal[slot] on the device, then copy all 16 device scalars to `host` and wait.
static double read_scalar(const CgRun &c, const double *part, int np, double *scal, int slot, hipError_t *err,
                          double *host = nullptr) {
    double h[16];
    for (int k = 0; k < 16; ++k) h[k] = NAN;
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(kThreads), 0, c.st, part, np, scal, slot);
    *err = hipGetLastError();
    if (*err == hipSuccess) *err = hipMemcpyAsync(h, scal, sizeof(h), hipMemcpyDeviceToHost, c.st);
    if (*err == hipSuccess) *err = hipStreamSynchronize(c.st);
    if (host) memcpy(host, h, sizeof(h));
    return h[slot];
}

// Generic driver. SH: sloppy spinor policy (SpF64 for the plain FP64 solve).
template <class SH>
static hipError_t cg_T(const CgRun &c, grid_cg_stats *stats, int *status) {
    const bool mixed = c.sloppy != GRID_F64;
    const CgLayout L = cg_layout(c.g, c.sloppy, c.link_fmt);
    char *ws = c.ws;
    const int n = c.g.n5;
    const int np = static_cast<int>((static_cast<long>(n) + kThreads - 1) / kThreads < kRedBlocks
                                        ? (static_cast<long>(n) + kThreads - 1) / kThreads
                                        : kRedBlocks);
    const dim3 grid(np), block(kThreads);
    void *r = ws + L.r, *q = ws + L.q, *t = ws + L.t;
    double *part = reinterpret_cast<double *>(ws + L.part);
    double *rr[2] = {part, part + kRedBlocks};
    double *pq = part + 2 * kRedBlocks, *ptrue = part + 3 * kRedBlocks, *plo = part + 4 * kRedBlocks;
    double *scal = reinterpret_cast<double *>(ws + L.scal);
    // sloppy vectors (FP64 mode: p in FP64 and r doubles as r_hat)
    void *ph = mixed ? ws + L.ph : ws + L.p;
    void *rh = mixed ? ws + L.rh : r;
    void *qh = mixed ? ws + L.qh : q;
    void *th = mixed ? ws + L.th : t;
    float *phs = c.sloppy == GRID_F16S ? reinterpret_cast<float *>(ws + L.phs) : nullptr;
    float *rhs = c.sloppy == GRID_F16S ? reinterpret_cast<float *>(ws + L.rhs) : nullptr;
    float *qhs = c.sloppy == GRID_F16S ? reinterpret_cast<float *>(ws + L.qhs) : nullptr;
    float *ths = c.sloppy == GRID_F16S ? reinterpret_cast<float *>(ws + L.ths) : nullptr;
    void *xh = mixed ? ws + L.xh : nullptr;
    const void *ulo = mixed ? ws + L.ulo : c.U;
    const int lo_fmt = mixed ? c.link_fmt : GRID_L18;
    hipError_t err;

    // |b|
    hipLaunchKernelGGL((k_dot<SpF64, SpF64>), grid, block, 0, c.st, c.b, nullptr, c.b, nullptr, n, ptrue);
    HIPCHK(hipGetLastError());
    const double bnorm = sqrt(read_scalar(c, ptrue, np, scal, 8, &err));
    HIPCHK(err);
    stats->iterations = 0;
    stats->reliable_updates = 0;
    stats->converged = 0;
    *status = GRID_OK;
    if (bnorm == 0.0) {
        HIPCHK(hipMemsetAsync(c.x, 0, static_cast<size_t>(n) * 192, c.st));
        stats->converged = 1;
        stats->true_residual = 0.0;
        return hipStreamSynchronize(c.st);
    }
    if (mixed) {
        HIPCHK(launch_convert_links(c.U, ws + L.ulo, c.sloppy, c.link_fmt, 1, static_cast<long>(c.g.vol) * 4, c.st));
        HIPCHK(hipMemsetAsync(xh, 0, static_cast<size_t>(n) * 96, c.st));
    }
    // r = b - A x;  r_hat = p = lo(r)
    auto true_residual = [&](bool to_lo, int parity) -> hipError_t {
        HIPCHK(apply_op(c, c.U, GRID_F64, GRID_L18, c.x, nullptr, t, nullptr, 0));
        HIPCHK(apply_op(c, c.U, GRID_F64, GRID_L18, t, nullptr, q, nullptr, 1));
        if (mixed) {
            hipLaunchKernelGGL((k_residual<SH>), grid, block, 0, c.st, c.b, q, r, n, ptrue, to_lo ? rh : nullptr,
                               to_lo ? rhs : nullptr, nullptr, nullptr, rr[parity]);
        } else {
            hipLaunchKernelGGL((k_residual<SpF64>), grid, block, 0, c.st, c.b, q, r, n, to_lo ? rr[parity] : ptrue,
                               nullptr, nullptr, nullptr, nullptr, nullptr);
        }
        return hipGetLastError();
    };
    HIPCHK(apply_op(c, c.U, GRID_F64, GRID_L18, c.x, nullptr, t, nullptr, 0));
    HIPCHK(apply_op(c, c.U, GRID_F64, GRID_L18, t, nullptr, q, nullptr, 1));
    if (mixed) {
        hipLaunchKernelGGL((k_residual<SH>), grid, block, 0, c.st, c.b, q, r, n, ptrue, rh, rhs, ph, phs, rr[1]);
    } else {
        hipLaunchKernelGGL((k_residual<SpF64>), grid, block, 0, c.st, c.b, q, r, n, rr[1], nullptr, nullptr, nullptr,
                           nullptr, nullptr);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(ph, r, static_cast<size_t>(n) * 192, hipMemcpyDeviceToDevice, c.st));
    }
    HIPCHK(hipGetLastError());
    double rtrue = sqrt(read_scalar(c, mixed ? ptrue : rr[1], np, scal, 9, &err));
    HIPCHK(err);
    double maxr = rtrue;
    bool converged = rtrue <= c.tol * bnorm;
    int it = 0;
    const int check = c.check_every < 1 ? 1 : c.check_every;

    while (!converged && it < c.maxiter) {
        const int P = it & 1;
        // q_hat = A_lo p_hat
        HIPCHK(apply_op(c, ulo, c.sloppy, lo_fmt, ph, phs, th, ths, 0));
        HIPCHK(apply_op(c, ulo, c.sloppy, lo_fmt, th, ths, qh, qhs, 1));
        hipLaunchKernelGGL((k_dot<SH, SH>), grid, block, 0, c.st, ph, phs, qh, qhs, n, pq);
        HIPCHK(hipGetLastError());
        if (mixed)
            hipLaunchKernelGGL((k_update_xr<SpF32, SH, SH, SH>), grid, block, 0, c.st, xh, ph, phs, rh, rhs, qh, qhs, n,
                               rr[P ^ 1], pq, np, rr[P], scal);
        else
            hipLaunchKernelGGL((k_update_xr<SpF64, SpF64, SpF64, SpF64>), grid, block, 0, c.st, c.x, ph, nullptr, rh,
                               nullptr, qh, nullptr, n, rr[P ^ 1], pq, np, rr[P], scal);
        HIPCHK(hipGetLastError());
        ++it;
        if (it % check == 0 || it == c.maxiter) {
            double sc[16];
            const double rn = sqrt(read_scalar(c, rr[P], np, scal, 10, &err, sc));
            HIPCHK(err);
            const double pqh = sc[1];
            if (!isfinite(rn) || !(pqh > 0.0) || !isfinite(pqh)) {
                *status = GRID_EBREAKDOWN;
                break;
            }
            if (rn > maxr) maxr = rn;
            const bool small = rn <= c.tol * bnorm;
            if (small || (mixed && rn < c.delta * maxr)) {
                // reliable update / residual replacement in FP64
                if (mixed) {
                    hipLaunchKernelGGL(k_accum_x, grid, block, 0, c.st, c.x, xh, n);
                    HIPCHK(hipGetLastError());
                }
                HIPCHK(true_residual(true, P));
                ++stats->reliable_updates;
                rtrue = sqrt(read_scalar(c, mixed ? ptrue : rr[P], np, scal, 9, &err));
                HIPCHK(err);
                if (rtrue <= c.tol * bnorm) {
                    converged = true;
                    break;
                }
                maxr = rtrue;
            }
        }
        hipLaunchKernelGGL((k_update_p<SH, SH>), grid, block, 0, c.st, rh, rhs, ph, phs, n, rr[P ^ 1], rr[P], np, scal);
        HIPCHK(hipGetLastError());
    }
    if (mixed && !converged) {
        hipLaunchKernelGGL(k_accum_x, grid, block, 0, c.st, c.x, xh, n);
        HIPCHK(hipGetLastError());
    }
    // final FP64 true residual
    HIPCHK(true_residual(false, 0));
    rtrue = sqrt(read_scalar(c, ptrue, np, scal, 9, &err));
    HIPCHK(err);
    stats->iterations = it;
    stats->true_residual = rtrue / bnorm;
    stats->converged = stats->true_residual <= c.tol ? 1 : 0;
    if (*status == GRID_OK && !stats->converged) *status = GRID_ENOCONV;
    return hipSuccess;
}

hipError_t run_cg(const void *U, const void *b, void *x, const GeomDev &g, int kind, double diag, double mf,
                  const grid_cg_params &p, void *ws, hipStream_t st, grid_cg_stats *stats, int *status) {
    CgRun c;
    c.U = U;
    c.b = b;
    c.x = x;
    c.g = g;
    c.kind = kind;
    c.diag = diag;
    c.mf = mf;
    c.tol = p.tol;
    c.maxiter = p.maxiter;
    c.sloppy = p.sloppy_prec;
    c.link_fmt = p.link_fmt;
    c.delta = p.delta;
    c.check_every = p.check_every;
    c.ws = static_cast<char *>(ws);
    c.st = st;
    const auto t0 = std::chrono::steady_clock::now();
    hipError_t e;
    if (p.sloppy_prec == GRID_F64)
        e = cg_T<SpF64>(c, stats, status);
    else if (p.sloppy_prec == GRID_F32)
        e = cg_T<SpF32>(c, stats, status);
    else
        e = cg_T<SpF16S>(c, stats, status);
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return e;
}

}  // namespace gridmi
