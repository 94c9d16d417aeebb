// Conjugate gradient on the normal equations Op^dagger Op x = b (Section 4 lists CG), in FP64 or
// in mixed precision with reliable updates (sloppy FP32 / FP16-storage iterations, FP64 solution,
// source and true residuals).
//
// Device side, one iteration: the vector work rides on the operator's last kernel (the Wilson,
// Shamir and Moebius domain-wall operators and the even-odd Schur operator all take the fused
// epilogues):
//   t = op p, writing the per-block partials of |t|^2 (= <p, A p>);    one block sum -> <p,Ap>
//   r -= alpha op^dagger t in the second application's epilogue (alpha = rho / <p,Ap> from the
//        device scalars), writing the partials of |r|^2;              one block sum -> rho
//   update_px: x += alpha p; p = r + beta p (beta = rho_new / rho_old).
// A p is never stored: per iteration 6 vectors of streaming traffic beyond the two operator
// applications' own, against 10 for separate dot, x/r-update and p-update kernels. The partials
// are summed in a fixed order and rho is double-buffered by iteration parity; alpha and beta never
// leave the device. No atomics: results are bitwise reproducible run to run.
//
// Host side: launches the iteration, reads |r|^2 back once every `check_every` iterations, and
// performs a reliable update (x += x_hat, r = b - A x in FP64, r_hat = lo(r)) when the sloppy
// residual fell below delta times its maximum since the last update, or below the target.
// The solve stops only on an FP64 true residual <= tol |b|.
//
// With params.graph the check_every iterations between two host reads (their last x/p update
// excepted, which follows the check) are recorded once into a HIP graph per starting parity on a
// stream the solver creates, then replayed on the caller's stream: one launch per segment in
// place of about six per iteration. The recorded kernels and arguments are those of the direct
// path (all workspace pointers are fixed for the solve), so results are bitwise identical.
#include <chrono>
#include <type_traits>
#include <math.h>
#include <string.h>

#include "device.h"
#include "launch.h"

namespace gridmi {

constexpr int kRedBlocks = 1024;   // maximum number of reduction partials
static_assert(kNormScratch >= kRedBlocks + 1, "norm scratch holds the partials and the sum");
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

// ---------------------------------------------------------------------------------------------
// Streaming vector kernels. FP64 and FP32 vectors have no per-site structure the update needs, so
// they are processed as flat arrays of 16-byte chunks (one complex double or two complex floats):
// consecutive lanes touch consecutive 16 bytes. FP16-storage vectors are processed in units of
// one 16-byte code chunk (4 complex numbers, a third of a site) with 21 sites (63 lanes) per
// wavefront, so the three lanes of a site can agree on the site's new scale when re-encoding.
// ---------------------------------------------------------------------------------------------

__device__ __forceinline__ double dot2(double2 a, double2 b) { return a.x * b.x + a.y * b.y; }
__device__ __forceinline__ double dot2(float4 a, float4 b) {
    return double(a.x) * double(b.x) + double(a.y) * double(b.y) + double(a.z) * double(b.z) + double(a.w) * double(b.w);
}
__device__ __forceinline__ double2 axpy2(double al, double2 x, double2 y) { return make_double2(y.x + al * x.x, y.y + al * x.y); }
__device__ __forceinline__ float4 axpy2(double al, float4 x, float4 y) {
    const float a = static_cast<float>(al);
    return make_float4(y.x + a * x.x, y.y + a * x.y, y.z + a * x.z, y.w + a * x.w);
}

template <typename V>
__global__ void __launch_bounds__(kThreads)
k_dot_flat(const V *__restrict__ a, const V *__restrict__ b, long n, double *__restrict__ part) {
    __shared__ double sm[4];
    double acc = 0.0;
    for (long i = static_cast<long>(blockIdx.x) * kThreads + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * kThreads)
        acc += dot2(a[i], b[i]);
    const double t = block_sum(acc, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Fused sequence: alpha = scal[so] / scal[sq], beta = scal[sn] / scal[so];
// mode bit 0: x += alpha p; bit 1: p = r + beta p (p read once for both).
template <typename V>
__global__ void __launch_bounds__(kThreads)
k_update_px_flat(V *__restrict__ x, V *__restrict__ p, const V *__restrict__ r, long n, const double *__restrict__ scal,
                 int so, int sn, int sq, int mode) {
    const double rho = scal[so];
    const double alpha = rho / scal[sq], beta = scal[sn] / rho;
    for (long i = static_cast<long>(blockIdx.x) * kThreads + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * kThreads) {
        const V pv = p[i];
        if (mode & 1) x[i] = axpy2(alpha, pv, x[i]);
        if (mode & 2) p[i] = axpy2(beta, pv, r[i]);
    }
}

// r = b - q in FP64 (flat, one complex per chunk), |r|^2 partials.
__global__ void __launch_bounds__(kThreads)
k_residual_f64(const double2 *__restrict__ b, const double2 *__restrict__ q, double2 *__restrict__ r, long n,
               double *__restrict__ part) {
    __shared__ double sm[4];
    double acc = 0.0;
    for (long i = static_cast<long>(blockIdx.x) * kThreads + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * kThreads) {
        const double2 bv = b[i], qv = q[i];
        const double2 rv = make_double2(bv.x - qv.x, bv.y - qv.y);
        r[i] = rv;
        acc += dot2(rv, rv);
    }
    const double t = block_sum(acc, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// r = b - q in FP64 plus FP32 copies lo (and lo2) of r; chunk i covers two complex numbers.
__global__ void __launch_bounds__(kThreads)
k_residual_f32lo(const double2 *__restrict__ b, const double2 *__restrict__ q, double2 *__restrict__ r, float4 *__restrict__ lo,
                 float4 *__restrict__ lo2, long n, double *__restrict__ part, double *__restrict__ part_lo) {
    __shared__ double sm[4];
    double acc = 0.0, acc_lo = 0.0;
    for (long i = static_cast<long>(blockIdx.x) * kThreads + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * kThreads) {
        const double2 b0 = b[2 * i], b1 = b[2 * i + 1], q0 = q[2 * i], q1 = q[2 * i + 1];
        const double2 r0 = make_double2(b0.x - q0.x, b0.y - q0.y), r1 = make_double2(b1.x - q1.x, b1.y - q1.y);
        r[2 * i] = r0;
        r[2 * i + 1] = r1;
        acc += dot2(r0, r0) + dot2(r1, r1);
        const float4 l = make_float4(static_cast<float>(r0.x), static_cast<float>(r0.y), static_cast<float>(r1.x),
                                     static_cast<float>(r1.y));
        lo[i] = l;
        if (lo2) lo2[i] = l;
        acc_lo += dot2(l, l);
    }
    double t = block_sum(acc, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
    t = block_sum(acc_lo, sm);
    if (threadIdx.x == 0) part_lo[blockIdx.x] = t;
}

// x += x_hat (FP32), x_hat = 0; chunk i of x_hat covers two complex numbers of x.
__global__ void __launch_bounds__(kThreads) k_accum_x(double2 *__restrict__ x, float4 *__restrict__ xh, long n) {
    for (long i = static_cast<long>(blockIdx.x) * kThreads + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * kThreads) {
        const float4 h = xh[i];
        const double2 x0 = x[2 * i], x1 = x[2 * i + 1];
        x[2 * i] = make_double2(x0.x + double(h.x), x0.y + double(h.y));
        x[2 * i + 1] = make_double2(x1.x + double(h.z), x1.y + double(h.w));
        xh[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// ---- FP16 storage: units of 8 halves (4 complex) + the site scale ----

__device__ __forceinline__ void unit_decode(uint4 w, float s, float v[8]) {
    const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        v[2 * j] = half_bits_to_float(ww[j] & 0xffffu) * s;
        v[2 * j + 1] = half_bits_to_float(ww[j] >> 16) * s;
    }
}

// Encode a unit with the site maximum taken over the three lanes 3r..3r+2 of the site (all 64
// lanes execute the shuffles); returns the code chunk and the site scale.
__device__ __forceinline__ uint4 unit_encode(const float v[8], float &site_max) {
    float m = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) m = fmaxf(m, fabsf(v[j]));
    const int lane = threadIdx.x & 63, r3 = 3 * (lane / 3);
    m = fmaxf(__shfl(m, r3, 64), fmaxf(__shfl(m, r3 + 1, 64), __shfl(m, r3 + 2, 64)));
    site_max = m;
    const float inv = m > 0.f ? 1.0f / m : 0.f;
    uint32_t w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) w[j] = scaled_half_bits(v[2 * j], inv) | (scaled_half_bits(v[2 * j + 1], inv) << 16);
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// Unit position in the FP16 kernels' loop: 21 sites per wavefront, unit = site * 3 + lane % 3;
// lane 63 (and lanes past the last site) shadow a valid unit but store nothing.
struct UnitPos {
    long su, unit;
    int sub;
    bool ok;
};

__device__ __forceinline__ UnitPos unit_pos(long sb, long nsites) {
    const int lane = threadIdx.x & 63;
    const long site = sb + lane / 3;
    UnitPos u;
    u.ok = lane < 63 && site < nsites;
    u.su = u.ok ? site : sb;
    u.sub = lane < 63 ? lane % 3 : 0;
    u.unit = u.su * 3 + u.sub;
    return u;
}

__device__ __forceinline__ long unit_first() {
    return (static_cast<long>(blockIdx.x) * (kThreads / 64) + (threadIdx.x >> 6)) * 21;
}
__device__ __forceinline__ long unit_stride() { return static_cast<long>(gridDim.x) * (kThreads / 64) * 21; }

// FP16-storage form of k_update_px_flat (x_hat in FP32, p re-encoded).
__global__ void __launch_bounds__(kThreads)
k_update_px_f16(float4 *__restrict__ xh, uint4 *__restrict__ p, float *__restrict__ ps, const uint4 *__restrict__ r,
                const float *__restrict__ rs, long nsites, const double *__restrict__ scal, int so, int sn, int sq,
                int mode) {
    const double rho = scal[so];
    const float al = static_cast<float>(rho / scal[sq]), be = static_cast<float>(scal[sn] / rho);
    for (long sb = unit_first(); sb < nsites; sb += unit_stride()) {
        const UnitPos u = unit_pos(sb, nsites);
        float pv[8];
        unit_decode(p[u.unit], ps[u.su], pv);
        if ((mode & 1) && u.ok) {
            float4 x0 = xh[2 * u.unit], x1 = xh[2 * u.unit + 1];
            xh[2 * u.unit] = make_float4(x0.x + al * pv[0], x0.y + al * pv[1], x0.z + al * pv[2], x0.w + al * pv[3]);
            xh[2 * u.unit + 1] = make_float4(x1.x + al * pv[4], x1.y + al * pv[5], x1.z + al * pv[6], x1.w + al * pv[7]);
        }
        if (mode & 2) {
            float rv[8];
            unit_decode(r[u.unit], rs[u.su], rv);
#pragma unroll
            for (int j = 0; j < 8; ++j) pv[j] = rv[j] + be * pv[j];
            float m;
            const uint4 code = unit_encode(pv, m);
            if (u.ok) {
                p[u.unit] = code;
                if (u.sub == 0) ps[u.su] = m;
            }
        }
    }
}

// r = b - q (FP64) with |r|^2 partials, and FP16 copies lo (and lo2) with |lo|^2 partials.
__global__ void __launch_bounds__(kThreads)
k_residual_f16lo(const double2 *__restrict__ b, const double2 *__restrict__ q, double2 *__restrict__ r, uint4 *__restrict__ lo,
                 float *__restrict__ los, uint4 *__restrict__ lo2, float *__restrict__ lo2s, long nsites,
                 double *__restrict__ part, double *__restrict__ part_lo) {
    __shared__ double sm[4];
    double acc = 0.0, acc_lo = 0.0;
    for (long sb = unit_first(); sb < nsites; sb += unit_stride()) {
        const UnitPos u = unit_pos(sb, nsites);
        float v[8];
        double d = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double2 bv = b[4 * u.unit + j], qv = q[4 * u.unit + j];
            const double2 rv = make_double2(bv.x - qv.x, bv.y - qv.y);
            if (u.ok) r[4 * u.unit + j] = rv;
            d += dot2(rv, rv);
            v[2 * j] = static_cast<float>(rv.x);
            v[2 * j + 1] = static_cast<float>(rv.y);
        }
        float m;
        const uint4 code = unit_encode(v, m);
        if (u.ok) {
            acc += d;
            lo[u.unit] = code;
            if (u.sub == 0) los[u.su] = m;
            if (lo2) {
                lo2[u.unit] = code;
                if (u.sub == 0) lo2s[u.su] = m;
            }
            float dv[8];
            unit_decode(code, m, dv);
            double dl = 0.0;
#pragma unroll
            for (int j = 0; j < 8; ++j) dl += double(dv[j]) * double(dv[j]);
            acc_lo += dl;
        }
    }
    double t = block_sum(acc, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
    t = block_sum(acc_lo, sm);
    if (threadIdx.x == 0) part_lo[blockIdx.x] = t;
}

// Partials of |a - b|^2 over FP64 chunks.
__global__ void __launch_bounds__(kThreads)
k_diff_norm2(const double2 *__restrict__ a, const double2 *__restrict__ b, long n, double *__restrict__ part) {
    __shared__ double sm[4];
    double acc = 0.0;
    for (long i = static_cast<long>(blockIdx.x) * kThreads + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * kThreads) {
        const double2 u = a[i], v = b[i];
        const double dx = u.x - v.x, dy = u.y - v.y;
        acc += dx * dx + dy * dy;
    }
    const double t = block_sum(acc, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Final sum of partials into scal[slot] (one block).
__global__ void __launch_bounds__(kThreads) k_sum(const double *__restrict__ part, int np, double *__restrict__ scal, int slot) {
    __shared__ double sm[4];
    const double t = sum_partials(part, np, sm);
    if (threadIdx.x == 0) scal[slot] = t;
}

// Final sum of many partials (the fused epilogues write one per operator block, up to tens of
// thousands): 1024 threads with eight independent accumulators each keep the loads in flight.
// The order is fixed, so the sum is reproducible.
constexpr int kWideThreads = 1024;
__global__ void __launch_bounds__(kWideThreads)
k_sum_wide(const double *__restrict__ part, int np, double *__restrict__ scal, int slot) {
    __shared__ double sm[kWideThreads / 64];
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int k = threadIdx.x;
    for (; k + 7 * kWideThreads < np; k += 8 * kWideThreads) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] += part[k + j * kWideThreads];
    }
    for (; k < np; k += kWideThreads) a[0] += part[k];
    double v = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kWideThreads / 64; ++w) t += sm[w];
        scal[slot] = t;
    }
}

// Launch helpers per sloppy precision (FP64 mode uses SpF64 for everything).
template <class SH>
struct Vec;

template <>
struct Vec<SpF64> {
    static void update_px(dim3 g, hipStream_t st, void *x, void *p, float *, const void *r, const float *, long n5,
                          const double *scal, int so, int sn, int sq, int mode) {
        hipLaunchKernelGGL(k_update_px_flat<double2>, g, dim3(kThreads), 0, st, static_cast<double2 *>(x),
                           static_cast<double2 *>(p), static_cast<const double2 *>(r), n5 * 12, scal, so, sn, sq, mode);
    }
};

template <>
struct Vec<SpF32> {
    static void update_px(dim3 g, hipStream_t st, void *x, void *p, float *, const void *r, const float *, long n5,
                          const double *scal, int so, int sn, int sq, int mode) {
        hipLaunchKernelGGL(k_update_px_flat<float4>, g, dim3(kThreads), 0, st, static_cast<float4 *>(x),
                           static_cast<float4 *>(p), static_cast<const float4 *>(r), n5 * 6, scal, so, sn, sq, mode);
    }
    static void residual_lo(dim3 g, hipStream_t st, const void *b, const void *q, void *r, void *lo, float *, void *lo2,
                            float *, long n5, double *part, double *part_lo) {
        hipLaunchKernelGGL(k_residual_f32lo, g, dim3(kThreads), 0, st, static_cast<const double2 *>(b),
                           static_cast<const double2 *>(q), static_cast<double2 *>(r), static_cast<float4 *>(lo),
                           static_cast<float4 *>(lo2), n5 * 6, part, part_lo);
    }
};

template <>
struct Vec<SpF16S> {
    static void update_px(dim3 g, hipStream_t st, void *x, void *p, float *ps, const void *r, const float *rs, long n5,
                          const double *scal, int so, int sn, int sq, int mode) {
        hipLaunchKernelGGL(k_update_px_f16, g, dim3(kThreads), 0, st, static_cast<float4 *>(x), static_cast<uint4 *>(p),
                           ps, static_cast<const uint4 *>(r), rs, n5, scal, so, sn, sq, mode);
    }
    static void residual_lo(dim3 g, hipStream_t st, const void *b, const void *q, void *r, void *lo, float *los, void *lo2,
                            float *lo2s, long n5, double *part, double *part_lo) {
        hipLaunchKernelGGL(k_residual_f16lo, g, dim3(kThreads), 0, st, static_cast<const double2 *>(b),
                           static_cast<const double2 *>(q), static_cast<double2 *>(r), static_cast<uint4 *>(lo), los,
                           static_cast<uint4 *>(lo2), lo2s, n5, part, part_lo);
    }
};

// --------------------------------------------------------------------------------------------
// Workspace layout
// --------------------------------------------------------------------------------------------

static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct CgLayout {
    size_t r, q, t;                       // FP64 vectors
    size_t p;                             // FP64 mode: search direction
    size_t xh;                            // mixed: FP32 x_hat
    size_t ph, rh, th;                    // mixed: sloppy vectors
    size_t phs, rhs, ths;                 // mixed F16S: scales
    size_t ulo;                           // mixed: sloppy links
    size_t u, uh, uhs;                    // operator temporaries (FP64, sloppy, sloppy scales)
    size_t part;                          // partials: rr[2], true  (3 x kRedBlocks)
    size_t opp;                           // fused-epilogue partials (one per operator block)
    size_t scal;                          // 16 doubles
    size_t total;
};

static CgLayout cg_layout(long nsites, long nlinks, int sloppy, int link_fmt, bool op_tmp, long nparts) {
    CgLayout L;
    memset(&L, 0, sizeof(L));
    const size_t n = static_cast<size_t>(nsites);
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
        L.th = take(n * sb);
        if (sloppy == GRID_F16S) {
            L.phs = take(n * 4);
            L.rhs = take(n * 4);
            L.ths = take(n * 4);
        }
        const size_t rows = link_fmt == GRID_L12 ? 2 : 3;
        const size_t cb = sloppy == GRID_F32 ? 8 : 4;
        L.ulo = take(static_cast<size_t>(nlinks) * rows * 3 * cb);
    }
    if (op_tmp) {
        L.u = take(n * 192);
        if (sloppy != GRID_F64) {
            L.uh = take(n * (sloppy == GRID_F32 ? 96 : 48));
            if (sloppy == GRID_F16S) L.uhs = take(n * 4);
        }
    }
    L.part = take(3 * kRedBlocks * sizeof(double));
    if (nparts > 0) L.opp = take(static_cast<size_t>(nparts) * sizeof(double));
    L.scal = take(16 * sizeof(double));
    L.total = off;
    return L;
}

size_t cg_workspace_bytes_n(long nsites, long nlinks, int sloppy, int link_fmt, long nparts) {
    return cg_layout(nsites, nlinks, sloppy, link_fmt, false, nparts).total;
}

// The full-lattice solve keeps one operator temporary per precision (the Moebius operator's
// intermediate field) and room for the fused epilogues' partial sums.
size_t cg_workspace_bytes(const GeomDev &g, int sloppy, int link_fmt) {
    return cg_layout(g.n5, static_cast<long>(g.vol) * 4, sloppy, link_fmt, true, fused_parts_max(g.n5, g.L[3])).total;
}

// --------------------------------------------------------------------------------------------
// Driver
// --------------------------------------------------------------------------------------------

struct CgRun {
    const void *U;
    const void *b;
    void *x;
    long n;              // 5D sites of the system
    long nlinks;         // links (for the sloppy copy)
    CgOp op;             // A = op^dagger op
    double tol;
    int maxiter;
    int sloppy;
    int link_fmt;
    double delta;
    int check_every;
    bool graph;          // replay recorded iteration segments
    char *ws;
    hipStream_t st;
    bool op_tmp;         // workspace holds the operator temporaries
    long nparts;         // room for the fused epilogues' partials
};

// Capture stream of the calling host thread on the current device: created on first use and kept
// for the life of the process, so a solve creates no stream, and a capture in one host thread
// never meets another thread's.
hipError_t capture_stream(hipStream_t *s) {
    constexpr int kMaxDevices = 64;
    thread_local hipStream_t streams[kMaxDevices] = {};
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    if (!streams[dev]) {
        const hipError_t e2 = hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking);
        if (e2 != hipSuccess) return e2;
    }
    *s = streams[dev];
    return hipSuccess;
}

// Recorded iteration segments of one solve, by starting parity; released with the solve (the
// recorded kernels name this solve's fields and workspace). The caller's stream is drained before
// the executables are destroyed (the normal exits have already synchronised it; an error exit may
// leave replays in flight).
struct SegmentGraphs {
    hipStream_t user;
    hipStream_t cs = nullptr;
    hipGraphExec_t ex[2] = {nullptr, nullptr};
    explicit SegmentGraphs(hipStream_t s) : user(s) {}
    SegmentGraphs(const SegmentGraphs &) = delete;
    SegmentGraphs &operator=(const SegmentGraphs &) = delete;
    ~SegmentGraphs() {
        if (ex[0] || ex[1]) (void)hipStreamSynchronize(user);
        for (hipGraphExec_t e : ex)
            if (e) (void)hipGraphExecDestroy(e);
    }
};

#define HIPCHK(x)                               \
    do {                                        \
        hipError_t e_ = (x);                    \
        if (e_ != hipSuccess) return e_;        \
    } while (0)

static hipError_t apply_op(const CgRun &c, const void *U, int prec, int fmt, const void *in, const float *ins, void *out,
                           float *outs, int dag) {
    return c.op.apply(c.op.ctx, U, prec, fmt, in, ins, out, outs, dag, c.st);
}

// The full-lattice operator (Wilson D, Shamir M or Moebius M).
struct FullOp {
    GeomDev g;
    int kind;
    double diag, mf;
    double M5, b5, c5;
    void *tmp[2];      // Moebius intermediate field: FP64, sloppy
    float *tmps;       // sloppy FP16 scales
};

static DhopArgs full_args(const FullOp &o, const void *U, int prec, int fmt, const void *in, const float *ins,
                          void *out, float *outs, int dag, hipStream_t st) {
    DhopArgs a;
    a.U = U;
    a.psi = in;
    a.psi_scale = ins;
    a.out = out;
    a.out_scale = outs;
    a.g = o.g;
    a.prec = prec;
    a.link_fmt = fmt;
    a.kind = o.kind;
    a.dag = dag;
    a.diag = o.diag;
    a.mf = o.mf;
    a.stream = st;
    return a;
}

static hipError_t full_apply(const void *ctx, const void *U, int prec, int fmt, const void *in, const float *ins, void *out,
                             float *outs, int dag, hipStream_t st) {
    const FullOp &o = *static_cast<const FullOp *>(ctx);
    const DhopArgs a = full_args(o, U, prec, fmt, in, ins, out, outs, dag, st);
    if (o.kind == GRID_MOBIUS)
        return launch_mobius(a, o.M5, o.b5, o.c5, o.tmp[prec == GRID_F64 ? 0 : 1], prec == GRID_F16S ? o.tmps : nullptr);
    return launch_dhop(a);
}

// Wilson / Shamir / Moebius domain-wall operator with a fused epilogue on its last kernel.
static hipError_t full_apply_fused(const void *ctx, const void *U, int prec, int fmt, const void *in, const float *ins,
                                   void *out, float *outs, int dag, int fuse, const FuseDev &fz, long *nparts,
                                   hipStream_t st) {
    const FullOp &o = *static_cast<const FullOp *>(ctx);
    if (o.kind != GRID_WILSON && o.kind != GRID_DWF && o.kind != GRID_MOBIUS) return hipErrorInvalidValue;
    DhopArgs a = full_args(o, U, prec, fmt, in, ins, out, outs, dag, st);
    a.fuse = fuse;
    a.fz = fz;
    if (o.kind == GRID_MOBIUS)
        return launch_mobius(a, o.M5, o.b5, o.c5, o.tmp[prec == GRID_F64 ? 0 : 1], prec == GRID_F16S ? o.tmps : nullptr,
                             nparts);
    *nparts = dhop_blocks(a);
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
    const CgLayout L = cg_layout(c.n, c.nlinks, c.sloppy, c.link_fmt, c.op_tmp, c.nparts);
    char *ws = c.ws;
    const int n = static_cast<int>(c.n);
    const int np = static_cast<int>((static_cast<long>(n) + kThreads - 1) / kThreads < kRedBlocks
                                        ? (static_cast<long>(n) + kThreads - 1) / kThreads
                                        : kRedBlocks);
    const dim3 grid(np), block(kThreads);
    if (!c.op.apply_fused || c.nparts <= 0) return hipErrorInvalidValue;
    void *r = ws + L.r, *q = ws + L.q, *t = ws + L.t;
    double *part = reinterpret_cast<double *>(ws + L.part);
    double *rr[2] = {part, part + kRedBlocks};
    double *ptrue = part + 2 * kRedBlocks;
    double *scal = reinterpret_cast<double *>(ws + L.scal);
    // sloppy vectors (FP64 mode: p in FP64 and r doubles as r_hat)
    void *ph = mixed ? ws + L.ph : ws + L.p;
    void *rh = mixed ? ws + L.rh : r;
    void *th = mixed ? ws + L.th : t;
    float *phs = c.sloppy == GRID_F16S ? reinterpret_cast<float *>(ws + L.phs) : nullptr;
    float *rhs = c.sloppy == GRID_F16S ? reinterpret_cast<float *>(ws + L.rhs) : nullptr;
    float *ths = c.sloppy == GRID_F16S ? reinterpret_cast<float *>(ws + L.ths) : nullptr;
    void *xh = mixed ? ws + L.xh : nullptr;
    void *xs = mixed ? xh : c.x;   // the vector the iterations update
    const void *ulo = mixed ? ws + L.ulo : c.U;
    const int lo_fmt = mixed ? c.link_fmt : GRID_L18;
    hipError_t err;
    // device scalars <p,Ap> and rho (by iteration parity); the operator kernels' partials
    constexpr int kSlotPQ = 11, kSlotRho = 12;
    double *opp = reinterpret_cast<double *>(ws + L.opp);
    auto sum_to = [&](hipStream_t s, const double *pp, long cnt, int slot) -> hipError_t {
        hipLaunchKernelGGL(k_sum_wide, dim3(1), dim3(kWideThreads), 0, s, pp, static_cast<int>(cnt), scal, slot);
        return hipGetLastError();
    };

    // |b|
    hipLaunchKernelGGL(k_dot_flat<double2>, grid, block, 0, c.st, static_cast<const double2 *>(c.b),
                       static_cast<const double2 *>(c.b), static_cast<long>(n) * 12, ptrue);
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
        HIPCHK(launch_convert_links(c.U, ws + L.ulo, c.sloppy, c.link_fmt, 1, c.nlinks, c.st));
        HIPCHK(hipMemsetAsync(xh, 0, static_cast<size_t>(n) * 96, c.st));
    }
    // r = b - A x;  r_hat = p = lo(r)
    auto true_residual = [&](bool to_lo, int parity) -> hipError_t {
        HIPCHK(apply_op(c, c.U, GRID_F64, GRID_L18, c.x, nullptr, t, nullptr, 0));
        HIPCHK(apply_op(c, c.U, GRID_F64, GRID_L18, t, nullptr, q, nullptr, 1));
        if (mixed && to_lo) {
            if constexpr (!std::is_same<SH, SpF64>::value)
                Vec<SH>::residual_lo(grid, c.st, c.b, q, r, rh, rhs, nullptr, nullptr, n, ptrue, rr[parity]);
        } else {
            hipLaunchKernelGGL(k_residual_f64, grid, block, 0, c.st, static_cast<const double2 *>(c.b),
                               static_cast<const double2 *>(q), static_cast<double2 *>(r), static_cast<long>(n) * 12,
                               (!mixed && to_lo) ? rr[parity] : ptrue);
        }
        return hipGetLastError();
    };
    HIPCHK(apply_op(c, c.U, GRID_F64, GRID_L18, c.x, nullptr, t, nullptr, 0));
    HIPCHK(apply_op(c, c.U, GRID_F64, GRID_L18, t, nullptr, q, nullptr, 1));
    if (mixed) {
        if constexpr (!std::is_same<SH, SpF64>::value)
            Vec<SH>::residual_lo(grid, c.st, c.b, q, r, rh, rhs, ph, phs, n, ptrue, rr[1]);
    } else {
        hipLaunchKernelGGL(k_residual_f64, grid, block, 0, c.st, static_cast<const double2 *>(c.b),
                           static_cast<const double2 *>(q), static_cast<double2 *>(r), static_cast<long>(n) * 12, rr[1]);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(ph, r, static_cast<size_t>(n) * 192, hipMemcpyDeviceToDevice, c.st));
    }
    HIPCHK(hipGetLastError());
    HIPCHK(sum_to(c.st, rr[1], np, kSlotRho + 1));
    double rtrue = sqrt(read_scalar(c, mixed ? ptrue : rr[1], np, scal, 9, &err));
    HIPCHK(err);
    double maxr = rtrue;
    bool converged = rtrue <= c.tol * bnorm;
    int it = 0;
    const int check = c.check_every < 1 ? 1 : c.check_every;

    // one sloppy step on stream s, parity P: t = op p with |t|^2 = <p, A p>, then
    // r -= alpha op^dagger t with |r|^2 (x follows in step_px)
    auto step_xr = [&](hipStream_t s, int P) -> hipError_t {
        long nb = 0;
        FuseDev f1;
        f1.part = opp;
        HIPCHK(c.op.apply_fused(c.op.ctx, ulo, c.sloppy, lo_fmt, ph, phs, th, ths, 0, kFuseNorm, f1, &nb, s));
        HIPCHK(sum_to(s, opp, nb, kSlotPQ));
        FuseDev f2;
        f2.r = rh;
        f2.r_scale = rhs;
        f2.scal = scal;
        f2.num = kSlotRho + (P ^ 1);
        f2.den = kSlotPQ;
        f2.part = opp;
        HIPCHK(c.op.apply_fused(c.op.ctx, ulo, c.sloppy, lo_fmt, th, ths, rh, rhs, 1, kFuseAxpy, f2, &nb, s));
        return sum_to(s, opp, nb, kSlotRho + P);
    };
    // mode 3: x += alpha p and p = r + beta p; mode 1 / 2: either half
    auto step_px = [&](hipStream_t s, int P, int mode) -> hipError_t {
        Vec<SH>::update_px(grid, s, xs, ph, phs, rh, rhs, n, scal, kSlotRho + (P ^ 1), kSlotRho + P, kSlotPQ, mode);
        return hipGetLastError();
    };
    // record the segment of `check` steps starting at parity P0
    SegmentGraphs seg(c.st);
    auto record = [&](int P0) -> hipError_t {
        if (!seg.cs) HIPCHK(capture_stream(&seg.cs));
        HIPCHK(hipStreamBeginCapture(seg.cs, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int i = 0; i < check && e == hipSuccess; ++i) {
            e = step_xr(seg.cs, (P0 + i) & 1);
            if (e == hipSuccess && i + 1 < check) e = step_px(seg.cs, (P0 + i) & 1, 3);
        }
        hipGraph_t gr = nullptr;
        const hipError_t e2 = hipStreamEndCapture(seg.cs, &gr);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&seg.ex[P0], gr, nullptr, nullptr, 0);
        if (gr) (void)hipGraphDestroy(gr);
        return e;
    };

    while (!converged && it < c.maxiter) {
        int P = it & 1;
        if (c.graph && it % check == 0 && it + check <= c.maxiter) {
            if (!seg.ex[P]) HIPCHK(record(P));
            HIPCHK(hipGraphLaunch(seg.ex[P], c.st));
            it += check;
            P = (it - 1) & 1;
        } else {
            HIPCHK(step_xr(c.st, P));
            ++it;
        }
        bool x_done = false;   // alpha p already added to x
        if (it % check == 0 || it == c.maxiter) {
            // |r|^2 and <p,Ap> are already summed on the device
            double sc[16];
            for (int k = 0; k < 16; ++k) sc[k] = NAN;
            HIPCHK(hipMemcpyAsync(sc, scal, sizeof(sc), hipMemcpyDeviceToHost, c.st));
            HIPCHK(hipStreamSynchronize(c.st));
            const double rn = sqrt(sc[kSlotRho + P]);
            const double pqh = sc[kSlotPQ];
            if (!isfinite(rn) || !(pqh > 0.0) || !isfinite(pqh)) {
                *status = GRID_EBREAKDOWN;
                break;
            }
            if (rn > maxr) maxr = rn;
            const bool small = rn <= c.tol * bnorm;
            if (small || (mixed && rn < c.delta * maxr)) {
                // reliable update / residual replacement in FP64
                HIPCHK(step_px(c.st, P, 1));
                x_done = true;
                if (mixed) {
                    hipLaunchKernelGGL(k_accum_x, grid, block, 0, c.st, static_cast<double2 *>(c.x),
                                       static_cast<float4 *>(xh), static_cast<long>(n) * 6);
                    HIPCHK(hipGetLastError());
                }
                HIPCHK(true_residual(true, P));
                HIPCHK(sum_to(c.st, rr[P], np, kSlotRho + P));
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
        HIPCHK(step_px(c.st, P, x_done ? 2 : 3));
    }
    if (mixed && !converged) {
        hipLaunchKernelGGL(k_accum_x, grid, block, 0, c.st, static_cast<double2 *>(c.x), static_cast<float4 *>(xh),
                           static_cast<long>(n) * 6);
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

hipError_t run_cg_op(const CgOp &op, const void *U, const void *b, void *x, long nsites, long nlinks,
                     const grid_cg_params &p, void *ws, hipStream_t st, grid_cg_stats *stats, int *status,
                     bool op_tmp, long nparts) {
    CgRun c;
    c.op_tmp = op_tmp;
    c.nparts = nparts;
    c.U = U;
    c.b = b;
    c.x = x;
    c.n = nsites;
    c.nlinks = nlinks;
    c.op = op;
    c.tol = p.tol;
    c.maxiter = p.maxiter;
    c.sloppy = p.sloppy_prec;
    c.link_fmt = p.link_fmt;
    c.delta = p.delta;
    c.check_every = p.check_every;
    c.graph = p.graph != 0;
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

hipError_t run_cg(const void *U, const void *b, void *x, const GeomDev &g, const grid_op &opd, const grid_cg_params &p,
                  void *ws, hipStream_t st, grid_cg_stats *stats, int *status) {
    FullOp o;
    o.g = g;
    o.kind = opd.kind;
    o.diag = opd.kind == GRID_WILSON ? 4.0 + opd.mass : 5.0 - opd.M5;
    o.mf = opd.mf;
    o.M5 = opd.M5;
    o.b5 = opd.b5;
    o.c5 = opd.c5;
    const long nparts = fused_parts_max(g.n5, g.L[3]);
    const CgLayout L = cg_layout(g.n5, static_cast<long>(g.vol) * 4, p.sloppy_prec, p.link_fmt, true, nparts);
    char *w = static_cast<char *>(ws);
    o.tmp[0] = w + L.u;
    o.tmp[1] = p.sloppy_prec != GRID_F64 ? w + L.uh : nullptr;
    o.tmps = p.sloppy_prec == GRID_F16S ? reinterpret_cast<float *>(w + L.uhs) : nullptr;
    CgOp op;
    op.apply = full_apply;
    op.ctx = &o;
    if (opd.kind == GRID_WILSON || opd.kind == GRID_DWF || opd.kind == GRID_MOBIUS) op.apply_fused = full_apply_fused;
    return run_cg_op(op, U, b, x, g.n5, static_cast<long>(g.vol) * 4, p, ws, st, stats, status, true, nparts);
}

hipError_t dot_re(const void *a, const void *b, long n, double *part, hipStream_t st, double *result) {
    const int np = static_cast<int>((n + kThreads - 1) / kThreads < kRedBlocks ? (n + kThreads - 1) / kThreads
                                                                                : kRedBlocks);
    if (n == 0) {
        *result = 0.0;
        return hipSuccess;
    }
    hipLaunchKernelGGL(k_dot_flat<double2>, dim3(np), dim3(kThreads), 0, st, static_cast<const double2 *>(a),
                       static_cast<const double2 *>(b), n * 12, part);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(kThreads), 0, st, part, np, part + kRedBlocks, 0);
    HIPCHK(hipGetLastError());
    double h = 0.0;
    HIPCHK(hipMemcpyAsync(&h, part + kRedBlocks, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *result = h;
    return hipSuccess;
}

// ||a - b||^2 (b may be NULL) over n FP64 spinor sites, summed deterministically; waits for the
// stream. `part` holds kRedBlocks + 16 doubles of device scratch.
hipError_t norm2_diff(const void *a, const void *b, long n, double *part, hipStream_t st, double *result) {
    const int np = static_cast<int>((n + kThreads - 1) / kThreads < kRedBlocks ? (n + kThreads - 1) / kThreads
                                                                                : kRedBlocks);
    if (n == 0) {
        *result = 0.0;
        return hipSuccess;
    }
    if (b)
        hipLaunchKernelGGL(k_diff_norm2, dim3(np), dim3(kThreads), 0, st, static_cast<const double2 *>(a),
                           static_cast<const double2 *>(b), n * 12, part);
    else
        hipLaunchKernelGGL(k_dot_flat<double2>, dim3(np), dim3(kThreads), 0, st, static_cast<const double2 *>(a),
                           static_cast<const double2 *>(a), n * 12, part);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(kThreads), 0, st, part, np, part + kRedBlocks, 0);
    HIPCHK(hipGetLastError());
    double h = 0.0;
    HIPCHK(hipMemcpyAsync(&h, part + kRedBlocks, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *result = h;
    return hipSuccess;
}

}  // namespace gridmi
