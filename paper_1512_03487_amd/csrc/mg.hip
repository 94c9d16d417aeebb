// Two-level aggregation multigrid for the Wilson operator D = (4 + m) - H/2 and the generic
// coarse stencil it runs on. The paper's stencil support is illustrated by exactly such a
// coarse-grid operator of an adaptive multigrid inverter (Section 2.4), and multigrid-
// preconditioned GCR is among its algorithms (Section 4); the construction below is the standard
// one, with these conventions:
//
//   aggregates  blocks of b = (bx, by, bz, bt) fine sites, coarse extents Lc = L / b (periodic);
//   basis       nvec fine vectors, orthonormalised per aggregate and chirality (spins 0,1 / 2,3)
//               by Gram-Schmidt in the order k = 0, 1, ...; coarse component n = chi nvec + k,
//               N = 2 nvec per coarse site;
//   P, R = P^+  prolongation (P v)(x) = sum_k phi_k(x)|chi v(xc)[chi nvec + k], restriction its adjoint;
//   A_c = R D P as a 9-point stencil (A_c v)(xc) = sum_d A_d(xc) v(xc + e_d), d = 0 self,
//               1 + 2 mu (+mu), 2 + 2 mu (-mu); a hop from fine x in +mu leaves the aggregate
//               iff x_mu mod b_mu = b_mu - 1 (then it belongs to A_{1+2mu}, else to A_0).
//               Storage [xc][d][column j][row i] complex double, so that lanes over rows read
//               contiguous memory; A_c^+ = G5 A_c G5 with G5 = +1 / -1 on the two chiralities.
//   K(r)        one two-level cycle: r_c = R r, at most n_c CGNR iterations on A_c from zero
//               (stopping below tol_c times the starting normal residual), z = P e_c, then nu
//               minimal-residual steps on D z = r;
//   solver      flexible GCR(m) with K, modified Gram-Schmidt on the w = D z, true residual at
//               every restart and at the end.
// With params.graph the coarse solve of a cycle (a fixed kernel sequence: its control stays on the
// device) is recorded once per solve and replayed in every cycle.
//
// The coarse CGNR keeps its scalars on the device (per-block partial sums re-summed in a fixed
// order by every block of the next kernel, a stop flag read by every kernel), so a cycle costs
// no host synchronisation below the fine level; the outer GCR reads its inner products back.
#include <math.h>
#include <string.h>

#include <chrono>

#include "device.h"
#include "launch.h"

namespace gridmi {

namespace {

constexpr int kMgThreads = 256;
constexpr int kMgParts = 1024;     // maximum per-block partials of a fine-vector reduction

struct MgDims {
    int L[4];      // fine extents
    int b[4];      // aggregate extents
    int Lc[4];     // coarse extents
    int vol;       // fine volume
    int vc;        // coarse volume
    int nb;        // fine sites per aggregate
    int nvec;
    int N;
};

__device__ __forceinline__ double2 cmul2(double2 a, double2 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ double2 cmulc2(double2 a, double2 b) {   // conj(a) b
    return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double2 add2(double2 a, double2 b) { return {a.x + b.x, a.y + b.y}; }

// Coarse neighbour of xc in stencil direction d (0 self, 1 + 2 mu: +mu, 2 + 2 mu: -mu).
__device__ __forceinline__ int coarse_nb(const int Lc[4], int xc, int d) {
    if (d == 0) return xc;
    const int mu = (d - 1) >> 1;
    const bool fwd = ((d - 1) & 1) == 0;
    int stride = 1;
    for (int m = 0; m < mu; ++m) stride *= Lc[m];
    const int c = (xc / stride) % Lc[mu];
    const int c2 = fwd ? (c + 1 == Lc[mu] ? 0 : c + 1) : (c == 0 ? Lc[mu] - 1 : c - 1);
    return xc + (c2 - c) * stride;
}

__device__ __forceinline__ int opposite(int d) { return d == 0 ? 0 : (((d - 1) & 1) ? d - 1 : d + 1); }

// Fine site of in-aggregate index f of coarse site xc (f: x fastest within the block).
__device__ __forceinline__ int fine_site(const MgDims &m, int xc, int f, int x[4]) {
    int r = xc, q = f;
    for (int mu = 0; mu < 4; ++mu) {
        const int c = r % m.Lc[mu];
        r /= m.Lc[mu];
        const int o = q % m.b[mu];
        q /= m.b[mu];
        x[mu] = c * m.b[mu] + o;
    }
    return x[0] + m.L[0] * (x[1] + m.L[1] * (x[2] + m.L[2] * x[3]));
}

__device__ __forceinline__ int coarse_of(const MgDims &m, int x4) {
    int r = x4, xc = 0, stride = 1;
    for (int mu = 0; mu < 4; ++mu) {
        const int c = r % m.L[mu];
        r /= m.L[mu];
        xc += (c / m.b[mu]) * stride;
        stride *= m.Lc[mu];
    }
    return xc;
}

// Sum of one double2 per thread over the block, in a fixed order; every thread gets the result.
__device__ double2 block_sum2(double2 v, double2 *sm) {
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] = add2(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    const double2 r = sm[0];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------------------------
// Generic coarse stencil: one block per coarse site; thread (group g, row i) sums the (d, j) pairs
// p = g, g + G, ... of the 9 N products A_d[i][j] v(xc + e_d)[j]; the G partial rows are then
// added in a fixed order. g5: apply G5 to the input and the output (A_c^+ = G5 A_c G5).
// dag: the true adjoint, (A^+ v)(xc) = sum_d A_d(xc - e_d)^+ v(xc - e_d).
// ctl (nullable): skip the launch when ctl[1 + par] <= ctl[0] (the coarse solver has converged).
// TA: the element type of A (double2, or float2 for the FP32 copy the FP32 cycle reads; the
// products and sums are FP64 either way).
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ double2 ld2(const double2 &v) { return v; }
__device__ __forceinline__ double2 ld2(const float2 &v) { return {double(v.x), double(v.y)}; }

struct CoarseGeo {
    int Lc[4];
    int vc;
    int N;
    int nvec;   // G5 split (N / 2)
};

template <typename TA>
__global__ void __launch_bounds__(kMgThreads)
k_coarse_stencil(const TA *__restrict__ A, const double2 *__restrict__ v, double2 *__restrict__ out, CoarseGeo cg,
                 int dag, int g5, const double *__restrict__ ctl, int par) {
    if (ctl && ctl[1 + par] <= ctl[0]) return;
    __shared__ double2 vnb[9 * 64];
    __shared__ double2 part[kMgThreads];
    const int xc = blockIdx.x, N = cg.N, t = threadIdx.x;
    const int G = kMgThreads / N;
    for (int e = t; e < 9 * N; e += kMgThreads) {
        const int d = e / N, j = e - d * N;
        const int y = coarse_nb(cg.Lc, xc, dag ? opposite(d) : d);
        double2 w = v[static_cast<size_t>(y) * N + j];
        if (g5 && j >= cg.nvec) w = {-w.x, -w.y};
        vnb[e] = w;
    }
    __syncthreads();
    const int g = t / N, i = t - g * N;
    double2 acc = {0.0, 0.0};
    if (g < G) {
        for (int p = g; p < 9 * N; p += G) {
            const int d = p / N, j = p - d * N;
            if (!dag) {
                const double2 a = ld2(A[((static_cast<size_t>(xc) * 9 + d) * N + j) * N + i]);
                acc = add2(acc, cmul2(a, vnb[p]));
            } else {
                const int y = coarse_nb(cg.Lc, xc, opposite(d));
                const double2 a = ld2(A[((static_cast<size_t>(y) * 9 + d) * N + i) * N + j]);
                acc = add2(acc, cmulc2(a, vnb[p]));
            }
        }
    }
    part[t] = acc;
    __syncthreads();
    if (t < N) {
        double2 s = part[t];
        for (int gg = 1; gg < G; ++gg) s = add2(s, part[gg * N + t]);
        if (g5 && t >= cg.nvec) s = {-s.x, -s.y};
        out[static_cast<size_t>(xc) * N + t] = s;
    }
}

hipError_t coarse_stencil(const void *A, const void *v, void *out, const CoarseGeo &cg, int dag, int g5,
                          const double *ctl, int par, hipStream_t st, bool a32 = false) {
    if (a32)
        hipLaunchKernelGGL(k_coarse_stencil<float2>, dim3(cg.vc), dim3(kMgThreads), 0, st,
                           static_cast<const float2 *>(A), static_cast<const double2 *>(v),
                           static_cast<double2 *>(out), cg, dag, g5, ctl, par);
    else
        hipLaunchKernelGGL(k_coarse_stencil<double2>, dim3(cg.vc), dim3(kMgThreads), 0, st,
                           static_cast<const double2 *>(A), static_cast<const double2 *>(v),
                           static_cast<double2 *>(out), cg, dag, g5, ctl, par);
    return hipGetLastError();
}

// out[i] = (float2)in[i], i < n (the FP32 copy of the coarse operator).
__global__ void __launch_bounds__(256) k_narrow2(const double2 *__restrict__ in, float2 *__restrict__ out, long n) {
    const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = {static_cast<float>(in[i].x), static_cast<float>(in[i].y)};
}

// ---------------------------------------------------------------------------------------------
// Restriction, prolongation and the blockwise Gram-Schmidt of the basis.
// vecs: nvec fine fields [k][V][4][3] complex double.
// ---------------------------------------------------------------------------------------------
// The basis may be read from an FP32 copy (TB = float2, the cycle in FP32); arithmetic in FP64.

template <typename TB>
__global__ void __launch_bounds__(kMgThreads)
k_mg_restrict(const TB *__restrict__ vecs, const double2 *__restrict__ psi, double2 *__restrict__ vc, MgDims m) {
    __shared__ double2 part[kMgThreads];
    const int xc = blockIdx.x, N = m.N, t = threadIdx.x;
    const int G = kMgThreads / N;
    const int g = t / N, n = t - g * N;
    double2 acc = {0.0, 0.0};
    if (g < G) {
        const int chi = n / m.nvec, k = n - chi * m.nvec;
        const TB *ph = vecs + static_cast<size_t>(k) * m.vol * 12;
        for (int f = g; f < m.nb; f += G) {
            int x[4];
            const size_t o = static_cast<size_t>(fine_site(m, xc, f, x)) * 12 + chi * 6;
#pragma unroll
            for (int e = 0; e < 6; ++e) acc = add2(acc, cmulc2(ld2(ph[o + e]), psi[o + e]));
        }
    }
    part[t] = acc;
    __syncthreads();
    if (t < N) {
        double2 s = part[t];
        for (int gg = 1; gg < G; ++gg) s = add2(s, part[gg * N + t]);
        vc[static_cast<size_t>(xc) * N + t] = s;
    }
}

template <typename TB>
__global__ void __launch_bounds__(kMgThreads)
k_mg_prolong(const TB *__restrict__ vecs, const double2 *__restrict__ vc, double2 *__restrict__ out, MgDims m) {
    const long id = static_cast<long>(blockIdx.x) * kMgThreads + threadIdx.x;
    if (id >= static_cast<long>(m.vol) * 12) return;
    const int x4 = static_cast<int>(id / 12), e = static_cast<int>(id - static_cast<long>(x4) * 12);
    const int chi = e / 6;
    const double2 *c = vc + static_cast<size_t>(coarse_of(m, x4)) * m.N + chi * m.nvec;
    double2 acc = {0.0, 0.0};
    for (int k = 0; k < m.nvec; ++k) acc = add2(acc, cmul2(ld2(vecs[static_cast<size_t>(k) * m.vol * 12 + id]), c[k]));
    out[id] = acc;
}

// One block per (aggregate, chirality): modified Gram-Schmidt of the nvec restrictions, in place.
__global__ void __launch_bounds__(kMgThreads) k_mg_orth(double2 *__restrict__ vecs, MgDims m) {
    __shared__ double2 sm[kMgThreads];
    const int xc = blockIdx.x >> 1, chi = blockIdx.x & 1;
    const int E = m.nb * 6;
    const size_t vs = static_cast<size_t>(m.vol) * 12;
    auto at = [&](int e) -> size_t {
        const int f = e / 6, r = e - f * 6;
        int x[4];
        return static_cast<size_t>(fine_site(m, xc, f, x)) * 12 + chi * 6 + r;
    };
    for (int k = 0; k < m.nvec; ++k) {
        double2 *vk = vecs + k * vs;
        for (int j = 0; j < k; ++j) {
            const double2 *qj = vecs + j * vs;
            double2 c = {0.0, 0.0};
            for (int e = threadIdx.x; e < E; e += kMgThreads) {
                const size_t o = at(e);
                c = add2(c, cmulc2(qj[o], vk[o]));
            }
            c = block_sum2(c, sm);
            for (int e = threadIdx.x; e < E; e += kMgThreads) {
                const size_t o = at(e);
                const double2 p = cmul2(c, qj[o]);
                vk[o] = {vk[o].x - p.x, vk[o].y - p.y};
            }
            __syncthreads();
        }
        double2 nn = {0.0, 0.0};
        for (int e = threadIdx.x; e < E; e += kMgThreads) {
            const size_t o = at(e);
            nn.x += vk[o].x * vk[o].x + vk[o].y * vk[o].y;
        }
        nn = block_sum2(nn, sm);
        const double inv = nn.x > 0.0 ? 1.0 / sqrt(nn.x) : 0.0;
        for (int e = threadIdx.x; e < E; e += kMgThreads) {
            const size_t o = at(e);
            vk[o] = {vk[o].x * inv, vk[o].y * inv};
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------------
// Galerkin coarse operator, one column j = (chi', k') at a time.
// k_mg_dirhop: H[d][x] = -1/2 (1 - gamma_mu) U_mu(x) t(x + mu) (d = 2 mu) or
// -1/2 (1 + gamma_mu) U_mu(x - mu)^+ t(x - mu) (d = 2 mu + 1), t = phi_k' on the spins of chi'.
// Chiral basis: gamma_mu = [[0, A_mu], [A_mu^+, 0]], A = -i s1, -i s2, -i s3, 1.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void gamma_apply(int mu, const double2 in[4][3], double2 out[4][3]) {
    for (int c = 0; c < 3; ++c) {
        const double2 u0 = in[0][c], u1 = in[1][c], l0 = in[2][c], l1 = in[3][c];
        double2 a0, a1, b0, b1;   // upper = A lower, lower = A^+ upper
        if (mu == 0) {            // A = [[0, -i], [-i, 0]], A^+ = [[0, i], [i, 0]]
            a0 = {l1.y, -l1.x};
            a1 = {l0.y, -l0.x};
            b0 = {-u1.y, u1.x};
            b1 = {-u0.y, u0.x};
        } else if (mu == 1) {     // A = [[0, -1], [1, 0]], A^+ = [[0, 1], [-1, 0]]
            a0 = {-l1.x, -l1.y};
            a1 = l0;
            b0 = u1;
            b1 = {-u0.x, -u0.y};
        } else if (mu == 2) {     // A = [[-i, 0], [0, i]], A^+ = [[i, 0], [0, -i]]
            a0 = {l0.y, -l0.x};
            a1 = {-l1.y, l1.x};
            b0 = {-u0.y, u0.x};
            b1 = {u1.y, -u1.x};
        } else {                  // A = 1
            a0 = l0;
            a1 = l1;
            b0 = u0;
            b1 = u1;
        }
        out[0][c] = a0;
        out[1][c] = a1;
        out[2][c] = b0;
        out[3][c] = b1;
    }
}

__global__ void __launch_bounds__(kMgThreads)
k_mg_dirhop(const double2 *__restrict__ U, const double2 *__restrict__ phi, int chi, double2 *__restrict__ H, GeomDev g) {
    const long id = static_cast<long>(blockIdx.x) * kMgThreads + threadIdx.x;
    if (id >= static_cast<long>(g.vol) * 8) return;
    const int d = static_cast<int>(id % 8), x4 = static_cast<int>(id / 8);
    const int mu = d >> 1;
    const bool fwd = (d & 1) == 0;
    int nb[8];
    neighbours(g, x4, nb);
    const int y = fwd ? nb[2 * mu] : nb[2 * mu + 1];
    const double2 *u = U + (static_cast<size_t>(fwd ? x4 : y) * 4 + mu) * 9;
    double2 t[4][3], ut[4][3], gt[4][3];
    for (int s = 0; s < 4; ++s)
        for (int c = 0; c < 3; ++c)
            t[s][c] = ((s >> 1) == chi) ? phi[static_cast<size_t>(y) * 12 + s * 3 + c] : double2{0.0, 0.0};
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
            double2 acc = {0.0, 0.0};
            for (int b = 0; b < 3; ++b)
                acc = add2(acc, fwd ? cmul2(u[a * 3 + b], t[s][b]) : cmulc2(u[b * 3 + a], t[s][b]));
            ut[s][a] = acc;
        }
    gamma_apply(mu, ut, gt);
    const double sg = fwd ? -1.0 : 1.0;   // (1 - gamma) forward, (1 + gamma) backward
    double2 *o = H + (static_cast<size_t>(d) * g.vol + x4) * 12;
    for (int s = 0; s < 4; ++s)
        for (int c = 0; c < 3; ++c)
            o[s * 3 + c] = {-0.5 * (ut[s][c].x + sg * gt[s][c].x), -0.5 * (ut[s][c].y + sg * gt[s][c].y)};
}

// Column j of every A_d(xc): thread (group g, row n) over the aggregate's fine sites.
__global__ void __launch_bounds__(kMgThreads)
k_mg_coarse_col(const double2 *__restrict__ vecs, const double2 *__restrict__ phi, int chi2,
                const double2 *__restrict__ H, double2 *__restrict__ A, MgDims m, double diag, int j) {
    __shared__ double2 part[kMgThreads];
    const int xc = blockIdx.x, N = m.N, t = threadIdx.x;
    const int G = kMgThreads / N;
    const int g = t / N, n = t - g * N;
    double2 acc[9];
    for (int d = 0; d < 9; ++d) acc[d] = {0.0, 0.0};
    if (g < G) {
        const int chi = n / m.nvec, k = n - chi * m.nvec;
        const double2 *ph = vecs + static_cast<size_t>(k) * m.vol * 12;
        for (int f = g; f < m.nb; f += G) {
            int x[4];
            const int x4 = fine_site(m, xc, f, x);
            const size_t o = static_cast<size_t>(x4) * 12 + chi * 6;
            double2 q[6];
            for (int e = 0; e < 6; ++e) q[e] = ph[o + e];
            if (chi == chi2)
                for (int e = 0; e < 6; ++e) {
                    const double2 p = cmulc2(q[e], phi[o + e]);
                    acc[0] = {acc[0].x + diag * p.x, acc[0].y + diag * p.y};
                }
            for (int d = 0; d < 8; ++d) {
                const int mu = d >> 1;
                const bool fwd = (d & 1) == 0;
                const int r = x[mu] % m.b[mu];
                const bool face = fwd ? (r == m.b[mu] - 1) : (r == 0);
                const double2 *h = H + (static_cast<size_t>(d) * m.vol + x4) * 12 + chi * 6;
                double2 c = {0.0, 0.0};
                for (int e = 0; e < 6; ++e) c = add2(c, cmulc2(q[e], h[e]));
                const int dd = face ? 1 + d : 0;
                acc[dd] = add2(acc[dd], c);
            }
        }
    }
    for (int d = 0; d < 9; ++d) {
        part[t] = acc[d];
        __syncthreads();
        if (t < N) {
            double2 s = part[t];
            for (int gg = 1; gg < G; ++gg) s = add2(s, part[gg * N + t]);
            A[((static_cast<size_t>(xc) * 9 + d) * N + j) * N + t] = s;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------------
// Vector kernels (complex double, n elements).
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kMgThreads)
k_zdot_part(const double2 *__restrict__ a, const double2 *__restrict__ b, long n, double2 *__restrict__ part) {
    __shared__ double2 sm[kMgThreads];
    double2 acc = {0.0, 0.0};
    for (long i = static_cast<long>(blockIdx.x) * kMgThreads + threadIdx.x; i < n;
         i += static_cast<long>(gridDim.x) * kMgThreads)
        acc = add2(acc, cmulc2(a[i], b[i]));
    acc = block_sum2(acc, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Two inner products in one pass: part[b] = <a1, b1>, part[kMgParts + b] = <a2, b2>.
__global__ void __launch_bounds__(kMgThreads)
k_zdot2_part(const double2 *__restrict__ a1, const double2 *__restrict__ b1, const double2 *__restrict__ a2,
             const double2 *__restrict__ b2, long n, double2 *__restrict__ part) {
    __shared__ double2 sm[kMgThreads];
    double2 c1 = {0.0, 0.0}, c2 = {0.0, 0.0};
    for (long i = static_cast<long>(blockIdx.x) * kMgThreads + threadIdx.x; i < n;
         i += static_cast<long>(gridDim.x) * kMgThreads) {
        c1 = add2(c1, cmulc2(a1[i], b1[i]));
        c2 = add2(c2, cmulc2(a2[i], b2[i]));
    }
    c1 = block_sum2(c1, sm);
    c2 = block_sum2(c2, sm);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = c1;
        part[kMgParts + blockIdx.x] = c2;
    }
}

// FP32 forms for the FP32 smoother (inner products accumulated in FP64).
__device__ __forceinline__ double2 up2(float2 v) { return {double(v.x), double(v.y)}; }
__global__ void __launch_bounds__(kMgThreads)
k_zdot2_part_f(const float2 *__restrict__ a1, const float2 *__restrict__ b1, const float2 *__restrict__ a2,
               const float2 *__restrict__ b2, long n, double2 *__restrict__ part) {
    __shared__ double2 sm[kMgThreads];
    double2 c1 = {0.0, 0.0}, c2 = {0.0, 0.0};
    for (long i = static_cast<long>(blockIdx.x) * kMgThreads + threadIdx.x; i < n;
         i += static_cast<long>(gridDim.x) * kMgThreads) {
        c1 = add2(c1, cmulc2(up2(a1[i]), up2(b1[i])));
        c2 = add2(c2, cmulc2(up2(a2[i]), up2(b2[i])));
    }
    c1 = block_sum2(c1, sm);
    c2 = block_sum2(c2, sm);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = c1;
        part[kMgParts + blockIdx.x] = c2;
    }
}

// minimal-residual step in FP32: alpha = sc[0] / Re sc[1]; y += alpha x, y2 -= alpha x2
__global__ void __launch_bounds__(kMgThreads)
k_mr_step_f(float2 *__restrict__ y, const float2 *__restrict__ x, float2 *__restrict__ y2, const float2 *__restrict__ x2,
            const double2 *__restrict__ sc, long n) {
    const float ar = static_cast<float>(sc[0].x / sc[1].x), ai = static_cast<float>(sc[0].y / sc[1].x);
    for (long i = static_cast<long>(blockIdx.x) * kMgThreads + threadIdx.x; i < n;
         i += static_cast<long>(gridDim.x) * kMgThreads) {
        const float2 xv = x[i], x2v = x2[i];
        float2 a = y[i], b = y2[i];
        a.x += ar * xv.x - ai * xv.y;
        a.y += ar * xv.y + ai * xv.x;
        b.x -= ar * x2v.x - ai * x2v.y;
        b.y -= ar * x2v.y + ai * x2v.x;
        y[i] = a;
        y2[i] = b;
    }
}

// out = a - b (FP32)
__global__ void __launch_bounds__(kMgThreads)
k_zsub_f(float2 *__restrict__ out, const float2 *__restrict__ a, const float2 *__restrict__ b, long n) {
    for (long i = static_cast<long>(blockIdx.x) * kMgThreads + threadIdx.x; i < n;
         i += static_cast<long>(gridDim.x) * kMgThreads)
        out[i] = {a[i].x - b[i].x, a[i].y - b[i].y};
}

// One block: thread t adds partials t, t + 256, ... then a tree sum (fixed order).
__global__ void __launch_bounds__(kMgThreads)
k_zsum(const double2 *__restrict__ part, int np, double2 *__restrict__ out) {
    __shared__ double2 sm[kMgThreads];
    double2 s = {0.0, 0.0};
    for (int i = threadIdx.x; i < np; i += kMgThreads) s = add2(s, part[i]);
    s = block_sum2(s, sm);
    if (threadIdx.x == 0) *out = s;
}

// y += a x; if x2: y2 += a2 x2 (two independent updates in one pass)
__global__ void __launch_bounds__(kMgThreads)
k_zaxpy2(double2 *__restrict__ y, const double2 *__restrict__ x, double2 a, double2 *__restrict__ y2,
         const double2 *__restrict__ x2, double2 a2, long n) {
    for (long i = static_cast<long>(blockIdx.x) * kMgThreads + threadIdx.x; i < n;
         i += static_cast<long>(gridDim.x) * kMgThreads) {
        y[i] = add2(y[i], cmul2(a, x[i]));
        if (y2) y2[i] = add2(y2[i], cmul2(a2, x2[i]));
    }
}

// The same two updates with the coefficient taken from device scalars sc (no read-back):
// mode 0: y += -sc[0] x, y2 += -sc[0] x2 (Gram-Schmidt, sc[0] = <x, y>);
// mode 1: alpha = sc[0] / Re sc[1]; y += alpha x, y2 += -alpha x2 (minimal residual,
//         sc[0] = <t, s>, sc[1] = <t, t>).
__global__ void __launch_bounds__(kMgThreads)
k_zaxpy2_dev(double2 *__restrict__ y, const double2 *__restrict__ x, double2 *__restrict__ y2,
             const double2 *__restrict__ x2, const double2 *__restrict__ sc, int mode, long n) {
    double2 a, a2;
    if (mode == 0) {
        a = {-sc[0].x, -sc[0].y};
        a2 = a;
    } else {
        a = {sc[0].x / sc[1].x, sc[0].y / sc[1].x};
        a2 = {-a.x, -a.y};
    }
    for (long i = static_cast<long>(blockIdx.x) * kMgThreads + threadIdx.x; i < n;
         i += static_cast<long>(gridDim.x) * kMgThreads) {
        y[i] = add2(y[i], cmul2(a, x[i]));
        y2[i] = add2(y2[i], cmul2(a2, x2[i]));
    }
}

// out = a - b
__global__ void __launch_bounds__(kMgThreads)
k_zsub(double2 *__restrict__ out, const double2 *__restrict__ a, const double2 *__restrict__ b, long n) {
    for (long i = static_cast<long>(blockIdx.x) * kMgThreads + threadIdx.x; i < n;
         i += static_cast<long>(gridDim.x) * kMgThreads)
        out[i] = {a[i].x - b[i].x, a[i].y - b[i].y};
}

// out = gamma5 v on a fine field (n = 12 V complex elements; spins 2, 3 change sign); out may be v
__global__ void __launch_bounds__(kMgThreads) k_zg5(double2 *out, const double2 *v, long n) {
    for (long i = static_cast<long>(blockIdx.x) * kMgThreads + threadIdx.x; i < n;
         i += static_cast<long>(gridDim.x) * kMgThreads) {
        const double sg = (i % 12) >= 6 ? -1.0 : 1.0;
        out[i] = {sg * v[i].x, sg * v[i].y};
    }
}

// y *= s, y2 *= s
__global__ void __launch_bounds__(kMgThreads)
k_zscale2(double2 *__restrict__ y, double2 *__restrict__ y2, double s, long n) {
    for (long i = static_cast<long>(blockIdx.x) * kMgThreads + threadIdx.x; i < n;
         i += static_cast<long>(gridDim.x) * kMgThreads) {
        y[i] = {y[i].x * s, y[i].y * s};
        if (y2) y2[i] = {y2[i].x * s, y2[i].y * s};
    }
}

// ---------------------------------------------------------------------------------------------
// Coarse CGNR with device scalars. ctl[0] = stop (tol_c^2 rho_0), ctl[1 + P] = rho entering an
// iteration of parity P. Partials: pq (<p, q>) and rr (|r|^2), np per set, in `part`.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ double sum_parts(const double *p, int np) {
    double s = 0.0;
    for (int i = 0; i < np; ++i) s += p[i];
    return s;
}

__global__ void __launch_bounds__(kMgThreads)
k_cdot_re(const double2 *__restrict__ a, const double2 *__restrict__ b, long n, double *__restrict__ part,
          const double *__restrict__ ctl, int par) {
    if (ctl && ctl[1 + par] <= ctl[0]) return;
    __shared__ double2 sm[kMgThreads];
    double2 acc = {0.0, 0.0};
    for (long i = static_cast<long>(blockIdx.x) * kMgThreads + threadIdx.x; i < n;
         i += static_cast<long>(gridDim.x) * kMgThreads)
        acc.x += a[i].x * b[i].x + a[i].y * b[i].y;
    acc = block_sum2(acc, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = acc.x;
}

// p = r; e = 0 (a kernel rather than a copy and a fill, so the sequence can be recorded)
__global__ void __launch_bounds__(kMgThreads)
k_ccg_start(double2 *__restrict__ p, const double2 *__restrict__ r, double2 *__restrict__ e, long n) {
    for (long i = static_cast<long>(blockIdx.x) * kMgThreads + threadIdx.x; i < n;
         i += static_cast<long>(gridDim.x) * kMgThreads) {
        p[i] = r[i];
        e[i] = {0.0, 0.0};
    }
}

// rho_0 = sum of parts; ctl[0] = tol^2 rho_0; ctl[1] = rho_0
__global__ void k_ccg_init(const double *__restrict__ part, int np, double tol, double *__restrict__ ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double r0 = sum_parts(part, np);
        ctl[0] = tol * tol * r0;
        ctl[1] = r0;
    }
}

// alpha = rho / <p, q>; e += alpha p; r -= alpha q; |r|^2 partials
__global__ void __launch_bounds__(kMgThreads)
k_ccg_update(double2 *__restrict__ e, double2 *__restrict__ r, const double2 *__restrict__ p,
             const double2 *__restrict__ q, long n, const double *__restrict__ pq, double *__restrict__ rr, int np,
             const double *__restrict__ ctl, int par) {
    if (ctl[1 + par] <= ctl[0]) return;
    __shared__ double2 sm[kMgThreads];
    const double alpha = ctl[1 + par] / sum_parts(pq, np);
    double2 acc = {0.0, 0.0};
    for (long i = static_cast<long>(blockIdx.x) * kMgThreads + threadIdx.x; i < n;
         i += static_cast<long>(gridDim.x) * kMgThreads) {
        e[i] = {e[i].x + alpha * p[i].x, e[i].y + alpha * p[i].y};
        const double2 ri = {r[i].x - alpha * q[i].x, r[i].y - alpha * q[i].y};
        r[i] = ri;
        acc.x += ri.x * ri.x + ri.y * ri.y;
    }
    acc = block_sum2(acc, sm);
    if (threadIdx.x == 0) rr[blockIdx.x] = acc.x;
}

// beta = rho' / rho; p = r + beta p; ctl[1 + (par ^ 1)] = rho' (or rho when already stopped)
__global__ void __launch_bounds__(kMgThreads)
k_ccg_p(double2 *__restrict__ p, const double2 *__restrict__ r, long n, const double *__restrict__ rr, int np,
        double *__restrict__ ctl, int par) {
    const double rho = ctl[1 + par];
    if (rho <= ctl[0]) {
        if (blockIdx.x == 0 && threadIdx.x == 0) ctl[1 + (par ^ 1)] = rho;
        return;
    }
    const double rho2 = sum_parts(rr, np);
    const double beta = rho2 / rho;
    for (long i = static_cast<long>(blockIdx.x) * kMgThreads + threadIdx.x; i < n;
         i += static_cast<long>(gridDim.x) * kMgThreads)
        p[i] = {r[i].x + beta * p[i].x, r[i].y + beta * p[i].y};
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl[1 + (par ^ 1)] = rho2;
}

int vec_blocks(long n) {
    const long b = (n + kMgThreads - 1) / kMgThreads;
    return static_cast<int>(b < kMgParts ? (b > 0 ? b : 1) : kMgParts);
}

#define MGCHK(x)                                \
    do {                                        \
        hipError_t e_ = (x);                    \
        if (e_ != hipSuccess) return e_;        \
    } while (0)

// Workspace layout of the solver and the setup (bytes, 256-aligned regions).
struct MgLayout {
    size_t fv, cv;          // one fine / coarse vector
    size_t r, s, t, u, Z, W;   // fine (Z, W: restart vectors each; u: the pCG preconditioner's)
    size_t rc, ec, cr, cp, cq, cq1;
    size_t part, scal;      // 2 x kMgParts double2, 16 double2
    size_t z32 = 0, s32 = 0, t32 = 0, r32 = 0, u32 = 0, v32 = 0, a32 = 0;   // FP32 cycle (cycle_prec GRID_F32)
    size_t solve_end;
    size_t H, xb, cg, setup_end;   // setup: 8 directional fields, CG solution, CG workspace
    size_t total;
};

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

MgLayout mg_layout(const MgDims &m, int restart, int setup_prec, int cycle_prec) {
    MgLayout L;
    L.fv = al256(static_cast<size_t>(m.vol) * 192);
    L.cv = al256(static_cast<size_t>(m.vc) * m.N * 16);
    size_t o = 0;
    L.r = o; o += L.fv;
    L.s = o; o += L.fv;
    L.t = o; o += L.fv;
    L.u = o; o += L.fv;
    L.Z = o; o += L.fv * restart;
    L.W = o; o += L.fv * restart;
    L.rc = o; o += L.cv;
    L.ec = o; o += L.cv;
    L.cr = o; o += L.cv;
    L.cp = o; o += L.cv;
    L.cq = o; o += L.cv;
    L.cq1 = o; o += L.cv;
    L.part = o; o += al256(2 * kMgParts * sizeof(double2));
    L.scal = o; o += al256(16 * sizeof(double2));
    if (cycle_prec == GRID_F32) {
        // FP32 smoother: z, s, t, r in FP32 and the FP32 links
        const size_t hv = al256(static_cast<size_t>(m.vol) * 96);
        L.z32 = o; o += hv;
        L.s32 = o; o += hv;
        L.t32 = o; o += hv;
        L.r32 = o; o += hv;
        L.u32 = o; o += al256(static_cast<size_t>(m.vol) * 4 * 72);
        L.v32 = o; o += al256(static_cast<size_t>(m.nvec) * m.vol * 96);   // the basis for R and P
        L.a32 = o; o += al256(static_cast<size_t>(m.vc) * 9 * m.N * m.N * sizeof(float2));   // coarse A
    }
    L.solve_end = o;
    o = 0;
    L.H = o; o += 8 * L.fv;
    L.xb = o; o += L.fv;
    L.cg = o;
    GeomDev g;
    for (int mu = 0; mu < 4; ++mu) g.L[mu] = m.L[mu];
    g.Ls = 1;
    g.vol = m.vol;
    g.n5 = m.vol;
    o += al256(cg_workspace_bytes(g, setup_prec, GRID_L18));
    L.setup_end = o;
    L.total = L.solve_end > L.setup_end ? L.solve_end : L.setup_end;
    return L;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------------------------
struct MgCtx {
    MgDims m;
    GeomDev g;
    double mass;
    const grid_mg_params *p;
    char *ws;
    MgLayout L;
    hipStream_t st;
    long nf, ncv;   // complex elements of a fine / coarse vector
    // the coarse solve recorded once per solve (params.graph): executable and recording stream
    hipGraphExec_t coarse_exec = nullptr;
    hipStream_t rec = nullptr;

    double2 *f(size_t off) const { return reinterpret_cast<double2 *>(ws + off); }
    float2 *h(size_t off) const { return reinterpret_cast<float2 *>(ws + off); }
    double2 *part() const { return f(L.part); }
    double2 *scal() const { return f(L.scal); }

    // the FP32 smoother's D (FP32 links converted once per solve) and vector steps
    hipError_t D32(const void *in, void *out) const {
        DhopArgs a;
        a.U = ws + L.u32;
        a.psi = in;
        a.psi_scale = nullptr;
        a.out = out;
        a.out_scale = nullptr;
        a.g = g;
        a.prec = GRID_F32;
        a.link_fmt = GRID_L18;
        a.kind = GRID_WILSON;
        a.dag = 0;
        a.diag = 4.0 + mass;
        a.mf = 0.0;
        a.stream = st;
        return launch_dhop(a);
    }
    hipError_t mr_step_f(float2 *z, float2 *s, const float2 *t, long n) const {
        const int nb = vec_blocks(n);
        hipLaunchKernelGGL(k_zdot2_part_f, dim3(nb), dim3(kMgThreads), 0, st, t, s, t, t, n, part());
        MGCHK(hipGetLastError());
        hipLaunchKernelGGL(k_zsum, dim3(1), dim3(kMgThreads), 0, st, part(), nb, scal());
        MGCHK(hipGetLastError());
        hipLaunchKernelGGL(k_zsum, dim3(1), dim3(kMgThreads), 0, st, part() + kMgParts, nb, scal() + 1);
        MGCHK(hipGetLastError());
        hipLaunchKernelGGL(k_mr_step_f, dim3(nb), dim3(kMgThreads), 0, st, z, s, s, t,
                           static_cast<const double2 *>(scal()), n);
        return hipGetLastError();
    }

    hipError_t D(const void *U, const void *in, void *out, int dag = 0) const {
        DhopArgs a;
        a.U = U;
        a.psi = in;
        a.psi_scale = nullptr;
        a.out = out;
        a.out_scale = nullptr;
        a.g = g;
        a.prec = GRID_F64;
        a.link_fmt = GRID_L18;
        a.kind = GRID_WILSON;
        a.dag = dag;
        a.diag = 4.0 + mass;
        a.mf = 0.0;
        a.stream = st;
        return launch_dhop(a);
    }
    // <a, b> over n complex elements, read back (waits for the stream)
    hipError_t zdot(const double2 *a, const double2 *b, long n, double2 *res) const {
        const int nb = vec_blocks(n);
        hipLaunchKernelGGL(k_zdot_part, dim3(nb), dim3(kMgThreads), 0, st, a, b, n, part());
        MGCHK(hipGetLastError());
        hipLaunchKernelGGL(k_zsum, dim3(1), dim3(kMgThreads), 0, st, part(), nb, scal());
        MGCHK(hipGetLastError());
        MGCHK(hipMemcpyAsync(res, scal(), sizeof(double2), hipMemcpyDeviceToHost, st));
        return hipStreamSynchronize(st);
    }
    // <a1, b1> and <a2, b2> in one pass and one read-back
    hipError_t zdot2(const double2 *a1, const double2 *b1, const double2 *a2, const double2 *b2, long n,
                     double2 res[2]) const {
        const int nb = vec_blocks(n);
        hipLaunchKernelGGL(k_zdot2_part, dim3(nb), dim3(kMgThreads), 0, st, a1, b1, a2, b2, n, part());
        MGCHK(hipGetLastError());
        hipLaunchKernelGGL(k_zsum, dim3(1), dim3(kMgThreads), 0, st, part(), nb, scal());
        MGCHK(hipGetLastError());
        hipLaunchKernelGGL(k_zsum, dim3(1), dim3(kMgThreads), 0, st, part() + kMgParts, nb, scal() + 1);
        MGCHK(hipGetLastError());
        MGCHK(hipMemcpyAsync(res, scal(), 2 * sizeof(double2), hipMemcpyDeviceToHost, st));
        return hipStreamSynchronize(st);
    }
    // <a, b> (and <a2, b2>) into the device scalars only, for a following axpy2_dev
    hipError_t zdot_dev(const double2 *a, const double2 *b, long n) const {
        const int nb = vec_blocks(n);
        hipLaunchKernelGGL(k_zdot_part, dim3(nb), dim3(kMgThreads), 0, st, a, b, n, part());
        MGCHK(hipGetLastError());
        hipLaunchKernelGGL(k_zsum, dim3(1), dim3(kMgThreads), 0, st, part(), nb, scal());
        return hipGetLastError();
    }
    hipError_t zdot2_dev(const double2 *a1, const double2 *b1, const double2 *a2, const double2 *b2, long n) const {
        const int nb = vec_blocks(n);
        hipLaunchKernelGGL(k_zdot2_part, dim3(nb), dim3(kMgThreads), 0, st, a1, b1, a2, b2, n, part());
        MGCHK(hipGetLastError());
        hipLaunchKernelGGL(k_zsum, dim3(1), dim3(kMgThreads), 0, st, part(), nb, scal());
        MGCHK(hipGetLastError());
        hipLaunchKernelGGL(k_zsum, dim3(1), dim3(kMgThreads), 0, st, part() + kMgParts, nb, scal() + 1);
        return hipGetLastError();
    }
    hipError_t axpy2_dev(double2 *y, const double2 *x, double2 *y2, const double2 *x2, int mode, long n) const {
        hipLaunchKernelGGL(k_zaxpy2_dev, dim3(vec_blocks(n)), dim3(kMgThreads), 0, st, y, x, y2, x2,
                           static_cast<const double2 *>(scal()), mode, n);
        return hipGetLastError();
    }
    hipError_t axpy2(double2 *y, const double2 *x, double2 a, double2 *y2, const double2 *x2, double2 a2, long n) const {
        hipLaunchKernelGGL(k_zaxpy2, dim3(vec_blocks(n)), dim3(kMgThreads), 0, st, y, x, a, y2, x2, a2, n);
        return hipGetLastError();
    }
    hipError_t sub(double2 *out, const double2 *a, const double2 *b, long n) const {
        hipLaunchKernelGGL(k_zsub, dim3(vec_blocks(n)), dim3(kMgThreads), 0, st, out, a, b, n);
        return hipGetLastError();
    }
    hipError_t g5(double2 *out, const double2 *v) const {
        hipLaunchKernelGGL(k_zg5, dim3(vec_blocks(nf)), dim3(kMgThreads), 0, st, out, v, nf);
        return hipGetLastError();
    }
};

static bool mg_dims(const GeomDev &g, const grid_mg_params &p, MgDims *m) {
    m->vol = g.vol;
    m->vc = 1;
    m->nb = 1;
    for (int mu = 0; mu < 4; ++mu) {
        m->L[mu] = g.L[mu];
        m->b[mu] = p.block[mu];
        if (p.block[mu] < 1 || g.L[mu] % p.block[mu]) return false;
        m->Lc[mu] = g.L[mu] / p.block[mu];
        m->vc *= m->Lc[mu];
        m->nb *= p.block[mu];
    }
    m->nvec = p.nvec;
    m->N = 2 * p.nvec;
    return true;
}

size_t mg_workspace_bytes(const GeomDev &g, const grid_mg_params &p) {
    MgDims m;
    if (!mg_dims(g, p, &m)) return 0;
    return mg_layout(m, p.restart, p.setup_prec, p.cycle_prec).total;
}

static CoarseGeo coarse_geo(const MgDims &m) {
    CoarseGeo c;
    for (int mu = 0; mu < 4; ++mu) c.Lc[mu] = m.Lc[mu];
    c.vc = m.vc;
    c.N = m.N;
    c.nvec = m.nvec;
    return c;
}

hipError_t launch_coarse_stencil(const void *A, const void *v, void *out, const int Lc[4], int N, int dag,
                                 hipStream_t st) {
    CoarseGeo c;
    c.vc = 1;
    for (int mu = 0; mu < 4; ++mu) {
        c.Lc[mu] = Lc[mu];
        c.vc *= Lc[mu];
    }
    c.N = N;
    c.nvec = N / 2;
    return coarse_stencil(A, v, out, c, dag, 0, nullptr, 0, st);
}

hipError_t launch_mg_restrict(const void *vecs, const void *psi, void *vc, const GeomDev &g, const grid_mg_params &p,
                              hipStream_t st) {
    MgDims m;
    mg_dims(g, p, &m);
    hipLaunchKernelGGL(k_mg_restrict<double2>, dim3(m.vc), dim3(kMgThreads), 0, st, static_cast<const double2 *>(vecs),
                       static_cast<const double2 *>(psi), static_cast<double2 *>(vc), m);
    return hipGetLastError();
}

hipError_t launch_mg_prolong(const void *vecs, const void *vc, void *psi, const GeomDev &g, const grid_mg_params &p,
                             hipStream_t st) {
    MgDims m;
    mg_dims(g, p, &m);
    const long n = static_cast<long>(m.vol) * 12;
    hipLaunchKernelGGL(k_mg_prolong<double2>, dim3(static_cast<unsigned>((n + kMgThreads - 1) / kMgThreads)), dim3(kMgThreads), 0,
                       st, static_cast<const double2 *>(vecs), static_cast<const double2 *>(vc),
                       static_cast<double2 *>(psi), m);
    return hipGetLastError();
}

hipError_t run_mg_basis(const void *U, void *vecs, const GeomDev &g, double mass, const grid_mg_params &p, void *ws,
                        hipStream_t st) {
    MgDims m;
    mg_dims(g, p, &m);
    const MgLayout L = mg_layout(m, p.restart, p.setup_prec, p.cycle_prec);
    char *w = static_cast<char *>(ws);
    double2 *V = static_cast<double2 *>(vecs);
    const long nf = static_cast<long>(m.vol) * 12;
    if (p.setup_rounds > 0 && p.setup_iters > 0) {
        grid_op op = {};
        op.kind = GRID_WILSON;
        op.mass = mass;
        grid_cg_params cp = {};
        cp.tol = 1e-300;
        cp.maxiter = p.setup_iters;
        cp.sloppy_prec = p.setup_prec;   // the near-null vectors need no FP64 iterations
        cp.link_fmt = GRID_L18;
        cp.delta = 0.1;
        cp.check_every = p.setup_iters;
        cp.graph = 0;
        double2 *x = reinterpret_cast<double2 *>(w + L.xb);
        double *part = reinterpret_cast<double *>(w + L.H);   // the directional fields are not used here
        for (int round = 0; round < p.setup_rounds; ++round)
            for (int k = 0; k < m.nvec; ++k) {
                double2 *vk = V + static_cast<size_t>(k) * nf;
                MGCHK(hipMemsetAsync(x, 0, static_cast<size_t>(nf) * sizeof(double2), st));
                grid_cg_stats cst;
                int status = 0;
                MGCHK(run_cg(U, vk, x, g, op, cp, w + L.cg, st, &cst, &status));
                double n2 = 0.0;
                MGCHK(norm2_diff(x, nullptr, m.vol, part, st, &n2));
                const double inv = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
                MGCHK(hipMemcpyAsync(vk, x, static_cast<size_t>(nf) * sizeof(double2), hipMemcpyDeviceToDevice, st));
                hipLaunchKernelGGL(k_zscale2, dim3(vec_blocks(nf)), dim3(kMgThreads), 0, st, vk,
                                   static_cast<double2 *>(nullptr), inv, nf);
                MGCHK(hipGetLastError());
            }
    }
    hipLaunchKernelGGL(k_mg_orth, dim3(2 * m.vc), dim3(kMgThreads), 0, st, V, m);
    MGCHK(hipGetLastError());
    return hipSuccess;
}

hipError_t run_mg_coarse_op(const void *U, const void *vecs, void *A, const GeomDev &g, double mass,
                            const grid_mg_params &p, void *ws, hipStream_t st) {
    MgDims m;
    mg_dims(g, p, &m);
    const MgLayout L = mg_layout(m, p.restart, p.setup_prec, p.cycle_prec);
    double2 *H = reinterpret_cast<double2 *>(static_cast<char *>(ws) + L.H);
    const double2 *V = static_cast<const double2 *>(vecs);
    const long nf = static_cast<long>(m.vol) * 12;
    const long nh = static_cast<long>(m.vol) * 8;
    for (int chi2 = 0; chi2 < 2; ++chi2)
        for (int k2 = 0; k2 < m.nvec; ++k2) {
            const double2 *phi = V + static_cast<size_t>(k2) * nf;
            hipLaunchKernelGGL(k_mg_dirhop, dim3(static_cast<unsigned>((nh + kMgThreads - 1) / kMgThreads)),
                               dim3(kMgThreads), 0, st, static_cast<const double2 *>(U), phi, chi2, H, g);
            MGCHK(hipGetLastError());
            hipLaunchKernelGGL(k_mg_coarse_col, dim3(m.vc), dim3(kMgThreads), 0, st, V, phi, chi2, H,
                               static_cast<double2 *>(A), m, 4.0 + mass, chi2 * m.nvec + k2);
            MGCHK(hipGetLastError());
        }
    return hipSuccess;
}

// One two-level cycle z = K(r) (z: fine, r: fine; uses s, t, rc, ec, cr, cp, cq, cq1).
static hipError_t mg_cycle(const MgCtx &c, const void *U, const double2 *V, const void *A, const double2 *r, double2 *z) {
    const MgDims &m = c.m;
    const CoarseGeo cg = coarse_geo(m);
    double2 *rc = c.f(c.L.rc), *ec = c.f(c.L.ec), *cr = c.f(c.L.cr), *cp = c.f(c.L.cp), *cq = c.f(c.L.cq),
            *cq1 = c.f(c.L.cq1);
    double *ctl = reinterpret_cast<double *>(c.scal()) + 4;
    double *pq = reinterpret_cast<double *>(c.part()), *rr = pq + kMgParts;
    const long n = c.ncv;
    const int nb = vec_blocks(n);
    // r_c = R r
    const float2 *V32 = c.p->cycle_prec == GRID_F32 ? c.h(c.L.v32) : nullptr;
    const bool a32 = V32 != nullptr;
    const void *Ac = a32 ? static_cast<const void *>(c.h(c.L.a32)) : A;
    if (V32)
        hipLaunchKernelGGL(k_mg_restrict<float2>, dim3(m.vc), dim3(kMgThreads), 0, c.st, V32, r, rc, m);
    else
        hipLaunchKernelGGL(k_mg_restrict<double2>, dim3(m.vc), dim3(kMgThreads), 0, c.st, V, r, rc, m);
    MGCHK(hipGetLastError());
    // coarse CGNR from e_c = 0: cr = A^+ r_c = G5 A G5 r_c; cp = cr; then the iterations, every
    // scalar on the device (the same kernels and arguments in every cycle of the solve)
    auto coarse_solve = [&](hipStream_t s) -> hipError_t {
        MGCHK(coarse_stencil(Ac, rc, cr, cg, 0, 1, nullptr, 0, s, a32));
        hipLaunchKernelGGL(k_ccg_start, dim3(nb), dim3(kMgThreads), 0, s, cp, cr, ec, n);
        MGCHK(hipGetLastError());
        hipLaunchKernelGGL(k_cdot_re, dim3(nb), dim3(kMgThreads), 0, s, cr, cr, n, rr, static_cast<const double *>(nullptr),
                           0);
        MGCHK(hipGetLastError());
        hipLaunchKernelGGL(k_ccg_init, dim3(1), dim3(64), 0, s, rr, nb, c.p->coarse_tol, ctl);
        MGCHK(hipGetLastError());
        for (int i = 0; i < c.p->coarse_iters; ++i) {
            const int P = i & 1;
            MGCHK(coarse_stencil(Ac, cp, cq1, cg, 0, 0, ctl, P, s, a32));
            MGCHK(coarse_stencil(Ac, cq1, cq, cg, 0, 1, ctl, P, s, a32));
            hipLaunchKernelGGL(k_cdot_re, dim3(nb), dim3(kMgThreads), 0, s, cp, cq, n, pq, ctl, P);
            MGCHK(hipGetLastError());
            hipLaunchKernelGGL(k_ccg_update, dim3(nb), dim3(kMgThreads), 0, s, ec, cr, cp, cq, n, pq, rr, nb, ctl, P);
            MGCHK(hipGetLastError());
            hipLaunchKernelGGL(k_ccg_p, dim3(nb), dim3(kMgThreads), 0, s, cp, cr, n, rr, nb, ctl, P);
            MGCHK(hipGetLastError());
        }
        return hipSuccess;
    };
    if (!c.p->graph) {
        MGCHK(coarse_solve(c.st));
    } else {
        if (!c.coarse_exec) {
            MgCtx &mc = const_cast<MgCtx &>(c);
            if (!mc.rec) MGCHK(capture_stream(&mc.rec));
            MGCHK(hipStreamBeginCapture(mc.rec, hipStreamCaptureModeThreadLocal));
            hipError_t e = coarse_solve(mc.rec);
            hipGraph_t gr = nullptr;
            const hipError_t e2 = hipStreamEndCapture(mc.rec, &gr);
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) e = hipGraphInstantiate(&mc.coarse_exec, gr, nullptr, nullptr, 0);
            if (gr) (void)hipGraphDestroy(gr);
            MGCHK(e);
        }
        MGCHK(hipGraphLaunch(c.coarse_exec, c.st));
    }
    // z = P e_c
    const long nf = c.nf;
    if (V32)
        hipLaunchKernelGGL(k_mg_prolong<float2>, dim3(static_cast<unsigned>((nf + kMgThreads - 1) / kMgThreads)),
                           dim3(kMgThreads), 0, c.st, V32, ec, z, m);
    else
        hipLaunchKernelGGL(k_mg_prolong<double2>, dim3(static_cast<unsigned>((nf + kMgThreads - 1) / kMgThreads)),
                           dim3(kMgThreads), 0, c.st, V, ec, z, m);
    MGCHK(hipGetLastError());
    // MR smoothing on D z = r, in FP32 (cycle_prec): z and r narrowed, z widened after
    if (c.p->smooth_iters > 0 && c.p->cycle_prec == GRID_F32) {
        float2 *z32 = c.h(c.L.z32), *s32 = c.h(c.L.s32), *t32 = c.h(c.L.t32), *r32 = c.h(c.L.r32);
        MGCHK(launch_convert_spinor(z, GRID_F64, nullptr, z32, GRID_F32, nullptr, m.vol, c.st));
        MGCHK(launch_convert_spinor(r, GRID_F64, nullptr, r32, GRID_F32, nullptr, m.vol, c.st));
        MGCHK(c.D32(z32, t32));
        hipLaunchKernelGGL(k_zsub_f, dim3(vec_blocks(nf)), dim3(kMgThreads), 0, c.st, s32, r32, t32, nf);
        MGCHK(hipGetLastError());
        for (int it = 0; it < c.p->smooth_iters; ++it) {
            MGCHK(c.D32(s32, t32));
            MGCHK(c.mr_step_f(z32, s32, t32, nf));
        }
        return launch_convert_spinor(z32, GRID_F32, nullptr, z, GRID_F64, nullptr, m.vol, c.st);
    }
    if (c.p->smooth_iters > 0) {
        double2 *s = c.f(c.L.s), *t = c.f(c.L.t);
        MGCHK(c.D(U, z, t));
        MGCHK(c.sub(s, r, t, nf));
        // alpha = <t, s> / |t|^2 stays on the device: z += alpha s, s -= alpha t
        for (int it = 0; it < c.p->smooth_iters; ++it) {
            MGCHK(c.D(U, s, t));
            MGCHK(c.zdot2_dev(t, s, t, t, nf));
            MGCHK(c.axpy2_dev(z, s, s, t, 1, nf));
        }
    }
    return hipSuccess;
}

// Flexible GCR on D x = b with z_k = K(r) (pcg = false), or multigrid pCG: flexible CG on the normal
// equations D^dagger D x = D^dagger b with z_k = M(rho) = K(G5 K(G5 rho)), rho = D^dagger r. In the
// pCG, N-conjugating z_k against the kept directions p_j (N = D^dagger D) is orthogonalising D z_k
// against the D p_j, and alpha = <p, rho> / <p, N p> = <D p, r> / |D p|^2, so both run the same loop
// over (z_j, w_j = D z_j) with r = b - D x, and differ in the preconditioned vector only.
hipError_t run_mg_solve(const void *U, const void *vecs, const void *A, const void *b, void *x, const GeomDev &g,
                        double mass, const grid_mg_params &p, void *ws, hipStream_t st, grid_cg_stats *stats,
                        int *status, bool pcg) {
    const auto t0 = std::chrono::steady_clock::now();
    MgCtx c;
    struct Release {   // the recorded coarse solve, after the caller's stream has drained
        MgCtx &c;
        ~Release() {
            if (c.coarse_exec) {
                (void)hipStreamSynchronize(c.st);
                (void)hipGraphExecDestroy(c.coarse_exec);
            }
        }
    } release{c};
    mg_dims(g, p, &c.m);
    c.g = g;
    c.mass = mass;
    c.p = &p;
    c.ws = static_cast<char *>(ws);
    c.L = mg_layout(c.m, p.restart, p.setup_prec, p.cycle_prec);
    c.st = st;
    c.nf = static_cast<long>(g.vol) * 12;
    c.ncv = static_cast<long>(c.m.vc) * c.m.N;
    const long nf = c.nf;
    if (p.cycle_prec == GRID_F32) {
        MGCHK(launch_convert_links(U, c.ws + c.L.u32, GRID_F32, GRID_L18, 0, static_cast<long>(g.vol) * 4, st));
        MGCHK(launch_convert_spinor(vecs, GRID_F64, nullptr, c.ws + c.L.v32, GRID_F32, nullptr,
                                    static_cast<long>(c.m.nvec) * g.vol, st));
        const long na = static_cast<long>(c.m.vc) * 9 * c.m.N * c.m.N;
        hipLaunchKernelGGL(k_narrow2, dim3(static_cast<unsigned>((na + 255) / 256)), dim3(256), 0, st,
                           static_cast<const double2 *>(A), c.h(c.L.a32), na);
        MGCHK(hipGetLastError());
    }
    const double2 *V = static_cast<const double2 *>(vecs);
    const double2 *bb = static_cast<const double2 *>(b);
    double2 *xx = static_cast<double2 *>(x);
    double2 *r = c.f(c.L.r), *t = c.f(c.L.t);
    auto Z = [&](int k) { return c.f(c.L.Z + k * c.L.fv); };
    auto W = [&](int k) { return c.f(c.L.W + k * c.L.fv); };
    *status = GRID_OK;
    stats->iterations = 0;
    stats->reliable_updates = 0;
    stats->converged = 0;
    double2 d;
    MGCHK(c.zdot(bb, bb, nf, &d));
    const double bn = sqrt(d.x);
    auto true_res = [&]() -> hipError_t {
        MGCHK(c.D(U, xx, t));
        return c.sub(r, bb, t, nf);
    };
    MGCHK(true_res());
    MGCHK(c.zdot(r, r, nf, &d));
    double rn = sqrt(d.x);
    int it = 0, k = 0;
    while (rn > p.tol * bn && it < p.maxiter) {
        double2 *zk = Z(k), *wk = W(k);
        if (pcg) {
            double2 *u = c.f(c.L.u);
            MGCHK(c.D(U, r, u, 1));   // rho = D^dagger r
            MGCHK(c.g5(u, u));
            MGCHK(mg_cycle(c, U, V, A, u, zk));
            MGCHK(c.g5(zk, zk));
            MGCHK(mg_cycle(c, U, V, A, zk, u));
            MGCHK(hipMemcpyAsync(zk, u, static_cast<size_t>(nf) * sizeof(double2), hipMemcpyDeviceToDevice, st));
        } else {
            MGCHK(mg_cycle(c, U, V, A, r, zk));
        }
        MGCHK(c.D(U, zk, wk));
        // modified Gram-Schmidt, beta_j = <w_j, w> on the device: w -= beta_j w_j, z -= beta_j z_j
        for (int j = 0; j < k; ++j) {
            MGCHK(c.zdot_dev(W(j), wk, nf));
            MGCHK(c.axpy2_dev(wk, W(j), zk, Z(j), 0, nf));
        }
        // |w|^2 and <w, r> in one pass; w, z scaled to |w| = 1, alpha = <w, r> / |w|
        double2 d2[2];
        MGCHK(c.zdot2(wk, wk, wk, r, nf, d2));
        const double nw = d2[0].x;
        if (!(nw > 0.0) || !isfinite(nw)) {
            *status = GRID_EBREAKDOWN;
            break;
        }
        const double inv = 1.0 / sqrt(nw);
        hipLaunchKernelGGL(k_zscale2, dim3(vec_blocks(nf)), dim3(kMgThreads), 0, st, wk, zk, inv, nf);
        MGCHK(hipGetLastError());
        const double2 alpha = {d2[1].x * inv, d2[1].y * inv};
        MGCHK(c.axpy2(xx, zk, alpha, r, wk, {-alpha.x, -alpha.y}, nf));
        ++it;
        ++k;
        if (k == p.restart) {
            k = 0;
            ++stats->reliable_updates;   // restarts
            MGCHK(true_res());
        }
        MGCHK(c.zdot(r, r, nf, &d));
        rn = sqrt(d.x);
    }
    MGCHK(true_res());
    MGCHK(c.zdot(r, r, nf, &d));
    stats->iterations = it;
    stats->true_residual = bn > 0.0 ? sqrt(d.x) / bn : 0.0;
    stats->converged = stats->true_residual <= p.tol ? 1 : 0;
    if (*status == GRID_OK && !stats->converged) *status = GRID_ENOCONV;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return hipSuccess;
}

}  // namespace gridmi
