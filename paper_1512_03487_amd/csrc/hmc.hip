// Hybrid Monte Carlo molecular dynamics (HMC is among the algorithms the paper lists, Section 4):
// Wilson plaquette gauge action and its force, the su(3) exponential link update, the kinetic
// energy, and leapfrog, Omelyan and force-gradient integrators whose fermion force is the
// pseudofermion force of the hopping-term adjoint (CG solve recomputed at every force evaluation).
//
// Conventions (shared with the fermion force of grid_dhop_backward):
//   S_G = beta sum_{x, mu<nu} (1 - Re tr P_munu(x) / 3),
//   P_munu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dagger U_nu(x)^dagger;
//   F = TA(G U^dagger), G = dS/dRe U + i dS/dIm U, so d/de S(exp(e X) U)|0 = Re tr(F^dagger X);
//   for S_G: F_mu(x) = (beta/3) TA(U_mu(x) A_mu(x)), A_mu the sum of the six staples;
//   K = sum tr(P^dagger P), dU/dt = P U, dP/dt = -F/2 (H = K + S conserved);
//   S_F = phi^dagger (M^dagger M)^-1 phi, dS_F/dU = -2 G_{c=-1/2}(chi = M X, psi = X).
#include <chrono>
#include <string.h>

#include "device.h"
#include "launch.h"

namespace gridmi {

typedef Cx<double> M3[3][3];

__device__ __forceinline__ void load_link(const double2 *__restrict__ U, size_t link, M3 u) {
    const double2 *q = U + link * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double2 v = q[k];
        u[k / 3][k % 3] = {v.x, v.y};
    }
}

__device__ __forceinline__ void store_link(double2 *__restrict__ U, size_t link, const M3 u) {
    double2 *q = U + link * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) q[k] = make_double2(u[k / 3][k % 3].r, u[k / 3][k % 3].i);
}

// c = a b (A: a^dagger when DA, B: b^dagger when DB)
template <bool DA, bool DB>
__device__ __forceinline__ void mm(const M3 a, const M3 b, M3 c) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Cx<double> s = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const Cx<double> x = DA ? cconj(a[k][i]) : a[i][k];
                const Cx<double> y = DB ? cconj(b[j][k]) : b[k][j];
                s = cmac(s, x, y);
            }
            c[i][j] = s;
        }
}

__device__ __forceinline__ void madd(M3 a, const M3 b) {
#pragma unroll
    for (int k = 0; k < 9; ++k) a[k / 3][k % 3] = cadd(a[k / 3][k % 3], b[k / 3][k % 3]);
}

__device__ __forceinline__ int nbr(const GeomDev &g, int x4, int mu, int dir) {
    int stride = 1;
    for (int k = 0; k < mu; ++k) stride *= g.L[k];
    const int c = (x4 / stride) % g.L[mu];
    if (dir > 0) return c == g.L[mu] - 1 ? x4 - (g.L[mu] - 1) * stride : x4 + stride;
    return c == 0 ? x4 + (g.L[mu] - 1) * stride : x4 - stride;
}

// F_mu(x) = scale * (beta / 3) TA(U_mu(x) A_mu(x)); one thread per link.
__global__ void __launch_bounds__(256)
k_gauge_force(const double2 *__restrict__ U, double2 *__restrict__ F, GeomDev g, double beta, double scale, int accumulate) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= g.vol * 4) return;
    const int mu = t & 3, x4 = t >> 2;
    const int xpm = nbr(g, x4, mu, +1);
    M3 A, u1, u2, u3, w, v;
#pragma unroll
    for (int k = 0; k < 9; ++k) A[k / 3][k % 3] = {0.0, 0.0};
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        // upper staple U_nu(x+mu) U_mu(x+nu)^dagger U_nu(x)^dagger
        const int xpn = nbr(g, x4, nu, +1);
        load_link(U, static_cast<size_t>(xpm) * 4 + nu, u1);
        load_link(U, static_cast<size_t>(xpn) * 4 + mu, u2);
        load_link(U, static_cast<size_t>(x4) * 4 + nu, u3);
        mm<false, true>(u1, u2, w);
        mm<false, true>(w, u3, v);
        madd(A, v);
        // lower staple U_nu(x+mu-nu)^dagger U_mu(x-nu)^dagger U_nu(x-nu)
        const int xmn = nbr(g, x4, nu, -1);
        const int xpmmn = nbr(g, xpm, nu, -1);
        load_link(U, static_cast<size_t>(xpmmn) * 4 + nu, u1);
        load_link(U, static_cast<size_t>(xmn) * 4 + mu, u2);
        load_link(U, static_cast<size_t>(xmn) * 4 + nu, u3);
        mm<true, true>(u1, u2, w);
        mm<false, false>(w, u3, v);
        madd(A, v);
    }
    load_link(U, static_cast<size_t>(t), u1);
    mm<false, false>(u1, A, w);
    // TA(w) = (w - w^dagger)/2 - tr(w - w^dagger)/6
    const double imtr = w[0][0].i + w[1][1].i + w[2][2].i;
    const double c = scale * beta / 3.0;
    M3 f;
    if (accumulate) load_link(F, static_cast<size_t>(t), f);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            Cx<double> x = {0.5 * (w[a][b].r - w[b][a].r), 0.5 * (w[a][b].i + w[b][a].i)};
            if (a == b) x.i -= imtr / 3.0;
            x = {c * x.r, c * x.i};
            f[a][b] = accumulate ? cadd(f[a][b], x) : x;
        }
    store_link(F, static_cast<size_t>(t), f);
}

// U <- exp(eps P) U per link: Taylor series to order 16 of X / 2^k with |X| / 2^k < 1/2
// (Frobenius norm), then k squarings (scaling and squaring).
__global__ void __launch_bounds__(256)
k_link_exp(double2 *__restrict__ U, const double2 *__restrict__ P, double eps, long nlinks) {
    const long l = static_cast<long>(blockIdx.x) * 256 + threadIdx.x;
    if (l >= nlinks) return;
    M3 X, E, T, u, r;
    load_link(P, l, X);
    double n2 = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) n2 += X[k / 3][k % 3].r * X[k / 3][k % 3].r + X[k / 3][k % 3].i * X[k / 3][k % 3].i;
    double nrm = fabs(eps) * sqrt(n2);
    int sq = 0;
    while (nrm > 0.5 && sq < 30) {
        nrm *= 0.5;
        ++sq;
    }
    const double sc = eps * ldexp(1.0, -sq);
#pragma unroll
    for (int k = 0; k < 9; ++k) X[k / 3][k % 3] = cscale(sc, X[k / 3][k % 3]);
    // Horner: E = I + X (I + X/2 (I + X/3 (... (I + X/16))))
#pragma unroll
    for (int k = 0; k < 9; ++k) E[k / 3][k % 3] = {k % 4 == 0 ? 1.0 : 0.0, 0.0};
    for (int n = 16; n >= 1; --n) {
        mm<false, false>(X, E, T);
        const double inv = 1.0 / n;
#pragma unroll
        for (int k = 0; k < 9; ++k) E[k / 3][k % 3] = {(k % 4 == 0 ? 1.0 : 0.0) + inv * T[k / 3][k % 3].r,
                                                       inv * T[k / 3][k % 3].i};
    }
    for (int k = 0; k < sq; ++k) {
        mm<false, false>(E, E, T);
#pragma unroll
        for (int j = 0; j < 9; ++j) E[j / 3][j % 3] = T[j / 3][j % 3];
    }
    load_link(U, l, u);
    mm<false, false>(E, u, r);
    store_link(U, l, r);
}

// y += a x over n doubles.
__global__ void __launch_bounds__(256) k_daxpy(double *__restrict__ y, const double *__restrict__ x, double a, long n) {
    for (long i = static_cast<long>(blockIdx.x) * 256 + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * 256)
        y[i] += a * x[i];
}

__device__ __forceinline__ double hsum(double v, double *sm) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    return (sm[0] + sm[1]) + (sm[2] + sm[3]);
}

// Per-block partial sums of Re tr P_munu(x) over mu < nu (one thread per site).
__global__ void __launch_bounds__(256) k_plaq(const double2 *__restrict__ U, GeomDev g, double *__restrict__ part) {
    __shared__ double sm[4];
    double acc = 0.0;
    for (int x4 = blockIdx.x * 256 + threadIdx.x; x4 < g.vol; x4 += gridDim.x * 256) {
        M3 a, b, c, d, w, v;
        for (int mu = 0; mu < 4; ++mu) {
            const int xpm = nbr(g, x4, mu, +1);
            load_link(U, static_cast<size_t>(x4) * 4 + mu, a);
            for (int nu = mu + 1; nu < 4; ++nu) {
                const int xpn = nbr(g, x4, nu, +1);
                load_link(U, static_cast<size_t>(xpm) * 4 + nu, b);
                load_link(U, static_cast<size_t>(xpn) * 4 + mu, c);
                load_link(U, static_cast<size_t>(x4) * 4 + nu, d);
                mm<false, false>(a, b, w);
                mm<false, true>(w, c, v);
                // Re tr(v d^dagger)
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int k = 0; k < 3; ++k) acc += v[i][k].r * d[i][k].r + v[i][k].i * d[i][k].i;
            }
        }
    }
    const double t = hsum(acc, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Per-block partial sums of sum |x|^2 over n doubles.
__global__ void __launch_bounds__(256) k_sumsq(const double *__restrict__ x, long n, double *__restrict__ part) {
    __shared__ double sm[4];
    double acc = 0.0;
    for (long i = static_cast<long>(blockIdx.x) * 256 + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * 256)
        acc += x[i] * x[i];
    const double t = hsum(acc, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(256) k_sum_part(const double *__restrict__ part, int np, double *__restrict__ out) {
    __shared__ double sm[4];
    double v = 0.0;
    for (int k = threadIdx.x; k < np; k += 256) v += part[k];
    const double t = hsum(v, sm);
    if (threadIdx.x == 0) *out = t;
}

constexpr int kHmcParts = 1024;

static hipError_t reduce_to_host(double *part, int np, hipStream_t st, double *result) {
    hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(256), 0, st, part, np, part + kHmcParts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double h = 0.0;
    e = hipMemcpyAsync(&h, part + kHmcParts, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    *result = h;
    return e;
}

#define HMCCHK(x)                               \
    do {                                        \
        hipError_t e_ = (x);                    \
        if (e_ != hipSuccess) return e_;        \
    } while (0)

hipError_t launch_gauge_force(const void *U, void *F, const GeomDev &g, double beta, double scale, int accumulate,
                              hipStream_t st) {
    if (g.vol == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gauge_force, dim3((g.vol * 4 + 255) / 256), dim3(256), 0, st, static_cast<const double2 *>(U),
                       static_cast<double2 *>(F), g, beta, scale, accumulate);
    return hipGetLastError();
}

hipError_t launch_link_exp(void *U, const void *P, double eps, long nlinks, hipStream_t st) {
    if (nlinks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_link_exp, dim3(static_cast<unsigned>((nlinks + 255) / 256)), dim3(256), 0, st,
                       static_cast<double2 *>(U), static_cast<const double2 *>(P), eps, nlinks);
    return hipGetLastError();
}

static hipError_t daxpy(void *y, const void *x, double a, long n, hipStream_t st) {
    const long blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    hipLaunchKernelGGL(k_daxpy, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, static_cast<double *>(y),
                       static_cast<const double *>(x), a, n);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------------------------
// Molecular dynamics
// ----------------------------------------------------------------------------------------------

static size_t al256(size_t v) { return (v + 255) & ~size_t(255); }

struct MdLayout {
    size_t F, Ff, X, Y, T, Ud, part, cg, total;   // Ud: displaced links (force-gradient integrator)
};

static MdLayout md_layout(const GeomDev &g, const grid_md_params &p) {
    MdLayout L;
    memset(&L, 0, sizeof(L));
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off = al256(off + b);
        return o;
    };
    const size_t lb = static_cast<size_t>(g.vol) * 4 * 144;
    const size_t sb = static_cast<size_t>(g.n5) * 192;
    L.F = take(lb);
    L.Ff = take(lb);
    L.X = take(sb);
    L.Y = take(sb);
    L.T = p.fermion.kind == GRID_MOBIUS ? take(sb) : 0;   // Moebius: the intermediate of M X, then B X
    L.Ud = p.integrator == GRID_FORCE_GRADIENT ? take(lb) : 0;
    L.part = take((kHmcParts + 16) * sizeof(double));
    L.cg = off;
    L.total = off + cg_workspace_bytes(g, p.cg.sloppy_prec, p.cg.link_fmt);
    return L;
}

size_t md_workspace_bytes(const GeomDev &g, const grid_md_params &p) { return md_layout(g, p).total; }

struct MdRun {
    void *U;
    const void *phi;   // NULL: pure gauge
    GeomDev g;
    grid_md_params p;
    char *ws;
    MdLayout L;
    hipStream_t st;
    grid_md_stats *stats;
};

// X = (M^dagger M)^-1 phi (warm start from the previous X), Y = M X; for the Moebius operator also
// T = B X, the field the links meet in M's hopping term -H B / 2.
static hipError_t fermion_solve(MdRun &r) {
    int status = GRID_OK;
    grid_cg_stats cs;
    memset(&cs, 0, sizeof(cs));
    HMCCHK(run_cg(r.U, r.phi, r.ws + r.L.X, r.g, r.p.fermion, r.p.cg, r.ws + r.L.cg, r.st, &cs, &status));
    r.stats->solves += 1;
    r.stats->cg_iterations += cs.iterations;
    if (status != GRID_OK) r.stats->failed_solves += 1;
    DhopArgs a;
    a.U = r.U;
    a.psi = r.ws + r.L.X;
    a.psi_scale = nullptr;
    a.out = r.ws + r.L.Y;
    a.out_scale = nullptr;
    a.g = r.g;
    a.prec = GRID_F64;
    a.link_fmt = GRID_L18;
    a.kind = r.p.fermion.kind;
    a.dag = 0;
    a.diag = r.p.fermion.kind == GRID_WILSON ? 4.0 + r.p.fermion.mass : 5.0 - r.p.fermion.M5;
    a.mf = r.p.fermion.mf;
    a.stream = r.st;
    if (r.p.fermion.kind != GRID_MOBIUS) return launch_dhop(a);
    const grid_op &op = r.p.fermion;
    HMCCHK(launch_mobius(a, op.M5, op.b5, op.c5, r.ws + r.L.T, nullptr));
    return launch_s5axpy(GRID_F64, r.ws + r.L.X, nullptr, nullptr, nullptr, r.ws + r.L.T, nullptr, r.g.n5, r.g.Ls,
                         op.b5, op.c5, 0.0, 0.0, op.mf, 0, r.st);
}

// The pseudofermion force into the Ff buffer (phi != NULL).
static hipError_t fermion_force(MdRun &r) {
    HMCCHK(fermion_solve(r));
    LinkGradArgs a;
    a.U = r.U;
    a.chi = r.ws + r.L.Y;
    a.psi = r.ws + (r.p.fermion.kind == GRID_MOBIUS ? r.L.T : r.L.X);
    a.G = r.ws + r.L.Ff;
    a.g = r.g;
    a.prec = GRID_F64;
    a.dag = 0;
    a.force_mode = 1;
    a.coef = 1.0;   // dS_F/dU = -2 G_{c=-1/2}(M X, X or B X) = G_{c=1}
    a.stream = r.st;
    return launch_link_grad(a);
}

// F = gauge force + fermion force (su(3), the convention above) into the F buffer.
static hipError_t total_force(MdRun &r) {
    HMCCHK(launch_gauge_force(r.U, r.ws + r.L.F, r.g, r.p.beta, 1.0, 0, r.st));
    if (!r.phi) return hipSuccess;
    HMCCHK(fermion_force(r));
    return daxpy(r.ws + r.L.F, r.ws + r.L.Ff, 1.0, static_cast<long>(r.g.vol) * 4 * 18, r.st);
}

hipError_t run_md_leapfrog(void *U, void *P, const void *phi, const GeomDev &g, const grid_md_params &p, void *ws,
                           hipStream_t st, grid_md_stats *stats) {
    const auto t0 = std::chrono::steady_clock::now();
    MdRun r;
    r.U = U;
    r.phi = phi;
    r.g = g;
    r.p = p;
    r.ws = static_cast<char *>(ws);
    r.L = md_layout(g, p);
    r.st = st;
    r.stats = stats;
    memset(stats, 0, sizeof(*stats));
    if (p.n_steps == 0) return hipSuccess;   // zero steps integrate over zero time
    const long nd = static_cast<long>(g.vol) * 4 * 18;
    if (phi) HMCCHK(hipMemsetAsync(r.ws + r.L.X, 0, static_cast<size_t>(g.n5) * 192, st));
    if (p.n_inner > 1) {
        // Two time scales: the fermion kicks of a leapfrog (P -= e/2 f_F; gauge integration over e;
        // P -= e/2 f_F), Omelyan (P -= l e f_F; e/2; P -= (1 - 2 l) e f_F; e/2; P -= l e f_F) or
        // force-gradient (P -= e/6 f_F; e/2; P -= 2e/3 f_F(U'); e/2; P -= e/6 f_F, with
        // U' = exp(-(e^2/24) f_F(U)) U) outer step, each gauge integration over tau being n_inner
        // leapfrog steps of h = tau / n_inner with the gauge force alone. Consecutive fermion kicks
        // (across outer steps) and consecutive gauge kicks (inside one integration) act at the same
        // U and are merged.
        constexpr double lam = 0.1931833275037836;
        const long nl = static_cast<long>(g.vol) * 4;
        auto gauge_integrate = [&](double tau) -> hipError_t {
            const double h = tau / p.n_inner;
            HMCCHK(launch_gauge_force(U, r.ws + r.L.F, g, p.beta, 1.0, 0, st));
            HMCCHK(daxpy(P, r.ws + r.L.F, -0.25 * h, nd, st));
            for (int j = 0; j < p.n_inner; ++j) {
                HMCCHK(launch_link_exp(U, P, h, nl, st));
                HMCCHK(launch_gauge_force(U, r.ws + r.L.F, g, p.beta, 1.0, 0, st));
                HMCCHK(daxpy(P, r.ws + r.L.F, (j == p.n_inner - 1 ? -0.25 : -0.5) * h, nd, st));
            }
            return hipSuccess;
        };
        auto fermion_kick = [&](double c) -> hipError_t {   // P -= c e F_F / 2
            if (!phi) return hipSuccess;
            HMCCHK(fermion_force(r));
            return daxpy(P, r.ws + r.L.Ff, -0.5 * c * p.eps, nd, st);
        };
        // force-gradient outer kick: P -= 2e/3 f_F(U'), U' = exp(-(e^2/24) f_F(U)) U in the Ud copy
        auto fermion_fg_kick = [&]() -> hipError_t {
            if (!phi) return hipSuccess;
            void *Ud = r.ws + r.L.Ud;
            HMCCHK(fermion_force(r));
            HMCCHK(hipMemcpyAsync(Ud, U, static_cast<size_t>(nl) * 144, hipMemcpyDeviceToDevice, st));
            HMCCHK(launch_link_exp(Ud, r.ws + r.L.Ff, -0.5 * p.eps * p.eps / 24.0, nl, st));
            r.U = Ud;
            const hipError_t e = fermion_force(r);
            r.U = U;
            HMCCHK(e);
            return daxpy(P, r.ws + r.L.Ff, -0.5 * 2.0 * p.eps / 3.0, nd, st);
        };
        const bool omelyan = p.integrator == GRID_OMELYAN, fg = p.integrator == GRID_FORCE_GRADIENT;
        HMCCHK(fermion_kick(omelyan ? lam : fg ? 1.0 / 6.0 : 0.5));
        for (int i = 0; i < p.n_steps; ++i) {
            const bool last = i == p.n_steps - 1;
            if (fg) {
                HMCCHK(gauge_integrate(0.5 * p.eps));
                HMCCHK(fermion_fg_kick());
                HMCCHK(gauge_integrate(0.5 * p.eps));
                HMCCHK(fermion_kick(last ? 1.0 / 6.0 : 2.0 / 6.0));
            } else if (omelyan) {
                HMCCHK(gauge_integrate(0.5 * p.eps));
                HMCCHK(fermion_kick(1.0 - 2.0 * lam));
                HMCCHK(gauge_integrate(0.5 * p.eps));
                HMCCHK(fermion_kick(last ? lam : 2.0 * lam));
            } else {
                HMCCHK(gauge_integrate(p.eps));
                HMCCHK(fermion_kick(last ? 0.5 : 1.0));
            }
        }
        HMCCHK(hipStreamSynchronize(st));
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return hipSuccess;
    }
    if (p.integrator == GRID_FORCE_GRADIENT) {
        // per step: P -= e/6 f(U); U <- exp(e/2 P) U; P -= 2e/3 f(U'), U' = exp(-(e^2/24) f(U)) U;
        // U <- exp(e/2 P) U; P -= e/6 f(U), f = F/2; consecutive outer kicks merged: 3 n + 1
        // force evaluations
        const long nl = static_cast<long>(g.vol) * 4;
        void *Ud = r.ws + r.L.Ud;
        HMCCHK(total_force(r));
        HMCCHK(daxpy(P, r.ws + r.L.F, -0.5 * p.eps / 6.0, nd, st));
        for (int i = 0; i < p.n_steps; ++i) {
            HMCCHK(launch_link_exp(U, P, 0.5 * p.eps, nl, st));
            HMCCHK(total_force(r));
            HMCCHK(hipMemcpyAsync(Ud, U, static_cast<size_t>(nl) * 144, hipMemcpyDeviceToDevice, st));
            HMCCHK(launch_link_exp(Ud, r.ws + r.L.F, -0.5 * p.eps * p.eps / 24.0, nl, st));
            r.U = Ud;   // the force at the displaced links
            const hipError_t e = total_force(r);
            r.U = U;
            HMCCHK(e);
            HMCCHK(daxpy(P, r.ws + r.L.F, -0.5 * 2.0 * p.eps / 3.0, nd, st));
            HMCCHK(launch_link_exp(U, P, 0.5 * p.eps, nl, st));
            HMCCHK(total_force(r));
            HMCCHK(daxpy(P, r.ws + r.L.F, -0.5 * (i == p.n_steps - 1 ? 1.0 : 2.0) * p.eps / 6.0, nd, st));
        }
        HMCCHK(hipStreamSynchronize(st));
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return hipSuccess;
    }
    if (p.integrator == GRID_OMELYAN) {
        // the closing kick of a step and the opening kick of the next act at the same U and are
        // merged: 2 n + 1 force evaluations
        constexpr double lam = 0.1931833275037836;
        const long nl = static_cast<long>(g.vol) * 4;
        HMCCHK(total_force(r));
        HMCCHK(daxpy(P, r.ws + r.L.F, -0.5 * lam * p.eps, nd, st));
        for (int i = 0; i < p.n_steps; ++i) {
            HMCCHK(launch_link_exp(U, P, 0.5 * p.eps, nl, st));
            HMCCHK(total_force(r));
            HMCCHK(daxpy(P, r.ws + r.L.F, -0.5 * (1.0 - 2.0 * lam) * p.eps, nd, st));
            HMCCHK(launch_link_exp(U, P, 0.5 * p.eps, nl, st));
            HMCCHK(total_force(r));
            HMCCHK(daxpy(P, r.ws + r.L.F, -0.5 * (i == p.n_steps - 1 ? lam : 2.0 * lam) * p.eps, nd, st));
        }
        HMCCHK(hipStreamSynchronize(st));
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return hipSuccess;
    }
    // P -= (eps / 2) F / 2
    HMCCHK(total_force(r));
    HMCCHK(daxpy(P, r.ws + r.L.F, -0.25 * p.eps, nd, st));
    for (int i = 0; i < p.n_steps; ++i) {
        HMCCHK(launch_link_exp(U, P, p.eps, static_cast<long>(g.vol) * 4, st));
        HMCCHK(total_force(r));
        HMCCHK(daxpy(P, r.ws + r.L.F, (i == p.n_steps - 1 ? -0.25 : -0.5) * p.eps, nd, st));
    }
    HMCCHK(hipStreamSynchronize(st));
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return hipSuccess;
}

// ----------------------------------------------------------------------------------------------
// Two-flavour pseudofermion action on its own (the fermion part of the HMC action, Section 4):
// X = (Op^dagger Op)^-1 phi, S = Re <phi, X> by the fixed-order FP64 reduction, and the gradients
// scaled by the caller's upstream factor: dS/dU = -2 G_{c=-1/2}(chi = Op X, psi = X) = G_{c=1}
// (raw, or TA(dS/dU U^dagger)) and dS/dphi = 2 X.
// ----------------------------------------------------------------------------------------------

// y = a x over n doubles.
__global__ void __launch_bounds__(256) k_dscal(double *__restrict__ y, const double *__restrict__ x, double a, long n) {
    for (long i = static_cast<long>(blockIdx.x) * 256 + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * 256)
        y[i] = a * x[i];
}

struct PfLayout {
    size_t Y, T, part, cg, total;
};

static PfLayout pf_layout(const GeomDev &g, const grid_cg_params &p) {
    PfLayout L;
    size_t off = 0;
    L.Y = off;
    off = al256(off + static_cast<size_t>(g.n5) * 192);
    L.T = off;   // Moebius: the intermediate of M X, then B X
    off = al256(off + static_cast<size_t>(g.n5) * 192);
    L.part = off;
    off = al256(off + (kHmcParts + 16) * sizeof(double));
    L.cg = off;
    L.total = off + cg_workspace_bytes(g, p.sloppy_prec, p.link_fmt);
    return L;
}

size_t pf_workspace_bytes(const GeomDev &g, const grid_cg_params &p) { return pf_layout(g, p).total; }

hipError_t run_pseudofermion(const void *U, const void *phi, void *X, const GeomDev &g, const grid_op &op,
                             const grid_cg_params &p, double grad_scale, double *S, void *dS_dU, int force_mode,
                             void *dS_dphi, void *ws, hipStream_t st, grid_cg_stats *stats, int *status) {
    const PfLayout L = pf_layout(g, p);
    char *w = static_cast<char *>(ws);
    HMCCHK(run_cg(U, phi, X, g, op, p, w + L.cg, st, stats, status));
    if (S) HMCCHK(dot_re(phi, X, g.n5, reinterpret_cast<double *>(w + L.part), st, S));
    if (dS_dU) {
        DhopArgs a;
        a.U = U;
        a.psi = X;
        a.psi_scale = nullptr;
        a.out = w + L.Y;
        a.out_scale = nullptr;
        a.g = g;
        a.prec = GRID_F64;
        a.link_fmt = GRID_L18;
        a.kind = op.kind;
        a.dag = 0;
        a.diag = op.kind == GRID_WILSON ? 4.0 + op.mass : 5.0 - op.M5;
        a.mf = op.mf;
        a.stream = st;
        const void *psi_g = X;
        if (op.kind == GRID_MOBIUS) {
            // M depends on the links through -H B / 2: dS/dU = -2 G(M X, B X)
            HMCCHK(launch_mobius(a, op.M5, op.b5, op.c5, w + L.T, nullptr));
            HMCCHK(launch_s5axpy(GRID_F64, X, nullptr, nullptr, nullptr, w + L.T, nullptr, g.n5, g.Ls, op.b5, op.c5,
                                 0.0, 0.0, op.mf, 0, st));
            psi_g = w + L.T;
        } else {
            HMCCHK(launch_dhop(a));
        }
        LinkGradArgs la;
        la.U = U;
        la.chi = w + L.Y;
        la.psi = psi_g;
        la.G = dS_dU;
        la.g = g;
        la.prec = GRID_F64;
        la.dag = 0;
        la.force_mode = force_mode;
        la.coef = grad_scale;   // -2 G_{c=-1/2} = G_{c=1}, times the upstream factor
        la.stream = st;
        HMCCHK(launch_link_grad(la));
    }
    if (dS_dphi && g.n5 > 0) {
        const long n = static_cast<long>(g.n5) * 24;
        const long blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
        hipLaunchKernelGGL(k_dscal, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, static_cast<double *>(dS_dphi),
                           static_cast<const double *>(X), 2.0 * grad_scale, n);
        HMCCHK(hipGetLastError());
    }
    return hipSuccess;
}

// energies[0..3] = K, S_G, S_F, H.
hipError_t run_hmc_energy(const void *U, const void *P, const void *phi, const GeomDev &g, const grid_md_params &p,
                          void *ws, hipStream_t st, double energies[4], grid_md_stats *stats) {
    MdRun r;
    r.U = const_cast<void *>(U);
    r.phi = phi;
    r.g = g;
    r.p = p;
    r.ws = static_cast<char *>(ws);
    r.L = md_layout(g, p);
    r.st = st;
    r.stats = stats;
    memset(stats, 0, sizeof(*stats));
    double *part = reinterpret_cast<double *>(r.ws + r.L.part);
    const long nd = static_cast<long>(g.vol) * 4 * 18;
    // K = sum |P|^2
    const int npk = static_cast<int>((nd + 255) / 256 < kHmcParts ? (nd + 255) / 256 : kHmcParts);
    hipLaunchKernelGGL(k_sumsq, dim3(npk), dim3(256), 0, st, static_cast<const double *>(P), nd, part);
    HMCCHK(hipGetLastError());
    double K = 0.0;
    HMCCHK(reduce_to_host(part, npk, st, &K));
    // S_G = beta (6 V - sum Re tr P / 3)
    const int npp = (g.vol + 255) / 256 < kHmcParts ? (g.vol + 255) / 256 : kHmcParts;
    hipLaunchKernelGGL(k_plaq, dim3(npp), dim3(256), 0, st, static_cast<const double2 *>(U), g, part);
    HMCCHK(hipGetLastError());
    double rt = 0.0;
    HMCCHK(reduce_to_host(part, npp, st, &rt));
    const double SG = p.beta * (6.0 * g.vol - rt / 3.0);
    double SF = 0.0;
    if (phi) {
        HMCCHK(hipMemsetAsync(r.ws + r.L.X, 0, static_cast<size_t>(g.n5) * 192, st));
        HMCCHK(fermion_solve(r));
        HMCCHK(dot_re(phi, r.ws + r.L.X, g.n5, part, st, &SF));
    }
    energies[0] = K;
    energies[1] = SG;
    energies[2] = SF;
    energies[3] = K + SG + SF;
    return hipSuccess;
}

}  // namespace gridmi
