// Link gradient and su(3) force of the hopping term (the adjoint HMC's fermion force needs,
// Section 4).
//
// For L = Re <g, c H psi> the complex gradient dL/dRe U + i dL/dIm U of link U_mu(x) is
//   G_mu(x) = c sum_{s, spin} { [(1 + EF gamma_mu) g(x)] psi(x+mu)^dagger
//                             + psi(x) [(1 - EF gamma_mu) g(x+mu)]^dagger },
// EF = -1 for H and +1 for H^dagger. Because (1 + e gamma) v = [h; e A^dagger h] with
// h = v_up + e A v_dn, a spin trace of [(1 + e gamma) v] w^dagger equals the two-spin sum
// h(v) h(w)^dagger of the projected half-spinors (with the same e), so each term is a sum of two
// 3x3 outer products of half-spinors. One thread per (4D site, mu), one mu per wavefront; the
// fifth coordinate is summed inside the thread; no atomics, so results are bitwise reproducible.
#include "device.h"
#include "launch.h"

namespace gridmi {

// Records come through the wavefront's LDS slot (coalesced chunk loads, then each lane reads its
// own record back); the four records of a step are all requested before the first is staged.
template <int MU, int EF, class SP, typename C>
__device__ __forceinline__ void grad_mu(const void *chi, const void *psi, int x4, int xp, int Ls, chunk_t *lds,
                                        Cx<C> G[3][3]) {
    Cx<C> p[4][3], hg[2][3], hp[2][3];
    for (int s = 0; s < Ls; ++s) {
        Fetch<SP> f0, f1, f2, f3;
        fetch<SP>(chi, nullptr, x4 * Ls + s, f0);
        fetch<SP>(psi, nullptr, xp * Ls + s, f1);
        fetch<SP>(psi, nullptr, x4 * Ls + s, f2);
        fetch<SP>(chi, nullptr, xp * Ls + s, f3);
        // [(1 + EF gamma) g(x)] psi(x+mu)^dagger
        stage<SP>(f0, lds, p);
        project<MU, EF>(p, hg);
        stage<SP>(f1, lds, p);
        project<MU, EF>(p, hp);
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) G[a][b] = cmac(G[a][b], hg[k][a], cconj(hp[k][b]));
        // psi(x) [(1 - EF gamma) g(x+mu)]^dagger
        stage<SP>(f2, lds, p);
        project<MU, -EF>(p, hp);
        stage<SP>(f3, lds, p);
        project<MU, -EF>(p, hg);
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) G[a][b] = cmac(G[a][b], hp[k][a], cconj(hg[k][b]));
    }
}

template <class SP, bool DAG>
__global__ void __launch_bounds__(256)
k_link_grad(const void *__restrict__ U, const void *__restrict__ chi, const void *__restrict__ psi, void *__restrict__ Gout,
            GeomDev g, double coef, int force_mode) {
    using C = typename SP::C;
    __shared__ chunk_t sm[4][64 * stage_pitch<SP>()];
    chunk_t *lds = sm[threadIdx.x >> 6];
    // A block covers 64 consecutive sites; wavefront mu computes their direction-mu links, so
    // the direction is uniform across a wavefront (no divergent switch) and the four wavefronts
    // reading chi(x) and psi(x) share them through the CU's L1.
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int mu = threadIdx.x >> 6;
    const int x4r = lb * 64 + (threadIdx.x & 63);
    const bool live = x4r < g.vol;
    const int x4 = live ? x4r : g.vol - 1;   // idle lanes take part in the wave's gathers
    const int t = x4 * 4 + mu;               // link index: site-major, direction fastest
    int nb[8];
    neighbours(g, x4, nb);
    Cx<C> G[3][3];
#pragma unroll
    for (int k = 0; k < 9; ++k) G[k / 3][k % 3] = {C(0), C(0)};
    constexpr int EF = DAG ? +1 : -1;
    switch (mu) {
        case 0: grad_mu<0, EF, SP, C>(chi, psi, x4, nb[0], g.Ls, lds, G); break;
        case 1: grad_mu<1, EF, SP, C>(chi, psi, x4, nb[2], g.Ls, lds, G); break;
        case 2: grad_mu<2, EF, SP, C>(chi, psi, x4, nb[4], g.Ls, lds, G); break;
        default: grad_mu<3, EF, SP, C>(chi, psi, x4, nb[6], g.Ls, lds, G); break;
    }
    const C c = static_cast<C>(coef);
#pragma unroll
    for (int k = 0; k < 9; ++k) G[k / 3][k % 3] = cscale(c, G[k / 3][k % 3]);
    if (force_mode) {
        // F = TA(G U^dagger), TA(A) = (A - A^dagger)/2 - tr(A - A^dagger)/6
        Cx<C> u[3][3], m[3][3];
        if constexpr (sizeof(C) == 8)
            LkF64<3>::load(U, static_cast<size_t>(t), u);
        else
            LkF32<3>::load(U, static_cast<size_t>(t), u);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                Cx<C> s = cmul(G[a][0], cconj(u[b][0]));
                s = cmac(s, G[a][1], cconj(u[b][1]));
                s = cmac(s, G[a][2], cconj(u[b][2]));
                m[a][b] = s;
            }
        // tr(A - A^dagger) = 2 i Im tr A
        const C imtr = m[0][0].i + m[1][1].i + m[2][2].i;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                Cx<C> f = {C(0.5) * (m[a][b].r - m[b][a].r), C(0.5) * (m[a][b].i + m[b][a].i)};
                if (a == b) f.i -= imtr / C(3);
                G[a][b] = f;
            }
    }
    if (!live) return;
    if constexpr (sizeof(C) == 8) {
        double2 *q = reinterpret_cast<double2 *>(Gout) + static_cast<size_t>(t) * 9;
#pragma unroll
        for (int k = 0; k < 9; ++k) q[k] = make_double2(G[k / 3][k % 3].r, G[k / 3][k % 3].i);
    } else {
        float2 *q = reinterpret_cast<float2 *>(Gout) + static_cast<size_t>(t) * 9;
#pragma unroll
        for (int k = 0; k < 9; ++k)
            q[k] = make_float2(static_cast<float>(G[k / 3][k % 3].r), static_cast<float>(G[k / 3][k % 3].i));
    }
}

hipError_t launch_link_grad(const LinkGradArgs &a) {
    if (a.g.vol == 0) return hipSuccess;
    const int blocks = (a.g.vol + 63) / 64;
    const dim3 grid(blocks), block(256);
    if (a.prec == GRID_F64) {
        if (a.dag)
            hipLaunchKernelGGL((k_link_grad<SpF64, true>), grid, block, 0, a.stream, a.U, a.chi, a.psi, a.G, a.g, a.coef,
                               a.force_mode);
        else
            hipLaunchKernelGGL((k_link_grad<SpF64, false>), grid, block, 0, a.stream, a.U, a.chi, a.psi, a.G, a.g,
                               a.coef, a.force_mode);
    } else if (a.prec == GRID_F32) {
        if (a.dag)
            hipLaunchKernelGGL((k_link_grad<SpF32, true>), grid, block, 0, a.stream, a.U, a.chi, a.psi, a.G, a.g, a.coef,
                               a.force_mode);
        else
            hipLaunchKernelGGL((k_link_grad<SpF32, false>), grid, block, 0, a.stream, a.U, a.chi, a.psi, a.G, a.g,
                               a.coef, a.force_mode);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gridmi
