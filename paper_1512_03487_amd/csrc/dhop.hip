// Wilson hopping term, Wilson operator and Shamir domain-wall operator (gfx950).
//
// One thread per 4D site (Ls = 1) or per 5D site (4D site, s) with s the fastest index, so a
// wavefront covers 64 / Ls consecutive 4D sites: the link loads of a 4D site are the same
// address for its Ls lanes, and the neighbour spinors of consecutive s are contiguous.
// For each of the 8 directions the neighbour spinor is spin-projected on load to a two-spin
// half-spinor (12 reals), multiplied by the link (or its adjoint) and reconstructed into the
// accumulator: 8 x (12 + 132) + 7 x 24 = 1320 flops per site. The output is written with
// non-temporal stores (Section 2.4: streaming stores in the final write).
#include "device.h"
#include "launch.h"

namespace gridmi {

template <int MU, int EF, class SP, class LK, typename C>
__device__ __forceinline__ void hop_dir(Cx<C> acc[4][3], const void *__restrict__ U, const void *__restrict__ psi,
                                        const float *__restrict__ psi_scale, int x4, const int nb[8], int Ls, int s) {
    Cx<C> p[4][3], h[2][3], u[3][3], chi[2][3];
    // forward: (1 + EF gamma_mu) U_mu(x) psi(x + mu)
    SP::load(psi, psi_scale, static_cast<size_t>(nb[2 * MU]) * Ls + s, p);
    project<MU, EF>(p, h);
    LK::load(U, static_cast<size_t>(x4) * 4 + MU, u);
    su3_mul(u, h, chi);
    reconstruct_add<MU, EF>(acc, chi);
    // backward: (1 - EF gamma_mu) U_mu(x - mu)^dagger psi(x - mu)
    SP::load(psi, psi_scale, static_cast<size_t>(nb[2 * MU + 1]) * Ls + s, p);
    project<MU, -EF>(p, h);
    LK::load(U, static_cast<size_t>(nb[2 * MU + 1]) * 4 + MU, u);
    su3_adj_mul(u, h, chi);
    reconstruct_add<MU, -EF>(acc, chi);
}

template <class SP, class LK, bool DAG, int KIND>
__global__ void __launch_bounds__(256)
k_dhop(const void *__restrict__ U, const void *__restrict__ psi, const float *__restrict__ psi_scale,
       void *__restrict__ out, float *__restrict__ out_scale, GeomDev g, double diag, double mf) {
    using C = typename SP::C;
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int t = lb * 256 + threadIdx.x;
    if (t >= g.n5) return;
    const int Ls = g.Ls;
    const int s = t % Ls;
    const int x4 = t / Ls;
    int nb[8];
    neighbours(g, x4, nb);

    Cx<C> acc[4][3];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k / 3][k % 3] = {C(0), C(0)};
    // H uses (1 - gamma) forward and (1 + gamma) backward; H^dagger the opposite.
    constexpr int EF = DAG ? +1 : -1;
    hop_dir<0, EF, SP, LK, C>(acc, U, psi, psi_scale, x4, nb, Ls, s);
    hop_dir<1, EF, SP, LK, C>(acc, U, psi, psi_scale, x4, nb, Ls, s);
    hop_dir<2, EF, SP, LK, C>(acc, U, psi, psi_scale, x4, nb, Ls, s);
    hop_dir<3, EF, SP, LK, C>(acc, U, psi, psi_scale, x4, nb, Ls, s);

    if (KIND == GRID_HOP) {
        SP::store(out, out_scale, t, acc);
        return;
    }
    // D = (4 + m) - H/2;  M = (5 - M5) - H/2 - (fifth-dimension hopping)
    Cx<C> p[4][3];
    SP::load(psi, psi_scale, t, p);
    const C d = static_cast<C>(diag);
    const C half = static_cast<C>(0.5);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const Cx<C> a = acc[k / 3][k % 3], v = p[k / 3][k % 3];
        acc[k / 3][k % 3] = {d * v.r - half * a.r, d * v.i - half * a.i};
    }
    if (KIND == GRID_DWF) {
        // M:   - P_- psi~_{s+1} - P_+ psi~_{s-1};  M^dagger: - P_+ psi~_{s+1} - P_- psi~_{s-1}
        // walls: psi~_{Ls} = -mf psi_0, psi~_{-1} = -mf psi_{Ls-1}
        const int sp = (s == Ls - 1) ? 0 : s + 1;
        const int sm = (s == 0) ? Ls - 1 : s - 1;
        const C fp = (s == Ls - 1) ? static_cast<C>(-mf) : C(1);
        const C fm = (s == 0) ? static_cast<C>(-mf) : C(1);
        const int hup = DAG ? 0 : 1;   // chiral half taken from s + 1 (0: spins 0,1; 1: spins 2,3)
        const int hdn = 1 - hup;       // chiral half taken from s - 1
        Cx<C> q[2][3];
        SP::load_half(psi, psi_scale, static_cast<size_t>(x4) * Ls + sp, hup, q);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            Cx<C> &o = acc[2 * hup + k / 3][k % 3];
            o = {o.r - fp * q[k / 3][k % 3].r, o.i - fp * q[k / 3][k % 3].i};
        }
        SP::load_half(psi, psi_scale, static_cast<size_t>(x4) * Ls + sm, hdn, q);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            Cx<C> &o = acc[2 * hdn + k / 3][k % 3];
            o = {o.r - fm * q[k / 3][k % 3].r, o.i - fm * q[k / 3][k % 3].i};
        }
    }
    SP::store(out, out_scale, t, acc);
}

template <class SP, class LK>
static hipError_t launch_T(const DhopArgs &a) {
    const int blocks = (a.g.n5 + 255) / 256;
    const dim3 grid(blocks), block(256);
    hipStream_t st = a.stream;
#define GRIDMI_LAUNCH(DAG, KIND)                                                                          \
    hipLaunchKernelGGL((k_dhop<SP, LK, DAG, KIND>), grid, block, 0, st, a.U, a.psi, a.psi_scale, a.out, \
                       a.out_scale, a.g, a.diag, a.mf)
    switch (a.kind * 2 + (a.dag ? 1 : 0)) {
        case GRID_HOP * 2 + 0: GRIDMI_LAUNCH(false, GRID_HOP); break;
        case GRID_HOP * 2 + 1: GRIDMI_LAUNCH(true, GRID_HOP); break;
        case GRID_WILSON * 2 + 0: GRIDMI_LAUNCH(false, GRID_WILSON); break;
        case GRID_WILSON * 2 + 1: GRIDMI_LAUNCH(true, GRID_WILSON); break;
        case GRID_DWF * 2 + 0: GRIDMI_LAUNCH(false, GRID_DWF); break;
        case GRID_DWF * 2 + 1: GRIDMI_LAUNCH(true, GRID_DWF); break;
        default: return hipErrorInvalidValue;
    }
#undef GRIDMI_LAUNCH
    return hipGetLastError();
}

hipError_t launch_dhop(const DhopArgs &a) {
    if (a.g.n5 == 0) return hipSuccess;
    switch (a.prec * 2 + a.link_fmt) {
        case GRID_F64 * 2 + GRID_L18: return launch_T<SpF64, LkF64<3>>(a);
        case GRID_F64 * 2 + GRID_L12: return launch_T<SpF64, LkF64<2>>(a);
        case GRID_F32 * 2 + GRID_L18: return launch_T<SpF32, LkF32<3>>(a);
        case GRID_F32 * 2 + GRID_L12: return launch_T<SpF32, LkF32<2>>(a);
        case GRID_F16S * 2 + GRID_L18: return launch_T<SpF16S, LkF16<3>>(a);
        case GRID_F16S * 2 + GRID_L12: return launch_T<SpF16S, LkF16<2>>(a);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gridmi
