// Wilson hopping term, Wilson operator and Shamir domain-wall operator (gfx950).
//
// Work decomposition. A thread owns one 5D "column" q = (x, y, z, s) of a time slice (s is the
// fifth coordinate, fastest, so Ls consecutive lanes share a 4D site and its links; Ls = 1 for
// 4D fields) and walks T consecutive time slices t0 .. t0 + T - 1. Along the walk the t-hop terms
// are carried in registers: the backward hop of slice t, U_t(x, t-1)^dagger h(psi(x, t-1)), is
// computed at step t-1 from the link and spinor that step loads anyway, so each psi record and
// each U_t link is read once per walk instead of three and two times.
//
// Coalescing. The fields are site-major (a site's 12 complex numbers are contiguous), so a lane
// reading its own neighbour record touches a partial cache line per instruction. Neighbour
// records are therefore gathered per wavefront through LDS: lane l loads 16-byte chunk
// c = k*64 + l of the 64 records the wave needs (record c / chunks), i.e. consecutive lanes read
// consecutive addresses, and writes it to a padded LDS slot; each lane then reads its own record
// back. This is the MI355X form of Grid's observation (Section 2.1-2.2) that many small matrix-
// vector products in parallel, one per SIMD lane, need a data layout or staging that feeds the
// lanes contiguously.
//
// Per site: 8 x (spin projection 12 + SU(3) x half-spinor 132) + 7 x 24 reconstruction = 1320
// flops. Blocks are numbered so that each XCD receives a contiguous range of (time segment,
// column block) pairs, time segment slowest, i.e. a slab of time slices per XCD.
#include "device.h"
#include "launch.h"

namespace gridmi {

constexpr int kWaves = 4;   // wavefronts per block

// 3D neighbours of column index col (x fastest): nb[2 mu] = col + mu-hat, nb[2 mu + 1] = col - mu-hat.
__device__ __forceinline__ void neighbours3(const GeomDev &g, int col, int nb[6]) {
    int r = col, stride = 1;
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
        const int L = g.L[mu];
        const int c = (mu < 2) ? r % L : r;
        r = (mu < 2) ? r / L : 0;
        nb[2 * mu] = col + ((c == L - 1) ? (1 - L) * stride : stride);
        nb[2 * mu + 1] = col + ((c == 0) ? (L - 1) * stride : -stride);
        stride *= L;
    }
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Coalesced wavefront gather of spinor records through LDS, in two phases so that the global
// loads of the next gather can be in flight while the current direction computes:
//   fetch: lane l loads 16-byte chunk c = k*64 + l of the 64 records the wave needs (record
//          c / chunks, the record index of that lane obtained by a cross-lane shuffle), so
//          consecutive lanes read consecutive addresses;
//   stage: the chunks go to padded LDS slots and each lane reads its own record back.
// All 64 lanes must take part with a valid record index.
// 16-byte chunk as a native vector type (HIP's uint4 wraps a union, which keeps the in-flight
// chunks from being promoted to registers).
typedef unsigned int chunk_t __attribute__((ext_vector_type(4)));

template <class SP>
struct Fetch {
    chunk_t w[SP::kChunks];
    float s;
};

template <class SP>
__device__ __forceinline__ void fetch(const void *__restrict__ base, const float *__restrict__ scale, int rec,
                                      Fetch<SP> &f) {
    constexpr int CH = SP::kChunks;
    const int lane = threadIdx.x & 63;
    const chunk_t *src = reinterpret_cast<const chunk_t *>(base);
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const int c = k * 64 + lane;
        const int r = c / CH, j = c - (c / CH) * CH;
        const int n = __shfl(rec, r, 64);
        f.w[k] = src[static_cast<size_t>(n) * CH + j];
    }
    f.s = SP::kScaled ? scale[rec] : 1.0f;
}

template <class SP>
__device__ __forceinline__ void stage(const Fetch<SP> &f, chunk_t *lds, Cx<typename SP::C> p[4][3]) {
    constexpr int CH = SP::kChunks;
    constexpr int PITCH = CH + 1;   // padded record pitch (16-byte units) against bank conflicts
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const int c = k * 64 + lane;
        const int r = c / CH, j = c - (c / CH) * CH;
        lds[r * PITCH + j] = f.w[k];
    }
    wave_sync();
    uint4 w[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const chunk_t v = lds[lane * PITCH + k];
        w[k] = make_uint4(v.x, v.y, v.z, v.w);
    }
    wave_sync();
    SP::unpack(w, f.s, p);
}

template <class SP>
__device__ __forceinline__ void gather(const void *__restrict__ base, const float *__restrict__ scale, int rec, chunk_t *lds,
                                       Cx<typename SP::C> p[4][3]) {
    Fetch<SP> f;
    fetch<SP>(base, scale, rec, f);
    stage<SP>(f, lds, p);
}

// Pin the accumulator in registers at this point of the program. The only use of the result is
// the store of live lanes, so without this the compiler sinks all arithmetic below the last
// gather (which every lane must execute) and keeps every gathered record live at once.
template <typename C>
__device__ __forceinline__ void pin(Cx<C> a[4][3]) {
#pragma unroll
    for (int j = 0; j < 12; ++j) __asm__ volatile("" : "+v"(a[j / 3][j % 3].r), "+v"(a[j / 3][j % 3].i));
}

// acc += (1 + E gamma_MU) V psi with V = U (ADJ false) or U^dagger (ADJ true)
template <int MU, int E, bool ADJ, typename C>
__device__ __forceinline__ void hop_term(Cx<C> acc[4][3], const Cx<C> p[4][3], const Cx<C> u[3][3]) {
    Cx<C> h[2][3], chi[2][3];
    project<MU, E>(p, h);
    if (ADJ)
        su3_adj_mul(u, h, chi);
    else
        su3_mul(u, h, chi);
    reconstruct_add<MU, E>(acc, chi);
    pin(acc);
    // One direction at a time: hoisting later directions' loads above this point would raise
    // per-wave parallelism at a larger cost in occupancy.
    __builtin_amdgcn_sched_barrier(0);
}

template <class SP, class LK, bool DAG, int KIND>
__global__ void __launch_bounds__(256)
k_dhop(const void *__restrict__ U, const void *__restrict__ psi, const float *__restrict__ psi_scale,
       void *__restrict__ out, float *__restrict__ out_scale, GeomDev g, int T, double diag, double mf) {
    using C = typename SP::C;
    __shared__ chunk_t sm[kWaves][64 * (SP::kChunks + 1)];
    chunk_t *lds = sm[threadIdx.x >> 6];

    const int Ls = g.Ls;
    const int V3 = g.L[0] * g.L[1] * g.L[2];
    const int nq = V3 * Ls;                 // 5D sites per time slice
    const int nbc = (nq + 255) / 256;       // column blocks per slice
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int seg = lb / nbc, cb = lb - seg * nbc;
    const int q = cb * 256 + threadIdx.x;
    const bool live = q < nq;
    const int qq = live ? q : 0;            // idle lanes still take part in the wave's gathers
    const int col = qq / Ls, s = qq - (qq / Ls) * Ls;
    int nb[6];
    neighbours3(g, col, nb);
    const int Lt = g.L[3];
    const int t0 = seg * T;
    // H: (1 - gamma) forward, (1 + gamma) backward; H^dagger the opposite.
    constexpr int EF = DAG ? +1 : -1;

    Cx<C> chi_b[2][3], hb[2][3], p[4][3], u[3][3];
    {
        // backward t-hop of slice t0: U_t(x, t0 - 1)^dagger h(psi(x, t0 - 1))
        const int tm = (t0 == 0) ? Lt - 1 : t0 - 1;
        gather<SP>(psi, psi_scale, tm * nq + qq, lds, p);
        project<3, -EF>(p, hb);
        LK::load(U, (static_cast<size_t>(tm) * V3 + col) * 4 + 3, u);
        su3_adj_mul(u, hb, chi_b);
        gather<SP>(psi, psi_scale, t0 * nq + qq, lds, p);
        project<3, -EF>(p, hb);
    }
    // Records gathered per step, in order: psi(x, t+1), the six spatial neighbours at t, and the
    // centre psi(x, t) for the Wilson / domain-wall epilogue. The next record's loads are issued
    // before the current direction computes.
    constexpr int NREC = (KIND == GRID_HOP) ? 7 : 8;
#pragma unroll 1
    for (int k = 0; k < T; ++k) {
        const int t = t0 + k;
        const int off = t * nq;
        const size_t loff = static_cast<size_t>(t) * V3;
        const int tn = (t == Lt - 1) ? 0 : t + 1;
        int rec[NREC];
        rec[0] = tn * nq + qq;
#pragma unroll
        for (int d = 0; d < 6; ++d) rec[1 + d] = off + nb[d] * Ls + s;
        if (KIND != GRID_HOP) rec[7] = off + qq;
        Fetch<SP> f;
        fetch<SP>(psi, psi_scale, rec[0], f);
        Cx<C> acc[4][3];
#pragma unroll
        for (int j = 0; j < 12; ++j) acc[j / 3][j % 3] = {C(0), C(0)};
        reconstruct_add<3, -EF>(acc, chi_b);
#pragma unroll
        for (int i = 0; i < NREC; ++i) {
            stage<SP>(f, lds, p);
            // link of this direction first, then the next record: loads complete in issue order
            const int mu = (i == 0) ? 3 : (i - 1) / 2;
            const bool bwd = (i >= 1 && i <= 6 && ((i - 1) & 1));
            if (i <= 6) LK::load(U, (loff + (bwd ? nb[i - 1] : col)) * 4 + mu, u);
            if (i + 1 < NREC) fetch<SP>(psi, psi_scale, rec[i + 1], f);
            if (i == 0) {
                hop_term<3, EF, false>(acc, p, u);
                su3_adj_mul(u, hb, chi_b);       // backward t-hop of the next slice, same link
                project<3, -EF>(p, hb);
            } else if (i == 1) {
                hop_term<0, EF, false>(acc, p, u);
            } else if (i == 2) {
                hop_term<0, -EF, true>(acc, p, u);
            } else if (i == 3) {
                hop_term<1, EF, false>(acc, p, u);
            } else if (i == 4) {
                hop_term<1, -EF, true>(acc, p, u);
            } else if (i == 5) {
                hop_term<2, EF, false>(acc, p, u);
            } else if (i == 6) {
                hop_term<2, -EF, true>(acc, p, u);
            } else {
                // D = (4 + m) - H/2;  M = (5 - M5) - H/2 - (fifth-dimension hopping)
                const C dg = static_cast<C>(diag);
                const C half = static_cast<C>(0.5);
#pragma unroll
                for (int j = 0; j < 12; ++j) {
                    const Cx<C> a = acc[j / 3][j % 3], v = p[j / 3][j % 3];
                    acc[j / 3][j % 3] = {dg * v.r - half * a.r, dg * v.i - half * a.i};
                }
            }
        }
        if (KIND == GRID_DWF) {
            // M:   - P_- psi~_{s+1} - P_+ psi~_{s-1};  M^dagger: - P_+ psi~_{s+1} - P_- psi~_{s-1}
            // walls: psi~_{Ls} = -mf psi_0, psi~_{-1} = -mf psi_{Ls-1}
            const int sp = (s == Ls - 1) ? 0 : s + 1;
            const int sm1 = (s == 0) ? Ls - 1 : s - 1;
            const C fp = (s == Ls - 1) ? static_cast<C>(-mf) : C(1);
            const C fm = (s == 0) ? static_cast<C>(-mf) : C(1);
            const int hup = DAG ? 0 : 1;   // chiral half taken from s + 1 (0: spins 0,1; 1: spins 2,3)
            const int hdn = 1 - hup;
            const size_t site4 = static_cast<size_t>(off) + static_cast<size_t>(col) * Ls;
            Cx<C> qh[2][3];
            SP::load_half(psi, psi_scale, site4 + sp, hup, qh);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                Cx<C> &o = acc[2 * hup + j / 3][j % 3];
                o = {o.r - fp * qh[j / 3][j % 3].r, o.i - fp * qh[j / 3][j % 3].i};
            }
            SP::load_half(psi, psi_scale, site4 + sm1, hdn, qh);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                Cx<C> &o = acc[2 * hdn + j / 3][j % 3];
                o = {o.r - fm * qh[j / 3][j % 3].r, o.i - fm * qh[j / 3][j % 3].i};
            }
        }
        if (live) SP::store(out, out_scale, static_cast<size_t>(off) + q, acc);
    }
}

// Steps per thread: the longest walk (a divisor of Lt) that still leaves enough blocks to fill
// the chip; small lattices use T = 1.
static int choose_steps(const GeomDev &g) {
    constexpr long kMinBlocks = 1024;
    const long nbc = (static_cast<long>(g.L[0]) * g.L[1] * g.L[2] * g.Ls + 255) / 256;
    int best = 1;
    for (int T = 1; T <= g.L[3]; ++T)
        if (g.L[3] % T == 0 && nbc * (g.L[3] / T) >= kMinBlocks) best = T;
    return best;
}

template <class SP, class LK>
static hipError_t launch_T(const DhopArgs &a) {
    const int T = choose_steps(a.g);
    const long nbc = (static_cast<long>(a.g.L[0]) * a.g.L[1] * a.g.L[2] * a.g.Ls + 255) / 256;
    const dim3 grid(static_cast<unsigned>(nbc * (a.g.L[3] / T))), block(256);
    hipStream_t st = a.stream;
#define GRIDMI_LAUNCH(DAG, KIND)                                                                          \
    hipLaunchKernelGGL((k_dhop<SP, LK, DAG, KIND>), grid, block, 0, st, a.U, a.psi, a.psi_scale, a.out, \
                       a.out_scale, a.g, T, a.diag, a.mf)
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
