// Tiled time-walk schedule of the hopping operator on 4D fields (gfx950).
//
// Why a third schedule. The column walk fetches each spinor record once per use (eight times)
// and each link once per lane, so it requests several times the compulsory bytes per site. Here
// neighbour reuse happens in LDS instead (Grid's observation, Section 3, that a neighbour spinor
// is used eight times, turned into on-chip reuse). It serves 4D fields in FP16 storage, where it
// is the fastest schedule measured.
//
// A block owns a TX x TY x TZ tile of (x, y, z) columns, one thread per column (a wavefront per
// z-plane of the tile), and walks T time slices. Per slice every thread writes its own record
// psi(x, t) to LDS, and the halo faces of slice t (loaded with coalesced 16-byte pieces during the
// previous slice) go beside it; the six spatial hops read LDS. The forward time neighbour
// psi(x, t + 1) is the thread's next centre and stays in registers; the backward time hop
// U_t(x, t-1)^dagger h(psi(x, t-1)) is formed one step ahead from the record and link already in
// hand and carried, as in the column walk. Links: a wavefront stages one direction's 64 links in
// its LDS area with coalesced loads (LinkStage) while the previous direction computes.
//
// Per site: 8 x (12 + 132) + 7 x 24 = 1320 flops, the convention of the flop counts quoted for
// this operator.
#include <type_traits>

#include "device.h"
#include "launch.h"

namespace gridmi {

template <int TX, int TY, int TZ>
struct TileShape {
    static constexpr int N = TX * TY * TZ;                 // interior columns = threads
    static constexpr int HX = TY * TZ, HY = TX * TZ, HZ = TX * TY;
    static constexpr int NH = 2 * (HX + HY + HZ);         // halo records (faces only)
    // halo slots after the interior: -x, +x, -y, +y, -z, +z faces
    static constexpr int XM = 0, XP = HX, YM = 2 * HX, YP = 2 * HX + HY, ZM = 2 * (HX + HY), ZP = ZM + HZ;
};

struct TileDev {
    int ntx, nty, ntz;   // tiles per direction
    int T;               // time slices per block
};

// Record of LDS slot `slot` (16-byte chunks at the record pitch), decoded into p.
template <class SP>
__device__ __forceinline__ void lds_record(const chunk_t *base, const float *sbase, int slot, Cx<typename SP::C> p[4][3]) {
    constexpr int CH = SP::kChunks;
    uint4 w[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const chunk_t v = base[slot * CH + k];
        w[k] = make_uint4(v.x, v.y, v.z, v.w);
    }
    SP::unpack(w, SP::kScaled ? sbase[slot] : 1.0f, p);
}

// Global chunk offset (relative to the start of a time slice) of chunk c of the tile's loads:
// c < N CH are the interior rows (row-major z, y, x, then chunk), the rest the halo faces.
template <int TX, int TY, int TZ, int CH>
__device__ __forceinline__ int tile_chunk_offset(const GeomDev &g, int x0, int y0, int z0, int c) {
    using S = TileShape<TX, TY, TZ>;
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2];
    int x, y, z, j;
    if (c < S::N * CH) {
        const int row = c / (TX * CH), off = c - row * (TX * CH);
        const int ry = row % TY, rz = row / TY;
        const int rx = off / CH;
        j = off - rx * CH;
        x = x0 + rx;
        y = y0 + ry;
        z = z0 + rz;
    } else {
        c -= S::N * CH;
        const int r = c / CH;
        j = c - r * CH;
        const int xm = x0 == 0 ? Lx - 1 : x0 - 1, xp = x0 + TX == Lx ? 0 : x0 + TX;
        const int ym = y0 == 0 ? Ly - 1 : y0 - 1, yp = y0 + TY == Ly ? 0 : y0 + TY;
        const int zm = z0 == 0 ? Lz - 1 : z0 - 1, zp = z0 + TZ == Lz ? 0 : z0 + TZ;
        if (r < S::YM) {                 // x faces: index over (y, z)
            const int i = r < S::XP ? r : r - S::XP;
            x = r < S::XP ? xm : xp;
            y = y0 + i % TY;
            z = z0 + i / TY;
        } else if (r < S::ZM) {          // y faces: index over (x, z)
            const int i = r < S::YP ? r - S::YM : r - S::YP;
            y = r < S::YP ? ym : yp;
            x = x0 + i % TX;
            z = z0 + i / TX;
        } else {                         // z faces: index over (x, y)
            const int i = r < S::ZP ? r - S::ZM : r - S::ZP;
            z = r < S::ZP ? zm : zp;
            x = x0 + i % TX;
            y = y0 + i / TX;
        }
    }
    return ((z * Ly + y) * Lx + x) * CH + j;
}

// Coalesced staging of one direction's links for a wavefront's 64 sites: the links of consecutive
// sites are LB-byte pieces at a 4 LB stride (site-major, four directions per site), so consecutive
// lanes load consecutive units of the same or the next link (unit = the largest of 16, 8, 4 bytes
// dividing LB), write them to the wavefront's LDS area in link order, and each lane then decodes
// its own link. A lane loading its own link directly instead touches a different cache line in
// every lane, which the vector-memory path serves several times slower.
template <class LK>
struct LinkStage {
    static constexpr int LB = LK::kBytes;
    static constexpr int kUnit = LB % 16 == 0 ? 16 : LB % 8 == 0 ? 8 : 4;
    static constexpr int kUnits = LB / kUnit;            // units per link = units per lane
    typedef unsigned int u2v __attribute__((ext_vector_type(2)));
    using T = std::conditional_t<kUnit == 16, chunk_t, std::conditional_t<kUnit == 8, u2v, uint32_t>>;
};

template <class SP, class LK, bool DAG, int KIND, int FUSE, int TX, int TY, int TZ>
__global__ void __launch_bounds__(TX * TY * TZ) __attribute__((amdgpu_waves_per_eu(2)))
k_dhop_tile(const void *__restrict__ U, const void *__restrict__ psi, const float *__restrict__ psi_scale, void *out,
            float *out_scale, GeomDev g, TileDev td, double diag, FuseDev fz) {
    using C = typename SP::C;
    using S = TileShape<TX, TY, TZ>;
    using LS = LinkStage<LK>;
    using LU = typename LS::T;
    static_assert(TX * TY == 64, "one wavefront per z-plane of the tile");
    constexpr int N = S::N, CH = SP::kChunks, NU = LS::kUnits;
    constexpr int KH = (S::NH * CH + N - 1) / N;         // halo chunks per thread
    __shared__ chunk_t sb[N * CH];                       // interior records of slice t
    __shared__ chunk_t sh[S::NH * CH];                   // halo records of slice t
    __shared__ float sbs[SP::kScaled ? N : 1];           // FP16 storage: per-record scales
    __shared__ float shs[SP::kScaled ? S::NH : 1];
    __shared__ LU sl[TZ][64 * NU];                       // per-wavefront link staging

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int ntiles = td.ntx * td.nty * td.ntz;
    const int seg = lb / ntiles, tile = lb - seg * ntiles;
    const int x0 = (tile % td.ntx) * TX, y0 = ((tile / td.ntx) % td.nty) * TY, z0 = (tile / (td.ntx * td.nty)) * TZ;
    const int cx = tid % TX, cy = (tid / TX) % TY, cz = tid / (TX * TY);
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
    const int V3 = Lx * Ly * Lz;
    const int x = x0 + cx, y = y0 + cy, z = z0 + cz;
    const int col = (z * Ly + y) * Lx + x;
    const int t0 = seg * td.T;
    constexpr int EF = DAG ? +1 : -1;

    // halo chunk offsets of this thread's loads (slice-relative, fixed along the walk)
    int hoff[KH];
#pragma unroll
    for (int k = 0; k < KH; ++k) {
        const int c = N * CH + k * N + tid;
        hoff[k] = c < (N + S::NH) * CH ? tile_chunk_offset<TX, TY, TZ, CH>(g, x0, y0, z0, c) : -1;
    }
    int hrec = -1;   // FP16 storage: this thread's halo scale
    if constexpr (SP::kScaled) {
        static_assert(!SP::kScaled || S::NH <= N, "one halo scale per thread");
        if (tid < S::NH) hrec = tile_chunk_offset<TX, TY, TZ, 1>(g, x0, y0, z0, N + tid);
    }
    // neighbour slots (LDS): interior slot or halo slot (>= N)
    const int own = tid;
    const int nxp = cx < TX - 1 ? own + 1 : N + S::XP + cy + TY * cz;
    const int nxm = cx > 0 ? own - 1 : N + S::XM + cy + TY * cz;
    const int nyp = cy < TY - 1 ? own + TX : N + S::YP + cx + TX * cz;
    const int nym = cy > 0 ? own - TX : N + S::YM + cx + TX * cz;
    const int nzp = cz < TZ - 1 ? own + TX * TY : N + S::ZP + cx + TX * cy;
    const int nzm = cz > 0 ? own - TX * TY : N + S::ZM + cx + TX * cy;
    // link staging: byte offset (within a time slice) of this lane's units of the forward link
    // of direction 0, and whether the unit's site sits on x = 0 / y = 0 (backward hops wrap)
    unsigned lofs[NU];
    unsigned wrapx = 0, wrapy = 0;
#pragma unroll
    for (int k = 0; k < NU; ++k) {
        const int u = k * 64 + lane, i = u / NU, j = u - (u / NU) * NU;
        const int xi = x0 + (i % TX), yi = y0 + (i / TX);
        lofs[k] = static_cast<unsigned>(((z * Ly + yi) * Lx + xi) * 4) * LS::LB + j * LS::kUnit;
        wrapx |= (xi == 0 ? 1u : 0u) << k;
        wrapy |= (yi == 0 ? 1u : 0u) << k;
    }
    const bool wrapz = z == 0;   // uniform over the wavefront
    LU *stage = sl[wv];
    const char *ub = static_cast<const char *>(U);
    // units of link U_mu(site - BWD mu-hat) at slice t for this lane's staging slots
    auto link_units = [&](int t, int mu, bool bwd, LU w[NU]) {
        const size_t tb = static_cast<size_t>(t) * V3 * 4 * LS::LB;
#pragma unroll
        for (int k = 0; k < NU; ++k) {
            long off = static_cast<long>(lofs[k]) + mu * LS::LB;
            if (bwd) {
                if (mu == 0) off += ((wrapx >> k) & 1) ? static_cast<long>(Lx - 1) * 4 * LS::LB : -4L * LS::LB;
                else if (mu == 1) off += ((wrapy >> k) & 1) ? static_cast<long>(Ly - 1) * Lx * 4 * LS::LB
                                                           : -static_cast<long>(Lx) * 4 * LS::LB;
                else off += wrapz ? static_cast<long>(Lz - 1) * Ly * Lx * 4 * LS::LB
                                  : -static_cast<long>(Ly) * Lx * 4 * LS::LB;
            }
            w[k] = *reinterpret_cast<const LU *>(ub + tb + off);
        }
    };
    // staged units -> LDS -> this lane's link
    auto link_take = [&](const LU w[NU], Cx<C> uu[3][3]) {
#pragma unroll
        for (int k = 0; k < NU; ++k) stage[k * 64 + lane] = w[k];
        wave_sync();
        LK::load(stage, lane, uu);
        wave_sync();   // every lane has its link before the area is reused
    };

    const chunk_t *src = reinterpret_cast<const chunk_t *>(psi);
    chunk_t wh[KH];
    float shv = 1.0f;
    auto issue_halo = [&](int t) {
        const size_t cbase = static_cast<size_t>(t) * V3 * CH;
#pragma unroll
        for (int j = 0; j < KH; ++j)
            if (hoff[j] >= 0) wh[j] = src[cbase + hoff[j]];
        if constexpr (SP::kScaled)
            if (hrec >= 0) shv = psi_scale[static_cast<size_t>(t) * V3 + hrec];
    };
    // raw record (chunks + scale) of this thread's column at slice tt
    auto own_raw = [&](int tt, uint4 w[CH], float &sc) {
        const size_t r = static_cast<size_t>(tt) * V3 + col;
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const chunk_t v = src[r * CH + j];
            w[j] = make_uint4(v.x, v.y, v.z, v.w);
        }
        sc = SP::kScaled ? psi_scale[r] : 1.0f;
    };
    Cx<C> chi_b[2][3], u[3][3], p[4][3];
    uint4 Pw[CH];      // centre record psi(x, t), raw
    float Ps = 1.0f;
    LU lw[NU];
    {
        // prologue: the backward time hop of slice t0, U_t(x, t0 - 1)^dagger h(psi(x, t0 - 1)),
        // the centre record psi(x, t0) and slice t0's halo
        const int tm = t0 == 0 ? Lt - 1 : t0 - 1;
        link_units(tm, 3, false, lw);
        SP::load(psi, psi_scale, static_cast<size_t>(tm) * V3 + col, p);
        own_raw(t0, Pw, Ps);
        issue_halo(t0);
        link_take(lw, u);
        Cx<C> hb[2][3];
        project<3, -EF>(p, hb);
        su3_adj_mul(u, hb, chi_b);
        link_units(t0, 0, false, lw);
    }
    [[maybe_unused]] double n2 = 0.0;
#pragma unroll 1
    for (int k = 0; k < td.T; ++k) {
        const int t = t0 + k;
        const int tn = t == Lt - 1 ? 0 : t + 1;
        // stage this thread's centre record and its share of the halo of slice t
#pragma unroll
        for (int j = 0; j < CH; ++j) sb[tid * CH + j] = chunk_t{Pw[j].x, Pw[j].y, Pw[j].z, Pw[j].w};
        if constexpr (SP::kScaled) sbs[tid] = Ps;
#pragma unroll
        for (int j = 0; j < KH; ++j)
            if (hoff[j] >= 0) sh[j * N + tid] = wh[j];
        if constexpr (SP::kScaled)
            if (hrec >= 0) shs[tid] = shv;
        __syncthreads();
        // the forward time neighbour psi(x, t + 1) (the next centre) and the next halo
        uint4 Qw[CH];
        float Qs = 1.0f;
        own_raw(tn, Qw, Qs);
        if (k + 1 < td.T) issue_halo(tn);
        auto rec = [&](int slot, Cx<C> q[4][3]) {
            if (slot < N)
                lds_record<SP>(sb, sbs, slot, q);
            else
                lds_record<SP>(sh, shs, slot - N, q);
        };
        Cx<C> acc[4][3];
#pragma unroll
        for (int j = 0; j < 12; ++j) acc[j / 3][j % 3] = {C(0), C(0)};
        reconstruct_add<3, -EF>(acc, chi_b);
        // spatial hops: links of the next direction are in flight while this one computes
        link_take(lw, u);
        link_units(t, 0, true, lw);
        rec(nxp, p);
        hop_term<0, EF, false>(acc, p, u);
        link_take(lw, u);
        link_units(t, 1, false, lw);
        rec(nxm, p);
        hop_term<0, -EF, true>(acc, p, u);
        link_take(lw, u);
        link_units(t, 1, true, lw);
        rec(nyp, p);
        hop_term<1, EF, false>(acc, p, u);
        link_take(lw, u);
        link_units(t, 2, false, lw);
        rec(nym, p);
        hop_term<1, -EF, true>(acc, p, u);
        link_take(lw, u);
        link_units(t, 2, true, lw);
        rec(nzp, p);
        hop_term<2, EF, false>(acc, p, u);
        link_take(lw, u);
        link_units(t, 3, false, lw);
        rec(nzm, p);
        hop_term<2, -EF, true>(acc, p, u);
        // forward time hop psi(x, t + 1) with U_t(x, t); the same link carries the backward time
        // hop of slice t + 1, U_t(x, t)^dagger h(psi(x, t))
        link_take(lw, u);
        if (k + 1 < td.T) link_units(tn, 0, false, lw);
        Cx<C> P[4][3];
        lds_record<SP>(sb, sbs, own, P);   // the centre psi(x, t), as staged
        {
            Cx<C> h[2][3], ch[2][3];
            SP::unpack(Qw, Qs, p);
            project<3, EF>(p, h);
            su3_mul(u, h, ch);
            reconstruct_add<3, EF>(acc, ch);
            project<3, -EF>(P, h);
            su3_adj_mul(u, h, chi_b);
        }
        if constexpr (KIND != GRID_HOP) {
            // D = (4 + m) - H/2
            const C dg = static_cast<C>(diag), half = static_cast<C>(0.5);
#pragma unroll
            for (int j = 0; j < 12; ++j) {
                const Cx<C> a = acc[j / 3][j % 3], v = P[j / 3][j % 3];
                acc[j / 3][j % 3] = {dg * v.r - half * a.r, dg * v.i - half * a.i};
            }
        }
        const size_t q = static_cast<size_t>(t) * V3 + col;
        if constexpr (FUSE == kFuseAxpy) {
            // r - alpha op psi; r may alias out: this thread reads its own record before storing it
            Cx<C> rv[4][3];
            SP::load(fz.r, fz.r_scale, q, rv);
            const C al = static_cast<C>(fz.scal[fz.num] / fz.scal[fz.den]);
#pragma unroll
            for (int j = 0; j < 12; ++j) {
                const Cx<C> a = acc[j / 3][j % 3], b = rv[j / 3][j % 3];
                acc[j / 3][j % 3] = {b.r - al * a.r, b.i - al * a.i};
            }
        }
        if constexpr (FUSE == kFuseNone)
            SP::store(out, out_scale, q, acc);
        else
            n2 += SP::store_n2(out, out_scale, q, acc);
#pragma unroll
        for (int j = 0; j < CH; ++j) Pw[j] = Qw[j];
        Ps = Qs;
        __syncthreads();   // the next slice overwrites the records read here
    }
    if constexpr (FUSE != kFuseNone) {
        n2 = wave_sum64(n2);
        constexpr int NW = N / 64;
        __shared__ double fred[NW];
        if ((tid & 63) == 0) fred[tid >> 6] = n2;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) s += fred[w];
            fz.part[blockIdx.x] = s;
        }
    }
}

// 4D: tile 8 x 8 x 4 (256 threads), walks of the longest divisor of Lt that keeps >= 1024 blocks
// (>= 1 otherwise).
constexpr int kTX = 8, kTY = 8, kTZ = 4;
static TileDev tile_dev(const GeomDev &g) {
    TileDev td;
    td.ntx = g.L[0] / kTX;
    td.nty = g.L[1] / kTY;
    td.ntz = g.L[2] / kTZ;
    const long ntiles = static_cast<long>(td.ntx) * td.nty * td.ntz;
    td.T = 1;
    for (int T = 1; T <= g.L[3]; ++T)
        if (g.L[3] % T == 0 && ntiles * (g.L[3] / T) >= 1024) td.T = T;
    return td;
}

// 4D FP16 storage only (86 against 93 us for the column walk, 74 against 132 us for the
// direction-parallel kernel at 32^4). 4D FP32 fields, 12-real links included, run faster on the
// direction-parallel kernel with its blocks as 4 x 2 x 2 x 2 boxes (32^4 12-real: 122.0 against
// 132.1 us here; 18-real: the eight direction wavefronts read a site's four links at about the
// same time, whereas this walk reads them one direction after another).
static bool tile4_applies(const DhopArgs &a) {
    const bool prec_ok = a.prec == GRID_F16S;
    return !a.custom && a.g.Ls == 1 && prec_ok && a.g.L[0] % kTX == 0 && a.g.L[1] % kTY == 0 &&
           a.g.L[2] % kTZ == 0 && (a.kind == GRID_HOP || a.kind == GRID_WILSON);
}

bool tile_applies(const DhopArgs &a) { return tile4_applies(a); }

long tile_blocks(const DhopArgs &a) {
    const TileDev td = tile_dev(a.g);
    return static_cast<long>(td.ntx) * td.nty * td.ntz * (a.g.L[3] / td.T);
}

template <class SP, class LK>
static hipError_t launch_tile_t(const DhopArgs &a) {
    const TileDev td = tile_dev(a.g);
    const dim3 grid(static_cast<unsigned>(tile_blocks(a))), block(kTX * kTY * kTZ);
    hipStream_t st = a.stream;
#define GRIDMI_LAUNCH(DAG, KIND, FUSE)                                                                          \
    hipLaunchKernelGGL((k_dhop_tile<SP, LK, DAG, KIND, FUSE, kTX, kTY, kTZ>), grid, block, 0, st, a.U, a.psi,      \
                       a.psi_scale, a.out, a.out_scale, a.g, td, a.diag, a.fz)
    if (a.fuse != kFuseNone) {
        switch (a.kind * 4 + a.fuse * 2 + (a.dag ? 1 : 0)) {
            case GRID_WILSON * 4 + kFuseNorm * 2 + 0: GRIDMI_LAUNCH(false, GRID_WILSON, kFuseNorm); break;
            case GRID_WILSON * 4 + kFuseAxpy * 2 + 1: GRIDMI_LAUNCH(true, GRID_WILSON, kFuseAxpy); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (a.kind * 2 + (a.dag ? 1 : 0)) {
        case GRID_HOP * 2 + 0: GRIDMI_LAUNCH(false, GRID_HOP, kFuseNone); break;
        case GRID_HOP * 2 + 1: GRIDMI_LAUNCH(true, GRID_HOP, kFuseNone); break;
        case GRID_WILSON * 2 + 0: GRIDMI_LAUNCH(false, GRID_WILSON, kFuseNone); break;
        case GRID_WILSON * 2 + 1: GRIDMI_LAUNCH(true, GRID_WILSON, kFuseNone); break;
        default: return hipErrorInvalidValue;
    }
#undef GRIDMI_LAUNCH
    return hipGetLastError();
}

hipError_t launch_tile(const DhopArgs &a) {
    switch (a.prec * 2 + a.link_fmt) {
        case GRID_F32 * 2 + GRID_L12: return launch_tile_t<SpF32, LkF32<2>>(a);
        case GRID_F16S * 2 + GRID_L18: return launch_tile_t<SpF16S, LkF16<3>>(a);
        case GRID_F16S * 2 + GRID_L12: return launch_tile_t<SpF16S, LkF16<2>>(a);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gridmi
