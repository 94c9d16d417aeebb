// Wilson hopping term, Wilson operator and Shamir domain-wall operator (gfx950).
//
// Two schedules of the same operator share this file; launch_dhop picks one by field type.
//
// Direction-parallel schedule (4D fields in FP64 and FP32). A block owns 32 consecutive 5D sites of a traversal order and runs 8
// wavefronts, one per hopping direction (mu = 0..3, forward and backward). In phase 1 wavefront d
// computes, for every site of the block, the spin-projected neighbour h = (1 -/+ gamma_mu) psi and
// its parallel transport chi = U h (forward) or U^dagger h (backward); two lanes share a site, one
// per spin of the half-spinor, so every lane does one 3x3 complex matrix-vector product. In FP64
// the two lanes of a site are l and l + 32 and split the link's loads between them (measured
// faster for FP64, slower for FP32, which keeps lanes 2 l and 2 l + 1 and whole-link loads). The
// eight chi per site meet in LDS, and in phase 2 sixteen lanes per site (twelve active, one per
// output spin-colour component) reconstruct the lower spins, sum the directions, apply the
// Wilson or domain-wall diagonal and fifth-dimension terms and store the component. All eight
// neighbour records and links of a site are in flight at once, which is what feeds HBM when the
// lattice is small (a 16^4 lattice has only 65536 sites for 256 compute units).
//
// Coalescing. The fields are site-major (a site's 12 complex numbers are contiguous), so a lane
// reading its own neighbour record touches a partial cache line per instruction. Neighbour
// records are therefore gathered per wavefront through LDS: consecutive lanes read consecutive
// 16-byte chunks of the 32 records the wavefront needs and write them to padded LDS slots, from
// which each lane reads the spins it projects. This is the MI355X form of Grid's observation
// (Sections 2.1-2.2) that many small matrix-vector products in parallel, one per SIMD lane, need
// a data layout or staging that feeds the lanes contiguously.
//
// Traversal. Blocks are renumbered so that each XCD receives a contiguous range of the traversal
// order, which is one of 8 sub-lattices (x, y and z halved) swept along t: a record's eight uses
// then fall within a few cross-sections of that sub-lattice and mostly stay in the XCD's L2, and
// only the sub-lattice faces are read by two XCDs.
//
// Per site: 8 x (spin projection 12 + SU(3) x half-spinor 132) + 7 x 24 reconstruction = 1320
// flops, the convention of the flop counts quoted for this operator.
#include "device.h"
#include "launch.h"

namespace gridmi {

constexpr int kSites = 32;           // 5D sites per block
constexpr int kDirs = 8;             // wavefronts per block, one per hopping direction
constexpr int kBlock = kDirs * 64;   // threads per block

// Division by a launch-invariant divisor d >= 1 for 0 <= n < 2^31: q = (umulhi(n, m) + n) >> l with
// l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1 (Granlund and Montgomery's division by
// invariant integers; n + umulhi(n, m) < 2^32 because n < 2^31).
struct FastDiv {
    uint32_t m, l;
};

static FastDiv make_fastdiv(int d) {
    uint32_t l = 0;
    while ((1u << l) < static_cast<uint32_t>(d)) ++l;
    const uint64_t m = ((uint64_t(1) << 32) * ((uint64_t(1) << l) - static_cast<uint64_t>(d))) / static_cast<uint64_t>(d) + 1;
    return {static_cast<uint32_t>(m), l};
}

__device__ __forceinline__ int fdiv(int n, FastDiv f) {
    return static_cast<int>((__umulhi(static_cast<uint32_t>(n), f.m) + static_cast<uint32_t>(n)) >> f.l);
}

// Traversal order: 8 XCD domains, one per contiguous eighth of the block order (x halved for
// checkerboard output).
//   mode 0: the halves of x and y and the halves or quarters of z (quarters: 16 domains, two per
//           XCD);
//           inside a domain s, x, y, z, t (t slowest, so the domain is swept along t with a
//           fraction of a time slice as cross-section); domain slowest;
//   mode 1: slabs of Lt / 8 time slices; inside s, x, y, t, z (z slowest); slab slowest;
//   mode 2: one domain in memory order s, x, y, z, t.
// With `box` (mode 0, 4D FP32 fields) the domain is covered by 4 x 2 x 2 x 2 boxes of 32 sites, one
// per block, in x, y, z, t order.
// For checkerboard output (cbp = 0 / 1) the site of parity cbp in each x pair is taken.
struct Trav {
    FastDiv ls, e0, e1, e2, e3;
    int en0, en1, en2, en3;   // domain extents
    int box;                  // mode 0 on 4D fields: blocks are 4 x 2 x 2 x 2 boxes of the domain
    FastDiv b0, b1, b2, b3;   // boxes per domain extent
    int bn0, bn1, bn2, bn3;
    int mode;
    int cbp;                  // output checkerboard, -1 for the full lattice
    int nout;                 // 5D sites written
};

// Block boxes of the direction-parallel kernel on 4D FP32 fields: a block's 32 sites as a 4 x 2 x
// 2 x 2 box instead of two x-rows of 16 (their 256 neighbour records are 144 distinct ones instead
// of 196, and fewer partial lines of links). Measured at 32^4: 142.5 -> 136.0 us in FP32; other
// shapes (8x2x2x1, 4x4x2x1, 4x2x4x1, 2x2x2x4) 141-153 us; FP64 is faster with rows (274 against
// 276-292 us), so it keeps them.
constexpr int kBox0 = 4, kBox1 = 2, kBox2 = 2, kBox3 = 2;
static_assert(kBox0 * kBox1 * kBox2 * kBox3 == 32, "a box holds a block's 32 sites");

// Traversal index j -> coordinates, 4D site and s.
__device__ __forceinline__ void trav_decode(const GeomDev &g, const Trav &tr, int j, int x[4], int &site4, int &s) {
    if (tr.box) {
        // 32 consecutive sites form a kBox0 x kBox1 x kBox2 x kBox3 box; boxes in x, y, z, t order,
        // domain slowest
        s = 0;
        const int k = j & 31;
        int b = j >> 5, q;
        q = fdiv(b, tr.b0);
        x[0] = (b - q * tr.bn0) * kBox0 + (k % kBox0);
        b = q;
        q = fdiv(b, tr.b1);
        x[1] = (b - q * tr.bn1) * kBox1 + (k / kBox0) % kBox1;
        b = q;
        q = fdiv(b, tr.b2);
        x[2] = (b - q * tr.bn2) * kBox2 + (k / (kBox0 * kBox1)) % kBox2;
        b = q;
        q = fdiv(b, tr.b3);
        x[3] = (b - q * tr.bn3) * kBox3 + k / (kBox0 * kBox1 * kBox2);
        x[0] += (q & 1) * tr.en0;
        x[1] += ((q >> 1) & 1) * tr.en1;
        x[2] += (q >> 2) * tr.en2;
        site4 = x[0] + g.L[0] * (x[1] + g.L[1] * (x[2] + g.L[2] * x[3]));
        return;
    }
    int q = fdiv(j, tr.ls);
    s = j - q * g.Ls;
    j = q;
    q = fdiv(j, tr.e0);
    x[0] = j - q * tr.en0;
    j = q;
    q = fdiv(j, tr.e1);
    x[1] = j - q * tr.en1;
    j = q;
    if (tr.mode == 1) {
        q = fdiv(j, tr.e3);
        x[3] = j - q * tr.en3;
        j = q;
        q = fdiv(j, tr.e2);
        x[2] = j - q * tr.en2;
        x[3] += q * tr.en3;
    } else {
        q = fdiv(j, tr.e2);
        x[2] = j - q * tr.en2;
        j = q;
        q = fdiv(j, tr.e3);
        x[3] = j - q * tr.en3;
        // domain index q (0 in mode 2)
        x[0] += (q & 1) * tr.en0;
        x[1] += ((q >> 1) & 1) * tr.en1;
        x[2] += (q >> 2) * tr.en2;   // up to 3 when z is quartered
    }
    if (tr.cbp >= 0) x[0] = 2 * x[0] + ((x[1] + x[2] + x[3] + tr.cbp) & 1);
    site4 = x[0] + g.L[0] * (x[1] + g.L[1] * (x[2] + g.L[2] * x[3]));
}

template <int MU>
__device__ __forceinline__ int stride_of(const GeomDev &g) {
    return MU == 0 ? 1 : MU == 1 ? g.L[0] : MU == 2 ? g.L[0] * g.L[1] : g.L[0] * g.L[1] * g.L[2];
}

// The split link load of a link type (FP64 links only; a placeholder otherwise).
template <class LK, bool S>
struct SplitOf {
    using type = SplitLoad<uint32_t, 1>;
};
template <class LK>
struct SplitOf<LK, true> {
    using type = SplitLoad<typename LK::E, LK::kN>;
};

// Phase 1, direction (MU, BWD): chi = U_mu(x) h(psi(x + mu)) or U_mu(x - mu)^dagger h(psi(x - mu))
// with h = (1 + E gamma_mu) psi projected; lane spin sp of the half-spinor. The result goes to
// the wavefront's LDS area as red[site][sp][colour].
template <class SP, class LK, int MU, bool BWD, int E>
__device__ __forceinline__ void dir_term(const void *__restrict__ U, const void *__restrict__ psi,
                                         const float *__restrict__ psi_scale, const GeomDev &g, const int x[4],
                                         int site4, int s, int sl, int sp, int cbin, chunk_t *lds) {
    using C = typename SP::C;
    constexpr int CH = SP::kChunks, PITCH = CH + 1;
    const int lane = threadIdx.x & 63;
    const int L = g.L[MU], st = stride_of<MU>(g);
    const int nb4 = BWD ? (x[MU] == 0 ? site4 + (L - 1) * st : site4 - st)
                        : (x[MU] == L - 1 ? site4 - (L - 1) * st : site4 + st);
    const int rec = (nb4 >> cbin) * g.Ls + s;   // checkerboard input: half-volume index
    // coalesced fetch of the 32 records (record r is named by lane r (split) or 2r)
    constexpr bool kSplit = sizeof(C) == 8;
    const chunk_t *src = reinterpret_cast<const chunk_t *>(psi);
    constexpr int NCH = kSites * CH, NK = (NCH + 63) / 64;
    chunk_t w[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        const int c = k * 64 + lane;
        const int cc = c < NCH ? c : 0;
        const int r = cc / CH, j = cc - r * CH;
        const int n = __shfl(rec, kSplit ? r : 2 * r, 64);
        w[k] = src[static_cast<size_t>(n) * CH + j];
    }
    const float sc = SP::kScaled ? psi_scale[rec] : 1.0f;
    const size_t link = static_cast<size_t>(BWD ? nb4 : site4) * 4 + MU;
    Cx<C> u[3][3];
    [[maybe_unused]] typename SplitOf<LK, kSplit>::type lk;
    if constexpr (kSplit) {
        lk.issue(LK::elems(U, link), sp);
        // every load of this direction is issued before anything waits on one
        __builtin_amdgcn_sched_barrier(0);
    } else {
        LK::load(U, link, u);
    }
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        const int c = k * 64 + lane;
        if (c < NCH) {
            const int r = c / CH, j = c - r * CH;
            lds[r * PITCH + j] = w[k];
        }
    }
    wave_sync();
    // h_sp = psi_sp + E * phase * psi_src
    const chunk_t *rp = lds + sl * PITCH;
    const int srcs = (MU < 2) ? 3 - sp : 2 + sp;
    const C e = static_cast<C>(E);
    const C sg = sp ? C(1) : C(-1);
    Cx<C> h[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const Cx<C> pu = Elem<SP>::get(rp, sp * 3 + c, sc);
        const Cx<C> pd = Elem<SP>::get(rp, srcs * 3 + c, sc);
        if (MU == 0)        // -i
            h[c] = {pu.r + e * pd.i, pu.i - e * pd.r};
        else if (MU == 1)   // -1 (sp 0), +1 (sp 1)
            h[c] = {pu.r + e * sg * pd.r, pu.i + e * sg * pd.i};
        else if (MU == 2)   // -i (sp 0), +i (sp 1)
            h[c] = {pu.r - e * sg * pd.i, pu.i + e * sg * pd.r};
        else
            h[c] = {pu.r + e * pd.r, pu.i + e * pd.i};
    }
    wave_sync();   // every lane has read its record before the area is reused for chi
    if constexpr (kSplit) {
        typename LK::E e[LK::kN];
        lk.finish(e);
        LK::decode(e, u);
    }
    Cx<C> *red = reinterpret_cast<Cx<C> *>(lds);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        Cx<C> acc;
        if (BWD) {
            acc = cmulc(u[0][a], h[0]);
            acc = cmacc(acc, u[1][a], h[1]);
            acc = cmacc(acc, u[2][a], h[2]);
        } else {
            acc = cmul(u[a][0], h[0]);
            acc = cmac(acc, u[a][1], h[1]);
            acc = cmac(acc, u[a][2], h[2]);
        }
        red[(sl * 2 + sp) * 3 + a] = acc;
    }
}

template <class SP, class LK, bool DAG, int KIND, int FUSE>
__global__ void __launch_bounds__(kBlock)
k_dhop_dir(const void *__restrict__ U, const void *__restrict__ psi, const float *__restrict__ psi_scale,
           const void *__restrict__ yv, const float *__restrict__ y_scale, void *out, float *out_scale, GeomDev g,
           Trav tr, double diag, double mf, double beta, double cs, FuseDev fz) {
    using C = typename SP::C;
    constexpr int PITCH = SP::kChunks + 1;
    __shared__ chunk_t sm[kDirs][kSites * PITCH];
    __shared__ int2 sinfo[kSites];   // (4D site, s) of the block's sites, for phase 2
    __shared__ double fred[kDirs];   // fused epilogue: per-wavefront sums and their arrival count
    __shared__ int fcount;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int base = xcd_block(blockIdx.x, gridDim.x) * kSites;
    // H: (1 - gamma) forward, (1 + gamma) backward; H^dagger the opposite.
    constexpr int EF = DAG ? +1 : -1;
    {
        constexpr bool kSplit = sizeof(C) == 8;   // lanes l, l + 32 share site l in FP64
        const int sl = kSplit ? (lane & 31) : (lane >> 1), sp = kSplit ? (lane >> 5) : (lane & 1);
        const int j = min(base + sl, tr.nout - 1);   // idle lanes of a ragged block still take part
        int x[4], site4, s;
        trav_decode(g, tr, j, x, site4, s);
        if (wv == 0 && sp == 0) sinfo[sl] = make_int2(site4, s);
        if (FUSE != kFuseNone && threadIdx.x == 0) fcount = 0;
        chunk_t *lds = sm[wv];
        const int cbin = tr.cbp >= 0 ? 1 : 0;
        switch (wv) {
            case 0: dir_term<SP, LK, 0, false, EF>(U, psi, psi_scale, g, x, site4, s, sl, sp, cbin, lds); break;
            case 1: dir_term<SP, LK, 0, true, -EF>(U, psi, psi_scale, g, x, site4, s, sl, sp, cbin, lds); break;
            case 2: dir_term<SP, LK, 1, false, EF>(U, psi, psi_scale, g, x, site4, s, sl, sp, cbin, lds); break;
            case 3: dir_term<SP, LK, 1, true, -EF>(U, psi, psi_scale, g, x, site4, s, sl, sp, cbin, lds); break;
            case 4: dir_term<SP, LK, 2, false, EF>(U, psi, psi_scale, g, x, site4, s, sl, sp, cbin, lds); break;
            case 5: dir_term<SP, LK, 2, true, -EF>(U, psi, psi_scale, g, x, site4, s, sl, sp, cbin, lds); break;
            case 6: dir_term<SP, LK, 3, false, EF>(U, psi, psi_scale, g, x, site4, s, sl, sp, cbin, lds); break;
            default: dir_term<SP, LK, 3, true, -EF>(U, psi, psi_scale, g, x, site4, s, sl, sp, cbin, lds); break;
        }
    }
    __syncthreads();
    // Phase 2: lane (site sl, component k = 3 a + c); lanes 12..15 of a site are idle.
    const int sl = threadIdx.x >> 4, k16 = threadIdx.x & 15;
    const int j = base + sl;
    const bool live = j < tr.nout && k16 < 12;
    const int k = k16 < 12 ? k16 : 0;
    const int a = k / 3, c = k - 3 * (k / 3);
    const bool up = a < 2;
    const int a2 = a - 2;
    const C sgn = up ? C(1) : C(-1);
    Cx<C> acc = {C(0), C(0)};
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        // upper: chi_f[a] + chi_b[a]; lower: EF * phase * (chi_f - chi_b)[src]
        int src;
        C pr, pi;   // phase of the lower reconstruction, times EF
        if (mu == 0) { src = 1 - a2; pr = 0; pi = EF; }                         // i
        else if (mu == 1) { src = 1 - a2; pr = a2 ? -EF : EF; pi = 0; }         // +1 / -1
        else if (mu == 2) { src = a2; pr = 0; pi = a2 ? -EF : EF; }             // i / -i
        else { src = a2; pr = EF; pi = 0; }                                     // 1
        if (up) { src = a; pr = 1; pi = 0; }
        const Cx<C> *rf = reinterpret_cast<const Cx<C> *>(sm[2 * mu]);
        const Cx<C> *rb = reinterpret_cast<const Cx<C> *>(sm[2 * mu + 1]);
        const Cx<C> f = rf[(sl * 2 + src) * 3 + c], b = rb[(sl * 2 + src) * 3 + c];
        const Cx<C> d = {f.r + sgn * b.r, f.i + sgn * b.i};
        acc = {acc.r + pr * d.r - pi * d.i, acc.i + pr * d.i + pi * d.r};
    }
    const int2 si = sinfo[sl];
    const int site4o = si.x >> (tr.cbp >= 0 ? 1 : 0), s = si.y;   // output (checkerboard) 4D index
    const size_t q = static_cast<size_t>(site4o) * g.Ls + s;
    const C bt = static_cast<C>(beta);
    if (KIND == GRID_HOP) {
        acc = {bt * acc.r, bt * acc.i};
    } else {
        // D = (4 + m) - H/2;  M = (5 - M5) - H/2 - (fifth-dimension hopping); the diagonal part
        // acts on y (= psi on the full lattice), H is scaled by beta (= -1/2 there)
        const Cx<C> v = global_elem<SP>(yv, y_scale, q, k);
        const C dg = static_cast<C>(diag);
        acc = {dg * v.r + bt * acc.r, dg * v.i + bt * acc.i};
    }
    if (KIND == GRID_DWF) {
        // M:   - P_- psi~_{s+1} - P_+ psi~_{s-1};  M^dagger: - P_+ psi~_{s+1} - P_- psi~_{s-1}
        // walls: psi~_{Ls} = -mf psi_0, psi~_{-1} = -mf psi_{Ls-1}
        const int Ls = g.Ls;
        const int hup = DAG ? 0 : 1;   // chiral half taken from s + 1 (0: spins 0,1; 1: spins 2,3)
        const bool from_up = (a >> 1) == hup;
        const int s2 = from_up ? (s == Ls - 1 ? 0 : s + 1) : (s == 0 ? Ls - 1 : s - 1);
        const C f = static_cast<C>(cs) *
                    (from_up ? (s == Ls - 1 ? static_cast<C>(-mf) : C(1)) : (s == 0 ? static_cast<C>(-mf) : C(1)));
        const Cx<C> v = global_elem<SP>(yv, y_scale, static_cast<size_t>(site4o) * Ls + s2, k);
        acc = {acc.r - f * v.r, acc.i - f * v.i};
    }
    if constexpr (FUSE == kFuseNone) {
        store_elem<SP>(out, out_scale, q, k, acc, live);
    } else {
        if constexpr (FUSE == kFuseAxpy) {
            // r - alpha op psi; r may alias out: this lane reads its own element (and the site
            // scale) before any lane of the site stores
            const Cx<C> rv = global_elem<SP>(fz.r, fz.r_scale, q, k);
            const C al = static_cast<C>(fz.scal[fz.num] / fz.scal[fz.den]);
            acc = {rv.r - al * acc.r, rv.i - al * acc.i};
        }
        // Block sum without a block barrier: each wavefront posts its sum and counts itself in;
        // the last one to arrive adds the eight in a fixed order (reproducible whichever it is).
        const double n2 = wave_sum64(stored_n2<SP>(acc, live));
        if (lane == 0) {
            fred[wv] = n2;
            if (__hip_atomic_fetch_add(&fcount, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP) == kDirs - 1) {
                double t = 0.0;
#pragma unroll
                for (int w = 0; w < kDirs; ++w) t += fred[w];
                fz.part[blockIdx.x] = t;
            }
        }
        store_elem<SP>(out, out_scale, q, k, acc, live);
    }
}

// XCD domains: halves of x and y and quarters of z when the extents allow (16 domains, two
// consecutive ones per XCD), else halves of x, y, z, else slabs of t when Lt is a multiple of 8,
// else a single domain.
static Trav make_trav(const GeomDev &g, int cb, bool boxes = false) {
    Trav tr{};
    tr.cbp = cb;
    tr.nout = cb >= 0 ? g.n5 / 2 : g.n5;
    int e[4] = {cb >= 0 ? g.L[0] / 2 : g.L[0], g.L[1], g.L[2], g.L[3]};
    if (e[0] % 2 == 0 && e[1] % 2 == 0 && e[2] % 4 == 0) {
        // quartering z halves the cross-section an XCD sweeps along t: a time slice of it (records
        // and links) and the previous one then fit the XCD's L2 together, so the t-neighbours'
        // records and links are reused from it (32^4 FP32: reads 1.43 -> 1.30 times the compulsory
        // bytes), at the price of two more z-faces per domain
        tr.mode = 0;
        e[0] /= 2;
        e[1] /= 2;
        e[2] /= 4;
    } else if (e[0] % 2 == 0 && e[1] % 2 == 0 && e[2] % 2 == 0) {
        tr.mode = 0;
        e[0] /= 2;
        e[1] /= 2;
        e[2] /= 2;
    } else if (e[3] % 8 == 0) {
        tr.mode = 1;
        e[3] /= 8;
    } else {
        tr.mode = 2;
    }
    tr.ls = make_fastdiv(g.Ls);
    tr.en0 = e[0];
    tr.en1 = e[1];
    tr.en2 = e[2];
    tr.en3 = e[3];
    tr.e0 = make_fastdiv(e[0]);
    tr.e1 = make_fastdiv(e[1]);
    tr.e2 = make_fastdiv(e[2]);
    tr.e3 = make_fastdiv(e[3]);
    tr.box = (boxes && tr.mode == 0 && g.Ls == 1 && cb < 0 && e[0] % kBox0 == 0 && e[1] % kBox1 == 0 && e[2] % kBox2 == 0 &&
              e[3] % kBox3 == 0) ? 1 : 0;
    tr.bn0 = e[0] / kBox0;
    tr.bn1 = e[1] / kBox1;
    tr.bn2 = e[2] / kBox2;
    tr.bn3 = e[3] / kBox3;
    if (tr.box) {
        tr.b0 = make_fastdiv(tr.bn0);
        tr.b1 = make_fastdiv(tr.bn1);
        tr.b2 = make_fastdiv(tr.bn2);
        tr.b3 = make_fastdiv(tr.bn3);
    }
    return tr;
}

template <class SP, class LK>
static hipError_t launch_dir(const DhopArgs &a) {
    const Trav tr = make_trav(a.g, a.custom ? a.cb : -1, a.prec == GRID_F32);
    const long nblocks = (static_cast<long>(tr.nout) + kSites - 1) / kSites;
    const void *y = a.custom ? a.y : a.psi;
    const float *ys = a.custom ? a.y_scale : a.psi_scale;
    const double beta = a.custom ? a.beta : (a.kind == GRID_HOP ? 1.0 : -0.5);
    const double cs = a.custom ? a.cs : 1.0;
    const dim3 grid(static_cast<unsigned>(nblocks)), block(kBlock);
    hipStream_t st = a.stream;
#define GRIDMI_LAUNCH(DAG, KIND, FUSE)                                                                    \
    hipLaunchKernelGGL((k_dhop_dir<SP, LK, DAG, KIND, FUSE>), grid, block, 0, st, a.U, a.psi, a.psi_scale, y, ys, \
                       a.out, a.out_scale, a.g, tr, a.diag, a.mf, beta, cs, a.fz)
    if (a.fuse != kFuseNone) {
        switch (a.kind * 4 + a.fuse * 2 + (a.dag ? 1 : 0)) {
            case GRID_WILSON * 4 + kFuseNorm * 2 + 0: GRIDMI_LAUNCH(false, GRID_WILSON, kFuseNorm); break;
            case GRID_DWF * 4 + kFuseNorm * 2 + 0: GRIDMI_LAUNCH(false, GRID_DWF, kFuseNorm); break;
            case GRID_WILSON * 4 + kFuseAxpy * 2 + 1: GRIDMI_LAUNCH(true, GRID_WILSON, kFuseAxpy); break;
            case GRID_DWF * 4 + kFuseAxpy * 2 + 1: GRIDMI_LAUNCH(true, GRID_DWF, kFuseAxpy); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (a.kind * 2 + (a.dag ? 1 : 0)) {
        case GRID_HOP * 2 + 0: GRIDMI_LAUNCH(false, GRID_HOP, kFuseNone); break;
        case GRID_HOP * 2 + 1: GRIDMI_LAUNCH(true, GRID_HOP, kFuseNone); break;
        case GRID_WILSON * 2 + 0: GRIDMI_LAUNCH(false, GRID_WILSON, kFuseNone); break;
        case GRID_WILSON * 2 + 1: GRIDMI_LAUNCH(true, GRID_WILSON, kFuseNone); break;
        case GRID_DWF * 2 + 0: GRIDMI_LAUNCH(false, GRID_DWF, kFuseNone); break;
        case GRID_DWF * 2 + 1: GRIDMI_LAUNCH(true, GRID_DWF, kFuseNone); break;
        default: return hipErrorInvalidValue;
    }
#undef GRIDMI_LAUNCH
    return hipGetLastError();
}

// ============================================================================================
// Column-walk schedule (domain-wall fields and FP16 storage).
//
// A thread owns one 5D "column" q = (x, y, z, s) of a time slice (s fastest, so Ls consecutive
// lanes share a 4D site and its links) and walks T consecutive time slices t0 .. t0 + T - 1.
// Along the walk the t-hop terms are carried in registers: the backward hop of slice t,
// U_t(x, t-1)^dagger h(psi(x, t-1)), is computed at step t-1 from the link and spinor that step
// loads anyway, so each psi record and each U_t link is read once per walk. Neighbour records are
// gathered per wavefront through LDS (64 records per gather), and the gather of the next record is
// in flight while the current direction computes. With one thread per 5D site this schedule
// spends far fewer instructions per site than the direction-parallel one, which is what the
// ALU-heavy FP16 decode and the Ls-fold link reuse of the fifth dimension need.
// ============================================================================================

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


template <class SP, class LK, bool DAG, int KIND, int FUSE>
__global__ void __launch_bounds__(256)
k_dhop_walk(const void *__restrict__ U, const void *__restrict__ psi, const float *__restrict__ psi_scale,
       const void *__restrict__ yv, const float *__restrict__ y_scale, void *out, float *out_scale, GeomDev g, int T,
       double diag, double mf, double cs, double b5, double c5, FuseDev fz) {
    using C = typename SP::C;
    // Moebius (KIND GRID_MOBIUS, y = psi, Ls dividing 64): M psi gathers chi = B psi, B = b5 + c5 S,
    // for the hopping records (stage_b5) and ends like the domain-wall operator with diag =
    // 1 + (4 - M5) b5 and cs = 1 - (4 - M5) c5; M^dagger psi forms w = (4 - M5) psi - H^dagger psi / 2
    // (diag = 4 - M5) and then b5 w + psi + S^dagger (c5 w - psi) across the column's lanes.
    constexpr bool MOBF = KIND == GRID_MOBIUS && !DAG;
    constexpr bool MOBA = KIND == GRID_MOBIUS && DAG;
    __shared__ chunk_t sm[kWaves][64 * stage_pitch<SP>()];
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
    // Moebius: the column's lanes of s + 1 and s - 1 and the wall factors
    int lp = 0, lm = 0;
    C mb5 = C(0), mc5 = C(0), wp = C(1), wm = C(1);
    if constexpr (KIND == GRID_MOBIUS) {
        const int lane = threadIdx.x & 63, sl = lane % Ls, lbase = lane - sl;
        lp = lbase + (sl == Ls - 1 ? 0 : sl + 1);
        lm = lbase + (sl == 0 ? Ls - 1 : sl - 1);
        mb5 = static_cast<C>(b5);
        mc5 = static_cast<C>(c5);
        wp = sl == Ls - 1 ? static_cast<C>(-mf) : C(1);
        wm = sl == 0 ? static_cast<C>(-mf) : C(1);
    }

    Cx<C> chi_b[2][3], hb[2][3], p[4][3], u[3][3];
    {
        // backward t-hop of slice t0: U_t(x, t0 - 1)^dagger h(psi(x, t0 - 1))
        const int tm = (t0 == 0) ? Lt - 1 : t0 - 1;
        if constexpr (MOBF)
            gather_b5<SP>(psi, psi_scale, tm * nq + qq, lds, p, lp, lm, mb5, mc5 * wp, mc5 * wm);
        else
            gather<SP>(psi, psi_scale, tm * nq + qq, lds, p);
        project<3, -EF>(p, hb);
        LK::load(U, (static_cast<size_t>(tm) * V3 + col) * 4 + 3, u);
        su3_adj_mul(u, hb, chi_b);
        if constexpr (MOBF)
            gather_b5<SP>(psi, psi_scale, t0 * nq + qq, lds, p, lp, lm, mb5, mc5 * wp, mc5 * wm);
        else
            gather<SP>(psi, psi_scale, t0 * nq + qq, lds, p);
        project<3, -EF>(p, hb);
    }
    // Records gathered per step, in order: psi(x, t+1), the six spatial neighbours at t, and the
    // centre y(x, t) for the Wilson / domain-wall epilogue (y = psi but for the Moebius operator's
    // hopping pass). The next record's loads are issued before the current direction computes.
    constexpr int NREC = (KIND == GRID_HOP) ? 7 : 8;
    [[maybe_unused]] double n2 = 0.0;   // fused epilogue: this thread's |out|^2
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
        if constexpr (NREC == 8) rec[7] = off + qq;
        Fetch<SP> f;
        fetch<SP>(psi, psi_scale, rec[0], f);
        Cx<C> acc[4][3];
#pragma unroll
        for (int j = 0; j < 12; ++j) acc[j / 3][j % 3] = {C(0), C(0)};
        reconstruct_add<3, -EF>(acc, chi_b);
#pragma unroll
        for (int i = 0; i < NREC; ++i) {
            if (MOBF && i < 7)
                stage_b5<SP>(f, lds, p, lp, lm, mb5, mc5 * wp, mc5 * wm);
            else
                stage<SP>(f, lds, p);
            // link of this direction first, then the next record: loads complete in issue order
            const int mu = (i == 0) ? 3 : (i - 1) / 2;
            const bool bwd = (i >= 1 && i <= 6 && ((i - 1) & 1));
            if (i <= 6) LK::load(U, (loff + (bwd ? nb[i - 1] : col)) * 4 + mu, u);
            if (i + 1 < NREC) {
                if (i + 1 == 7)   // only when NREC == 8
                    fetch<SP>(yv, y_scale, rec[NREC - 1], f);
                else
                    fetch<SP>(psi, psi_scale, rec[i + 1], f);
            }
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
        if constexpr (MOBA) {
            // M^dagger psi = b5 w + psi + S^dagger v with v = c5 w - psi, w = acc and psi = p (the
            // centre record); (S^dagger v)_s = P_+ v~_{s+1} + P_- v~_{s-1}
            Cx<C> v[4][3], h[2][3];
#pragma unroll
            for (int j = 0; j < 12; ++j) {
                const Cx<C> a = acc[j / 3][j % 3], c = p[j / 3][j % 3];
                v[j / 3][j % 3] = {mc5 * a.r - c.r, mc5 * a.i - c.i};
                acc[j / 3][j % 3] = {mb5 * a.r + c.r, mb5 * a.i + c.i};
            }
            column_half<SP>(lds, v, 0, lp, h);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                Cx<C> &o = acc[j / 3][j % 3];
                o = {o.r + wp * h[j / 3][j % 3].r, o.i + wp * h[j / 3][j % 3].i};
            }
            column_half<SP>(lds, v, 1, lm, h);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                Cx<C> &o = acc[2 + j / 3][j % 3];
                o = {o.r + wm * h[j / 3][j % 3].r, o.i + wm * h[j / 3][j % 3].i};
            }
        }
        if (KIND == GRID_DWF || MOBF) {
            // M:   - P_- y~_{s+1} - P_+ y~_{s-1};  M^dagger: - P_+ y~_{s+1} - P_- y~_{s-1}, times cs
            // walls: y~_{Ls} = -mf y_0, y~_{-1} = -mf y_{Ls-1}
            const int sp = (s == Ls - 1) ? 0 : s + 1;
            const int sm1 = (s == 0) ? Ls - 1 : s - 1;
            const C c5 = static_cast<C>(cs);
            const C fp = (s == Ls - 1) ? c5 * static_cast<C>(-mf) : c5;
            const C fm = (s == 0) ? c5 * static_cast<C>(-mf) : c5;
            const int hup = DAG ? 0 : 1;   // chiral half taken from s + 1 (0: spins 0,1; 1: spins 2,3)
            const int hdn = 1 - hup;
            const size_t site4 = static_cast<size_t>(off) + static_cast<size_t>(col) * Ls;
            Cx<C> qh[2][3];
            SP::load_half(yv, y_scale, site4 + sp, hup, qh);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                Cx<C> &o = acc[2 * hup + j / 3][j % 3];
                o = {o.r - fp * qh[j / 3][j % 3].r, o.i - fp * qh[j / 3][j % 3].i};
            }
            SP::load_half(yv, y_scale, site4 + sm1, hdn, qh);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                Cx<C> &o = acc[2 * hdn + j / 3][j % 3];
                o = {o.r - fm * qh[j / 3][j % 3].r, o.i - fm * qh[j / 3][j % 3].i};
            }
        }
        if constexpr (FUSE == kFuseAxpy) {
            // r - alpha op psi; r may alias out: the wavefront gathers its own records before storing
            Cx<C> rv[4][3];
            gather<SP>(fz.r, fz.r_scale, off + qq, lds, rv);
            const C al = static_cast<C>(fz.scal[fz.num] / fz.scal[fz.den]);
#pragma unroll
            for (int j = 0; j < 12; ++j) {
                const Cx<C> a = acc[j / 3][j % 3], b = rv[j / 3][j % 3];
                acc[j / 3][j % 3] = {b.r - al * a.r, b.i - al * a.i};
            }
        }
        if constexpr (FUSE == kFuseNone) {
            if (live) SP::store(out, out_scale, static_cast<size_t>(off) + q, acc);
        } else {
            if (live) n2 += SP::store_n2(out, out_scale, static_cast<size_t>(off) + q, acc);
        }
    }
    if constexpr (FUSE != kFuseNone) {
        n2 = wave_sum64(n2);
        __shared__ double fred[4];
        if ((threadIdx.x & 63) == 0) fred[threadIdx.x >> 6] = n2;
        __syncthreads();
        if (threadIdx.x == 0) fz.part[blockIdx.x] = (fred[0] + fred[1]) + (fred[2] + fred[3]);
    }
}

// Same-step column walk (5D full-lattice fields, y = psi): step k finishes out(t) with its forward
// t-hop and builds most of out(t+1) from the records of slice t+1 that the same step brings in
// (the thread's own record, then the six spatial neighbours), so every use of a record of slice
// t+1 -- forward neighbour and centre in its own column, spatial neighbour in the adjacent columns,
// some of which belong to other blocks of the XCD -- falls within one step of the walk. In the
// column walk above the neighbouring columns read a record one step after its own column loaded
// it, and with a 5D time slice several times the size of an XCD's L2 the other resident blocks'
// traffic has often evicted it by then. The partial sum of out(t+1) is carried in registers in
// units of beta (its diagonal and fifth-dimension parts divided by beta) and one scale finishes it.
template <class SP, class LK, bool DAG, int KIND, int FUSE>
__global__ void __launch_bounds__(256)
k_dhop_walk2(const void *__restrict__ U, const void *__restrict__ psi, const float *__restrict__ psi_scale,
             void *out, float *out_scale, GeomDev g, int T, double diag, double mf, FuseDev fz) {
    using C = typename SP::C;
    static_assert(KIND == GRID_HOP || KIND == GRID_WILSON || KIND == GRID_DWF, "plain operators only");
    __shared__ chunk_t sm[kWaves][64 * stage_pitch<SP>()];
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
    // out = beta (H psi + (diag psi - S psi) / beta), beta = 1 for H and -1/2 for D and M
    const C bt = KIND == GRID_HOP ? C(1) : C(-0.5);
    const C dgb = static_cast<C>(diag) / bt;
    // fifth-dimension hop of M (M^dagger: P_+ and P_- exchanged), walls -mf, divided by beta
    const C fpb = ((s == Ls - 1) ? static_cast<C>(-mf) : C(1)) / bt;
    const C fmb = ((s == 0) ? static_cast<C>(-mf) : C(1)) / bt;
    const int sp = (s == Ls - 1) ? 0 : s + 1, sm1 = (s == 0) ? Ls - 1 : s - 1;

    Cx<C> A[4][3], hb[2][3], p[4][3], u[3][3];
    // the diagonal and fifth-dimension parts of out(tt) from the centre record p = psi(x, tt)
    auto diag_part = [&](int tt) {
        if constexpr (KIND != GRID_HOP) {
#pragma unroll
            for (int j = 0; j < 12; ++j) {
                Cx<C> &o = A[j / 3][j % 3];
                o = {o.r + dgb * p[j / 3][j % 3].r, o.i + dgb * p[j / 3][j % 3].i};
            }
        }
        if constexpr (KIND == GRID_DWF) {
            const int hup = DAG ? 0 : 1;   // chiral half taken from s + 1 (0: spins 0,1; 1: spins 2,3)
            const size_t site4 = static_cast<size_t>(tt) * nq + static_cast<size_t>(col) * Ls;
            Cx<C> qh[2][3];
            SP::load_half(psi, psi_scale, site4 + sp, hup, qh);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                Cx<C> &o = A[2 * hup + j / 3][j % 3];
                o = {o.r - fpb * qh[j / 3][j % 3].r, o.i - fpb * qh[j / 3][j % 3].i};
            }
            SP::load_half(psi, psi_scale, site4 + sm1, 1 - hup, qh);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                Cx<C> &o = A[2 * (1 - hup) + j / 3][j % 3];
                o = {o.r - fmb * qh[j / 3][j % 3].r, o.i - fmb * qh[j / 3][j % 3].i};
            }
        }
    };
    // the six spatial hops of slice tt into A (records fetched one ahead of the one in use)
    auto spatial = [&](int tt) {
        const int off = tt * nq;
        const size_t loff = static_cast<size_t>(tt) * V3;
        Fetch<SP> f;
        fetch<SP>(psi, psi_scale, off + nb[0] * Ls + s, f);
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            stage<SP>(f, lds, p);
            const int mu = d / 2;
            const bool bwd = d & 1;
            LK::load(U, (loff + (bwd ? nb[d] : col)) * 4 + mu, u);
            if (d + 1 < 6) fetch<SP>(psi, psi_scale, off + nb[d + 1] * Ls + s, f);
            if (d == 0) hop_term<0, EF, false>(A, p, u);
            else if (d == 1) hop_term<0, -EF, true>(A, p, u);
            else if (d == 2) hop_term<1, EF, false>(A, p, u);
            else if (d == 3) hop_term<1, -EF, true>(A, p, u);
            else if (d == 4) hop_term<2, EF, false>(A, p, u);
            else hop_term<2, -EF, true>(A, p, u);
        }
    };

    {
        // out(t0) without its forward t-hop: backward t-hop from psi(x, t0 - 1), centre, spatial
        const int tm = (t0 == 0) ? Lt - 1 : t0 - 1;
        gather<SP>(psi, psi_scale, tm * nq + qq, lds, p);
        project<3, -EF>(p, hb);
        LK::load(U, (static_cast<size_t>(tm) * V3 + col) * 4 + 3, u);
        Cx<C> chi[2][3];
        su3_adj_mul(u, hb, chi);
#pragma unroll
        for (int j = 0; j < 12; ++j) A[j / 3][j % 3] = {C(0), C(0)};
        reconstruct_add<3, -EF>(A, chi);
        gather<SP>(psi, psi_scale, t0 * nq + qq, lds, p);
        project<3, -EF>(p, hb);
        diag_part(t0);
        spatial(t0);
    }
    [[maybe_unused]] double n2 = 0.0;   // fused epilogue: this thread's |out|^2
#pragma unroll 1
    for (int k = 0; k < T; ++k) {
        const int t = t0 + k;
        const int tn = (t == Lt - 1) ? 0 : t + 1;
        // psi(x, t + 1): the forward t-hop that finishes out(t)
        gather<SP>(psi, psi_scale, tn * nq + qq, lds, p);
        LK::load(U, (static_cast<size_t>(t) * V3 + col) * 4 + 3, u);
        hop_term<3, EF, false>(A, p, u);
#pragma unroll
        for (int j = 0; j < 12; ++j) A[j / 3][j % 3] = {bt * A[j / 3][j % 3].r, bt * A[j / 3][j % 3].i};
        const int off = t * nq;
        if constexpr (FUSE == kFuseAxpy) {
            // r - alpha op psi; r may alias out: the wavefront gathers its own records before storing
            Cx<C> rv[4][3];
            gather<SP>(fz.r, fz.r_scale, off + qq, lds, rv);
            const C al = static_cast<C>(fz.scal[fz.num] / fz.scal[fz.den]);
#pragma unroll
            for (int j = 0; j < 12; ++j) {
                const Cx<C> a = A[j / 3][j % 3], b = rv[j / 3][j % 3];
                A[j / 3][j % 3] = {b.r - al * a.r, b.i - al * a.i};
            }
        }
        if constexpr (FUSE == kFuseNone) {
            if (live) SP::store(out, out_scale, static_cast<size_t>(off) + q, A);
        } else {
            if (live) n2 += SP::store_n2(out, out_scale, static_cast<size_t>(off) + q, A);
        }
        if (k + 1 == T) break;
        // out(t + 1): backward t-hop U_t(x, t)^dagger h(psi(x, t)), centre, spatial hops
        Cx<C> chi[2][3];
        su3_adj_mul(u, hb, chi);
#pragma unroll
        for (int j = 0; j < 12; ++j) A[j / 3][j % 3] = {C(0), C(0)};
        reconstruct_add<3, -EF>(A, chi);
        project<3, -EF>(p, hb);
        diag_part(tn);
        spatial(tn);
    }
    if constexpr (FUSE != kFuseNone) {
        n2 = wave_sum64(n2);
        __shared__ double fred[4];
        if ((threadIdx.x & 63) == 0) fred[threadIdx.x >> 6] = n2;
        __syncthreads();
        if (threadIdx.x == 0) fz.part[blockIdx.x] = (fred[0] + fred[1]) + (fred[2] + fred[3]);
    }
}

// Column walk on checkerboard fields (the even-odd form): out (parity cb) = Diag(y) + beta H psi,
// psi of parity 1 - cb, y and out of parity cb. A checkerboard field holds one site per x-pair, at
// (full 4D index) / 2. A thread owns (xh, y, z, s) and walks T slices; its physical x shifts with
// t (x = 2 xh + ((cb + y + z + t) & 1)), so the backward t-hop cannot be carried from the previous
// step and both t-neighbours are gathered: 8 neighbour records (+ y) and 8 links per step.
//
// Moebius Schur operator (kinds kMobHop, kMobDiag; Ls dividing 64, so a wavefront holds whole
// fifth-dimension columns): without dag the gathered records become B psi = b5 psi + c5 S psi
// (stage_b5) and out = beta H B psi (kMobHop) or diag y - cs S y + beta H B psi (kMobDiag); with
// dag, h = beta H^dagger psi and out = B^dagger h = b5 h + S^dagger (c5 h) (kMobHop) or
// diag y + b5 h + S^dagger (c5 h - cs y) (kMobDiag), S^dagger taken across the column's lanes.
template <class SP, class LK, bool DAG, int KIND, int FUSE>
__global__ void __launch_bounds__(256)
k_dhop_walk_cb(const void *__restrict__ U, const void *__restrict__ psi, const float *__restrict__ psi_scale,
               const void *__restrict__ yv, const float *__restrict__ y_scale, void *out, float *out_scale, GeomDev g,
               int T, int cbp, double diag, double mf, double beta, double cs, double b5, double c5, FuseDev fz) {
    using C = typename SP::C;
    constexpr bool MOB = KIND == kMobHop || KIND == kMobDiag || KIND == kMobHopInv;
    constexpr bool MOBF = MOB && !DAG;
    constexpr bool MOBA = MOB && DAG;
    __shared__ chunk_t sm[kWaves][64 * stage_pitch<SP>()];
    chunk_t *lds = sm[threadIdx.x >> 6];

    const int Ls = g.Ls, Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
    const int Lxh = Lx / 2;
    const int V3h = Lxh * Ly * Lz;          // checkerboard sites per slice
    const int nq = V3h * Ls;                // 5D checkerboard sites per slice
    const int nbc = (nq + 255) / 256;
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int seg = lb / nbc, cbk = lb - seg * nbc;
    const int q = cbk * 256 + threadIdx.x;
    const bool live = q < nq;
    const int qq = live ? q : 0;            // idle lanes still take part in the wave's gathers
    const int colh = qq / Ls, s = qq - (qq / Ls) * Ls;
    const int xh = colh % Lxh, yz = colh / Lxh;
    const int y = yz % Ly, z = yz / Ly;
    const int rowh = yz * Lxh;              // checkerboard index of the row (0, y, z)
    const int yp = (y == Ly - 1) ? 0 : y + 1, ym = (y == 0) ? Ly - 1 : y - 1;
    const int zp = (z == Lz - 1) ? 0 : z + 1, zm = (z == 0) ? Lz - 1 : z - 1;
    const int V3 = Lx * Ly * Lz;
    const int t0 = seg * T;
    constexpr int EF = DAG ? +1 : -1;
    constexpr int NREC = (KIND == GRID_HOP || KIND == kMobHop || KIND == kHopInv || KIND == kMobHopInv) ? 8 : 9;
    [[maybe_unused]] double n2 = 0.0;   // fused epilogue: this thread's |out|^2
    // Moebius: the column's lanes of s + 1 and s - 1 and the wall factors
    int lp = 0, lm = 0;
    C mb5 = C(0), mc5 = C(0), wp = C(1), wm = C(1);
    if constexpr (MOB) {
        const int lane = threadIdx.x & 63, sl = lane % Ls, lbase = lane - sl;
        lp = lbase + (sl == Ls - 1 ? 0 : sl + 1);
        lm = lbase + (sl == 0 ? Ls - 1 : sl - 1);
        mb5 = static_cast<C>(b5);
        mc5 = static_cast<C>(c5);
        wp = sl == Ls - 1 ? static_cast<C>(-mf) : C(1);
        wm = sl == 0 ? static_cast<C>(-mf) : C(1);
    }

    Cx<C> p[4][3], u[3][3];
#pragma unroll 1
    for (int k = 0; k < T; ++k) {
        const int t = t0 + k;
        const int tn = (t == Lt - 1) ? 0 : t + 1, tm = (t == 0) ? Lt - 1 : t - 1;
        const int x = 2 * xh + ((cbp + y + z + t) & 1);
        const int xp = (x == Lx - 1) ? 0 : x + 1, xm = (x == 0) ? Lx - 1 : x - 1;
        const int offh = t * V3h;
        const int oq = (offh + colh) * Ls + s;   // output (and y) record
        // records: +t, -t, +x, -x, +y, -y, +z, -z (the input field), then y
        int rec[NREC];
        rec[0] = (tn * V3h + colh) * Ls + s;
        rec[1] = (tm * V3h + colh) * Ls + s;
        rec[2] = (offh + rowh + (xp >> 1)) * Ls + s;
        rec[3] = (offh + rowh + (xm >> 1)) * Ls + s;
        rec[4] = (offh + (z * Ly + yp) * Lxh + xh) * Ls + s;
        rec[5] = (offh + (z * Ly + ym) * Lxh + xh) * Ls + s;
        rec[6] = (offh + (zp * Ly + y) * Lxh + xh) * Ls + s;
        rec[7] = (offh + (zm * Ly + y) * Lxh + xh) * Ls + s;
        if constexpr (NREC == 9) rec[8] = oq;
        // links, full-lattice index: U_mu(x) forward, U_mu(x - mu) backward
        const size_t f4 = (static_cast<size_t>(t) * Lz + z) * Ly * Lx + static_cast<size_t>(y) * Lx + x;
        const size_t row4 = f4 - x;
        size_t lk[8];
        lk[0] = f4 * 4 + 3;
        lk[1] = ((static_cast<size_t>(tm) * Lz + z) * Ly * Lx + static_cast<size_t>(y) * Lx + x) * 4 + 3;
        lk[2] = f4 * 4 + 0;
        lk[3] = (row4 + xm) * 4 + 0;
        lk[4] = f4 * 4 + 1;
        lk[5] = (f4 - static_cast<size_t>(y) * Lx + static_cast<size_t>(ym) * Lx) * 4 + 1;
        lk[6] = f4 * 4 + 2;
        lk[7] = (f4 - static_cast<size_t>(z) * Ly * Lx + static_cast<size_t>(zm) * Ly * Lx) * 4 + 2;
        Fetch<SP> f;
        fetch<SP>(psi, psi_scale, rec[0], f);
        Cx<C> acc[4][3];
#pragma unroll
        for (int j = 0; j < 12; ++j) acc[j / 3][j % 3] = {C(0), C(0)};
#pragma unroll
        for (int i = 0; i < NREC; ++i) {
            if (MOBF && i < 8)
                stage_b5<SP>(f, lds, p, lp, lm, mb5, mc5 * wp, mc5 * wm);
            else
                stage<SP>(f, lds, p);
            // link of this direction first, then the next record: loads complete in issue order
            if (i < 8) LK::load(U, lk[i], u);
            if (i + 1 < 8)
                fetch<SP>(psi, psi_scale, rec[i + 1], f);
            else if (i + 1 < NREC)
                fetch<SP>(yv, y_scale, rec[i + 1], f);
            if (i == 0) hop_term<3, EF, false>(acc, p, u);
            else if (i == 1) hop_term<3, -EF, true>(acc, p, u);
            else if (i == 2) hop_term<0, EF, false>(acc, p, u);
            else if (i == 3) hop_term<0, -EF, true>(acc, p, u);
            else if (i == 4) hop_term<1, EF, false>(acc, p, u);
            else if (i == 5) hop_term<1, -EF, true>(acc, p, u);
            else if (i == 6) hop_term<2, EF, false>(acc, p, u);
            else if (i == 7) hop_term<2, -EF, true>(acc, p, u);
            else if (!MOB) {
                // the diagonal part of `kind` on y, H scaled by beta
                const C dg = static_cast<C>(diag), bt = static_cast<C>(beta);
#pragma unroll
                for (int j = 0; j < 12; ++j) {
                    const Cx<C> a = acc[j / 3][j % 3], v = p[j / 3][j % 3];
                    acc[j / 3][j % 3] = {dg * v.r + bt * a.r, dg * v.i + bt * a.i};
                }
            }
        }
        if (KIND == GRID_HOP || KIND == kMobHop || KIND == kHopInv || KIND == kMobHopInv || MOBA) {
            const C bt = static_cast<C>(beta);
#pragma unroll
            for (int j = 0; j < 12; ++j) acc[j / 3][j % 3] = {bt * acc[j / 3][j % 3].r, bt * acc[j / 3][j % 3].i};
        }
        if constexpr (KIND == kHopInv) {
            const int lane = threadIdx.x & 63, sl = lane % Ls;
            column_m5inv<SP>(lds, acc, sl, lane - sl, Ls, static_cast<C>(1.0 / diag), static_cast<C>(mf), DAG);
        }
        if (MOBF && KIND == kMobDiag) {
            // diag y + beta H B psi (y = p, the last record staged)
            const C dg = static_cast<C>(diag), bt = static_cast<C>(beta);
#pragma unroll
            for (int j = 0; j < 12; ++j) {
                const Cx<C> a = acc[j / 3][j % 3], v = p[j / 3][j % 3];
                acc[j / 3][j % 3] = {dg * v.r + bt * a.r, dg * v.i + bt * a.i};
            }
        }
        if constexpr (MOBA) {
            // out = diag y + b5 h + S^dagger v, v = c5 h - cs y (y = 0 for kMobHop), h = acc;
            // (S^dagger v)_s = P_+ v~_{s+1} + P_- v~_{s-1}
            const C dg = static_cast<C>(diag), csc = static_cast<C>(cs);
            Cx<C> v[4][3], hh[2][3];
#pragma unroll
            for (int j = 0; j < 12; ++j) {
                const Cx<C> h = acc[j / 3][j % 3];
                Cx<C> yy = {C(0), C(0)};
                if (KIND == kMobDiag) yy = p[j / 3][j % 3];
                v[j / 3][j % 3] = {mc5 * h.r - csc * yy.r, mc5 * h.i - csc * yy.i};
                acc[j / 3][j % 3] = {mb5 * h.r + dg * yy.r, mb5 * h.i + dg * yy.i};
            }
            column_half<SP>(lds, v, 0, lp, hh);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                Cx<C> &o = acc[j / 3][j % 3];
                o = {o.r + wp * hh[j / 3][j % 3].r, o.i + wp * hh[j / 3][j % 3].i};
            }
            column_half<SP>(lds, v, 1, lm, hh);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                Cx<C> &o = acc[2 + j / 3][j % 3];
                o = {o.r + wm * hh[j / 3][j % 3].r, o.i + wm * hh[j / 3][j % 3].i};
            }
        }
        if constexpr (KIND == kMobHopInv) {
            const int lane = threadIdx.x & 63, sl = lane % Ls;
            column_m5inv<SP>(lds, acc, sl, lane - sl, Ls, static_cast<C>(1.0 / diag), static_cast<C>(mf), DAG);
        }
        if (KIND == GRID_DWF || (MOBF && KIND == kMobDiag)) {
            // - cs (P_- y~_{s+1} + P_+ y~_{s-1}) (M; P_+ and P_- exchanged for M^dagger), walls -mf
            const int sp = (s == Ls - 1) ? 0 : s + 1;
            const int sm1 = (s == 0) ? Ls - 1 : s - 1;
            const C csc = static_cast<C>(cs);
            const C fp = csc * ((s == Ls - 1) ? static_cast<C>(-mf) : C(1));
            const C fm = csc * ((s == 0) ? static_cast<C>(-mf) : C(1));
            const int hup = DAG ? 0 : 1;   // chiral half taken from s + 1 (0: spins 0,1; 1: spins 2,3)
            const int hdn = 1 - hup;
            const size_t site4 = static_cast<size_t>(offh + colh) * Ls;
            Cx<C> qh[2][3];
            SP::load_half(yv, y_scale, site4 + sp, hup, qh);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                Cx<C> &o = acc[2 * hup + j / 3][j % 3];
                o = {o.r - fp * qh[j / 3][j % 3].r, o.i - fp * qh[j / 3][j % 3].i};
            }
            SP::load_half(yv, y_scale, site4 + sm1, hdn, qh);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                Cx<C> &o = acc[2 * hdn + j / 3][j % 3];
                o = {o.r - fm * qh[j / 3][j % 3].r, o.i - fm * qh[j / 3][j % 3].i};
            }
        }
        if constexpr (FUSE == kFuseAxpy) {
            // r - alpha op psi; r may alias out: the wavefront gathers its own records before storing
            Cx<C> rv[4][3];
            gather<SP>(fz.r, fz.r_scale, oq, lds, rv);
            const C al = static_cast<C>(fz.scal[fz.num] / fz.scal[fz.den]);
#pragma unroll
            for (int j = 0; j < 12; ++j) {
                const Cx<C> a = acc[j / 3][j % 3], b = rv[j / 3][j % 3];
                acc[j / 3][j % 3] = {b.r - al * a.r, b.i - al * a.i};
            }
        }
        if constexpr (FUSE == kFuseNone) {
            if (live) SP::store(out, out_scale, static_cast<size_t>(oq), acc);
        } else {
            if (live) n2 += SP::store_n2(out, out_scale, static_cast<size_t>(oq), acc);
        }
    }
    if constexpr (FUSE != kFuseNone) {
        n2 = wave_sum64(n2);
        __shared__ double fred[4];
        if ((threadIdx.x & 63) == 0) fred[threadIdx.x >> 6] = n2;
        __syncthreads();
        if (threadIdx.x == 0) fz.part[blockIdx.x] = (fred[0] + fred[1]) + (fred[2] + fred[3]);
    }
}

// Steps per thread: the longest walk (a divisor of Lt) that still leaves enough blocks to fill
// the chip; small lattices use T = 1.
static int choose_steps(const GeomDev &g) {
    // Measured: the longest walk that still gives >= 4096 blocks, but at least two slices (a walk
    // of one slice cannot carry the backward t-hop and reads twice the records).
    constexpr long kMinBlocks = 4096;
    const long nbc = (static_cast<long>(g.L[0]) * g.L[1] * g.L[2] * g.Ls + 255) / 256;
    int best = 1;
    for (int T = 1; T <= g.L[3]; ++T)
        if (g.L[3] % T == 0 && nbc * (g.L[3] / T) >= kMinBlocks) best = T;
    if (best < 2)
        for (int T = 2; T <= g.L[3]; ++T)
            if (g.L[3] % T == 0) {
                if (nbc * (g.L[3] / T) >= 1024) best = T;
                break;
            }
    return best;
}

// The fused Moebius operator runs on the full-lattice column walk (FP32 and FP16-storage 5D fields)
// when whole fifth-dimension columns fit a wavefront.
bool walk_mobius_applies(const DhopArgs &a) {
    return a.kind == GRID_MOBIUS && !a.custom && a.g.Ls >= 2 && 64 % a.g.Ls == 0 &&
           (a.prec == GRID_F32 || a.prec == GRID_F16S);
}

// The same-step walk takes the plain operators on 5D fields (y = psi).
static bool use_walk2(const DhopArgs &a) {
    return !a.custom && a.g.Ls > 1 && (a.kind == GRID_HOP || a.kind == GRID_WILSON || a.kind == GRID_DWF);
}

template <class SP, class LK>
static hipError_t launch_walk2(const DhopArgs &a) {
    const int T = choose_steps(a.g);
    const long nbc = (static_cast<long>(a.g.L[0]) * a.g.L[1] * a.g.L[2] * a.g.Ls + 255) / 256;
    const dim3 grid(static_cast<unsigned>(nbc * (a.g.L[3] / T))), block(256);
    hipStream_t st = a.stream;
#define GRIDMI_LAUNCH(DAG, KIND, FUSE)                                                                       \
    hipLaunchKernelGGL((k_dhop_walk2<SP, LK, DAG, KIND, FUSE>), grid, block, 0, st, a.U, a.psi, a.psi_scale, a.out, \
                       a.out_scale, a.g, T, a.diag, a.mf, a.fz)
    if (a.fuse != kFuseNone) {
        switch (a.kind * 4 + a.fuse * 2 + (a.dag ? 1 : 0)) {
            case GRID_WILSON * 4 + kFuseNorm * 2 + 0: GRIDMI_LAUNCH(false, GRID_WILSON, kFuseNorm); break;
            case GRID_DWF * 4 + kFuseNorm * 2 + 0: GRIDMI_LAUNCH(false, GRID_DWF, kFuseNorm); break;
            case GRID_WILSON * 4 + kFuseAxpy * 2 + 1: GRIDMI_LAUNCH(true, GRID_WILSON, kFuseAxpy); break;
            case GRID_DWF * 4 + kFuseAxpy * 2 + 1: GRIDMI_LAUNCH(true, GRID_DWF, kFuseAxpy); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (a.kind * 2 + (a.dag ? 1 : 0)) {
        case GRID_HOP * 2 + 0: GRIDMI_LAUNCH(false, GRID_HOP, kFuseNone); break;
        case GRID_HOP * 2 + 1: GRIDMI_LAUNCH(true, GRID_HOP, kFuseNone); break;
        case GRID_WILSON * 2 + 0: GRIDMI_LAUNCH(false, GRID_WILSON, kFuseNone); break;
        case GRID_WILSON * 2 + 1: GRIDMI_LAUNCH(true, GRID_WILSON, kFuseNone); break;
        case GRID_DWF * 2 + 0: GRIDMI_LAUNCH(false, GRID_DWF, kFuseNone); break;
        case GRID_DWF * 2 + 1: GRIDMI_LAUNCH(true, GRID_DWF, kFuseNone); break;
        default: return hipErrorInvalidValue;
    }
#undef GRIDMI_LAUNCH
    return hipGetLastError();
}

template <class SP, class LK>
static hipError_t launch_walk(const DhopArgs &a) {
    if (use_walk2(a)) return launch_walk2<SP, LK>(a);
    const int T = choose_steps(a.g);
    const long nbc = (static_cast<long>(a.g.L[0]) * a.g.L[1] * a.g.L[2] * a.g.Ls + 255) / 256;
    const dim3 grid(static_cast<unsigned>(nbc * (a.g.L[3] / T))), block(256);
    hipStream_t st = a.stream;
    const void *y = a.custom ? a.y : a.psi;
    const float *ys = a.custom ? a.y_scale : a.psi_scale;
    const double cs = (a.custom || a.kind == GRID_MOBIUS) ? a.cs : 1.0;
#define GRIDMI_LAUNCH(DAG, KIND, FUSE)                                                                    \
    hipLaunchKernelGGL((k_dhop_walk<SP, LK, DAG, KIND, FUSE>), grid, block, 0, st, a.U, a.psi, a.psi_scale, y, ys,  \
                       a.out, a.out_scale, a.g, T, a.diag, a.mf, cs, a.b5, a.c5, a.fz)
    if (a.kind == GRID_MOBIUS && !walk_mobius_applies(a)) return hipErrorInvalidValue;
    if (a.fuse != kFuseNone) {
        switch (a.kind * 4 + a.fuse * 2 + (a.dag ? 1 : 0)) {
            case GRID_WILSON * 4 + kFuseNorm * 2 + 0: GRIDMI_LAUNCH(false, GRID_WILSON, kFuseNorm); break;
            case GRID_DWF * 4 + kFuseNorm * 2 + 0: GRIDMI_LAUNCH(false, GRID_DWF, kFuseNorm); break;
            case GRID_MOBIUS * 4 + kFuseNorm * 2 + 0: GRIDMI_LAUNCH(false, GRID_MOBIUS, kFuseNorm); break;
            case GRID_WILSON * 4 + kFuseAxpy * 2 + 1: GRIDMI_LAUNCH(true, GRID_WILSON, kFuseAxpy); break;
            case GRID_DWF * 4 + kFuseAxpy * 2 + 1: GRIDMI_LAUNCH(true, GRID_DWF, kFuseAxpy); break;
            case GRID_MOBIUS * 4 + kFuseAxpy * 2 + 1: GRIDMI_LAUNCH(true, GRID_MOBIUS, kFuseAxpy); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (a.kind * 2 + (a.dag ? 1 : 0)) {
        case GRID_HOP * 2 + 0: GRIDMI_LAUNCH(false, GRID_HOP, kFuseNone); break;
        case GRID_HOP * 2 + 1: GRIDMI_LAUNCH(true, GRID_HOP, kFuseNone); break;
        case GRID_WILSON * 2 + 0: GRIDMI_LAUNCH(false, GRID_WILSON, kFuseNone); break;
        case GRID_WILSON * 2 + 1: GRIDMI_LAUNCH(true, GRID_WILSON, kFuseNone); break;
        case GRID_DWF * 2 + 0: GRIDMI_LAUNCH(false, GRID_DWF, kFuseNone); break;
        case GRID_DWF * 2 + 1: GRIDMI_LAUNCH(true, GRID_DWF, kFuseNone); break;
        case GRID_MOBIUS * 2 + 0: GRIDMI_LAUNCH(false, GRID_MOBIUS, kFuseNone); break;
        case GRID_MOBIUS * 2 + 1: GRIDMI_LAUNCH(true, GRID_MOBIUS, kFuseNone); break;
        default: return hipErrorInvalidValue;
    }
#undef GRIDMI_LAUNCH
    return hipGetLastError();
}

// Checkerboard walk: blocks of 256 column sites, walks of the longest divisor of Lt that keeps at
// least 2048 blocks (no carried term, so a longer walk only amortises the index set-up).
static long walk_cb_nbc(const GeomDev &g) {
    return (static_cast<long>(g.L[0] / 2) * g.L[1] * g.L[2] * g.Ls + 255) / 256;
}
static int choose_steps_cb(const GeomDev &g) {
    const long nbc = walk_cb_nbc(g);
    int best = 1;
    for (int T = 1; T <= g.L[3]; ++T)
        if (g.L[3] % T == 0 && nbc * (g.L[3] / T) >= 2048) best = T;
    return best;
}

template <class SP, class LK>
static hipError_t launch_walk_cb(const DhopArgs &a) {
    const int T = choose_steps_cb(a.g);
    const dim3 grid(static_cast<unsigned>(walk_cb_nbc(a.g) * (a.g.L[3] / T))), block(256);
    hipStream_t st = a.stream;
#define GRIDMI_LAUNCH(DAG, KIND, FUSE)                                                                    \
    hipLaunchKernelGGL((k_dhop_walk_cb<SP, LK, DAG, KIND, FUSE>), grid, block, 0, st, a.U, a.psi, a.psi_scale, \
                       a.y, a.y_scale, a.out, a.out_scale, a.g, T, a.cb, a.diag, a.mf, a.beta, a.cs, a.b5, a.c5, a.fz)
    const bool mob = a.kind == kMobHop || a.kind == kMobDiag || a.kind == kHopInv || a.kind == kMobHopInv;
    if (mob && !(a.g.Ls >= 2 && 64 % a.g.Ls == 0)) return hipErrorInvalidValue;
    if (a.fuse != kFuseNone) {
        switch (a.kind * 4 + a.fuse * 2 + (a.dag ? 1 : 0)) {
            case GRID_WILSON * 4 + kFuseNorm * 2 + 0: GRIDMI_LAUNCH(false, GRID_WILSON, kFuseNorm); break;
            case GRID_DWF * 4 + kFuseNorm * 2 + 0: GRIDMI_LAUNCH(false, GRID_DWF, kFuseNorm); break;
            case kMobDiag * 4 + kFuseNorm * 2 + 0: GRIDMI_LAUNCH(false, kMobDiag, kFuseNorm); break;
            case GRID_WILSON * 4 + kFuseAxpy * 2 + 1: GRIDMI_LAUNCH(true, GRID_WILSON, kFuseAxpy); break;
            case GRID_DWF * 4 + kFuseAxpy * 2 + 1: GRIDMI_LAUNCH(true, GRID_DWF, kFuseAxpy); break;
            case kMobDiag * 4 + kFuseAxpy * 2 + 1: GRIDMI_LAUNCH(true, kMobDiag, kFuseAxpy); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (a.kind * 2 + (a.dag ? 1 : 0)) {
        case GRID_HOP * 2 + 0: GRIDMI_LAUNCH(false, GRID_HOP, kFuseNone); break;
        case GRID_HOP * 2 + 1: GRIDMI_LAUNCH(true, GRID_HOP, kFuseNone); break;
        case GRID_WILSON * 2 + 0: GRIDMI_LAUNCH(false, GRID_WILSON, kFuseNone); break;
        case GRID_WILSON * 2 + 1: GRIDMI_LAUNCH(true, GRID_WILSON, kFuseNone); break;
        case GRID_DWF * 2 + 0: GRIDMI_LAUNCH(false, GRID_DWF, kFuseNone); break;
        case GRID_DWF * 2 + 1: GRIDMI_LAUNCH(true, GRID_DWF, kFuseNone); break;
        case kMobHop * 2 + 0: GRIDMI_LAUNCH(false, kMobHop, kFuseNone); break;
        case kMobHop * 2 + 1: GRIDMI_LAUNCH(true, kMobHop, kFuseNone); break;
        case kMobDiag * 2 + 0: GRIDMI_LAUNCH(false, kMobDiag, kFuseNone); break;
        case kMobDiag * 2 + 1: GRIDMI_LAUNCH(true, kMobDiag, kFuseNone); break;
        case kHopInv * 2 + 0: GRIDMI_LAUNCH(false, kHopInv, kFuseNone); break;
        case kHopInv * 2 + 1: GRIDMI_LAUNCH(true, kHopInv, kFuseNone); break;
        case kMobHopInv * 2 + 0: GRIDMI_LAUNCH(false, kMobHopInv, kFuseNone); break;
        case kMobHopInv * 2 + 1: GRIDMI_LAUNCH(true, kMobHopInv, kFuseNone); break;
        default: return hipErrorInvalidValue;
    }
#undef GRIDMI_LAUNCH
    return hipGetLastError();
}

// Schedules: column walk for FP16 storage and 5D FP32 fields (full lattice, or checkerboard
// fields in the even-odd form), direction-parallel otherwise (measured faster there). The
// full-lattice walk also takes the custom form with a separate y and beta = -1/2 (the Moebius
// operator's hopping pass).
static bool walk_prec(const DhopArgs &a) { return a.prec == GRID_F16S || (a.prec == GRID_F32 && a.g.Ls > 1); }
static bool use_walk(const DhopArgs &a) {
    return walk_prec(a) && (!a.custom || (a.cb < 0 && a.kind != GRID_HOP && a.beta == -0.5));
}
static bool use_walk_cb(const DhopArgs &a) { return a.custom && a.cb >= 0 && walk_prec(a); }

template <class SP, class LK>
static hipError_t launch_sched(const DhopArgs &a) {
    if (a.kind == GRID_MOBIUS && !walk_mobius_applies(a)) return hipErrorInvalidValue;
    if ((a.kind == kMobHop || a.kind == kMobDiag || a.kind == kHopInv || a.kind == kMobHopInv) && !use_walk_cb(a))
        return hipErrorInvalidValue;
    if (tile_applies(a)) return launch_tile(a);
    if (use_walk(a)) return launch_walk<SP, LK>(a);
    if (use_walk_cb(a)) return launch_walk_cb<SP, LK>(a);
    return launch_dir<SP, LK>(a);
}

long dhop_blocks(const DhopArgs &a) {
    if (tile_applies(a)) return tile_blocks(a);
    if (use_walk(a)) {
        const long nbc = (static_cast<long>(a.g.L[0]) * a.g.L[1] * a.g.L[2] * a.g.Ls + 255) / 256;
        return nbc * (a.g.L[3] / choose_steps(a.g));
    }
    if (use_walk_cb(a)) return walk_cb_nbc(a.g) * (a.g.L[3] / choose_steps_cb(a.g));
    const Trav tr = make_trav(a.g, a.custom ? a.cb : -1);
    return (static_cast<long>(tr.nout) + kSites - 1) / kSites;
}

long dhop_blocks_max(long n5, int Lt) {
    // direction-parallel: ceil(n5 / 32); column walks: at most ceil(n5 / Lt / 256) * Lt
    return (n5 + kSites - 1) / kSites + Lt;
}

hipError_t launch_dhop(const DhopArgs &a) {
    if (a.g.n5 == 0) return hipSuccess;
    switch (a.prec * 2 + a.link_fmt) {
        case GRID_F64 * 2 + GRID_L18: return launch_sched<SpF64, LkF64<3>>(a);
        case GRID_F64 * 2 + GRID_L12: return launch_sched<SpF64, LkF64<2>>(a);
        case GRID_F32 * 2 + GRID_L18: return launch_sched<SpF32, LkF32<3>>(a);
        case GRID_F32 * 2 + GRID_L12: return launch_sched<SpF32, LkF32<2>>(a);
        case GRID_F16S * 2 + GRID_L18: return launch_sched<SpF16S, LkF16<3>>(a);
        case GRID_F16S * 2 + GRID_L12: return launch_sched<SpF16S, LkF16<2>>(a);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gridmi
