// Even-odd (red-black) preconditioning of the Wilson and domain-wall operators.
//
// Grid objects may be single-checkerboard (Section 2.2): a field holding only the sites of one
// parity p = (x + y + z + t) mod 2. Here such a field stores site (x, y, z, t) at the half-volume
// index (x / 2) + (Lx / 2)(y + Ly(z + Lz t)), i.e. the full site index divided by two, with the
// Ls fifth-dimension records of a 4D site contiguous as in full fields; all four extents are even.
//
// The hopping term connects the two parities only, so with o = odd, e = even
//   M = [[M_ee, M_eo], [M_oe, M_oo]],  M_eo = -H_eo / 2,  M_oe = -H_oe / 2,
//   M_ee = M_oo = (4 + m) for Wilson and the fifth-dimension operator M5 for domain wall,
// and M x = b is solved through the Schur complement on the even sites
//   Mhat = M_ee - M_eo M_oo^-1 M_oe = M_ee - H_eo M_oo^-1 H_oe / 4,
//   bhat = b_e - M_eo M_oo^-1 b_o = b_e + H_eo M_oo^-1 b_o / 2,
//   Mhat^dagger Mhat x_e = Mhat^dagger bhat (CG),   x_o = M_oo^-1 (b_o + H_oe x_e / 2).
//
// M5 per 4D site and chirality is (5 - M5) minus a cyclic shift in s with -m_f on the wrap: the
// lower spins take psi_{s+1} (psi_{Ls} = -m_f psi_0), the upper spins psi_{s-1}
// (psi_{-1} = -m_f psi_{Ls-1}); the adjoint swaps the two. Its inverse is applied in closed form:
// for d y_s - y_{s+1} = b_s (s < Ls-1), d y_{Ls-1} + m_f y_0 = b_{Ls-1},
//   y_0 = [sum_k b_k d^-(k+1)] / (1 + m_f d^-Ls),  y_{Ls-1} = (b_{Ls-1} - m_f y_0) / d,
//   y_s = (b_s + y_{s+1}) / d  for s = Ls-2 .. 1,
// and mirrored in s for the other chirality (the recurrences are stable for |d| > 1).
//
// Moebius (M = D_W B + 1 - S, B = b5 + c5 S): the hopping term enters as M_eo = -H_eo B / 2,
// M_oe = -H_oe B / 2, and M_ee = M_oo = (4 - M5) B + 1 - S = alpha - beta S with
// alpha = 1 + (4 - M5) b5, beta = 1 - (4 - M5) c5: per chirality the same cyclic bidiagonal
// system, so M_oo^-1 = (1 / beta) (alpha / beta - S)^-1 (d = alpha / beta), the factor 1 / beta
// folded into the s-local pass that follows (M_oo = alpha when beta = 0). Then
//   Mhat = M_ee - H_eo B M_oo^-1 H_oe B / 4,   Mhat^dagger = M_ee^dagger - B^dagger H_eo^dagger
//   (M_oo^dagger)^-1 B^dagger H_oe^dagger / 4,
//   bhat = b_e + H_eo B M_oo^-1 b_o / 2,   x_o = M_oo^-1 (b_o + H_oe B x_e / 2).
#include <chrono>
#include <string.h>

#include "device.h"
#include "launch.h"

namespace gridmi {

constexpr int kM5invSites = 4;   // 4D sites per block (16 lanes each, one wavefront)
constexpr int kM5invMaxLs = 64;

typedef unsigned int m5chunk_t __attribute__((ext_vector_type(4)));

// LDS of one block: the block's 4 x Ls input records as stored (16-byte chunks), then, for FP16
// storage only, the FP16 site scales and a separate result area (FP64 / FP32 results overwrite
// their own input element: lane k reads b_s[k] before it writes y_s[k]).
template <class SP>
static size_t m5inv_lds_bytes(int Ls) {
    size_t b = static_cast<size_t>(kM5invSites) * Ls * SP::kChunks * 16;
    if (SP::kScaled) b += static_cast<size_t>(kM5invSites) * Ls * (sizeof(float) + 12 * sizeof(Cx<float>));
    return b;
}

template <class SP>
__global__ void __launch_bounds__(64)
k_m5inv(const void *__restrict__ psi, const float *__restrict__ psi_scale, void *__restrict__ out,
        float *__restrict__ out_scale, long n4, int Ls, double diag, double mf, int dag) {
    using C = typename SP::C;
    constexpr int CH = SP::kChunks;
    extern __shared__ m5chunk_t smem[];
    const int lane = threadIdx.x;
    const long h0 = static_cast<long>(blockIdx.x) * kM5invSites;
    const int nsite = static_cast<int>(n4 - h0 < kM5invSites ? n4 - h0 : kM5invSites);
    // Stage the block's nsite * Ls consecutive records: coalesced 16-byte loads, eight in flight
    // per lane, so the s recurrences below read LDS instead of waiting on one load per step.
    m5chunk_t *xin = smem;
    const int nch = nsite * Ls * CH;
    const m5chunk_t *src = reinterpret_cast<const m5chunk_t *>(psi) + static_cast<size_t>(h0) * Ls * CH;
    for (int c0 = 0; c0 < nch; c0 += 8 * 64) {
        m5chunk_t w[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int c = c0 + j * 64 + lane;
            if (c < nch) w[j] = src[c];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int c = c0 + j * 64 + lane;
            if (c < nch) xin[c] = w[j];
        }
    }
    [[maybe_unused]] float *scl = reinterpret_cast<float *>(xin + kM5invSites * Ls * CH);
    if constexpr (SP::kScaled) {
        for (int r = lane; r < nsite * Ls; r += 64) scl[r] = psi_scale[static_cast<size_t>(h0) * Ls + r];
    }
    __syncthreads();

    const int sl = lane >> 4, k16 = lane & 15;
    const bool live = sl < nsite && k16 < 12;
    const int sli = sl < nsite ? sl : 0;   // idle lanes compute on a valid site, store nothing
    const int k = k16 < 12 ? k16 : 0;
    // non-adjoint: lower spins couple to s + 1, upper spins to s - 1; the adjoint swaps them
    const bool plus = ((k / 3) >= 2) != (dag != 0);
    const C d = static_cast<C>(diag), m = static_cast<C>(mf);
    const C dinv = C(1) / d;
    C dl = C(1);
    for (int i = 0; i < Ls; ++i) dl *= dinv;
    const C den = C(1) + m * dl;
    const m5chunk_t *rec0 = xin + static_cast<size_t>(sli) * Ls * CH;
    auto b_at = [&](int s) -> Cx<C> {
        return Elem<SP>::get(rec0 + s * CH, k, SP::kScaled ? scl[sli * Ls + s] : 1.0f);
    };
    // results: in place over the input element (FP64 / FP32), else the separate area
    Cx<C> *yb = SP::kScaled ? reinterpret_cast<Cx<C> *>(scl + kM5invSites * Ls) + static_cast<size_t>(sli) * Ls * 12
                            : reinterpret_cast<Cx<C> *>(xin) + static_cast<size_t>(sli) * Ls * 12;
    const bool wr = live;
    auto put = [&](int s, Cx<C> v) {
        if (wr) yb[s * 12 + k] = v;
    };
    // y_s solves the cyclic bidiagonal system of one chirality: first the corner value from the
    // Horner sum over all s, then back substitution. Every b_s is read before y_s is written.
    if (plus) {
        Cx<C> S = {C(0), C(0)};
        for (int s = Ls - 1; s >= 0; --s) {
            const Cx<C> b = b_at(s);
            S = {(S.r + b.r) * dinv, (S.i + b.i) * dinv};
        }
        const Cx<C> y0 = {S.r / den, S.i / den};
        if (Ls > 1) {
            Cx<C> b = b_at(Ls - 1);
            Cx<C> y = {(b.r - m * y0.r) * dinv, (b.i - m * y0.i) * dinv};
            put(Ls - 1, y);
            for (int s = Ls - 2; s >= 1; --s) {
                b = b_at(s);
                y = {(b.r + y.r) * dinv, (b.i + y.i) * dinv};
                put(s, y);
            }
        }
        put(0, y0);
    } else {
        Cx<C> S = {C(0), C(0)};
        for (int s = 0; s < Ls; ++s) {
            const Cx<C> b = b_at(s);
            S = {(S.r + b.r) * dinv, (S.i + b.i) * dinv};
        }
        const Cx<C> yl = {S.r / den, S.i / den};
        if (Ls > 1) {
            Cx<C> b = b_at(0);
            Cx<C> y = {(b.r - m * yl.r) * dinv, (b.i - m * yl.i) * dinv};
            put(0, y);
            for (int s = 1; s <= Ls - 2; ++s) {
                b = b_at(s);
                y = {(b.r + y.r) * dinv, (b.i + y.i) * dinv};
                put(s, y);
            }
        }
        put(Ls - 1, yl);
    }
    __syncthreads();
    const size_t base = static_cast<size_t>(h0 + sli) * Ls;
    for (int s = 0; s < Ls; ++s) {
        const Cx<C> v = yb[s * 12 + k];
        store_elem<SP>(out, out_scale, base + s, k, v, live);
    }
}

hipError_t launch_m5inv(const void *psi, const float *psi_scale, void *out, float *out_scale, long n4, int Ls,
                        double diag, double mf, int dag, int prec, hipStream_t stream) {
    if (n4 == 0) return hipSuccess;
    if (Ls < 1 || Ls > kM5invMaxLs) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>((n4 + kM5invSites - 1) / kM5invSites)), block(64);
    if (prec == GRID_F64)
        hipLaunchKernelGGL(k_m5inv<SpF64>, grid, block, m5inv_lds_bytes<SpF64>(Ls), stream, psi, psi_scale, out,
                           out_scale, n4, Ls, diag, mf, dag);
    else if (prec == GRID_F32)
        hipLaunchKernelGGL(k_m5inv<SpF32>, grid, block, m5inv_lds_bytes<SpF32>(Ls), stream, psi, psi_scale, out,
                           out_scale, n4, Ls, diag, mf, dag);
    else
        hipLaunchKernelGGL(k_m5inv<SpF16S>, grid, block, m5inv_lds_bytes<SpF16S>(Ls), stream, psi, psi_scale, out,
                           out_scale, n4, Ls, diag, mf, dag);
    return hipGetLastError();
}

// Copy between a full FP64 field and one checkerboard of it (to_cb: full -> checkerboard).
__global__ void __launch_bounds__(256)
k_cb_copy(const double2 *__restrict__ src, double2 *__restrict__ dst, GeomDev g, int parity, int to_cb, long nchunks) {
    const long i = static_cast<long>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= nchunks) return;
    const long rec = i / 12;
    const int c = static_cast<int>(i - rec * 12);
    const long h = rec / g.Ls;
    const int s = static_cast<int>(rec - h * g.Ls);
    const int lxh = g.L[0] / 2;
    long r = h / lxh;
    const int xh = static_cast<int>(h - r * lxh);
    const int y = static_cast<int>(r % g.L[1]);
    r /= g.L[1];
    const int z = static_cast<int>(r % g.L[2]);
    const int t = static_cast<int>(r / g.L[2]);
    const int x = 2 * xh + ((y + z + t + parity) & 1);
    const long full = (x + static_cast<long>(g.L[0]) * (y + static_cast<long>(g.L[1]) * (z + static_cast<long>(g.L[2]) * t))) *
                          g.Ls + s;
    if (to_cb)
        dst[i] = src[full * 12 + c];
    else
        dst[full * 12 + c] = src[i];
}

static hipError_t cb_copy(const void *src, void *dst, const GeomDev &g, int parity, int to_cb, hipStream_t st) {
    const long n = static_cast<long>(g.n5 / 2) * 12;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cb_copy, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st,
                       static_cast<const double2 *>(src), static_cast<double2 *>(dst), g, parity, to_cb, n);
    return hipGetLastError();
}

#define EOCHK(x)                                \
    do {                                        \
        hipError_t e_ = (x);                    \
        if (e_ != hipSuccess) return e_;        \
    } while (0)

// out (checkerboard cb) = diagonal part of `kind` (coefficient dg) on y + beta * H psi.
static hipError_t hop_cb(const void *U, int prec, int fmt, const GeomDev &g, int kind, int dag, double dg, double mf,
                         int cb, const void *psi, const float *psis, const void *y, const float *ys, double beta, void *out,
                         float *outs, hipStream_t st, int fuse = kFuseNone, const FuseDev *fz = nullptr,
                         long *nparts = nullptr, double cs = 1.0, double b5 = 1.0, double c5 = 0.0) {
    DhopArgs a;
    a.U = U;
    a.psi = psi;
    a.psi_scale = psis;
    a.out = out;
    a.out_scale = outs;
    a.g = g;
    a.prec = prec;
    a.link_fmt = fmt;
    a.kind = kind;
    a.dag = dag;
    a.diag = dg;
    a.mf = mf;
    a.stream = st;
    a.custom = true;
    a.cb = cb;
    a.y = y;
    a.y_scale = ys;
    a.beta = beta;
    a.cs = cs;
    a.b5 = b5;
    a.c5 = c5;
    if (fuse != kFuseNone) {
        a.fuse = fuse;
        a.fz = *fz;
        *nparts = dhop_blocks(a);
    }
    return launch_dhop(a);
}

// The Schur operator Mhat (dag: Mhat^dagger) on even checkerboard fields, with two temporaries
// per precision class (index 0: FP64, 1: the sloppy precision).
struct EoOp {
    GeomDev g;
    int kind;
    double diag, mf;
    double b5 = 1.0, c5 = 0.0, alpha = 0.0, beta = 0.0;   // Moebius: M_ee = alpha - beta S
    void *t1[2], *t2[2];
    float *t1s, *t2s;   // sloppy FP16 scales
};

// Moebius: out = (alpha / beta - S)^-1 in (S^dagger when dag), returning the factor f (1 / beta)
// that makes f out = M_oo^-1 in; with beta = 0, out = in and f = 1 / alpha.
static hipError_t mob_ee_inv(const EoOp &o, int prec, const void *in, const float *ins, void *out, float *outs, int dag,
                             hipStream_t st, double *f) {
    const long n4 = o.g.vol / 2;
    if (o.beta == 0.0) {
        *f = 1.0 / o.alpha;
        return launch_s5axpy(prec, in, ins, nullptr, nullptr, out, outs, n4 * o.g.Ls, o.g.Ls, 1.0, 0.0, 0.0, 0.0, o.mf, dag,
                             st);
    }
    *f = 1.0 / o.beta;
    return launch_m5inv(in, ins, out, outs, n4, o.g.Ls, o.alpha / o.beta, o.mf, dag, prec, st);
}

// Moebius Schur operator (see the header): two kernels on the checkerboard column walk when it
// takes the Moebius kinds, else five (with separate s-local passes and the M_ee inverse); the last
// carries the fused epilogue.
static hipError_t eo_apply_mobius(const EoOp &o, const void *U, int prec, int fmt, const void *in, const float *ins,
                                  void *out, float *outs, int dag, int fuse, const FuseDev *fz, long *nparts,
                                  hipStream_t st) {
    const int ix = prec == GRID_F64 ? 0 : 1;
    void *t1 = o.t1[ix], *t2 = o.t2[ix];
    float *t1s = prec == GRID_F16S ? o.t1s : nullptr, *t2s = prec == GRID_F16S ? o.t2s : nullptr;
    const long n5 = static_cast<long>(o.g.vol / 2) * o.g.Ls;
    const int Ls = o.g.Ls;
    double f = 1.0;
    if (mob_cb_applies(prec, Ls)) {
        // two kernels: B folded into the checkerboard walks (gathered records, or across the column
        // after the hop for the adjoint), the first also applying (alpha / beta - S)^-1 across the
        // column (M_oo = alpha when beta = 0: no inverse, f = 1 / alpha)
        const bool inv = o.beta != 0.0;
        f = inv ? 1.0 / o.beta : 1.0 / o.alpha;
        EOCHK(hop_cb(U, prec, fmt, o.g, inv ? kMobHopInv : kMobHop, dag, inv ? o.alpha / o.beta : 0.0, o.mf, 1, in,
                     ins, nullptr, nullptr, 1.0, t2, t2s, st, kFuseNone, nullptr, nullptr, 1.0, o.b5, o.c5));
        return hop_cb(U, prec, fmt, o.g, kMobDiag, dag, o.alpha, o.mf, 0, t2, t2s, in, ins, -0.25 * f, out, outs, st,
                      fuse, fz, nparts, o.beta, o.b5, o.c5);
    }
    if (!dag) {
        EOCHK(launch_s5axpy(prec, in, ins, nullptr, nullptr, t1, t1s, n5, Ls, o.b5, o.c5, 0.0, 0.0, o.mf, 0, st));
        EOCHK(hop_cb(U, prec, fmt, o.g, GRID_HOP, 0, 0.0, o.mf, 1, t1, t1s, nullptr, nullptr, 1.0, t2, t2s, st));
        EOCHK(mob_ee_inv(o, prec, t2, t2s, t1, t1s, 0, st, &f));
        EOCHK(launch_s5axpy(prec, t1, t1s, nullptr, nullptr, t2, t2s, n5, Ls, f * o.b5, f * o.c5, 0.0, 0.0, o.mf, 0, st));
        // out = alpha in - beta S in - H_eo t2 / 4
        return hop_cb(U, prec, fmt, o.g, GRID_DWF, 0, o.alpha, o.mf, 0, t2, t2s, in, ins, -0.25, out, outs, st, fuse, fz,
                      nparts, o.beta);
    }
    EOCHK(hop_cb(U, prec, fmt, o.g, GRID_HOP, 1, 0.0, o.mf, 1, in, ins, nullptr, nullptr, 1.0, t1, t1s, st));
    EOCHK(launch_s5axpy(prec, t1, t1s, nullptr, nullptr, t2, t2s, n5, Ls, o.b5, o.c5, 0.0, 0.0, o.mf, 1, st));
    EOCHK(mob_ee_inv(o, prec, t2, t2s, t1, t1s, 1, st, &f));
    EOCHK(hop_cb(U, prec, fmt, o.g, GRID_HOP, 1, 0.0, o.mf, 0, t1, t1s, nullptr, nullptr, 1.0, t2, t2s, st));
    // out = alpha in - beta S^dagger in - (b5 t2 + c5 S^dagger t2) f / 4
    if (fuse != kFuseNone) *nparts = s5_blocks(n5);
    return launch_s5axpy(prec, in, ins, t2, t2s, out, outs, n5, Ls, o.alpha, -o.beta, -0.25 * f * o.b5,
                         -0.25 * f * o.c5, o.mf, 1, st, fuse, fz ? *fz : FuseDev());
}

static hipError_t eo_apply_fz(const void *ctx, const void *U, int prec, int fmt, const void *in, const float *ins,
                              void *out, float *outs, int dag, int fuse, const FuseDev *fz, long *nparts,
                              hipStream_t st) {
    const EoOp &o = *static_cast<const EoOp *>(ctx);
    if (o.kind == GRID_MOBIUS) return eo_apply_mobius(o, U, prec, fmt, in, ins, out, outs, dag, fuse, fz, nparts, st);
    const int ix = prec == GRID_F64 ? 0 : 1;
    float *t1s = prec == GRID_F16S ? o.t1s : nullptr, *t2s = prec == GRID_F16S ? o.t2s : nullptr;
    if (o.kind == GRID_DWF && mob_cb_applies(prec, o.g.Ls)) {
        // M5^-1 H_oe in by one checkerboard walk (the inverse formed across the column's lanes)
        EOCHK(hop_cb(U, prec, fmt, o.g, kHopInv, dag, o.diag, o.mf, 1, in, ins, nullptr, nullptr, 1.0, o.t2[ix], t2s,
                     st));
        return hop_cb(U, prec, fmt, o.g, GRID_DWF, dag, o.diag, o.mf, 0, o.t2[ix], t2s, in, ins, -0.25, out, outs, st,
                      fuse, fz, nparts);
    }
    // t1 = H_oe in
    EOCHK(hop_cb(U, prec, fmt, o.g, GRID_HOP, dag, 0.0, o.mf, 1, in, ins, nullptr, nullptr, 1.0, o.t1[ix], t1s, st));
    const void *src = o.t1[ix];
    const float *srcs = t1s;
    if (o.kind == GRID_DWF) {
        EOCHK(launch_m5inv(o.t1[ix], t1s, o.t2[ix], t2s, o.g.vol / 2, o.g.Ls, o.diag, o.mf, dag, prec, st));
        src = o.t2[ix];
        srcs = t2s;
    }
    // out = M_ee in - H_eo M_oo^-1 H_oe in / 4  (Wilson: M_oo^-1 = 1 / (4 + m) folded into beta)
    const double beta = o.kind == GRID_WILSON ? -0.25 / o.diag : -0.25;
    return hop_cb(U, prec, fmt, o.g, o.kind, dag, o.diag, o.mf, 0, src, srcs, in, ins, beta, out, outs, st, fuse, fz,
                  nparts);
}

static hipError_t eo_apply(const void *ctx, const void *U, int prec, int fmt, const void *in, const float *ins, void *out,
                           float *outs, int dag, hipStream_t st) {
    return eo_apply_fz(ctx, U, prec, fmt, in, ins, out, outs, dag, kFuseNone, nullptr, nullptr, st);
}

// Mhat with the conjugate gradient's fused epilogue on its last kernel.
static hipError_t eo_apply_fused(const void *ctx, const void *U, int prec, int fmt, const void *in, const float *ins,
                                 void *out, float *outs, int dag, int fuse, const FuseDev &fz, long *nparts,
                                 hipStream_t st) {
    return eo_apply_fz(ctx, U, prec, fmt, in, ins, out, outs, dag, fuse, &fz, nparts, st);
}

static size_t al256(size_t v) { return (v + 255) & ~size_t(255); }

struct EoLayout {
    size_t be, bo, bhat, rhs, xe, xo, t1, t2, t1h, t2h, t1hs, t2hs, norm, cg, total;
};

static EoLayout eo_layout(const GeomDev &g, int sloppy, int link_fmt) {
    EoLayout L;
    memset(&L, 0, sizeof(L));
    const size_t n = static_cast<size_t>(g.n5 / 2);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = al256(off + bytes);
        return o;
    };
    // be and bo adjacent: together they hold a full FP64 field for the final residual
    L.be = take(2 * n * 192);
    L.bo = L.be + n * 192;
    L.bhat = take(n * 192);
    L.rhs = take(n * 192);
    // xe and xo adjacent: a full FP64 field (the Moebius residual's intermediate) once x is assembled
    L.xe = take(2 * n * 192);
    L.xo = L.xe + n * 192;
    L.t1 = take(n * 192);
    L.t2 = take(n * 192);
    if (sloppy != GRID_F64) {
        const size_t sb = sloppy == GRID_F32 ? 96 : 48;
        L.t1h = take(n * sb);
        L.t2h = take(n * sb);
        if (sloppy == GRID_F16S) {
            L.t1hs = take(n * 4);
            L.t2hs = take(n * 4);
        }
    }
    L.norm = take(kNormScratch * sizeof(double));
    L.cg = off;
    L.total = off + cg_workspace_bytes_n(static_cast<long>(n), static_cast<long>(g.vol) * 4, sloppy, link_fmt,
                                         fused_parts_max(static_cast<long>(n), g.L[3]));
    return L;
}

size_t solve_eo_workspace_bytes(const GeomDev &g, int sloppy, int link_fmt) { return eo_layout(g, sloppy, link_fmt).total; }

hipError_t run_solve_eo(const void *U, const void *b, void *x, const GeomDev &g, const grid_op &opd,
                        const grid_cg_params &p, void *ws, hipStream_t st, grid_cg_stats *stats, int *status) {
    const int kind = opd.kind;
    const double mf = opd.mf;
    const double diag = kind == GRID_WILSON ? 4.0 + opd.mass : 5.0 - opd.M5;
    const auto t0 = std::chrono::steady_clock::now();
    const EoLayout L = eo_layout(g, p.sloppy_prec, p.link_fmt);
    char *w = static_cast<char *>(ws);
    void *be = w + L.be, *bo = w + L.bo, *bhat = w + L.bhat, *rhs = w + L.rhs, *xe = w + L.xe, *xo = w + L.xo;
    double *norm = reinterpret_cast<double *>(w + L.norm);
    const long n = g.n5 / 2;
    *status = GRID_OK;
    memset(stats, 0, sizeof(*stats));

    double bb = 0.0;
    EOCHK(norm2_diff(b, nullptr, g.n5, norm, st, &bb));
    if (bb == 0.0) {
        EOCHK(hipMemsetAsync(x, 0, static_cast<size_t>(g.n5) * 192, st));
        EOCHK(hipStreamSynchronize(st));
        stats->converged = 1;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return hipSuccess;
    }
    EoOp o;
    o.g = g;
    o.kind = kind;
    o.diag = diag;
    o.mf = mf;
    o.t1[0] = w + L.t1;
    o.t2[0] = w + L.t2;
    o.t1[1] = p.sloppy_prec != GRID_F64 ? w + L.t1h : nullptr;
    o.t2[1] = p.sloppy_prec != GRID_F64 ? w + L.t2h : nullptr;
    o.t1s = p.sloppy_prec == GRID_F16S ? reinterpret_cast<float *>(w + L.t1hs) : nullptr;
    o.t2s = p.sloppy_prec == GRID_F16S ? reinterpret_cast<float *>(w + L.t2hs) : nullptr;
    if (kind == GRID_MOBIUS) {
        o.b5 = opd.b5;
        o.c5 = opd.c5;
        o.alpha = 1.0 + (4.0 - opd.M5) * opd.b5;
        o.beta = 1.0 - (4.0 - opd.M5) * opd.c5;
    }
    const long n5h = n;

    EOCHK(cb_copy(b, be, g, 0, 1, st));
    EOCHK(cb_copy(b, bo, g, 1, 1, st));
    // bhat = b_e + H_eo M_oo^-1 b_o / 2  (Moebius: H_eo B M_oo^-1 b_o / 2)
    const void *src = bo;
    double beta = 0.5 / diag;
    if (kind == GRID_MOBIUS) {
        double f = 1.0;
        EOCHK(mob_ee_inv(o, GRID_F64, bo, nullptr, o.t1[0], nullptr, 0, st, &f));
        EOCHK(launch_s5axpy(GRID_F64, o.t1[0], nullptr, nullptr, nullptr, o.t2[0], nullptr, n5h, g.Ls, f * o.b5,
                            f * o.c5, 0.0, 0.0, mf, 0, st));
        src = o.t2[0];
        beta = 0.5;
    } else if (kind == GRID_DWF) {
        EOCHK(launch_m5inv(bo, nullptr, o.t1[0], nullptr, g.vol / 2, g.Ls, diag, mf, 0, GRID_F64, st));
        src = o.t1[0];
        beta = 0.5;
    }
    EOCHK(hop_cb(U, GRID_F64, GRID_L18, g, GRID_WILSON, 0, 1.0, mf, 0, src, nullptr, be, nullptr, beta, bhat, nullptr, st));
    // rhs = Mhat^dagger bhat; initial guess: the even part of x
    EOCHK(eo_apply(&o, U, GRID_F64, GRID_L18, bhat, nullptr, rhs, nullptr, 1, st));
    EOCHK(cb_copy(x, xe, g, 0, 1, st));
    CgOp op;
    op.apply = eo_apply;
    op.apply_fused = eo_apply_fused;
    op.ctx = &o;
    grid_cg_stats cs;
    memset(&cs, 0, sizeof(cs));
    EOCHK(run_cg_op(op, U, rhs, xe, n, static_cast<long>(g.vol) * 4, p, w + L.cg, st, &cs, status, false,
                    fused_parts_max(static_cast<long>(n), g.L[3])));
    // x_o = M_oo^-1 (b_o + H_oe x_e / 2)  (Moebius: M_oo^-1 (b_o + H_oe B x_e / 2))
    if (kind == GRID_MOBIUS) {
        double f = 1.0;
        EOCHK(launch_s5axpy(GRID_F64, xe, nullptr, nullptr, nullptr, o.t2[0], nullptr, n5h, g.Ls, o.b5, o.c5, 0.0, 0.0,
                            mf, 0, st));
        EOCHK(hop_cb(U, GRID_F64, GRID_L18, g, GRID_WILSON, 0, 1.0, mf, 1, o.t2[0], nullptr, bo, nullptr, 0.5, o.t1[0],
                     nullptr, st));
        EOCHK(mob_ee_inv(o, GRID_F64, o.t1[0], nullptr, o.t2[0], nullptr, 0, st, &f));
        EOCHK(launch_s5axpy(GRID_F64, o.t2[0], nullptr, nullptr, nullptr, xo, nullptr, n5h, g.Ls, f, 0.0, 0.0, 0.0, mf, 0,
                            st));
    } else if (kind == GRID_DWF) {
        EOCHK(hop_cb(U, GRID_F64, GRID_L18, g, GRID_WILSON, 0, 1.0, mf, 1, xe, nullptr, bo, nullptr, 0.5, o.t1[0], nullptr,
                     st));
        EOCHK(launch_m5inv(o.t1[0], nullptr, xo, nullptr, g.vol / 2, g.Ls, diag, mf, 0, GRID_F64, st));
    } else {
        EOCHK(hop_cb(U, GRID_F64, GRID_L18, g, GRID_WILSON, 0, 1.0 / diag, mf, 1, xe, nullptr, bo, nullptr, 0.5 / diag, xo,
                     nullptr, st));
    }
    EOCHK(cb_copy(xe, x, g, 0, 0, st));
    EOCHK(cb_copy(xo, x, g, 1, 0, st));
    // true residual of the full system, in FP64 (be|bo now hold M x)
    DhopArgs a;
    a.U = U;
    a.psi = x;
    a.psi_scale = nullptr;
    a.out = be;
    a.out_scale = nullptr;
    a.g = g;
    a.prec = GRID_F64;
    a.link_fmt = GRID_L18;
    a.kind = kind;
    a.dag = 0;
    a.diag = diag;
    a.mf = mf;
    a.stream = st;
    if (kind == GRID_MOBIUS)
        EOCHK(launch_mobius(a, opd.M5, opd.b5, opd.c5, xe, nullptr));   // xe | xo: a full-field temporary
    else
        EOCHK(launch_dhop(a));
    double rr = 0.0;
    EOCHK(norm2_diff(b, be, g.n5, norm, st, &rr));
    stats->iterations = cs.iterations;
    stats->reliable_updates = cs.reliable_updates;
    stats->converged = cs.converged;
    stats->true_residual = sqrt(rr / bb);
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return hipSuccess;
}

}  // namespace gridmi
