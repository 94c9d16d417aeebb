// Moebius (Cayley) domain-wall operator, one of the five-dimensional chiral fermion actions the
// paper lists (Section 4):
//   M = D_W B + 1 - S,  D_W = (4 - M5) - H/2,  B = b5 + c5 S,
//   (S psi)_s = P_- psi~_{s+1} + P_+ psi~_{s-1}, psi~_{Ls} = -mf psi_0, psi~_{-1} = -mf psi_{Ls-1},
//   M^dagger = B^dagger D_W^dagger + 1 - S^dagger, S^dagger with P_+ and P_- exchanged.
// M psi is one s-local pass chi = B psi followed by one hopping pass whose epilogue adds the
// 4D-diagonal rest, (4 - M5) chi + psi - S psi = (1 + b5 (4 - M5)) psi - (1 - c5 (4 - M5)) S psi;
// M^dagger psi is one hopping pass phi = D_W^dagger psi followed by the s-local
// b5 phi + c5 S^dagger phi + psi - S^dagger psi. b5 = 1, c5 = 0 is the Shamir operator.
// FP32 and FP16-storage fields whose Ls divides 64 take one column-walk kernel instead (the
// s-local parts formed across the lanes of a fifth-dimension column, see k_dhop_walk), which
// saves the intermediate field's write and read.
#include "device.h"
#include "launch.h"

namespace gridmi {

constexpr int kS5Sites = 16;   // 5D sites per block, 16 lanes each (12 active, one per component)

// out = a1 u + a2 S u + a3 v + a4 S v (S^dagger when dag); v may be NULL (a3 = a4 = 0).
// FUSE: the conjugate gradient's epilogue (see FuseDev): |out|^2 partials, and with kFuseAxpy
// out = r - alpha (...) (r may be out: each element is read by the lane that overwrites it).
template <class SP, int FUSE>
__global__ void __launch_bounds__(256)
k_s5axpy(const void *__restrict__ u, const float *__restrict__ us, const void *__restrict__ v,
         const float *__restrict__ vs, void *out, float *outs, long n5, int Ls, double a1, double a2, double a3,
         double a4, double mf, int dag, FuseDev fz) {
    using C = typename SP::C;
    const long q = static_cast<long>(blockIdx.x) * kS5Sites + (threadIdx.x >> 4);
    const int k16 = threadIdx.x & 15;
    const bool live = q < n5 && k16 < 12;
    const long qq = q < n5 ? q : n5 - 1;
    const int k = k16 < 12 ? k16 : 0;
    const int s = static_cast<int>(qq % Ls);
    // lower spins take s + 1 and upper spins s - 1 (S); S^dagger exchanges them
    const bool plus = ((k / 3) >= 2) != (dag != 0);
    const int s2 = plus ? (s == Ls - 1 ? 0 : s + 1) : (s == 0 ? Ls - 1 : s - 1);
    const bool wall = plus ? (s == Ls - 1) : (s == 0);
    const C w = wall ? static_cast<C>(-mf) : C(1);
    const long q2 = qq - s + s2;
    const Cx<C> u0 = global_elem<SP>(u, us, qq, k), u1 = global_elem<SP>(u, us, q2, k);
    const C c1 = static_cast<C>(a1), c2 = static_cast<C>(a2) * w;
    Cx<C> r = {c1 * u0.r + c2 * u1.r, c1 * u0.i + c2 * u1.i};
    if (v) {
        const Cx<C> v0 = global_elem<SP>(v, vs, qq, k), v1 = global_elem<SP>(v, vs, q2, k);
        const C c3 = static_cast<C>(a3), c4 = static_cast<C>(a4) * w;
        r = {r.r + c3 * v0.r + c4 * v1.r, r.i + c3 * v0.i + c4 * v1.i};
    }
    if constexpr (FUSE != kFuseNone) {
        if constexpr (FUSE == kFuseAxpy) {
            const Cx<C> rv = global_elem<SP>(fz.r, fz.r_scale, qq, k);
            const C al = static_cast<C>(fz.scal[fz.num] / fz.scal[fz.den]);
            r = {rv.r - al * r.r, rv.i - al * r.i};
        }
        // block sum before the stores (the barrier then waits for no store)
        const double n2 = wave_sum64(stored_n2<SP>(r, live));
        __shared__ double fred[4];
        if ((threadIdx.x & 63) == 0) fred[threadIdx.x >> 6] = n2;
        __syncthreads();
        if (threadIdx.x == 0) fz.part[blockIdx.x] = (fred[0] + fred[1]) + (fred[2] + fred[3]);
    }
    store_elem<SP>(out, outs, qq, k, r, live);
}

long s5_blocks(long n5) { return (n5 + kS5Sites - 1) / kS5Sites; }

template <int FUSE>
static void s5axpy_prec(int prec, dim3 grid, hipStream_t st, const void *u, const float *us, const void *v,
                        const float *vs, void *out, float *outs, long n5, int Ls, double a1, double a2, double a3,
                        double a4, double mf, int dag, const FuseDev &fz) {
    const dim3 block(256);
    if (prec == GRID_F64)
        hipLaunchKernelGGL((k_s5axpy<SpF64, FUSE>), grid, block, 0, st, u, us, v, vs, out, outs, n5, Ls, a1, a2, a3, a4,
                           mf, dag, fz);
    else if (prec == GRID_F32)
        hipLaunchKernelGGL((k_s5axpy<SpF32, FUSE>), grid, block, 0, st, u, us, v, vs, out, outs, n5, Ls, a1, a2, a3, a4,
                           mf, dag, fz);
    else
        hipLaunchKernelGGL((k_s5axpy<SpF16S, FUSE>), grid, block, 0, st, u, us, v, vs, out, outs, n5, Ls, a1, a2, a3,
                           a4, mf, dag, fz);
}

hipError_t launch_s5axpy(int prec, const void *u, const float *us, const void *v, const float *vs, void *out,
                         float *outs, long n5, int Ls, double a1, double a2, double a3, double a4, double mf, int dag,
                         hipStream_t st, int fuse, const FuseDev &fz) {
    if (n5 == 0) return hipSuccess;
    const dim3 grid(static_cast<unsigned>(s5_blocks(n5)));
    if (fuse == kFuseAxpy)
        s5axpy_prec<kFuseAxpy>(prec, grid, st, u, us, v, vs, out, outs, n5, Ls, a1, a2, a3, a4, mf, dag, fz);
    else if (fuse == kFuseNone)
        s5axpy_prec<kFuseNone>(prec, grid, st, u, us, v, vs, out, outs, n5, Ls, a1, a2, a3, a4, mf, dag, fz);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

long fused_parts_max(long n5, int Lt) {
    const long d = dhop_blocks_max(n5, Lt), m = s5_blocks(n5);
    return d > m ? d : m;
}

hipError_t launch_mobius(const DhopArgs &a, double M5, double b5, double c5, void *tmp, float *tmp_scale,
                         long *nparts) {
    const double d4 = 4.0 - M5;
    const long n5 = a.g.n5;
    // a fused epilogue (a.fuse: norm with dag = 0, r update with dag = 1) goes to the last kernel
    if (a.fuse != kFuseNone && (!nparts || a.fuse != (a.dag ? kFuseAxpy : kFuseNorm))) return hipErrorInvalidValue;
    DhopArgs h = a;
    h.kind = GRID_MOBIUS;
    h.custom = false;
    h.b5 = b5;
    h.c5 = c5;
    h.diag = a.dag ? d4 : 1.0 + b5 * d4;
    h.cs = 1.0 - c5 * d4;
    if (walk_mobius_applies(h)) {
        // one column-walk kernel: B folded into the records it gathers (M) or applied across the
        // column's lanes after the hop (M^dagger); tmp is not used
        if (h.fuse != kFuseNone) *nparts = dhop_blocks(h);
        return launch_dhop(h);
    }
    h.custom = true;
    h.cb = -1;
    h.beta = -0.5;
    if (!a.dag) {
        // chi = B psi;  out = -H chi / 2 + (1 + b5 d4) psi - (1 - c5 d4) S psi
        hipError_t e = launch_s5axpy(a.prec, a.psi, a.psi_scale, nullptr, nullptr, tmp, tmp_scale, n5, a.g.Ls, b5, c5, 0.0,
                                     0.0, a.mf, 0, a.stream);
        if (e != hipSuccess) return e;
        h.kind = GRID_DWF;
        h.psi = tmp;
        h.psi_scale = tmp_scale;
        h.y = a.psi;
        h.y_scale = a.psi_scale;
        h.diag = 1.0 + b5 * d4;
        h.cs = 1.0 - c5 * d4;
        if (h.fuse != kFuseNone) *nparts = dhop_blocks(h);
        return launch_dhop(h);
    }
    h.fuse = kFuseNone;
    // phi = D_W^dagger psi;  out = b5 phi + c5 S^dagger phi + psi - S^dagger psi
    h.kind = GRID_WILSON;
    h.y = a.psi;
    h.y_scale = a.psi_scale;
    h.diag = d4;
    h.out = tmp;
    h.out_scale = tmp_scale;
    hipError_t e = launch_dhop(h);
    if (e != hipSuccess) return e;
    if (a.fuse != kFuseNone) *nparts = s5_blocks(n5);
    return launch_s5axpy(a.prec, tmp, tmp_scale, a.psi, a.psi_scale, a.out, a.out_scale, n5, a.g.Ls, b5, c5, 1.0, -1.0,
                         a.mf, 1, a.stream, a.fuse, a.fz);
}

}  // namespace gridmi
