// C ABI of libgrid_mi: host-side argument validation, dispatch to the kernel launchers, status
// codes and a thread-local error message. Every check runs before the first HIP call, so a
// rejected call has no effect on the device.
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "launch.h"

using namespace gridmi;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int ok() {
    g_err[0] = '\0';
    return GRID_OK;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(GRID_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Geometry: every extent >= 2, Ls >= 1, and V * Ls * 4 below 2^31 (kernel indices are 32-bit).
int check_geom(const grid_geom *geom, GeomDev *g) {
    if (!geom) return fail(GRID_EINVAL, "geom is NULL");
    int64_t vol = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (geom->dims[mu] < 2) return fail(GRID_ESHAPE, "dims[%d] = %d is below 2", mu, geom->dims[mu]);
        vol *= geom->dims[mu];
        if (vol > (int64_t(1) << 30)) return fail(GRID_ESHAPE, "lattice volume too large");
    }
    if (geom->Ls < 1) return fail(GRID_ESHAPE, "Ls = %d is below 1", geom->Ls);
    if (vol * geom->Ls * 4 >= (int64_t(1) << 31)) return fail(GRID_ESHAPE, "V * Ls too large for 32-bit indexing");
    for (int mu = 0; mu < 4; ++mu) g->L[mu] = geom->dims[mu];
    g->Ls = geom->Ls;
    g->vol = static_cast<int>(vol);
    g->n5 = static_cast<int>(vol * geom->Ls);
    return GRID_OK;
}

int check_ptr(const void *p, const char *name, uintptr_t align) {
    if (!p) return fail(GRID_EINVAL, "%s is NULL", name);
    if (reinterpret_cast<uintptr_t>(p) % align) return fail(GRID_EALIGN, "%s is not %d-byte aligned", name, (int)align);
    return GRID_OK;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    if (!a || !b || !na || !nb) return false;
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
    return a0 < b0 + nb && b0 < a0 + na;
}

size_t spinor_site_bytes(int prec) { return prec == GRID_F64 ? 192 : prec == GRID_F32 ? 96 : 48; }
size_t link_bytes(int prec, int fmt) {
    const size_t rows = fmt == GRID_L12 ? 2 : 3;
    const size_t cbytes = prec == GRID_F64 ? 16 : prec == GRID_F32 ? 8 : 4;
    return rows * 3 * cbytes;
}

int check_prec(int prec) {
    if (prec != GRID_F64 && prec != GRID_F32 && prec != GRID_F16S) return fail(GRID_EDTYPE, "unknown precision %d", prec);
    return GRID_OK;
}
int check_fmt(int fmt) {
    if (fmt != GRID_L18 && fmt != GRID_L12) return fail(GRID_EDTYPE, "unknown link format %d", fmt);
    return GRID_OK;
}

// Spinor (+ scale for F16S) argument check.
int check_spinor(const void *p, const float *scale, int prec, const char *name, const char *sname) {
    int rc = check_ptr(p, name, 16);
    if (rc) return rc;
    if (prec == GRID_F16S) return check_ptr(scale, sname, 4);
    if (scale) return fail(GRID_EINVAL, "%s must be NULL unless prec is GRID_F16S", sname);
    return GRID_OK;
}

#define TRY(x)                   \
    do {                         \
        int rc_ = (x);           \
        if (rc_) return rc_;     \
    } while (0)

// Checkerboard fields need every extent even (the parity of a site is then well defined across
// the periodic boundary, and x pairs up).
int check_even(const GeomDev &g) {
    for (int mu = 0; mu < 4; ++mu)
        if (g.L[mu] % 2) return fail(GRID_ESHAPE, "checkerboard fields need even extents (dims[%d] = %d)", mu, g.L[mu]);
    return GRID_OK;
}

// Operator and parameter checks shared by the solvers.
int check_solver_args(const GeomDev &g, const grid_op *op, const grid_cg_params *params, const grid_cg_stats *stats) {
    if (!op || !params || !stats) return fail(GRID_EINVAL, "op, params and stats must not be NULL");
    if (op->kind != GRID_WILSON && op->kind != GRID_DWF && op->kind != GRID_MOBIUS)
        return fail(GRID_EINVAL, "the solvers take GRID_WILSON, GRID_DWF or GRID_MOBIUS (got kind %d)", op->kind);
    if (op->kind == GRID_WILSON && g.Ls != 1) return fail(GRID_ESHAPE, "GRID_WILSON needs Ls == 1 (got %d)", g.Ls);
    TRY(check_prec(params->sloppy_prec));
    TRY(check_fmt(params->link_fmt));
    if (!(params->tol > 0.0) || params->maxiter < 0 || params->check_every < 1)
        return fail(GRID_EINVAL, "need tol > 0, maxiter >= 0 and check_every >= 1");
    if (params->sloppy_prec != GRID_F64 && !(params->delta > 0.0 && params->delta < 1.0))
        return fail(GRID_EINVAL, "reliable-update delta must lie in (0, 1)");
    return GRID_OK;
}

// Molecular-dynamics parameter and buffer checks.
int check_md(const GeomDev &g, const grid_md_params *p, const void *phi) {
    if (!p) return fail(GRID_EINVAL, "params is NULL");
    if (!isfinite(p->beta) || !isfinite(p->eps) || p->n_steps < 0)
        return fail(GRID_EINVAL, "need finite beta and eps and n_steps >= 0");
    if (p->integrator != GRID_LEAPFROG && p->integrator != GRID_OMELYAN && p->integrator != GRID_FORCE_GRADIENT)
        return fail(GRID_EINVAL, "unknown integrator %d", p->integrator);
    if (p->n_inner < 0) return fail(GRID_EINVAL, "n_inner = %d is negative", p->n_inner);
    if (phi) {
        if (p->fermion.kind != GRID_WILSON && p->fermion.kind != GRID_DWF && p->fermion.kind != GRID_MOBIUS)
            return fail(GRID_EINVAL, "the fermion force takes GRID_WILSON, GRID_DWF or GRID_MOBIUS (got kind %d)",
                        p->fermion.kind);
        grid_cg_stats dummy;
        TRY(check_solver_args(g, &p->fermion, &p->cg, &dummy));
    } else {
        TRY(check_prec(p->cg.sloppy_prec));
        TRY(check_fmt(p->cg.link_fmt));
    }
    return GRID_OK;
}

int check_md_buffers(const GeomDev &g, const grid_md_params *p, const void *U, const void *P, const void *phi,
                     const void *ws, size_t ws_bytes) {
    TRY(check_ptr(U, "U", 16));
    TRY(check_ptr(P, "P", 16));
    if (phi) TRY(check_ptr(phi, "phi", 16));
    TRY(check_ptr(ws, "workspace", 256));
    const size_t need = md_workspace_bytes(g, *p);
    if (ws_bytes < need) return fail(GRID_ESPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    const size_t lb = static_cast<size_t>(g.vol) * 4 * 144, sb = static_cast<size_t>(g.n5) * 192;
    if (overlap(U, lb, P, lb) || overlap(ws, need, U, lb) || overlap(ws, need, P, lb) ||
        (phi && (overlap(phi, sb, U, lb) || overlap(phi, sb, P, lb) || overlap(ws, need, phi, sb))))
        return fail(GRID_EINVAL, "U, P, phi and workspace must not overlap");
    return GRID_OK;
}

// Multigrid parameters and buffers (4D Wilson, FP64).
int check_mg(const GeomDev &g, const grid_op *op, const grid_mg_params *p) {
    if (!p) return fail(GRID_EINVAL, "params is NULL");
    if (g.Ls != 1) return fail(GRID_ESHAPE, "multigrid takes 4D fields (Ls = %d)", g.Ls);
    if (op && op->kind != GRID_WILSON) return fail(GRID_EINVAL, "multigrid takes GRID_WILSON (got kind %d)", op->kind);
    int64_t nb = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (p->block[mu] < 1 || g.L[mu] % p->block[mu])
            return fail(GRID_ESHAPE, "block[%d] = %d does not divide dims[%d] = %d", mu, p->block[mu], mu, g.L[mu]);
        nb *= p->block[mu];
    }
    if (p->nvec < 1 || p->nvec > 32) return fail(GRID_EINVAL, "nvec = %d outside 1..32", p->nvec);
    if (p->nvec > 6 * nb) return fail(GRID_EINVAL, "nvec = %d exceeds the 6 x %d dimensions of an aggregate chirality",
                                      p->nvec, (int)nb);
    if (p->setup_rounds < 0 || p->setup_iters < 0 || p->coarse_iters < 0 || p->smooth_iters < 0 || p->maxiter < 0)
        return fail(GRID_EINVAL, "iteration counts must be >= 0");
    if (p->restart < 1 || p->restart > 64) return fail(GRID_EINVAL, "restart = %d outside 1..64", p->restart);
    if (!(p->tol > 0.0) || !(p->coarse_tol >= 0.0)) return fail(GRID_EINVAL, "need tol > 0 and coarse_tol >= 0");
    TRY(check_prec(p->setup_prec));
    if (p->cycle_prec != GRID_F64 && p->cycle_prec != GRID_F32)
        return fail(GRID_EDTYPE, "cycle_prec must be GRID_F64 or GRID_F32 (got %d)", p->cycle_prec);
    return GRID_OK;
}

int check_ws(const void *ws, size_t bytes, size_t need) {
    TRY(check_ptr(ws, "workspace", 256));
    if (bytes < need) return fail(GRID_EINVAL, "workspace of %zu bytes, %zu needed", bytes, need);
    return GRID_OK;
}

// Normal operator M^dagger M: argument checks (tmp == NULL skips those of tmp) and the two launches.
int check_mdag_m(const GeomDev &g, const void *U, const void *psi, const float *psi_scale, const void *out,
                 const float *out_scale, const void *tmp, const float *tmp_scale, int prec, int link_fmt) {
    TRY(check_prec(prec));
    TRY(check_fmt(link_fmt));
    TRY(check_ptr(U, "U", 16));
    TRY(check_spinor(psi, psi_scale, prec, "psi", "psi_scale"));
    TRY(check_spinor(out, out_scale, prec, "out", "out_scale"));
    const size_t sb = spinor_site_bytes(prec) * static_cast<size_t>(g.n5);
    const size_t ub = link_bytes(prec, link_fmt) * static_cast<size_t>(g.vol) * 4;
    const size_t cb = prec == GRID_F16S ? sizeof(float) * static_cast<size_t>(g.n5) : 0;
    if (overlap(out, sb, psi, sb) || overlap(out, sb, U, ub)) return fail(GRID_EINVAL, "out overlaps psi or U");
    if (cb && (overlap(out_scale, cb, psi_scale, cb) || overlap(out_scale, cb, out, sb) ||
               overlap(out_scale, cb, psi, sb)))
        return fail(GRID_EINVAL, "out_scale overlaps an input or out");
    if (tmp) {
        TRY(check_spinor(tmp, tmp_scale, prec, "tmp", "tmp_scale"));
        if (overlap(tmp, sb, psi, sb) || overlap(tmp, sb, out, sb) || overlap(tmp, sb, U, ub))
            return fail(GRID_EINVAL, "tmp overlaps psi, out or U");
        if (cb && (overlap(tmp_scale, cb, psi_scale, cb) || overlap(tmp_scale, cb, out_scale, cb) ||
                   overlap(tmp_scale, cb, tmp, sb)))
            return fail(GRID_EINVAL, "tmp_scale overlaps another field");
    } else if (tmp_scale) {
        return fail(GRID_EINVAL, "tmp_scale without tmp");
    }
    return GRID_OK;
}

hipError_t launch_mdag_m(const GeomDev &g, const void *U, const void *psi, const float *psi_scale, void *out,
                         float *out_scale, void *tmp, float *tmp_scale, double M5, double mf, int prec, int link_fmt,
                         hipStream_t st) {
    DhopArgs a;
    a.U = U;
    a.psi = psi;
    a.psi_scale = psi_scale;
    a.out = tmp;
    a.out_scale = tmp_scale;
    a.g = g;
    a.prec = prec;
    a.link_fmt = link_fmt;
    a.kind = GRID_DWF;
    a.dag = 0;
    a.diag = 5.0 - M5;
    a.mf = mf;
    a.stream = st;
    hipError_t e = launch_dhop(a);
    if (e != hipSuccess) return e;
    a.psi = tmp;
    a.psi_scale = tmp_scale;
    a.out = out;
    a.out_scale = out_scale;
    a.dag = 1;
    return launch_dhop(a);
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Static scratch of the entry points that allocate nothing (callers that cannot call hipMalloc:
// code under stream capture, tight serving loops). Each device holds its own copy from module load
// until the process ends; its address on a device is looked up once, with that device current, and
// kept. In host code `scratch` names a host-side stand-in, never passed to a kernel or copy.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

int scratch_of_current_device(char **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(GRID_EINVAL, "device %d beyond the %d the library serves", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(GRID_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = static_cast<char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return GRID_OK;
}

}  // namespace

extern "C" {

const char *grid_last_error(void) { return g_err; }

int grid_version(void) { return 100; }

int grid_dhop(const void *U, const void *psi, const float *psi_scale, void *out, float *out_scale, const grid_geom *geom,
              const grid_op *op, int prec, int link_fmt, void *stream) {
    GeomDev g;
    TRY(check_geom(geom, &g));
    if (!op) return fail(GRID_EINVAL, "op is NULL");
    TRY(check_prec(prec));
    TRY(check_fmt(link_fmt));
    if (op->kind == GRID_MOBIUS) return fail(GRID_EINVAL, "GRID_MOBIUS needs a temporary: use grid_mobius");
    if (op->kind != GRID_HOP && op->kind != GRID_WILSON && op->kind != GRID_DWF)
        return fail(GRID_EINVAL, "unknown operator kind %d", op->kind);
    if (op->kind == GRID_WILSON && g.Ls != 1) return fail(GRID_ESHAPE, "GRID_WILSON needs Ls == 1 (got %d)", g.Ls);
    TRY(check_ptr(U, "U", 16));
    TRY(check_spinor(psi, psi_scale, prec, "psi", "psi_scale"));
    TRY(check_spinor(out, out_scale, prec, "out", "out_scale"));
    const size_t sb = spinor_site_bytes(prec) * static_cast<size_t>(g.n5);
    const size_t ub = link_bytes(prec, link_fmt) * static_cast<size_t>(g.vol) * 4;
    const size_t cb = prec == GRID_F16S ? sizeof(float) * static_cast<size_t>(g.n5) : 0;
    if (overlap(out, sb, psi, sb) || overlap(out, sb, U, ub)) return fail(GRID_EINVAL, "out overlaps psi or U");
    if (cb && (overlap(out_scale, cb, psi_scale, cb) || overlap(out_scale, cb, out, sb) ||
               overlap(out_scale, cb, psi, sb)))
        return fail(GRID_EINVAL, "out_scale overlaps an input or out");

    DhopArgs a;
    a.U = U;
    a.psi = psi;
    a.psi_scale = psi_scale;
    a.out = out;
    a.out_scale = out_scale;
    a.g = g;
    a.prec = prec;
    a.link_fmt = link_fmt;
    a.kind = op->kind;
    a.dag = op->dag ? 1 : 0;
    a.diag = op->kind == GRID_WILSON ? 4.0 + op->mass : (op->kind == GRID_DWF ? 5.0 - op->M5 : 0.0);
    a.mf = op->mf;
    a.stream = static_cast<hipStream_t>(stream);
    hipError_t e = launch_dhop(a);
    if (e != hipSuccess) return hip_fail(e, "grid_dhop launch");
    return ok();
}

int grid_mobius(const void *U, const void *psi, const float *psi_scale, void *out, float *out_scale, void *tmp,
                float *tmp_scale, const grid_geom *geom, const grid_op *op, int prec, int link_fmt, void *stream) {
    GeomDev g;
    TRY(check_geom(geom, &g));
    if (!op) return fail(GRID_EINVAL, "op is NULL");
    if (op->kind != GRID_MOBIUS) return fail(GRID_EINVAL, "grid_mobius needs op->kind == GRID_MOBIUS");
    TRY(check_prec(prec));
    TRY(check_fmt(link_fmt));
    TRY(check_ptr(U, "U", 16));
    TRY(check_spinor(psi, psi_scale, prec, "psi", "psi_scale"));
    TRY(check_spinor(out, out_scale, prec, "out", "out_scale"));
    TRY(check_spinor(tmp, tmp_scale, prec, "tmp", "tmp_scale"));
    const size_t sb = spinor_site_bytes(prec) * static_cast<size_t>(g.n5);
    const size_t ub = link_bytes(prec, link_fmt) * static_cast<size_t>(g.vol) * 4;
    const size_t cb = prec == GRID_F16S ? sizeof(float) * static_cast<size_t>(g.n5) : 0;
    if (overlap(out, sb, psi, sb) || overlap(out, sb, U, ub) || overlap(tmp, sb, psi, sb) || overlap(tmp, sb, out, sb) ||
        overlap(tmp, sb, U, ub))
        return fail(GRID_EINVAL, "out, tmp, psi and U must not overlap");
    if (cb && (overlap(out_scale, cb, psi_scale, cb) || overlap(tmp_scale, cb, psi_scale, cb) ||
               overlap(tmp_scale, cb, out_scale, cb)))
        return fail(GRID_EINVAL, "scale arrays overlap");
    DhopArgs a;
    a.U = U;
    a.psi = psi;
    a.psi_scale = psi_scale;
    a.out = out;
    a.out_scale = out_scale;
    a.g = g;
    a.prec = prec;
    a.link_fmt = link_fmt;
    a.kind = GRID_MOBIUS;
    a.dag = op->dag ? 1 : 0;
    a.diag = 0.0;
    a.mf = op->mf;
    a.stream = static_cast<hipStream_t>(stream);
    hipError_t e = launch_mobius(a, op->M5, op->b5, op->c5, tmp, tmp_scale);
    if (e != hipSuccess) return hip_fail(e, "grid_mobius launch");
    return ok();
}

int grid_dwf_mdag_m(const void *U, const void *psi, const float *psi_scale, void *out, float *out_scale, void *tmp,
                    float *tmp_scale, const grid_geom *geom, double M5, double mf, int prec, int link_fmt,
                    void *stream) {
    GeomDev g;
    TRY(check_geom(geom, &g));
    TRY(check_mdag_m(g, U, psi, psi_scale, out, out_scale, tmp, tmp_scale, prec, link_fmt));
    hipError_t e = launch_mdag_m(g, U, psi, psi_scale, out, out_scale, tmp, tmp_scale, M5, mf, prec, link_fmt,
                                 static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "grid_dwf_mdag_m launch");
    return ok();
}

int grid_dwf_mdag_m_noalloc(const void *U, const void *psi, const float *psi_scale, void *out, float *out_scale,
                            const grid_geom *geom, double M5, double mf, int prec, int link_fmt, void *stream) {
    GeomDev g;
    TRY(check_geom(geom, &g));
    TRY(check_mdag_m(g, U, psi, psi_scale, out, out_scale, nullptr, nullptr, prec, link_fmt));
    const size_t tb = align256(spinor_site_bytes(prec) * static_cast<size_t>(g.n5));
    const size_t need = tb + (prec == GRID_F16S ? sizeof(float) * static_cast<size_t>(g.n5) : 0);
    if (need > kScratchBytes)
        return fail(GRID_ESPACE, "M psi needs %zu bytes of scratch, above the library's static %zu bytes", need,
                    kScratchBytes);
    char *sp = nullptr;
    TRY(scratch_of_current_device(&sp));
    hipError_t e = launch_mdag_m(g, U, psi, psi_scale, out, out_scale, sp, prec == GRID_F16S ? reinterpret_cast<float *>(sp + tb) : nullptr,
                                 M5, mf, prec, link_fmt, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "grid_dwf_mdag_m_noalloc launch");
    return ok();
}

int grid_dhop_backward(const void *U, const void *psi, const void *grad_out, void *grad_psi, void *grad_U,
                       const grid_geom *geom, const grid_op *op, int prec, int force_mode, void *stream) {
    GeomDev g;
    TRY(check_geom(geom, &g));
    if (!op) return fail(GRID_EINVAL, "op is NULL");
    if (prec != GRID_F64 && prec != GRID_F32) return fail(GRID_EDTYPE, "grid_dhop_backward takes GRID_F64 or GRID_F32");
    if (op->kind != GRID_HOP && op->kind != GRID_WILSON && op->kind != GRID_DWF)
        return fail(GRID_EINVAL, "unknown operator kind %d", op->kind);
    if (op->kind == GRID_WILSON && g.Ls != 1) return fail(GRID_ESHAPE, "GRID_WILSON needs Ls == 1 (got %d)", g.Ls);
    if (force_mode != 0 && force_mode != 1) return fail(GRID_EINVAL, "force_mode must be 0 or 1");
    TRY(check_ptr(U, "U", 16));
    TRY(check_ptr(psi, "psi", 16));
    TRY(check_ptr(grad_out, "grad_out", 16));
    if (!grad_psi && !grad_U) return fail(GRID_EINVAL, "grad_psi and grad_U are both NULL");
    const size_t sb = spinor_site_bytes(prec) * static_cast<size_t>(g.n5);
    const size_t ub = link_bytes(prec, GRID_L18) * static_cast<size_t>(g.vol) * 4;
    if (grad_psi) {
        TRY(check_ptr(grad_psi, "grad_psi", 16));
        if (overlap(grad_psi, sb, grad_out, sb) || overlap(grad_psi, sb, psi, sb) || overlap(grad_psi, sb, U, ub))
            return fail(GRID_EINVAL, "grad_psi overlaps an input");
    }
    if (grad_U) {
        TRY(check_ptr(grad_U, "grad_U", 16));
        if (overlap(grad_U, ub, grad_out, sb) || overlap(grad_U, ub, psi, sb) || overlap(grad_U, ub, U, ub) ||
            overlap(grad_U, ub, grad_psi, sb))
            return fail(GRID_EINVAL, "grad_U overlaps an input or grad_psi");
    }
    if (grad_psi) {
        grid_op adj = *op;
        adj.dag = op->dag ? 0 : 1;
        TRY(grid_dhop(U, grad_out, nullptr, grad_psi, nullptr, geom, &adj, prec, GRID_L18, stream));
    }
    if (grad_U) {
        LinkGradArgs a;
        a.U = U;
        a.chi = grad_out;
        a.psi = psi;
        a.G = grad_U;
        a.g = g;
        a.prec = prec;
        a.dag = op->dag ? 1 : 0;
        a.force_mode = force_mode;
        a.coef = op->kind == GRID_HOP ? 1.0 : -0.5;
        a.stream = static_cast<hipStream_t>(stream);
        hipError_t e = launch_link_grad(a);
        if (e != hipSuccess) return hip_fail(e, "grid_dhop_backward launch");
    }
    return ok();
}

size_t grid_cg_workspace_bytes(const grid_geom *geom, const grid_cg_params *params) {
    GeomDev g;
    if (check_geom(geom, &g) || !params) return 0;
    if (check_prec(params->sloppy_prec) || check_fmt(params->link_fmt)) return 0;
    return cg_workspace_bytes(g, params->sloppy_prec, params->link_fmt);
}

int grid_cg(const void *U, const void *b, void *x, const grid_geom *geom, const grid_op *op, const grid_cg_params *params,
            void *workspace, size_t ws_bytes, grid_cg_stats *stats, void *stream) {
    GeomDev g;
    TRY(check_geom(geom, &g));
    TRY(check_solver_args(g, op, params, stats));
    TRY(check_ptr(U, "U", 16));
    TRY(check_ptr(b, "b", 16));
    TRY(check_ptr(x, "x", 16));
    TRY(check_ptr(workspace, "workspace", 256));
    const size_t need = cg_workspace_bytes(g, params->sloppy_prec, params->link_fmt);
    if (ws_bytes < need) return fail(GRID_ESPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    const size_t sb = static_cast<size_t>(g.n5) * 192, ub = static_cast<size_t>(g.vol) * 4 * 144;
    if (overlap(x, sb, b, sb) || overlap(x, sb, U, ub) || overlap(workspace, need, x, sb) ||
        overlap(workspace, need, b, sb) || overlap(workspace, need, U, ub))
        return fail(GRID_EINVAL, "x, b, U and workspace must not overlap");
    int status = GRID_OK;
    memset(stats, 0, sizeof(*stats));
    hipError_t e = run_cg(U, b, x, g, *op, *params, workspace, static_cast<hipStream_t>(stream), stats, &status);
    if (e != hipSuccess) return hip_fail(e, "grid_cg");
    if (status == GRID_ENOCONV)
        return fail(GRID_ENOCONV, "CG stopped after %d iterations at true residual %.3e", stats->iterations,
                    stats->true_residual);
    if (status == GRID_EBREAKDOWN) return fail(GRID_EBREAKDOWN, "CG breakdown after %d iterations", stats->iterations);
    return ok();
}

int grid_dhop_cb(const void *U, const void *psi, const float *psi_scale, const void *y, const float *y_scale, void *out,
                 float *out_scale, const grid_geom *geom, const grid_op *op, int out_parity, double beta, int prec,
                 int link_fmt, void *stream) {
    GeomDev g;
    TRY(check_geom(geom, &g));
    TRY(check_even(g));
    if (!op) return fail(GRID_EINVAL, "op is NULL");
    TRY(check_prec(prec));
    TRY(check_fmt(link_fmt));
    if (op->kind != GRID_HOP && op->kind != GRID_WILSON && op->kind != GRID_DWF)
        return fail(GRID_EINVAL, "unknown operator kind %d", op->kind);
    if (op->kind == GRID_WILSON && g.Ls != 1) return fail(GRID_ESHAPE, "GRID_WILSON needs Ls == 1 (got %d)", g.Ls);
    if (out_parity != 0 && out_parity != 1) return fail(GRID_EINVAL, "out_parity must be 0 or 1");
    TRY(check_ptr(U, "U", 16));
    TRY(check_spinor(psi, psi_scale, prec, "psi", "psi_scale"));
    TRY(check_spinor(out, out_scale, prec, "out", "out_scale"));
    if (op->kind == GRID_HOP) {
        if (y || y_scale) return fail(GRID_EINVAL, "y must be NULL for GRID_HOP");
    } else {
        TRY(check_spinor(y, y_scale, prec, "y", "y_scale"));
    }
    const size_t nh = static_cast<size_t>(g.n5 / 2);
    const size_t sb = spinor_site_bytes(prec) * nh;
    const size_t ub = link_bytes(prec, link_fmt) * static_cast<size_t>(g.vol) * 4;
    const size_t cb = prec == GRID_F16S ? sizeof(float) * nh : 0;
    if (overlap(out, sb, psi, sb) || overlap(out, sb, U, ub) || overlap(out, sb, y, y ? sb : 0))
        return fail(GRID_EINVAL, "out overlaps psi, y or U");
    if (cb && (overlap(out_scale, cb, psi_scale, cb) || overlap(out_scale, cb, y_scale, y_scale ? cb : 0) ||
               overlap(out_scale, cb, out, sb) || overlap(out_scale, cb, psi, sb)))
        return fail(GRID_EINVAL, "out_scale overlaps an input or out");
    DhopArgs a;
    a.U = U;
    a.psi = psi;
    a.psi_scale = psi_scale;
    a.out = out;
    a.out_scale = out_scale;
    a.g = g;
    a.prec = prec;
    a.link_fmt = link_fmt;
    a.kind = op->kind;
    a.dag = op->dag ? 1 : 0;
    a.diag = op->kind == GRID_WILSON ? 4.0 + op->mass : (op->kind == GRID_DWF ? 5.0 - op->M5 : 0.0);
    a.mf = op->mf;
    a.stream = static_cast<hipStream_t>(stream);
    a.custom = true;
    a.cb = out_parity;
    a.y = y;
    a.y_scale = y_scale;
    a.beta = beta;
    hipError_t e = launch_dhop(a);
    if (e != hipSuccess) return hip_fail(e, "grid_dhop_cb launch");
    return ok();
}

int grid_m5inv(const void *psi, const float *psi_scale, void *out, float *out_scale, long n4, int Ls, double M5,
               double mf, int dag, int prec, void *stream) {
    TRY(check_prec(prec));
    if (Ls < 1 || Ls > 64) return fail(GRID_ESHAPE, "grid_m5inv needs 1 <= Ls <= 64 (got %d)", Ls);
    if (n4 < 0 || n4 * Ls * 4 >= (long(1) << 31)) return fail(GRID_ESHAPE, "n4 out of range");
    if (!(fabs(5.0 - M5) > 1.0)) return fail(GRID_EINVAL, "grid_m5inv needs |5 - M5| > 1 (got M5 = %g)", M5);
    TRY(check_spinor(psi, psi_scale, prec, "psi", "psi_scale"));
    TRY(check_spinor(out, out_scale, prec, "out", "out_scale"));
    const size_t sb = spinor_site_bytes(prec) * static_cast<size_t>(n4) * Ls;
    if (overlap(out, sb, psi, sb)) return fail(GRID_EINVAL, "out overlaps psi");
    if (out_scale && (overlap(out_scale, 4 * n4 * Ls, psi, sb) || overlap(out_scale, 4 * n4 * Ls, out, sb) ||
                      overlap(out_scale, 4 * n4 * Ls, psi_scale, psi_scale ? 4 * n4 * Ls : 0)))
        return fail(GRID_EINVAL, "out_scale overlaps another buffer");
    hipError_t e = launch_m5inv(psi, psi_scale, out, out_scale, n4, Ls, 5.0 - M5, mf, dag ? 1 : 0, prec,
                                static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "grid_m5inv launch");
    return ok();
}

size_t grid_solve_eo_workspace_bytes(const grid_geom *geom, const grid_cg_params *params) {
    GeomDev g;
    if (check_geom(geom, &g) || check_even(g) || !params) return 0;
    if (check_prec(params->sloppy_prec) || check_fmt(params->link_fmt)) return 0;
    return solve_eo_workspace_bytes(g, params->sloppy_prec, params->link_fmt);
}

int grid_solve_eo(const void *U, const void *b, void *x, const grid_geom *geom, const grid_op *op,
                  const grid_cg_params *params, void *workspace, size_t ws_bytes, grid_cg_stats *stats, void *stream) {
    GeomDev g;
    TRY(check_geom(geom, &g));
    TRY(check_even(g));
    TRY(check_solver_args(g, op, params, stats));
    if (op->kind == GRID_DWF) {
        if (g.Ls > 64) return fail(GRID_ESHAPE, "grid_solve_eo needs Ls <= 64 for the domain-wall M5 inverse");
        if (!(fabs(5.0 - op->M5) > 1.0)) return fail(GRID_EINVAL, "grid_solve_eo needs |5 - M5| > 1");
    } else if (op->kind == GRID_MOBIUS) {
        if (g.Ls > 64) return fail(GRID_ESHAPE, "grid_solve_eo needs Ls <= 64 for the Moebius M_ee inverse");
        const double alpha = 1.0 + (4.0 - op->M5) * op->b5, beta = 1.0 - (4.0 - op->M5) * op->c5;
        if (beta != 0.0 ? !(fabs(alpha / beta) > 1.0) : !(alpha != 0.0))
            return fail(GRID_EINVAL,
                        "grid_solve_eo needs |alpha / beta| > 1 (alpha = 1 + (4 - M5) b5 = %g, beta = 1 - (4 - M5) c5 = "
                        "%g), or beta = 0 and alpha != 0",
                        alpha, beta);
    } else if (!(fabs(4.0 + op->mass) > 0.0)) {
        return fail(GRID_EINVAL, "grid_solve_eo needs 4 + mass != 0");
    }
    TRY(check_ptr(U, "U", 16));
    TRY(check_ptr(b, "b", 16));
    TRY(check_ptr(x, "x", 16));
    TRY(check_ptr(workspace, "workspace", 256));
    const size_t need = solve_eo_workspace_bytes(g, params->sloppy_prec, params->link_fmt);
    if (ws_bytes < need) return fail(GRID_ESPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    const size_t sb = static_cast<size_t>(g.n5) * 192, ub = static_cast<size_t>(g.vol) * 4 * 144;
    if (overlap(x, sb, b, sb) || overlap(x, sb, U, ub) || overlap(workspace, need, x, sb) ||
        overlap(workspace, need, b, sb) || overlap(workspace, need, U, ub))
        return fail(GRID_EINVAL, "x, b, U and workspace must not overlap");
    int status = GRID_OK;
    memset(stats, 0, sizeof(*stats));
    hipError_t e = run_solve_eo(U, b, x, g, *op, *params, workspace, static_cast<hipStream_t>(stream), stats, &status);
    if (e != hipSuccess) return hip_fail(e, "grid_solve_eo");
    if (status == GRID_ENOCONV)
        return fail(GRID_ENOCONV, "CG stopped after %d iterations (full residual %.3e)", stats->iterations,
                    stats->true_residual);
    if (status == GRID_EBREAKDOWN) return fail(GRID_EBREAKDOWN, "CG breakdown after %d iterations", stats->iterations);
    return ok();
}

// ---- Hybrid Monte Carlo ----

size_t grid_md_workspace_bytes(const grid_geom *geom, const grid_md_params *params) {
    GeomDev g;
    if (check_geom(geom, &g) || !params) return 0;
    if (check_prec(params->cg.sloppy_prec) || check_fmt(params->cg.link_fmt)) return 0;
    return md_workspace_bytes(g, *params);
}

int grid_gauge_force(const void *U, void *F, const grid_geom *geom, double beta, void *stream) {
    GeomDev g;
    TRY(check_geom(geom, &g));
    TRY(check_ptr(U, "U", 16));
    TRY(check_ptr(F, "F", 16));
    const size_t lb = static_cast<size_t>(g.vol) * 4 * 144;
    if (overlap(U, lb, F, lb)) return fail(GRID_EINVAL, "F overlaps U");
    hipError_t e = launch_gauge_force(U, F, g, beta, 1.0, 0, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "grid_gauge_force launch");
    return ok();
}

int grid_link_exp(void *U, const void *P, double eps, long n_links, void *stream) {
    if (n_links < 0 || n_links >= (long(1) << 31)) return fail(GRID_ESHAPE, "n_links out of range");
    TRY(check_ptr(U, "U", 16));
    TRY(check_ptr(P, "P", 16));
    if (overlap(U, 144 * n_links, P, 144 * n_links)) return fail(GRID_EINVAL, "P overlaps U");
    hipError_t e = launch_link_exp(U, P, eps, n_links, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "grid_link_exp launch");
    return ok();
}

int grid_md_leapfrog(void *U, void *P, const void *phi, const grid_geom *geom, const grid_md_params *params,
                     void *workspace, size_t ws_bytes, grid_md_stats *stats, void *stream) {
    GeomDev g;
    TRY(check_geom(geom, &g));
    TRY(check_md(g, params, phi));
    if (!stats) return fail(GRID_EINVAL, "stats is NULL");
    TRY(check_md_buffers(g, params, U, P, phi, workspace, ws_bytes));
    hipError_t e = run_md_leapfrog(U, P, phi, g, *params, workspace, static_cast<hipStream_t>(stream), stats);
    if (e != hipSuccess) return hip_fail(e, "grid_md_leapfrog");
    return ok();
}

size_t grid_pseudofermion_workspace_bytes(const grid_geom *geom, const grid_cg_params *params) {
    GeomDev g;
    if (!params || check_geom(geom, &g) != GRID_OK) return 0;
    if (check_prec(params->sloppy_prec) != GRID_OK || check_fmt(params->link_fmt) != GRID_OK) return 0;
    return pf_workspace_bytes(g, *params);
}

int grid_pseudofermion_action(const void *U, const void *phi, void *X, const grid_geom *geom, const grid_op *op,
                              const grid_cg_params *params, double grad_scale, double *S, void *dS_dU, int force_mode,
                              void *dS_dphi, void *workspace, size_t ws_bytes, grid_cg_stats *stats, void *stream) {
    GeomDev g;
    TRY(check_geom(geom, &g));
    TRY(check_solver_args(g, op, params, stats));
    if (op->kind != GRID_WILSON && op->kind != GRID_DWF && op->kind != GRID_MOBIUS)
        return fail(GRID_EINVAL, "the pseudofermion action takes GRID_WILSON, GRID_DWF or GRID_MOBIUS (got kind %d)",
                    op->kind);
    if (force_mode != 0 && force_mode != 1) return fail(GRID_EINVAL, "force_mode must be 0 or 1 (got %d)", force_mode);
    if (!isfinite(grad_scale)) return fail(GRID_EINVAL, "grad_scale must be finite");
    TRY(check_ptr(U, "U", 16));
    TRY(check_ptr(phi, "phi", 16));
    TRY(check_ptr(X, "X", 16));
    if (dS_dU) TRY(check_ptr(dS_dU, "dS_dU", 16));
    if (dS_dphi) TRY(check_ptr(dS_dphi, "dS_dphi", 16));
    TRY(check_ptr(workspace, "workspace", 256));
    const size_t need = pf_workspace_bytes(g, *params);
    if (ws_bytes < need) return fail(GRID_ESPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    const size_t sb = static_cast<size_t>(g.n5) * 192, ub = static_cast<size_t>(g.vol) * 4 * 144;
    const void *bufs[6] = {U, phi, X, dS_dU, dS_dphi, workspace};
    const size_t sizes[6] = {ub, sb, sb, ub, sb, need};
    for (int i = 2; i < 6; ++i)        // outputs against every other buffer (inputs may share memory)
        for (int j = 0; j < 6; ++j)
            if (j != i && overlap(bufs[i], sizes[i], bufs[j], sizes[j]))
                return fail(GRID_EINVAL, "X, dS_dU, dS_dphi and workspace must not overlap each other or U, phi");
    int status = GRID_OK;
    memset(stats, 0, sizeof(*stats));
    hipError_t e = run_pseudofermion(U, phi, X, g, *op, *params, grad_scale, S, dS_dU, force_mode, dS_dphi, workspace,
                                     static_cast<hipStream_t>(stream), stats, &status);
    if (e != hipSuccess) return hip_fail(e, "grid_pseudofermion_action");
    if (status == GRID_ENOCONV)
        return fail(GRID_ENOCONV, "the solve stopped after %d iterations at true residual %.3e", stats->iterations,
                    stats->true_residual);
    if (status == GRID_EBREAKDOWN) return fail(GRID_EBREAKDOWN, "CG breakdown after %d iterations", stats->iterations);
    return ok();
}

int grid_hmc_energy(const void *U, const void *P, const void *phi, const grid_geom *geom, const grid_md_params *params,
                    void *workspace, size_t ws_bytes, double energies[4], grid_md_stats *stats, void *stream) {
    GeomDev g;
    TRY(check_geom(geom, &g));
    TRY(check_md(g, params, phi));
    if (!stats || !energies) return fail(GRID_EINVAL, "stats and energies must not be NULL");
    TRY(check_md_buffers(g, params, U, P, phi, workspace, ws_bytes));
    hipError_t e = run_hmc_energy(U, P, phi, g, *params, workspace, static_cast<hipStream_t>(stream), energies, stats);
    if (e != hipSuccess) return hip_fail(e, "grid_hmc_energy");
    return ok();
}

int grid_convert_spinor(const void *src, int src_prec, const float *src_scale, void *dst, int dst_prec, float *dst_scale,
                        long n_sites, void *stream) {
    TRY(check_prec(src_prec));
    TRY(check_prec(dst_prec));
    if (n_sites < 0 || n_sites >= (long(1) << 31)) return fail(GRID_ESHAPE, "n_sites out of range");
    TRY(check_spinor(src, src_scale, src_prec, "src", "src_scale"));
    TRY(check_spinor(dst, dst_scale, dst_prec, "dst", "dst_scale"));
    const size_t sa = spinor_site_bytes(src_prec) * n_sites, sd = spinor_site_bytes(dst_prec) * n_sites;
    if (overlap(src, sa, dst, sd)) return fail(GRID_EINVAL, "dst overlaps src");
    if (dst_scale && (overlap(dst_scale, 4 * n_sites, src, sa) || overlap(dst_scale, 4 * n_sites, dst, sd) ||
                      overlap(dst_scale, 4 * n_sites, src_scale, src_scale ? 4 * n_sites : 0)))
        return fail(GRID_EINVAL, "dst_scale overlaps another buffer");
    hipError_t e = launch_convert_spinor(src, src_prec, src_scale, dst, dst_prec, dst_scale, n_sites,
                                         static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "grid_convert_spinor launch");
    return ok();
}

int grid_convert_links(const void *src, void *dst, int dst_prec, int dst_fmt, int reunitarise, long n_links,
                       void *stream) {
    TRY(check_prec(dst_prec));
    TRY(check_fmt(dst_fmt));
    if (n_links < 0 || n_links >= (long(1) << 31)) return fail(GRID_ESHAPE, "n_links out of range");
    TRY(check_ptr(src, "src", 16));
    TRY(check_ptr(dst, "dst", 16));
    if (overlap(src, 144 * n_links, dst, link_bytes(dst_prec, dst_fmt) * n_links))
        return fail(GRID_EINVAL, "dst overlaps src");
    hipError_t e = launch_convert_links(src, dst, dst_prec, dst_fmt, reunitarise, n_links, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "grid_convert_links launch");
    return ok();
}

int grid_coarse_stencil(const void *A, const void *v, void *out, const int coarse_dims[4], int N, int dag,
                        void *stream) {
    if (!coarse_dims) return fail(GRID_EINVAL, "coarse_dims is NULL");
    int64_t vc = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (coarse_dims[mu] < 1) return fail(GRID_ESHAPE, "coarse_dims[%d] = %d is below 1", mu, coarse_dims[mu]);
        vc *= coarse_dims[mu];
        if (vc > (int64_t(1) << 24)) return fail(GRID_ESHAPE, "coarse volume too large");
    }
    if (N < 1 || N > 64) return fail(GRID_EINVAL, "N = %d outside 1..64", N);
    TRY(check_ptr(A, "A", 16));
    TRY(check_ptr(v, "v", 16));
    TRY(check_ptr(out, "out", 16));
    const size_t vb = static_cast<size_t>(vc) * N * 16;
    if (overlap(v, vb, out, vb) || overlap(A, vb * 9 * N, out, vb)) return fail(GRID_EINVAL, "out overlaps an input");
    hipError_t e = launch_coarse_stencil(A, v, out, coarse_dims, N, dag ? 1 : 0, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "grid_coarse_stencil launch");
    return ok();
}

size_t grid_mg_workspace_bytes(const grid_geom *geom, const grid_mg_params *params) {
    GeomDev g;
    if (check_geom(geom, &g) || check_mg(g, nullptr, params)) return 0;
    return mg_workspace_bytes(g, *params);
}

int grid_mg_basis(const void *U, void *vecs, const grid_geom *geom, const grid_op *op, const grid_mg_params *params,
                  void *workspace, size_t ws_bytes, void *stream) {
    GeomDev g;
    TRY(check_geom(geom, &g));
    if (!op) return fail(GRID_EINVAL, "op is NULL");
    TRY(check_mg(g, op, params));
    TRY(check_ptr(U, "U", 16));
    TRY(check_ptr(vecs, "vecs", 16));
    TRY(check_ws(workspace, ws_bytes, mg_workspace_bytes(g, *params)));
    const size_t fb = static_cast<size_t>(g.vol) * 192;
    if (overlap(vecs, fb * params->nvec, workspace, ws_bytes) || overlap(vecs, fb * params->nvec, U, 4 * 144 * g.vol))
        return fail(GRID_EINVAL, "vecs overlaps U or the workspace");
    hipError_t e = run_mg_basis(U, vecs, g, op->mass, *params, workspace, static_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "grid_mg_basis");
    return ok();
}

int grid_mg_coarse_op(const void *U, const void *vecs, void *A, const grid_geom *geom, const grid_op *op,
                      const grid_mg_params *params, void *workspace, size_t ws_bytes, void *stream) {
    GeomDev g;
    TRY(check_geom(geom, &g));
    if (!op) return fail(GRID_EINVAL, "op is NULL");
    TRY(check_mg(g, op, params));
    TRY(check_ptr(U, "U", 16));
    TRY(check_ptr(vecs, "vecs", 16));
    TRY(check_ptr(A, "A", 16));
    TRY(check_ws(workspace, ws_bytes, mg_workspace_bytes(g, *params)));
    int64_t vc = 1;
    for (int mu = 0; mu < 4; ++mu) vc *= g.L[mu] / params->block[mu];
    const size_t N = 2 * static_cast<size_t>(params->nvec);
    const size_t ab = static_cast<size_t>(vc) * 9 * N * N * 16;
    if (overlap(A, ab, vecs, static_cast<size_t>(g.vol) * 192 * params->nvec) || overlap(A, ab, workspace, ws_bytes) ||
        overlap(A, ab, U, 4 * 144 * static_cast<size_t>(g.vol)))
        return fail(GRID_EINVAL, "A overlaps another buffer");
    hipError_t e = run_mg_coarse_op(U, vecs, A, g, op->mass, *params, workspace, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "grid_mg_coarse_op");
    return ok();
}

int grid_mg_restrict(const void *vecs, const void *psi, void *vc, const grid_geom *geom, const grid_mg_params *params,
                     void *stream) {
    GeomDev g;
    TRY(check_geom(geom, &g));
    TRY(check_mg(g, nullptr, params));
    TRY(check_ptr(vecs, "vecs", 16));
    TRY(check_ptr(psi, "psi", 16));
    TRY(check_ptr(vc, "vc", 16));
    hipError_t e = launch_mg_restrict(vecs, psi, vc, g, *params, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "grid_mg_restrict launch");
    return ok();
}

int grid_mg_prolong(const void *vecs, const void *vc, void *psi, const grid_geom *geom, const grid_mg_params *params,
                    void *stream) {
    GeomDev g;
    TRY(check_geom(geom, &g));
    TRY(check_mg(g, nullptr, params));
    TRY(check_ptr(vecs, "vecs", 16));
    TRY(check_ptr(vc, "vc", 16));
    TRY(check_ptr(psi, "psi", 16));
    if (overlap(psi, static_cast<size_t>(g.vol) * 192, vecs, static_cast<size_t>(g.vol) * 192 * params->nvec))
        return fail(GRID_EINVAL, "psi overlaps vecs");
    hipError_t e = launch_mg_prolong(vecs, vc, psi, g, *params, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "grid_mg_prolong launch");
    return ok();
}

static int mg_solve_entry(const char *name, const char *method, bool pcg, const void *U, const void *vecs,
                          const void *A, const void *b, void *x, const grid_geom *geom, const grid_op *op,
                          const grid_mg_params *params, void *workspace, size_t ws_bytes, grid_cg_stats *stats,
                          void *stream) {
    GeomDev g;
    TRY(check_geom(geom, &g));
    if (!op || !stats) return fail(GRID_EINVAL, "op and stats must not be NULL");
    TRY(check_mg(g, op, params));
    TRY(check_ptr(U, "U", 16));
    TRY(check_ptr(vecs, "vecs", 16));
    TRY(check_ptr(A, "A", 16));
    TRY(check_ptr(b, "b", 16));
    TRY(check_ptr(x, "x", 16));
    TRY(check_ws(workspace, ws_bytes, mg_workspace_bytes(g, *params)));
    const size_t fb = static_cast<size_t>(g.vol) * 192;
    if (overlap(x, fb, b, fb) || overlap(x, fb, workspace, ws_bytes) || overlap(x, fb, vecs, fb * params->nvec))
        return fail(GRID_EINVAL, "x overlaps another buffer");
    memset(stats, 0, sizeof(*stats));
    int status = GRID_OK;
    hipError_t e = run_mg_solve(U, vecs, A, b, x, g, op->mass, *params, workspace, static_cast<hipStream_t>(stream),
                                stats, &status, pcg);
    if (e != hipSuccess) return hip_fail(e, name);
    if (status == GRID_ENOCONV)
        return fail(GRID_ENOCONV, "%s stopped at relative residual %.3e after %d iterations", method,
                    stats->true_residual, stats->iterations);
    if (status == GRID_EBREAKDOWN)
        return fail(GRID_EBREAKDOWN, "%s breakdown after %d iterations", method, stats->iterations);
    return ok();
}

int grid_mg_solve(const void *U, const void *vecs, const void *A, const void *b, void *x, const grid_geom *geom,
                  const grid_op *op, const grid_mg_params *params, void *workspace, size_t ws_bytes,
                  grid_cg_stats *stats, void *stream) {
    return mg_solve_entry("grid_mg_solve", "GCR", false, U, vecs, A, b, x, geom, op, params, workspace, ws_bytes, stats,
                          stream);
}

int grid_mg_pcg(const void *U, const void *vecs, const void *A, const void *b, void *x, const grid_geom *geom,
                const grid_op *op, const grid_mg_params *params, void *workspace, size_t ws_bytes,
                grid_cg_stats *stats, void *stream) {
    return mg_solve_entry("grid_mg_pcg", "pCG", true, U, vecs, A, b, x, geom, op, params, workspace, ws_bytes, stats,
                          stream);
}

}  // extern "C"
