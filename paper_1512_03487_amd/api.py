"""Torch-facing wrappers of the C ABI (argument marshalling only; every step runs in HIP kernels).

Fields are torch tensors on a ROCm device in the site-major layout of include/grid_mi.h:

* 4D spinor ``(Lt, Lz, Ly, Lx, 4, 3)`` and 5D spinor ``(Lt, Lz, Ly, Lx, Ls, 4, 3)``: complex128
  (FP64) or complex64 (FP32); FP16 storage is an :class:`F16Spinor` (half codes with a trailing
  re/im axis plus one float32 scale per site).
* links ``(Lt, Lz, Ly, Lx, 4, 3, 3)`` (18-real) or ``(..., 4, 2, 3)`` (12-real), complex128 /
  complex64, or float16 with a trailing re/im axis for FP16 storage.

All calls are asynchronous on torch's current stream except :func:`cg`.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import (GRID_DWF, GRID_F16S, GRID_F32, GRID_F64, GRID_HOP, GRID_L12, GRID_L18, GRID_MOBIUS, GRID_WILSON,
                   GridCgParams, GridCgStats, GridGeom, GridMdParams, GridMdStats, GridMgParams, GridOp, check,
                   load)

_KIND = {"hop": GRID_HOP, "wilson": GRID_WILSON, "dwf": GRID_DWF, "mobius": GRID_MOBIUS}
_PREC = {"f64": GRID_F64, "f32": GRID_F32, "f16s": GRID_F16S}
_FMT = {"L18": GRID_L18, "L12": GRID_L12}


@dataclass
class F16Spinor:
    """FP16-storage spinor: ``codes`` float16 (site shape + (4, 3, 2)), ``scale`` float32 (site shape)."""
    codes: torch.Tensor
    scale: torch.Tensor

    @property
    def shape(self):
        return tuple(self.codes.shape[:-1])

    @property
    def device(self):
        return self.codes.device

    @staticmethod
    def empty(site_shape, device) -> "F16Spinor":
        return F16Spinor(torch.empty(tuple(site_shape) + (4, 3, 2), dtype=torch.float16, device=device),
                         torch.empty(tuple(site_shape), dtype=torch.float32, device=device))


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _need_cuda(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on a GPU device")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def spinor_prec(psi) -> int:
    if isinstance(psi, F16Spinor):
        _need_cuda(psi.codes, "psi.codes")
        _need_cuda(psi.scale, "psi.scale")
        return GRID_F16S
    _need_cuda(psi, "psi")
    if psi.dtype == torch.complex128:
        return GRID_F64
    if psi.dtype == torch.complex64:
        return GRID_F32
    raise TypeError(f"unsupported spinor dtype {psi.dtype}")


def geom_of(psi) -> GridGeom:
    shape = psi.shape
    if len(shape) == 6 and tuple(shape[4:]) == (4, 3):
        lt, lz, ly, lx = shape[:4]
        ls = 1
    elif len(shape) == 7 and tuple(shape[5:]) == (4, 3):
        lt, lz, ly, lx, ls = shape[:5]
    else:
        raise ValueError(f"spinor shape {tuple(shape)} is neither (Lt,Lz,Ly,Lx,4,3) nor (Lt,Lz,Ly,Lx,Ls,4,3)")
    g = GridGeom()
    g.dims[:] = [int(lx), int(ly), int(lz), int(lt)]
    g.Ls = int(ls)
    return g


def link_format(U, prec: int) -> int:
    _need_cuda(U, "U")
    want = {GRID_F64: torch.complex128, GRID_F32: torch.complex64, GRID_F16S: torch.float16}[prec]
    if U.dtype != want:
        raise TypeError(f"links must be {want} for this spinor precision (got {U.dtype})")
    tail = tuple(U.shape[4:]) if prec != GRID_F16S else tuple(U.shape[4:-1])
    if tail == (4, 3, 3):
        return GRID_L18
    if tail == (4, 2, 3):
        return GRID_L12
    raise ValueError(f"link shape {tuple(U.shape)} is not (..., 4, 3, 3) or (..., 4, 2, 3)")


def _check_like(t, ref, name, ref_name="psi"):
    """Raise unless t is a field of ref's kind, shape, dtype and device (checked before any launch)."""
    if isinstance(ref, F16Spinor):
        if not isinstance(t, F16Spinor):
            raise TypeError(f"{name} must be an F16Spinor like {ref_name}")
        pairs = ((t.codes, ref.codes, ".codes"), (t.scale, ref.scale, ".scale"))
    else:
        if isinstance(t, F16Spinor) or not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor like {ref_name}")
        pairs = ((t, ref, ""),)
    for a, b, sfx in pairs:
        _need_cuda(a, name + sfx)
        if a.dtype != b.dtype:
            raise TypeError(f"{name}{sfx} has dtype {a.dtype}, {ref_name}{sfx} has {b.dtype}")
        if tuple(a.shape) != tuple(b.shape):
            raise ValueError(f"{name}{sfx} has shape {tuple(a.shape)}, {ref_name}{sfx} has {tuple(b.shape)}")
        if a.device != b.device:
            raise ValueError(f"{name}{sfx} is on {a.device}, {ref_name}{sfx} on {b.device}")


def _check_links(U, psi, name="U"):
    """The links' site shape and device must be psi's (full-lattice fields)."""
    sites = tuple(psi.shape[:4])
    if tuple(U.shape[:4]) != sites:
        raise ValueError(f"{name} has site shape {tuple(U.shape[:4])}, the spinor has {sites}")
    dev = psi.device
    if U.device != dev:
        raise ValueError(f"{name} is on {U.device}, the spinor on {dev}")


def _check_workspace(ws, ref):
    _need_cuda(ws, "workspace")
    if ws.device != ref.device:
        raise ValueError(f"workspace is on {ws.device}, the fields on {ref.device}")


def _data_scale(psi):
    if isinstance(psi, F16Spinor):
        return psi.codes, psi.scale
    return psi, None


def _empty_like(psi):
    if isinstance(psi, F16Spinor):
        return F16Spinor.empty(psi.shape[:-2], psi.device)
    return torch.empty_like(psi)


def make_op(kind="hop", dag=False, mass=0.0, M5=1.8, mf=0.01, b5=1.0, c5=0.0) -> GridOp:
    op = GridOp()
    op.kind = _KIND[kind] if isinstance(kind, str) else int(kind)
    op.dag = int(bool(dag))
    op.mass, op.M5, op.mf = float(mass), float(M5), float(mf)
    op.b5, op.c5 = float(b5), float(c5)
    return op


def dhop(U, psi, kind="hop", dag=False, mass=0.0, M5=1.8, mf=0.01, out=None):
    """Apply H (kind "hop"), the Wilson D ("wilson") or the domain-wall M ("dwf"), or an adjoint."""
    prec = spinor_prec(psi)
    fmt = link_format(U, prec)
    g = geom_of(psi)
    _check_links(U, psi)
    if out is None:
        out = _empty_like(psi)
    else:
        _check_like(out, psi, "out")
    pd, ps = _data_scale(psi)
    od, os_ = _data_scale(out)
    op = make_op(kind, dag, mass, M5, mf)
    check(load().grid_dhop(_ptr(U), _ptr(pd), _ptr(ps), _ptr(od), _ptr(os_), ctypes.byref(g), ctypes.byref(op),
                           prec, fmt, _stream(pd.device)))
    return out


def wilson(U, psi, mass, dag=False, out=None):
    return dhop(U, psi, "wilson", dag=dag, mass=mass, out=out)


def dwf(U, psi, M5, mf, dag=False, out=None):
    return dhop(U, psi, "dwf", dag=dag, M5=M5, mf=mf, out=out)


def mobius(U, psi, M5, mf, b5, c5, dag=False, out=None, tmp=None):
    """Moebius domain-wall M psi (or M^dagger psi), M = D_W (b5 + c5 S) + 1 - S; see include/grid_mi.h."""
    prec = spinor_prec(psi)
    fmt = link_format(U, prec)
    g = geom_of(psi)
    _check_links(U, psi)
    for t, n in ((out, "out"), (tmp, "tmp")):
        if t is not None:
            _check_like(t, psi, n)
    out = _empty_like(psi) if out is None else out
    tmp = _empty_like(psi) if tmp is None else tmp
    pd, ps = _data_scale(psi)
    od, os_ = _data_scale(out)
    td, ts = _data_scale(tmp)
    op = make_op("mobius", dag, 0.0, M5, mf, b5, c5)
    check(load().grid_mobius(_ptr(U), _ptr(pd), _ptr(ps), _ptr(od), _ptr(os_), _ptr(td), _ptr(ts), ctypes.byref(g),
                             ctypes.byref(op), prec, fmt, _stream(pd.device)))
    return out


def dwf_mdag_m(U, psi, M5, mf, out=None, tmp=None):
    """M^dagger M psi for the domain-wall operator."""
    prec = spinor_prec(psi)
    fmt = link_format(U, prec)
    g = geom_of(psi)
    _check_links(U, psi)
    for t, n in ((out, "out"), (tmp, "tmp")):
        if t is not None:
            _check_like(t, psi, n)
    out = _empty_like(psi) if out is None else out
    tmp = _empty_like(psi) if tmp is None else tmp
    pd, ps = _data_scale(psi)
    od, os_ = _data_scale(out)
    td, ts = _data_scale(tmp)
    check(load().grid_dwf_mdag_m(_ptr(U), _ptr(pd), _ptr(ps), _ptr(od), _ptr(os_), _ptr(td), _ptr(ts),
                                 ctypes.byref(g), float(M5), float(mf), prec, fmt, _stream(pd.device)))
    return out


def dwf_mdag_m_noalloc(U, psi, M5, mf, out):
    """M^dagger M psi into the caller's out with no device allocation by the library (M psi goes to
    its static 64 MiB scratch; larger fields are rejected). Calls overlapping on one device race."""
    prec = spinor_prec(psi)
    fmt = link_format(U, prec)
    g = geom_of(psi)
    _check_links(U, psi)
    _check_like(out, psi, "out")
    pd, ps = _data_scale(psi)
    od, os_ = _data_scale(out)
    check(load().grid_dwf_mdag_m_noalloc(_ptr(U), _ptr(pd), _ptr(ps), _ptr(od), _ptr(os_), ctypes.byref(g),
                                         float(M5), float(mf), prec, fmt, _stream(pd.device)))
    return out


def cg_params(tol=1e-10, maxiter=20000, sloppy="f64", link_fmt="L18", delta=0.1, check_every=10,
              graph=False) -> GridCgParams:
    p = GridCgParams()
    p.tol, p.maxiter = float(tol), int(maxiter)
    p.sloppy_prec = _PREC[sloppy] if isinstance(sloppy, str) else int(sloppy)
    p.link_fmt = _FMT[link_fmt] if isinstance(link_fmt, str) else int(link_fmt)
    p.delta, p.check_every = float(delta), int(check_every)
    p.graph = 1 if graph else 0
    return p


def cg_workspace_bytes(b, **params) -> int:
    g = geom_of(b)
    p = cg_params(**params)
    return int(load().grid_cg_workspace_bytes(ctypes.byref(g), ctypes.byref(p)))


def cg(U, b, kind="dwf", mass=0.0, M5=1.8, mf=0.01, x0=None, workspace=None, raise_on_fail=True, b5=1.0, c5=0.0,
       **params):
    """Solve Op^dagger Op x = b (Op = D for kind "wilson", M for "dwf", M_mob for "mobius"); FP64 U, b, x.

    ``params``: tol, maxiter, sloppy ("f64" | "f32" | "f16s"), link_fmt ("L18" | "L12"), delta,
    check_every. Returns (x, stats dict). Synchronous.
    """
    if spinor_prec(b) != GRID_F64 or link_format(U, GRID_F64) != GRID_L18:
        raise TypeError("cg takes complex128 b and complex128 18-real links")
    g = geom_of(b)
    _check_links(U, b)
    if x0 is not None:
        _check_like(x0, b, "x0", "b")
    p = cg_params(**params)
    need = int(load().grid_cg_workspace_bytes(ctypes.byref(g), ctypes.byref(p)))
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=b.device)
    else:
        _check_workspace(workspace, b)
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    op = make_op(kind, False, mass, M5, mf, b5, c5)
    st = GridCgStats()
    rc = load().grid_cg(_ptr(U), _ptr(b), _ptr(x), ctypes.byref(g), ctypes.byref(op), ctypes.byref(p),
                        _ptr(workspace), ctypes.c_size_t(workspace.numel()), ctypes.byref(st), _stream(b.device))
    stats = {"iterations": st.iterations, "reliable_updates": st.reliable_updates, "converged": bool(st.converged),
             "true_residual": st.true_residual, "seconds": st.seconds, "status": rc}
    if rc != 0 and raise_on_fail:
        check(rc)
    return x, stats


def pseudofermion_action(U, phi, kind="wilson", mass=0.1, M5=1.8, mf=0.01, x0=None, grad_scale=1.0, want_S=True,
                         want_U=False, force=False, want_phi=False, workspace=None, raise_on_fail=True, b5=1.0,
                         c5=0.0, **params):
    """Two-flavour pseudofermion action S = Re phi^dagger (Op^dagger Op)^-1 phi (Op = D, the Shamir
    M or the Moebius M with b5, c5; FP64).

    Returns (S, X, dS_dU, dS_dphi, stats): S a float (None unless want_S), X the solution, and the
    gradients scaled by grad_scale (None unless asked for); force=True gives the su(3) projection
    of dS/dU. Every value is computed by the library (grid_pseudofermion_action). Synchronous.
    """
    if spinor_prec(phi) != GRID_F64 or link_format(U, GRID_F64) != GRID_L18:
        raise TypeError("pseudofermion_action takes complex128 phi and complex128 18-real links")
    g = geom_of(phi)
    _check_links(U, phi)
    if x0 is not None:
        _check_like(x0, phi, "x0", "phi")
    p = cg_params(**params)
    need = int(load().grid_pseudofermion_workspace_bytes(ctypes.byref(g), ctypes.byref(p)))
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=phi.device)
    else:
        _check_workspace(workspace, phi)
    X = torch.zeros_like(phi) if x0 is None else x0.clone()
    gU = torch.empty(tuple(phi.shape[:4]) + (4, 3, 3), dtype=torch.complex128, device=phi.device) if want_U else None
    gphi = torch.empty_like(phi) if want_phi else None
    op = make_op(kind, False, mass, M5, mf, b5, c5)
    S = ctypes.c_double(0.0)
    st = GridCgStats()
    rc = load().grid_pseudofermion_action(_ptr(U), _ptr(phi), _ptr(X), ctypes.byref(g), ctypes.byref(op),
                                          ctypes.byref(p), float(grad_scale), ctypes.byref(S) if want_S else None,
                                          _ptr(gU), int(bool(force)), _ptr(gphi), _ptr(workspace),
                                          ctypes.c_size_t(workspace.numel()), ctypes.byref(st), _stream(phi.device))
    stats = {"iterations": st.iterations, "reliable_updates": st.reliable_updates, "converged": bool(st.converged),
             "true_residual": st.true_residual, "seconds": st.seconds, "status": rc}
    if rc != 0 and raise_on_fail:
        check(rc)
    return (S.value if want_S else None), X, gU, gphi, stats


def _geom_cb(U, psi) -> GridGeom:
    """Geometry of a checkerboard field (x extent Lx / 2) checked against full-lattice links."""
    g = geom_of(psi)
    g.dims[0] = 2 * g.dims[0]
    if tuple(U.shape[:4]) != (g.dims[3], g.dims[2], g.dims[1], g.dims[0]):
        raise ValueError(f"checkerboard field {tuple(psi.shape)} does not match links {tuple(U.shape)}")
    return g


def dhop_cb(U, psi, out_parity, kind="hop", y=None, beta=1.0, dag=False, mass=0.0, M5=1.8, mf=0.01, out=None):
    """Checkerboard hopping term: out (parity p) = beta H psi (parity 1 - p) + Diag_kind(y).

    Checkerboard fields have shape (Lt, Lz, Ly, Lx/2[, Ls], 4, 3); see include/grid_mi.h.
    """
    prec = spinor_prec(psi)
    fmt = link_format(U, prec)
    g = _geom_cb(U, psi)
    if U.device != psi.device:
        raise ValueError(f"U is on {U.device}, psi on {psi.device}")
    if out is None:
        out = _empty_like(psi)
    else:
        _check_like(out, psi, "out")
    if y is not None:
        _check_like(y, psi, "y")
    pd, ps = _data_scale(psi)
    yd, ys = _data_scale(y) if y is not None else (None, None)
    od, os_ = _data_scale(out)
    op = make_op(kind, dag, mass, M5, mf)
    check(load().grid_dhop_cb(_ptr(U), _ptr(pd), _ptr(ps), _ptr(yd), _ptr(ys), _ptr(od), _ptr(os_), ctypes.byref(g),
                              ctypes.byref(op), int(out_parity), float(beta), prec, fmt, _stream(pd.device)))
    return out


def m5inv(psi, M5, mf, dag=False, out=None):
    """Inverse of the domain-wall fifth-dimension operator on a full or checkerboard 5D field."""
    prec = spinor_prec(psi)
    shape = psi.shape
    if len(shape) != 7:
        raise ValueError("m5inv takes a 5D field (..., Ls, 4, 3)")
    n4 = int(shape[0]) * int(shape[1]) * int(shape[2]) * int(shape[3])
    if out is not None:
        _check_like(out, psi, "out")
    out = _empty_like(psi) if out is None else out
    pd, ps = _data_scale(psi)
    od, os_ = _data_scale(out)
    check(load().grid_m5inv(_ptr(pd), _ptr(ps), _ptr(od), _ptr(os_), n4, int(shape[4]), float(M5), float(mf),
                            int(bool(dag)), prec, _stream(pd.device)))
    return out


def solve_eo_workspace_bytes(b, **params) -> int:
    g = geom_of(b)
    p = cg_params(**params)
    return int(load().grid_solve_eo_workspace_bytes(ctypes.byref(g), ctypes.byref(p)))


def solve_eo(U, b, kind="dwf", mass=0.0, M5=1.8, mf=0.01, x0=None, workspace=None, raise_on_fail=True, b5=1.0, c5=0.0,
             **params):
    """Solve Op x = b (Op = D, the Shamir M or the Moebius M with b5, c5) with even-odd
    preconditioned CG; FP64 full-lattice U, b, x.

    Returns (x, stats); stats["true_residual"] is |b - Op x| / |b|. Synchronous.
    """
    if spinor_prec(b) != GRID_F64 or link_format(U, GRID_F64) != GRID_L18:
        raise TypeError("solve_eo takes complex128 b and complex128 18-real links")
    g = geom_of(b)
    _check_links(U, b)
    if x0 is not None:
        _check_like(x0, b, "x0", "b")
    p = cg_params(**params)
    need = int(load().grid_solve_eo_workspace_bytes(ctypes.byref(g), ctypes.byref(p)))
    if need == 0:
        raise ValueError("invalid geometry or parameters for solve_eo (every extent must be even)")
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=b.device)
    else:
        _check_workspace(workspace, b)
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    op = make_op(kind, False, mass, M5, mf, b5, c5)
    st = GridCgStats()
    rc = load().grid_solve_eo(_ptr(U), _ptr(b), _ptr(x), ctypes.byref(g), ctypes.byref(op), ctypes.byref(p),
                              _ptr(workspace), ctypes.c_size_t(workspace.numel()), ctypes.byref(st), _stream(b.device))
    stats = {"iterations": st.iterations, "reliable_updates": st.reliable_updates, "converged": bool(st.converged),
             "true_residual": st.true_residual, "seconds": st.seconds, "status": rc}
    if rc != 0 and raise_on_fail:
        check(rc)
    return x, stats


def _geom_links(U, Ls=1) -> GridGeom:
    if U.dtype != torch.complex128 or tuple(U.shape[4:]) != (4, 3, 3):
        raise TypeError("HMC takes complex128 links (Lt, Lz, Ly, Lx, 4, 3, 3)")
    _need_cuda(U, "U")
    g = GridGeom()
    g.dims[:] = [int(U.shape[3]), int(U.shape[2]), int(U.shape[1]), int(U.shape[0])]
    g.Ls = int(Ls)
    return g


def gauge_force(U, beta, out=None):
    """su(3) force of the Wilson plaquette action on every link."""
    g = _geom_links(U)
    if out is not None:
        _check_like(out, U, "out", "U")
    F = torch.empty_like(U) if out is None else out
    check(load().grid_gauge_force(_ptr(U), _ptr(F), ctypes.byref(g), float(beta), _stream(U.device)))
    return F


def link_exp(U, P, eps):
    """U <- exp(eps P) U in place (returns U)."""
    _geom_links(U)
    _check_like(P, U, "P", "U")
    check(load().grid_link_exp(_ptr(U), _ptr(P), float(eps), U.numel() // 9, _stream(U.device)))
    return U


def md_params(beta, eps=0.1, n_steps=10, kind="dwf", mass=0.0, M5=1.8, mf=0.01, integrator="leapfrog",
              n_inner=1, b5=1.0, c5=0.0, **cg) -> GridMdParams:
    p = GridMdParams()
    p.beta, p.eps, p.n_steps = float(beta), float(eps), int(n_steps)
    p.integrator = {"leapfrog": 0, "omelyan": 1, "force_gradient": 2}[integrator]
    p.n_inner = int(n_inner)
    p.fermion = make_op(kind, False, mass, M5, mf, b5, c5)
    p.cg = cg_params(**cg)
    return p


def _md_setup(U, phi, workspace, p, P=None):
    Ls = 1
    if phi is not None:
        if spinor_prec(phi) != GRID_F64:
            raise TypeError("phi must be complex128")
        Ls = geom_of(phi).Ls
        _check_links(U, phi)
    g = _geom_links(U, Ls)
    if P is not None:
        _check_like(P, U, "P", "U")
    if workspace is not None:
        _check_workspace(workspace, U)
    need = int(load().grid_md_workspace_bytes(ctypes.byref(g), ctypes.byref(p)))
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=U.device)
    return g, workspace


def md_leapfrog(U, P, beta, eps, n_steps, phi=None, workspace=None, **kw):
    """Molecular dynamics of (U, P) in place (integrator="leapfrog" | "omelyan" | "force_gradient" in
    kw); phi adds the pseudofermion force. Returns stats."""
    p = md_params(beta, eps, n_steps, **kw)
    g, workspace = _md_setup(U, phi, workspace, p, P)
    st = GridMdStats()
    check(load().grid_md_leapfrog(_ptr(U), _ptr(P), _ptr(phi), ctypes.byref(g), ctypes.byref(p), _ptr(workspace),
                                  ctypes.c_size_t(workspace.numel()), ctypes.byref(st), _stream(U.device)))
    return {"solves": st.solves, "cg_iterations": st.cg_iterations, "failed_solves": st.failed_solves,
            "seconds": st.seconds}


def hmc_energy(U, P, beta, phi=None, workspace=None, **kw):
    """{"K", "S_G", "S_F", "H"} in FP64."""
    p = md_params(beta, **kw)
    g, workspace = _md_setup(U, phi, workspace, p, P)
    st = GridMdStats()
    e = (ctypes.c_double * 4)()
    check(load().grid_hmc_energy(_ptr(U), _ptr(P), _ptr(phi), ctypes.byref(g), ctypes.byref(p), _ptr(workspace),
                                 ctypes.c_size_t(workspace.numel()), e, ctypes.byref(st), _stream(U.device)))
    return {"K": e[0], "S_G": e[1], "S_F": e[2], "H": e[3]}


def dhop_backward(U, psi, grad_out, kind="hop", dag=False, mass=0.0, M5=1.8, mf=0.01, want_psi=True, want_U=True,
                  force=False):
    """Gradients of L = Re <grad_out, Op psi>: (Op^dagger grad_out, dL/dU or its su(3) force)."""
    prec = spinor_prec(psi)
    if prec == GRID_F16S or spinor_prec(grad_out) != prec:
        raise TypeError("dhop_backward takes FP64 or FP32 spinors of one precision")
    if link_format(U, prec) != GRID_L18:
        raise TypeError("dhop_backward takes 18-real links")
    g = geom_of(psi)
    _check_links(U, psi)
    _check_like(grad_out, psi, "grad_out")
    gp = torch.empty_like(psi) if want_psi else None
    gu = torch.empty(tuple(psi.shape[:4]) + (4, 3, 3), dtype=psi.dtype, device=psi.device) if want_U else None
    op = make_op(kind, dag, mass, M5, mf)
    check(load().grid_dhop_backward(_ptr(U), _ptr(psi), _ptr(grad_out), _ptr(gp), _ptr(gu), ctypes.byref(g),
                                    ctypes.byref(op), prec, int(bool(force)), _stream(psi.device)))
    return gp, gu


def convert_spinor(x, to: str):
    """Change a spinor's storage precision: to = "f64" | "f32" | "f16s"."""
    src_prec = spinor_prec(x)
    dst_prec = _PREC[to]
    xd, xs = _data_scale(x)
    site_shape = x.shape[:-2]
    n = 1
    for d in site_shape:
        n *= int(d)
    if dst_prec == GRID_F16S:
        out = F16Spinor.empty(site_shape, xd.device)
    else:
        out = torch.empty(tuple(site_shape) + (4, 3), dtype=torch.complex128 if dst_prec == GRID_F64 else torch.complex64,
                          device=xd.device)
    od, os_ = _data_scale(out)
    check(load().grid_convert_spinor(_ptr(xd), src_prec, _ptr(xs), _ptr(od), dst_prec, _ptr(os_), n, _stream(xd.device)))
    return out


def convert_links(U, prec="f32", fmt="L18", reunitarise=False):
    """Narrow / compress / reunitarise FP64 18-real links."""
    if link_format(U, GRID_F64) != GRID_L18:
        raise TypeError("convert_links takes complex128 18-real links")
    dst_prec, dst_fmt = _PREC[prec], _FMT[fmt]
    rows = 3 if dst_fmt == GRID_L18 else 2
    lead = tuple(U.shape[:5])
    if dst_prec == GRID_F16S:
        out = torch.empty(lead + (rows, 3, 2), dtype=torch.float16, device=U.device)
    else:
        out = torch.empty(lead + (rows, 3), dtype=torch.complex128 if dst_prec == GRID_F64 else torch.complex64,
                          device=U.device)
    n = U.numel() // 9
    check(load().grid_convert_links(_ptr(U), _ptr(out), dst_prec, dst_fmt, int(bool(reunitarise)), n,
                                    _stream(U.device)))
    return out


def version() -> int:
    return int(load().grid_version())


# --------------------------------------------------------------------------------------------
# Generic coarse stencil and two-level multigrid for the Wilson operator (FP64).
# Coarse fields are (Lct, Lcz, Lcy, Lcx, N) complex128; the coarse operator is
# (Lct, Lcz, Lcy, Lcx, 9, N, N) with A[..., d, j, i] = element (row i, column j) of A_d.
# --------------------------------------------------------------------------------------------

def mg_params(block=(2, 2, 2, 2), nvec=6, setup_rounds=2, setup_iters=8, coarse_iters=40, coarse_tol=0.05,
              smooth_iters=2, restart=8, maxiter=500, tol=1e-10, graph=True, setup_prec="f64",
              cycle_prec="f64") -> GridMgParams:
    p = GridMgParams()
    for mu in range(4):
        p.block[mu] = int(block[mu])
    p.nvec, p.setup_rounds, p.setup_iters = int(nvec), int(setup_rounds), int(setup_iters)
    p.coarse_iters, p.coarse_tol, p.smooth_iters = int(coarse_iters), float(coarse_tol), int(smooth_iters)
    p.restart, p.maxiter, p.tol = int(restart), int(maxiter), float(tol)
    p.graph = 1 if graph else 0
    p.setup_prec = _PREC[setup_prec]
    p.cycle_prec = _PREC[cycle_prec]
    return p


def _coarse_shape(psi_or_U, block, N):
    shape = psi_or_U.shape if hasattr(psi_or_U, "shape") else psi_or_U
    lt, lz, ly, lx = shape[:4]
    bx, by, bz, bt = block
    return (lt // bt, lz // bz, ly // by, lx // bx, N)


def _mg_ws(U, p, workspace):
    g = geom_of_links(U)
    if workspace is not None:
        _check_workspace(workspace, U)
    need = int(load().grid_mg_workspace_bytes(ctypes.byref(g), ctypes.byref(p)))
    if need == 0:
        check(load().grid_mg_restrict(None, None, None, ctypes.byref(g), ctypes.byref(p), None))
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=U.device)
    return g, workspace


def _check_vecs(vecs, U):
    """Basis vectors (nvec, Lt, Lz, Ly, Lx, 4, 3) complex128 on U's lattice and device."""
    _need_cuda(vecs, "vecs")
    if vecs.dtype != torch.complex128 or vecs.dim() != 7 or tuple(vecs.shape[5:]) != (4, 3):
        raise ValueError("vecs must be complex128 (nvec, Lt, Lz, Ly, Lx, 4, 3)")
    if tuple(vecs.shape[1:5]) != tuple(U.shape[:4]) or vecs.device != U.device:
        raise ValueError(f"vecs {tuple(vecs.shape)} on {vecs.device} do not match U {tuple(U.shape)} on {U.device}")


def _check_coarse_op(A, U, block, N):
    _need_cuda(A, "A")
    want = _coarse_shape(U, block, N)[:4] + (9, N, N)
    if A.dtype != torch.complex128 or tuple(A.shape) != want or A.device != U.device:
        raise ValueError(f"A must be complex128 {want} on {U.device}")


def geom_of_links(U) -> GridGeom:
    _need_cuda(U, "U")
    if U.dtype != torch.complex128 or tuple(U.shape[4:]) != (4, 3, 3):
        raise TypeError("multigrid takes complex128 links (Lt, Lz, Ly, Lx, 4, 3, 3)")
    g = GridGeom()
    lt, lz, ly, lx = U.shape[:4]
    g.dims[:] = [lx, ly, lz, lt]
    g.Ls = 1
    return g


def coarse_stencil(A, v, dag=False, out=None):
    """out = A v (dag: A^dagger v) for a 9-point coarse stencil (see the layout above)."""
    _need_cuda(A, "A")
    _need_cuda(v, "v")
    N = int(v.shape[-1])
    if A.dtype != torch.complex128 or v.dtype != torch.complex128 or tuple(A.shape) != tuple(v.shape[:4]) + (9, N, N):
        raise ValueError("A must be complex128 (Lct, Lcz, Lcy, Lcx, 9, N, N) and v (Lct, Lcz, Lcy, Lcx, N)")
    out = torch.empty_like(v) if out is None else out
    lt, lz, ly, lx = v.shape[:4]
    cd = (ctypes.c_int * 4)(lx, ly, lz, lt)
    check(load().grid_coarse_stencil(_ptr(A), _ptr(v), _ptr(out), cd, N, int(bool(dag)), _stream(v.device)))
    return out


def mg_basis(U, vecs, mass, workspace=None, **params):
    """In place: near-null improvement of the caller's vecs (nvec, Lt, Lz, Ly, Lx, 4, 3) and blockwise
    Gram-Schmidt. Returns vecs."""
    p = mg_params(nvec=int(vecs.shape[0]), **params)
    _check_vecs(vecs, U)
    g, workspace = _mg_ws(U, p, workspace)
    op = make_op("wilson", False, mass)
    check(load().grid_mg_basis(_ptr(U), _ptr(vecs), ctypes.byref(g), ctypes.byref(op), ctypes.byref(p), _ptr(workspace),
                               ctypes.c_size_t(workspace.numel()), _stream(U.device)))
    return vecs


def mg_coarse_op(U, vecs, mass, workspace=None, out=None, **params):
    """Galerkin coarse operator R D P as a (Lct, Lcz, Lcy, Lcx, 9, N, N) complex128 tensor."""
    nvec = int(vecs.shape[0])
    p = mg_params(nvec=nvec, **params)
    _check_vecs(vecs, U)
    g, workspace = _mg_ws(U, p, workspace)
    cs = _coarse_shape(U, p.block, 2 * nvec)
    if out is not None:
        _check_coarse_op(out, U, p.block, 2 * nvec)
    A = torch.empty(cs[:4] + (9, 2 * nvec, 2 * nvec), dtype=torch.complex128, device=U.device) if out is None else out
    op = make_op("wilson", False, mass)
    check(load().grid_mg_coarse_op(_ptr(U), _ptr(vecs), _ptr(A), ctypes.byref(g), ctypes.byref(op), ctypes.byref(p),
                                   _ptr(workspace), ctypes.c_size_t(workspace.numel()), _stream(U.device)))
    return A


def mg_restrict(vecs, psi, block):
    nvec = int(vecs.shape[0])
    p = mg_params(block=block, nvec=nvec)
    if spinor_prec(psi) != GRID_F64:
        raise TypeError("mg_restrict takes a complex128 psi")
    g = geom_of(psi)
    _check_vecs(vecs, psi)
    vc = torch.empty(_coarse_shape(psi, block, 2 * nvec), dtype=torch.complex128, device=psi.device)
    check(load().grid_mg_restrict(_ptr(vecs), _ptr(psi), _ptr(vc), ctypes.byref(g), ctypes.byref(p),
                                  _stream(psi.device)))
    return vc


def mg_prolong(vecs, vc, block):
    nvec = int(vecs.shape[0])
    p = mg_params(block=block, nvec=nvec)
    _need_cuda(vecs, "vecs")
    _need_cuda(vc, "vc")
    want = _coarse_shape(vecs.shape[1:], block, 2 * nvec)
    if vc.dtype != torch.complex128 or tuple(vc.shape) != want or vc.device != vecs.device:
        raise ValueError(f"vc must be complex128 {want} on {vecs.device}")
    psi = torch.empty(tuple(vecs.shape[1:]), dtype=torch.complex128, device=vecs.device)
    g = geom_of(psi)
    check(load().grid_mg_prolong(_ptr(vecs), _ptr(vc), _ptr(psi), ctypes.byref(g), ctypes.byref(p),
                                 _stream(psi.device)))
    return psi


def _mg_solve_call(fn, U, vecs, A, b, mass, x0, workspace, raise_on_fail, params):
    nvec = int(vecs.shape[0])
    p = mg_params(nvec=nvec, **params)
    _check_vecs(vecs, U)
    _check_coarse_op(A, U, p.block, 2 * nvec)
    if spinor_prec(b) != GRID_F64:
        raise TypeError("the multigrid solvers take a complex128 b")
    _check_links(U, b)
    if x0 is not None:
        _check_like(x0, b, "x0", "b")
    g, workspace = _mg_ws(U, p, workspace)
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    op = make_op("wilson", False, mass)
    st = GridCgStats()
    rc = getattr(load(), fn)(_ptr(U), _ptr(vecs), _ptr(A), _ptr(b), _ptr(x), ctypes.byref(g), ctypes.byref(op),
                             ctypes.byref(p), _ptr(workspace), ctypes.c_size_t(workspace.numel()), ctypes.byref(st),
                             _stream(b.device))
    stats = {"iterations": st.iterations, "restarts": st.reliable_updates, "converged": bool(st.converged),
             "true_residual": st.true_residual, "seconds": st.seconds, "status": rc}
    if rc != 0 and raise_on_fail:
        check(rc)
    return x, stats


def mg_solve(U, vecs, A, b, mass, x0=None, workspace=None, raise_on_fail=True, **params):
    """D x = b by multigrid-preconditioned flexible GCR. Returns (x, stats)."""
    return _mg_solve_call("grid_mg_solve", U, vecs, A, b, mass, x0, workspace, raise_on_fail, params)


def mg_pcg(U, vecs, A, b, mass, x0=None, workspace=None, raise_on_fail=True, **params):
    """D x = b by multigrid-preconditioned flexible CG on the normal equations. Returns (x, stats)."""
    return _mg_solve_call("grid_mg_pcg", U, vecs, A, b, mass, x0, workspace, raise_on_fail, params)


def mg_workspace_bytes(U, **params) -> int:
    p = mg_params(**params)
    g = geom_of_links(U)
    return int(load().grid_mg_workspace_bytes(ctypes.byref(g), ctypes.byref(p)))
