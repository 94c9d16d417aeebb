"""ctypes binding of libgrid_mi.so (the C ABI declared in include/grid_mi.h).

The library is built in-tree by ``paper_1512_03487_amd.build``. Loading fails loudly when it is
missing: there is no CPU fallback for any entry point.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrid_mi.so")

GRID_OK, GRID_EINVAL, GRID_ESHAPE, GRID_EDTYPE, GRID_EALIGN = 0, -1, -2, -3, -4
GRID_EHIP, GRID_ENOCONV, GRID_EBREAKDOWN, GRID_ESPACE = -5, -6, -7, -8
GRID_F64, GRID_F32, GRID_F16S = 0, 1, 2
GRID_L18, GRID_L12 = 0, 1
GRID_HOP, GRID_WILSON, GRID_DWF, GRID_MOBIUS = 0, 1, 2, 3
GRID_LEAPFROG, GRID_OMELYAN, GRID_FORCE_GRADIENT = 0, 1, 2

#: every symbol include/grid_mi.h declares
EXPORTS = ("grid_dhop", "grid_mobius", "grid_dwf_mdag_m", "grid_dwf_mdag_m_noalloc", "grid_cg_workspace_bytes", "grid_cg", "grid_dhop_backward",
           "grid_dhop_cb", "grid_m5inv", "grid_solve_eo_workspace_bytes", "grid_solve_eo",
           "grid_md_workspace_bytes", "grid_gauge_force", "grid_link_exp", "grid_md_leapfrog", "grid_hmc_energy",
           "grid_pseudofermion_workspace_bytes", "grid_pseudofermion_action",
           "grid_convert_spinor", "grid_convert_links", "grid_coarse_stencil", "grid_mg_workspace_bytes",
           "grid_mg_basis", "grid_mg_coarse_op", "grid_mg_restrict", "grid_mg_prolong", "grid_mg_solve",
           "grid_mg_pcg", "grid_last_error", "grid_version")


class GridGeom(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("Ls", ctypes.c_int)]


class GridOp(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("dag", ctypes.c_int), ("mass", ctypes.c_double),
                ("M5", ctypes.c_double), ("mf", ctypes.c_double), ("b5", ctypes.c_double), ("c5", ctypes.c_double)]


class GridCgParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int), ("sloppy_prec", ctypes.c_int),
                ("link_fmt", ctypes.c_int), ("delta", ctypes.c_double), ("check_every", ctypes.c_int),
                ("graph", ctypes.c_int)]


class GridCgStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("reliable_updates", ctypes.c_int), ("converged", ctypes.c_int),
                ("true_residual", ctypes.c_double), ("seconds", ctypes.c_double)]


class GridMdParams(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("eps", ctypes.c_double), ("n_steps", ctypes.c_int), ("fermion", GridOp),
                ("cg", GridCgParams), ("integrator", ctypes.c_int), ("n_inner", ctypes.c_int)]


class GridMdStats(ctypes.Structure):
    _fields_ = [("solves", ctypes.c_int), ("cg_iterations", ctypes.c_int), ("failed_solves", ctypes.c_int),
                ("seconds", ctypes.c_double)]


class GridMgParams(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int * 4), ("nvec", ctypes.c_int), ("setup_rounds", ctypes.c_int),
                ("setup_iters", ctypes.c_int), ("coarse_iters", ctypes.c_int), ("coarse_tol", ctypes.c_double),
                ("smooth_iters", ctypes.c_int), ("restart", ctypes.c_int), ("maxiter", ctypes.c_int),
                ("tol", ctypes.c_double), ("graph", ctypes.c_int), ("setup_prec", ctypes.c_int),
                ("cycle_prec", ctypes.c_int)]


class GridError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"grid_mi error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libgrid_mi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1512_03487_amd.build` "
                          "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.grid_dhop.argtypes = [P, P, P, P, P, ctypes.POINTER(GridGeom), ctypes.POINTER(GridOp), I, I, P]
    lib.grid_dhop.restype = I
    lib.grid_mobius.argtypes = [P, P, P, P, P, P, P, ctypes.POINTER(GridGeom), ctypes.POINTER(GridOp), I, I, P]
    lib.grid_mobius.restype = I
    lib.grid_dwf_mdag_m.argtypes = [P, P, P, P, P, P, P, ctypes.POINTER(GridGeom), D, D, I, I, P]
    lib.grid_dwf_mdag_m.restype = I
    lib.grid_dwf_mdag_m_noalloc.argtypes = [P, P, P, P, P, ctypes.POINTER(GridGeom), D, D, I, I, P]
    lib.grid_dwf_mdag_m_noalloc.restype = I
    lib.grid_cg_workspace_bytes.argtypes = [ctypes.POINTER(GridGeom), ctypes.POINTER(GridCgParams)]
    lib.grid_cg_workspace_bytes.restype = ctypes.c_size_t
    lib.grid_cg.argtypes = [P, P, P, ctypes.POINTER(GridGeom), ctypes.POINTER(GridOp), ctypes.POINTER(GridCgParams),
                            P, ctypes.c_size_t, ctypes.POINTER(GridCgStats), P]
    lib.grid_cg.restype = I
    lib.grid_dhop_backward.argtypes = [P, P, P, P, P, ctypes.POINTER(GridGeom), ctypes.POINTER(GridOp), I, I, P]
    lib.grid_dhop_backward.restype = I
    lib.grid_dhop_cb.argtypes = [P, P, P, P, P, P, P, ctypes.POINTER(GridGeom), ctypes.POINTER(GridOp), I, D, I, I, P]
    lib.grid_dhop_cb.restype = I
    lib.grid_m5inv.argtypes = [P, P, P, P, ctypes.c_long, I, D, D, I, I, P]
    lib.grid_m5inv.restype = I
    lib.grid_solve_eo_workspace_bytes.argtypes = [ctypes.POINTER(GridGeom), ctypes.POINTER(GridCgParams)]
    lib.grid_solve_eo_workspace_bytes.restype = ctypes.c_size_t
    lib.grid_solve_eo.argtypes = [P, P, P, ctypes.POINTER(GridGeom), ctypes.POINTER(GridOp),
                                  ctypes.POINTER(GridCgParams), P, ctypes.c_size_t, ctypes.POINTER(GridCgStats), P]
    lib.grid_solve_eo.restype = I
    lib.grid_md_workspace_bytes.argtypes = [ctypes.POINTER(GridGeom), ctypes.POINTER(GridMdParams)]
    lib.grid_md_workspace_bytes.restype = ctypes.c_size_t
    lib.grid_gauge_force.argtypes = [P, P, ctypes.POINTER(GridGeom), D, P]
    lib.grid_gauge_force.restype = I
    lib.grid_link_exp.argtypes = [P, P, D, ctypes.c_long, P]
    lib.grid_link_exp.restype = I
    lib.grid_md_leapfrog.argtypes = [P, P, P, ctypes.POINTER(GridGeom), ctypes.POINTER(GridMdParams), P,
                                     ctypes.c_size_t, ctypes.POINTER(GridMdStats), P]
    lib.grid_md_leapfrog.restype = I
    lib.grid_hmc_energy.argtypes = [P, P, P, ctypes.POINTER(GridGeom), ctypes.POINTER(GridMdParams), P,
                                    ctypes.c_size_t, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(GridMdStats), P]
    lib.grid_hmc_energy.restype = I
    lib.grid_pseudofermion_workspace_bytes.argtypes = [ctypes.POINTER(GridGeom), ctypes.POINTER(GridCgParams)]
    lib.grid_pseudofermion_workspace_bytes.restype = ctypes.c_size_t
    lib.grid_pseudofermion_action.argtypes = [P, P, P, ctypes.POINTER(GridGeom), ctypes.POINTER(GridOp),
                                              ctypes.POINTER(GridCgParams), D, ctypes.POINTER(ctypes.c_double), P, I,
                                              P, P, ctypes.c_size_t, ctypes.POINTER(GridCgStats), P]
    lib.grid_pseudofermion_action.restype = I
    lib.grid_convert_spinor.argtypes = [P, I, P, P, I, P, ctypes.c_long, P]
    lib.grid_convert_spinor.restype = I
    lib.grid_convert_links.argtypes = [P, P, I, I, I, ctypes.c_long, P]
    lib.grid_convert_links.restype = I
    G, MP = ctypes.POINTER(GridGeom), ctypes.POINTER(GridMgParams)
    lib.grid_coarse_stencil.argtypes = [P, P, P, ctypes.POINTER(ctypes.c_int), I, I, P]
    lib.grid_coarse_stencil.restype = I
    lib.grid_mg_workspace_bytes.argtypes = [G, MP]
    lib.grid_mg_workspace_bytes.restype = ctypes.c_size_t
    lib.grid_mg_basis.argtypes = [P, P, G, ctypes.POINTER(GridOp), MP, P, ctypes.c_size_t, P]
    lib.grid_mg_basis.restype = I
    lib.grid_mg_coarse_op.argtypes = [P, P, P, G, ctypes.POINTER(GridOp), MP, P, ctypes.c_size_t, P]
    lib.grid_mg_coarse_op.restype = I
    lib.grid_mg_restrict.argtypes = [P, P, P, G, MP, P]
    lib.grid_mg_restrict.restype = I
    lib.grid_mg_prolong.argtypes = [P, P, P, G, MP, P]
    lib.grid_mg_prolong.restype = I
    lib.grid_mg_solve.argtypes = [P, P, P, P, P, G, ctypes.POINTER(GridOp), MP, P, ctypes.c_size_t,
                                  ctypes.POINTER(GridCgStats), P]
    lib.grid_mg_solve.restype = I
    lib.grid_mg_pcg.argtypes = lib.grid_mg_solve.argtypes
    lib.grid_mg_pcg.restype = I
    lib.grid_last_error.argtypes = []
    lib.grid_last_error.restype = ctypes.c_char_p
    lib.grid_version.argtypes = []
    lib.grid_version.restype = I
    _lib = lib
    return lib


def check(rc: int) -> int:
    """Raise GridError for a negative status (GRID_ENOCONV / GRID_EBREAKDOWN included)."""
    if rc != GRID_OK:
        raise GridError(rc, load().grid_last_error().decode())
    return rc


def last_error() -> str:
    return load().grid_last_error().decode()
