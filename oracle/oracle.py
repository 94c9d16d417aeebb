"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Python face of ``oracle.c`` (loaded with ctypes) plus the few oracle pieces that are plain numpy:
the FP16 storage codec, 12-real link compression and FP64 reunitarisation. Only the test-suite,
the smoke check and the benchmark's CPU-baseline leg may import this module. The product library
(``paper_1512_03487_amd``) never imports it, and it imports nothing from the product.

Every function evaluates its definition directly; the definitions are stated in ``oracle.c`` and in
the docstrings below. Arrays follow the site-major layout of ``paper_1512_03487_amd.fields``
(x fastest among sites, the per-site tensor innermost); all arithmetic is complex128.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile oracle.c with gcc into oracle/liboracle.so (always recompiles)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           _SRC, "-o", _LIB_PATH + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    lib.oracle_gamma.argtypes = [ctypes.c_int, P]
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_hop.argtypes = [P, P, P, P, ctypes.c_int, ctypes.c_int]
    lib.oracle_wilson.argtypes = [P, P, P, P, ctypes.c_double, ctypes.c_int]
    lib.oracle_dwf.argtypes = [P, P, P, P, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.oracle_normal.argtypes = [P, P, P, P, P, P]
    lib.oracle_cg.argtypes = [P, P, P, P, P, ctypes.c_double, ctypes.c_int, P]
    lib.oracle_cg.restype = ctypes.c_int
    lib.oracle_link_grad.argtypes = [P, P, P, P, ctypes.c_int, ctypes.c_double, ctypes.c_int]
    lib.oracle_force.argtypes = [P, P, P, ctypes.c_long]
    lib.oracle_sites.argtypes = [P, P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_int, P, ctypes.c_long]
    _lib = lib
    return lib


class _OpStruct(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("Ls", ctypes.c_int), ("mass", ctypes.c_double),
                ("M5", ctypes.c_double), ("mf", ctypes.c_double)]


@dataclass(frozen=True)
class Op:
    """Fermion operator: ``Op.wilson(mass)`` (D) or ``Op.dwf(Ls, M5, mf)`` (Shamir M)."""
    kind: int
    Ls: int = 1
    mass: float = 0.0
    M5: float = 0.0
    mf: float = 0.0

    @staticmethod
    def wilson(mass: float) -> "Op":
        return Op(kind=0, Ls=1, mass=float(mass))

    @staticmethod
    def dwf(Ls: int, M5: float, mf: float) -> "Op":
        return Op(kind=1, Ls=int(Ls), M5=float(M5), mf=float(mf))

    def _c(self):
        return _OpStruct(self.kind, self.Ls, self.mass, self.M5, self.mf)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(field) -> np.ndarray:
    lt, lz, ly, lx = field.shape[:4]
    return np.array([lx, ly, lz, lt], dtype=np.int32)


def _ls(psi) -> int:
    return 1 if psi.ndim == 6 else int(psi.shape[4])


def threads() -> int:
    """OpenMP threads the oracle runs with."""
    return int(_load().oracle_threads())


def gamma(which: int) -> np.ndarray:
    """Dirac matrix: which = 0..3 gives gamma_{which+1} (direction x, y, z, t), 4 gives gamma_5."""
    out = np.zeros((4, 4), dtype=np.complex128)
    _load().oracle_gamma(int(which), _ptr(out))
    return out


def hop(U, psi, dag: bool = False) -> np.ndarray:
    """H psi (or H^dagger psi) on a 4D or 5D spinor (same links on every fifth slice)."""
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    _load().oracle_hop(_ptr(U), _ptr(psi), _ptr(out), _ptr(_dims(psi)), _ls(psi), int(bool(dag)))
    return out


def wilson(U, psi, mass: float, dag: bool = False) -> np.ndarray:
    """D psi or D^dagger psi with D = (4 + m) - H/2."""
    U, psi = _c128(U), _c128(psi)
    if psi.ndim != 6:
        raise ValueError("Wilson operator takes a 4D spinor")
    out = np.empty_like(psi)
    _load().oracle_wilson(_ptr(U), _ptr(psi), _ptr(out), _ptr(_dims(psi)), float(mass), int(bool(dag)))
    return out


def dwf(U, psi, M5: float, mf: float, dag: bool = False) -> np.ndarray:
    """Shamir domain-wall M psi or M^dagger psi on a 5D spinor (Lt,Lz,Ly,Lx,Ls,4,3)."""
    U, psi = _c128(U), _c128(psi)
    if psi.ndim != 7:
        raise ValueError("domain-wall operator takes a 5D spinor")
    out = np.empty_like(psi)
    _load().oracle_dwf(_ptr(U), _ptr(psi), _ptr(out), _ptr(_dims(psi)), _ls(psi), float(M5),
                       float(mf), int(bool(dag)))
    return out


def apply(op: Op, U, psi, dag: bool = False) -> np.ndarray:
    if op.kind == 0:
        return wilson(U, psi, op.mass, dag)
    return dwf(U, psi, op.M5, op.mf, dag)


def sites(U, psi, idx, kind: str = "hop", dag: bool = False, mass: float = 0.0, M5: float = 0.0,
          mf: float = 0.0) -> np.ndarray:
    """The operator at selected sites only: idx are flat site indices (x * Ls + s for 5D).

    kind "hop" (H), "wilson" (D, 4D only) or "dwf" (M). Returns (len(idx), 4, 3) complex128.
    """
    U, psi = _c128(U), _c128(psi)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty((len(idx), 4, 3), dtype=np.complex128)
    k = {"hop": 0, "wilson": 1, "dwf": 2}[kind]
    _load().oracle_sites(_ptr(U), _ptr(psi), _ptr(out), _ptr(_dims(psi)), _ls(psi), k, float(mass), float(M5),
                         float(mf), int(bool(dag)), _ptr(idx), len(idx))
    return out


def normal(op: Op, U, psi) -> np.ndarray:
    """Op^dagger Op psi."""
    U, psi = _c128(U), _c128(psi)
    out, tmp = np.empty_like(psi), np.empty_like(psi)
    c = op._c()
    _load().oracle_normal(_ptr(U), _ptr(psi), _ptr(out), _ptr(tmp), _ptr(_dims(psi)), ctypes.byref(c))
    return out


def true_residual(op: Op, U, b, x) -> float:
    """|b - Op^dagger Op x| / |b| in FP64."""
    r = _c128(b) - normal(op, U, x)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def cg(op: Op, U, b, tol: float = 1e-10, maxiter: int = 20000, x0=None):
    """CG (Hestenes-Stiefel) on Op^dagger Op x = b. Returns (x, status, iterations, true relres).

    status 0: converged (true relative residual <= tol), 1: maxiter reached, 2: breakdown.
    """
    U, b = _c128(U), _c128(b)
    x = np.zeros_like(b) if x0 is None else _c128(x0).copy()
    stats = np.zeros(2)
    c = op._c()
    st = _load().oracle_cg(_ptr(U), _ptr(b), _ptr(x), _ptr(_dims(b)), ctypes.byref(c), float(tol),
                           int(maxiter), _ptr(stats))
    return x, int(st), int(stats[0]), float(stats[1])


def link_grad(chi, psi, c: float = 1.0, dag: bool = False) -> np.ndarray:
    """dL/dU (complex, dL/dRe + i dL/dIm) of L = Re <chi, c H psi> (H^dagger if dag).

    Shape (Lt,Lz,Ly,Lx,4,3,3); for 5D fields the fifth coordinate is summed.
    """
    chi, psi = _c128(chi), _c128(psi)
    G = np.empty(psi.shape[:4] + (4, 3, 3), dtype=np.complex128)
    _load().oracle_link_grad(_ptr(chi), _ptr(psi), _ptr(G), _ptr(_dims(psi)), _ls(psi), float(c),
                             int(bool(dag)))
    return G


def force(G, U) -> np.ndarray:
    """F = TA(G U^dagger) per link (traceless anti-Hermitian part)."""
    G, U = _c128(G), _c128(U)
    F = np.empty_like(G)
    _load().oracle_force(_ptr(G), _ptr(U), _ptr(F), int(G.size // 9))
    return F


def pseudofermion(op: Op, U, phi, tol: float = 1e-14, maxiter: int = 20000):
    """S = phi^dagger (Op^dagger Op)^-1 phi and dS/dU, recomputing the solve.

    With X = (Op^dagger Op)^-1 phi and Y = Op X, dS = -2 Re <Y, dOp X>, and Op's link dependence is
    its hopping part -H/2, so dS/dU = -2 G(chi = Y, psi = X) with G the link gradient at c = -1/2.
    Returns (S, dS/dU, X).
    """
    X, st, _, _ = cg(op, U, phi, tol=tol, maxiter=maxiter)
    if st != 0:
        raise RuntimeError(f"oracle CG did not converge (status {st})")
    Y = apply(op, U, X)
    S = float(np.vdot(_c128(phi), X).real)
    dS = -2.0 * link_grad(Y, X, c=-0.5)
    return S, dS, X


# ---------------------------------------------------------------------------------------------
# Storage codecs (numpy). Floating-point decisions are taken in float32, as the encoder defines.
# ---------------------------------------------------------------------------------------------

def fp16_encode(psi, site_axes: int):
    """FP16 storage with one float32 scale per site.

    ``psi`` is complex; the trailing ``site_axes`` axes (e.g. 2 for (4, 3)) form one site.
    The values are first rounded to float32; the site scale is s = max |Re|, |Im| over the site
    (float32); with r = float32(1 / s) (correctly rounded), each real is stored as
    float16(float32(v) * r) rounded to nearest even; s = 0 stores zeros. Returns (codes as
    float16 with a trailing re/im axis, scales float32).
    """
    psi = np.asarray(psi)
    re = np.stack([psi.real, psi.imag], axis=-1).astype(np.float32)
    lead = re.shape[: re.ndim - site_axes - 1]
    flat = re.reshape(lead + (-1,))
    s = np.max(np.abs(flat), axis=-1).astype(np.float32)
    safe = np.where(s > 0, s, np.float32(1)).astype(np.float32)
    r = (np.float32(1.0) / safe).astype(np.float32)
    q = (flat * r[..., None]).astype(np.float32).astype(np.float16)
    q = np.where(s[..., None] > 0, q, np.float16(0))
    return q.reshape(re.shape), s


def fp16_decode(codes, scales) -> np.ndarray:
    """Inverse of fp16_encode: float32(code) * scale, returned as complex128."""
    c = np.asarray(codes).astype(np.float32)
    s = np.asarray(scales).astype(np.float32)
    extra = c.ndim - s.ndim
    v = c * s.reshape(s.shape + (1,) * extra)
    return v[..., 0].astype(np.float64) + 1j * v[..., 1].astype(np.float64)


def compress12(U) -> np.ndarray:
    """Keep rows 0 and 1 of every SU(3) link: (..., 3, 3) -> (..., 2, 3)."""
    return np.ascontiguousarray(np.asarray(U)[..., :2, :])


def reconstruct12(U12) -> np.ndarray:
    """Rebuild row 2 = conj(row0 x row1) (exact for SU(3): the cofactor equals the conjugate)."""
    U12 = np.asarray(U12)
    r0, r1 = U12[..., 0, :], U12[..., 1, :]
    r2 = np.conj(np.cross(r0, r1))
    return np.concatenate([U12, r2[..., None, :]], axis=-2)


def reunitarise(U) -> np.ndarray:
    """Project a near-SU(3) matrix back to SU(3) in FP64.

    Normalise row 0; remove row 0's component from row 1 (Gram-Schmidt) and normalise it;
    row 2 = conj(row0 x row1).
    """
    U = np.asarray(U, dtype=np.complex128)
    r0 = U[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = U[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


# ---------------------------------------------------------------------------------------------
# Analytic operation counts (flops per site, the usual hopping-term convention).
# ---------------------------------------------------------------------------------------------

#: H per 4D site: 8 directions x (12 projection + 132 SU(3) x half-spinor) + 7 x 24 accumulation.
FLOPS_HOP = 8 * (12 + 132) + 7 * 24
#: Wilson D = (4 + m) psi - H psi / 2: +48 flops for the diagonal term (24 mul + 24 fma).
FLOPS_WILSON = FLOPS_HOP + 48
#: Domain-wall M per 5D site: H, the diagonal term and the two chirally projected s +- 1 terms.
FLOPS_DWF = FLOPS_HOP + 96
