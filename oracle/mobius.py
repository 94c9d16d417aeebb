"""Moebius domain-wall operator -- FP64 CPU oracle, TEST INFRASTRUCTURE ONLY.

The paper lists five-dimensional chiral fermions among Grid's actions (Section 4). The Moebius
(Cayley) form generalises the Shamir operator with two coefficients b5, c5:

    M = D_W B + (1 - S),   B = b5 + c5 S,   D_W = (4 - M5) - H / 2,
    (S psi)_s = P_- psi~_{s+1} + P_+ psi~_{s-1},   psi~_{Ls} = -mf psi_0,  psi~_{-1} = -mf psi_{Ls-1},

so M psi = -H chi / 2 + (4 - M5) chi + psi - S psi with chi = b5 psi + c5 S psi, and
M^dagger = B^dagger D_W^dagger + 1 - S^dagger with S^dagger = P_+ S_+ + P_- S_- (the projectors
exchanged). b5 = 1, c5 = 0 is the Shamir operator of ``oracle.dwf``.

Composed from the pinned ``oracle.hop`` and plain numpy shifts; used only by the test-suite.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import oracle as _o


@dataclass(frozen=True)
class MobiusOp:
    """The Moebius operator's parameters, as the fermion of an HMC oracle run."""
    M5: float
    mf: float
    b5: float
    c5: float


def shift5(psi, mf: float, dag: bool = False) -> np.ndarray:
    """S psi (S^dagger psi if dag) on a 5D field (..., Ls, 4, 3)."""
    psi = np.asarray(psi, dtype=np.complex128)
    up = np.roll(psi, -1, axis=-3).copy()     # psi~_{s+1}
    up[..., -1, :, :] *= -mf
    dn = np.roll(psi, 1, axis=-3).copy()      # psi~_{s-1}
    dn[..., 0, :, :] *= -mf
    out = np.empty_like(psi)
    lower, upper = slice(2, 4), slice(0, 2)
    from_up, from_dn = (upper, lower) if dag else (lower, upper)
    out[..., from_up, :] = up[..., from_up, :]
    out[..., from_dn, :] = dn[..., from_dn, :]
    return out


def mobius(U, psi, M5: float, mf: float, b5: float, c5: float, dag: bool = False) -> np.ndarray:
    """M psi or M^dagger psi for the Moebius operator (definition in the module docstring)."""
    psi = np.asarray(psi, dtype=np.complex128)
    if not dag:
        chi = b5 * psi + c5 * shift5(psi, mf)
        return -0.5 * _o.hop(U, chi) + (4.0 - M5) * chi + psi - shift5(psi, mf)
    phi = (4.0 - M5) * psi - 0.5 * _o.hop(U, psi, True)
    return b5 * phi + c5 * shift5(phi, mf, True) + psi - shift5(psi, mf, True)


def normal(U, psi, M5: float, mf: float, b5: float, c5: float) -> np.ndarray:
    """M^dagger M psi."""
    return mobius(U, mobius(U, psi, M5, mf, b5, c5), M5, mf, b5, c5, True)


def cg(U, b, M5: float, mf: float, b5: float, c5: float, tol: float = 1e-13, maxiter: int = 20000):
    """Textbook CG (Hestenes-Stiefel) on M^dagger M x = b from x = 0, stopping when the true
    relative residual |b - M^dagger M x| / |b| is <= tol. Returns (x, iterations)."""
    b = np.asarray(b, dtype=np.complex128)
    A = lambda v: normal(U, v, M5, mf, b5, c5)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = np.vdot(r, r).real
    bn = np.sqrt(np.vdot(b, b).real)
    for it in range(1, maxiter + 1):
        Ap = A(p)
        alpha = rr / np.vdot(p, Ap).real
        x += alpha * p
        r -= alpha * Ap
        rr_new = np.vdot(r, r).real
        if np.sqrt(rr_new) <= tol * bn and np.linalg.norm(b - A(x)) <= tol * bn:
            return x, it
        p = r + (rr_new / rr) * p
        rr = rr_new
    raise RuntimeError("Moebius oracle CG did not converge")


def pseudofermion(U, phi, M5: float, mf: float, b5: float, c5: float, tol: float = 1e-13):
    """S = Re phi^dagger (M^dagger M)^-1 phi and dS/dU for the Moebius M, the solve recomputed.

    M depends on the links only through its hopping part -H B / 2 (B = b5 + c5 S acts on the fifth
    coordinate), so with X = (M^dagger M)^-1 phi and Y = M X, dS = -2 Re <Y, dM X> gives
    dS/dU = -2 G(chi = Y, psi = B X), G the link gradient at c = -1/2. Returns (S, dS/dU, X).
    """
    X, _ = cg(U, phi, M5, mf, b5, c5, tol=tol)
    Y = mobius(U, X, M5, mf, b5, c5)
    S = float(np.vdot(np.asarray(phi, dtype=np.complex128), X).real)
    BX = b5 * X + c5 * shift5(X, mf)
    return S, -2.0 * _o.link_grad(Y, BX, c=-0.5), X
