"""Hybrid Monte Carlo pieces -- FP64 CPU oracle, TEST INFRASTRUCTURE ONLY.

HMC is named by the paper among the algorithms Grid provides (Section 4). Definitions used:

* Wilson gauge action S_G = beta sum_{x, mu < nu} (1 - Re tr P_munu(x) / 3) with the plaquette
  P_munu(x) = U_mu(x) U_nu(x + mu) U_mu(x + nu)^dagger U_nu(x)^dagger.
* Forces follow the fermion-force convention: F = TA(G U^dagger) with G = dS/dRe U + i dS/dIm U,
  so that d/de S(exp(e X) U)|0 = Re tr(F^dagger X) for X in su(3). For S_G, G_mu(x) = -(beta/3)
  A_mu(x)^dagger with A_mu(x) the sum of the six staples that close U_mu(x) into plaquettes.
* Momenta P in su(3) per link, kinetic energy K = sum tr(P^dagger P) (a Gaussian refresh draws
  P = i h_a lambda_a / 2 with h_a ~ N(0, 1)); H = K + S_G (+ S_F).
* Equations of motion dU/dt = P U, dP/dt = -F / 2, which conserve H; the leapfrog integrator
  P -= (e/2) F/2, then n times {U <- exp(e P) U; P -= e F/2} with the last momentum step halved.
* exp of an anti-Hermitian matrix through the eigendecomposition of the Hermitian -i X.

Composed from the pinned C oracle (``oracle.force``, ``oracle.pseudofermion``) and numpy; used only
by the test-suite.
"""
from __future__ import annotations

import numpy as np

from . import mobius as _mob
from . import oracle as _o

_AX = {0: 3, 1: 2, 2: 1, 3: 0}   # numpy axis of direction mu in (Lt, Lz, Ly, Lx, ...)


def _sh(field, mu, k):
    """field(x + k mu-hat), periodic."""
    return np.roll(field, -k, axis=_AX[mu])


def _dag(a):
    return np.conj(np.swapaxes(a, -1, -2))


def _mm(*ms):
    out = ms[0]
    for m in ms[1:]:
        out = np.einsum("...ij,...jk->...ik", out, m)
    return out


def plaquette_field(U, mu, nu):
    Um, Un = U[..., mu, :, :], U[..., nu, :, :]
    return _mm(Um, _sh(Un, mu, 1), _dag(_sh(Um, nu, 1)), _dag(Un))


def plaquette(U) -> float:
    """Average of Re tr P_munu / 3 over sites and the six planes."""
    tot, n = 0.0, 0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            P = plaquette_field(U, mu, nu)
            tot += float(np.trace(P, axis1=-2, axis2=-1).real.sum())
            n += P.shape[0] * P.shape[1] * P.shape[2] * P.shape[3]
    return tot / (3.0 * n)


def gauge_action(U, beta: float) -> float:
    s = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            s += float((1.0 - np.trace(plaquette_field(U, mu, nu), axis1=-2, axis2=-1).real / 3.0).sum())
    return beta * s


def staples(U, mu):
    """A_mu(x): sum over nu != mu of the upper and lower staples, Re tr(U_mu A_mu) = the plaquettes."""
    Um = U[..., mu, :, :]
    A = np.zeros_like(Um)
    for nu in range(4):
        if nu == mu:
            continue
        Un = U[..., nu, :, :]
        A += _mm(_sh(Un, mu, 1), _dag(_sh(Um, nu, 1)), _dag(Un))
        Un_m = _sh(Un, nu, -1)
        A += _mm(_dag(_sh(Un_m, mu, 1)), _dag(_sh(Um, nu, -1)), Un_m)
    return A


def gauge_force(U, beta: float) -> np.ndarray:
    """F = TA(G U^dagger) with G = dS_G/dU = -(beta/3) A^dagger."""
    G = np.empty_like(U)
    for mu in range(4):
        G[..., mu, :, :] = -(beta / 3.0) * _dag(staples(U, mu))
    return _o.force(G, U)


def su3_exp(X):
    """exp(X) per matrix for anti-Hermitian X."""
    w, v = np.linalg.eigh(-1j * X)
    return np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * w), v.conj())


def kinetic(P) -> float:
    return float(np.sum(np.abs(P) ** 2))


def fermion_force(U, fermion):
    """(S_F, F_F) for S_F = phi^dagger (M^dagger M)^-1 phi; fermion = (Op, phi), Op an
    ``oracle.Op`` (Wilson D or Shamir M) or an ``oracle.mobius.MobiusOp``."""
    op, phi = fermion
    if isinstance(op, _mob.MobiusOp):
        S, dS, _ = _mob.pseudofermion(U, phi, op.M5, op.mf, op.b5, op.c5, tol=1e-12)
    else:
        S, dS, _ = _o.pseudofermion(op, U, phi, tol=1e-12)
    return S, _o.force(dS, U)


def md_force(U, beta, fermion=None):
    """dP/dt = -md_force: half the total su(3) force."""
    F = gauge_force(U, beta)
    if fermion is not None:
        F = F + fermion_force(U, fermion)[1]
    return 0.5 * F


def hamiltonian(U, P, beta, fermion=None) -> float:
    H = kinetic(P) + gauge_action(U, beta)
    if fermion is not None:
        H += fermion_force(U, fermion)[0]
    return H


OMELYAN_LAMBDA = 0.1931833275037836   # Omelyan, Mryglod and Folk's second-order minimum-norm value


def omelyan(U, P, beta: float, eps: float, n: int, fermion=None):
    """Second-order minimum-norm integrator: per step P -= l e F/2; U <- exp(e/2 P) U;
    P -= (1 - 2 l) e F/2; U <- exp(e/2 P) U; P -= l e F/2 (l = OMELYAN_LAMBDA)."""
    lam = OMELYAN_LAMBDA
    U, P = np.array(U, dtype=np.complex128), np.array(P, dtype=np.complex128)

    def drift(U, P):
        return np.einsum("...ij,...jk->...ik", su3_exp(0.5 * eps * P), U)
    for _ in range(n):
        P = P - lam * eps * md_force(U, beta, fermion)
        U = drift(U, P)
        P = P - (1.0 - 2.0 * lam) * eps * md_force(U, beta, fermion)
        U = drift(U, P)
        P = P - lam * eps * md_force(U, beta, fermion)
    return U, P


def force_gradient(U, P, beta: float, eps: float, n: int, fermion=None):
    """Force-gradient integrator (Omelyan, Mryglod and Folk's fourth-order PQPQP scheme with the
    force-gradient term, in the Hessian-free form of Yin and Mawhinney): per step
    P -= e/6 f(U); U <- exp(e/2 P) U; P -= 2e/3 f(U'), U' = exp(-(e^2/24) f(U)) U;
    U <- exp(e/2 P) U; P -= e/6 f(U), with f = md_force (dP/dt = -f)."""
    U, P = np.array(U, dtype=np.complex128), np.array(P, dtype=np.complex128)

    def drift(U, P, t):
        return np.einsum("...ij,...jk->...ik", su3_exp(t * P), U)
    for _ in range(n):
        P = P - (eps / 6.0) * md_force(U, beta, fermion)
        U = drift(U, P, 0.5 * eps)
        Ud = drift(U, md_force(U, beta, fermion), -eps * eps / 24.0)
        P = P - (2.0 * eps / 3.0) * md_force(Ud, beta, fermion)
        U = drift(U, P, 0.5 * eps)
        P = P - (eps / 6.0) * md_force(U, beta, fermion)
    return U, P


def gauge_md_force(U, beta):
    return 0.5 * gauge_force(U, beta)


def fermion_md_force(U, fermion):
    return np.zeros_like(U) if fermion is None else 0.5 * fermion_force(U, fermion)[1]


def nested_leapfrog(U, P, beta: float, eps: float, n: int, fermion, n_inner: int):
    """Two time scales (Sexton and Weingarten): per outer step P -= e/2 f_F(U), then n_inner
    leapfrog steps of size e / n_inner with the gauge force alone, then P -= e/2 f_F(U)."""
    U, P = np.array(U, dtype=np.complex128), np.array(P, dtype=np.complex128)
    h = eps / n_inner
    for _ in range(n):
        P = P - 0.5 * eps * fermion_md_force(U, fermion)
        for _ in range(n_inner):
            P = P - 0.5 * h * gauge_md_force(U, beta)
            U = np.einsum("...ij,...jk->...ik", su3_exp(h * P), U)
            P = P - 0.5 * h * gauge_md_force(U, beta)
        P = P - 0.5 * eps * fermion_md_force(U, fermion)
    return U, P


def _inner_leapfrog(U, P, beta: float, tau: float, n_inner: int):
    """n_inner leapfrog steps of size tau / n_inner with the gauge force alone."""
    h = tau / n_inner
    for _ in range(n_inner):
        P = P - 0.5 * h * gauge_md_force(U, beta)
        U = np.einsum("...ij,...jk->...ik", su3_exp(h * P), U)
        P = P - 0.5 * h * gauge_md_force(U, beta)
    return U, P


def nested_omelyan(U, P, beta: float, eps: float, n: int, fermion, n_inner: int):
    """Two time scales with an Omelyan outer step: per outer step P -= l e f_F(U); the gauge system
    integrated over e/2 by n_inner leapfrog steps; P -= (1 - 2 l) e f_F(U); again e/2 of gauge
    integration; P -= l e f_F(U) (l = OMELYAN_LAMBDA)."""
    lam = OMELYAN_LAMBDA
    U, P = np.array(U, dtype=np.complex128), np.array(P, dtype=np.complex128)
    for _ in range(n):
        P = P - lam * eps * fermion_md_force(U, fermion)
        U, P = _inner_leapfrog(U, P, beta, 0.5 * eps, n_inner)
        P = P - (1.0 - 2.0 * lam) * eps * fermion_md_force(U, fermion)
        U, P = _inner_leapfrog(U, P, beta, 0.5 * eps, n_inner)
        P = P - lam * eps * fermion_md_force(U, fermion)
    return U, P


def nested_force_gradient(U, P, beta: float, eps: float, n: int, fermion, n_inner: int):
    """Two time scales with a force-gradient outer step: per outer step P -= e/6 f_F(U); the gauge
    system integrated over e/2 by n_inner leapfrog steps; P -= 2e/3 f_F(U') with the displaced
    links U' = exp(-(e^2/24) f_F(U)) U (the outer force's gradient term, as in force_gradient());
    again e/2 of gauge integration; P -= e/6 f_F(U)."""
    U, P = np.array(U, dtype=np.complex128), np.array(P, dtype=np.complex128)
    for _ in range(n):
        P = P - (eps / 6.0) * fermion_md_force(U, fermion)
        U, P = _inner_leapfrog(U, P, beta, 0.5 * eps, n_inner)
        Ud = np.einsum("...ij,...jk->...ik", su3_exp(-(eps * eps / 24.0) * fermion_md_force(U, fermion)), U)
        P = P - (2.0 * eps / 3.0) * fermion_md_force(Ud, fermion)
        U, P = _inner_leapfrog(U, P, beta, 0.5 * eps, n_inner)
        P = P - (eps / 6.0) * fermion_md_force(U, fermion)
    return U, P


def leapfrog(U, P, beta: float, eps: float, n: int, fermion=None):
    U, P = np.array(U, dtype=np.complex128), np.array(P, dtype=np.complex128)
    if n == 0:   # zero steps integrate over zero time
        return U, P
    P = P - 0.5 * eps * md_force(U, beta, fermion)
    for i in range(n):
        U = np.einsum("...ij,...jk->...ik", su3_exp(eps * P), U)
        P = P - (0.5 if i == n - 1 else 1.0) * eps * md_force(U, beta, fermion)
    return U, P
