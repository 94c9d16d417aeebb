"""Pins of the Moebius domain-wall oracle (oracle.mobius).

Fixed against the free-field momentum-space form of the operator, a dense matrix assembled entry
by entry from the textbook hopping term, the Shamir operator it must reduce to, and the
R5 gamma5 hermiticity every domain-wall operator of this family has.
"""
import numpy as np
import pytest

import oracle.oracle as O
from oracle import mobius as MB
from paper_1512_03487_amd import fields as F
from tests.lattice_testlib import (GAMMA5, I4, P_MINUS, P_PLUS, TEXTBOOK_GAMMA, dense_hop, momentum, plane_wave, rel,
                                   spin_apply)

B5, C5 = 1.5, 0.5


@pytest.mark.parametrize("dag", [False, True])
def test_reduces_to_shamir(dag):
    dims, Ls = (2, 4, 2, 4), 6
    U = F.gauge_field(dims, seed=1, kind="haar")
    psi = F.spinor_field(dims, seed=2, Ls=Ls)
    assert rel(MB.mobius(U, psi, 1.8, 0.04, 1.0, 0.0, dag), O.dwf(U, psi, 1.8, 0.04, dag)) < 1e-14


@pytest.mark.parametrize("dag", [False, True])
def test_free_field_fourier_blocks(dag):
    """U = 1, psi_s = e^{ip.x} u_s: D_W acts as -M5 + sum(1 - cos p) + i gamma.sin p on each u_s."""
    dims, Ls, M5, mf = (4, 4, 4, 4), 5, 1.8, 0.03
    U = F.gauge_field(dims, kind="unit")
    rng = np.random.default_rng(8)
    for n in [(0, 0, 0, 0), (1, 0, 2, 3), (3, 1, 0, 1)]:
        p = momentum(dims, n)
        u = rng.standard_normal((Ls, 4, 3)) + 1j * rng.standard_normal((Ls, 4, 3))
        W = (-M5 + np.sum(1 - np.cos(p))) * I4 + 1j * sum(TEXTBOOK_GAMMA[mu] * np.sin(p[mu]) for mu in range(4))

        def S(v, adj):
            Pup, Pdn = (P_PLUS, P_MINUS) if adj else (P_MINUS, P_PLUS)
            out = np.empty_like(v)
            for s in range(Ls):
                up = v[(s + 1) % Ls] * (-mf if s == Ls - 1 else 1.0)
                dn = v[(s - 1) % Ls] * (-mf if s == 0 else 1.0)
                out[s] = Pup @ up + Pdn @ dn
            return out

        if not dag:
            chi = B5 * u + C5 * S(u, False)
            expect = np.einsum("ij,sjc->sic", W, chi) + u - S(u, False)
        else:
            phi = np.einsum("ij,sjc->sic", W.conj().T, u)
            expect = B5 * phi + C5 * S(phi, True) + u - S(u, True)
        got = MB.mobius(U, plane_wave(dims, n, u), M5, mf, B5, C5, dag)
        assert np.max(np.abs(got - plane_wave(dims, n, expect))) < 1e-13


def test_dense_brute_force_and_adjoint():
    dims, Ls, M5, mf = (2, 2, 2, 2), 4, 1.8, 0.05
    U = F.gauge_field(dims, seed=1, kind="haar")
    V = int(np.prod(dims))
    H = dense_hop(U, False).reshape(V, 12, V, 12)
    n = V * Ls * 12
    Dw = np.zeros((V, Ls, 12, V, Ls, 12), dtype=complex)
    for s in range(Ls):
        Dw[:, s, :, :, s, :] = -0.5 * H
    Dw = Dw.reshape(n, n) + (4.0 - M5) * np.eye(n)
    S5p, S5m = np.zeros((Ls, Ls)), np.zeros((Ls, Ls))
    for s in range(Ls):
        S5p[s, (s + 1) % Ls] = -mf if s == Ls - 1 else 1.0
        S5m[s, (s - 1) % Ls] = -mf if s == 0 else 1.0
    I3 = np.eye(3)
    S = np.kron(np.eye(V), np.kron(S5p, np.kron(P_MINUS, I3)) + np.kron(S5m, np.kron(P_PLUS, I3)))
    M = Dw @ (B5 * np.eye(n) + C5 * S) + np.eye(n) - S
    psi = F.spinor_field(dims, seed=2, Ls=Ls)
    assert np.max(np.abs(MB.mobius(U, psi, M5, mf, B5, C5).ravel() - M @ psi.ravel())) < 1e-13
    assert np.max(np.abs(MB.mobius(U, psi, M5, mf, B5, C5, True).ravel() - M.conj().T @ psi.ravel())) < 1e-13


def test_adjoint_inner_product():
    """<chi, M psi> = <M^dagger chi, psi> on a lattice too large for the dense check. (Unlike the
    Shamir operator, M is not R5 gamma5-hermitian for c5 != 0: D_W and S do not commute.)"""
    dims, Ls = (4, 4, 2, 4), 6
    U = F.gauge_field(dims, seed=1, kind="haar")
    psi = F.spinor_field(dims, seed=2, Ls=Ls)
    chi = F.spinor_field(dims, seed=3, Ls=Ls)
    a = np.vdot(chi, MB.mobius(U, psi, 1.8, 0.02, B5, C5))
    b = np.vdot(MB.mobius(U, chi, 1.8, 0.02, B5, C5, True), psi)
    assert abs(a - b) < 1e-13 * abs(a)

    def G5(v):
        return spin_apply(GAMMA5, v[..., ::-1, :, :])
    # the Shamir limit keeps R5 gamma5 hermiticity
    lhs = MB.mobius(U, psi, 1.8, 0.02, 1.0, 0.0, True)
    assert rel(lhs, G5(MB.mobius(U, G5(psi), 1.8, 0.02, 1.0, 0.0))) < 1e-14


def _dense_mobius(U, shape, **kw):
    n = int(np.prod(shape))
    M = np.empty((n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        M[:, j] = MB.mobius(U, e.reshape(shape), **kw).ravel()
    return M


def test_pseudofermion_shamir_limit():
    """b5 = 1, c5 = 0: the Moebius pseudofermion action and force are the domain-wall ones of the C
    oracle."""
    dims, Ls = (2, 2, 2, 2), 4
    U = F.gauge_field(dims, seed=1, kind="haar")
    phi = F.spinor_field(dims, seed=5, Ls=Ls)
    S, dS, _ = MB.pseudofermion(U, phi, 1.8, 0.1, 1.0, 0.0)
    S0, dS0, _ = O.pseudofermion(O.Op.dwf(Ls, 1.8, 0.1), U, phi)
    assert abs(S - S0) < 1e-10 * abs(S0)
    assert np.linalg.norm(dS - dS0) < 1e-9 * np.linalg.norm(dS0)


def test_pseudofermion_dense_and_fd():
    """b5 = 1.5, c5 = 0.5 at 2^4 x 4: S against a dense solve, and the su(3) force against a
    central finite difference of the dense S along a random su(3) direction."""
    from tests.lattice_testlib import su3_exp
    dims, Ls = (2, 2, 2, 2), 4
    kw = dict(M5=1.8, mf=0.1, b5=1.5, c5=0.5)
    U = F.gauge_field(dims, seed=1, kind="haar")
    phi = F.spinor_field(dims, seed=5, Ls=Ls)
    S, dS, _ = MB.pseudofermion(U, phi, **kw)

    def S_dense(UU):
        M = _dense_mobius(UU, phi.shape, **kw)
        return np.vdot(phi.ravel(), np.linalg.solve(M.conj().T @ M, phi.ravel())).real
    assert abs(S - S_dense(U)) < 1e-10 * abs(S)
    Xd = F.random_su3_algebra(dims, seed=8)
    eps = 1e-4
    fd = (S_dense(su3_exp(eps * Xd) @ U) - S_dense(su3_exp(-eps * Xd) @ U)) / (2 * eps)
    an = np.sum(np.einsum("...ij,...ij->...", O.force(dS, U).conj(), Xd).real)
    assert abs(fd - an) < 1e-6 * abs(an)
