"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test fixes the oracle to a closed form, an invariant, a textbook object or a brute-force
evaluation, chosen so that a plausible slip (a dropped term, a flipped sign, a swapped
forward/backward neighbour, a transposed link, a wrong axis) fails at least one of them.
"""
import itertools

import numpy as np
import pytest

import oracle.oracle as O
from paper_1512_03487_amd import fields as F
from tests.lattice_testlib import (GAMMA5, I4, P_MINUS, P_PLUS, TEXTBOOK_GAMMA, dense_dwf, dense_wilson,
                                   dims_of, momentum, plane_wave, rel, shift, spin_apply, su3_exp)


# ----------------------------------------------------------------------------------- gammas ---

def test_gamma_basis_is_the_textbook_chiral_basis():
    for mu in range(4):
        np.testing.assert_array_equal(O.gamma(mu), TEXTBOOK_GAMMA[mu])
    np.testing.assert_allclose(O.gamma(4), GAMMA5, atol=0)


def test_clifford_algebra_and_hermiticity():
    g = [O.gamma(mu) for mu in range(4)]
    for mu, nu in itertools.product(range(4), range(4)):
        anti = g[mu] @ g[nu] + g[nu] @ g[mu]
        np.testing.assert_allclose(anti, 2 * (mu == nu) * I4, atol=1e-15)
    for mu in range(4):
        np.testing.assert_allclose(g[mu], g[mu].conj().T, atol=0)
        np.testing.assert_allclose(O.gamma(4) @ g[mu], -g[mu] @ O.gamma(4), atol=1e-15)


# ------------------------------------------------------------------------------ free field (P1) ---

@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (3, 4, 5, 6)])
def test_free_field_plane_waves(dims):
    """U = 1: D e^{ip.x} u = [m + sum(1 - cos p) + i sum gamma_mu sin p_mu] e^{ip.x} u."""
    mass = 0.1
    U = F.gauge_field(dims, kind="unit")
    rng = np.random.default_rng(11)
    for n in [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1), (1, 2, 3, 1), (2, 1, 1, 3)]:
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi = plane_wave(dims, n, u)
        p = momentum(dims, n)
        K = (mass + np.sum(1 - np.cos(p))) * I4 + 1j * sum(TEXTBOOK_GAMMA[mu] * np.sin(p[mu]) for mu in range(4))
        expect = plane_wave(dims, n, K @ u)
        got = O.wilson(U, psi, mass)
        assert np.max(np.abs(got - expect)) < 1e-13
        # D^dagger has the conjugate symbol
        got_dag = O.wilson(U, psi, mass, dag=True)
        expect_dag = plane_wave(dims, n, K.conj().T @ u)
        assert np.max(np.abs(got_dag - expect_dag)) < 1e-13


def test_free_field_spectrum_dense():
    """Eigenvalues of the free D on 3^4 are m + sum(1 - cos p) +- i sqrt(sum sin^2 p), 6 times each."""
    dims, mass = (3, 3, 3, 3), 0.1
    U = F.gauge_field(dims, kind="unit")
    n = int(np.prod(dims)) * 12
    D = np.zeros((n, n), dtype=complex)
    e = np.zeros(n, dtype=complex)
    for k in range(n):                  # columns from the oracle applied to unit vectors
        e[:] = 0
        e[k] = 1
        D[:, k] = O.wilson(U, e.reshape(3, 3, 3, 3, 4, 3), mass).ravel()
    ev = np.linalg.eigvals(D)
    expect = []
    for nn in itertools.product(range(3), repeat=4):
        p = momentum(dims, nn)
        re, im = mass + np.sum(1 - np.cos(p)), np.sqrt(np.sum(np.sin(p) ** 2))
        expect += [re + 1j * im] * 6 + [re - 1j * im] * 6
    key = lambda z: (round(z.real, 8), round(z.imag, 8))
    got = sorted(ev, key=key)
    exp = sorted(expect, key=key)
    assert np.max(np.abs(np.array(got) - np.array(exp))) < 1e-10


def test_cshift_derivative_identity():
    """0.5 (psi(x + y) - psi(x - y)) = i sin(p_y) psi for a plane wave (Section 2.3's example)."""
    dims = (4, 6, 4, 4)
    psi = plane_wave(dims, (0, 1, 0, 0), np.ones((4, 3)))
    d = 0.5 * (shift(psi, 1, +1) - shift(psi, 1, -1))
    np.testing.assert_allclose(d, 1j * np.sin(2 * np.pi / 6) * psi, atol=1e-14)


# ------------------------------------------------------------------- invariants (P2, P3) ---

@pytest.fixture(scope="module")
def haar44():
    dims = (4, 4, 4, 4)
    return dims, F.gauge_field(dims, seed=1, kind="haar"), F.spinor_field(dims, seed=2), F.spinor_field(dims, seed=3)


def test_gamma5_hermiticity(haar44):
    dims, U, psi, chi = haar44
    m = 0.1
    lhs = np.vdot(chi, O.wilson(U, psi, m))
    g5Dg5chi = spin_apply(GAMMA5, O.wilson(U, spin_apply(GAMMA5, chi), m))
    rhs = np.vdot(g5Dg5chi, psi)
    scale = np.linalg.norm(chi) * np.linalg.norm(O.wilson(U, psi, m))
    assert abs(lhs - rhs) < 1e-14 * scale
    # and the dag flag is the adjoint
    assert abs(lhs - np.vdot(O.wilson(U, chi, m, dag=True), psi)) < 1e-14 * scale
    # H^dagger = gamma5 H gamma5 as operators
    np.testing.assert_allclose(O.hop(U, psi, dag=True), spin_apply(GAMMA5, O.hop(U, spin_apply(GAMMA5, psi))),
                               atol=1e-13)


def test_gauge_covariance(haar44):
    dims, U, psi, _ = haar44
    g = F.gauge_transform(dims, seed=4)
    Up = np.empty_like(U)
    for mu in range(4):
        Up[..., mu, :, :] = g @ U[..., mu, :, :] @ shift(g, mu, +1).conj().swapaxes(-1, -2)
    psip = np.einsum("...ab,...sb->...sa", g, psi)
    lhs = O.wilson(Up, psip, 0.1)
    rhs = np.einsum("...ab,...sb->...sa", g, O.wilson(U, psi, 0.1))
    assert np.max(np.abs(lhs - rhs)) < 1e-13


def test_not_covariant_under_a_wrong_transform(haar44):
    """Control: transforming the links with g(x - mu) instead of g(x + mu) breaks covariance."""
    dims, U, psi, _ = haar44
    g = F.gauge_transform(dims, seed=4)
    Up = np.empty_like(U)
    for mu in range(4):
        Up[..., mu, :, :] = g @ U[..., mu, :, :] @ shift(g, mu, -1).conj().swapaxes(-1, -2)
    psip = np.einsum("...ab,...sb->...sa", g, psi)
    lhs = O.wilson(Up, psip, 0.1)
    rhs = np.einsum("...ab,...sb->...sa", g, O.wilson(U, psi, 0.1))
    assert np.max(np.abs(lhs - rhs)) > 1e-3


# ------------------------------------------------------------------------- brute force (P4) ---

@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 3, 4, 5)])
@pytest.mark.parametrize("dag", [False, True])
def test_dense_brute_force_wilson(dims, dag):
    U = F.gauge_field(dims, seed=1, kind="haar")
    psi = F.spinor_field(dims, seed=2)
    D = dense_wilson(U, 0.1, dag)
    expect = (D @ psi.ravel()).reshape(psi.shape)
    assert np.max(np.abs(O.wilson(U, psi, 0.1, dag) - expect)) < 1e-13
    if dag:
        np.testing.assert_allclose(D, dense_wilson(U, 0.1, False).conj().T, atol=1e-15)


# ------------------------------------------------------------------------ SU(3) fields (P6) ---

def test_haar_links_are_su3_and_haar():
    u = F.haar_su3(F.make_rng(7), 20000)
    np.testing.assert_allclose(u.conj().swapaxes(-1, -2) @ u, np.broadcast_to(np.eye(3), u.shape), atol=1e-13)
    np.testing.assert_allclose(np.linalg.det(u), 1.0, atol=1e-13)
    tr = np.trace(u, axis1=-2, axis2=-1)
    n = len(tr)
    # Haar moments on SU(3): E tr U = 0, E |tr U|^2 = 1 (Var |tr U|^2 = 1 for SU(3), fourth moment 2)
    assert abs(tr.mean()) < 5 * np.sqrt(1.0 / n)
    assert abs(np.mean(np.abs(tr) ** 2) - 1.0) < 5 * np.sqrt(1.0 / n)


def test_weak_links_are_su3_near_identity():
    u = F.weak_su3(F.make_rng(8), 4000, eps=0.3)
    np.testing.assert_allclose(u.conj().swapaxes(-1, -2) @ u, np.broadcast_to(np.eye(3), u.shape), atol=1e-13)
    np.testing.assert_allclose(np.linalg.det(u), 1.0, atol=1e-13)
    # |1 - U| = O(eps): mean of Re tr U / 3 close to 1 - eps^2 <h^2>/... > 0.9
    assert np.mean(np.trace(u, axis1=-2, axis2=-1).real) / 3 > 0.9


def test_link_compression_and_reunitarisation():
    U = F.gauge_field((4, 4, 4, 4), seed=1, kind="haar")
    np.testing.assert_allclose(O.reconstruct12(O.compress12(U)), U, atol=1e-14)
    # reunitarisation: fixed point on SU(3), projects a perturbed matrix back onto SU(3)
    np.testing.assert_allclose(O.reunitarise(U), U, atol=1e-14)
    rng = np.random.default_rng(3)
    noisy = U + 1e-4 * (rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape))
    R = O.reunitarise(noisy)
    np.testing.assert_allclose(R.conj().swapaxes(-1, -2) @ R, np.broadcast_to(np.eye(3), R.shape), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-14)
    assert np.max(np.abs(R - U)) < 1e-3
    # and a rounded-to-float32 link reunitarised in FP64 is much closer to SU(3) than the rounded one
    U32 = U.astype(np.complex64).astype(np.complex128)
    R32 = O.reunitarise(U32)
    def dev(M):
        return np.max(np.abs(M.conj().swapaxes(-1, -2) @ M - np.eye(3)))
    assert dev(R32) < 1e-14 < dev(U32)


# ------------------------------------------------------------------------------ DWF (P7, P8) ---

@pytest.mark.parametrize("dag", [False, True])
def test_dwf_fourier_blocks(dag):
    """U = 1, psi_s = e^{ip.x} u_s: M acts on (u_s) as a closed-form 4 Ls x 4 Ls block."""
    dims, Ls, M5, mf = (4, 4, 4, 4), 6, 1.8, 0.01
    U = F.gauge_field(dims, kind="unit")
    rng = np.random.default_rng(5)
    for n in [(0, 0, 0, 0), (1, 0, 2, 3), (3, 1, 0, 1)]:
        p = momentum(dims, n)
        u = rng.standard_normal((Ls, 4, 3)) + 1j * rng.standard_normal((Ls, 4, 3))
        W = (1 - M5 + np.sum(1 - np.cos(p))) * I4 + 1j * sum(TEXTBOOK_GAMMA[mu] * np.sin(p[mu]) for mu in range(4))
        if dag:
            W = W.conj().T
        Pup, Pdn = (P_PLUS, P_MINUS) if dag else (P_MINUS, P_PLUS)
        expect = np.empty_like(u)
        for s in range(Ls):
            up = u[(s + 1) % Ls] * (-mf if s == Ls - 1 else 1.0)
            dn = u[(s - 1) % Ls] * (-mf if s == 0 else 1.0)
            expect[s] = W @ u[s] - Pup @ up - Pdn @ dn
        got = O.dwf(U, plane_wave(dims, n, u), M5, mf, dag)
        assert np.max(np.abs(got - plane_wave(dims, n, expect))) < 1e-13


def test_dwf_reduces_to_wilson_at_ls1():
    """Ls = 1: both walls give +mf psi, so M = D_W with m = 1 - M5 + mf."""
    dims = (4, 4, 2, 4)
    U = F.gauge_field(dims, seed=1, kind="haar")
    psi = F.spinor_field(dims, seed=2)
    got = O.dwf(U, psi[..., None, :, :], 1.8, 0.01)[..., 0, :, :]
    np.testing.assert_allclose(got, O.wilson(U, psi, 1 - 1.8 + 0.01), atol=1e-13)


def test_dwf_r5g5_hermiticity_and_adjoint():
    dims, Ls = (4, 4, 4, 4), 8
    U = F.gauge_field(dims, seed=1, kind="haar")
    psi = F.spinor_field(dims, seed=2, Ls=Ls)
    chi = F.spinor_field(dims, seed=3, Ls=Ls)
    M5, mf = 1.8, 0.01
    def G5(v):
        return spin_apply(GAMMA5, v[..., ::-1, :, :])
    lhs = np.vdot(chi, O.dwf(U, psi, M5, mf))
    scale = np.linalg.norm(chi) * np.linalg.norm(psi) * 10
    assert abs(lhs - np.vdot(G5(O.dwf(U, G5(chi), M5, mf)), psi)) < 1e-14 * scale
    assert abs(lhs - np.vdot(O.dwf(U, chi, M5, mf, dag=True), psi)) < 1e-14 * scale
    # M^dagger = Gamma5 M Gamma5 as operators
    np.testing.assert_allclose(O.dwf(U, psi, M5, mf, dag=True), G5(O.dwf(U, G5(psi), M5, mf)), atol=1e-13)


@pytest.mark.parametrize("dag", [False, True])
def test_dwf_dense_brute_force(dag):
    dims, Ls, M5, mf = (2, 2, 2, 2), 4, 1.8, 0.01
    U = F.gauge_field(dims, seed=1, kind="haar")
    psi = F.spinor_field(dims, seed=2, Ls=Ls)
    M = dense_dwf(U, Ls, M5, mf, dag)
    expect = (M @ psi.ravel()).reshape(psi.shape)
    assert np.max(np.abs(O.dwf(U, psi, M5, mf, dag) - expect)) < 1e-13
    if not dag:
        A = M.conj().T @ M
        np.testing.assert_allclose(A, A.conj().T, atol=1e-12)
        assert np.min(np.linalg.eigvalsh(A)) > 0


# ---------------------------------------------------------------------------------- CG (P9) ---

@pytest.mark.parametrize("kind", ["wilson", "dwf"])
def test_cg_against_dense_solve(kind):
    dims = (2, 2, 2, 2)
    U = F.gauge_field(dims, seed=1, kind="haar")
    if kind == "wilson":
        op = O.Op.wilson(0.1)
        b = F.spinor_field(dims, seed=3)
        M = dense_wilson(U, 0.1)
    else:
        op = O.Op.dwf(4, 1.8, 0.01)
        b = F.spinor_field(dims, seed=3, Ls=4)
        M = dense_dwf(U, 4, 1.8, 0.01)
    A = M.conj().T @ M
    xs = np.linalg.solve(A, b.ravel())
    x, st, it, res = O.cg(op, U, b, tol=1e-12, maxiter=5000)
    assert st == 0 and res <= 1e-12
    # independent true residual from the dense matrix
    assert np.linalg.norm(b.ravel() - A @ x.ravel()) / np.linalg.norm(b) <= 1e-12
    assert rel(x.ravel(), xs) <= np.linalg.cond(A) * 1e-12


def test_cg_reports_maxiter_and_warm_start():
    dims = (2, 2, 2, 2)
    U = F.gauge_field(dims, seed=1, kind="haar")
    op = O.Op.dwf(4, 1.8, 0.01)
    b = F.spinor_field(dims, seed=3, Ls=4)
    x, st, it, res = O.cg(op, U, b, tol=1e-12, maxiter=3)
    assert st == 1 and it == 3 and res > 1e-12
    x2, st2, it2, res2 = O.cg(op, U, b, tol=1e-12, maxiter=5000, x0=x)
    assert st2 == 0 and res2 <= 1e-12


# --------------------------------------------------------------------------- gradients (P10) ---

@pytest.fixture(scope="module")
def weak44():
    dims = (4, 4, 4, 4)
    return (dims, F.gauge_field(dims, seed=1, kind="weak"), F.spinor_field(dims, seed=2),
            F.spinor_field(dims, seed=3))


def test_link_gradient_componentwise_fd(weak44):
    """L = Re <chi, D psi> is linear in each complex link entry: FD gives dL/dRe, dL/dIm exactly."""
    dims, U, psi, chi = weak44
    m = 0.1
    G = O.link_grad(chi, psi, c=-0.5)
    L = lambda UU: np.vdot(chi, O.wilson(UU, psi, m)).real
    rng = np.random.default_rng(1)
    for _ in range(6):
        t, z, y, x = (int(v) for v in rng.integers(0, 4, 4))
        mu, a, b = int(rng.integers(4)), int(rng.integers(3)), int(rng.integers(3))
        for unit in (1.0, 1j):
            Up, Um = U.copy(), U.copy()
            Up[t, z, y, x, mu, a, b] += 1e-3 * unit
            Um[t, z, y, x, mu, a, b] -= 1e-3 * unit
            fd = (L(Up) - L(Um)) / 2e-3
            want = G[t, z, y, x, mu, a, b].real if unit == 1.0 else G[t, z, y, x, mu, a, b].imag
            assert abs(fd - want) < 1e-9 * max(1.0, abs(want))


def test_force_fd_along_su3(weak44):
    """d/de L(exp(e X) U) at 0 equals sum Re tr(F^dagger X), F = TA(G U^dagger), central FD in FP64."""
    dims, U, psi, chi = weak44
    m = 0.1
    G = O.link_grad(chi, psi, c=-0.5)
    Fo = O.force(G, U)
    # F is in su(3): anti-Hermitian and traceless
    np.testing.assert_allclose(Fo, -Fo.conj().swapaxes(-1, -2), atol=1e-14)
    assert np.max(np.abs(np.trace(Fo, axis1=-2, axis2=-1))) < 1e-13
    X = F.random_su3_algebra(dims, seed=6)
    eps = 1e-4
    L = lambda UU: np.vdot(chi, O.wilson(UU, psi, m)).real
    fd = (L(su3_exp(eps * X) @ U) - L(su3_exp(-eps * X) @ U)) / (2 * eps)
    an = np.sum(np.einsum("...ij,...ij->...", Fo.conj(), X).real)
    assert abs(fd - an) < 1e-6 * abs(an)
    # grad_psi = D^dagger chi: FD along a random complex direction
    d = F.spinor_field(dims, seed=9)
    Lp = lambda pp: np.vdot(chi, O.wilson(U, pp, m)).real
    fdp = (Lp(psi + 1e-3 * d) - Lp(psi - 1e-3 * d)) / 2e-3
    assert abs(fdp - np.vdot(O.wilson(U, chi, m, dag=True), d).real) < 1e-9 * abs(fdp)


def test_force_gauge_covariance(weak44):
    """Under U -> g U g(x+mu)^dag, chi, psi -> g chi, g psi: F_mu(x) -> g(x) F_mu(x) g(x)^dag."""
    dims, U, psi, chi = weak44
    g = F.gauge_transform(dims, seed=4)
    Up = np.empty_like(U)
    for mu in range(4):
        Up[..., mu, :, :] = g @ U[..., mu, :, :] @ shift(g, mu, +1).conj().swapaxes(-1, -2)
    tr = lambda v: np.einsum("...ab,...sb->...sa", g, v)
    F1 = O.force(O.link_grad(chi, psi, c=-0.5), U)
    F2 = O.force(O.link_grad(tr(chi), tr(psi), c=-0.5), Up)
    gg = g[..., None, :, :]
    np.testing.assert_allclose(F2, gg @ F1 @ gg.conj().swapaxes(-1, -2), atol=1e-12)


def test_dag_link_gradient_fd(weak44):
    """The dag variant differentiates L = Re <chi, D^dagger psi>."""
    dims, U, psi, chi = weak44
    G = O.link_grad(chi, psi, c=-0.5, dag=True)
    X = F.random_su3_algebra(dims, seed=7)
    eps = 1e-4
    L = lambda UU: np.vdot(chi, O.wilson(UU, psi, 0.1, dag=True)).real
    fd = (L(su3_exp(eps * X) @ U) - L(su3_exp(-eps * X) @ U)) / (2 * eps)
    an = np.sum(np.einsum("...ij,...ij->...", O.force(G, U).conj(), X).real)
    assert abs(fd - an) < 1e-6 * abs(an)


def test_dwf_link_gradient_fd():
    dims, Ls = (4, 4, 2, 2), 4
    U = F.gauge_field(dims, seed=1, kind="weak")
    psi, chi = F.spinor_field(dims, seed=2, Ls=Ls), F.spinor_field(dims, seed=3, Ls=Ls)
    G = O.link_grad(chi, psi, c=-0.5)
    X = F.random_su3_algebra(dims, seed=7)
    eps = 1e-4
    L = lambda UU: np.vdot(chi, O.dwf(UU, psi, 1.8, 0.01)).real
    fd = (L(su3_exp(eps * X) @ U) - L(su3_exp(-eps * X) @ U)) / (2 * eps)
    an = np.sum(np.einsum("...ij,...ij->...", O.force(G, U).conj(), X).real)
    assert abs(fd - an) < 1e-6 * abs(an)


# ------------------------------------------------------------------ pseudofermion force (P11) ---

def test_pseudofermion_dense_and_fd():
    dims = (2, 2, 2, 2)
    U = F.gauge_field(dims, seed=1, kind="haar")
    phi = F.spinor_field(dims, seed=5)
    op = O.Op.wilson(0.1)
    S, dS, X = O.pseudofermion(op, U, phi)
    D = dense_wilson(U, 0.1)
    S_dense = np.vdot(phi.ravel(), np.linalg.solve(D.conj().T @ D, phi.ravel())).real
    assert abs(S - S_dense) < 1e-10 * abs(S_dense)
    Xd = F.random_su3_algebra(dims, seed=8)
    eps = 1e-4
    def Sof(UU):
        Dd = dense_wilson(UU, 0.1)
        return np.vdot(phi.ravel(), np.linalg.solve(Dd.conj().T @ Dd, phi.ravel())).real
    fd = (Sof(su3_exp(eps * Xd) @ U) - Sof(su3_exp(-eps * Xd) @ U)) / (2 * eps)
    an = np.sum(np.einsum("...ij,...ij->...", O.force(dS, U).conj(), Xd).real)
    assert abs(fd - an) < 1e-6 * abs(an)


def test_pseudofermion_fd_44():
    dims = (4, 4, 4, 4)
    U = F.gauge_field(dims, seed=1, kind="haar")
    phi = F.spinor_field(dims, seed=5)
    op = O.Op.wilson(0.1)
    S, dS, _ = O.pseudofermion(op, U, phi)
    Xd = F.random_su3_algebra(dims, seed=8)
    eps = 1e-4
    Sp = O.pseudofermion(op, su3_exp(eps * Xd) @ U, phi)[0]
    Sm = O.pseudofermion(op, su3_exp(-eps * Xd) @ U, phi)[0]
    fd = (Sp - Sm) / (2 * eps)
    an = np.sum(np.einsum("...ij,...ij->...", O.force(dS, U).conj(), Xd).real)
    assert abs(fd - an) < 1e-6 * abs(an)


# ----------------------------------------------------------------------------- codecs (P12) ---

def test_fp16_codec_bound_and_exact_max():
    psi = F.spinor_field((4, 4, 4, 4), seed=2, Ls=4) * np.exp(np.random.default_rng(0).uniform(-8, 8, (4, 4, 4, 4, 4, 1, 1)))
    q, s = O.fp16_encode(psi, site_axes=2)
    assert q.dtype == np.float16 and s.dtype == np.float32 and s.shape == psi.shape[:5]
    back = O.fp16_decode(q, s)
    v32 = psi.astype(np.complex64)
    err = np.maximum(np.abs(back.real - v32.real), np.abs(back.imag - v32.imag))
    assert np.all(err <= (2.0 ** -11) * (1 + 2.0 ** -10) * s[..., None, None])
    # the largest real of each site is coded as exactly +-1
    amax = np.max(np.abs(q.reshape(q.shape[:5] + (-1,)).astype(np.float32)), axis=-1)
    np.testing.assert_array_equal(amax, 1.0)
    # zero sites stay zero
    z = np.zeros((2, 4, 3), dtype=complex)
    qz, sz = O.fp16_encode(z, site_axes=2)
    assert np.all(sz == 0) and np.all(qz == 0) and np.all(O.fp16_decode(qz, sz) == 0)


def test_float32_rounding_bound():
    psi = F.spinor_field((4, 4, 4, 4), seed=2)
    r = psi.astype(np.complex64).astype(np.complex128)
    assert np.max(np.abs(r.real - psi.real) / np.abs(psi.real)) <= 2.0 ** -24


def test_sampled_sites_match_whole_field():
    """The sampled evaluation is the same per-site definition as the whole-field one."""
    dims, Ls = (4, 2, 3, 2), 3
    U = F.gauge_field(dims, seed=1, kind="haar")
    psi4, psi5 = F.spinor_field(dims, seed=2), F.spinor_field(dims, seed=2, Ls=Ls)
    idx4 = np.array([0, 5, 17, 47])
    idx5 = np.array([0, 7, 50, 143])
    np.testing.assert_array_equal(O.sites(U, psi4, idx4, "hop", dag=True), O.hop(U, psi4, dag=True).reshape(-1, 4, 3)[idx4])
    np.testing.assert_array_equal(O.sites(U, psi4, idx4, "wilson", mass=0.1), O.wilson(U, psi4, 0.1).reshape(-1, 4, 3)[idx4])
    np.testing.assert_array_equal(O.sites(U, psi5, idx5, "dwf", M5=1.8, mf=0.01),
                                  O.dwf(U, psi5, 1.8, 0.01).reshape(-1, 4, 3)[idx5])
