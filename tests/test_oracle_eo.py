"""Pins of the even-odd (red-black) oracle pieces.

The checkerboard operators are compositions of the already pinned full-lattice oracle; these tests
fix the compositions themselves: the checkerboard bookkeeping, the parity structure of H, the
fifth-dimension operator against the C oracle's domain-wall operator, its inverse, and the Schur
complement solve against a solve of the full system.
"""
import numpy as np
import pytest

import oracle.oracle as O
from oracle import eo
from paper_1512_03487_amd import fields as F
from tests.lattice_testlib import rel


def _rand5(dims, Ls, seed):
    return F.spinor_field(dims, seed=seed, Ls=Ls)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 4, 6, 8)])
def test_pick_embed_roundtrip_and_parity(dims):
    psi = F.spinor_field(dims, seed=2)
    e, o = eo.pick(psi, 0), eo.pick(psi, 1)
    lx, ly, lz, lt = dims
    assert e.shape == (lt, lz, ly, lx // 2, 4, 3)
    np.testing.assert_array_equal(eo.embed(e, 0) + eo.embed(o, 1), psi)
    par = eo.parity(psi.shape[:4])
    assert np.all(eo.embed(e, 0)[par == 1] == 0) and np.all(eo.embed(o, 1)[par == 0] == 0)
    # storage order: index (x // 2) of each row, the full site index halved
    t, z, y = 1, 1, 1
    xs = [x for x in range(lx) if (x + y + z + t) % 2 == 0]
    np.testing.assert_array_equal(e[t, z, y], psi[t, z, y, xs])


def test_odd_extent_rejected():
    with pytest.raises(ValueError):
        eo.pick(F.spinor_field((3, 4, 4, 4), seed=2), 0)


@pytest.mark.parametrize("dag", [False, True])
def test_hopping_term_changes_parity(dag):
    """H maps a field living on one parity to a field living on the other only."""
    dims = (4, 4, 4, 4)
    U = F.gauge_field(dims, seed=1)
    psi = F.spinor_field(dims, seed=2)
    par = eo.parity(psi.shape[:4])
    for p in (0, 1):
        out = O.hop(U, eo.embed(eo.pick(psi, p), p), dag)
        assert np.max(np.abs(out[par == p])) == 0
        np.testing.assert_allclose(eo.pick(out, 1 - p), eo.hop_cb(U, eo.pick(psi, p), 1 - p, dag), atol=0)
    # the two checkerboard blocks rebuild the full H
    full = O.hop(U, psi, dag)
    rebuilt = eo.merge(eo.hop_cb(U, eo.pick(psi, 1), 0, dag), eo.hop_cb(U, eo.pick(psi, 0), 1, dag))
    assert rel(rebuilt, full) < 1e-15


@pytest.mark.parametrize("dag", [False, True])
@pytest.mark.parametrize("Ls", [1, 2, 5])
def test_m5_is_dwf_minus_hopping(Ls, dag):
    """M = M5 - H/2 with the C oracle's M: fixes M5's projectors, shifts and wall factors."""
    dims, M5, mf = (2, 2, 4, 2), 1.8, 0.07
    U = F.gauge_field(dims, seed=1)
    psi = _rand5(dims, Ls, 3)
    lhs = eo.m5(psi, M5, mf, dag) - 0.5 * O.hop(U, psi, dag)
    assert rel(lhs, O.dwf(U, psi, M5, mf, dag)) < 1e-14


@pytest.mark.parametrize("dag", [False, True])
@pytest.mark.parametrize("Ls", [1, 2, 8])
def test_m5_inverse(Ls, dag):
    dims, M5, mf = (2, 2, 2, 2), 1.8, 0.05
    psi = _rand5(dims, Ls, 4)
    assert rel(eo.m5(eo.m5inv(psi, M5, mf, dag), M5, mf, dag), psi) < 1e-14
    assert rel(eo.m5inv(eo.m5(psi, M5, mf, dag), M5, mf, dag), psi) < 1e-14
    # the adjoint really is the adjoint: <chi, M5 psi> = <M5^dagger chi, psi>
    chi = _rand5(dims, Ls, 5)
    a = np.vdot(chi, eo.m5(psi, M5, mf))
    b = np.vdot(eo.m5(chi, M5, mf, True), psi)
    assert abs(a - b) < 1e-12 * abs(a)


@pytest.mark.parametrize("kind", ["wilson", "dwf"])
def test_schur_adjoint(kind):
    dims = (2, 2, 2, 4)
    U = F.gauge_field(dims, seed=1)
    Ls = 1 if kind == "wilson" else 4
    x = eo.pick(_rand5(dims, Ls, 6) if Ls > 1 else F.spinor_field(dims, seed=6), 0)
    y = eo.pick(_rand5(dims, Ls, 7) if Ls > 1 else F.spinor_field(dims, seed=7), 0)
    kw = dict(mass=0.1) if kind == "wilson" else dict(M5=1.8, mf=0.1)
    a = np.vdot(y, eo.schur(U, x, kind, **kw))
    b = np.vdot(eo.schur(U, y, kind, dag=True, **kw), x)
    assert abs(a - b) < 1e-13 * abs(a)


def _dense(apply, shape):
    n = int(np.prod(shape))
    cols = []
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        cols.append(apply(e.reshape(shape)).ravel())
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("kind", ["wilson", "dwf"])
def test_schur_complement_solve_equals_full_solve(kind):
    """x_e = Mhat^-1 bhat and x_o = M_oo^-1 (b_o - M_oe x_e) solve M x = b (dense, tiny lattice)."""
    dims = (2, 2, 2, 2)
    U = F.gauge_field(dims, seed=1)
    if kind == "wilson":
        kw, b = dict(mass=0.1), F.spinor_field(dims, seed=3)
        op = O.Op.wilson(0.1)
    else:
        kw, b = dict(M5=1.8, mf=0.1), _rand5(dims, 4, 3)
        op = O.Op.dwf(4, 1.8, 0.1)
    M = _dense(lambda v: O.apply(op, U, v), b.shape)
    x_full = np.linalg.solve(M, b.ravel()).reshape(b.shape)
    bh = eo.source(U, b, kind, **kw)
    Mh = _dense(lambda v: eo.schur(U, v, kind, **kw), bh.shape)
    x_e = np.linalg.solve(Mh, bh.ravel()).reshape(bh.shape)
    x = eo.merge(x_e, eo.odd_solution(U, b, x_e, kind, **kw))
    assert rel(x, x_full) < 1e-12
    assert rel(O.apply(op, U, x), b) < 1e-12


MOB = dict(M5=1.8, mf=0.1, b5=1.5, c5=0.5)


def test_mobius_diagonal_block_is_the_operator_without_hopping():
    """M_ee read off the full Moebius operator equals the matrix of its s-local part, the dense
    inverse inverts it, and the Shamir limit gives the domain-wall M5 (whose projectors and walls
    the C oracle fixes)."""
    dims, Ls = (2, 2, 2, 4), 4
    U = F.gauge_field(dims, seed=1)
    psi = eo.pick(_rand5(dims, Ls, 3), 0)
    blk = eo.mobius_block(U, psi, 0, 0, **MOB)
    A = eo.mobius_diag_matrix(Ls, MOB["M5"], MOB["mf"], MOB["b5"], MOB["c5"])
    direct = np.einsum("ij,...jc->...ic", A, psi.reshape(psi.shape[:4] + (Ls * 4, 3))).reshape(psi.shape)
    assert rel(blk, direct) < 1e-14
    assert rel(eo.mobius_diag_inv(blk, MOB["M5"], MOB["mf"], MOB["b5"], MOB["c5"]), psi) < 1e-13
    shamir = eo.mobius_block(U, psi, 0, 0, M5=1.8, mf=0.1, b5=1.0, c5=0.0)
    assert rel(shamir, eo.m5(psi, 1.8, 0.1)) < 1e-14
    for dag in (False, True):
        assert rel(eo.mobius_diag_inv(eo.mobius_block(U, psi, 0, 0, dag=dag, **MOB), MOB["M5"], MOB["mf"], MOB["b5"],
                                      MOB["c5"], dag), psi) < 1e-13


def test_mobius_schur_shamir_limit_and_adjoint():
    dims, Ls = (2, 2, 2, 4), 4
    U = F.gauge_field(dims, seed=1)
    x = eo.pick(_rand5(dims, Ls, 6), 0)
    y = eo.pick(_rand5(dims, Ls, 7), 0)
    # b5 = 1, c5 = 0 is the Shamir operator: the same Schur complement as the domain-wall one
    for dag in (False, True):
        a = eo.schur_mobius(U, x, 1.8, 0.1, 1.0, 0.0, dag)
        assert rel(a, eo.schur(U, x, "dwf", M5=1.8, mf=0.1, dag=dag)) < 1e-13
    a = np.vdot(y, eo.schur_mobius(U, x, **MOB))
    b = np.vdot(eo.schur_mobius(U, y, dag=True, **MOB), x)
    assert abs(a - b) < 1e-13 * abs(a)


def test_mobius_schur_complement_solve_equals_full_solve():
    """Moebius 2^4 x 4: x_e = Mhat^-1 bhat and x_o = M_oo^-1 (b_o - M_oe x_e) solve M x = b, with
    M the dense matrix of the full-lattice Moebius oracle."""
    from oracle import mobius as mob
    dims, Ls = (2, 2, 2, 2), 4
    U = F.gauge_field(dims, seed=1)
    b = _rand5(dims, Ls, 3)
    M = _dense(lambda v: mob.mobius(U, v, **MOB), b.shape)
    x_full = np.linalg.solve(M, b.ravel()).reshape(b.shape)
    bh = eo.source_mobius(U, b, **MOB)
    Mh = _dense(lambda v: eo.schur_mobius(U, v, **MOB), bh.shape)
    x_e = np.linalg.solve(Mh, bh.ravel()).reshape(bh.shape)
    x = eo.merge(x_e, eo.odd_solution_mobius(U, b, x_e, **MOB))
    assert rel(x, x_full) < 1e-12
    assert rel(mob.mobius(U, x, **MOB), b) < 1e-12
