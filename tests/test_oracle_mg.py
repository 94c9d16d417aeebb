"""Pins of the multigrid oracle (oracle.mg): block orthonormalisation (QR properties), the
Galerkin coarse operator against a brute-force R D P built column by column from the pinned
Wilson operator, a free-field closed form (coarse Wilson operator with shifted mass and hopping
scaled by 1/b), gamma5-hermiticity, gauge invariance, the stencil adjoint, Galerkin orthogonality
of the coarse-grid correction, the coarse CGNR, the MR smoother, and the preconditioned GCR's
solution against CG. Multigrid pCG: textbook CG iterates with the identity preconditioner, its
preconditioner without smoothing equal to the dense P (A_c^dagger A_c)^-1 R (Hermitian, positive),
one step with an exact preconditioner, and its solution against CG with and without restarts.
"""
import numpy as np
import pytest

import oracle.oracle as O
from oracle import mg
from paper_1512_03487_amd import fields as F

# chiral basis written out independently of the oracle: gamma_k = [[0, -i s_k], [i s_k, 0]],
# gamma_4 = [[0, 1], [1, 0]]
_S = [np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]])]
_Z = np.zeros((2, 2))
GAMMA = [np.block([[_Z, -1j * s], [1j * s, _Z]]) for s in _S] + [np.block([[_Z, np.eye(2)], [np.eye(2), _Z]])]


def _vecs(dims, nvec, seed=11):
    return np.stack([F.spinor_field(dims, seed=seed + k) for k in range(nvec)])


def _dense_coarse(A):
    """Dense matrix of the stencil by applying it to unit coarse vectors."""
    shp = A.shape[:4] + (A.shape[-1],)
    n = int(np.prod(shp))
    M = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        M[:, j] = mg.coarse_apply(A, e.reshape(shp)).ravel()
    return M


def test_orthonormalise_is_blockwise_qr():
    dims, block, nvec = (4, 4, 2, 4), (2, 2, 2, 2), 4
    v = _vecs(dims, nvec)
    q = mg.orthonormalise(v, block)
    cd = mg.coarse_dims(dims, block)
    rng = np.random.default_rng(3)
    vc = rng.standard_normal((cd[3], cd[2], cd[1], cd[0], 2 * nvec)) + 1j * rng.standard_normal(
        (cd[3], cd[2], cd[1], cd[0], 2 * nvec))
    # P^dagger P = 1
    assert np.max(np.abs(mg.restrict(q, mg.prolong(q, vc, block), block) - vc)) < 1e-13
    # triangular: <q_j, v_k> = 0 for j > k on every aggregate and chirality, real positive for j = k
    c = np.stack([mg.restrict(q, v[k], block) for k in range(nvec)])    # c[k][..., chi nvec + j]
    for chi in (0, 1):
        for k in range(nvec):
            for j in range(nvec):
                cj = c[k][..., chi * nvec + j]
                if j > k:
                    assert np.max(np.abs(cj)) < 1e-13
                if j == k:
                    assert np.max(np.abs(cj.imag)) < 1e-13 and np.min(cj.real) > 0
    # span preserved: v_k = sum_{j <= k} <q_j, v_k> q_j, chirality by chirality
    for k in range(nvec):
        back = mg.prolong(q, c[k], block)
        assert np.max(np.abs(back - v[k])) < 1e-12


def test_free_field_constant_basis_gives_the_coarse_wilson_operator():
    """Unit links and a basis constant on each aggregate (one vector per upper/lower spin pair and
    colour): A_0 = 4 + m - sum_mu (b_mu - 1)/b_mu, A_{+mu} = -(1 - gamma_mu)/(2 b_mu),
    A_{-mu} = -(1 + gamma_mu)/(2 b_mu), component n = 3 spin + colour."""
    dims, block, m = (8, 4, 4, 6), (2, 4, 1, 3), 0.1
    U = F.gauge_field(dims, kind="unit")
    shp = F.lattice_shape(dims)
    v = np.zeros((6,) + shp + (4, 3), dtype=np.complex128)
    for k in range(6):
        sp, c = divmod(k, 3)
        v[k][..., sp, c] = 1.0
        v[k][..., 2 + sp, c] = 1.0
    q = mg.orthonormalise(v, block)
    A = mg.coarse_operator(U, q, m, block)
    I3 = np.eye(3)
    A0 = (4 + m - sum((b - 1) / b for b in block)) * np.eye(12)
    assert np.max(np.abs(A[..., 0, :, :] - A0)) < 1e-13
    for mu in range(4):
        fwd = -np.kron(np.eye(4) - GAMMA[mu], I3) / (2 * block[mu])
        bwd = -np.kron(np.eye(4) + GAMMA[mu], I3) / (2 * block[mu])
        assert np.max(np.abs(A[..., 1 + 2 * mu, :, :] - fwd)) < 1e-13, mu
        assert np.max(np.abs(A[..., 2 + 2 * mu, :, :] - bwd)) < 1e-13, mu


@pytest.mark.parametrize("dims,block", [((8, 4, 2, 4), (2, 2, 2, 2)), ((4, 6, 4, 2), (1, 3, 2, 2))])
def test_stencil_equals_brute_force_galerkin(dims, block):
    """The stencil (split by hop direction and aggregate faces) equals R D P computed column by
    column with the pinned Wilson operator, and its adjoint is the conjugate transpose."""
    nvec, m = 3, 0.2
    U = F.gauge_field(dims, seed=1, kind="haar")
    q = mg.orthonormalise(_vecs(dims, nvec), block)
    A = mg.coarse_operator(U, q, m, block)
    M = _dense_coarse(A)
    cd = mg.coarse_dims(dims, block)
    shp = (cd[3], cd[2], cd[1], cd[0], 2 * nvec)
    n = int(np.prod(shp))
    G = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        G[:, j] = mg.restrict(q, O.wilson(U, mg.prolong(q, e.reshape(shp), block), m), block).ravel()
    assert np.max(np.abs(M - G)) < 1e-13 * np.max(np.abs(G))
    # adjoint of the stencil, and gamma5-hermiticity G5 A G5 = A^dagger
    Md = np.zeros_like(M)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        Md[:, j] = mg.coarse_apply(A, e.reshape(shp), dag=True).ravel()
    assert np.max(np.abs(Md - M.conj().T)) < 1e-13 * np.max(np.abs(M))
    g5 = np.tile(np.r_[np.ones(nvec), -np.ones(nvec)], n // (2 * nvec))
    assert np.max(np.abs(g5[:, None] * M * g5[None, :] - M.conj().T)) < 1e-13 * np.max(np.abs(M))


def test_coarse_operator_is_gauge_invariant():
    dims, block, nvec, m = (4, 4, 4, 4), (2, 2, 2, 2), 3, 0.1
    U = F.gauge_field(dims, seed=1, kind="haar")
    g = F.gauge_transform(dims, seed=4)
    Ug = np.empty_like(U)
    for mu, ax in ((0, 3), (1, 2), (2, 1), (3, 0)):
        Ug[..., mu, :, :] = np.einsum("...ij,...jk,...lk->...il", g, U[..., mu, :, :], np.roll(g, -1, axis=ax).conj())
    v = _vecs(dims, nvec)
    vg = np.einsum("...ab,k...sb->k...sa", g, v)
    A = mg.coarse_operator(U, mg.orthonormalise(v, block), m, block)
    Ag = mg.coarse_operator(Ug, mg.orthonormalise(vg, block), m, block)
    assert np.max(np.abs(A - Ag)) < 1e-13


def test_coarse_correction_is_galerkin_orthogonal_and_cgnr_solves():
    dims, block, nvec, m = (4, 4, 4, 4), (2, 2, 2, 2), 3, 0.1
    U = F.gauge_field(dims, seed=1, kind="haar")
    q = mg.orthonormalise(_vecs(dims, nvec), block)
    A = mg.coarse_operator(U, q, m, block)
    r = F.spinor_field(dims, seed=3)
    rc = mg.restrict(q, r, block)
    shp = rc.shape
    ec = np.linalg.solve(_dense_coarse(A), rc.ravel()).reshape(shp)
    z = mg.prolong(q, ec, block)
    # R (r - D P A_c^-1 R r) = 0
    assert np.max(np.abs(mg.restrict(q, r - O.wilson(U, z, m), block))) < 1e-12 * np.max(np.abs(rc))
    # CGNR run to a tight tolerance reproduces the dense solve
    e2 = mg.coarse_cgnr(A, rc, 500, 1e-13)
    assert np.linalg.norm(e2 - ec) < 1e-10 * np.linalg.norm(ec)
    # and stops early on a loose one, with its normal residual below that bound
    e3 = mg.coarse_cgnr(A, rc, 500, 0.1)
    nr = np.linalg.norm(mg.coarse_apply(A, rc - mg.coarse_apply(A, e3), dag=True))
    assert nr <= 0.1 * np.linalg.norm(mg.coarse_apply(A, rc, dag=True))


def test_mr_smoothing_never_increases_the_residual():
    dims, block, nvec, m = (4, 4, 4, 4), (2, 2, 2, 2), 3, 0.1
    U = F.gauge_field(dims, seed=1, kind="haar")
    q = mg.orthonormalise(_vecs(dims, nvec), block)
    A = mg.coarse_operator(U, q, m, block)
    r = F.spinor_field(dims, seed=3)
    res = [np.linalg.norm(r - O.wilson(U, mg.precondition(U, q, A, r, m, block, 20, 0.1, nu), m))
           for nu in range(5)]
    assert all(b <= a * (1 + 1e-14) for a, b in zip(res, res[1:])), res
    assert res[-1] < res[0]
    # one MR step leaves a residual orthogonal to t = D s (its defining property)
    z0 = mg.precondition(U, q, A, r, m, block, 20, 0.1, 0)
    z1 = mg.precondition(U, q, A, r, m, block, 20, 0.1, 1)
    t = O.wilson(U, r - O.wilson(U, z0, m), m)
    s1 = r - O.wilson(U, z1, m)
    assert abs(np.vdot(t, s1)) < 1e-12 * np.linalg.norm(t) * np.linalg.norm(s1)


def test_preconditioned_gcr_solves_the_wilson_system():
    """x from multigrid-preconditioned GCR has |b - D x| <= tol |b| and agrees with the CG solution
    of D^dagger D x = D^dagger b within the condition number times the tolerances; the setup's
    near-null vectors cut the iteration count against random ones."""
    dims, block, nvec, m = (4, 4, 4, 4), (2, 2, 2, 2), 6, 0.2
    U = F.gauge_field(dims, seed=1, kind="weak")
    b = F.spinor_field(dims, seed=3)
    op = O.Op.wilson(m)
    v0 = _vecs(dims, nvec)
    counts = {}
    for rounds in (0, 2):
        q = mg.orthonormalise(mg.near_null(U, v0, m, rounds, 8) if rounds else v0, block)
        A = mg.coarse_operator(U, q, m, block)
        x, it, res = mg.fgcr(U, q, A, b, m, block, tol=1e-10, restart=8, coarse_iters=40, coarse_tol=0.05,
                             smooth_iters=2)
        assert res <= 1e-10 and O.true_residual(op, U, O.wilson(U, b, m, dag=True), x) < 1e-8
        counts[rounds] = it
    xc, st, _, _ = O.cg(op, U, O.wilson(U, b, m, dag=True), tol=1e-12)
    assert st == 0 and np.linalg.norm(x - xc) < 1e-7 * np.linalg.norm(xc)
    assert counts[2] < counts[0], counts


def test_fcg_without_preconditioner_is_textbook_cg():
    """With the identity in place of the cycle (and no restart within the steps compared), the
    flexible CG's iterates are those of plain CG on D^dagger D x = D^dagger b."""
    dims, m = (4, 4, 2, 4), 0.1
    U = F.gauge_field(dims, seed=1, kind="haar")
    b = F.spinor_field(dims, seed=3)
    q = mg.orthonormalise(_vecs(dims, 2), (2, 2, 2, 2))
    A = mg.coarse_operator(U, q, m, (2, 2, 2, 2))
    for k in (1, 2, 5):
        x, it, _ = mg.fcg(U, q, A, b, m, (2, 2, 2, 2), tol=1e-300, maxiter=k, restart=16, precondition=False)
        xc, _, _, _ = O.cg(O.Op.wilson(m), U, O.wilson(U, b, m, dag=True), tol=1e-300, maxiter=k)
        assert it == k and np.linalg.norm(x - xc) < 1e-11 * np.linalg.norm(xc), k


def test_coarse_part_of_the_pcg_preconditioner():
    """Without smoothing and with the coarse systems solved tightly, M = K G5 K G5 is
    P A_c^-1 G5 A_c^-1 G5 R = P (A_c^dagger A_c)^-1 R: equal to that dense formula, Hermitian and
    positive."""
    dims, block, nvec, m = (4, 4, 4, 4), (2, 2, 2, 2), 3, 0.1
    U = F.gauge_field(dims, seed=1, kind="haar")
    q = mg.orthonormalise(_vecs(dims, nvec), block)
    A = mg.coarse_operator(U, q, m, block)
    Ad = _dense_coarse(A)
    a, r = F.spinor_field(dims, seed=3), F.spinor_field(dims, seed=4)
    Mr = mg.normal_cycle(U, q, A, r, m, block, 2000, 1e-14, 0)
    Ma = mg.normal_cycle(U, q, A, a, m, block, 2000, 1e-14, 0)
    rc = mg.restrict(q, r, block)
    ref = mg.prolong(q, np.linalg.solve(Ad.conj().T @ Ad, rc.ravel()).reshape(rc.shape), block)
    assert np.linalg.norm(Mr - ref) < 1e-10 * np.linalg.norm(ref)
    assert abs(np.vdot(a, Mr) - np.conj(np.vdot(r, Ma))) < 1e-10 * abs(np.vdot(a, Mr))
    assert np.vdot(r, Mr).real > 0 and abs(np.vdot(r, Mr).imag) < 1e-10 * np.vdot(r, Mr).real


def test_fcg_with_an_exact_cycle_converges_in_one_step():
    """One-site aggregates with nvec = 6 make P unitary and A_c = R D P the whole operator; the
    preconditioner without smoothing then applies (D^dagger D)^-1 and the flexible CG stops after
    one step."""
    dims, m = (2, 2, 2, 4), 0.2
    U = F.gauge_field(dims, seed=1, kind="weak")
    b = F.spinor_field(dims, seed=3)
    block = (1, 1, 1, 1)
    q = mg.orthonormalise(_vecs(dims, 6), block)
    A = mg.coarse_operator(U, q, m, block)
    x, it, res = mg.fcg(U, q, A, b, m, block, tol=1e-10, coarse_iters=5000, coarse_tol=1e-14, smooth_iters=0)
    assert it == 1 and res <= 1e-10


def test_multigrid_pcg_solves_the_wilson_system():
    """Multigrid pCG reaches |b - D x| <= tol |b|, agrees with the CG solution, and takes fewer
    iterations than CG on the same normal equations."""
    dims, block, nvec, m = (4, 4, 4, 4), (2, 2, 2, 2), 6, 0.05
    U = F.gauge_field(dims, seed=1, kind="weak")
    b = F.spinor_field(dims, seed=3)
    q = mg.orthonormalise(mg.near_null(U, _vecs(dims, nvec), m, 2, 8), block)
    A = mg.coarse_operator(U, q, m, block)
    x, it, res = mg.fcg(U, q, A, b, m, block, tol=1e-10, restart=64, coarse_iters=40, coarse_tol=0.05,
                        smooth_iters=2)
    assert res <= 1e-10
    xc, st, its_cg, _ = O.cg(O.Op.wilson(m), U, O.wilson(U, b, m, dag=True), tol=1e-12)
    assert st == 0 and np.linalg.norm(x - xc) < 1e-7 * np.linalg.norm(xc)
    assert 2 * it < its_cg, (it, its_cg)
    # restarts from the true residual every four directions: still converges
    x4, it4, res4 = mg.fcg(U, q, A, b, m, block, tol=1e-10, maxiter=400, restart=4, coarse_iters=40,
                           coarse_tol=0.05, smooth_iters=2)
    assert res4 <= 1e-10 and np.linalg.norm(x4 - xc) < 1e-7 * np.linalg.norm(xc)
