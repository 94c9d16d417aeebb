"""GPU parity of the coarse stencil and the multigrid entry points (grid_coarse_stencil,
grid_mg_basis, grid_mg_restrict, grid_mg_prolong, grid_mg_coarse_op, grid_mg_solve, grid_mg_pcg)
against the FP64 oracle (oracle.mg), through the C ABI.

Tolerances: the linear maps (stencil, R, P, Galerkin operator, Gram-Schmidt of a given set)
1e-13 relative (FP64, summation order only); the setup's near-null vectors 1e-9 (sixteen CG
iterations on each side, different summation orders); GCR iterates after three steps 1e-9; the
full solve is gated on the oracle-recomputed true residual and the iteration count.
"""
import numpy as np
import pytest

import oracle.oracle as O
from oracle import mg
from paper_1512_03487_amd import fields as F

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _announce():
    print("\n[gpu] test_gpu_mg", flush=True)


def _gm():
    import paper_1512_03487_amd as gm
    return gm


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _vecs(dims, nvec, seed=11):
    return np.stack([F.spinor_field(dims, seed=seed + k) for k in range(nvec)])


@pytest.mark.parametrize("cdims,N", [((4, 2, 3, 2), 12), ((2, 1, 3, 4), 24), ((3, 3, 1, 1), 64), ((1, 1, 1, 2), 1)])
def test_coarse_stencil(gpu, cdims, N):
    from tests.gpu_util import dev, host
    gm = _gm()
    rng = np.random.default_rng(7)
    shp = (cdims[3], cdims[2], cdims[1], cdims[0])
    A = rng.standard_normal(shp + (9, N, N)) + 1j * rng.standard_normal(shp + (9, N, N))
    v = rng.standard_normal(shp + (N,)) + 1j * rng.standard_normal(shp + (N,))
    A_nat = np.ascontiguousarray(np.swapaxes(A, -1, -2))    # device layout [d][j][i] -> oracle [d][i][j]
    for dag in (False, True):
        got = host(gm.coarse_stencil(dev(A), dev(v), dag=dag))
        assert _rel(got, mg.coarse_apply(A_nat, v, dag=dag)) <= 1e-13, dag


@pytest.mark.parametrize("dims,block,nvec", [((4, 4, 4, 4), (2, 2, 2, 2), 6), ((4, 6, 2, 4), (1, 3, 2, 2), 3),
                                             ((4, 4, 2, 2), (4, 2, 2, 1), 1)])
def test_orthonormalise_restrict_prolong(gpu, dims, block, nvec):
    from tests.gpu_util import dev, host
    gm = _gm()
    U = F.gauge_field(dims, seed=1, kind="haar")
    v = _vecs(dims, nvec)
    vd = dev(v)
    gm.mg_basis(dev(U), vd, 0.1, block=block, setup_rounds=0)
    q = mg.orthonormalise(v, block)
    assert _rel(host(vd), q) <= 1e-13
    psi = F.spinor_field(dims, seed=2)
    vc = host(gm.mg_restrict(dev(q), dev(psi), block))
    assert _rel(vc, mg.restrict(q, psi, block)) <= 1e-13
    back = host(gm.mg_prolong(dev(q), dev(vc), block))
    assert _rel(back, mg.prolong(q, vc, block)) <= 1e-13


def test_near_null_setup(gpu):
    from tests.gpu_util import dev, host
    gm = _gm()
    dims, block, nvec, m = (4, 4, 4, 4), (2, 2, 2, 2), 4, 0.2
    U = F.gauge_field(dims, seed=1, kind="weak")
    v = _vecs(dims, nvec)
    vd = dev(v)
    gm.mg_basis(dev(U), vd, m, block=block, setup_rounds=2, setup_iters=8)
    ref = mg.orthonormalise(mg.near_null(U, v, m, 2, 8), block)
    assert _rel(host(vd), ref) <= 1e-9


def test_fp32_cycle(gpu):
    """The cycle in FP32 (minimal-residual smoother with FP32 links and FP64 inner products; R, P
    and the coarse solve reading FP32 copies of the basis and of A): the flexible GCR still reaches
    1e-10 (checked by the oracle) in about as many outer iterations."""
    from tests.gpu_util import dev, host
    gm = _gm()
    dims, block, nvec, m = (8, 8, 8, 8), (4, 4, 4, 4), 8, 0.05
    U = F.gauge_field(dims, seed=1, kind="weak")
    b = F.spinor_field(dims, seed=3)
    Ud = dev(U)
    qd = dev(_vecs(dims, nvec))
    gm.mg_basis(Ud, qd, m, block=block, setup_rounds=3, setup_iters=10)
    Ad = gm.mg_coarse_op(Ud, qd, m, block=block)
    its = {}
    for prec in ("f64", "f32"):
        x, st = gm.mg_solve(Ud, qd, Ad, dev(b), m, block=block, restart=8, coarse_iters=50, coarse_tol=0.05,
                            smooth_iters=4, cycle_prec=prec)
        res = float(np.linalg.norm(b - O.wilson(U, host(x), m)) / np.linalg.norm(b))
        assert st["converged"] and res <= 1.05e-10, (prec, res)
        its[prec] = st["iterations"]
    assert abs(its["f32"] - its["f64"]) <= 2, its


@pytest.mark.parametrize("setup_prec", ["f32", "f16s"])
def test_mixed_precision_setup(gpu, setup_prec):
    """Setup CG in mixed precision: the near-null vectors stay close to the FP64 setup's (the
    sloppy iterations perturb them at the sloppy precision's rounding level), and the basis still
    gives a converged multigrid solve in about as many outer iterations."""
    from tests.gpu_util import dev, host
    gm = _gm()
    dims, block, nvec, m = (8, 8, 8, 8), (4, 4, 4, 4), 8, 0.05
    U = F.gauge_field(dims, seed=1, kind="weak")
    b = F.spinor_field(dims, seed=3)
    Ud = dev(U)
    out, its = {}, {}
    for prec in ("f64", setup_prec):
        qd = dev(_vecs(dims, nvec))
        gm.mg_basis(Ud, qd, m, block=block, setup_rounds=3, setup_iters=10, setup_prec=prec)
        out[prec] = host(qd)
        Ad = gm.mg_coarse_op(Ud, qd, m, block=block)
        x, st = gm.mg_solve(Ud, qd, Ad, dev(b), m, block=block, restart=8, coarse_iters=50, coarse_tol=0.05)
        res = float(np.linalg.norm(b - O.wilson(U, host(x), m)) / np.linalg.norm(b))
        assert st["converged"] and res <= 1.05e-10, (prec, res)
        its[prec] = st["iterations"]
    assert _rel(out[setup_prec], out["f64"]) <= (1e-4 if setup_prec == "f32" else 5e-2), _rel(out[setup_prec], out["f64"])
    assert abs(its[setup_prec] - its["f64"]) <= 2, its


@pytest.mark.parametrize("dims,block,nvec,kind", [((8, 4, 2, 4), (2, 2, 2, 2), 3, "haar"),
                                                  ((4, 6, 4, 2), (1, 3, 2, 2), 4, "weak"),
                                                  ((4, 4, 4, 4), (4, 2, 1, 2), 2, "haar")])
def test_coarse_operator(gpu, dims, block, nvec, kind):
    from tests.gpu_util import dev, host
    gm = _gm()
    m = 0.1
    U = F.gauge_field(dims, seed=1, kind=kind)
    q = mg.orthonormalise(_vecs(dims, nvec), block)
    A = host(gm.mg_coarse_op(dev(U), dev(q), m, block=block))
    ref = mg.coarse_operator(U, q, m, block)
    assert np.max(np.abs(np.swapaxes(A, -1, -2) - ref)) <= 1e-13 * np.max(np.abs(ref))


def _setup(dims, block, nvec, m, kind="weak"):
    U = F.gauge_field(dims, seed=1, kind=kind)
    q = mg.orthonormalise(mg.near_null(U, _vecs(dims, nvec), m, 2, 8), block)
    return U, q, mg.coarse_operator(U, q, m, block)


def test_gcr_iterates_match_the_oracle(gpu):
    """Three preconditioned GCR steps (no convergence): the iterate equals the oracle's."""
    from tests.gpu_util import dev, host
    gm = _gm()
    dims, block, nvec, m = (4, 4, 4, 4), (2, 2, 2, 2), 6, 0.2
    U, q, A = _setup(dims, block, nvec, m)
    b = F.spinor_field(dims, seed=3)
    kw = dict(block=block, restart=2, coarse_iters=30, coarse_tol=0.05, smooth_iters=2)
    x, st = gm.mg_solve(dev(U), dev(q), dev(np.ascontiguousarray(np.swapaxes(A, -1, -2))), dev(b), m, maxiter=3,
                        raise_on_fail=False, **kw)
    xo, ito, _ = mg.fgcr(U, q, A, b, m, block, tol=1e-10, maxiter=3, restart=2, coarse_iters=30, coarse_tol=0.05,
                         smooth_iters=2)
    assert st["iterations"] == ito == 3
    assert _rel(host(x), xo) <= 1e-9


@pytest.mark.parametrize("dims,block,nvec,restart", [((4, 4, 4, 4), (2, 2, 2, 2), 6, 8), ((8, 4, 4, 4), (2, 2, 2, 2), 4, 4)])
@pytest.mark.parametrize("cycle_prec", ["f64", "f32"])
def test_mg_solve(gpu, dims, block, nvec, restart, cycle_prec):
    """Solves D x = b to 1e-10 (checked by the oracle) in as many outer iterations as the oracle's
    flexible GCR (within one; within two with the FP32 cycle, a slightly different preconditioner)."""
    from tests.gpu_util import dev, host
    gm = _gm()
    m = 0.2
    U, q, A = _setup(dims, block, nvec, m)
    b = F.spinor_field(dims, seed=3)
    Ud, qd = dev(U), dev(q)
    Ad = gm.mg_coarse_op(Ud, qd, m, block=block)
    x, st = gm.mg_solve(Ud, qd, Ad, dev(b), m, block=block, restart=restart, coarse_iters=40, tol=1e-10,
                        cycle_prec=cycle_prec)
    assert st["converged"]
    res = float(np.linalg.norm(b - O.wilson(U, host(x), m)) / np.linalg.norm(b))
    assert res <= 1.05e-10 and abs(res - st["true_residual"]) <= 1e-3 * res
    _, ito, _ = mg.fgcr(U, q, A, b, m, block, tol=1e-10, restart=restart, coarse_iters=40, coarse_tol=0.05,
                        smooth_iters=2)
    assert abs(st["iterations"] - ito) <= (1 if cycle_prec == "f64" else 2), (st["iterations"], ito)


def test_mg_full_pipeline_on_device(gpu):
    """Setup, coarse operator and solve all on the device from the same random vectors: solves
    D x = b to 1e-10 in fewer outer iterations than with an unimproved (random) basis."""
    from tests.gpu_util import dev, host
    gm = _gm()
    dims, block, nvec, m = (8, 8, 8, 8), (4, 4, 4, 4), 8, 0.05
    U = F.gauge_field(dims, seed=1, kind="weak")
    b = F.spinor_field(dims, seed=3)
    Ud = dev(U)
    its = {}
    for rounds in (0, 3):
        qd = dev(_vecs(dims, nvec))
        gm.mg_basis(Ud, qd, m, block=block, setup_rounds=rounds, setup_iters=10)
        Ad = gm.mg_coarse_op(Ud, qd, m, block=block)
        x, st = gm.mg_solve(Ud, qd, Ad, dev(b), m, block=block, restart=8, coarse_iters=50, coarse_tol=0.05)
        res = float(np.linalg.norm(b - O.wilson(U, host(x), m)) / np.linalg.norm(b))
        assert st["converged"] and res <= 1.05e-10
        its[rounds] = st["iterations"]
    assert its[3] < its[0], its


def test_recorded_coarse_solve_matches_direct_launches(gpu):
    """grid_mg_params.graph replays the coarse solve recorded once per solve: x, the iteration count
    and the residual equal those of direct launches bit for bit, for two solves in a row."""
    from tests.gpu_util import dev
    gm = _gm()
    dims, block, nvec, m = (8, 4, 4, 4), (2, 2, 2, 2), 4, 0.2
    U, q, A = _setup(dims, block, nvec, m)
    Ud, qd = dev(U), dev(q)
    Ad = gm.mg_coarse_op(Ud, qd, m, block=block)
    for seed in (3, 4):
        b = dev(F.spinor_field(dims, seed=seed))
        kw = dict(block=block, restart=4, coarse_iters=25, coarse_tol=0.05)
        x0, s0 = gm.mg_solve(Ud, qd, Ad, b, m, graph=False, **kw)
        x1, s1 = gm.mg_solve(Ud, qd, Ad, b, m, graph=True, **kw)
        assert s0["iterations"] == s1["iterations"] and s0["true_residual"] == s1["true_residual"]
        assert bool((x0 == x1).all())


def test_pcg_iterates_match_the_oracle(gpu):
    """Three multigrid pCG steps with a restart after two (no convergence): the iterate equals the
    oracle's flexible CG, written in CG form (N-conjugate directions, rho updated by N p)."""
    from tests.gpu_util import dev, host
    gm = _gm()
    dims, block, nvec, m = (4, 4, 4, 4), (2, 2, 2, 2), 6, 0.2
    U, q, A = _setup(dims, block, nvec, m)
    b = F.spinor_field(dims, seed=3)
    x, st = gm.mg_pcg(dev(U), dev(q), dev(np.ascontiguousarray(np.swapaxes(A, -1, -2))), dev(b), m, maxiter=3,
                      block=block, restart=2, coarse_iters=30, coarse_tol=0.05, smooth_iters=2, raise_on_fail=False)
    xo, ito, _ = mg.fcg(U, q, A, b, m, block, tol=1e-10, maxiter=3, restart=2, coarse_iters=30, coarse_tol=0.05,
                        smooth_iters=2)
    assert st["iterations"] == ito == 3 and st["restarts"] == 1
    assert _rel(host(x), xo) <= 1e-9


@pytest.mark.parametrize("dims,block,nvec,cycle_prec", [((4, 4, 4, 4), (2, 2, 2, 2), 6, "f64"),
                                                        ((8, 4, 4, 4), (2, 2, 2, 2), 4, "f64"),
                                                        ((8, 4, 4, 4), (2, 2, 2, 2), 4, "f32")])
def test_mg_pcg_solve(gpu, dims, block, nvec, cycle_prec):
    """Multigrid pCG solves D x = b to 1e-10 (checked by the oracle) in as many iterations as the
    oracle's flexible CG (within one; within three with the FP32 cycle, a slightly different
    preconditioner), and its graph-recorded coarse solves give the same x."""
    from tests.gpu_util import dev, host
    gm = _gm()
    m = 0.2
    U, q, A = _setup(dims, block, nvec, m)
    b = F.spinor_field(dims, seed=3)
    Ud, qd = dev(U), dev(q)
    Ad = gm.mg_coarse_op(Ud, qd, m, block=block)
    kw = dict(restart=8, coarse_iters=40, coarse_tol=0.05, smooth_iters=2, tol=1e-10)
    x, st = gm.mg_pcg(Ud, qd, Ad, dev(b), m, block=block, graph=False, cycle_prec=cycle_prec, **kw)
    assert st["converged"]
    res = float(np.linalg.norm(b - O.wilson(U, host(x), m)) / np.linalg.norm(b))
    assert res <= 1.05e-10 and abs(res - st["true_residual"]) <= 1e-3 * res
    _, ito, _ = mg.fcg(U, q, A, b, m, block, **kw)
    assert abs(st["iterations"] - ito) <= (1 if cycle_prec == "f64" else 3), (st["iterations"], ito)
    x1, s1 = gm.mg_pcg(Ud, qd, Ad, dev(b), m, block=block, graph=True, cycle_prec=cycle_prec, **kw)
    assert s1["iterations"] == st["iterations"] and bool((x1 == x).all())


@pytest.mark.parametrize("solver", ["mg_solve", "mg_pcg"])
def test_mg_status_warm_start_and_zero_source(gpu, solver):
    """Both multigrid solvers: stopping at maxiter returns GRID_ENOCONV with the iterate so far; a
    warm start at the converged solution takes no iterations; a zero source returns x = 0."""
    import torch
    from paper_1512_03487_amd import _lib
    from tests.gpu_util import dev
    gm = _gm()
    dims, block, nvec, m = (4, 4, 4, 4), (2, 2, 2, 2), 6, 0.2
    U, q, A = _setup(dims, block, nvec, m)
    b = dev(F.spinor_field(dims, seed=3))
    Ud, qd = dev(U), dev(q)
    Ad = gm.mg_coarse_op(Ud, qd, m, block=block)
    fn = getattr(gm, solver)
    kw = dict(block=block, restart=8, coarse_iters=40, coarse_tol=0.05, smooth_iters=2, tol=1e-10)
    x2, st2 = fn(Ud, qd, Ad, b, m, maxiter=2, raise_on_fail=False, **kw)
    assert st2["status"] == _lib.GRID_ENOCONV and st2["iterations"] == 2 and not st2["converged"]
    assert 1e-10 < st2["true_residual"] < 1.0
    x, st = fn(Ud, qd, Ad, b, m, **kw)
    assert st["converged"]
    x1, st1 = fn(Ud, qd, Ad, b, m, x0=x, **kw)
    assert st1["iterations"] == 0 and st1["converged"] and bool((x1 == x).all())
    x0, st0 = fn(Ud, qd, Ad, torch.zeros_like(b), m, **kw)
    assert st0["iterations"] == 0 and bool((x0 == 0).all())
