"""GPU parity of the even-odd entry points (grid_dhop_cb, grid_m5inv, grid_solve_eo) against the
FP64 oracle's even-odd compositions (oracle.eo), called through the C ABI.

Tolerances as for the full-lattice operator: FP64 1e-13, FP32 1e-6 against the oracle on the
FP32-rounded inputs, FP16 storage 2e-3.
"""
import numpy as np
import pytest

import oracle.oracle as O
from oracle import eo
from paper_1512_03487_amd import fields as F

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-13, "f32": 1e-6, "f16s": 2e-3}


def _gm():
    import paper_1512_03487_amd as gm
    return gm


@pytest.fixture(scope="module", autouse=True)
def _announce():
    print("\n[gpu] test_gpu_eo", flush=True)


@pytest.mark.parametrize("dims,Ls", [((4, 4, 4, 4), 1), ((2, 4, 6, 8), 1), ((4, 2, 2, 4), 5), ((2, 2, 4, 4), 8)])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
def test_dhop_cb(gpu, dims, Ls, prec):
    from tests.gpu_util import as_prec, host, rel
    gm = _gm()
    U = F.gauge_field(dims, seed=1, kind="haar")
    psi = F.spinor_field(dims, seed=2, Ls=Ls if Ls > 1 else None)
    y = F.spinor_field(dims, seed=3, Ls=Ls if Ls > 1 else None)
    for p in (0, 1):
        Uk, pk, Ur, pr = as_prec(U, eo.pick(psi, 1 - p), prec)
        _, yk, _, yr = as_prec(U, eo.pick(y, p), prec)
        for dag in (False, True):
            got = host(gm.dhop_cb(Uk, pk, p, "hop", beta=0.75, dag=dag))
            assert rel(got, 0.75 * eo.hop_cb(Ur, pr, p, dag)) <= TOL[prec], (p, dag, "hop")
            if Ls == 1:
                got = host(gm.dhop_cb(Uk, pk, p, "wilson", y=yk, beta=-0.3, mass=0.1, dag=dag))
                ref = 4.1 * yr - 0.3 * eo.hop_cb(Ur, pr, p, dag)
            else:
                got = host(gm.dhop_cb(Uk, pk, p, "dwf", y=yk, beta=-0.25, M5=1.8, mf=0.05, dag=dag))
                ref = eo.m5(yr, 1.8, 0.05, dag) - 0.25 * eo.hop_cb(Ur, pr, p, dag)
            assert rel(got, ref) <= TOL[prec], (p, dag, "diag")


def _pick_dev(x, p):
    """Parity-p checkerboard (Lt, Lz, Ly, Lx/2, ...) of a full device field (Lt, Lz, Ly, Lx, ...)."""
    import torch
    Lt, Lz, Ly, Lx = x.shape[:4]
    ar = lambda n: torch.arange(n, device=x.device)
    xs = 2 * ar(Lx // 2).view(1, 1, 1, -1) + ((p + ar(Lt).view(-1, 1, 1, 1) + ar(Lz).view(1, -1, 1, 1)
                                                 + ar(Ly).view(1, 1, -1, 1)) & 1)
    idx = xs.view(xs.shape + (1,) * (x.dim() - 4)).expand((Lt, Lz, Ly, Lx // 2) + tuple(x.shape[4:]))
    return torch.gather(x, 3, idx).contiguous()


@pytest.mark.parametrize("prec", ["f32", "f16s"])
def test_dhop_cb_long_walks_match_full_lattice(gpu, prec):
    """24^4 x 12 (checkerboard walks of three slices over many blocks): H couples only opposite
    parities and the diagonal and fifth-dimension parts are parity-local, so the checkerboard
    operator on (psi of parity 1 - p, y of parity p) equals the full-lattice operator on the field
    holding both, restricted to parity p. The two sides run different kernels."""
    import torch
    from tests.gpu_util import cached
    gm = _gm()
    dev = torch.device("cuda:0")
    dims, Ls = (24, 24, 24, 24), 12
    U = torch.from_numpy(cached("gauge", dims, 1, kind="haar")).to(dev)
    g = torch.Generator(device=dev).manual_seed(11)
    shape = (dims[3], dims[2], dims[1], dims[0], Ls, 4, 3)
    full = torch.complex(torch.randn(shape, generator=g, device=dev), torch.randn(shape, generator=g, device=dev))
    if prec == "f32":
        Uk, fk = U.to(torch.complex64), full
        pick = _pick_dev
        as32 = lambda v: v
        tol = 1e-5
    else:
        Uk, fk = gm.convert_links(U, "f16s", "L12"), gm.convert_spinor(full, "f16s")
        pick = lambda v, p: gm.F16Spinor(_pick_dev(v.codes, p), _pick_dev(v.scale, p))
        as32 = lambda v: gm.convert_spinor(v, "f32")
        tol = 4e-3
    for dag in (False, True):
        ref_full = as32(gm.dwf(Uk, fk, 1.8, 0.05, dag=dag))
        hop_full = as32(gm.dhop(Uk, fk, "hop", dag=dag))
        for p in (0, 1):
            got = as32(gm.dhop_cb(Uk, pick(fk, 1 - p), p, "dwf", y=pick(fk, p), beta=-0.5, M5=1.8, mf=0.05, dag=dag))
            ref = _pick_dev(ref_full, p)
            assert float((got - ref).norm() / ref.norm()) <= tol, (prec, dag, p, "dwf")
            # the hopping term alone: at parity-p sites H sees only the parity 1 - p part
            got = as32(gm.dhop_cb(Uk, pick(fk, 1 - p), p, "hop", dag=dag))
            ref = _pick_dev(hop_full, p)
            assert float((got - ref).norm() / ref.norm()) <= tol, (prec, dag, p, "hop")


@pytest.mark.parametrize("prec", ["f32", "f16s"])
def test_dhop_cb_compressed_links(gpu, prec):
    from tests.gpu_util import as_prec, host, rel
    gm = _gm()
    dims = (4, 4, 2, 6)
    U = F.gauge_field(dims, seed=1, kind="haar")
    psi = F.spinor_field(dims, seed=2, Ls=4)
    Uk, pk, Ur, pr = as_prec(U, eo.pick(psi, 0), prec, "L12")
    got = host(gm.dhop_cb(Uk, pk, 1, "hop", beta=1.0, dag=True))
    assert rel(got, eo.hop_cb(Ur, pr, 1, True)) <= TOL[prec]


@pytest.mark.parametrize("Ls", [1, 3, 8, 16, 64])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
def test_m5inv(gpu, Ls, prec):
    from tests.gpu_util import as_prec, host, rel
    gm = _gm()
    dims = (2, 2, 2, 4) if Ls == 64 else (2, 4, 2, 4)
    U = F.gauge_field(dims, seed=1)
    psi = F.spinor_field(dims, seed=4, Ls=Ls)
    if Ls == 1:
        psi = psi.reshape(psi.shape[:4] + (1, 4, 3))
    _, pk, _, pr = as_prec(U, psi, prec)
    for dag in (False, True):
        got = host(gm.m5inv(pk, 1.8, 0.05, dag=dag))
        assert rel(got, eo.m5inv(pr, 1.8, 0.05, dag)) <= TOL[prec], (Ls, dag)
    # checkerboard-shaped input (half the sites)
    _, pk, _, pr = as_prec(U, eo.pick(psi, 1), prec)
    assert rel(host(gm.m5inv(pk, 1.8, 0.05)), eo.m5inv(pr, 1.8, 0.05)) <= TOL[prec]


@pytest.mark.parametrize("Ls", [5, 16])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
def test_m5inv_ragged_block(gpu, Ls, prec):
    """7 4D sites: the last block of 4 sites holds 3 (its staged records and its stores stop there)."""
    from tests.gpu_util import as_prec, host, rel
    gm = _gm()
    dims = (7, 1, 1, 1)
    U = F.gauge_field(dims, seed=1)
    psi = F.spinor_field(dims, seed=6, Ls=Ls)
    _, pk, _, pr = as_prec(U, psi, prec)
    for dag in (False, True):
        got = host(gm.m5inv(pk, 1.8, 0.05, dag=dag))
        assert rel(got, eo.m5inv(pr, 1.8, 0.05, dag)) <= TOL[prec], (Ls, dag)


def _kw(kind):
    return dict(mass=0.1) if kind == "wilson" else dict(M5=1.8, mf=0.1)


def _oracle_op(kind, Ls):
    return O.Op.wilson(0.1) if kind == "wilson" else O.Op.dwf(Ls, 1.8, 0.1)


@pytest.mark.parametrize("kind,dims,Ls", [("wilson", (4, 4, 4, 4), 1), ("wilson", (2, 4, 6, 8), 1),
                                          ("dwf", (4, 4, 4, 4), 8), ("dwf", (2, 2, 4, 6), 4), ("dwf", (2, 4, 2, 4), 6)])
@pytest.mark.parametrize("sloppy,fmt", [("f64", "L18"), ("f32", "L18"), ("f16s", "L12")])
def test_solve_eo(gpu, kind, dims, Ls, sloppy, fmt):
    from tests.gpu_util import dev, host, rel
    gm = _gm()
    U = F.gauge_field(dims, seed=1, kind="haar")
    b = F.spinor_field(dims, seed=3, Ls=Ls if Ls > 1 else None)
    tol = 1e-12
    x, st = gm.solve_eo(dev(U), dev(b), kind, tol=tol, sloppy=sloppy, link_fmt=fmt, **_kw(kind))
    xh = host(x)
    assert st["converged"] and st["status"] == 0
    # the CG criterion, checked with the oracle's Schur operator: |Mhat^+(bhat - Mhat x_e)| <= tol |Mhat^+ bhat|
    kw = _kw(kind)
    bh = eo.source(U, b, kind, **kw)
    xe = eo.pick(xh, 0)
    rhs = eo.schur(U, bh, kind, dag=True, **kw)
    rn = np.linalg.norm(rhs - eo.schur(U, eo.schur(U, xe, kind, **kw), kind, dag=True, **kw)) / np.linalg.norm(rhs)
    assert rn <= 1.05 * tol, rn
    # odd sites are the reconstruction from the even ones
    assert rel(eo.pick(xh, 1), eo.odd_solution(U, b, xe, kind, **kw)) <= 1e-12
    # reported full residual is the oracle's
    r_full = rel(O.apply(_oracle_op(kind, Ls), U, xh), b)
    assert abs(r_full - st["true_residual"]) <= 1e-3 * r_full + 1e-15
    assert r_full <= 1e-9


MOB_CASES = {"mobius": dict(M5=1.8, mf=0.1, b5=1.5, c5=0.5),      # alpha = 4.3, beta = -0.1
             "beta0": dict(M5=2.0, mf=0.1, b5=1.5, c5=0.5),       # beta = 0: M_ee = alpha = 4
             "shamir": dict(M5=1.8, mf=0.1, b5=1.0, c5=0.0)}      # the domain-wall M


@pytest.mark.parametrize("case", sorted(MOB_CASES))
@pytest.mark.parametrize("dims,Ls", [((4, 4, 4, 4), 8), ((2, 2, 4, 6), 4), ((2, 4, 2, 4), 6)])
@pytest.mark.parametrize("sloppy,fmt", [("f64", "L18"), ("f32", "L18"), ("f16s", "L12")])
def test_solve_eo_mobius(gpu, case, dims, Ls, sloppy, fmt):
    """Even-odd CG for the Moebius operator, checked with the oracle's Moebius blocks: the CG
    criterion on the Schur system, the odd-site reconstruction and the full residual. Ls = 4, 8
    take the three-kernel Schur operator in FP32 / FP16 storage, Ls = 6 the five-kernel one."""
    from oracle import mobius as OM
    from tests.gpu_util import dev, host, rel
    gm = _gm()
    kw = MOB_CASES[case]
    U = F.gauge_field(dims, seed=1, kind="haar")
    b = F.spinor_field(dims, seed=3, Ls=Ls)
    tol = 1e-12
    print(f"[gpu] solve_eo mobius {case} {dims} Ls={Ls} {sloppy}", flush=True)
    x, st = gm.solve_eo(dev(U), dev(b), "mobius", tol=tol, sloppy=sloppy, link_fmt=fmt, **kw)
    xh = host(x)
    assert st["converged"] and st["status"] == 0
    bh = eo.source_mobius(U, b, **kw)
    xe = eo.pick(xh, 0)
    rhs = eo.schur_mobius(U, bh, dag=True, **kw)
    rn = np.linalg.norm(rhs - eo.schur_mobius(U, eo.schur_mobius(U, xe, **kw), dag=True, **kw)) / np.linalg.norm(rhs)
    assert rn <= 1.05 * tol, rn
    assert rel(eo.pick(xh, 1), eo.odd_solution_mobius(U, b, xe, **kw)) <= 1e-12
    r_full = rel(OM.mobius(U, xh, **kw), b)
    assert abs(r_full - st["true_residual"]) <= 1e-3 * r_full + 1e-15
    assert r_full <= 1e-9


def test_solve_eo_mobius_matches_shamir_and_cg(gpu):
    """b5 = 1, c5 = 0 is the Shamir operator: the Moebius even-odd solution equals the domain-wall
    one, and the Moebius even-odd solve takes fewer iterations than CG on M^+ M."""
    from tests.gpu_util import dev, host, rel
    gm = _gm()
    dims, Ls = (4, 4, 4, 4), 8
    U, b = dev(F.gauge_field(dims, seed=1, kind="haar")), dev(F.spinor_field(dims, seed=3, Ls=Ls))
    xm, _ = gm.solve_eo(U, b, "mobius", M5=1.8, mf=0.1, b5=1.0, c5=0.0, tol=1e-12)
    xd, _ = gm.solve_eo(U, b, "dwf", M5=1.8, mf=0.1, tol=1e-12)
    assert rel(host(xm), host(xd)) <= 1e-10
    kw = dict(M5=1.8, mf=0.1, b5=1.5, c5=0.5)
    _, st_eo = gm.solve_eo(U, b, "mobius", tol=1e-10, **kw)
    mdb = gm.mobius(U, b, dag=True, **kw)
    _, st_full = gm.cg(U, mdb, "mobius", tol=1e-10, **kw)
    assert st_eo["iterations"] < 0.8 * st_full["iterations"], (st_eo["iterations"], st_full["iterations"])


def test_solve_eo_needs_fewer_iterations(gpu):
    """The even-odd system converges in fewer iterations than CG on M^+ M for the same M x = b."""
    from tests.gpu_util import dev, host, rel
    gm = _gm()
    dims, Ls = (4, 4, 4, 4), 8
    U = F.gauge_field(dims, seed=1, kind="haar")
    b = F.spinor_field(dims, seed=3, Ls=Ls)
    Ud, bd = dev(U), dev(b)
    _, st_eo = gm.solve_eo(Ud, bd, "dwf", M5=1.8, mf=0.1, tol=1e-10)
    mdb = gm.dwf(Ud, bd, 1.8, 0.1, dag=True)
    x, st_full = gm.cg(Ud, mdb, "dwf", M5=1.8, mf=0.1, tol=1e-10)
    assert rel(O.dwf(U, host(x), 1.8, 0.1), b) < 1e-7
    assert st_eo["iterations"] < 0.8 * st_full["iterations"], (st_eo["iterations"], st_full["iterations"])


def test_solve_eo_zero_source_and_warm_start(gpu):
    import torch
    from tests.gpu_util import dev
    gm = _gm()
    dims = (4, 4, 4, 4)
    U = dev(F.gauge_field(dims, seed=1, kind="haar"))
    b = torch.zeros((4, 4, 4, 4, 4, 4, 3), dtype=torch.complex128, device="cuda:0")
    x, st = gm.solve_eo(U, b, "dwf", M5=1.8, mf=0.1)
    assert st["converged"] and float(x.abs().max()) == 0.0
    b = dev(F.spinor_field(dims, seed=3, Ls=4))
    x, st = gm.solve_eo(U, b, "dwf", M5=1.8, mf=0.1, tol=1e-10)
    x2, st2 = gm.solve_eo(U, b, "dwf", M5=1.8, mf=0.1, tol=1e-10, x0=x)
    assert st2["iterations"] <= 2 and st2["true_residual"] <= 1e-8


@pytest.mark.slow
@pytest.mark.parametrize("sloppy,fmt", [("f64", "L18"), ("f32", "L18"), ("f16s", "L12")])
def test_config2_dwf_16_4_ls16_eo(gpu, sloppy, fmt):
    """The 16^4 x 16 domain-wall workload (M5 = 1.8, m_f = 0.01) solved for M x = b with even-odd CG."""
    from tests.gpu_util import cached, dev, host, rel
    gm = _gm()
    dims, Ls = (16, 16, 16, 16), 16
    U = cached("gauge", dims, 1, kind="haar")
    b = cached("spinor", dims, 3, Ls=Ls)
    x, st = gm.solve_eo(dev(U), dev(b), "dwf", M5=1.8, mf=0.01, tol=1e-10, sloppy=sloppy, link_fmt=fmt)
    r = rel(O.dwf(U, host(x), 1.8, 0.01), b)
    assert abs(r - st["true_residual"]) <= 1e-3 * r + 1e-15
    assert st["converged"] and r <= 1e-8, (r, st)
