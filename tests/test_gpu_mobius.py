"""GPU parity of the Moebius domain-wall operator (grid_mobius) and of CG on its normal equations
against the FP64 oracle (oracle.mobius), through the C ABI.

Tolerances: FP64 1e-13, FP32 1e-6 against the oracle on the FP32-rounded inputs, FP16 storage
4e-3 (the intermediate field chi = B psi is itself stored in FP16 with a per-site scale).
"""
import pytest

import oracle.oracle as O
from oracle import mobius as MB
from paper_1512_03487_amd import fields as F

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-13, "f32": 1e-6, "f16s": 4e-3}
B5, C5 = 1.5, 0.5


def _gm():
    import paper_1512_03487_amd as gm
    return gm


@pytest.fixture(scope="module", autouse=True)
def _announce():
    print("\n[gpu] test_gpu_mobius", flush=True)


@pytest.mark.parametrize("dims,Ls", [((4, 4, 4, 4), 8), ((2, 3, 4, 5), 5), ((4, 6, 2, 8), 4), ((2, 2, 2, 2), 1)])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
def test_mobius_operator(gpu, dims, Ls, prec):
    from tests.gpu_util import as_prec, host, rel
    gm = _gm()
    U = F.gauge_field(dims, seed=1, kind="haar")
    psi = F.spinor_field(dims, seed=2, Ls=Ls)
    if Ls == 1:
        psi = psi.reshape(psi.shape[:4] + (1, 4, 3))
    Uk, pk, Ur, pr = as_prec(U, psi, prec)
    for dag in (False, True):
        got = host(gm.mobius(Uk, pk, 1.8, 0.05, B5, C5, dag=dag))
        assert rel(got, MB.mobius(Ur, pr, 1.8, 0.05, B5, C5, dag)) <= TOL[prec], (dag,)


@pytest.mark.parametrize("prec", ["f32", "f16s"])
def test_mobius_compressed_links(gpu, prec):
    from tests.gpu_util import as_prec, host, rel
    gm = _gm()
    dims, Ls = (4, 4, 2, 6), 6
    U = F.gauge_field(dims, seed=1, kind="haar")
    psi = F.spinor_field(dims, seed=2, Ls=Ls)
    Uk, pk, Ur, pr = as_prec(U, psi, prec, "L12")
    for dag in (False, True):
        got = host(gm.mobius(Uk, pk, 1.8, 0.05, B5, C5, dag=dag))
        assert rel(got, MB.mobius(Ur, pr, 1.8, 0.05, B5, C5, dag)) <= TOL[prec]


@pytest.mark.parametrize("prec,tol", [("f64", 1e-14), ("f32", 1e-6)])
def test_shamir_limit_matches_grid_dhop(gpu, prec, tol):
    """b5 = 1, c5 = 0 reproduces the domain-wall operator of grid_dhop: in FP64 through the
    direction-parallel kernel's custom and standard forms, in FP32 through the column walk's
    (the same sums in another order, so agreement to rounding)."""
    from tests.gpu_util import as_prec, host, rel
    gm = _gm()
    dims, Ls = (4, 4, 4, 8), 8
    U, psi, _, _ = as_prec(F.gauge_field(dims, seed=1, kind="haar"), F.spinor_field(dims, seed=2, Ls=Ls), prec)
    for dag in (False, True):
        a = host(gm.mobius(U, psi, 1.8, 0.01, 1.0, 0.0, dag=dag))
        b = host(gm.dwf(U, psi, 1.8, 0.01, dag=dag))
        assert rel(a, b) <= tol, (dag,)


@pytest.mark.parametrize("sloppy,fmt", [("f64", "L18"), ("f32", "L18"), ("f16s", "L12")])
def test_mobius_cg(gpu, sloppy, fmt):
    from tests.gpu_util import dev, host, rel
    gm = _gm()
    dims, Ls = (4, 4, 4, 4), 8
    U = F.gauge_field(dims, seed=1, kind="haar")
    b = F.spinor_field(dims, seed=3, Ls=Ls)
    x, st = gm.cg(dev(U), dev(b), "mobius", M5=1.8, mf=0.1, b5=B5, c5=C5, tol=1e-10, sloppy=sloppy, link_fmt=fmt)
    assert st["converged"]
    r = rel(MB.normal(U, host(x), 1.8, 0.1, B5, C5), b)
    assert r <= 1.05e-10 and abs(r - st["true_residual"]) <= 1e-3 * r + 1e-16


@pytest.mark.parametrize("prec,fmt", [("f32", "L18"), ("f16s", "L12"), ("f16s", "L18"), ("f64", "L18")])
def test_mobius_16_4_ls16_bench_size(gpu, prec, fmt):
    """16^4 x 16, the size the benchmark times (the fused column walk over several time slices per
    thread in FP32 / FP16 storage, the two-pass form in FP64): M and M^dagger over the whole field,
    relative L2 and the worst per-site component error."""
    from tests.gpu_util import as_prec, cached, host, rel
    from tests.test_gpu_dhop import SITE_TOL, _site_err
    gm = _gm()
    dims, Ls = (16, 16, 16, 16), 16
    U = cached("gauge", dims, 1, kind="haar")
    psi = cached("spinor", dims, 2, Ls=Ls)
    Uk, pk, Ur, pr = as_prec(U, psi, prec, fmt)
    for dag in (False, True):
        got = host(gm.mobius(Uk, pk, 1.8, 0.01, B5, C5, dag=dag))
        ref = MB.mobius(Ur, pr, 1.8, 0.01, B5, C5, dag)
        assert rel(got, ref) <= TOL[prec], (prec, fmt, dag)
        assert _site_err(got.reshape(-1, 4, 3), ref.reshape(-1, 4, 3)) <= SITE_TOL[prec], (prec, fmt, dag)
