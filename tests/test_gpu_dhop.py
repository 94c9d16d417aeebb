"""GPU parity of grid_dhop / grid_dwf_mdag_m against the FP64 oracle (called through the C ABI).

Tolerances (relative L2 error over the whole field): FP64 1e-13, FP32 1e-6 against the oracle
evaluated on the FP32-rounded inputs, FP16 storage 2e-3 (the output itself is FP16-coded with a
per-site scale, error <= 2^-11 of the site maximum per component).
"""
import numpy as np
import pytest

import oracle.oracle as O
from paper_1512_03487_amd import fields as F

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-13, "f32": 1e-6, "f16s": 2e-3}


def _gm():
    import paper_1512_03487_amd as gm
    return gm


@pytest.fixture(scope="module", autouse=True)
def _announce():
    print("\n[gpu] test_gpu_dhop", flush=True)


def test_config0_wilson_d_and_ddag_4444(gpu):
    """4^4, Haar links, complex128, m = 0.1: D and D^dagger once."""
    from tests.gpu_util import dev, host, rel
    gm = _gm()
    dims = (4, 4, 4, 4)
    U, psi = F.gauge_field(dims, seed=1, kind="haar"), F.spinor_field(dims, seed=2)
    for dag in (False, True):
        out = host(gm.wilson(dev(U), dev(psi), 0.1, dag=dag))
        assert rel(out, O.wilson(U, psi, 0.1, dag)) <= 1e-13


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 3, 4, 5), (4, 6, 8, 10), (6, 4, 2, 8), (8, 8, 4, 3),
                                  (16, 8, 12, 4), (8, 4, 8, 2), (16, 8, 16, 6)])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("fmt", ["L18", "L12"])
def test_hop_and_wilson_parity(gpu, dims, prec, fmt):
    from tests.gpu_util import as_prec, host, rel
    gm = _gm()
    U = F.gauge_field(dims, seed=1, kind="haar")
    psi = F.spinor_field(dims, seed=2)
    Uk, pk, Ur, pr = as_prec(U, psi, prec, fmt)
    for dag in (False, True):
        got, ref = host(gm.dhop(Uk, pk, "hop", dag=dag)), O.hop(Ur, pr, dag)
        assert rel(got, ref) <= TOL[prec], (dims, prec, fmt, dag)
        assert _site_err(got.reshape(-1, 4, 3), ref.reshape(-1, 4, 3)) <= SITE_TOL[prec], (dims, prec, fmt, dag)
        got, ref = host(gm.wilson(Uk, pk, 0.1, dag=dag)), O.wilson(Ur, pr, 0.1, dag)
        assert rel(got, ref) <= TOL[prec], (dims, prec, fmt, dag)
        assert _site_err(got.reshape(-1, 4, 3), ref.reshape(-1, 4, 3)) <= SITE_TOL[prec], (dims, prec, fmt, dag)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_config1_16_4_weak_field_100_applications(gpu, prec):
    """16^4, weak-field links exp(0.3 i H): H applied 100 times to the same psi; each output equal."""
    import torch
    from tests.gpu_util import as_prec, host, rel
    gm = _gm()
    dims = (16, 16, 16, 16)
    U = F.gauge_field(dims, seed=1, kind="weak")
    psi = F.spinor_field(dims, seed=2)
    Uk, pk, Ur, pr = as_prec(U, psi, prec)
    first = gm.dhop(Uk, pk, "hop")
    out = torch.empty_like(first)
    for _ in range(100):
        gm.dhop(Uk, pk, "hop", out=out)
    torch.cuda.synchronize()
    assert torch.equal(out, first)     # bitwise reproducible
    assert rel(host(out), O.hop(Ur, pr)) <= TOL[prec]


@pytest.mark.parametrize("Ls", [1, 2, 5, 8, 16])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
def test_dwf_parity(gpu, Ls, prec):
    from tests.gpu_util import as_prec, host, rel
    gm = _gm()
    dims = (4, 4, 4, 6)
    U = F.gauge_field(dims, seed=1, kind="haar")
    psi = F.spinor_field(dims, seed=3, Ls=Ls)
    Uk, pk, Ur, pr = as_prec(U, psi, prec)
    for dag in (False, True):
        got, ref = host(gm.dwf(Uk, pk, 1.8, 0.01, dag=dag)), O.dwf(Ur, pr, 1.8, 0.01, dag)
        assert rel(got, ref) <= TOL[prec], (Ls, prec, dag)
        assert _site_err(got.reshape(-1, 4, 3), ref.reshape(-1, 4, 3)) <= SITE_TOL[prec], (Ls, prec, dag)
        # Ls-replicated hopping term on the 5D field
        got = host(gm.dhop(Uk, pk, "hop", dag=dag))
        assert rel(got, O.hop(Ur, pr, dag)) <= TOL[prec], (Ls, prec, dag)


@pytest.mark.parametrize("prec,fmt", [("f32", "L12"), ("f16s", "L12"), ("f32", "L18")])
def test_dwf_ls16_link_formats(gpu, prec, fmt):
    """Ls = 16 (one column of s-lanes per 16-lane row) on a lattice of several column blocks."""
    from tests.gpu_util import as_prec, host, rel
    gm = _gm()
    dims, Ls = (8, 4, 4, 6), 16
    U = F.gauge_field(dims, seed=4, kind="haar")
    psi = F.spinor_field(dims, seed=5, Ls=Ls)
    Uk, pk, Ur, pr = as_prec(U, psi, prec, fmt)
    for dag in (False, True):
        got = host(gm.dwf(Uk, pk, 1.8, 0.01, dag=dag))
        assert rel(got, O.dwf(Ur, pr, 1.8, 0.01, dag)) <= TOL[prec], (prec, fmt, dag)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_dwf_mdag_m(gpu, prec):
    from tests.gpu_util import as_prec, host, rel
    gm = _gm()
    dims, Ls = (4, 4, 6, 4), 8
    U = F.gauge_field(dims, seed=1, kind="haar")
    psi = F.spinor_field(dims, seed=3, Ls=Ls)
    Uk, pk, Ur, pr = as_prec(U, psi, prec)
    got = host(gm.dwf_mdag_m(Uk, pk, 1.8, 0.01))
    assert rel(got, O.normal(O.Op.dwf(Ls, 1.8, 0.01), Ur, pr)) <= 10 * TOL[prec]


# Per-component bound relative to the site scale s = max |Re|, |Im| over the site's 24 reals (of
# the oracle's output): FP16 storage codes the output with error <= 2^-11 s per component, plus the
# FP32 arithmetic; FP32 a few tens of roundings of terms of the inputs' size; FP64 likewise.
SITE_TOL = {"f64": 1e-12, "f32": 2.0 ** -16, "f16s": 2.0 ** -10}


def _site_err(got, ref) -> float:
    """max over sites of (max component error) / (site scale of ref)."""
    d = np.maximum(np.abs(got.real - ref.real), np.abs(got.imag - ref.imag)).reshape(len(ref), -1).max(axis=1)
    s = np.maximum(np.abs(ref.real), np.abs(ref.imag)).reshape(len(ref), -1).max(axis=1)
    return float(np.max(d / s))


def _sampled(gm, U, psi, prec, fmt, kind, n=4096, **kw):
    """(relative L2 error, worst per-site component error) on sampled sites, the first and last 64
    of them included, against the oracle evaluated site by site on the stored inputs."""
    from tests.gpu_util import as_prec, host, rel
    Uk, pk, Ur, pr = as_prec(U, psi, prec, fmt)
    got = host(gm.dhop(Uk, pk, kind, **kw)).reshape(-1, 4, 3)
    nsites = got.shape[0]
    rng = np.random.default_rng(0)
    idx = np.unique(np.concatenate([rng.integers(0, nsites, n), np.arange(64), np.arange(nsites - 64, nsites)]))
    ref = O.sites(Ur, pr, idx, kind, dag=kw.get("dag", False), mass=kw.get("mass", 0.0), M5=kw.get("M5", 0.0),
                  mf=kw.get("mf", 0.0))
    return rel(got[idx], ref), _site_err(got[idx], ref)


@pytest.mark.parametrize("dag", [False, True])
@pytest.mark.parametrize("prec,fmt", [("f32", "L18"), ("f32", "L12"), ("f16s", "L12"), ("f64", "L18")])
def test_config4_wilson_32_4_sampled(gpu, prec, fmt, dag):
    """32^4 (the throughput size), H and H^dagger: sampled sites, including the first and last 64."""
    gm = _gm()
    from tests.gpu_util import cached
    dims = (32, 32, 32, 32)
    U = cached("gauge", dims, 1, kind="haar")
    psi = cached("spinor", dims, 2)
    r, e = _sampled(gm, U, psi, prec, fmt, "hop", dag=dag)
    assert r <= TOL[prec] and e <= SITE_TOL[prec], (prec, fmt, dag, r, e)


@pytest.mark.parametrize("dag", [False, True])
@pytest.mark.parametrize("prec,fmt", [("f32", "L18"), ("f16s", "L12"), ("f32", "L12"), ("f16s", "L18")])
def test_config4_dwf_24_4_ls12_sampled(gpu, prec, fmt, dag):
    """24^4 x 12 domain wall, M and M^dagger, in the launch configuration the benchmark times (the
    column walk over three time slices per thread at this size)."""
    gm = _gm()
    from tests.gpu_util import cached
    dims = (24, 24, 24, 24)
    U = cached("gauge", dims, 1, kind="haar")
    psi = cached("spinor", dims, 3, Ls=12)
    r, e = _sampled(gm, U, psi, prec, fmt, "dwf", M5=1.8, mf=0.01, dag=dag)
    assert r <= TOL[prec] and e <= SITE_TOL[prec], (prec, fmt, dag, r, e)


def test_bitwise_determinism_dwf(gpu):
    import torch
    from tests.gpu_util import as_prec
    gm = _gm()
    dims = (8, 8, 8, 8)
    U = F.gauge_field(dims, seed=1, kind="haar")
    psi = F.spinor_field(dims, seed=3, Ls=8)
    for prec in ("f64", "f32", "f16s"):
        Uk, pk, _, _ = as_prec(U, psi, prec)
        a = gm.dwf(Uk, pk, 1.8, 0.01)
        b = gm.dwf(Uk, pk, 1.8, 0.01)
        torch.cuda.synchronize()
        if prec == "f16s":
            assert torch.equal(a.codes, b.codes) and torch.equal(a.scale, b.scale)
        else:
            assert torch.equal(a, b)


def test_zero_input_gives_zero_output(gpu):
    """Degenerate input: a zero spinor (FP16 scale 0) maps to zero in every precision."""
    from tests.gpu_util import as_prec, host
    gm = _gm()
    dims = (4, 4, 2, 2)
    U = F.gauge_field(dims, seed=1, kind="haar")
    psi = np.zeros(F.lattice_shape(dims) + (3, 4, 3), dtype=np.complex128)
    for prec in ("f64", "f32", "f16s"):
        Uk, pk, _, _ = as_prec(U, psi, prec)
        assert np.all(host(gm.dwf(Uk, pk, 1.8, 0.01)) == 0)
