"""GPU CG (FP64 and mixed precision) checked by the oracle: the true residual of every returned x
is recomputed on the CPU in FP64, and small systems are compared with the oracle's own solve.

A CG solution is unique only up to the tolerance, so x is compared with the oracle solution for
information (relative difference bounded by the condition number times tol), and the gate is
the oracle-recomputed true residual.
"""
import numpy as np
import pytest

import oracle.oracle as O
from paper_1512_03487_amd import fields as F

pytestmark = pytest.mark.gpu

TOL = 1e-10
# the oracle's recomputation differs from the kernel's own FP64 residual by rounding only
RES_SLACK = 1.05


@pytest.fixture(scope="module", autouse=True)
def _announce():
    print("\n[gpu] test_gpu_cg", flush=True)


def test_wilson_fp64_cg_4444(gpu):
    import paper_1512_03487_amd as gm
    from tests.gpu_util import dev
    dims = (4, 4, 4, 4)
    U, b = F.gauge_field(dims, seed=1, kind="haar"), F.spinor_field(dims, seed=3)
    x, st = gm.cg(dev(U), dev(b), kind="wilson", mass=0.1, tol=TOL, sloppy="f64", check_every=1)
    x = x.cpu().numpy()
    op = O.Op.wilson(0.1)
    assert st["converged"] and st["true_residual"] <= TOL
    assert O.true_residual(op, U, b, x) <= RES_SLACK * TOL
    xo, sto, ito, reso = O.cg(op, U, b, tol=TOL)
    assert sto == 0
    print(f"wilson 4^4: gpu {st['iterations']} it, oracle {ito} it, |x-xo|/|xo| = "
          f"{np.linalg.norm(x - xo) / np.linalg.norm(xo):.2e}")
    assert abs(st["iterations"] - ito) <= max(3, ito // 20)


@pytest.mark.parametrize("sloppy", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("kind", ["wilson", "dwf"])
def test_cg_ragged_blocks(gpu, kind, sloppy):
    """Full-lattice Wilson / domain-wall solves (operator epilogues carry r -= alpha A p and the
    norms) on a lattice whose site count fills neither operator schedule's blocks evenly."""
    import paper_1512_03487_amd as gm
    from tests.gpu_util import dev
    dims, Ls = (6, 4, 5, 6), (1 if kind == "wilson" else 3)
    U = F.gauge_field(dims, seed=7, kind="haar")
    b = F.spinor_field(dims, seed=8, Ls=Ls) if Ls > 1 else F.spinor_field(dims, seed=8)
    kw = dict(mass=0.1) if kind == "wilson" else dict(M5=1.8, mf=0.05)
    x, st = gm.cg(dev(U), dev(b), kind=kind, tol=TOL, sloppy=sloppy, check_every=4, **kw)
    op = O.Op.wilson(0.1) if kind == "wilson" else O.Op.dwf(Ls, 1.8, 0.05)
    res = O.true_residual(op, U, b, x.cpu().numpy())
    print(f"{kind} {sloppy} ragged: {st['iterations']} it, {st['reliable_updates']} RU, oracle residual {res:.2e}")
    assert st["converged"] and res <= RES_SLACK * TOL
    if sloppy == "f64":
        _, sto, ito, _ = O.cg(op, U, b, tol=TOL)
        assert sto == 0 and abs(st["iterations"] - ito) <= max(3, ito // 20), (st["iterations"], ito)


@pytest.mark.parametrize("dims", [(8, 8, 4, 6), (16, 8, 8, 4)])
@pytest.mark.parametrize("sloppy,fmt", [("f32", "L18"), ("f32", "L12"), ("f16s", "L12")])
def test_wilson_cg_tiled_lattices(gpu, dims, sloppy, fmt):
    """Mixed-precision Wilson solves on lattices the tiled time walk covers (x, y multiples of 8, z
    of 4): its fused epilogues carry the norms and r -= alpha A p; one tile per slice in the first
    (every face wraps onto the tile itself)."""
    import paper_1512_03487_amd as gm
    from tests.gpu_util import dev
    U = F.gauge_field(dims, seed=7, kind="haar")
    b = F.spinor_field(dims, seed=8)
    x, st = gm.cg(dev(U), dev(b), kind="wilson", mass=0.1, tol=TOL, sloppy=sloppy, link_fmt=fmt, check_every=4)
    res = O.true_residual(O.Op.wilson(0.1), U, b, x.cpu().numpy())
    print(f"wilson {dims} {sloppy} {fmt}: {st['iterations']} it, {st['reliable_updates']} RU, residual {res:.2e}")
    assert st["converged"] and res <= RES_SLACK * TOL


@pytest.mark.parametrize("sloppy,fmt", [("f64", "L18"), ("f32", "L18"), ("f32", "L12"), ("f16s", "L18"),
                                        ("f16s", "L12")])
def test_dwf_cg_modes(gpu, sloppy, fmt):
    import paper_1512_03487_amd as gm
    from tests.gpu_util import dev
    dims, Ls = (4, 4, 4, 8), 8
    U, b = F.gauge_field(dims, seed=1, kind="haar"), F.spinor_field(dims, seed=3, Ls=Ls)
    x, st = gm.cg(dev(U), dev(b), kind="dwf", M5=1.8, mf=0.01, tol=TOL, sloppy=sloppy, link_fmt=fmt,
                  delta=0.1, check_every=5)
    op = O.Op.dwf(Ls, 1.8, 0.01)
    res = O.true_residual(op, U, b, x.cpu().numpy())
    print(f"dwf {sloppy}/{fmt}: {st['iterations']} it, {st['reliable_updates']} reliable updates, "
          f"kernel residual {st['true_residual']:.2e}, oracle residual {res:.2e}")
    assert st["converged"] and res <= RES_SLACK * TOL


def test_warm_start_and_zero_source(gpu):
    import torch
    import paper_1512_03487_amd as gm
    from tests.gpu_util import dev
    dims, Ls = (4, 4, 4, 4), 4
    U, b = F.gauge_field(dims, seed=1, kind="haar"), F.spinor_field(dims, seed=3, Ls=Ls)
    Ud, bd = dev(U), dev(b)
    x1, st1 = gm.cg(Ud, bd, kind="dwf", tol=1e-4)
    x2, st2 = gm.cg(Ud, bd, kind="dwf", tol=TOL, x0=x1)
    x3, st3 = gm.cg(Ud, bd, kind="dwf", tol=TOL)
    assert st2["converged"] and st2["iterations"] < st3["iterations"]
    assert O.true_residual(O.Op.dwf(Ls, 1.8, 0.01), U, b, x2.cpu().numpy()) <= RES_SLACK * TOL
    z, stz = gm.cg(Ud, torch.zeros_like(bd), kind="dwf", tol=TOL)
    assert stz["converged"] and stz["iterations"] == 0 and torch.count_nonzero(z) == 0


def test_maxiter_and_breakdown_status(gpu):
    import paper_1512_03487_amd as gm
    from paper_1512_03487_amd import _lib
    from tests.gpu_util import dev
    dims, Ls = (4, 4, 4, 4), 4
    U, b = F.gauge_field(dims, seed=1, kind="haar"), F.spinor_field(dims, seed=3, Ls=Ls)
    x, st = gm.cg(dev(U), dev(b), kind="dwf", tol=TOL, maxiter=7, check_every=3, raise_on_fail=False)
    assert st["status"] == _lib.GRID_ENOCONV and st["iterations"] == 7 and not st["converged"]
    bad = b.copy()
    bad[0, 0, 0, 0, 0, 0, 0] = np.nan      # the host-detected breakdown path (NaN residual)
    x, st = gm.cg(dev(U), dev(bad), kind="dwf", tol=TOL, check_every=2, raise_on_fail=False)
    assert st["status"] == _lib.GRID_EBREAKDOWN
    with pytest.raises(_lib.GridError):
        gm.cg(dev(U), dev(b), kind="dwf", tol=TOL, maxiter=2)


@pytest.mark.slow
@pytest.mark.parametrize("sloppy", ["f64", "f32", "f16s"])
def test_config2_dwf_16_4_ls16(gpu, sloppy):
    """16^4 x 16, M5 = 1.8, mf = 0.01, Haar links: true residual 1e-10, recomputed by the oracle."""
    import paper_1512_03487_amd as gm
    from tests.gpu_util import cached, dev
    dims, Ls = (16, 16, 16, 16), 16
    U, b = cached("gauge", dims, 1, kind="haar"), cached("spinor", dims, 3, Ls=Ls)
    x, st = gm.cg(dev(U), dev(b), kind="dwf", M5=1.8, mf=0.01, tol=TOL, sloppy=sloppy,
                  link_fmt="L12" if sloppy == "f16s" else "L18")
    res = O.true_residual(O.Op.dwf(Ls, 1.8, 0.01), U, b, x.cpu().numpy())
    print(f"config2 {sloppy}: {st['iterations']} it, {st['reliable_updates']} RU, {st['seconds']:.3f} s, "
          f"oracle residual {res:.3e}", flush=True)
    assert st["converged"] and res <= RES_SLACK * TOL


@pytest.mark.slow
@pytest.mark.parametrize("sloppy,fmt", [("f32", "L18"), ("f16s", "L12")])
def test_dwf_cg_24_4_ls12(gpu, sloppy, fmt):
    """24^4 x 12 (the throughput size: sloppy iterations on three-slice walks with the fused
    epilogues), M5 = 1.8, mf = 0.01, Haar links, to a true residual of 1e-8 recomputed by the
    oracle."""
    import paper_1512_03487_amd as gm
    from tests.gpu_util import cached, dev
    dims, Ls, tol = (24, 24, 24, 24), 12, 1e-8
    U, b = cached("gauge", dims, 1, kind="haar"), cached("spinor", dims, 3, Ls=Ls)
    x, st = gm.cg(dev(U), dev(b), kind="dwf", M5=1.8, mf=0.01, tol=tol, sloppy=sloppy, link_fmt=fmt)
    res = O.true_residual(O.Op.dwf(Ls, 1.8, 0.01), U, b, x.cpu().numpy())
    print(f"dwf 24^4x12 {sloppy}: {st['iterations']} it, {st['reliable_updates']} RU, oracle residual {res:.3e}",
          flush=True)
    assert st["converged"] and res <= RES_SLACK * tol


@pytest.mark.parametrize("solver,kind,sloppy,check", [
    ("cg", "dwf", "f64", 10), ("cg", "dwf", "f32", 3), ("cg", "dwf", "f16s", 4), ("cg", "wilson", "f32", 7),
    ("cg", "mobius", "f32", 5), ("eo", "dwf", "f32", 3), ("eo", "wilson", "f16s", 6)])
def test_graph_segments_match_direct_launches(gpu, solver, kind, sloppy, check):
    """Recorded iteration segments (grid_cg_params.graph) replay the direct path's kernels with the
    same arguments: the solution, iteration count, reliable updates and residual are identical.
    Each solve replays a segment tens of times with the solver's host checks, reliable updates and
    synchronisations in between; an odd check_every exercises both starting parities."""
    import paper_1512_03487_amd as gm
    from tests.gpu_util import dev
    dims, Ls = (4, 4, 4, 8), (1 if kind == "wilson" else 8)
    U = dev(F.gauge_field(dims, seed=1, kind="haar"))
    b = dev(F.spinor_field(dims, seed=3, Ls=Ls) if Ls > 1 else F.spinor_field(dims, seed=3))
    kw = dict(kind=kind, mass=0.1, M5=1.8, mf=0.05, tol=TOL, sloppy=sloppy, check_every=check)
    if kind == "mobius":
        kw.update(b5=1.5, c5=0.5)
    run = gm.cg if solver == "cg" else gm.solve_eo
    out = [run(U, b, graph=g, **kw) for g in (False, True, True)]
    (x0, s0), (x1, s1), (x2, s2) = out
    for x, s in ((x1, s1), (x2, s2)):
        assert s["converged"] and s["iterations"] == s0["iterations"]
        assert s.get("reliable_updates") == s0.get("reliable_updates")
        assert s["true_residual"] == s0["true_residual"]
        assert bool((x == x0).all()), "graph replay differs from direct launches"
    assert s0["iterations"] > 2 * check


@pytest.mark.parametrize("solver,sloppy", [("cg", "f64"), ("cg", "f16s"), ("eo", "f16s"), ("mobius", "f32")])
def test_fused_reductions_reproducible(gpu, solver, sloppy):
    """The operators' fused norms and residual updates sum their partials in a fixed order (the
    last wavefront to arrive adds the block's sums in order): two identical solves give bitwise
    identical solutions, iteration counts and residuals."""
    import paper_1512_03487_amd as gm
    from tests.gpu_util import dev
    dims, Ls = (8, 4, 4, 6), 8
    U, b = F.gauge_field(dims, seed=2, kind="haar"), F.spinor_field(dims, seed=4, Ls=Ls)
    runs = []
    for _ in range(2):
        if solver == "eo":
            x, st = gm.solve_eo(dev(U), dev(b), kind="dwf", M5=1.8, mf=0.05, tol=TOL, sloppy=sloppy)
        elif solver == "mobius":
            x, st = gm.cg(dev(U), dev(b), "mobius", M5=1.8, mf=0.05, b5=1.5, c5=0.5, tol=TOL, sloppy=sloppy)
        else:
            x, st = gm.cg(dev(U), dev(b), kind="dwf", M5=1.8, mf=0.05, tol=TOL, sloppy=sloppy)
        runs.append((x.cpu().numpy(), st))
    (x0, s0), (x1, s1) = runs
    assert s0["converged"] and s0["iterations"] == s1["iterations"]
    assert s0["true_residual"] == s1["true_residual"]
    assert np.array_equal(x0, x1)
