"""GPU parity of the HMC entry points (grid_gauge_force, grid_link_exp, grid_hmc_energy,
grid_md_leapfrog) against the FP64 oracle (oracle.hmc), through the C ABI, plus the integrator's
reversibility and second-order energy error on the GPU.
"""
import numpy as np
import pytest

import oracle.oracle as O
from oracle import hmc as OH
from paper_1512_03487_amd import fields as F

pytestmark = pytest.mark.gpu

DWF = dict(kind="dwf", M5=1.8, mf=0.2)


def _gm():
    import paper_1512_03487_amd as gm
    return gm


@pytest.fixture(scope="module", autouse=True)
def _announce():
    print("\n[gpu] test_gpu_hmc", flush=True)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 4, 6, 3)])
def test_gauge_force(gpu, dims):
    from tests.gpu_util import dev, host, rel
    gm = _gm()
    U = F.gauge_field(dims, seed=1, kind="weak")
    assert rel(host(gm.gauge_force(dev(U), 5.7)), OH.gauge_force(U, 5.7)) <= 1e-13


def test_link_exp(gpu):
    from tests.gpu_util import dev, host, rel
    gm = _gm()
    dims = (2, 4, 2, 4)
    U = F.gauge_field(dims, seed=1, kind="haar")
    for scale in (0.05, 1.0, 7.0):     # small steps and ones that need squaring
        P = F.random_su3_algebra(dims, seed=6)
        Ud = dev(U)
        gm.link_exp(Ud, dev(P), scale)
        ref = np.einsum("...ij,...jk->...ik", OH.su3_exp(scale * P), U)
        assert rel(host(Ud), ref) <= 1e-13, scale


def test_energies(gpu):
    from tests.gpu_util import dev
    gm = _gm()
    dims, Ls = (4, 4, 4, 4), 4
    U = F.gauge_field(dims, seed=1, kind="weak")
    P = F.random_su3_algebra(dims, seed=7)
    phi = F.spinor_field(dims, seed=5, Ls=Ls)
    e = gm.hmc_energy(dev(U), dev(P), 5.5, dev(phi), tol=1e-12, **DWF)
    assert e["K"] == pytest.approx(OH.kinetic(P), rel=1e-13)
    assert e["S_G"] == pytest.approx(OH.gauge_action(U, 5.5), rel=1e-12)
    S_ref = OH.fermion_force(U, (O.Op.dwf(Ls, 1.8, 0.2), phi))[0]
    assert e["S_F"] == pytest.approx(S_ref, rel=1e-10)
    assert e["H"] == pytest.approx(e["K"] + e["S_G"] + e["S_F"], rel=1e-15)
    assert gm.hmc_energy(dev(U), dev(P), 5.5)["S_F"] == 0.0


@pytest.mark.parametrize("with_fermion", [False, True])
def test_leapfrog_matches_oracle(gpu, with_fermion):
    from tests.gpu_util import dev, host, rel
    gm = _gm()
    dims, Ls, beta = (2, 2, 2, 4), 4, 5.5
    U = F.gauge_field(dims, seed=1, kind="weak")
    P = F.random_su3_algebra(dims, seed=7)
    phi = F.spinor_field(dims, seed=5, Ls=Ls) if with_fermion else None
    Ud, Pd = dev(U), dev(P)
    st = gm.md_leapfrog(Ud, Pd, beta, 0.05, 4, dev(phi) if with_fermion else None, tol=1e-12, **DWF)
    ferm = (O.Op.dwf(Ls, 1.8, 0.2), phi) if with_fermion else None
    Ur, Pr = OH.leapfrog(U, P, beta, 0.05, 4, ferm)
    tol = 1e-12 if not with_fermion else 1e-8
    assert rel(host(Ud), Ur) <= tol and rel(host(Pd), Pr) <= tol
    assert st["failed_solves"] == 0 and st["solves"] == (5 if with_fermion else 0)


@pytest.mark.parametrize("with_fermion", [False, True])
def test_reversibility_and_energy_error(gpu, with_fermion):
    from tests.gpu_util import dev
    gm = _gm()
    dims, Ls, beta, tau = (4, 4, 4, 4), 4, 5.5, 0.5
    U = dev(F.gauge_field(dims, seed=1, kind="weak"))
    P = dev(F.random_su3_algebra(dims, seed=7))
    phi = dev(F.spinor_field(dims, seed=5, Ls=Ls)) if with_fermion else None
    kw = dict(tol=1e-12, **DWF)
    U1, P1 = U.clone(), P.clone()
    gm.md_leapfrog(U1, P1, beta, tau / 5, 5, phi, **kw)
    U2, P2 = U1.clone(), -P1
    gm.md_leapfrog(U2, P2, beta, tau / 5, 5, phi, **kw)
    tol = 1e-12 if not with_fermion else 1e-8
    assert float((U2 - U).abs().max()) < tol and float((P2 + P).abs().max()) < tol
    H0 = gm.hmc_energy(U, P, beta, phi, **kw)["H"]
    dH = []
    for n in (5, 10):
        Un, Pn = U.clone(), P.clone()
        gm.md_leapfrog(Un, Pn, beta, tau / n, n, phi, **kw)
        dH.append(abs(gm.hmc_energy(Un, Pn, beta, phi, **kw)["H"] - H0))
    assert 3.0 < dH[0] / dH[1] < 5.0, dH


def test_hmc_trajectories_pure_gauge(gpu):
    """Trajectories at beta = 5.7 from a weak-field start: the first trajectory's dH equals the
    oracle's for the same momenta; dH stays O(0.1) at eps = 1/80, most trajectories are accepted and
    the plaquette relaxes from its start."""
    import paper_1512_03487_amd.hmc as H
    from tests.gpu_util import dev
    dims, beta, eps, n = (4, 4, 4, 4), 5.7, 0.0125, 40
    U0 = F.gauge_field(dims, seed=1, kind="weak")
    P0 = H.gaussian_momenta(dims[::-1], np.random.default_rng(123))
    U1, P1 = OH.leapfrog(U0, P0, beta, eps, n)
    dH_ref = OH.hamiltonian(U1, P1, beta) - OH.hamiltonian(U0, P0, beta)
    rng = np.random.default_rng(123)
    U = dev(U0)
    acc = 0
    for k in range(4):
        U, ok, dH, info = H.trajectory(U, beta, eps, n, rng)
        if k == 0:
            assert dH == pytest.approx(dH_ref, rel=1e-8, abs=1e-10)
        acc += ok
        assert abs(dH) < 1.0
    assert acc >= 3
    assert abs(OH.plaquette(U.cpu().numpy()) - OH.plaquette(U0)) > 1e-3


@pytest.mark.parametrize("with_fermion", [False, True])
def test_omelyan_matches_oracle(gpu, with_fermion):
    from tests.gpu_util import dev, host, rel
    gm = _gm()
    dims, Ls, beta = (2, 2, 2, 4), 4, 5.5
    U = F.gauge_field(dims, seed=1, kind="weak")
    P = F.random_su3_algebra(dims, seed=7)
    phi = F.spinor_field(dims, seed=5, Ls=Ls) if with_fermion else None
    Ud, Pd = dev(U), dev(P)
    st = gm.md_leapfrog(Ud, Pd, beta, 0.1, 3, dev(phi) if with_fermion else None, tol=1e-12, integrator="omelyan",
                        **DWF)
    ferm = (O.Op.dwf(Ls, 1.8, 0.2), phi) if with_fermion else None
    Ur, Pr = OH.omelyan(U, P, beta, 0.1, 3, ferm)
    tol = 1e-12 if not with_fermion else 1e-8
    assert rel(host(Ud), Ur) <= tol and rel(host(Pd), Pr) <= tol
    assert st["solves"] == (7 if with_fermion else 0)


def test_omelyan_trajectory_and_reversibility(gpu):
    """A trajectory with the Omelyan integrator: dH equals the oracle's for the same momenta, and
    integrating back with -P returns to the start."""
    import paper_1512_03487_amd.hmc as H
    from tests.gpu_util import dev, host, rel
    gm = _gm()
    dims, beta, eps, n = (4, 4, 4, 4), 5.7, 0.05, 10
    U0 = F.gauge_field(dims, seed=1, kind="weak")
    P0 = H.gaussian_momenta(dims[::-1], np.random.default_rng(321))
    U1, P1 = OH.omelyan(U0, P0, beta, eps, n)
    dH_ref = OH.hamiltonian(U1, P1, beta) - OH.hamiltonian(U0, P0, beta)
    _, _, dH, _ = H.trajectory(dev(U0), beta, eps, n, np.random.default_rng(321), integrator="omelyan")
    assert dH == pytest.approx(dH_ref, rel=1e-8, abs=1e-10)
    Ud, Pd = dev(U0), dev(P0)
    gm.md_leapfrog(Ud, Pd, beta, eps, n, integrator="omelyan")
    Pd.neg_()
    gm.md_leapfrog(Ud, Pd, beta, eps, n, integrator="omelyan")
    assert rel(host(Ud), U0) <= 1e-12 and rel(host(Pd), -P0) <= 1e-12


@pytest.mark.parametrize("with_fermion", [False, True])
def test_force_gradient_matches_oracle(gpu, with_fermion):
    """Force-gradient steps equal the oracle's (which keeps consecutive outer kicks separate), with
    3 n + 1 force evaluations (solves) on the device, and integrating back with -P returns."""
    from tests.gpu_util import dev, host, rel
    gm = _gm()
    dims, Ls, beta = (2, 2, 2, 4), 4, 5.5
    U = F.gauge_field(dims, seed=1, kind="weak")
    P = F.random_su3_algebra(dims, seed=7)
    phi = F.spinor_field(dims, seed=5, Ls=Ls) if with_fermion else None
    Ud, Pd = dev(U), dev(P)
    kw = dict(tol=1e-12, integrator="force_gradient", **DWF)
    st = gm.md_leapfrog(Ud, Pd, beta, 0.1, 3, dev(phi) if with_fermion else None, **kw)
    ferm = (O.Op.dwf(Ls, 1.8, 0.2), phi) if with_fermion else None
    Ur, Pr = OH.force_gradient(U, P, beta, 0.1, 3, ferm)
    tol = 1e-12 if not with_fermion else 1e-8
    assert rel(host(Ud), Ur) <= tol and rel(host(Pd), Pr) <= tol
    assert st["solves"] == (10 if with_fermion else 0)
    Pd.neg_()
    gm.md_leapfrog(Ud, Pd, beta, 0.1, 3, dev(phi) if with_fermion else None, **kw)
    assert rel(host(Ud), U) <= 10 * tol and rel(host(Pd), -P) <= 10 * tol


@pytest.mark.parametrize("outer", ["leapfrog", "omelyan", "force_gradient"])
@pytest.mark.parametrize("with_fermion", [False, True])
def test_nested_time_scales_match_oracle(gpu, with_fermion, outer):
    """Two time scales (n_inner = 3) with leapfrog, Omelyan or force-gradient outer steps equal the
    oracle's nested integrators, with n + 1, 2 n + 1 or 3 n + 1 fermion solves; zero steps leave U
    and P unchanged."""
    from tests.gpu_util import dev, host, rel
    gm = _gm()
    dims, Ls, beta = (2, 2, 2, 4), 4, 5.5
    U = F.gauge_field(dims, seed=1, kind="weak")
    P = F.random_su3_algebra(dims, seed=7)
    phi = F.spinor_field(dims, seed=5, Ls=Ls) if with_fermion else None
    Ud, Pd = dev(U), dev(P)
    st = gm.md_leapfrog(Ud, Pd, beta, 0.1, 3, dev(phi) if with_fermion else None, tol=1e-12, n_inner=3,
                        integrator=outer, **DWF)
    ferm = (O.Op.dwf(Ls, 1.8, 0.2), phi) if with_fermion else None
    nested = {"leapfrog": OH.nested_leapfrog, "omelyan": OH.nested_omelyan,
              "force_gradient": OH.nested_force_gradient}[outer]
    Ur, Pr = nested(U, P, beta, 0.1, 3, ferm, 3)
    tol = 1e-12 if not with_fermion else 1e-8
    assert rel(host(Ud), Ur) <= tol and rel(host(Pd), Pr) <= tol
    assert st["solves"] == ({"leapfrog": 4, "omelyan": 7, "force_gradient": 10}[outer] if with_fermion else 0)
    U0, P0 = dev(U), dev(P)
    st = gm.md_leapfrog(U0, P0, beta, 0.1, 0, dev(phi) if with_fermion else None, tol=1e-12, n_inner=3,
                        integrator=outer, **DWF)
    assert bool((U0 == dev(U)).all()) and bool((P0 == dev(P)).all()) and st["solves"] == 0


@pytest.mark.parametrize("integrator,n,solves", [("leapfrog", 4, 5), ("force_gradient", 2, 7)])
def test_mobius_md_matches_oracle(gpu, integrator, n, solves):
    """Moebius fermions (b5 = 1.5, c5 = 0.5) in the molecular dynamics: the steps and the energy
    equal the oracle's (force -2 G(M X, B X) in the library, the Moebius CG in the oracle)."""
    from oracle.mobius import MobiusOp
    from tests.gpu_util import dev, host, rel
    gm = _gm()
    dims, Ls, beta = (2, 2, 2, 4), 4, 5.5
    mob = dict(kind="mobius", M5=1.8, mf=0.2, b5=1.5, c5=0.5)
    U = F.gauge_field(dims, seed=1, kind="weak")
    P = F.random_su3_algebra(dims, seed=7)
    phi = F.spinor_field(dims, seed=5, Ls=Ls)
    Ud, Pd, phid = dev(U), dev(P), dev(phi)
    ferm = (MobiusOp(1.8, 0.2, 1.5, 0.5), phi)
    e = gm.hmc_energy(Ud, Pd, beta, phid, tol=1e-12, **mob)
    assert e["S_F"] == pytest.approx(OH.fermion_force(U, ferm)[0], rel=1e-10)
    st = gm.md_leapfrog(Ud, Pd, beta, 0.1, n, phid, tol=1e-12, integrator=integrator, **mob)
    step = OH.leapfrog if integrator == "leapfrog" else OH.force_gradient
    Ur, Pr = step(U, P, beta, 0.1, n, ferm)
    assert rel(host(Ud), Ur) <= 1e-8 and rel(host(Pd), Pr) <= 1e-8
    assert st["solves"] == solves and st["failed_solves"] == 0


def test_mobius_trajectory_two_time_scales(gpu):
    """A trajectory with a Moebius pseudofermion (phi = M^dagger eta) on two time scales (Omelyan
    outer steps, two inner gauge steps): dH equals the oracle's for the same momenta and source."""
    import paper_1512_03487_amd.hmc as H
    from oracle.mobius import MobiusOp, mobius
    from tests.gpu_util import dev
    dims, Ls, beta, eps, n = (2, 2, 2, 4), 4, 5.5, 0.1, 3
    U0 = F.gauge_field(dims, seed=1, kind="weak")
    rng = np.random.default_rng(77)
    P0 = H.gaussian_momenta(dims[::-1], rng)
    eta = H.gaussian_spinor(dims[::-1] + (Ls, 4, 3), rng)
    phi = mobius(U0, eta, 1.8, 0.2, 1.5, 0.5, dag=True)
    ferm = (MobiusOp(1.8, 0.2, 1.5, 0.5), phi)
    U1, P1 = OH.nested_omelyan(U0, P0, beta, eps, n, ferm, 2)
    dH_ref = OH.hamiltonian(U1, P1, beta, ferm) - OH.hamiltonian(U0, P0, beta, ferm)
    fermion = dict(kind="mobius", Ls=Ls, M5=1.8, mf=0.2, b5=1.5, c5=0.5)
    _, _, dH, info = H.trajectory(dev(U0), beta, eps, n, np.random.default_rng(77), fermion=fermion,
                                  integrator="omelyan", n_inner=2, tol=1e-12)
    assert dH == pytest.approx(dH_ref, rel=1e-7, abs=1e-9)
    assert info["md"]["solves"] == 2 * n + 1 and info["md"]["failed_solves"] == 0
