"""GPU adjoint kernels against the oracle gradient, plus autograd and the pseudofermion force.

Gradients use the convention dL/dRe + i dL/dIm (PyTorch's, for a real loss). The FP32 kernel is
compared with the oracle gradient on FP32-rounded inputs; central finite differences in FP32 at
eps = 1e-4 would carry ~1e-3 rounding noise, so the finite-difference checks are the oracle's pins
(FP64) and here the FP64 kernel is also checked against an FP64 central difference directly.
"""
import numpy as np
import pytest

import oracle.oracle as O
from paper_1512_03487_amd import fields as F

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-13, "f32": 2e-6}


@pytest.fixture(scope="module", autouse=True)
def _announce():
    print("\n[gpu] test_gpu_backward", flush=True)


def _inputs(dims, prec, Ls=None, kind="weak"):
    from tests.gpu_util import dev
    U = F.gauge_field(dims, seed=1, kind=kind)
    psi = F.spinor_field(dims, seed=2, Ls=Ls)
    chi = F.spinor_field(dims, seed=3, Ls=Ls)
    if prec == "f32":
        U, psi, chi = (a.astype(np.complex64) for a in (U, psi, chi))
    ref = tuple(a.astype(np.complex128) for a in (U, psi, chi))
    return (dev(U), dev(psi), dev(chi)), ref


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (12, 12, 12, 12), (2, 3, 4, 5)])
@pytest.mark.parametrize("dag", [False, True])
def test_wilson_backward(gpu, prec, dims, dag):
    import paper_1512_03487_amd as gm
    from tests.gpu_util import rel
    (U, psi, chi), (Ur, pr, cr) = _inputs(dims, prec)
    gp, gu = gm.dhop_backward(U, psi, chi, "wilson", dag=dag, mass=0.1)
    assert rel(gp.cpu().numpy(), O.wilson(Ur, cr, 0.1, dag=not dag)) <= TOL[prec]
    G = O.link_grad(cr, pr, c=-0.5, dag=dag)
    assert rel(gu.cpu().numpy(), G) <= TOL[prec]
    _, fu = gm.dhop_backward(U, psi, chi, "wilson", dag=dag, mass=0.1, want_psi=False, force=True)
    assert rel(fu.cpu().numpy(), O.force(G, Ur)) <= 5 * TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_hop_and_dwf_backward(gpu, prec):
    import paper_1512_03487_amd as gm
    from tests.gpu_util import rel
    (U, psi, chi), (Ur, pr, cr) = _inputs((4, 4, 2, 6), prec)
    gp, gu = gm.dhop_backward(U, psi, chi, "hop")
    assert rel(gp.cpu().numpy(), O.hop(Ur, cr, dag=True)) <= TOL[prec]
    assert rel(gu.cpu().numpy(), O.link_grad(cr, pr, c=1.0)) <= TOL[prec]
    (U, psi, chi), (Ur, pr, cr) = _inputs((4, 4, 2, 6), prec, Ls=6)
    for dag in (False, True):
        gp, gu = gm.dhop_backward(U, psi, chi, "dwf", dag=dag, M5=1.8, mf=0.01)
        assert rel(gp.cpu().numpy(), O.dwf(Ur, cr, 1.8, 0.01, dag=not dag)) <= TOL[prec]
        assert rel(gu.cpu().numpy(), O.link_grad(cr, pr, c=-0.5, dag=dag)) <= TOL[prec]


def test_config3_fd_on_gpu_fp64(gpu):
    """12^4: the FP64 kernel's force against an FP64 central difference of the oracle's L."""
    import paper_1512_03487_amd as gm
    from tests.lattice_testlib import su3_exp
    dims = (12, 12, 12, 12)
    (U, psi, chi), (Ur, pr, cr) = _inputs(dims, "f64")
    _, Fk = gm.dhop_backward(U, psi, chi, "wilson", mass=0.1, want_psi=False, force=True)
    X = F.random_su3_algebra(dims, seed=6)
    eps = 1e-4

    def L(UU):
        return float(np.vdot(cr, O.wilson(UU, pr, 0.1)).real)

    fd = (L(su3_exp(eps * X) @ Ur) - L(su3_exp(-eps * X) @ Ur)) / (2 * eps)
    an = float(np.sum(np.einsum("...ij,...ij->...", Fk.cpu().numpy().conj(), X).real))
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_autograd_dhopfn(gpu):
    import torch
    import paper_1512_03487_amd as gm
    from tests.gpu_util import rel
    (U, psi, chi), (Ur, pr, cr) = _inputs((4, 4, 4, 6), "f64")
    U = U.clone().requires_grad_(True)
    psi = psi.clone().requires_grad_(True)
    out = gm.DhopFn.apply(U, psi, "wilson", False, 0.1)
    loss = torch.vdot(chi.reshape(-1), out.reshape(-1)).real
    loss.backward()
    assert rel(psi.grad.cpu().numpy(), O.wilson(Ur, cr, 0.1, dag=True)) <= 1e-13
    assert rel(U.grad.cpu().numpy(), O.link_grad(cr, pr, c=-0.5)) <= 1e-13


def test_pseudofermion_force_8_4(gpu):
    """S = phi^dagger (D^dagger D)^-1 phi at 8^4 (Haar, m = 0.1): S, dS/dU and dS/dphi vs the oracle."""
    import torch
    import paper_1512_03487_amd as gm
    from tests.gpu_util import dev, rel
    dims = (8, 8, 8, 8)
    U = F.gauge_field(dims, seed=1, kind="haar")
    phi = F.spinor_field(dims, seed=5)
    S_ref, dS_ref, X_ref = O.pseudofermion(O.Op.wilson(0.1), U, phi, tol=1e-13)
    Ud = dev(U).requires_grad_(True)
    phid = dev(phi).requires_grad_(True)
    S = gm.PseudofermionActionFn.apply(Ud, phid, "wilson", 0.1, 1.8, 0.01, 1e-13)
    S.backward()
    assert abs(float(S) - S_ref) <= 1e-12 * abs(S_ref)
    assert rel(Ud.grad.cpu().numpy(), dS_ref) <= 1e-9
    assert rel(phid.grad.cpu().numpy(), 2 * X_ref) <= 1e-9
    F_gpu = O.force(Ud.grad.cpu().numpy(), U)
    assert rel(F_gpu, O.force(dS_ref, U)) <= 1e-9


def test_autograd_dhopfn_fp32_12_4(gpu):
    """12^4 weak field, FP32 DhopFn (Wilson D, m = 0.1): grad_psi and grad_U against the oracle
    gradient evaluated on the FP32-rounded inputs."""
    import torch
    import paper_1512_03487_amd as gm
    from tests.gpu_util import rel
    (U, psi, chi), (Ur, pr, cr) = _inputs((12, 12, 12, 12), "f32")
    U = U.clone().requires_grad_(True)
    psi = psi.clone().requires_grad_(True)
    out = gm.DhopFn.apply(U, psi, "wilson", False, 0.1)
    loss = torch.vdot(chi.reshape(-1), out.reshape(-1)).real
    loss.backward()
    assert rel(psi.grad.cpu().numpy(), O.wilson(Ur, cr, 0.1, dag=True)) <= TOL["f32"]
    assert rel(U.grad.cpu().numpy(), O.link_grad(cr, pr, c=-0.5)) <= TOL["f32"]


def _pf_case(kind):
    if kind == "wilson":
        dims, Ls, op, kw = (8, 8, 8, 8), None, O.Op.wilson(0.1), dict(mass=0.1)
    else:
        dims, Ls, op, kw = (4, 4, 4, 4), 8, O.Op.dwf(8, 1.8, 0.01), dict(M5=1.8, mf=0.01)
    U = F.gauge_field(dims, seed=1, kind="haar")
    phi = F.spinor_field(dims, seed=5, Ls=Ls)
    return U, phi, op, kw


@pytest.mark.parametrize("kind", ["wilson", "dwf"])
def test_pseudofermion_action_abi(gpu, kind):
    """grid_pseudofermion_action: S, the scaled dS/dU (raw and su(3)-projected) and dS/dphi against
    the oracle (Wilson 8^4, m = 0.1; domain wall 4^4 x 8, M5 = 1.8, mf = 0.01; Haar links)."""
    import paper_1512_03487_amd as gm
    from tests.gpu_util import dev, rel
    U, phi, op, kw = _pf_case(kind)
    S_ref, dS_ref, X_ref = O.pseudofermion(op, U, phi, tol=1e-13)
    Ud, phid = dev(U), dev(phi)
    S, X, gU, gphi, st = gm.pseudofermion_action(Ud, phid, kind, tol=1e-13, grad_scale=0.75, want_U=True,
                                                 want_phi=True, **kw)
    assert st["converged"]
    assert abs(S - S_ref) <= 1e-11 * abs(S_ref)
    assert rel(X.cpu().numpy(), X_ref) <= 1e-9
    assert rel(gU.cpu().numpy(), 0.75 * dS_ref) <= 1e-9
    assert rel(gphi.cpu().numpy(), 1.5 * X_ref) <= 1e-9
    S2, _, Fk, _, _ = gm.pseudofermion_action(Ud, phid, kind, tol=1e-13, want_U=True, force=True, **kw)
    assert S2 == S                                           # same solve from zero, same fixed-order sum
    assert rel(Fk.cpu().numpy(), O.force(dS_ref, U)) <= 1e-9


def test_pseudofermion_autograd_dwf(gpu):
    """PseudofermionActionFn on the domain-wall operator at 4^4 x 8: S and both gradients."""
    import paper_1512_03487_amd as gm
    from tests.gpu_util import dev, rel
    U, phi, op, kw = _pf_case("dwf")
    S_ref, dS_ref, X_ref = O.pseudofermion(op, U, phi, tol=1e-13)
    Ud = dev(U).requires_grad_(True)
    phid = dev(phi).requires_grad_(True)
    S = gm.PseudofermionActionFn.apply(Ud, phid, "dwf", 0.0, 1.8, 0.01, 1e-13)
    (3.0 * S).backward()
    assert abs(float(S) - S_ref) <= 1e-11 * abs(S_ref)
    assert rel(Ud.grad.cpu().numpy(), 3.0 * dS_ref) <= 1e-9
    assert rel(phid.grad.cpu().numpy(), 6.0 * X_ref) <= 1e-9


def test_pseudofermion_action_mobius(gpu):
    """The Moebius pseudofermion action (b5 = 1.5, c5 = 0.5, M5 = 1.8, mf = 0.1) at 4^4 x 8: S, X,
    dS/dU (raw and su(3)-projected) and dS/dphi through the ABI, and S and both gradients through
    PseudofermionActionFn, against the numpy Moebius oracle (its own CG to 1e-13)."""
    import paper_1512_03487_amd as gm
    from oracle import mobius as MB
    from tests.gpu_util import dev, rel
    dims, Ls = (4, 4, 4, 4), 8
    kw = dict(M5=1.8, mf=0.1, b5=1.5, c5=0.5)
    U = F.gauge_field(dims, seed=1, kind="haar")
    phi = F.spinor_field(dims, seed=5, Ls=Ls)
    S_ref, dS_ref, X_ref = MB.pseudofermion(U, phi, tol=1e-13, **kw)
    Ud, phid = dev(U), dev(phi)
    S, X, gU, gphi, st = gm.pseudofermion_action(Ud, phid, "mobius", tol=1e-13, grad_scale=0.75, want_U=True,
                                                 want_phi=True, **kw)
    assert st["converged"]
    assert abs(S - S_ref) <= 1e-11 * abs(S_ref)
    assert rel(X.cpu().numpy(), X_ref) <= 1e-9
    assert rel(gU.cpu().numpy(), 0.75 * dS_ref) <= 1e-9
    assert rel(gphi.cpu().numpy(), 1.5 * X_ref) <= 1e-9
    _, _, Fk, _, _ = gm.pseudofermion_action(Ud, phid, "mobius", tol=1e-13, want_U=True, force=True, **kw)
    assert rel(Fk.cpu().numpy(), O.force(dS_ref, U)) <= 1e-9
    Ug = dev(U).requires_grad_(True)
    phig = dev(phi).requires_grad_(True)
    Sa = gm.PseudofermionActionFn.apply(Ug, phig, "mobius", 0.0, 1.8, 0.1, 1e-13, "f64", 1.5, 0.5)
    (2.0 * Sa).backward()
    assert abs(float(Sa) - S_ref) <= 1e-11 * abs(S_ref)
    assert rel(Ug.grad.cpu().numpy(), 2.0 * dS_ref) <= 1e-9
    assert rel(phig.grad.cpu().numpy(), 4.0 * X_ref) <= 1e-9
