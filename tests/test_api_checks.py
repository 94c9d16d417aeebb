"""The torch wrappers reject mismatched fields before anything reaches the library.

The C ABI sees raw pointers only, so a link field of the wrong lattice, or an out / tmp / x0 /
grad_out of another shape or dtype, would be read or written out of bounds on the device. These
checks run on the host: the library loader is replaced by one that fails the test if it is ever
reached, and CPU tensors stand in for device tensors (the device guard is relaxed to a
contiguity check).
"""
import pytest
import torch

from paper_1512_03487_amd import api


class _NoLibrary:
    def __getattr__(self, name):
        raise AssertionError(f"library entry {name} reached despite invalid arguments")


@pytest.fixture(autouse=True)
def host_only(monkeypatch):
    def need(t, name):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    monkeypatch.setattr(api, "_need_cuda", need)
    monkeypatch.setattr(api, "load", lambda: _NoLibrary())


def spinor(dims=(4, 4, 4, 4), Ls=None, dtype=torch.complex128):
    lx, ly, lz, lt = dims
    shape = (lt, lz, ly, lx) + ((Ls,) if Ls else ()) + (4, 3)
    return torch.zeros(shape, dtype=dtype)


def links(dims=(4, 4, 4, 4), dtype=torch.complex128, rows=3):
    lx, ly, lz, lt = dims
    return torch.zeros((lt, lz, ly, lx, 4, rows, 3), dtype=dtype)


def test_dhop_rejects_links_of_another_lattice():
    with pytest.raises(ValueError, match="site shape"):
        api.dhop(links((4, 4, 4, 2)), spinor())


def test_dhop_rejects_bad_out():
    U, psi = links(), spinor()
    with pytest.raises(TypeError, match="dtype"):
        api.dhop(U, psi, out=spinor(dtype=torch.complex64))
    with pytest.raises(ValueError, match="shape"):
        api.dhop(U, psi, out=spinor((4, 4, 4, 2)))
    with pytest.raises(TypeError):
        api.dhop(U, psi, out=api.F16Spinor.empty((4, 4, 4, 4), "cpu"))


def test_fp16_out_must_match_codes_and_scales():
    U = torch.zeros((4, 4, 4, 4, 4, 2, 3, 2), dtype=torch.float16)
    psi = api.F16Spinor.empty((4, 4, 4, 4), "cpu")
    bad = api.F16Spinor(psi.codes.clone(), torch.zeros((4, 4, 4, 2), dtype=torch.float32))
    with pytest.raises(ValueError, match="scale"):
        api.dhop(U, psi, out=bad)
    with pytest.raises(TypeError):
        api.dhop(U, psi, out=spinor())


def test_mobius_and_normal_operator_reject_bad_tmp():
    U, psi = links(), spinor(Ls=4)
    with pytest.raises(ValueError, match="tmp"):
        api.mobius(U, psi, 1.8, 0.01, 1.5, 0.5, tmp=spinor(Ls=2))
    with pytest.raises(ValueError, match="out"):
        api.dwf_mdag_m(U, psi, 1.8, 0.01, out=spinor(Ls=2))
    with pytest.raises(ValueError, match="site shape"):
        api.dwf_mdag_m(links((2, 4, 4, 4)), psi, 1.8, 0.01)


def test_cg_and_solve_eo_reject_bad_x0_and_links():
    U, b = links(), spinor(Ls=4)
    with pytest.raises(ValueError, match="x0"):
        api.cg(U, b, x0=spinor(Ls=2))
    with pytest.raises(TypeError, match="x0"):
        api.cg(U, b, x0=spinor(Ls=4, dtype=torch.complex64))
    with pytest.raises(ValueError, match="site shape"):
        api.cg(links((4, 4, 2, 4)), b)
    with pytest.raises(ValueError, match="x0"):
        api.solve_eo(U, b, x0=spinor(Ls=2))


def test_backward_rejects_bad_grad_out():
    U, psi = links(), spinor()
    with pytest.raises(ValueError, match="grad_out"):
        api.dhop_backward(U, psi, spinor((2, 4, 4, 4)))
    with pytest.raises(ValueError, match="site shape"):
        api.dhop_backward(links((2, 4, 4, 4)), psi, spinor())


def test_checkerboard_rejects_bad_y_and_out():
    U = links()
    psi = spinor((2, 4, 4, 4))          # half the x extent
    with pytest.raises(ValueError, match="y"):
        api.dhop_cb(U, psi, 0, "wilson", y=spinor((4, 4, 4, 4)))
    with pytest.raises(TypeError, match="out"):
        api.dhop_cb(U, psi, 0, out=spinor((2, 4, 4, 4), dtype=torch.complex64))


def test_hmc_rejects_mismatched_momenta_and_pseudofermion():
    U = links()
    with pytest.raises(ValueError, match="P"):
        api.md_leapfrog(U, links((2, 4, 4, 4)), 5.0, 0.1, 2)
    with pytest.raises(ValueError, match="site shape"):
        api.md_leapfrog(U, links(), 5.0, 0.1, 2, phi=spinor((2, 4, 4, 4), Ls=4))
    with pytest.raises(ValueError, match="P"):
        api.link_exp(U, links((4, 4, 4, 2)), 0.1)


def test_multigrid_rejects_mismatched_fields():
    U = links()
    vecs = torch.zeros((2, 4, 4, 4, 4, 4, 3), dtype=torch.complex128)
    A = torch.zeros((2, 2, 2, 2, 9, 4, 4), dtype=torch.complex128)
    with pytest.raises(ValueError, match="vecs"):
        api.mg_solve(U, torch.zeros((2, 4, 4, 2, 4, 4, 3), dtype=torch.complex128), A, spinor(), 0.1)
    with pytest.raises(ValueError, match="A must be"):
        api.mg_solve(U, vecs, A[:1], spinor(), 0.1)
    with pytest.raises(ValueError, match="x0"):
        api.mg_solve(U, vecs, A, spinor(), 0.1, x0=spinor((2, 4, 4, 4)))
    with pytest.raises(ValueError, match="vc"):
        api.mg_prolong(vecs, torch.zeros((2, 2, 2, 2, 3), dtype=torch.complex128), (2, 2, 2, 2))
