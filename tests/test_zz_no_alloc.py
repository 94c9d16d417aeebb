"""grid_dwf_mdag_m_noalloc (M psi in the library's static scratch) against grid_dwf_mdag_m (M psi
in a caller's tmp): same kernels, so the outputs agree bit for bit, on two calls in a row, the
second with a smaller field, in every storage precision. Called through the C ABI."""
import pytest

from paper_1512_03487_amd import fields as F

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _announce():
    print("\n[gpu] test_zz_no_alloc", flush=True)


def _same(a, b):
    import torch
    if hasattr(a, "codes"):
        return torch.equal(a.codes, b.codes) and torch.equal(a.scale, b.scale)
    return torch.equal(a, b)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
def test_noalloc_matches_tmp_variant(gpu, prec):
    import torch
    import paper_1512_03487_amd as gm
    from tests.gpu_util import as_prec
    # a larger field first, then a smaller one: the second call must not see the first's scratch
    for dims, Ls in (((8, 8, 8, 8), 8), ((4, 4, 6, 4), 4)):
        U = F.gauge_field(dims, seed=1, kind="haar")
        psi = F.spinor_field(dims, seed=3, Ls=Ls)
        Uk, pk, _, _ = as_prec(U, psi, prec)
        ref = gm.dwf_mdag_m(Uk, pk, 1.8, 0.01)
        out = gm.api._empty_like(pk)
        gm.api.dwf_mdag_m_noalloc(Uk, pk, 1.8, 0.01, out)
        torch.cuda.synchronize()
        assert _same(out, ref), (prec, dims, Ls)

