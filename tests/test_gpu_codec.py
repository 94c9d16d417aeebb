"""GPU codecs against the oracle: bit-exact where the result is a code (FP16 storage, narrowing),
within FP64 rounding for reunitarisation."""
import numpy as np
import pytest

import oracle.oracle as O
from paper_1512_03487_amd import fields as F

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _announce():
    print("\n[gpu] test_gpu_codec", flush=True)


@pytest.mark.parametrize("Ls", [None, 7])
def test_spinor_fp16_encode_is_bit_exact(gpu, Ls):
    import paper_1512_03487_amd as gm
    from tests.gpu_util import dev
    dims = (4, 6, 2, 6)
    psi = F.spinor_field(dims, seed=2, Ls=Ls)
    # wide dynamic range across sites, and an all-zero site
    psi = psi * np.exp(np.random.default_rng(0).uniform(-10, 10, psi.shape[:-2]))[..., None, None]
    psi[0, 0, 0, 0] = 0
    codes, scale = O.fp16_encode(psi, site_axes=2)
    for src in (psi, psi.astype(np.complex64)):
        h = gm.convert_spinor(dev(src), "f16s")
        np.testing.assert_array_equal(h.scale.cpu().numpy(), scale)
        np.testing.assert_array_equal(h.codes.cpu().numpy().view(np.uint16), codes.view(np.uint16))
    # decode (exact: one float32 product per real)
    back = gm.convert_spinor(h, "f64").cpu().numpy()
    np.testing.assert_array_equal(back, O.fp16_decode(codes, scale))


def test_spinor_float_round_trip(gpu):
    import paper_1512_03487_amd as gm
    from tests.gpu_util import dev
    psi = F.spinor_field((4, 4, 4, 4), seed=2, Ls=3)
    f32 = gm.convert_spinor(dev(psi), "f32").cpu().numpy()
    np.testing.assert_array_equal(f32, psi.astype(np.complex64))
    back = gm.convert_spinor(dev(f32), "f64").cpu().numpy()
    np.testing.assert_array_equal(back, f32.astype(np.complex128))


def test_link_narrowing_and_compression(gpu):
    import paper_1512_03487_amd as gm
    from tests.gpu_util import dev, links_f16
    U = F.gauge_field((4, 4, 2, 6), seed=1, kind="haar")
    Ud = dev(U)
    np.testing.assert_array_equal(gm.convert_links(Ud, "f32", "L18").cpu().numpy(), U.astype(np.complex64))
    np.testing.assert_array_equal(gm.convert_links(Ud, "f32", "L12").cpu().numpy(), U[..., :2, :].astype(np.complex64))
    np.testing.assert_array_equal(gm.convert_links(Ud, "f64", "L12").cpu().numpy(), U[..., :2, :])
    h = gm.convert_links(Ud, "f16s", "L18").cpu().numpy()
    np.testing.assert_array_equal(h.view(np.uint16), links_f16(U).view(np.uint16))
    h12 = gm.convert_links(Ud, "f16s", "L12").cpu().numpy()
    np.testing.assert_array_equal(h12.view(np.uint16), links_f16(U)[..., :2, :, :].view(np.uint16))


def test_link_reunitarisation(gpu):
    import paper_1512_03487_amd as gm
    from tests.gpu_util import dev
    U = F.gauge_field((4, 4, 4, 4), seed=1, kind="haar")
    rng = np.random.default_rng(3)
    noisy = U + 1e-3 * (rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape))
    got = gm.convert_links(dev(noisy), "f64", "L18", reunitarise=True).cpu().numpy()
    np.testing.assert_allclose(got, O.reunitarise(noisy), atol=1e-14, rtol=0)
    # rounded to float32 after projection
    got32 = gm.convert_links(dev(noisy), "f32", "L18", reunitarise=True).cpu().numpy()
    np.testing.assert_allclose(got32, O.reunitarise(noisy).astype(np.complex64), atol=2e-7, rtol=0)
