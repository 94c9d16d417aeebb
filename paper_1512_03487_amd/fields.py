"""Seeded synthetic lattice fields shared by the HIP path's tests/benchmarks and the oracle's tests.

This module only draws random inputs. It holds none of the operator's arithmetic (no hopping term,
no gamma matrices, no solver), so the oracle and the HIP path stay independent: both receive the
same arrays from here and nothing else in common.

Conventions
-----------
* ``dims = (Lx, Ly, Lz, Lt)``: direction mu = 0, 1, 2, 3 is x, y, z, t.
* Fields are numpy arrays with the time coordinate slowest and x fastest among sites, the
  per-site tensor innermost ("site-major"):

  - gauge field ``U``: ``(Lt, Lz, Ly, Lx, 4, 3, 3)`` complex, ``U[..., mu, a, b]`` row-major 3x3;
  - 4D spinor: ``(Lt, Lz, Ly, Lx, 4, 3)`` complex (spin, colour);
  - 5D spinor: ``(Lt, Lz, Ly, Lx, Ls, 4, 3)`` complex, the fifth coordinate inside the 4D site.

* Random numbers come from ``numpy.random.Generator(PCG64(seed))``, consumed in memory order.

The lattice formulation is the Wilson / domain-wall fermion discretisation the paper's Grid
library implements (Section 4 lists the Wilson fermion action, five-dimensional chiral fermions
and periodic boundary conditions); the paper itself gives no generator recipe, so the recipes
below are the standard ones and are stated here in full.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "make_rng", "lattice_shape", "haar_su3", "weak_su3", "gauge_field", "spinor_field",
    "gauge_transform", "random_su3_algebra", "GELL_MANN",
]


def make_rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def lattice_shape(dims) -> tuple:
    """Site shape (Lt, Lz, Ly, Lx) for dims = (Lx, Ly, Lz, Lt)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    return (lt, lz, ly, lx)


# The eight Gell-Mann matrices (a basis of traceless Hermitian 3x3 matrices, tr(l_a l_b) = 2 d_ab).
GELL_MANN = np.zeros((8, 3, 3), dtype=np.complex128)
GELL_MANN[0][0, 1] = GELL_MANN[0][1, 0] = 1
GELL_MANN[1][0, 1], GELL_MANN[1][1, 0] = -1j, 1j
GELL_MANN[2][0, 0], GELL_MANN[2][1, 1] = 1, -1
GELL_MANN[3][0, 2] = GELL_MANN[3][2, 0] = 1
GELL_MANN[4][0, 2], GELL_MANN[4][2, 0] = -1j, 1j
GELL_MANN[5][1, 2] = GELL_MANN[5][2, 1] = 1
GELL_MANN[6][1, 2], GELL_MANN[6][2, 1] = -1j, 1j
GELL_MANN[7] = np.diag([1, 1, -2]) / np.sqrt(3)


def haar_su3(rng: np.random.Generator, n: int) -> np.ndarray:
    """n Haar-distributed SU(3) matrices, shape (n, 3, 3).

    Mezzadri's recipe (Notices AMS 54, 2007): QR of a complex Gaussian matrix with the phases of
    R's diagonal moved into Q gives Haar on U(3); dividing by the principal cube root of the
    determinant maps it to SU(3). That map commutes with left multiplication by SU(3), so the
    result is Haar on SU(3).
    """
    re = rng.standard_normal((n, 3, 3))
    im = rng.standard_normal((n, 3, 3))
    z = (re + 1j * im) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    u = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(u)
    return u / (det ** (1.0 / 3.0))[:, None, None]


def weak_su3(rng: np.random.Generator, n: int, eps: float = 0.3) -> np.ndarray:
    """n matrices exp(i eps H), H = sum_a h_a lambda_a / 2 with h_a ~ N(0, 1); shape (n, 3, 3).

    H is traceless Hermitian, so the exponential (taken through H's eigendecomposition) is SU(3).
    """
    h = rng.standard_normal((n, 8))
    herm = np.einsum("na,aij->nij", h, GELL_MANN) / 2.0
    w, v = np.linalg.eigh(herm)
    return np.einsum("nij,nj,nkj->nik", v, np.exp(1j * eps * w), v.conj())


def gauge_field(dims, seed: int = 1, kind: str = "haar", eps: float = 0.3) -> np.ndarray:
    """Gauge field of shape (Lt, Lz, Ly, Lx, 4, 3, 3), complex128.

    ``kind``: "haar" (hot, Haar random), "weak" (exp(i eps H) near the identity) or "unit".
    """
    shape = lattice_shape(dims) + (4,)
    n = int(np.prod(shape))
    if kind == "unit":
        u = np.broadcast_to(np.eye(3, dtype=np.complex128), (n, 3, 3)).copy()
    elif kind == "haar":
        u = haar_su3(make_rng(seed), n)
    elif kind == "weak":
        u = weak_su3(make_rng(seed), n, eps)
    else:
        raise ValueError(f"unknown gauge field kind {kind!r}")
    return np.ascontiguousarray(u.reshape(shape + (3, 3)))


def spinor_field(dims, seed: int = 2, Ls: int | None = None) -> np.ndarray:
    """Complex Gaussian spinor with Re, Im ~ N(0, 1/2) (so E|z|^2 = 1), complex128.

    Shape (Lt, Lz, Ly, Lx, 4, 3), or (Lt, Lz, Ly, Lx, Ls, 4, 3) when Ls is given.
    """
    shape = lattice_shape(dims) + ((int(Ls),) if Ls is not None else ()) + (4, 3)
    rng = make_rng(seed)
    x = rng.standard_normal(shape + (2,)) * np.sqrt(0.5)
    return np.ascontiguousarray(x[..., 0] + 1j * x[..., 1])


def gauge_transform(dims, seed: int = 4) -> np.ndarray:
    """A Haar-random SU(3) matrix per site, shape (Lt, Lz, Ly, Lx, 3, 3)."""
    shape = lattice_shape(dims)
    g = haar_su3(make_rng(seed), int(np.prod(shape)))
    return np.ascontiguousarray(g.reshape(shape + (3, 3)))


def random_su3_algebra(dims, seed: int = 6) -> np.ndarray:
    """A random element X = i sum_a h_a lambda_a / 2 of su(3) per link, shape (Lt,Lz,Ly,Lx,4,3,3).

    Used as a perturbation direction U -> exp(eps X) U in finite-difference checks.
    """
    shape = lattice_shape(dims) + (4,)
    h = make_rng(seed).standard_normal(shape + (8,))
    return np.ascontiguousarray(1j * np.einsum("...a,aij->...ij", h, GELL_MANN) / 2.0)
