"""Even-odd (red-black) decomposition -- FP64 CPU oracle, TEST INFRASTRUCTURE ONLY.

Grid objects may hold a single checkerboard of the lattice (Section 2.2). A site's parity is
p = (x + y + z + t) mod 2; a checkerboard field holds the sites of one parity with x halved:
site (x, y, z, t) sits at [t][z][y][x // 2] (every extent even), the per-site tensor (and the Ls
records of a 5D site) unchanged.

Everything here is composed from the pinned full-lattice oracle (``oracle.hop``, ``oracle.apply``)
and plain numpy: a checkerboard operator is the full operator applied to a field that is zero on
the other parity, restricted to the output parity. The domain-wall fifth-dimension operator M5 is
written out from its definition, and its inverse is a dense solve of the Ls x Ls system per
chirality (numpy.linalg.solve as the library step).

Only the test-suite uses this module; it shares nothing with the HIP library.
"""
from __future__ import annotations

import numpy as np

from . import oracle as _o


def parity(shape4) -> np.ndarray:
    """(Lt, Lz, Ly, Lx) array of site parities (x + y + z + t) mod 2."""
    lt, lz, ly, lx = shape4
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    return (x + y + z + t) % 2


def _xs(shape4, p):
    """x coordinate of the k-th parity-p site of each row: (Lt, Lz, Ly, Lx/2) integer array."""
    lt, lz, ly, lx = shape4
    if any(L % 2 for L in shape4):
        raise ValueError("checkerboard fields need even extents")
    t, z, y, k = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx // 2), indexing="ij")
    return t, z, y, 2 * k + ((y + z + t + p) % 2)


def pick(field, p: int) -> np.ndarray:
    """The parity-p checkerboard of a full field (Lt, Lz, Ly, Lx, ...)."""
    t, z, y, x = _xs(field.shape[:4], p)
    return np.ascontiguousarray(field[t, z, y, x])


def embed(cb, p: int) -> np.ndarray:
    """Full field equal to the checkerboard cb on parity p and zero on the other parity."""
    shape4 = cb.shape[:3] + (2 * cb.shape[3],)
    out = np.zeros(shape4 + cb.shape[4:], dtype=np.complex128)
    t, z, y, x = _xs(shape4, p)
    out[t, z, y, x] = cb
    return out


def hop_cb(U, psi_cb, out_parity: int, dag: bool = False) -> np.ndarray:
    """H_{p,1-p} psi: the hopping term from checkerboard 1 - p to checkerboard p."""
    full = embed(psi_cb, 1 - out_parity)
    return pick(_o.hop(U, full, dag), out_parity)


def m5(psi, M5: float, mf: float, dag: bool = False) -> np.ndarray:
    """Fifth-dimension part of the Shamir operator on a 5D field (..., Ls, 4, 3):

    (M5 psi)_s = (5 - M5) psi_s - P_- psi~_{s+1} - P_+ psi~_{s-1}, psi~_{Ls} = -mf psi_0,
    psi~_{-1} = -mf psi_{Ls-1}; the adjoint exchanges P_+ and P_-. P_+ keeps spins 0, 1 and
    P_- spins 2, 3 (gamma_5 = diag(1, 1, -1, -1)).
    """
    psi = np.asarray(psi, dtype=np.complex128)
    up = np.roll(psi, -1, axis=-3).copy()     # psi~_{s+1}
    up[..., -1, :, :] *= -mf
    dn = np.roll(psi, 1, axis=-3).copy()      # psi~_{s-1}
    dn[..., 0, :, :] *= -mf
    out = (5.0 - M5) * psi
    lower, upper = slice(2, 4), slice(0, 2)
    from_up, from_dn = (upper, lower) if dag else (lower, upper)
    out[..., from_up, :] -= up[..., from_up, :]
    out[..., from_dn, :] -= dn[..., from_dn, :]
    return out


def m5_matrix(Ls: int, M5: float, mf: float, plus: bool) -> np.ndarray:
    """Ls x Ls matrix of M5 on one chirality: plus couples s to s + 1, else s to s - 1."""
    A = (5.0 - M5) * np.eye(Ls, dtype=np.complex128)
    for s in range(Ls):
        if plus:
            A[s, (s + 1) % Ls] += -1.0 if s < Ls - 1 else mf
        else:
            A[s, (s - 1) % Ls] += -1.0 if s > 0 else mf
    return A


def m5inv(psi, M5: float, mf: float, dag: bool = False) -> np.ndarray:
    """M5^-1 psi (or (M5^dagger)^-1 psi) by a dense solve per chirality."""
    psi = np.asarray(psi, dtype=np.complex128)
    Ls = psi.shape[-3]
    lead = psi.shape[:-3]
    out = np.empty_like(psi)
    for spins, plus in ((slice(2, 4), not dag), (slice(0, 2), dag)):
        A = m5_matrix(Ls, M5, mf, plus)
        rhs = np.moveaxis(psi[..., spins, :], -3, 0).reshape(Ls, -1)
        sol = np.linalg.solve(A, rhs).reshape((Ls,) + lead + (2, 3))
        out[..., spins, :] = np.moveaxis(sol, 0, -3)
    return out


def diag(kind: str, y, mass: float = 0.0, M5: float = 1.8, mf: float = 0.01, dag: bool = False) -> np.ndarray:
    """The parity-diagonal block M_ee = M_oo: (4 + mass) for Wilson, M5 for domain wall."""
    if kind == "wilson":
        return (4.0 + mass) * np.asarray(y, dtype=np.complex128)
    return m5(y, M5, mf, dag)


def diag_inv(kind: str, y, mass: float = 0.0, M5: float = 1.8, mf: float = 0.01, dag: bool = False) -> np.ndarray:
    if kind == "wilson":
        return np.asarray(y, dtype=np.complex128) / (4.0 + mass)
    return m5inv(y, M5, mf, dag)


def schur(U, psi_e, kind: str, mass: float = 0.0, M5: float = 1.8, mf: float = 0.01, dag: bool = False) -> np.ndarray:
    """Mhat psi_e = M_ee psi_e - M_eo M_oo^-1 M_oe psi_e with M_eo = M_oe = -H/2 (adjoint if dag)."""
    t = hop_cb(U, psi_e, 1, dag)
    t = diag_inv(kind, t, mass, M5, mf, dag)
    return diag(kind, psi_e, mass, M5, mf, dag) - 0.25 * hop_cb(U, t, 0, dag)


def source(U, b, kind: str, mass: float = 0.0, M5: float = 1.8, mf: float = 0.01) -> np.ndarray:
    """bhat = b_e - M_eo M_oo^-1 b_o."""
    bo = diag_inv(kind, pick(b, 1), mass, M5, mf)
    return pick(b, 0) + 0.5 * hop_cb(U, bo, 0)


def odd_solution(U, b, x_e, kind: str, mass: float = 0.0, M5: float = 1.8, mf: float = 0.01) -> np.ndarray:
    """x_o = M_oo^-1 (b_o - M_oe x_e)."""
    return diag_inv(kind, pick(b, 1) + 0.5 * hop_cb(U, x_e, 1), mass, M5, mf)


def merge(x_e, x_o) -> np.ndarray:
    return embed(x_e, 0) + embed(x_o, 1)


# ---------------------------------------------------------------------------------------------
# Moebius domain wall (M = D_W (b5 + c5 S) + 1 - S, see oracle.mobius). Its blocks are read off
# the pinned full-lattice operator: a field living on parity q, mapped by M (or M^dagger) and
# restricted to parity p, is M_pq applied to it. The 4D-diagonal block M_ee = M_oo has no hopping
# term (it acts on the fifth coordinate and the chirality only, the same at every 4D site), so its
# inverse is a dense solve of the 4 Ls x 4 Ls matrix it has on one 4D site and colour, written
# out column by column from the operator itself.
# ---------------------------------------------------------------------------------------------

def mobius_block(U, psi_q, q: int, p: int, M5: float, mf: float, b5: float, c5: float,
                 dag: bool = False) -> np.ndarray:
    """M_pq psi_q (the blocks of M^dagger when dag) for checkerboard fields."""
    from . import mobius as _mob
    return pick(_mob.mobius(U, embed(psi_q, q), M5, mf, b5, c5, dag), p)


def mobius_diag_matrix(Ls: int, M5: float, mf: float, b5: float, c5: float, dag: bool = False) -> np.ndarray:
    """The (Ls, 4) x (Ls, 4) matrix of M_ee on one 4D site and colour: the Moebius operator of the
    module ``oracle.mobius`` with its hopping term dropped, applied to unit vectors."""
    from . import mobius as _mob
    n = Ls * 4
    A = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros((Ls, 4, 3), dtype=np.complex128)
        e[j // 4, j % 4, 0] = 1.0
        # M_ee psi = (4 - M5) B psi + psi - S psi (B^dagger D^dagger ... for the adjoint): the
        # Moebius operator with the hopping term dropped
        if not dag:
            v = (4.0 - M5) * (b5 * e + c5 * _mob.shift5(e, mf)) + e - _mob.shift5(e, mf)
        else:
            f = (4.0 - M5) * e
            v = b5 * f + c5 * _mob.shift5(f, mf, True) + e - _mob.shift5(e, mf, True)
        A[:, j] = v[:, :, 0].ravel()
    return A


def mobius_diag_inv(psi, M5: float, mf: float, b5: float, c5: float, dag: bool = False) -> np.ndarray:
    """M_ee^-1 psi (the adjoint's inverse when dag) by a dense solve per 4D site and colour."""
    psi = np.asarray(psi, dtype=np.complex128)
    Ls = psi.shape[-3]
    A = mobius_diag_matrix(Ls, M5, mf, b5, c5, dag)
    lead = psi.shape[:-3]
    rhs = np.moveaxis(psi, -1, 0).reshape(3, -1, Ls * 4)          # colour, sites, (s, spin)
    sol = np.linalg.solve(A, rhs.reshape(-1, Ls * 4).T).T.reshape(3, *lead, Ls, 4)
    return np.ascontiguousarray(np.moveaxis(sol, 0, -1))


def schur_mobius(U, psi_e, M5: float, mf: float, b5: float, c5: float, dag: bool = False) -> np.ndarray:
    """Mhat psi_e = M_ee psi_e - M_eo M_oo^-1 M_oe psi_e (Mhat^dagger, from the blocks of M^dagger,
    when dag)."""
    kw = dict(M5=M5, mf=mf, b5=b5, c5=c5, dag=dag)
    t = mobius_block(U, psi_e, 0, 1, **kw)
    t = mobius_diag_inv(t, M5, mf, b5, c5, dag)
    return mobius_block(U, psi_e, 0, 0, **kw) - mobius_block(U, t, 1, 0, **kw)


def source_mobius(U, b, M5: float, mf: float, b5: float, c5: float) -> np.ndarray:
    """bhat = b_e - M_eo M_oo^-1 b_o."""
    bo = mobius_diag_inv(pick(b, 1), M5, mf, b5, c5)
    return pick(b, 0) - mobius_block(U, bo, 1, 0, M5, mf, b5, c5)


def odd_solution_mobius(U, b, x_e, M5: float, mf: float, b5: float, c5: float) -> np.ndarray:
    """x_o = M_oo^-1 (b_o - M_oe x_e)."""
    return mobius_diag_inv(pick(b, 1) - mobius_block(U, x_e, 0, 1, M5, mf, b5, c5), M5, mf, b5, c5)
