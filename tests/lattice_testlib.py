"""Test-side textbook pieces used to pin the oracle and to compare the HIP path against it.

Nothing here is shared with the oracle or the product: the Dirac matrices are typed from the
textbook chiral-basis definition, the dense operators are assembled entry by entry, and the
plane waves and shifts are plain numpy.
"""
from __future__ import annotations

import numpy as np

# Pauli matrices and the Euclidean chiral-basis Dirac matrices, typed from their definition:
# gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] for k = 1, 2, 3 and gamma_4 = [[0, 1], [1, 0]].
SIGMA = [np.array([[0, 1], [1, 0]], dtype=complex),
         np.array([[0, -1j], [1j, 0]], dtype=complex),
         np.array([[1, 0], [0, -1]], dtype=complex)]
Z2 = np.zeros((2, 2), dtype=complex)
I2 = np.eye(2, dtype=complex)
TEXTBOOK_GAMMA = [np.block([[Z2, -1j * s], [1j * s, Z2]]) for s in SIGMA] + [np.block([[Z2, I2], [I2, Z2]])]
GAMMA5 = np.diag([1, 1, -1, -1]).astype(complex)
P_PLUS = np.diag([1, 1, 0, 0]).astype(complex)
P_MINUS = np.diag([0, 0, 1, 1]).astype(complex)
I4 = np.eye(4, dtype=complex)

# numpy axis of direction mu in a (Lt, Lz, Ly, Lx, ...) array
AXIS = {0: 3, 1: 2, 2: 1, 3: 0}


def dims_of(field):
    lt, lz, ly, lx = field.shape[:4]
    return (lx, ly, lz, lt)


def shift(field, mu, k):
    """field(x + k mu-hat), periodic (the paper's Cshift(field, mu, k))."""
    return np.roll(field, -k, axis=AXIS[mu])


def coords(dims):
    """Integer coordinates x_mu of every site, shape (4, Lt, Lz, Ly, Lx)."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.indices((lt, lz, ly, lx))
    return np.stack([x, y, z, t])


def plane_wave(dims, n, u):
    """psi(x) = exp(i p.x) u with p_mu = 2 pi n_mu / L_mu; u has shape (4, 3) or (Ls, 4, 3)."""
    c = coords(dims)
    phase = np.zeros(c.shape[1:])
    for mu in range(4):
        phase = phase + 2 * np.pi * n[mu] * c[mu] / dims[mu]
    return np.exp(1j * phase)[(...,) + (None,) * np.ndim(u)] * np.asarray(u)[None, None, None, None]


def momentum(dims, n):
    return np.array([2 * np.pi * n[mu] / dims[mu] for mu in range(4)])


def spin_apply(M, psi):
    """Apply a 4x4 spin matrix to every site (spin axis -2)."""
    return np.einsum("st,...ta->...sa", M, psi)


def site_index(dims, x):
    lx, ly, lz, lt = dims
    return ((x[3] % lt) * lz + (x[2] % lz)) * ly * lx + (x[1] % ly) * lx + (x[0] % lx)


def all_sites(dims):
    lx, ly, lz, lt = dims
    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    yield (x, y, z, t)


def link(U, x, mu):
    """U_mu(x) from a (Lt, Lz, Ly, Lx, 4, 3, 3) array at periodic coordinates x."""
    lx, ly, lz, lt = dims_of(U)
    return U[x[3] % lt, x[2] % lz, x[1] % ly, x[0] % lx, mu]


def dense_hop(U, dag=False):
    """Dense H (or H^dagger) assembled block by block, index = site * 12 + spin * 3 + colour."""
    dims = dims_of(U)
    V = int(np.prod(dims))
    H = np.zeros((12 * V, 12 * V), dtype=complex)
    sg = -1.0 if dag else 1.0
    for x in all_sites(dims):
        i = site_index(dims, x)
        for mu in range(4):
            xp = list(x); xp[mu] += 1
            xm = list(x); xm[mu] -= 1
            j, k = site_index(dims, xp), site_index(dims, xm)
            H[12 * i:12 * i + 12, 12 * j:12 * j + 12] += np.kron(I4 - sg * TEXTBOOK_GAMMA[mu], link(U, x, mu))
            H[12 * i:12 * i + 12, 12 * k:12 * k + 12] += np.kron(I4 + sg * TEXTBOOK_GAMMA[mu],
                                                                 link(U, xm, mu).conj().T)
    return H


def dense_wilson(U, mass, dag=False):
    H = dense_hop(U, dag)
    return (4.0 + mass) * np.eye(H.shape[0]) - 0.5 * H


def dense_dwf(U, Ls, M5, mf, dag=False):
    """Dense Shamir M (or M^dagger), index = (site * Ls + s) * 12 + spin * 3 + colour."""
    dims = dims_of(U)
    V = int(np.prod(dims))
    H = dense_hop(U, dag).reshape(V, 12, V, 12)
    n = V * Ls * 12
    M = np.zeros((V, Ls, 12, V, Ls, 12), dtype=complex)
    for s in range(Ls):
        M[:, s, :, :, s, :] = -0.5 * H
    M = M.reshape(n, n) + (5.0 - M5) * np.eye(n)
    # fifth-dimension hopping: -P_up psi~_{s+1} - P_dn psi~_{s-1} (P_up = P_- for M, P_+ for M^dag)
    Pup, Pdn = (P_PLUS, P_MINUS) if dag else (P_MINUS, P_PLUS)
    S5p = np.zeros((Ls, Ls))
    S5m = np.zeros((Ls, Ls))
    for s in range(Ls):
        S5p[s, (s + 1) % Ls] = -mf if s == Ls - 1 else 1.0
        S5m[s, (s - 1) % Ls] = -mf if s == 0 else 1.0
    I3 = np.eye(3)
    K = -(np.kron(S5p, np.kron(Pup, I3)) + np.kron(S5m, np.kron(Pdn, I3)))
    return M + np.kron(np.eye(V), K)


def su3_exp(X):
    """exp(X) for anti-Hermitian X (per matrix), via the eigendecomposition of -iX."""
    w, v = np.linalg.eigh(-1j * X)
    return np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * w), v.conj())


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
