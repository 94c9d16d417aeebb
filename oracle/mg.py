"""Two-level multigrid for the Wilson operator -- FP64 CPU oracle, TEST INFRASTRUCTURE ONLY.

The paper presents its generic stencil support with a coarse-grid operator of an adaptive multigrid
inverter as the example (Section 2.4, Stencil support) and lists multigrid-preconditioned CG and
GCR among the algorithms (Section 4). It prints no formulas; the definitions used here are the
standard aggregation-based construction, written out plainly:

* Aggregates: blocks of b = (bx, by, bz, bt) fine sites; fine x belongs to coarse site
  xc_mu = x_mu // b_mu on the coarse lattice Lc = L / b (periodic), coarse index
  xc0 + Lc0 (xc1 + Lc1 (xc2 + Lc2 xc3)) like the fine one.
* Chirality split: spins 0, 1 (chi = 0) and spins 2, 3 (chi = 1), the P+ / P- halves of the chiral
  basis. A coarse vector has N = 2 nvec components per coarse site, n = chi nvec + k.
* Basis: nvec fine vectors phi_k. On every aggregate and chirality their restrictions are
  orthonormalised by Gram-Schmidt in the order k = 0, 1, ... (the thin QR factorisation with a
  positive real diagonal), giving the columns of the prolongation P; restriction R = P^dagger.
* Coarse operator A_c = R D P (Galerkin), held as a 9-point stencil
  (A_c v)(xc) = sum_d A_d(xc) v(xc + e_d), d = 0 (self), 1 + 2 mu (e = +mu), 2 + 2 mu (e = -mu).
  A hop of D from fine x in direction +mu lands in the next aggregate iff x_mu mod b_mu = b_mu - 1;
  such terms form A_{1+2mu}, hops that stay inside the aggregate join A_0 with the diagonal
  (4 + m). Because the basis respects chirality, A_c^dagger = G5 A_c G5 with
  G5 = diag(+1 (chi = 0), -1 (chi = 1)).
* Near-null vectors: each phi_k is replaced `rounds` times by iters iterations of CG on
  D^dagger D phi' = phi (from zero), normalised to unit length, then block-orthonormalised.
* Preconditioner K(r) (one two-level cycle): r_c = R r; e_c from CGNR on A_c (at most n_c
  iterations from zero, stopping when the normal-equation residual falls below tol_c times its
  start); z = P e_c; then nu minimal-residual steps on D z = r (s = r - D z; t = D s;
  alpha = <t, s> / <t, t>; z += alpha s; s -= alpha t).
* Outer solver: flexible GCR with restart m on D x = b: z_k = K(r), w_k = D z_k, w_k and z_k
  orthogonalised against the previous w_j (modified Gram-Schmidt) and scaled to |w_k| = 1,
  alpha = <w_k, r>, x += alpha z_k, r -= alpha w_k; at each restart and at the end r = b - D x is
  recomputed; stop when |b - D x| <= tol |b|.
* Multigrid pCG: flexible preconditioned CG on the Hermitian positive definite normal equations
  N x = D^dagger b, N = D^dagger D, preconditioned with M(rho) = K(G5 K(G5 rho)), K the two-level
  cycle above and G5 = gamma5 on the fine field: since D^dagger = G5 D G5, G5 K G5 approximates
  D^-dagger and M approximates N^-1 = D^-1 D^-dagger (with no smoothing and exact coarse solves
  M = P (A_c^dagger A_c)^-1 R, Hermitian positive semidefinite). M varies between iterations (the
  MR and coarse CG coefficients depend on rho), so each search direction
  p_k = z_k - sum_j (<N p_j, z_k> / <p_j, N p_j>) p_j is made N-conjugate to every earlier one kept
  (up to m, then the process restarts from the true residual), alpha_k = <p_k, rho_k> /
  <p_k, N p_k>, x += alpha_k p_k, rho -= alpha_k N p_k (flexible CG in Notay's form); stop when
  |b - D x| <= tol |b|.

Inner products are <a, b> = sum conj(a) b. Only the test-suite uses this module.
"""
from __future__ import annotations

import numpy as np

from . import oracle as _o

_AX = {0: 3, 1: 2, 2: 1, 3: 0}   # numpy axis of direction mu in (Lt, Lz, Ly, Lx, ...)


def coarse_dims(dims, block):
    """Coarse (Lx, Ly, Lz, Lt) for fine dims (Lx, Ly, Lz, Lt) and block (bx, by, bz, bt)."""
    for L, b in zip(dims, block):
        if b < 1 or L % b:
            raise ValueError("every block extent must divide the lattice extent")
    return tuple(L // b for L, b in zip(dims, block))


def _blocks(field, block):
    """View (Lct, bt, Lcz, bz, Lcy, by, Lcx, bx, 4, 3) of a fine field (Lt, Lz, Ly, Lx, 4, 3)."""
    lt, lz, ly, lx = field.shape[:4]
    bx, by, bz, bt = block
    return field.reshape(lt // bt, bt, lz // bz, bz, ly // by, by, lx // bx, bx, 4, 3)


def _chi_part(field, chi):
    """The spins of chirality chi of a fine field, others zero."""
    out = np.zeros_like(field)
    out[..., 2 * chi:2 * chi + 2, :] = field[..., 2 * chi:2 * chi + 2, :]
    return out


def orthonormalise(vecs, block):
    """Block Gram-Schmidt of vecs (nvec, Lt, Lz, Ly, Lx, 4, 3) per aggregate and chirality, as the
    thin QR factorisation with positive real diagonal."""
    vecs = np.array(vecs, dtype=np.complex128)
    nvec = vecs.shape[0]
    lt, lz, ly, lx = vecs.shape[1:5]
    bx, by, bz, bt = block
    # (nvec, Lct, bt, Lcz, bz, Lcy, by, Lcx, bx, 4, 3) -> per aggregate and chirality a matrix
    v = vecs.reshape(nvec, lt // bt, bt, lz // bz, bz, ly // by, by, lx // bx, bx, 4, 3)
    out = np.empty_like(v)
    for chi in (0, 1):
        sub = v[..., 2 * chi:2 * chi + 2, :]                   # (..., 2, 3)
        # move the aggregate axes to the front and the in-aggregate axes together
        a = sub.transpose(1, 3, 5, 7, 2, 4, 6, 8, 9, 10, 0)    # (Lct,Lcz,Lcy,Lcx, bt,bz,by,bx,2,3, nvec)
        shp = a.shape
        m = a.reshape(shp[0] * shp[1] * shp[2] * shp[3], -1, nvec)
        q = np.empty_like(m)
        for i in range(m.shape[0]):
            Q, Rm = np.linalg.qr(m[i])
            ph = np.diag(Rm) / np.abs(np.diag(Rm))
            q[i] = Q * ph[None, :]
        q = q.reshape(shp).transpose(10, 0, 4, 1, 5, 2, 6, 3, 7, 8, 9)
        out[..., 2 * chi:2 * chi + 2, :] = q
    return out.reshape(vecs.shape)


def restrict(vecs, psi, block):
    """(R psi)(xc)[chi nvec + k] = sum over the aggregate and the spins of chi of conj(phi_k) psi."""
    nvec = vecs.shape[0]
    lt, lz, ly, lx = psi.shape[:4]
    cd = coarse_dims((lx, ly, lz, lt), block)
    out = np.zeros((cd[3], cd[2], cd[1], cd[0], 2 * nvec), dtype=np.complex128)
    pb = _blocks(psi, block)
    for k in range(nvec):
        vb = _blocks(vecs[k], block)
        for chi in (0, 1):
            prod = np.conj(vb[..., 2 * chi:2 * chi + 2, :]) * pb[..., 2 * chi:2 * chi + 2, :]
            out[..., chi * nvec + k] = prod.sum(axis=(1, 3, 5, 7, 8, 9))
    return out


def prolong(vecs, vc, block):
    """(P v)(x)[s][c] = sum_k phi_k(x)[s][c] v(xc(x))[chi(s) nvec + k]."""
    nvec = vecs.shape[0]
    bx, by, bz, bt = block
    out = np.zeros(vecs.shape[1:], dtype=np.complex128)
    for chi in (0, 1):
        for k in range(nvec):
            c = vc[..., chi * nvec + k]
            cf = np.repeat(np.repeat(np.repeat(np.repeat(c, bt, 0), bz, 1), by, 2), bx, 3)
            out[..., 2 * chi:2 * chi + 2, :] += vecs[k][..., 2 * chi:2 * chi + 2, :] * cf[..., None, None]
    return out


def _dir_hop(U, t, mu, fwd):
    """The single hop term of H in direction mu: (1 - gamma_mu) U_mu(x) t(x + mu) (fwd) or
    (1 + gamma_mu) U_mu(x - mu)^dagger t(x - mu)."""
    g = _o.gamma(mu)
    one = np.eye(4)
    ax = _AX[mu]
    if fwd:
        tn = np.roll(t, -1, axis=ax)
        ut = np.einsum("...ab,...sb->...sa", U[..., mu, :, :], tn)
        return np.einsum("st,...tb->...sb", one - g, ut)
    Un = np.roll(U[..., mu, :, :], 1, axis=ax)
    tn = np.roll(t, 1, axis=ax)
    ut = np.einsum("...ba,...sb->...sa", np.conj(Un), tn)
    return np.einsum("st,...tb->...sb", one + g, ut)


def _face_mask(shape4, block, mu, fwd):
    """Fine sites whose hop in direction +mu (fwd) / -mu leaves their aggregate."""
    lt, lz, ly, lx = shape4
    b = block[mu]
    coord = np.arange(shape4[_AX[mu]])
    on = (coord % b == b - 1) if fwd else (coord % b == 0)
    sh = [1, 1, 1, 1]
    sh[_AX[mu]] = shape4[_AX[mu]]
    return np.broadcast_to(on.reshape(sh), shape4)


def coarse_operator(U, vecs, mass, block):
    """A_c = R D P as the 9-point stencil, shape (Lct, Lcz, Lcy, Lcx, 9, N, N), A[..., d, i, j]."""
    nvec = vecs.shape[0]
    N = 2 * nvec
    shape4 = vecs.shape[1:5]
    cd = coarse_dims((shape4[3], shape4[2], shape4[1], shape4[0]), block)
    A = np.zeros((cd[3], cd[2], cd[1], cd[0], 9, N, N), dtype=np.complex128)
    for chi2 in (0, 1):
        for k2 in range(nvec):
            j = chi2 * nvec + k2
            t = _chi_part(vecs[k2], chi2)                   # P e_j on every aggregate at once
            parts = {0: (4.0 + mass) * t}
            for mu in range(4):
                for fwd in (True, False):
                    h = -0.5 * _dir_hop(U, t, mu, fwd)
                    face = _face_mask(shape4, block, mu, fwd)[..., None, None]
                    d = 1 + 2 * mu if fwd else 2 + 2 * mu
                    parts[d] = np.where(face, h, 0.0)
                    parts[0] = parts[0] + np.where(face, 0.0, h)
            for d, f in parts.items():
                A[..., d, :, j] = restrict(vecs, f, block)
    return A


def coarse_apply(A, v, dag=False):
    """(A v)(xc) = sum_d A_d(xc) v(xc + e_d); dag: (A^dagger v)(xc) = sum_d A_d(xc - e_d)^dagger v(xc - e_d)."""
    out = np.zeros_like(v)
    for d in range(9):
        if d == 0:
            shift = None
        else:
            mu, fwd = (d - 1) // 2, (d - 1) % 2 == 0
            shift = (_AX[mu], -1 if fwd else 1)
        if not dag:
            vn = v if shift is None else np.roll(v, shift[1], axis=shift[0])
            out += np.einsum("...ij,...j->...i", A[..., d, :, :], vn)
        else:
            # term of the adjoint reaching xc from xc - e_d
            An = A[..., d, :, :] if shift is None else np.roll(A[..., d, :, :], -shift[1], axis=shift[0])
            vn = v if shift is None else np.roll(v, -shift[1], axis=shift[0])
            out += np.einsum("...ji,...j->...i", np.conj(An), vn)
    return out


def gamma5_coarse(v):
    nvec = v.shape[-1] // 2
    out = v.copy()
    out[..., nvec:] *= -1.0
    return out


def _dot(a, b):
    return complex(np.vdot(a.ravel(), b.ravel()))


def coarse_cgnr(A, rc, iters, tol):
    """CG on A^dagger A e = A^dagger rc from zero; at most iters iterations, stop when the
    normal-equation residual is below tol times its start."""
    e = np.zeros_like(rc)
    r = coarse_apply(A, rc, dag=True)
    p = r.copy()
    rho = _dot(r, r).real
    stop = tol * tol * rho
    for _ in range(iters):
        if rho <= stop or rho == 0.0:
            break
        q = coarse_apply(A, coarse_apply(A, p), dag=True)
        alpha = rho / _dot(p, q).real
        e = e + alpha * p
        r = r - alpha * q
        rho_new = _dot(r, r).real
        p = r + (rho_new / rho) * p
        rho = rho_new
    return e


def near_null(U, vecs, mass, rounds, iters):
    """rounds x (iters CG iterations on D^dagger D from zero, unit normalisation)."""
    op = _o.Op.wilson(mass)
    out = np.array(vecs, dtype=np.complex128)
    for _ in range(rounds):
        for k in range(out.shape[0]):
            x, _, _, _ = _o.cg(op, U, out[k], tol=1e-300, maxiter=iters)
            out[k] = x / np.linalg.norm(x)
    return out


def precondition(U, vecs, A, r, mass, block, coarse_iters, coarse_tol, smooth_iters):
    rc = restrict(vecs, r, block)
    ec = coarse_cgnr(A, rc, coarse_iters, coarse_tol)
    z = prolong(vecs, ec, block)
    s = r - _o.wilson(U, z, mass)
    for _ in range(smooth_iters):
        t = _o.wilson(U, s, mass)
        alpha = _dot(t, s) / _dot(t, t)
        z = z + alpha * s
        s = s - alpha * t
    return z


def fgcr(U, vecs, A, b, mass, block, tol=1e-10, maxiter=200, restart=8, coarse_iters=50, coarse_tol=0.05,
         smooth_iters=3):
    """Flexible GCR with the two-level preconditioner; returns (x, iterations, |b - D x| / |b|)."""
    x = np.zeros_like(b)
    bn = np.linalg.norm(b)
    r = b.copy()
    it = 0
    Z, W = [], []
    while np.linalg.norm(r) > tol * bn and it < maxiter:
        z = precondition(U, vecs, A, r, mass, block, coarse_iters, coarse_tol, smooth_iters)
        w = _o.wilson(U, z, mass)
        for zj, wj in zip(Z, W):
            beta = _dot(wj, w)
            w = w - beta * wj
            z = z - beta * zj
        nw = np.linalg.norm(w)
        w, z = w / nw, z / nw
        alpha = _dot(w, r)
        x = x + alpha * z
        r = r - alpha * w
        Z.append(z)
        W.append(w)
        it += 1
        if len(Z) == restart:
            Z, W = [], []
            r = b - _o.wilson(U, x, mass)
    r = b - _o.wilson(U, x, mass)
    return x, it, float(np.linalg.norm(r) / bn)


def gamma5(v):
    """gamma5 v on a fine field: +1 on spins 0, 1 and -1 on spins 2, 3."""
    out = np.array(v, dtype=np.complex128)
    out[..., 2:4, :] *= -1
    return out


def normal(U, v, mass):
    """D^dagger D v."""
    return _o.wilson(U, _o.wilson(U, v, mass), mass, dag=True)


def normal_cycle(U, vecs, A, rho, mass, block, coarse_iters, coarse_tol, smooth_iters):
    """M(rho) = K(G5 K(G5 rho)), the pCG preconditioner."""
    y = gamma5(precondition(U, vecs, A, gamma5(rho), mass, block, coarse_iters, coarse_tol, smooth_iters))
    return precondition(U, vecs, A, y, mass, block, coarse_iters, coarse_tol, smooth_iters)


def fcg(U, vecs, A, b, mass, block, tol=1e-10, maxiter=200, restart=8, coarse_iters=50, coarse_tol=0.05,
        smooth_iters=2, precondition=True):
    """Multigrid-preconditioned flexible CG on D^dagger D x = D^dagger b (precondition=False: the
    identity in place of the cycle). Returns (x, iterations, |b - D x| / |b|)."""
    x = np.zeros_like(b)
    bn = np.linalg.norm(b)
    rho = _o.wilson(U, b, mass, dag=True)
    it = 0
    P, NP = [], []
    while np.linalg.norm(b - _o.wilson(U, x, mass)) > tol * bn and it < maxiter:
        z = normal_cycle(U, vecs, A, rho, mass, block, coarse_iters, coarse_tol, smooth_iters) \
            if precondition else rho.copy()
        p = z.copy()
        for pj, npj in zip(P, NP):
            p = p - (_dot(npj, z) / _dot(pj, npj)) * pj
        n_p = normal(U, p, mass)
        alpha = _dot(p, rho) / _dot(p, n_p)
        x = x + alpha * p
        rho = rho - alpha * n_p
        P.append(p)
        NP.append(n_p)
        it += 1
        if len(P) == restart:
            P, NP = [], []
            rho = _o.wilson(U, b - _o.wilson(U, x, mass), mass, dag=True)
    r = b - _o.wilson(U, x, mass)
    return x, it, float(np.linalg.norm(r) / bn)
