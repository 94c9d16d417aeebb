"""Hybrid Monte Carlo trajectories on top of the library's molecular-dynamics entry points.

The host draws the random numbers (Gaussian momenta, the pseudofermion source, the Metropolis
uniform) from a seeded numpy Generator and takes the accept / reject decision; every field
operation (forces, link updates, solves, energies) runs in the HIP library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api
from .fields import GELL_MANN


def gaussian_momenta(shape4, rng: np.random.Generator) -> np.ndarray:
    """P = i sum_a h_a lambda_a / 2 per link, h_a ~ N(0, 1): the distribution exp(-tr P^dagger P)."""
    h = rng.standard_normal(tuple(shape4) + (4, 8))
    return np.ascontiguousarray(1j * np.einsum("...a,aij->...ij", h, GELL_MANN) / 2.0)


def gaussian_spinor(shape, rng: np.random.Generator) -> np.ndarray:
    """Complex Gaussian with <|eta|^2> = 1 per component (re, im ~ N(0, 1/2))."""
    return ((rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)).astype(np.complex128)


def trajectory(U, beta, eps, n_steps, rng, fermion=None, integrator="leapfrog", **cg):
    """One HMC trajectory. fermion: None (pure gauge) or dict(kind, Ls, mass / M5, mf, b5, c5
    for "mobius") for a two-flavour pseudofermion phi = Op^dagger eta; integrator "leapfrog",
    "omelyan" or "force_gradient" (n_inner in cg for two time scales). Returns
    (U_new, accepted, dH, info); U is not modified."""
    dev = U.device
    shape4 = tuple(U.shape[:4])
    P = torch.from_numpy(gaussian_momenta(shape4, rng)).to(dev)
    phi, kw = None, {}
    if fermion is not None:
        f = dict(fermion)
        Ls = f.pop("Ls", 1)
        kw = dict(kind=f.pop("kind"), **f)
        site = shape4 + ((Ls,) if Ls > 1 else ()) + (4, 3)
        eta = torch.from_numpy(gaussian_spinor(site, rng)).to(dev)
        if kw["kind"] == "mobius":
            phi = api.mobius(U, eta, kw.get("M5", 1.8), kw.get("mf", 0.01), kw.get("b5", 1.0), kw.get("c5", 0.0),
                             dag=True)
        else:
            phi = api.dhop(U, eta, kw["kind"], dag=True, mass=kw.get("mass", 0.0), M5=kw.get("M5", 1.8),
                           mf=kw.get("mf", 0.01))
    e0 = api.hmc_energy(U, P, beta, phi, **kw, **cg)
    U1, P1 = U.clone(), P.clone()
    st = api.md_leapfrog(U1, P1, beta, eps, n_steps, phi, integrator=integrator, **kw, **cg)
    e1 = api.hmc_energy(U1, P1, beta, phi, **kw, **cg)
    dH = e1["H"] - e0["H"]
    accepted = bool(rng.uniform() < np.exp(-dH))
    return (U1 if accepted else U), accepted, dH, {"md": st, "start": e0, "end": e1}
