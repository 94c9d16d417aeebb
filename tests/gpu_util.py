"""Helpers for GPU parity tests: host <-> device marshalling and precision round-trips.

Inputs for every precision are derived on the host from the same FP64 seeded fields, so the
oracle can be evaluated on exactly the values the kernel reads.
"""
from __future__ import annotations

import numpy as np
import torch

import oracle.oracle as O

DEV = torch.device("cuda:0")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    if hasattr(t, "codes"):
        return O.fp16_decode(t.codes.cpu().numpy(), t.scale.cpu().numpy())
    return t.cpu().numpy()


def rel(a, b) -> float:
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def links_f16(U):
    """FP64 links -> half (re, im) via float32, as the library's narrowing does."""
    u32 = np.asarray(U).astype(np.complex64)
    return np.stack([u32.real, u32.imag], axis=-1).astype(np.float16)


def links_f16_decoded(U16):
    u = np.asarray(U16).astype(np.float64)
    return u[..., 0] + 1j * u[..., 1]


def as_prec(U, psi, prec: str, fmt: str = "L18"):
    """Device inputs in precision prec ("f64" | "f32" | "f16s") plus the FP64 values they hold.

    Returns (U_dev, psi_dev, U_ref, psi_ref): the oracle evaluated on (U_ref, psi_ref) is the exact
    result for the stored inputs.
    """
    from paper_1512_03487_amd import F16Spinor
    if prec == "f64":
        Uk, Ur = U, U
        pk, pr = dev(psi), psi
    elif prec == "f32":
        Uk = U.astype(np.complex64)
        Ur = Uk.astype(np.complex128)
        p32 = psi.astype(np.complex64)
        pk, pr = dev(p32), p32.astype(np.complex128)
    else:
        Uk = links_f16(U)
        Ur = links_f16_decoded(Uk)
        codes, scale = O.fp16_encode(psi, site_axes=2)
        pk = F16Spinor(dev(codes), dev(scale))
        pr = O.fp16_decode(codes, scale)
    if fmt == "L12":
        Uk = np.ascontiguousarray(Uk[..., :2, :, :] if prec == "f16s" else Uk[..., :2, :])
        # the kernel rebuilds row 2 from the stored rows, in its own precision
        rows = links_f16_decoded(Uk) if prec == "f16s" else Uk.astype(np.complex128)
        Ur = O.reconstruct12(rows)
    return dev(Uk), pk, Ur, pr


_cache = {}


def cached(what: str, dims, seed: int, **kw):
    """Seeded fields, generated once per process (large lattices take seconds to draw)."""
    from paper_1512_03487_amd import fields as F
    key = (what, tuple(dims), seed, tuple(sorted(kw.items())))
    if key not in _cache:
        if what == "gauge":
            a = F.gauge_field(dims, seed=seed, **kw)
        else:
            a = F.spinor_field(dims, seed=seed, **kw)
        a.setflags(write=False)
        _cache[key] = a
    return _cache[key]
