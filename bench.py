"""Benchmark: Wilson hopping operator GFLOP/s and HBM GB/s on one MI355X at the throughput size
(32^4, FP32), the domain-wall operator at 24^4 x 12, and the domain-wall CG time to a true
residual of 1e-10 in FP64 and in mixed precision.

One "step" is one application of the hopping operator H on a 32^4 lattice with FP32 spinors and
18-real FP32 links (Haar links, Gaussian spinor; 1320 flop per site). The timed loop rotates over
two independent (U, psi, out) buffer sets of 403 MB of inputs each, three times the 256 MB
last-level cache, so every application streams its inputs from HBM. It is timed after the
operator legs, with the device at its working clocks. Further legs (the
domain-wall operator on 24^4 x 12 in FP32 and FP16 storage with their own roofline records,
16^4 FP64, the CG on 16^4 x 16, the even-odd preconditioned solve, recorded-graph CG iterations,
multigrid and HMC kernels) are reported alongside.

Usage: python bench.py [--gpus 1] [--steps 100] [--warmup 10] [--no-cg] [--no-cpu] [--oracle-cg]
Prints one JSON line (progress lines go to stderr).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Dhop GFLOP/s & HBM GB/s (1320 flop/site); DWF CG time-to-1e-10 mixed vs FP64"
HBM_PEAK_GBS = 8000.0
FLOPS_HOP = 1320
# algorithmic bytes per site: read psi once, the 4 links of the site once, write out once
SPINOR_BYTES = {"f64": 192, "f32": 96, "f16s": 52}
LINK_BYTES = {("f64", "L18"): 144, ("f64", "L12"): 96, ("f32", "L18"): 72, ("f32", "L12"): 48,
              ("f16s", "L18"): 36, ("f16s", "L12"): 24}
# HBM traffic summaries (rocprofv3 FETCH_SIZE / WRITE_SIZE, copy-calibrated) of the timed kernels
TRAFFIC_FILES = {
    "hop_32^4_f32": os.path.join(ROOT, "profiles", "traffic_dhop_f32_32x32x32x32.txt"),
    "dwf_24^4x12_f32": os.path.join(ROOT, "profiles", "traffic_dwf_f32_24x24x24x24_ls12.txt"),
    "dwf_24^4x12_f16s_L12": os.path.join(ROOT, "profiles", "traffic_dwf_f16s_24x24x24x24_ls12.txt"),
    "dwf_24^4x12_f32_L12": os.path.join(ROOT, "profiles", "traffic_dwf_f32_L12_24x24x24x24_ls12.txt"),
    "dwf_24^4x12_f16s_L18": os.path.join(ROOT, "profiles", "traffic_dwf_f16s_L18_24x24x24x24_ls12.txt"),
}
ORACLE_CG_FILE = os.path.join(ROOT, "profiles", "oracle_cg_dwf_16x16x16x16_ls16.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1512_03487_amd", "csrc", f) for f in ("dhop.hip", "device.h")]
HEAD_DIMS = (32, 32, 32, 32)
HEAD_KERNEL = "k_dhop_dir<SpF32, LkF32<3>, hop>"


def progress(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def alg_bytes_per_site(prec: str, fmt: str, Ls: int) -> float:
    return 2 * SPINOR_BYTES[prec] + 4 * LINK_BYTES[(prec, fmt)] / Ls


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(name="hop_32^4_f32"):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it matches the source."""
    path = TRAFFIC_FILES[name]
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def make_sets(dims, prec, nsets, seed_u=1, seed_psi=2, kind="weak", Ls=None, fmt="L18"):
    """nsets device copies of one seeded (U, psi) pair (traffic does not depend on the values)."""
    import numpy as np
    import torch
    import paper_1512_03487_amd as gm
    from paper_1512_03487_amd import fields
    dev = torch.device("cuda:0")
    U = fields.gauge_field(dims, seed=seed_u, kind=kind)
    psi = fields.spinor_field(dims, seed=seed_psi, Ls=Ls)
    Ud = torch.from_numpy(U).to(dev)
    pd = torch.from_numpy(psi).to(dev)
    if prec == "f64":
        Uk = Ud if fmt == "L18" else Ud[..., :2, :].contiguous()
        pk = pd
    else:
        Uk = gm.convert_links(Ud, prec, fmt)
        pk = gm.convert_spinor(pd, prec)
    del Ud, pd
    sets = []
    for _ in range(nsets):
        if prec == "f16s":
            p = gm.F16Spinor(pk.codes.clone(), pk.scale.clone())
            o = gm.F16Spinor(torch.empty_like(pk.codes), torch.empty_like(pk.scale))
        else:
            p = pk.clone()
            o = torch.empty_like(pk)
        sets.append((Uk.clone(), p, o))
    torch.cuda.synchronize()
    return sets, (U, psi)


# Legs run their operator untimed for this long before timing it: after host-side set-up (the
# seeded fields are drawn on the host) the device has idled and its clocks have dropped, and the
# first tens of milliseconds of work then run up to 10 % slower.
SETTLE_S = 0.05


def settle(run, seconds=SETTLE_S):
    """Call run(i), i = 0, 1, ..., untimed until `seconds` of wall time have passed."""
    import torch
    t0 = time.perf_counter()
    i = 0
    while True:
        run(i)
        i += 1
        if i % 8 == 0:
            torch.cuda.synchronize()
            if time.perf_counter() - t0 >= seconds:
                break
    torch.cuda.synchronize()


def time_dhop(sets, steps, warmup, kind="hop", settle_s=0.0, **kw):
    """Average seconds per application over `steps` launches rotating over `sets` (HIP events),
    after `warmup` untimed ones (and, for legs, `settle_s` seconds of untimed ones before those)."""
    import torch
    import paper_1512_03487_amd as gm
    if settle_s > 0:
        settle(lambda i: gm.dhop(sets[i % len(sets)][0], sets[i % len(sets)][1], kind, out=sets[i % len(sets)][2], **kw),
               settle_s)
    for i in range(warmup):
        U, p, o = sets[i % len(sets)]
        gm.dhop(U, p, kind, out=o, **kw)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for i in range(steps):
        U, p, o = sets[i % len(sets)]
        gm.dhop(U, p, kind, out=o, **kw)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) * 1e-3 / steps, wall


def copy_reference(nbytes, nsets=12, steps=100, warmup=10):
    """A plain device copy moving `nbytes` per launch (half read, half written), its sources rotated
    over `nsets` buffers like the headline's inputs: what a launch of this size reaches from HBM."""
    import torch
    dev = torch.device("cuda:0")
    n = int(nbytes // 8)   # float32 elements per side
    srcs = [torch.ones(n, dtype=torch.float32, device=dev) for _ in range(nsets)]
    dst = torch.empty(n, dtype=torch.float32, device=dev)
    settle(lambda i: dst.copy_(srcs[i % nsets]))
    for i in range(warmup):
        dst.copy_(srcs[i % nsets])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        dst.copy_(srcs[i % nsets])
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / steps
    moved = 8 * n
    del srcs, dst
    return {"bytes_per_launch": moved, "us_per_launch": round(t * 1e6, 2), "gbs": round(moved / t / 1e9, 1),
            "roofline_frac": round(moved / t / 1e9 / HBM_PEAK_GBS, 4), "buffer_sets": nsets}


def link_force_leg(dims=(32, 32, 32, 32), steps=20, warmup=3, nsets=2):
    """The link force of the hopping term (grid_dhop_backward, FP32, su(3)-projected): per site it
    reads chi and psi (2 x 96 B) and the 4 links (288 B) and writes the 4 force matrices (288 B)."""
    import torch
    import paper_1512_03487_amd as gm
    from paper_1512_03487_amd import fields
    dev = torch.device("cuda:0")
    vol = dims[0] * dims[1] * dims[2] * dims[3]
    U = torch.from_numpy(fields.gauge_field(dims, seed=1, kind="haar")).to(dev).to(torch.complex64)
    g = torch.Generator(device=dev).manual_seed(3)
    shape = (dims[3], dims[2], dims[1], dims[0], 4, 3)
    sets = []
    for _ in range(nsets):
        mk = lambda: torch.complex(torch.randn(shape, generator=g, device=dev), torch.randn(shape, generator=g, device=dev))
        sets.append((U.clone(), mk(), mk()))
    settle(lambda i: gm.dhop_backward(sets[i % nsets][0], sets[i % nsets][1], sets[i % nsets][2], want_psi=False,
                                      force=True))
    for i in range(warmup):
        Uk, psi, chi = sets[i % nsets]
        gm.dhop_backward(Uk, psi, chi, want_psi=False, force=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        Uk, psi, chi = sets[i % nsets]
        gm.dhop_backward(Uk, psi, chi, want_psi=False, force=True)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / steps
    nbytes = (2 * 96 + 288 + 288) * vol
    del sets, U
    return {"lattice": list(dims), "prec": "f32", "us_per_launch": round(t * 1e6, 2),
            "alg_bytes_per_launch": nbytes, "alg_gbs": round(nbytes / t / 1e9, 1),
            "roofline_frac": round(nbytes / t / 1e9 / HBM_PEAK_GBS, 4), "buffer_sets": nsets}


def cb_leg(dims, Ls, prec, fmt, steps=50, warmup=5, nsets=4):
    """The even-odd hop with the domain-wall diagonal, out (parity 0) = M5 y - H psi / 4, on one
    checkerboard: per output 5D site it reads psi (the other parity) and y once, writes out once,
    and reads 8 links per 4D site (one parity's outputs touch every link)."""
    import torch
    import paper_1512_03487_amd as gm
    from paper_1512_03487_amd import fields
    dev = torch.device("cuda:0")
    Lt, Lz, Ly, Lx = dims[3], dims[2], dims[1], dims[0]
    U = torch.from_numpy(fields.gauge_field(dims, seed=1, kind="haar")).to(dev)
    Uk = U.to(torch.complex64) if prec == "f32" else gm.convert_links(U, "f16s", fmt)
    g = torch.Generator(device=dev).manual_seed(9)
    shape = (Lt, Lz, Ly, Lx // 2, Ls, 4, 3)

    def field():
        v = torch.complex(torch.randn(shape, generator=g, device=dev), torch.randn(shape, generator=g, device=dev))
        return v if prec == "f32" else gm.convert_spinor(v, "f16s")
    sets = [(field(), field(), field()) for _ in range(nsets)]
    run = lambda i: gm.dhop_cb(Uk, sets[i % nsets][0], 0, "dwf", y=sets[i % nsets][1], beta=-0.25, M5=1.8, mf=0.01,
                               out=sets[i % nsets][2])
    settle(run)
    for i in range(warmup):
        run(i)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        run(i)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / steps
    n5 = Lx // 2 * Ly * Lz * Lt * Ls
    nbytes = (3 * SPINOR_BYTES[prec] + 8 * LINK_BYTES[(prec, fmt)] / Ls) * n5
    del sets
    return {"lattice": list(dims), "Ls": Ls, "prec": prec, "links": fmt, "op": "dwf even-odd hop + diagonal",
            "us_per_launch": round(t * 1e6, 2), "alg_gbs": round(nbytes / t / 1e9, 1),
            "roofline_frac": round(nbytes / t / 1e9 / HBM_PEAK_GBS, 4), "buffer_sets": nsets}


def mobius_leg(dims, Ls, prec, steps, warmup, b5=1.5, c5=0.5, fmt="L18"):
    """Moebius operator M and M^dagger (grid_mobius); GB/s on the same algorithmic bytes as the
    Shamir operator (read psi and the links once, write out once)."""
    import torch
    import paper_1512_03487_amd as gm
    (U, p, o), = make_sets(dims, prec, 1, kind="haar", Ls=Ls, fmt=fmt)[0]
    tmp = gm.F16Spinor(torch.empty_like(p.codes), torch.empty_like(p.scale)) if prec == "f16s" else torch.empty_like(p)
    n5 = dims[0] * dims[1] * dims[2] * dims[3] * Ls
    out = {"lattice": list(dims), "Ls": Ls, "prec": prec, "links": fmt, "b5": b5, "c5": c5}
    for dag in (False, True):
        settle(lambda i: gm.mobius(U, p, 1.8, 0.01, b5, c5, dag=dag, out=o, tmp=tmp))
        for _ in range(warmup):
            gm.mobius(U, p, 1.8, 0.01, b5, c5, dag=dag, out=o, tmp=tmp)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            gm.mobius(U, p, 1.8, 0.01, b5, c5, dag=dag, out=o, tmp=tmp)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) * 1e-3 / steps
        gbs = alg_bytes_per_site(prec, fmt, Ls) * n5 / t / 1e9
        out["Mdag" if dag else "M"] = {"us_per_launch": round(t * 1e6, 2), "alg_gbs": round(gbs, 1),
                                       "roofline_frac": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def leg(dims, prec, fmt, kind, Ls, steps, warmup, min_bytes=600e6):
    sb = SPINOR_BYTES[prec] * (Ls or 1) + 4 * LINK_BYTES[(prec, fmt)]     # input bytes per site
    vol = dims[0] * dims[1] * dims[2] * dims[3]
    nsets = max(1, int(min_bytes // (sb * vol)) + 1)
    sets, _ = make_sets(dims, prec, nsets, kind="haar", Ls=Ls, fmt=fmt)
    t, _ = time_dhop(sets, steps, warmup, kind=kind, settle_s=SETTLE_S, M5=1.8, mf=0.01)
    n5 = vol * (Ls or 1)
    gbs = alg_bytes_per_site(prec, fmt, Ls or 1) * n5 / t / 1e9
    del sets
    return {"lattice": list(dims), "Ls": Ls or 1, "prec": prec, "links": fmt, "op": kind,
            "us_per_launch": round(t * 1e6, 2), "gflops": round(FLOPS_HOP * n5 / t / 1e9, 1),
            "alg_gbs": round(gbs, 1), "roofline_frac": round(gbs / HBM_PEAK_GBS, 4), "buffer_sets": nsets}


def cg_legs(keep_solutions=False):
    import torch
    import paper_1512_03487_amd as gm
    from paper_1512_03487_amd import fields
    dev = torch.device("cuda:0")
    dims, Ls = (16, 16, 16, 16), 16
    U = torch.from_numpy(fields.gauge_field(dims, seed=1, kind="haar")).to(dev)
    b = torch.from_numpy(fields.spinor_field(dims, seed=3, Ls=Ls)).to(dev)
    out = {"lattice": list(dims), "Ls": Ls, "M5": 1.8, "mf": 0.01, "tol": 1e-10}
    sols = {}
    # FP16-storage sloppy iterations with 18-real FP16 links: for the domain-wall walks faster than
    # 12-real links (the 12-real row reconstruction costs more than the bytes it saves)
    for name, sloppy, fmt in (("fp64", "f64", "L18"), ("mixed_f32", "f32", "L18"), ("mixed_f16s", "f16s", "L18")):
        ws = torch.empty(gm.cg_workspace_bytes(b, sloppy=sloppy, link_fmt=fmt), dtype=torch.uint8, device=dev)
        gm.cg(U, b, kind="dwf", M5=1.8, mf=0.01, tol=1e-10, sloppy=sloppy, link_fmt=fmt, workspace=ws,
              maxiter=20, raise_on_fail=False)   # warm-up: touches the workspace
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = gm.cg(U, b, kind="dwf", M5=1.8, mf=0.01, tol=1e-10, sloppy=sloppy, link_fmt=fmt, workspace=ws)
        torch.cuda.synchronize()
        out[name] = {"seconds": round(time.perf_counter() - t0, 4), "iterations": st["iterations"],
                     "reliable_updates": st["reliable_updates"], "true_residual": st["true_residual"],
                     "converged": st["converged"]}
        if name == "fp64":
            x64 = x
        else:
            # the solution is unique only up to the tolerance: its distance to the FP64 solve's
            out[name]["rel_error_vs_fp64_solution"] = float(torch.linalg.vector_norm(x - x64) /
                                                            torch.linalg.vector_norm(x64))
        sols[name] = x.cpu().numpy() if keep_solutions else None
        del ws, x
    mob = dict(kind="mobius", M5=1.8, mf=0.01, b5=1.5, c5=0.5, tol=1e-10)
    xm64 = None
    for name, sloppy in (("mobius_b1.5_c0.5_fp64", "f64"), ("mobius_b1.5_c0.5_mixed_f32", "f32")):
        ws = torch.empty(gm.cg_workspace_bytes(b, sloppy=sloppy), dtype=torch.uint8, device=dev)
        gm.cg(U, b, sloppy=sloppy, workspace=ws, maxiter=20, raise_on_fail=False, **mob)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = gm.cg(U, b, sloppy=sloppy, workspace=ws, **mob)
        torch.cuda.synchronize()
        out[name] = {"seconds": round(time.perf_counter() - t0, 4), "iterations": st["iterations"],
                     "reliable_updates": st["reliable_updates"], "true_residual": st["true_residual"],
                     "converged": st["converged"]}
        if xm64 is None:
            xm64 = x
        else:
            out[name]["rel_error_vs_fp64_solution"] = float(torch.linalg.vector_norm(x - xm64) /
                                                            torch.linalg.vector_norm(xm64))
        del ws, x
    del xm64
    out["speedup_mixed_f32"] = round(out["fp64"]["seconds"] / out["mixed_f32"]["seconds"], 2)
    out["speedup_mixed_f16s"] = round(out["fp64"]["seconds"] / out["mixed_f16s"]["seconds"], 2)
    return (out, sols) if keep_solutions else out


def eo_legs(kind="dwf"):
    """M x = b on the 16^4 x 16 domain-wall workload (kind "dwf": the Shamir M; "mobius": the
    Moebius M with b5 = 1.5, c5 = 0.5): CG on M^dagger M (source M^dagger b) against even-odd
    preconditioned CG, each in FP64 and mixed precision, to a normal-equation residual of 1e-10;
    the full residual |b - M x| / |b| is reported for both."""
    import torch
    import paper_1512_03487_amd as gm
    from paper_1512_03487_amd import fields
    dev = torch.device("cuda:0")
    dims, Ls = (16, 16, 16, 16), 16
    U = torch.from_numpy(fields.gauge_field(dims, seed=1, kind="haar")).to(dev)
    b = torch.from_numpy(fields.spinor_field(dims, seed=3, Ls=Ls)).to(dev)
    bn = float(torch.linalg.vector_norm(b))
    kw = dict(M5=1.8, mf=0.01) if kind == "dwf" else dict(M5=1.8, mf=0.01, b5=1.5, c5=0.5)
    out = {"lattice": list(dims), "Ls": Ls, **kw, "tol": 1e-10, "system": "M x = b"}

    def op(x, dag=False):
        return gm.dwf(U, x, dag=dag, **kw) if kind == "dwf" else gm.mobius(U, x, dag=dag, **kw)

    def full_res(x):
        return float(torch.linalg.vector_norm(op(x) - b)) / bn

    # FP16-storage sloppy iterations with 18-real FP16 links: for the domain-wall walks faster than
    # 12-real links (the 12-real row reconstruction costs more than the bytes it saves)
    for name, sloppy, fmt in (("fp64", "f64", "L18"), ("mixed_f32", "f32", "L18"), ("mixed_f16s", "f16s", "L18")):
        ws = torch.empty(gm.cg_workspace_bytes(b, sloppy=sloppy, link_fmt=fmt), dtype=torch.uint8, device=dev)
        gm.cg(U, b, kind=kind, tol=1e-10, sloppy=sloppy, link_fmt=fmt, workspace=ws, maxiter=20, raise_on_fail=False,
              **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c = op(b, dag=True)
        x, st = gm.cg(U, c, kind=kind, tol=1e-10, sloppy=sloppy, link_fmt=fmt, workspace=ws, **kw)
        torch.cuda.synchronize()
        t_full = time.perf_counter() - t0
        r_full = full_res(x)
        del ws, x, c
        ws = torch.empty(gm.solve_eo_workspace_bytes(b, sloppy=sloppy, link_fmt=fmt), dtype=torch.uint8, device=dev)
        gm.solve_eo(U, b, kind=kind, tol=1e-10, sloppy=sloppy, link_fmt=fmt, workspace=ws, maxiter=20,
                    raise_on_fail=False, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, ste = gm.solve_eo(U, b, kind=kind, tol=1e-10, sloppy=sloppy, link_fmt=fmt, workspace=ws, **kw)
        torch.cuda.synchronize()
        t_eo = time.perf_counter() - t0
        out[name] = {"cgnr": {"seconds": round(t_full, 4), "iterations": st["iterations"],
                              "full_residual": r_full},
                     "even_odd": {"seconds": round(t_eo, 4), "iterations": ste["iterations"],
                                  "full_residual": ste["true_residual"], "full_residual_recomputed": full_res(x)},
                     "speedup_even_odd": round(t_full / t_eo, 2)}
        if name == "fp64":
            x_eo64 = x
        else:
            out[name]["even_odd"]["rel_error_vs_fp64_solution"] = float(
                torch.linalg.vector_norm(x - x_eo64) / torch.linalg.vector_norm(x_eo64))
        del ws, x
    return out


# Bytes per 5D site and sloppy iteration beyond the two operator applications (each: input,
# output, links): the second one also reads r (its output is r - alpha op^dagger t), and the x/p
# update reads x_hat (FP32), p, r and writes x_hat, p. Spinors: FP32 96, FP16 storage 52 bytes.
CG_VEC_BYTES = {"f32": 96 + (2 * 96 + 2 * 96 + 96), "f16s": 52 + (2 * 96 + 2 * 52 + 52)}
OP_FLOPS = {"wilson": 1368, "dwf": 1416}


def cg_iteration_legs():
    """Throughput of sloppy CG iterations (two operator applications, the second carrying the r
    update, and the x/p update)
    on Wilson D^dagger D at 32^4 and domain-wall M^dagger M at 24^4 x 12, Haar links, FP32 and
    FP16-storage spinors, with the iterations between host checks replayed from recorded HIP graphs
    and, for comparison, launched directly. Per-iteration time = (t(120 its) - t(20 its)) / 100, so
    the setup, the initial and final FP64 residuals and the workspace touch drop out; no reliable
    update occurs (delta = tol = 1e-30)."""
    import torch
    import paper_1512_03487_amd as gm
    from paper_1512_03487_amd import fields
    dev = torch.device("cuda:0")
    out = {}
    for name, dims, Ls, kind, kw in (("wilson_32^4", (32, 32, 32, 32), None, "wilson", dict(mass=0.1)),
                                     ("dwf_24^4x12", (24, 24, 24, 24), 12, "dwf", dict(M5=1.8, mf=0.01))):
        U = torch.from_numpy(fields.gauge_field(dims, seed=1, kind="haar")).to(dev)
        b = torch.from_numpy(fields.spinor_field(dims, seed=3, Ls=Ls)).to(dev)
        n5 = dims[0] * dims[1] * dims[2] * dims[3] * (Ls or 1)
        res = {"lattice": list(dims), "Ls": Ls or 1, "op": f"{kind} normal operator", **kw}
        for sloppy, fmt in (("f32", "L18"), ("f16s", "L12" if kind == "wilson" else "L18")):
            ws = torch.empty(gm.cg_workspace_bytes(b, sloppy=sloppy, link_fmt=fmt), dtype=torch.uint8, device=dev)
            per = {}
            for graph in (True, False):
                def run(n):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    x, st = gm.cg(U, b, kind=kind, tol=1e-30, delta=1e-30, maxiter=n, sloppy=sloppy, link_fmt=fmt,
                                  check_every=10, graph=graph, workspace=ws, raise_on_fail=False, **kw)
                    torch.cuda.synchronize()
                    assert st["iterations"] == n and st["reliable_updates"] == 0
                    return time.perf_counter() - t0
                run(20)
                t20 = run(20)
                t_it = (run(120) - t20) / 100
                per["graph" if graph else "direct"] = t_it
                per["t20_graph" if graph else "t20_direct"] = t20
            t_it = per["graph"]
            nbytes = (2 * alg_bytes_per_site(sloppy, fmt, Ls or 1) + CG_VEC_BYTES[sloppy]) * n5
            res[f"{sloppy}_{fmt}"] = {
                "ms_per_iteration": round(t_it * 1e3, 4),
                "ms_per_iteration_direct_launches": round(per["direct"] * 1e3, 4),
                # recording and instantiating the two segment graphs of a solve (created per solve):
                # the 20-iteration solve's extra time over direct launches, less the replays' gain
                "graph_recording_ms_per_solve": round(
                    (per["t20_graph"] - per["t20_direct"] - 20 * (per["graph"] - per["direct"])) * 1e3, 3),
                "alg_bytes_per_iteration": int(nbytes),
                "alg_gbs": round(nbytes / t_it / 1e9, 1), "roofline_frac": round(nbytes / t_it / 1e9 / HBM_PEAK_GBS, 4),
                "op_gflops": round(2 * OP_FLOPS[kind] * n5 / t_it / 1e9, 1)}
            del ws
        out[name] = res
        del U, b
        torch.cuda.empty_cache()
    return out


PCG_RESTART = 16   # directions the multigrid pCG keeps before a restart


def mg_legs(mass=-0.1, nvec=12, block=(4, 4, 4, 4)):
    """Multigrid: (1) the generic coarse stencil on the 8^4 coarse lattice of a 32^4 lattice with
    4^4 aggregates, N = 24 (its bytes are the 9 N^2 matrices per coarse site plus v and out);
    (2) the Wilson system D x = b at 24^4, weak-field links, m = -0.1, to |b - D x| / |b| <= 1e-10:
    setup (near-null vectors and the Galerkin operator), multigrid-preconditioned GCR (coarse
    CGNR <= 8 iterations to 0.25, four MR smoothing steps) and multigrid pCG (the same cycle twice
    per iteration) against FP64 CG on D^dagger D x = D^dagger b."""
    import numpy as np
    import torch
    import paper_1512_03487_amd as gm
    from paper_1512_03487_amd import fields
    dev = torch.device("cuda:0")
    out = {}
    N = 2 * nvec
    cshape = (8, 8, 8, 8)
    g = torch.Generator(device="cpu").manual_seed(5)
    A = torch.complex(torch.randn(cshape + (9, N, N), generator=g, dtype=torch.float64),
                      torch.randn(cshape + (9, N, N), generator=g, dtype=torch.float64)).to(dev)
    v = torch.complex(torch.randn(cshape + (N,), generator=g, dtype=torch.float64),
                      torch.randn(cshape + (N,), generator=g, dtype=torch.float64)).to(dev)
    o = torch.empty_like(v)
    for _ in range(3):
        gm.coarse_stencil(A, v, out=o)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(50):
        gm.coarse_stencil(A, v, out=o)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / 50
    nbytes = (A.numel() + 2 * v.numel()) * 16
    out["coarse_stencil_8^4_N24"] = {"us_per_launch": round(t * 1e6, 2), "alg_bytes": int(nbytes),
                                     "alg_gbs": round(nbytes / t / 1e9, 1),
                                     "roofline_frac": round(nbytes / t / 1e9 / HBM_PEAK_GBS, 4),
                                     "gflops": round(8 * 9 * N * N * np.prod(cshape) / t / 1e9, 1)}
    del A, v, o
    dims = (24, 24, 24, 24)
    U = torch.from_numpy(fields.gauge_field(dims, seed=1, kind="weak")).to(dev)
    b = torch.from_numpy(fields.spinor_field(dims, seed=3)).to(dev)
    vec0 = torch.from_numpy(np.stack([fields.spinor_field(dims, seed=11 + k) for k in range(nvec)])).to(dev)
    kw = dict(block=block, restart=8, coarse_iters=8, coarse_tol=0.25, smooth_iters=4, tol=1e-10, setup_prec="f32",
              cycle_prec="f32")
    ws = torch.empty(gm.mg_workspace_bytes(U, nvec=nvec, **kw), dtype=torch.uint8, device=dev)
    res = {"lattice": list(dims), "mass": mass, "links": "weak field exp(0.3 i H)", "block": list(block), "nvec": nvec,
           "tol": 1e-10, "setup_prec": "f32", "cycle_prec": "f32"}
    vecs = vec0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gm.mg_basis(U, vecs, mass, workspace=ws, setup_rounds=3, setup_iters=20, **kw)
    Ac = gm.mg_coarse_op(U, vecs, mass, workspace=ws, **kw)
    torch.cuda.synchronize()
    res["setup_seconds"] = round(time.perf_counter() - t0, 4)
    c = gm.wilson(U, b, mass=mass, dag=True)
    wsc = torch.empty(gm.cg_workspace_bytes(c), dtype=torch.uint8, device=dev)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    kwp = dict(kw, restart=PCG_RESTART)
    wsp = torch.empty(gm.mg_workspace_bytes(U, nvec=nvec, **kwp), dtype=torch.uint8, device=dev)
    t_mg, t_cg, t_pcg = [], [], []
    for _ in range(3):   # alternate, keep the fastest of each (clock and first-touch effects)
        t, (x, st) = timed(lambda: gm.mg_solve(U, vecs, Ac, b, mass, workspace=ws, **kw))
        t_mg.append(t)
        t, (xp, stp) = timed(lambda: gm.mg_pcg(U, vecs, Ac, b, mass, workspace=wsp, **kwp))
        t_pcg.append(t)
        t, (xc, stc) = timed(lambda: gm.cg(U, c, kind="wilson", mass=mass, tol=1e-10, workspace=wsc))
        t_cg.append(t)
    full = float(torch.linalg.vector_norm(gm.wilson(U, xc, mass=mass) - b) / torch.linalg.vector_norm(b))
    res["mg_gcr"] = {"seconds": round(min(t_mg), 4), "iterations": st["iterations"],
                     "true_residual": st["true_residual"]}
    res["mg_pcg"] = {"seconds": round(min(t_pcg), 4), "iterations": stp["iterations"], "restart": PCG_RESTART,
                     "true_residual": stp["true_residual"]}
    res["cg_normal_fp64"] = {"seconds": round(min(t_cg), 4), "iterations": stc["iterations"],
                             "full_residual": full}
    res["speedup_mg"] = round(min(t_cg) / min(t_mg), 2)
    res["speedup_mg_pcg"] = round(min(t_cg) / min(t_pcg), 2)
    del ws, wsc, wsp
    out["wilson_24^4_solve"] = res
    return out


def hmc_legs():
    """Molecular-dynamics kernels on 16^4 (FP64): gauge force and link update per launch, and one
    5-step leapfrog with a two-flavour Ls = 8 domain-wall pseudofermion (FP32-sloppy solves)."""
    import torch
    import paper_1512_03487_amd as gm
    from paper_1512_03487_amd import fields
    dev = torch.device("cuda:0")
    dims = (16, 16, 16, 16)
    vol = 16 ** 4
    U = torch.from_numpy(fields.gauge_field(dims, seed=1, kind="weak")).to(dev)
    P = torch.from_numpy(fields.random_su3_algebra(dims, seed=7)).to(dev)
    out = {"lattice": list(dims)}

    def timed(fn, n=20):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / n

    F = torch.empty_like(U)
    t = timed(lambda: gm.gauge_force(U, 5.7, out=F))
    out["gauge_force"] = {"us_per_launch": round(t * 1e6, 2), "alg_gbs": round(2 * 576 * vol / t / 1e9, 1)}
    Uc = U.clone()
    t = timed(lambda: gm.link_exp(Uc, P, 1e-3))
    out["link_exp"] = {"us_per_launch": round(t * 1e6, 2), "alg_gbs": round(3 * 576 * vol / t / 1e9, 1)}
    Ls = 8
    phi = torch.from_numpy(fields.spinor_field(dims, seed=5, Ls=Ls)).to(dev)
    U1, P1 = U.clone(), P.clone()
    st = gm.md_leapfrog(U1, P1, 5.7, 0.02, 5, phi, kind="dwf", M5=1.8, mf=0.1, tol=1e-8, sloppy="f32")
    out["leapfrog_5_steps_dwf_ls8"] = {"seconds": round(st["seconds"], 4), "solves": st["solves"],
                                      "cg_iterations": st["cg_iterations"], "failed_solves": st["failed_solves"]}
    return out


def cpu_baseline(U_host, psi_host, seconds_target=15.0):
    """The FP64 oracle's H on the headline workload (the same Haar links and Gaussian spinor, FP32-
    rounded, in FP64), timed on the host cores for about seconds_target; plus the oracle on one
    thread, its domain-wall normal operator per application, and its full FP64 CG at 16^4 x 16
    as measured by `bench.py --oracle-cg` (the committed record, see oracle_cg_leg)."""
    import numpy as np
    from oracle import oracle as orc
    U = np.asarray(U_host).astype(np.complex64).astype(np.complex128)
    psi = np.asarray(psi_host).astype(np.complex64).astype(np.complex128)
    orc.hop(U, psi)    # load / warm
    n, t0 = 0, time.perf_counter()
    while True:
        orc.hop(U, psi)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds_target:
            break
    vol = int(np.prod(HEAD_DIMS))
    res = {"value": round(FLOPS_HOP * vol * n / el / 1e9, 3), "unit": "GFLOP/s", "cores": orc.threads(),
           "kind": "oracle",
           "sample": f"{n} applications of H on the 32^4 workload (FP32-rounded inputs, FP64 oracle, {el:.1f} s)",
           "cpu_model": _cpu_model()}
    del U, psi
    res["single_thread"] = _oracle_single_thread()
    from paper_1512_03487_amd import fields
    dims = (16, 16, 16, 16)
    U16 = fields.gauge_field(dims, seed=1, kind="haar")
    psi5 = fields.spinor_field(dims, seed=3, Ls=16)
    op = orc.Op.dwf(16, 1.8, 0.01)
    orc.normal(op, U16, psi5)
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        orc.normal(op, U16, psi5)
    res["dwf_mdag_m_16^4x16_seconds"] = round((time.perf_counter() - t0) / reps, 4)
    if os.path.exists(ORACLE_CG_FILE):
        rec = {}
        for line in open(ORACLE_CG_FILE):
            if line.startswith("{"):
                rec = json.loads(line)
        if rec:
            res["oracle_cg_16^4x16"] = dict(rec, source=os.path.relpath(ORACLE_CG_FILE, ROOT))
    return res


def oracle_cg_leg():
    """The FP64 oracle CG (Hestenes-Stiefel on M^dagger M, stopping on the true residual) on the
    16^4 x 16 domain-wall workload of the CG legs, timed to a true residual of 1e-10 on the host
    cores (minutes), and each GPU solution's distance to the oracle's solution."""
    import numpy as np
    from oracle import oracle as orc
    from paper_1512_03487_amd import fields
    _, sols = cg_legs(keep_solutions=True)
    dims, Ls = (16, 16, 16, 16), 16
    U = fields.gauge_field(dims, seed=1, kind="haar")
    b = fields.spinor_field(dims, seed=3, Ls=Ls)
    op = orc.Op.dwf(Ls, 1.8, 0.01)
    progress("oracle CG on 16^4 x 16 (minutes; the oracle reports every 25 iterations)")
    os.environ["ORACLE_CG_PROGRESS"] = "25"
    t0 = time.perf_counter()
    x, status, its, relres = orc.cg(op, U, b, tol=1e-10)
    el = time.perf_counter() - t0
    xn = float(np.linalg.norm(x))
    out = {"seconds": round(el, 2), "iterations": its, "status": status, "true_residual": relres,
           "cores": orc.threads(), "cpu_model": _cpu_model(), "lattice": list(dims), "Ls": Ls, "M5": 1.8,
           "mf": 0.01, "tol": 1e-10}
    for name, xs in sols.items():
        out[f"gpu_{name}_rel_error_vs_oracle"] = float(np.linalg.norm(xs - x) / xn)
        out[f"gpu_{name}_true_residual_by_oracle"] = orc.true_residual(op, U, b, xs)
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_single_thread(seconds_target=3.0):
    """The oracle's H on 16^4 with one OpenMP thread, in a CPU-only child process (the thread count
    is fixed when the oracle library loads). The inputs are plain random arrays: the time of H does
    not depend on the values."""
    code = (
        "import sys, time, numpy as np\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "from oracle import oracle as orc\n"
        "r = np.random.default_rng(7)\n"
        "d = (16, 16, 16, 16)\n"
        "U = r.standard_normal(d + (4, 3, 3)) + 1j * r.standard_normal(d + (4, 3, 3))\n"
        "psi = r.standard_normal(d + (4, 3)) + 1j * r.standard_normal(d + (4, 3))\n"
        "orc.hop(U, psi)\n"
        "n, t0 = 0, time.perf_counter()\n"
        "while True:\n"
        "    orc.hop(U, psi); n += 1; el = time.perf_counter() - t0\n"
        f"    if el >= {seconds_target}: break\n"
        "print(orc.threads(), n, el)\n")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120,
                             check=True).stdout.split()
        th, n, el = int(out[-3]), int(out[-2]), float(out[-1])
    except (subprocess.SubprocessError, ValueError, IndexError) as e:
        return {"error": str(e)[:200]}
    return {"value": round(FLOPS_HOP * 16 ** 4 * n / el / 1e9, 3), "unit": "GFLOP/s", "cores": th,
            "sample": f"{n} applications of H on 16^4 ({el:.1f} s)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-legs", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy three times (counter calibration)")
    ap.add_argument("--only-solvers", action="store_true",
                    help="profiling aid: run only the CG and even-odd solver legs and print them")
    ap.add_argument("--only-mg", action="store_true", help="profiling aid: run only the multigrid legs")
    ap.add_argument("--only-cg-iterations", action="store_true",
                    help="profiling aid: run only the recorded-graph CG iteration legs and print them")
    ap.add_argument("--only-dwf", action="store_true",
                    help="profiling aid: run only the 24^4 x 12 domain-wall operator legs and print them")
    ap.add_argument("--oracle-cg", action="store_true",
                    help="run the FP64 oracle CG on 16^4 x 16 to 1e-10 (minutes) and print its record")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (multi-GPU sharding is not built)",
              file=sys.stderr)
        sys.exit(2)
    if args.only_solvers:
        print(json.dumps({"cg_dwf_16^4x16": cg_legs(), "solve_dwf_16^4x16_even_odd": eo_legs(),
                          "solve_mobius_16^4x16_even_odd": eo_legs("mobius")}), flush=True)
        return
    if args.only_mg:
        print(json.dumps({"multigrid": mg_legs()}), flush=True)
        return
    if args.only_cg_iterations:
        print(json.dumps({"cg_iterations_graph": cg_iteration_legs()}), flush=True)
        return
    if args.only_dwf:
        print(json.dumps(dwf_config5(args.calibrate_copy)), flush=True)
        return
    if args.oracle_cg:
        print(json.dumps(oracle_cg_leg()), flush=True)
        return

    import torch
    dims = HEAD_DIMS
    vol = dims[0] * dims[1] * dims[2] * dims[3]
    bytes_launch = alg_bytes_per_site("f32", "L18", 1) * vol
    # The headline's fields are drawn on the host first and the operator legs run next, so the
    # headline's warmup and timed steps follow GPU work without an idle gap (after one, the first
    # hundred or so applications run up to 10 % slower while the clocks come back up).
    # 2 x 403 MB of inputs (FP32 links + psi) = 806 MB, three times the 256 MB MALL, so every
    # application streams its inputs from HBM
    nsets = 2
    sets, (U_host, psi_host) = make_sets(dims, "f32", nsets, kind="haar")
    dwf5 = None
    legs = {}
    if not args.no_legs:
        progress("domain-wall operator 24^4 x 12")
        dwf5 = dwf_config5(False)
        progress("operator legs")
        legs["hop_32^4_f32_L12"] = leg((32, 32, 32, 32), "f32", "L12", "hop", None, 50, 5)
        legs["hop_32^4_f16s_L12"] = leg((32, 32, 32, 32), "f16s", "L12", "hop", None, 50, 5)
        s16, _ = make_sets((16, 16, 16, 16), "f64", 12)
        t16, _ = time_dhop(s16, 100, 10, settle_s=SETTLE_S)
        del s16
        b16 = alg_bytes_per_site("f64", "L18", 1) * 16 ** 4
        legs["hop_16^4_f64"] = {"us_per_launch": round(t16 * 1e6, 2), "gflops": round(FLOPS_HOP * 16 ** 4 / t16 / 1e9, 1),
                                "alg_gbs": round(b16 / t16 / 1e9, 1),
                                "roofline_frac": round(b16 / t16 / 1e9 / HBM_PEAK_GBS, 4), "buffer_sets": 12,
                                "links": "weak field"}
        legs["hop_16^4_f32"] = leg((16, 16, 16, 16), "f32", "L18", "hop", None, 100, 10)
        legs["copy_same_bytes_as_hop_32^4_f32"] = copy_reference(bytes_launch, nsets=2, steps=50, warmup=5)
        legs["link_force_32^4_f32"] = link_force_leg()
        legs["dwf_eo_hop_16^4x16_f32"] = cb_leg((16, 16, 16, 16), 16, "f32", "L18")
        legs["dwf_eo_hop_16^4x16_f16s_L12"] = cb_leg((16, 16, 16, 16), 16, "f16s", "L12")
        legs["mobius_16^4x16_f32"] = mobius_leg((16, 16, 16, 16), 16, "f32", 50, 5)
        legs["mobius_16^4x16_f16s_L12"] = mobius_leg((16, 16, 16, 16), 16, "f16s", 50, 5, fmt="L12")
        legs["mobius_16^4x16_f64"] = mobius_leg((16, 16, 16, 16), 16, "f64", 20, 3)
        torch.cuda.empty_cache()
    progress("headline: H on 32^4 FP32")
    t, wall = time_dhop(sets, args.steps, args.warmup)
    del sets
    if args.calibrate_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    torch.cuda.empty_cache()
    achieved = bytes_launch / t / 1e9
    gflops = FLOPS_HOP * vol / t / 1e9
    cg = eo = eo_mob = cgi = mgl = None
    if not args.no_cg:
        progress("CG on 16^4 x 16")
        cg = cg_legs()
        progress("even-odd solves")
        eo = eo_legs()
        progress("even-odd Moebius solves")
        eo_mob = eo_legs("mobius")
        progress("recorded CG iterations")
        cgi = cg_iteration_legs()
        progress("multigrid")
        mgl = mg_legs()
    md = None
    if not args.no_legs:
        progress("HMC kernels")
        md = hmc_legs()
    cpu = None
    if not args.no_cpu:
        progress("oracle on the host cores")
        cpu = cpu_baseline(U_host, psi_host)
    del U_host, psi_host

    traffic = measured_traffic("hop_32^4_f32")
    rec = {
        "metric": METRIC,
        "value": round(gflops, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "Wilson hopping operator H, 32^4 periodic lattice, FP32 spinors and 18-real FP32 "
                               "links, Haar-random SU(3) links, Gaussian spinor, repeated applications",
                   "lattice": list(dims), "links": "L18", "buffer_sets": nsets, "flop_per_site": FLOPS_HOP},
        "hbm_gbs_algorithmic": round(achieved, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "alg_bytes_per_launch": int(bytes_launch),
                     "hbm_bytes_per_launch": traffic, "kernel": HEAD_KERNEL},
        "cpu_baseline": cpu,
        "dwf_24^4x12": dwf5,
        "legs": legs,
        "cg_dwf_16^4x16": cg,
        "solve_dwf_16^4x16_even_odd": eo,
        "solve_mobius_16^4x16_even_odd": eo_mob,
        "cg_iterations_graph": cgi,
        "multigrid": mgl,
        "hmc_16^4": md,
        "wall_s_timed": round(wall, 4),
    }
    print(json.dumps(rec), flush=True)


def dwf_config5(calibrate_copy=False):
    """The domain-wall operator M on 24^4 x 12 (M5 = 1.8, mf = 0.01, Haar links, Gaussian spinor),
    the throughput size of the domain-wall workload, in FP32 (18-real links) and FP16 storage
    (12-real FP16 links): time per application over buffer sets rotating through > 600 MB of
    inputs, GFLOP/s at 1320 per 5D site, and the HBM roofline record of its kernel (algorithmic
    bytes: psi and out once per 5D site, the links once per 4D site)."""
    import torch
    out = {"workload": "domain-wall operator M, 24^4 x Ls = 12, M5 = 1.8, mf = 0.01, Haar links, Gaussian spinor"}
    for name, prec, fmt, kern in (("f32", "f32", "L18", "k_dhop_walk2<SpF32, LkF32<3>, false, GRID_DWF, 0>"),
                                  ("f16s_L12", "f16s", "L12", "k_dhop_walk2<SpF16S, LkF16<2>, false, GRID_DWF, 0>"),
                                  ("f16s_L18", "f16s", "L18", "k_dhop_walk2<SpF16S, LkF16<3>, false, GRID_DWF, 0>"),
                                  ("f32_L12", "f32", "L12", "k_dhop_walk2<SpF32, LkF32<2>, false, GRID_DWF, 0>")):
        r = leg((24, 24, 24, 24), prec, fmt, "dwf", 12, 20, 3)
        key = f"dwf_24^4x12_{name}"
        traffic = measured_traffic(key) if key in TRAFFIC_FILES else None
        r["roofline"] = {"bound": "hbm", "achieved": r["alg_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": r["roofline_frac"], "traffic": traffic,
                         "alg_bytes_per_launch": int(alg_bytes_per_site(prec, fmt, 12) * 24 ** 4 * 12),
                         "kernel": kern}
        out[name] = r
        torch.cuda.empty_cache()
    if calibrate_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
    return out


if __name__ == "__main__":
    main()
