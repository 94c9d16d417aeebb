"""The C ABI library loads, exports every declared symbol, and validates arguments on the host.

These run without a GPU: every call below is rejected by host-side validation before any HIP
call, so the (fake, never dereferenced) device addresses are never touched.
"""
import ctypes
import os
import re

import pytest

from paper_1512_03487_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
A = 0x7f0000000000          # a 256-byte aligned fake address
P = ctypes.c_void_p


def declared_functions():
    text = open(os.path.join(ROOT, "include", "grid_mi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(grid_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def geom(dims=(4, 4, 4, 4), Ls=1):
    g = _lib.GridGeom()
    g.dims[:] = list(dims)
    g.Ls = Ls
    return g


def op(kind=_lib.GRID_HOP, dag=0, mass=0.1, M5=1.8, mf=0.01, b5=1.0, c5=0.0):
    return _lib.GridOp(kind, dag, mass, M5, mf, b5, c5)


def dhop(lib, U=A, psi=A + 0x10000000, ps=None, out=A + 0x20000000, os_=None, g=None, o=None, prec=0, fmt=0):
    g = g or geom()
    o = o or op()
    return lib.grid_dhop(P(U), P(psi), P(ps), P(out), P(os_), ctypes.byref(g), ctypes.byref(o), prec, fmt, None)


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert set(names) == set(_lib.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n
    assert lib.grid_version() == 100


def test_geometry_validation(lib):
    assert lib.grid_dhop(P(A), P(A), None, P(A), None, None, ctypes.byref(op()), 0, 0, None) == _lib.GRID_EINVAL
    assert dhop(lib, g=geom((4, 4, 1, 4))) == _lib.GRID_ESHAPE
    assert "dims[2]" in _lib.last_error()
    assert dhop(lib, g=geom((4, 4, 4, 4), Ls=0)) == _lib.GRID_ESHAPE
    assert dhop(lib, g=geom((1024, 1024, 1024, 2))) == _lib.GRID_ESHAPE
    assert dhop(lib, g=geom((64, 64, 64, 64), Ls=32)) == _lib.GRID_ESHAPE


def test_enum_and_pointer_validation(lib):
    assert dhop(lib, prec=7) == _lib.GRID_EDTYPE
    assert dhop(lib, fmt=5) == _lib.GRID_EDTYPE
    assert dhop(lib, o=op(kind=9)) == _lib.GRID_EINVAL
    assert dhop(lib, o=op(kind=_lib.GRID_WILSON), g=geom(Ls=4)) == _lib.GRID_ESHAPE
    assert dhop(lib, U=0) == _lib.GRID_EINVAL
    assert dhop(lib, psi=A + 8) == _lib.GRID_EALIGN
    assert dhop(lib, prec=_lib.GRID_F16S) == _lib.GRID_EINVAL            # missing scales
    assert dhop(lib, ps=A + 0x30000000) == _lib.GRID_EINVAL               # scale with FP64
    assert dhop(lib, out=A + 0x10000000 + 16) == _lib.GRID_EINVAL         # out overlaps psi
    assert "overlap" in _lib.last_error()


def test_backward_and_convert_validation(lib):
    g, o = geom(), op()
    assert lib.grid_dhop_backward(P(A), P(A + 0x1000000), P(A + 0x2000000), None, None, ctypes.byref(g),
                                  ctypes.byref(o), 0, 0, None) == _lib.GRID_EINVAL
    assert lib.grid_dhop_backward(P(A), P(A + 0x1000000), P(A + 0x2000000), P(A + 0x3000000), None, ctypes.byref(g),
                                  ctypes.byref(o), _lib.GRID_F16S, 0, None) == _lib.GRID_EDTYPE
    assert lib.grid_dhop_backward(P(A), P(A + 0x1000000), P(A + 0x2000000), P(A + 0x3000000), None, ctypes.byref(g),
                                  ctypes.byref(o), 0, 2, None) == _lib.GRID_EINVAL
    assert lib.grid_convert_spinor(P(A), 0, None, P(A + 0x1000000), 1, None, -1, None) == _lib.GRID_ESHAPE
    assert lib.grid_convert_spinor(P(A), 0, None, P(A + 0x1000000), 2, None, 16, None) == _lib.GRID_EINVAL
    assert lib.grid_convert_links(P(A), P(A + 16), 1, 0, 0, 16, None) == _lib.GRID_EINVAL   # overlap
    assert lib.grid_convert_links(P(A), P(A + 0x1000000), 3, 0, 0, 16, None) == _lib.GRID_EDTYPE


def test_cg_workspace_and_validation(lib):
    g = geom((4, 4, 4, 4), Ls=8)
    n = 4 ** 4 * 8
    p64 = _lib.GridCgParams(1e-10, 100, _lib.GRID_F64, _lib.GRID_L18, 0.1, 10)
    p16 = _lib.GridCgParams(1e-10, 100, _lib.GRID_F16S, _lib.GRID_L12, 0.1, 10)
    w64 = lib.grid_cg_workspace_bytes(ctypes.byref(g), ctypes.byref(p64))
    w16 = lib.grid_cg_workspace_bytes(ctypes.byref(g), ctypes.byref(p16))
    assert w64 >= 4 * n * 192 and w16 >= 3 * n * 192 + n * 96 + 4 * n * 52
    bad = _lib.GridCgParams(1e-10, 100, 9, 0, 0.1, 10)
    assert lib.grid_cg_workspace_bytes(ctypes.byref(g), ctypes.byref(bad)) == 0
    st = _lib.GridCgStats()
    o = op(kind=_lib.GRID_DWF)
    args = lambda ws, nbytes, p=p64, oo=o: (P(A), P(A + 0x1000000), P(A + 0x2000000), ctypes.byref(g), ctypes.byref(oo),
                                            ctypes.byref(p), P(ws), ctypes.c_size_t(nbytes), ctypes.byref(st), None)
    assert lib.grid_cg(*args(A + 0x4000000, w64 - 1)) == _lib.GRID_ESPACE
    assert lib.grid_cg(*args(A + 0x4000000 + 128, w64)) == _lib.GRID_EALIGN
    assert lib.grid_cg(*args(A + 0x1000000, w64)) == _lib.GRID_EINVAL                 # overlaps b
    assert lib.grid_cg(*args(A + 0x4000000, w64, oo=op(kind=_lib.GRID_HOP))) == _lib.GRID_EINVAL
    nodelta = _lib.GridCgParams(1e-10, 100, _lib.GRID_F32, _lib.GRID_L18, 1.5, 10)
    assert lib.grid_cg(*args(A + 0x4000000, w64 * 4, p=nodelta)) == _lib.GRID_EINVAL
    assert _lib.last_error()


def test_even_odd_validation(lib):
    g, go = geom((4, 4, 4, 4), Ls=4), geom((4, 3, 4, 4), Ls=4)
    o_hop, o_dwf = op(), op(kind=_lib.GRID_DWF)
    cb = lambda gg=g, oo=o_hop, y=None, par=0, prec=0, ps=None, os_=None: lib.grid_dhop_cb(
        P(A), P(A + 0x1000000), P(ps), P(y), None, P(A + 0x2000000), P(os_), ctypes.byref(gg), ctypes.byref(oo), par,
        ctypes.c_double(0.5), prec, 0, None)
    assert cb(gg=go) == _lib.GRID_ESHAPE and "even" in _lib.last_error()
    assert cb(par=2) == _lib.GRID_EINVAL
    assert cb(y=A + 0x3000000) == _lib.GRID_EINVAL                           # y with GRID_HOP
    assert cb(oo=o_dwf) == _lib.GRID_EINVAL                                  # y missing
    assert cb(oo=op(kind=_lib.GRID_WILSON), y=A + 0x3000000) == _lib.GRID_ESHAPE   # Wilson needs Ls 1
    assert cb(prec=_lib.GRID_F16S) == _lib.GRID_EINVAL                       # scales missing
    m5 = lambda Ls=8, M5=1.8, n4=16: lib.grid_m5inv(P(A), None, P(A + 0x1000000), None, n4, Ls, ctypes.c_double(M5),
                                                    ctypes.c_double(0.01), 0, 0, None)
    assert m5(Ls=65) == _lib.GRID_ESHAPE and m5(Ls=0) == _lib.GRID_ESHAPE
    assert m5(M5=4.5) == _lib.GRID_EINVAL                                    # |5 - M5| <= 1
    assert m5(n4=-1) == _lib.GRID_ESHAPE
    assert lib.grid_m5inv(P(A), None, P(A + 16), None, 16, 8, ctypes.c_double(1.8), ctypes.c_double(0.01), 0, 0,
                          None) == _lib.GRID_EINVAL                          # overlap


def test_solve_eo_workspace_and_validation(lib):
    g = geom((4, 4, 4, 4), Ls=8)
    n = 4 ** 4 * 8
    p64 = _lib.GridCgParams(1e-10, 100, _lib.GRID_F64, _lib.GRID_L18, 0.1, 10)
    w = lib.grid_solve_eo_workspace_bytes(ctypes.byref(g), ctypes.byref(p64))
    # eight checkerboard FP64 fields of its own plus the CG's four on the even checkerboard
    assert w >= 8 * (n // 2) * 192 + 4 * (n // 2) * 192
    assert lib.grid_solve_eo_workspace_bytes(ctypes.byref(geom((4, 4, 4, 5), Ls=8)), ctypes.byref(p64)) == 0
    st = _lib.GridCgStats()
    args = lambda gg=g, oo=op(kind=_lib.GRID_DWF), ws=A + 0x40000000, nbytes=w: (
        P(A), P(A + 0x10000000), P(A + 0x20000000), ctypes.byref(gg), ctypes.byref(oo), ctypes.byref(p64), P(ws),
        ctypes.c_size_t(nbytes), ctypes.byref(st), None)
    assert lib.grid_solve_eo(*args(gg=geom((4, 4, 6, 5), Ls=8))) == _lib.GRID_ESHAPE
    assert lib.grid_solve_eo(*args(gg=geom((4, 4, 4, 4), Ls=65))) == _lib.GRID_ESHAPE
    assert lib.grid_solve_eo(*args(oo=op(kind=_lib.GRID_DWF, M5=4.5))) == _lib.GRID_EINVAL
    assert lib.grid_solve_eo(*args(oo=op(kind=_lib.GRID_HOP))) == _lib.GRID_EINVAL
    assert lib.grid_solve_eo(*args(nbytes=w - 1)) == _lib.GRID_ESPACE
    assert lib.grid_solve_eo(*args(ws=A + 0x40000000 + 64)) == _lib.GRID_EALIGN


def test_mobius_validation(lib):
    g = geom((4, 4, 4, 4), Ls=8)
    mob = op(kind=_lib.GRID_MOBIUS, b5=1.5, c5=0.5)
    call = lambda oo=mob, tmp=A + 0x30000000, prec=0, ts=None: lib.grid_mobius(
        P(A), P(A + 0x10000000), None, P(A + 0x20000000), None, P(tmp), P(ts), ctypes.byref(g), ctypes.byref(oo), prec,
        0, None)
    assert call(oo=op(kind=_lib.GRID_DWF)) == _lib.GRID_EINVAL
    assert call(tmp=0) == _lib.GRID_EINVAL
    assert call(tmp=A + 0x10000000 + 64) == _lib.GRID_EINVAL                # tmp overlaps psi
    assert call(prec=_lib.GRID_F16S) == _lib.GRID_EINVAL                     # scales missing
    assert dhop(lib, o=mob, g=g) == _lib.GRID_EINVAL and "grid_mobius" in _lib.last_error()
    # the even-odd solver takes the Moebius kind when M_ee = alpha - beta S has a stable inverse:
    # alpha = 1 + (4 - M5) b5, beta = 1 - (4 - M5) c5 with |alpha / beta| > 1, or beta = 0 != alpha
    p64 = _lib.GridCgParams(1e-10, 100, _lib.GRID_F64, _lib.GRID_L18, 0.1, 10)
    st = _lib.GridCgStats()
    w = lib.grid_solve_eo_workspace_bytes(ctypes.byref(g), ctypes.byref(p64))
    eo = lambda oo, gg=g: lib.grid_solve_eo(P(A), P(A + 0x10000000), P(A + 0x20000000), ctypes.byref(gg),
                                            ctypes.byref(oo), ctypes.byref(p64), P(A + 0x40000000), ctypes.c_size_t(w),
                                            ctypes.byref(st), None)
    assert eo(op(kind=_lib.GRID_MOBIUS, b5=0.0, c5=0.0)) == _lib.GRID_EINVAL            # alpha = beta = 1
    assert "alpha" in _lib.last_error()
    assert eo(op(kind=_lib.GRID_MOBIUS, M5=2.0, b5=-0.5, c5=0.5)) == _lib.GRID_EINVAL    # beta = 0 = alpha
    assert eo(op(kind=_lib.GRID_MOBIUS, b5=1.5, c5=0.5), gg=geom((4, 4, 4, 4), Ls=65)) == _lib.GRID_ESHAPE


def test_md_validation(lib):
    g = geom((4, 4, 4, 4), Ls=4)
    cg = _lib.GridCgParams(1e-10, 100, _lib.GRID_F64, _lib.GRID_L18, 0.1, 10)
    p = _lib.GridMdParams(5.5, 0.05, 4, op(kind=_lib.GRID_DWF), cg)
    w = lib.grid_md_workspace_bytes(ctypes.byref(g), ctypes.byref(p))
    assert w >= 2 * 4 ** 4 * 4 * 144 + 2 * 4 ** 4 * 4 * 192
    st = _lib.GridMdStats()
    call = lambda pp=p, phi=A + 0x20000000, ws=A + 0x40000000, nb=w: lib.grid_md_leapfrog(
        P(A), P(A + 0x10000000), P(phi), ctypes.byref(g), ctypes.byref(pp), P(ws), ctypes.c_size_t(nb),
        ctypes.byref(st), None)
    assert call(nb=w - 1) == _lib.GRID_ESPACE
    assert call(ws=A + 0x40000000 + 32) == _lib.GRID_EALIGN
    assert call(pp=_lib.GridMdParams(5.5, 0.05, 4, op(kind=_lib.GRID_HOP), cg)) == _lib.GRID_EINVAL
    # the Moebius force needs one more 5D field (B X)
    pm = _lib.GridMdParams(5.5, 0.05, 4, op(kind=_lib.GRID_MOBIUS, b5=1.5, c5=0.5), cg)
    wm = lib.grid_md_workspace_bytes(ctypes.byref(g), ctypes.byref(pm))
    assert wm >= w + 4 ** 4 * 4 * 192
    assert call(pp=pm) == _lib.GRID_ESPACE
    assert call(pp=_lib.GridMdParams(5.5, 0.05, -1, op(kind=_lib.GRID_DWF), cg)) == _lib.GRID_EINVAL
    bad_int = _lib.GridMdParams(5.5, 0.05, 4, op(kind=_lib.GRID_DWF), cg, 3, 2)
    assert call(pp=bad_int) == _lib.GRID_EINVAL and "integrator" in _lib.last_error()
    neg_inner = _lib.GridMdParams(5.5, 0.05, 4, op(kind=_lib.GRID_DWF), cg, _lib.GRID_FORCE_GRADIENT, -1)
    assert call(pp=neg_inner) == _lib.GRID_EINVAL
    assert call(pp=_lib.GridMdParams(float("nan"), 0.05, 4, op(kind=_lib.GRID_DWF), cg)) == _lib.GRID_EINVAL
    assert call(phi=A + 0x10000000 + 64) == _lib.GRID_EINVAL                  # phi overlaps P
    assert lib.grid_link_exp(P(A), P(A + 16), ctypes.c_double(0.1), 16, None) == _lib.GRID_EINVAL
    assert lib.grid_gauge_force(P(A), P(A + 16), ctypes.byref(geom()), ctypes.c_double(5.5), None) == _lib.GRID_EINVAL


def test_ctypes_structs_match_the_c_header(tmp_path):
    """Every struct of include/grid_mi.h has the size and field offsets of its ctypes mirror, as a
    C compiler lays it out (gcc on the header itself)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    mirrors = {"grid_geom": _lib.GridGeom, "grid_op": _lib.GridOp, "grid_cg_params": _lib.GridCgParams,
               "grid_cg_stats": _lib.GridCgStats, "grid_md_params": _lib.GridMdParams,
               "grid_md_stats": _lib.GridMdStats, "grid_mg_params": _lib.GridMgParams}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "grid_mi.h"', 'int main(void) {']
    for cname, py in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict((" ".join(l.split()[:2]), int(l.split()[2]))
               for l in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines())
    for cname, py in mirrors.items():
        assert got[f"{cname} size"] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[f"{cname} {fname}"] == getattr(py, fname).offset, (cname, fname)


def mg_params(**kw):
    p = _lib.GridMgParams()
    for mu, b in enumerate(kw.get("block", (2, 2, 2, 2))):
        p.block[mu] = b
    p.nvec = kw.get("nvec", 4)
    p.setup_rounds, p.setup_iters = 1, 4
    p.coarse_iters, p.coarse_tol, p.smooth_iters = 10, 0.1, 1
    p.restart, p.maxiter, p.tol = kw.get("restart", 4), 10, 1e-8
    p.setup_prec = kw.get("setup_prec", _lib.GRID_F64)
    p.cycle_prec = kw.get("cycle_prec", _lib.GRID_F64)
    return p


def test_multigrid_validation(lib):
    g = geom()
    ok = mg_params()
    assert lib.grid_mg_workspace_bytes(ctypes.byref(g), ctypes.byref(ok)) > 0
    for bad in (mg_params(block=(3, 2, 2, 2)), mg_params(block=(0, 2, 2, 2)), mg_params(nvec=0), mg_params(nvec=33),
                mg_params(restart=0), mg_params(restart=65), mg_params(block=(1, 1, 1, 1), nvec=7),
                mg_params(setup_prec=3), mg_params(setup_prec=-1), mg_params(cycle_prec=_lib.GRID_F16S),
                mg_params(cycle_prec=7)):
        assert lib.grid_mg_workspace_bytes(ctypes.byref(g), ctypes.byref(bad)) == 0
    # a mixed-precision setup needs the sloppy vectors and links besides
    assert (lib.grid_mg_workspace_bytes(ctypes.byref(g), ctypes.byref(mg_params(setup_prec=_lib.GRID_F32)))
            >= lib.grid_mg_workspace_bytes(ctypes.byref(g), ctypes.byref(ok)))
    # an FP32 cycle also holds FP32 z, s, t, r, the links, the basis and the coarse operator (the
    # workspace is the larger of the solve's and the setup's; 16 restart vectors make it the solve's)
    vol, nvec, vc = 4**4, 4, 2**4
    fp32_cycle = 4 * vol * 96 + vol * 4 * 72 + nvec * vol * 96 + vc * 9 * (2 * nvec) ** 2 * 8
    w64 = lib.grid_mg_workspace_bytes(ctypes.byref(g), ctypes.byref(mg_params(restart=16)))
    w32 = lib.grid_mg_workspace_bytes(ctypes.byref(g), ctypes.byref(mg_params(restart=16, cycle_prec=_lib.GRID_F32)))
    assert w32 >= w64 + fp32_cycle
    op =_lib.GridOp(_lib.GRID_WILSON, 0, 0.1, 1.8, 0.01, 1.0, 0.0)
    dwf = _lib.GridOp(_lib.GRID_DWF, 0, 0.1, 1.8, 0.01, 1.0, 0.0)
    need = lib.grid_mg_workspace_bytes(ctypes.byref(g), ctypes.byref(ok))
    st = _lib.GridCgStats()
    assert lib.grid_mg_solve(P(A), P(A + 2**30), P(A + 2**31), P(A + 3 * 2**30), P(A + 2**32), ctypes.byref(g),
                             ctypes.byref(dwf), ctypes.byref(ok), P(A + 2**33), need, ctypes.byref(st), None) == _lib.GRID_EINVAL
    assert lib.grid_mg_solve(P(A), P(A + 2**30), P(A + 2**31), P(A + 3 * 2**30), P(A + 2**32), ctypes.byref(g),
                             ctypes.byref(op), ctypes.byref(ok), P(A + 2**33), need - 1, ctypes.byref(st), None) == _lib.GRID_EINVAL
    assert "workspace" in _lib.last_error()
    # the pCG entry shares the checks
    for kind, nb, code in ((dwf, need, _lib.GRID_EINVAL), (op, need - 1, _lib.GRID_EINVAL)):
        assert lib.grid_mg_pcg(P(A), P(A + 2**30), P(A + 2**31), P(A + 3 * 2**30), P(A + 2**32), ctypes.byref(g),
                               ctypes.byref(kind), ctypes.byref(ok), P(A + 2**33), nb, ctypes.byref(st), None) == code
    assert lib.grid_mg_pcg(P(A), P(A + 2**30), P(A + 2**31), P(A + 3 * 2**30), P(A + 3 * 2**30 + 64), ctypes.byref(g),
                           ctypes.byref(op), ctypes.byref(ok), P(A + 2**33), need, ctypes.byref(st), None) == _lib.GRID_EINVAL
    assert "x overlaps" in _lib.last_error()
    assert lib.grid_mg_basis(P(A), P(A + 2**30), ctypes.byref(geom(Ls=4)), ctypes.byref(op), ctypes.byref(ok),
                             P(A + 2**33), need, None) == _lib.GRID_ESHAPE
    cd = (ctypes.c_int * 4)(2, 2, 2, 2)
    assert lib.grid_coarse_stencil(P(A), P(A + 2**30), P(A + 2**31), cd, 65, 0, None) == _lib.GRID_EINVAL
    assert lib.grid_coarse_stencil(P(A), P(A + 2**30), P(A + 2**30), cd, 8, 0, None) == _lib.GRID_EINVAL
    cd0 = (ctypes.c_int * 4)(2, 0, 2, 2)
    assert lib.grid_coarse_stencil(P(A), P(A + 2**30), P(A + 2**31), cd0, 8, 0, None) == _lib.GRID_ESHAPE


def test_parameter_builders():
    """The Python parameter builders fill their ctypes structs without touching a GPU."""
    from paper_1512_03487_amd import api
    p = api.cg_params(tol=1e-9, sloppy="f16s", link_fmt="L12", graph=True)
    assert (p.sloppy_prec, p.link_fmt, p.graph) == (_lib.GRID_F16S, _lib.GRID_L12, 1)
    q = api.mg_params(block=(4, 4, 2, 2), nvec=8, setup_prec="f32")
    assert (tuple(q.block), q.nvec, q.setup_prec) == ((4, 4, 2, 2), 8, _lib.GRID_F32)
    assert api.mg_params().setup_prec == _lib.GRID_F64 and api.mg_params().cycle_prec == _lib.GRID_F64
    assert api.mg_params(cycle_prec="f32").cycle_prec == _lib.GRID_F32
    m = api.md_params(5.5, integrator="force_gradient", n_inner=1)
    assert m.integrator == _lib.GRID_FORCE_GRADIENT


def test_pseudofermion_action_validation(lib):
    g = geom((4, 4, 4, 4), Ls=4)
    n, nl = 4 ** 4 * 4, 4 ** 4 * 4
    p64 = _lib.GridCgParams(1e-10, 100, _lib.GRID_F64, _lib.GRID_L18, 0.1, 10)
    w = lib.grid_pseudofermion_workspace_bytes(ctypes.byref(g), ctypes.byref(p64))
    # the CG's workspace plus two FP64 fields (Op X, and the Moebius intermediate / B X)
    assert w >= lib.grid_cg_workspace_bytes(ctypes.byref(g), ctypes.byref(p64)) + 2 * n * 192
    assert lib.grid_pseudofermion_workspace_bytes(ctypes.byref(g), ctypes.byref(_lib.GridCgParams(1e-10, 100, 9, 0, 0.1,
                                                                                                  10))) == 0
    st = _lib.GridCgStats()
    S = ctypes.c_double()
    U, phi, X, dU, dphi, ws = A, A + 2**28, A + 2**29, A + 3 * 2**28, A + 2**30, A + 2**31

    def call(oo=op(kind=_lib.GRID_DWF), x=X, du=dU, dp=dphi, wsp=ws, nb=w, fm=0, scale=1.0, gg=g):
        return lib.grid_pseudofermion_action(P(U), P(phi), P(x), ctypes.byref(gg), ctypes.byref(oo),
                                             ctypes.byref(p64), ctypes.c_double(scale), ctypes.byref(S), P(du), fm,
                                             P(dp), P(wsp), ctypes.c_size_t(nb), ctypes.byref(st), None)
    assert call(oo=op(kind=_lib.GRID_HOP)) == _lib.GRID_EINVAL
    assert call(oo=op(kind=_lib.GRID_WILSON)) == _lib.GRID_ESHAPE            # Wilson needs Ls 1
    assert call(fm=2) == _lib.GRID_EINVAL
    assert call(scale=float("inf")) == _lib.GRID_EINVAL
    assert call(x=0) == _lib.GRID_EINVAL
    assert call(nb=w - 1) == _lib.GRID_ESPACE
    assert call(wsp=ws + 64) == _lib.GRID_EALIGN
    assert call(x=phi + 64) == _lib.GRID_EINVAL and "overlap" in _lib.last_error()   # X overlaps phi
    assert call(dp=X) == _lib.GRID_EINVAL                                    # dS/dphi overlaps X
    assert call(du=U + 16 * nl) == _lib.GRID_EINVAL                          # dS/dU overlaps U
    assert call(dp=dphi + 8) == _lib.GRID_EALIGN


def test_noalloc_normal_operator_validation(lib):
    """The allocation-free normal operator rejects fields whose M psi exceeds its static scratch,
    and bad arguments, on the host (nothing here reaches a HIP call)."""
    o, big = op(), geom((16, 16, 16, 16), Ls=8)         # 524288 sites: 96 MiB of M psi in FP64
    call = lambda g, prec=0, psi=A + 0x10000000, ps=None, out=A + 0x40000000, os_=None: lib.grid_dwf_mdag_m_noalloc(
        P(A), P(psi), P(ps), P(out), P(os_), ctypes.byref(g), ctypes.c_double(1.8), ctypes.c_double(0.01), prec, 0,
        None)
    assert call(big) == _lib.GRID_ESPACE and "scratch" in _lib.last_error()
    # FP16 storage at 16^4 x 16 fits (48 MiB of codes, 4 MiB of scales); 16^4 x 32 does not
    assert call(geom((16, 16, 16, 16), Ls=32), prec=_lib.GRID_F16S, ps=A + 0x80000000,
                os_=A + 0x90000000) == _lib.GRID_ESPACE
    assert call(geom((4, 4, 4, 4), Ls=4), out=A + 0x10000000 + 64) == _lib.GRID_EINVAL    # out overlaps psi
    assert call(geom((4, 4, 4, 4), Ls=4), prec=_lib.GRID_F16S) == _lib.GRID_EINVAL        # scales missing
    assert call(geom((4, 4, 4, 1), Ls=4)) == _lib.GRID_ESHAPE
