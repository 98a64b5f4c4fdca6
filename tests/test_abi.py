"""CPU checks of the boundary: the built HIP library loads and exports every
function declared in include/pcr.h; the binding's structs have the header's
layout; the oracle and the product share no code and neither imports the
other."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pcr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pcr_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ["pcr_dvf_compose", "pcr_warp_volume", "pcr_forward_project",
                     "pcr_backproject_residual", "pcr_cost_grad",
                     "pcr_reconstruct_from_projection", "pcr_localize_tumor"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1004_0014_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libpcr.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert lib.pcr_version  # callable without a device
    lib.pcr_version.restype = ctypes.c_char_p
    assert lib.pcr_version().startswith(b"pcr ")


def test_opts_default_without_device():
    from paper_1004_0014_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libpcr.so not built")
    o = _lib.default_opts()
    assert o.max_iter == 50 and o.max_backtracks == 30 and o.sigma == 1e-4 and o.beta == 0.5
    assert o.step_rule == _lib.PCR_STEP_SECANT


def _imports(path):
    out = []
    for dirpath, _, files in os.walk(path):
        for f in files:
            if f.endswith((".py", ".c", ".h", ".hip", ".cpp")):
                out.append((os.path.join(dirpath, f), open(os.path.join(dirpath, f)).read()))
    return out


def test_oracle_and_product_are_independent():
    for p, txt in _imports(os.path.join(ROOT, "oracle")):
        assert "paper_1004_0014_amd" not in txt and "pcr.h" not in txt, p
    for p, txt in _imports(os.path.join(ROOT, "paper_1004_0014_amd")):
        assert not re.search(r"^\s*(import|from)\s+oracle\b", txt, re.M), p
        assert "oracle.h" not in txt, p


def test_predict_w_is_polynomial_extrapolation():
    """pcr_predict_w (host-only): exact on sequences of the polynomial degree
    it uses; order 0 is the plain warm start."""
    import numpy as np
    from paper_1004_0014_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libpcr.so not built")
    t = np.array([0.0, 0.09, 0.2, 0.27])
    a, b, c = np.array([1.0, -2.0, 0.5]), np.array([3.0, 0.25, -1.0]), np.array([-0.7, 2.0, 4.0])
    lin = np.stack([a + b * ti for ti in t])
    quad = np.stack([a + b * ti + c * ti * ti for ti in t])
    tn = 0.36
    np.testing.assert_allclose(_lib.predict_w(lin, t, tn, 1), a + b * tn, rtol=1e-12)
    np.testing.assert_allclose(_lib.predict_w(quad, t, tn, 2), a + b * tn + c * tn * tn, rtol=1e-12)
    np.testing.assert_array_equal(_lib.predict_w(quad, t, tn, 0), quad[-1])
    np.testing.assert_array_equal(_lib.predict_w(quad[:1], t[:1], tn, 2), quad[0])
    with pytest.raises(_lib.PCRError):
        _lib.predict_w(quad, t[::-1], tn, 1)          # times must increase


# ctypes mirror of each boundary struct, by its C name
_STRUCTS = {"pcr_grid": "Grid", "pcr_geom": "Geom", "pcr_model": "Model",
            "pcr_solve_opts": "SolveOpts", "pcr_solve_stats": "SolveStats",
            "pcr_server_opts": "ServerOpts", "pcr_result": "Result"}


def test_binding_structs_match_the_header(tmp_path):
    """Every struct the binding passes across the boundary has the size and
    the field offsets the C compiler gives the header's declaration."""
    import shutil
    import subprocess
    from paper_1004_0014_amd import _lib
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "pcr.h"', "int main(void) {"]
    for cname, pyname in _STRUCTS.items():
        cls = getattr(_lib, pyname)
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f[0], cname, f[0]))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    cc = subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                        capture_output=True, text=True)
    assert cc.returncode == 0, cc.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, v = line.split()
            got[(a, b)] = int(v)
    for cname, pyname in _STRUCTS.items():
        cls = getattr(_lib, pyname)
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f in cls._fields_:
            assert got[(cname, f[0])] == getattr(cls, f[0]).offset, (cname, f[0])


def _fake_grid(n, spacing=1.0):
    from paper_1004_0014_amd import _lib
    g = _lib.Grid()
    g.n[:] = list(n)
    g.spacing_mm[:] = [spacing] * 3
    g.origin_mm[:] = [0.0, 0.0, 0.0]
    return g


def _fake_geom():
    from paper_1004_0014_amd import _lib
    G = _lib.Geom()
    G.angle_rad, G.sad_mm, G.sdd_mm = 0.3, 1000.0, 1500.0
    G.nu, G.nv, G.du_mm, G.dv_mm = 64, 48, 1.0, 1.0
    G.step_mm = 1.0
    return G


def test_march_addressing_limit_is_rejected_before_any_launch():
    """The FP32 march forms 32-bit byte offsets (image < 2 GiB).  An image
    beyond that is refused with PCR_EINVAL by validation, before the library
    touches a device: the device pointers passed here are never dereferenced
    (this runs without a GPU)."""
    import ctypes as C
    from paper_1004_0014_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libpcr.so not built")
    L = _lib.lib()
    fake = C.c_void_p(0x10000)
    # single channel: (1024+3)^2 (600+3) cells x 4 B = 2.54 GB
    g = _fake_grid((1024, 1024, 600))
    G = _fake_geom()
    st = L.pcr_forward_project(C.byref(g), C.byref(G), _lib.PCR_F32, fake, fake, None)
    assert st == _lib.PCR_EINVAL
    assert b"addressing" in L.pcr_last_error()
    # K = 4 fused image (6 FP32 channels, 24 B cells): 515 x 515 x 343 x 24 B = 2.18 GB
    m = _lib.Model(4, _lib.PCR_F32, fake.value, fake.value, None)
    h = C.c_void_p()
    g2 = _fake_grid((512, 512, 340))
    st = L.pcr_ctx_create(C.byref(g2), C.byref(m), _lib.PCR_F32, fake, _lib.PCR_F32, C.byref(h))
    assert st == _lib.PCR_EINVAL and not h.value
    assert b"addressing" in L.pcr_last_error()
    # the same grid in FP64 compute has 64-bit offsets: not refused for addressing
    # (what happens next needs a device)
    st = L.pcr_ctx_create(C.byref(g2), C.byref(m), _lib.PCR_F32, fake, _lib.PCR_F64, C.byref(h))
    assert not (st == _lib.PCR_EINVAL and b"addressing" in L.pcr_last_error())
    if h.value:
        L.pcr_ctx_destroy(h)


def test_noalloc_projection_refuses_oversized_grid_before_any_launch():
    """pcr_forward_project_noalloc keeps its padded copy in a fixed array of
    PCR_NOALLOC_SCRATCH_BYTES: a grid whose padded copy is larger returns
    PCR_EINVAL from validation, before the library touches a device (the
    pointers passed here are never dereferenced; this runs without a GPU)."""
    import ctypes as C
    from paper_1004_0014_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libpcr.so not built")
    L = _lib.lib()
    fake = C.c_void_p(0x10000)
    G = _fake_geom()
    # (400+3)^3 cells x 4 B = 262 MB > 64 MiB
    g = _fake_grid((400, 400, 400))
    st = L.pcr_forward_project_noalloc(C.byref(g), C.byref(G), _lib.PCR_F32, fake, fake, None)
    assert st == _lib.PCR_EINVAL and b"fixed scratch" in L.pcr_last_error()
    # FP64 doubles the cells' size: (256+3)^2 (100+3) x 8 B = 55 MB fits, (256+3)^2 (128+3) x 8 B does not
    g = _fake_grid((256, 256, 128))
    st = L.pcr_forward_project_noalloc(C.byref(g), C.byref(G), _lib.PCR_F64, fake, fake, None)
    assert st == _lib.PCR_EINVAL and b"fixed scratch" in L.pcr_last_error()


def test_march_step_limit_is_rejected_before_any_launch():
    """The FP32 march counts a ray's samples with an FP32 index, exact below
    2^24: a step so small that a ray through the grid would take 2^24
    samples or more is refused with PCR_EINVAL by validation, before the
    library touches a device (this runs without a GPU)."""
    import ctypes as C
    from paper_1004_0014_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libpcr.so not built")
    L = _lib.lib()
    fake = C.c_void_p(0x10000)
    g = _fake_grid((64, 64, 32))
    G = _fake_geom()
    G.step_mm = 1e-6      # a ~90 mm diagonal in 9e7 samples
    for fn in (L.pcr_forward_project, L.pcr_forward_project_noalloc):
        st = fn(C.byref(g), C.byref(G), _lib.PCR_F32, fake, fake, None)
        assert st == _lib.PCR_EINVAL
        assert b"too small for the FP32 march" in L.pcr_last_error()
