"""The allocation-free projection (pcr_forward_project_noalloc) against the
allocating one (pcr_forward_project), through the C ABI: the same kernels on
the same padded image, so the projections agree bit for bit.  Two calls in a
row, the second on a smaller grid (the fixed array keeps the first call's
contents, which the second must clear), in FP32 and FP64; a grid beyond the
array is refused before any launch."""
import ctypes as C
import math

import numpy as np
import pytest

from paper_1004_0014_amd import synth as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


def _case(n, spacing, nu, nv, pitch, angle_deg, dtype, seed):
    g = S.Grid(n, spacing)
    G = S.Geom(math.radians(angle_deg), nu, nv, pitch, pitch, 0.5 * min(spacing))
    vol = torch.tensor(S.phantom(g, seed=seed), dtype=dtype, device=DEV)
    return g, G, vol


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_projection_equals_allocating_projection(dtype):
    from paper_1004_0014_amd import _lib as L
    cases = [((96, 80, 56), (3.0, 3.0, 4.0), 160, 120, 2.0, 30.0, 1),
             ((40, 36, 28), (4.0, 4.0, 5.0), 72, 52, 3.0, 200.0, 2)]
    for n, sp, nu, nv, pitch, ang, seed in cases:
        g, G, vol = _case(n, sp, nu, nv, pitch, ang, dtype, seed)
        print("noalloc", dtype, n, (nu, nv), ang, flush=True)
        ref = L.forward_project(g, G, vol)
        out = torch.full((nv, nu), float("nan"), dtype=dtype, device=DEV)
        L.forward_project_noalloc(g, G, vol, out)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        assert np.isfinite(a).all()
        np.testing.assert_array_equal(a, b)
        assert np.abs(b).max() > 0


def test_noalloc_refuses_a_grid_beyond_the_array():
    from paper_1004_0014_amd import _lib as L
    lib = L.lib()
    g = L.make_grid(S.Grid((400, 400, 400), (1.0, 1.0, 1.0)))   # 403^3 x 4 B = 262 MB
    G = L.make_geom(S.Geom(0.3, 64, 48, 1.0, 1.0, 0.5))
    vol = torch.zeros(1, device=DEV)
    out = torch.zeros(1, device=DEV)
    st = lib.pcr_forward_project_noalloc(C.byref(g), C.byref(G), L.PCR_F32, C.c_void_p(vol.data_ptr()),
                                         C.c_void_p(out.data_ptr()), None)
    assert st == L.PCR_EINVAL
    assert b"fixed scratch" in lib.pcr_last_error()
