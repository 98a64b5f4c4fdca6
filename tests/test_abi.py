"""CPU checks of the boundary: the built HIP library loads and exports every
function declared in include/pcr.h; the oracle and the product share no
code and neither imports the other."""
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
