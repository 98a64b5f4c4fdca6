"""The HIP library against the oracle's stored outputs on a small seeded
problem (tests/golden/tiny_oracle.json): projection, cost and gradient,
a short solve and the tumour position, at the parity tolerances."""
import json
import os
import sys

import numpy as np
import pytest

from helpers import rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_golden  # noqa: E402

DEV = "cuda"


def test_library_matches_stored_oracle_outputs():
    from paper_1004_0014_amd import _lib as L
    stored = json.load(open(make_golden.OUT))
    g, G, f0, mean, U = make_golden.inputs()
    inp = stored["inputs"]
    f0_t = torch.tensor(f0, dtype=torch.float64, device=DEV)
    dm = L.DeviceModel(torch.tensor(mean, dtype=torch.float64, device=DEV),
                       torch.tensor(U, dtype=torch.float64, device=DEV))
    # FP64 storage and compute: agreement to rounding
    p = L.forward_project(g, G, f0_t).cpu().numpy()
    assert rel_l2(p, np.asarray(stored["projection_f0"])) <= 1e-12
    y = torch.tensor(stored["y"], dtype=torch.float64, device=DEV)
    ctx = L.Context(g, dm, f0_t, compute=torch.float64)
    J, grad = ctx.cost_grad(y, G, inp["w_eval"], *inp["ab_eval"])
    assert abs(J - stored["cost"]) <= 1e-10 * stored["cost"]
    assert rel_l2(grad, stored["grad"]) <= 1e-8
    opts = L.default_opts(max_iter=inp["solve_iterations"], step0=inp["solve_step0"])
    w, ab, st = ctx.reconstruct(y, G, np.zeros(inp["K"]), opts)
    assert st["iterations"] == stored["solve"]["iterations"]
    assert st["trials"] == stored["solve"]["trials"]
    assert rel_l2(w, stored["solve"]["w"]) <= 1e-7
    ctx.close()
    pos, status, it = L.localize_tumor(g, dm, stored["solve"]["w"], inp["p_ref_mm"])
    assert status == 0
    # both stop the fixed point once a step is below 1e-6 mm
    assert np.max(np.abs(np.asarray(pos) - stored["tumour_mm"])) <= 1e-5
    # FP32 storage and compute: the parity tolerances
    f0_32 = f0_t.float()
    dm32 = L.DeviceModel(dm.mean.float(), dm.U.float())
    p32 = L.forward_project(g, G, f0_32).cpu().double().numpy()
    assert rel_l2(p32, np.asarray(stored["projection_f0"])) <= 1e-5
    ctx = L.Context(g, dm32, f0_32)
    J, grad = ctx.cost_grad(y.float(), G, inp["w_eval"], *inp["ab_eval"])
    assert abs(J - stored["cost"]) <= 2e-5 * stored["cost"]
    assert rel_l2(grad, stored["grad"]) <= 1e-4
    w, ab, st = ctx.reconstruct(y.float(), G, np.zeros(inp["K"]), opts)
    assert rel_l2(w, stored["solve"]["w"]) <= 1e-3
    ctx.close()
