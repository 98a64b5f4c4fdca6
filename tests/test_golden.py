"""The oracle against its stored outputs on a small seeded problem
(tests/golden/tiny_oracle.json, written by tests/golden/make_golden.py):
any later change to the oracle's arithmetic fails here.  The oracle runs its
ray and voxel loops with OpenMP, so sums may be reordered: values are
compared to 1e-10 relative."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_golden  # noqa: E402


def _close(a, b, rtol=1e-10, atol=0.0):
    a, b = np.asarray(a, float), np.asarray(b, float)
    assert a.shape == b.shape
    assert np.all(np.abs(a - b) <= atol + rtol * np.maximum(np.abs(a), np.abs(b))), (a, b)


def test_oracle_matches_stored_outputs():
    stored = json.load(open(make_golden.OUT))
    now = make_golden.compute()
    scale = np.abs(np.asarray(stored["y"])).max()
    _close(now["y"], stored["y"], atol=1e-12 * scale)
    _close(now["projection_f0"], stored["projection_f0"], atol=1e-12 * scale)
    _close(now["cost"], stored["cost"])
    _close(now["grad"], stored["grad"], atol=1e-12 * np.abs(stored["grad"]).max())
    assert now["solve"]["iterations"] == stored["solve"]["iterations"]
    assert now["solve"]["trials"] == stored["solve"]["trials"]
    assert now["solve"]["status"] == stored["solve"]["status"]
    _close(now["solve"]["w"], stored["solve"]["w"], rtol=1e-9)
    _close(now["solve"]["ab"], stored["solve"]["ab"], rtol=1e-9)
    _close(now["tumour_mm"], stored["tumour_mm"], atol=1e-9)
    assert now["tumour_status"] == stored["tumour_status"] == 0
