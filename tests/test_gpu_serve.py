"""Serving engine on the GPU: continuous batching of solves for streams of
different volume and detector sizes.

* every result computed inside the mix equals (bitwise: the fused gradient
  path has fixed-order reductions and no atomics) the same request solved
  alone from the same warm start;
* streams are admitted by HBM footprint (PCR_EBUSY beyond the budget);
* a stale queued frame is dropped when a newer one of its stream arrives;
* warm starts can be snapshot and restored; streams can be removed;
* a served solve agrees with the FP64 oracle.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1004_0014_amd import synth as S
from helpers import rel_l2, rounded

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


def _L():
    from paper_1004_0014_amd import _lib
    return _lib


class SmallStream:
    """A small seeded stream: grid, K, detector, model, f0 and measured
    projections of consecutive frames (oracle-generated)."""

    def __init__(self, n, sp, K, nu, nv, du, n_frames, t0=0.0):
        L = _L()
        self.grid = S.Grid(n, sp)
        self.K = K
        self.m = S.pca_model(self.grid, K)
        self.f0_t, self.f0 = rounded(S.phantom(self.grid), torch.float32)
        self.mean_t, self.mean = rounded(self.m.mean, torch.float32)
        self.U_t, self.U = rounded(self.m.U, torch.float32)
        self.dm = L.DeviceModel(self.mean_t.to(DEV), self.U_t.to(DEV))
        self.df0 = self.f0_t.to(DEV)
        self.geoms, self.ys, self.y_np, self.w_true = [], [], [], []
        for j in range(n_frames):
            t = t0 + j / 11.0
            ang = math.radians((37.0 + 6.0 * t * 10) % 360)
            G = S.Geom(ang, nu, nv, du, du, 0.5 * min(sp))
            w = S.truth_w(self.m, S.breathing_phase(t))
            y = oracle.project(self.grid, G, oracle.warp(self.grid, self.f0,
                                                         oracle.compose(self.grid, self.mean, self.U, w)))
            self.geoms.append(G)
            self.y_np.append(y)
            self.ys.append(torch.tensor(y, dtype=torch.float32, device=DEV))
            self.w_true.append(w)
        self.opts = L.default_opts(max_iter=25, step0=self.m.step0, localize=1,
                                   p_ref_mm=S.tumor_center(self.grid))


@pytest.fixture(scope="module")
def streams():
    specs = [((40, 40, 32), (6.0, 6.0, 8.0), 2, 64, 48, 4.0),
             ((56, 48, 40), (4.5, 5.0, 6.0), 3, 96, 64, 3.0),
             ((64, 64, 48), (4.0, 4.0, 5.0), 3, 128, 96, 2.4),
             ((33, 45, 28), (7.0, 5.0, 8.0), 2, 80, 60, 3.6),
             ((72, 60, 36), (3.5, 4.0, 7.0), 3, 112, 80, 2.6)]
    return [SmallStream(*sp, n_frames=3, t0=0.13 * i) for i, sp in enumerate(specs)]


def test_mix_equals_alone_bitwise(streams):
    L = _L()
    srv = L.Server(hbm_budget_bytes=8 << 30, max_slots=3, drop_stale=False)
    sids = [srv.add_stream(st.grid, st.dm, st.df0, st.opts, np.zeros(st.K)) for st in streams]
    # interleave submissions of all streams (frames in order per stream)
    expect = {}
    for j in range(3):
        for st, sid in zip(streams, sids):
            rid = srv.submit(sid, st.ys[j], st.geoms[j])
            expect[rid] = (st, j)
    srv.drain()
    res = srv.poll(64)
    assert len(res) == len(expect)
    assert all(r["status"] in (0, -4) for r in res), [r["status"] for r in res]
    for r in res:
        st, j = expect[r["req_id"]]
        ctx = L.Context(st.grid, st.dm, st.df0)
        w, ab, sta = ctx.reconstruct(st.ys[j], st.geoms[j], r["w0"], st.opts)
        ctx.close()
        assert w == r["w"], (r["req_id"], w, r["w"])          # bitwise
        assert list(ab) == r["ab"]
        assert sta["iterations"] == r["iterations"] and sta["trials"] == r["trials"]
        assert sta["samples"] == r["samples"] > 0
        assert np.allclose(sta["tumor_mm"], r["tumor_mm"], rtol=0, atol=0)
    # warm starts chain: each stream's frame j started from its frame j-1 result
    by_stream = {}
    for r in sorted(res, key=lambda r: r["req_id"]):
        by_stream.setdefault(r["stream_id"], []).append(r)
    for rs in by_stream.values():
        for prev, cur in zip(rs, rs[1:]):
            assert cur["w0"] == prev["w"]
    srv.close()


def test_served_solve_matches_oracle(streams):
    L = _L()
    st = streams[2]
    srv = L.Server(hbm_budget_bytes=4 << 30, max_slots=2)
    sid = srv.add_stream(st.grid, st.dm, st.df0, st.opts, np.zeros(st.K))
    srv.submit(sid, st.ys[0], st.geoms[0])
    srv.drain()
    (r,) = srv.poll(4)
    wo, abo, sto, _ = oracle.solve(st.grid, st.geoms[0], st.f0, st.mean, st.U, st.y_np[0],
                                   np.zeros(st.K), oracle.SolveOpts(max_iter=25, step0=st.m.step0))
    assert rel_l2(r["w"], wo) <= 1e-3
    srv.close()


def test_admission_by_hbm_footprint(streams):
    L = _L()
    big, small = streams[4], streams[0]
    # small stream: 2 MB copies + 2 slots x 9 MB scratch = 20 MB; with the big
    # one (8 MB copies, 11 MB scratch per slot) 32 MB
    srv = L.Server(hbm_budget_bytes=25 << 20, max_slots=2)
    sid = srv.add_stream(small.grid, small.dm, small.df0, small.opts, np.zeros(small.K))
    with pytest.raises(L.PCRError) as e:
        srv.add_stream(big.grid, big.dm, big.df0, big.opts, np.zeros(big.K))
    assert e.value.status == L.PCR_EBUSY
    # the admitted stream still serves
    srv.submit(sid, small.ys[0], small.geoms[0])
    srv.drain()
    assert srv.poll(4)[0]["status"] in (0, -4)
    assert 0 < srv.device_bytes <= 25 << 20
    srv.close()


def test_stale_frame_dropped_and_state_restore(streams):
    L = _L()
    a, b = streams[4], streams[1]
    srv = L.Server(hbm_budget_bytes=8 << 30, max_slots=1, drop_stale=True)
    sa = srv.add_stream(a.grid, a.dm, a.df0, a.opts, np.zeros(a.K))
    sb = srv.add_stream(b.grid, b.dm, b.df0, b.opts, np.zeros(b.K))
    ra = srv.submit(sa, a.ys[0], a.geoms[0])          # takes the only slot
    rb1 = srv.submit(sb, b.ys[0], b.geoms[0])         # queued
    rb2 = srv.submit(sb, b.ys[1], b.geoms[1])         # supersedes rb1
    srv.drain()
    res = {r["req_id"]: r for r in srv.poll(8)}
    assert set(res) == {ra, rb1, rb2}
    assert res[rb1]["status"] == L.PCR_EBUSY          # dropped as stale
    assert res[rb2]["status"] in (0, -4) and res[ra]["status"] in (0, -4)
    # snapshot / restore of the warm start
    w = srv.get_w(sb, b.K)
    assert w == res[rb2]["w"]
    srv.set_w(sb, [0.0] * b.K)
    rb3 = srv.submit(sb, b.ys[2], b.geoms[2])
    srv.drain()
    r3 = srv.poll(4)[0]
    assert r3["req_id"] == rb3 and r3["w0"] == [0.0] * b.K
    srv.remove_stream(sa)
    with pytest.raises(L.PCRError):
        srv.submit(sa, a.ys[0], a.geoms[0])
    srv.close()


@pytest.mark.parametrize("order", [1, 2])
def test_predicted_warm_start(streams, order):
    """With predict_order > 0 a stream's next solve starts from the polynomial
    extrapolation of its last results to the new frame's submit time."""
    L = _L()
    st = streams[1]
    srv = L.Server(hbm_budget_bytes=4 << 30, max_slots=1, predict_order=order)
    sid = srv.add_stream(st.grid, st.dm, st.df0, st.opts, np.zeros(st.K))
    res = []
    for j in range(3):
        srv.submit(sid, st.ys[j], st.geoms[j])
        srv.drain()
        res += srv.poll(4)
    assert [r["status"] in (0, -4) for r in res] == [True] * 3
    # frame 1 has one result of history: plain warm start
    assert res[1]["w0"] == res[0]["w"]
    hist = res[:2]
    expect = L.predict_w([r["w"] for r in hist], [r["t_submit_s"] for r in hist],
                         res[2]["t_submit_s"], order)
    assert np.allclose(res[2]["w0"], expect, rtol=1e-12, atol=1e-12)
    srv.close()


def test_chained_step_size(streams):
    """With chain_step each solve's first trial uses the step size the
    stream's previous solve ended with; the result equals a blocking solve
    given that step size (opts.mu0)."""
    L = _L()
    st = streams[2]
    srv = L.Server(hbm_budget_bytes=4 << 30, max_slots=1, chain_step=True)
    sid = srv.add_stream(st.grid, st.dm, st.df0, st.opts, np.zeros(st.K))
    res = []
    for j in range(3):
        srv.submit(sid, st.ys[j], st.geoms[j])
        srv.drain()
        res += srv.poll(4)
    assert res[0]["mu0"] == 0.0 and res[0]["mu"] > 0
    for prev, cur in zip(res, res[1:]):
        assert cur["mu0"] == prev["mu"]
    ctx = L.Context(st.grid, st.dm, st.df0)
    opts = L.default_opts(max_iter=25, step0=st.m.step0, localize=1,
                          p_ref_mm=S.tumor_center(st.grid), mu0=res[2]["mu0"])
    w, ab, sta = ctx.reconstruct(st.ys[2], st.geoms[2], res[2]["w0"], opts)
    ctx.close()
    assert w == res[2]["w"] and sta["trials"] == res[2]["trials"]
    assert sta["mu"] == res[2]["mu"]
    srv.close()


def test_carried_move_with_predicted_start(streams):
    """With carry_move (and a predicted warm start) each solve's first trial
    moves w by the distance the stream's previous solve moved it, clamped to
    [1e-3, 1] x step0; the result equals a blocking solve given the same
    start and step0."""
    L = _L()
    st = streams[1]
    srv = L.Server(hbm_budget_bytes=4 << 30, max_slots=1, predict_order=1, carry_move=True)
    sid = srv.add_stream(st.grid, st.dm, st.df0, st.opts, np.zeros(st.K))
    res = []
    for j in range(3):
        srv.submit(sid, st.ys[j], st.geoms[j])
        srv.drain()
        res += srv.poll(4)
    assert [r["status"] in (0, -4) for r in res] == [True] * 3
    s0 = st.m.step0
    assert res[0]["step0"] == s0
    for prev, cur in zip(res, res[1:]):
        move = float(np.linalg.norm(np.array(prev["w"]) - np.array(prev["w0"])))
        assert abs(cur["step0"] - min(max(move, 1e-3 * s0), s0)) <= 1e-12 * s0
        assert cur["mu0"] == 0.0
    ctx = L.Context(st.grid, st.dm, st.df0)
    opts = L.default_opts(max_iter=25, step0=res[2]["step0"], localize=1,
                          p_ref_mm=S.tumor_center(st.grid))
    w, ab, sta = ctx.reconstruct(st.ys[2], st.geoms[2], res[2]["w0"], opts)
    ctx.close()
    assert w == res[2]["w"] and sta["trials"] == res[2]["trials"]
    srv.close()
    with pytest.raises(L.PCRError):
        L.Server(hbm_budget_bytes=4 << 30, max_slots=1, chain_step=True, carry_move=True)
