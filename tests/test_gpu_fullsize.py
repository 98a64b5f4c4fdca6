"""Parity at the full workload sizes, in the launch configuration the
benchmark uses (default tile shapes and layouts, rays clipped to the support
box of the warped image):

* paper scale (256x256x100 at 1.875x1.875x2.5 mm, K = 3, 512x384 detector at
  0.776 mm): the whole projection of the warped image, the fused cost and
  gradient, and a short warm-started solve, at an angle on each memory
  layout (30 deg x-fastest, 85 deg y-fastest);
* precision scale (256x256x128, K = 4, BF16 and FP16 storage): projection
  error against the FP64 oracle on the unrounded inputs and the fused cost;
* the largest serving size (512x512x160 over 480x480x320 mm, 1024x768
  detector): the projection on sampled rays, computed one by one by the
  oracle, and the fused cost of a K = 2 model;
* PCA training at paper scale (9 training DVFs of 3 x 6,553,600 FP32
  entries, K = 3), the size the benchmark measures, against the oracle's
  direct SVD of the same FP32 DVFs.
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


@pytest.fixture(scope="module")
def paper():
    g = S.grid_for("paper")
    m = S.pca_model(g, 3)
    f0_t, f0 = rounded(S.phantom(g), torch.float32)
    mean_t, mean = rounded(m.mean, torch.float32)
    U_t, U = rounded(m.U, torch.float32)
    L = _L()
    dm = L.DeviceModel(mean_t.to(DEV), U_t.to(DEV))
    return dict(g=g, m=m, f0=f0, mean=mean, U=U, df0=f0_t.to(DEV), dm=dm)


@pytest.mark.parametrize("angle", [30.0, 85.0])
def test_paper_scale_projection(paper, angle):
    L = _L()
    c = paper
    g, G = c["g"], S.geom_for("paper", math.radians(angle))
    w = S.truth_w(c["m"], 2.4)
    p = L.forward_project(g, G, L.warp_volume(g, c["df0"], L.dvf_compose(g, c["dm"], w)))
    f = oracle.warp(g, c["f0"], oracle.compose(g, c["mean"], c["U"], w))
    po = oracle.project(g, G, f)
    assert rel_l2(p.cpu().double().numpy(), po) <= 1e-5
    # and ray by ray on a seeded sample: FP32 sample positions are good to
    # ~1e-5 voxel, so a ray grazing a sharp edge carries an error of about
    # 1e-5 of the edge jump times a few samples -- bounded by 1e-5 of its own
    # value plus 1 % of the projection's largest value
    rng = np.random.default_rng(11)
    pn = p.cpu().double().numpy()
    pmax = float(np.abs(po).max())
    for iu, iv in zip(rng.integers(0, G.nu, 64), rng.integers(0, G.nv, 64)):
        ref = oracle.project_ray(g, G, f, int(iu), int(iv))
        assert abs(pn[iv, iu] - ref) <= 1e-5 * (abs(ref) + 0.01 * pmax)


@pytest.mark.parametrize("angle", [30.0, 85.0])
def test_paper_scale_fused_cost_grad(paper, angle):
    L = _L()
    c = paper
    g, G = c["g"], S.geom_for("paper", math.radians(angle))
    w_true = S.truth_w(c["m"], 2.4)
    y_np = oracle.project(g, G, oracle.warp(g, c["f0"], oracle.compose(g, c["mean"], c["U"], w_true)))
    y = torch.tensor(y_np, dtype=torch.float32, device=DEV)
    y_np = y.double().cpu().numpy()
    ctx = L.Context(g, c["dm"], c["df0"])
    for w in (0.85 * w_true, 1.2 * w_true):
        J, grad = ctx.cost_grad(y, G, w, 1.02, -0.01)
        Jo, go = oracle.cost_grad(g, G, c["f0"], c["mean"], c["U"], w, y_np, 1.02, -0.01)
        assert abs(J - Jo) <= 2e-5 * Jo, (J, Jo)
        assert rel_l2(grad, go) <= 1e-4, (grad, go)
    ctx.close()


def test_paper_scale_solve(paper):
    """Four Armijo iterations from the previous frame's true w (the warm start
    of the benchmark), against the oracle's solve with the same options."""
    L = _L()
    c = paper
    g = c["g"]
    i = 57                                     # projection 57 of the rotation
    cfg = S.config("paper")
    G = S.geom_for("paper", math.radians(i))
    w_true = S.truth_w(c["m"], S.breathing_phase(i / cfg["rate_hz"]))
    w_prev = S.truth_w(c["m"], S.breathing_phase((i - 1) / cfg["rate_hz"]))
    y_np = oracle.project(g, G, oracle.warp(g, c["f0"], oracle.compose(g, c["mean"], c["U"], w_true)))
    y = torch.tensor(y_np, dtype=torch.float32, device=DEV)
    y_np = y.double().cpu().numpy()
    ctx = L.Context(g, c["dm"], c["df0"])
    w, ab, st = ctx.reconstruct(y, G, w_prev, L.default_opts(max_iter=4, step0=c["m"].step0))
    ctx.close()
    wo, abo, sto, _ = oracle.solve(g, G, c["f0"], c["mean"], c["U"], y_np, w_prev,
                                   oracle.SolveOpts(max_iter=4, step0=c["m"].step0))
    assert st["iterations"] == sto["iterations"] and st["trials"] == sto["trials"]
    assert rel_l2(w, wo) <= 1e-3, (w, wo)
    assert abs(ab[0] - abo[0]) <= 1e-4 and abs(ab[1] - abo[1]) <= 1e-4 * max(1.0, abs(abo[1]))


@pytest.mark.parametrize("i", [100, 178])
def test_paper_scale_full_solve(paper, i):
    """Projection i of the rotation solved to the stopping rule (relative
    gradient 1e-4, at most 50 iterations), warm-started from the previous
    frame's true w, then the tumour localised, against the oracle's solve and
    localisation with the same options.  Frame 100 is a typical solve
    (~8 iterations in the benchmark); frame 178 is one of the slowest of the
    rotation (~40 iterations, near the turn of the breathing cycle).  Final w
    within 1e-3, (a, b) within 1e-4; the tumour follows the DVF, which moves
    by at most sum_k |dw_k| max|U_k| for a change dw of w, so the positions
    agree within 1e-3 sum_k |w_k| max|U_k| plus 1e-5 mm."""
    L = _L()
    c = paper
    g = c["g"]
    cfg = S.config("paper")
    G = S.geom_for("paper", math.radians(i))
    w_true = S.truth_w(c["m"], S.breathing_phase(i / cfg["rate_hz"]))
    w_prev = S.truth_w(c["m"], S.breathing_phase((i - 1) / cfg["rate_hz"]))
    y_np = oracle.project(g, G, oracle.warp(g, c["f0"], oracle.compose(g, c["mean"], c["U"], w_true)))
    y_t, y_np = rounded(y_np, torch.float32)
    p_ref = S.tumor_center(g)
    ctx = L.Context(g, c["dm"], c["df0"])
    w, ab, st = ctx.reconstruct(y_t.to(DEV), G, w_prev,
                                L.default_opts(max_iter=cfg["max_iter"], step0=c["m"].step0,
                                               localize=1, p_ref_mm=p_ref))
    ctx.close()
    print("frame %d: library %d iterations, %d trials, status %d" % (i, st["iterations"], st["trials"],
                                                                     st["status"]), flush=True)
    wo, abo, sto, _ = oracle.solve(g, G, c["f0"], c["mean"], c["U"], y_np, w_prev,
                                   oracle.SolveOpts(max_iter=cfg["max_iter"], step0=c["m"].step0))
    po, fst, _ = oracle.localize(g, c["mean"], c["U"], wo, p_ref)
    print("frame %d: oracle %d iterations, %d trials, status %d; w %.2e apart, tumour %.2e mm apart" % (
        i, sto["iterations"], sto["trials"], sto["status"], rel_l2(w, wo),
        np.linalg.norm(np.array(st["tumor_mm"]) - po)), flush=True)
    assert st["status"] == 0 and sto["status"] == 0
    assert rel_l2(w, wo) <= 1e-3, (w, wo)
    assert abs(ab[0] - abo[0]) <= 1e-4 and abs(ab[1] - abo[1]) <= 1e-4 * max(1.0, abs(abo[1]))
    umax = np.abs(c["U"]).reshape(len(wo), -1).max(axis=1)
    assert np.linalg.norm(np.array(st["tumor_mm"]) - po) <= 1e-3 * np.sum(np.abs(wo) * umax) + 1e-5


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_precision_scale_16bit(storage):
    L = _L()
    g = S.grid_for("precision")
    K = 4
    m = S.pca_model(g, K)
    f0 = S.phantom(g)
    dt = {"bf16": torch.bfloat16, "f16": torch.float16}[storage]
    if storage == "f16":
        scale = np.abs(m.U.reshape(K, -1)).max(axis=1)
        U_t, Ur = rounded(m.U / scale[:, None, None, None, None], dt)
        Ur = Ur * scale[:, None, None, None, None]
    else:
        scale = None
        U_t, Ur = rounded(m.U, dt)
    mean_t, meanr = rounded(m.mean, dt)
    f0_t, f0r = rounded(f0, dt)
    dm = L.DeviceModel(mean_t.to(DEV), U_t.to(DEV), scale=scale)
    G = S.geom_for("precision", math.radians(140.0))
    w = S.truth_w(m, 1.6)
    p = L.forward_project(g, G, L.warp_volume(g, f0_t.to(DEV), L.dvf_compose(g, dm, w)))
    p = p.cpu().double().numpy()
    po_r = oracle.project(g, G, oracle.warp(g, f0r, oracle.compose(g, meanr, Ur, w)))
    po = oracle.project(g, G, oracle.warp(g, f0, oracle.compose(g, m.mean, m.U, w)))
    assert rel_l2(p, po_r) <= 1e-5          # kernel error on the stored values
    assert rel_l2(p, po) <= 1e-2            # storage error against FP64 inputs
    # fused cost (FP32 image, and the FP16 image on request) against the
    # oracle on the stored values
    y = torch.tensor(po, dtype=torch.float32, device=DEV)
    Jo, go = oracle.cost_grad(g, G, f0r, meanr, Ur, 0.7 * w, y.double().cpu().numpy(), 1.0, 0.0)
    for image, tol_J, tol_g in ((torch.float32, 2e-5, 1e-4), (torch.float16, 2e-3, 1e-2)):
        ctx = L.Context(g, dm, f0_t.to(DEV), image_dtype=image)
        J, grad = ctx.cost_grad(y, G, 0.7 * w, 1.0, 0.0)
        ctx.close()
        assert abs(J - Jo) <= tol_J * Jo
        assert rel_l2(grad, go) <= tol_g


def test_largest_serving_size():
    L = _L()
    g = S.Grid((512, 512, 160), (480.0 / 512, 480.0 / 512, 320.0 / 160))
    G = S.Geom(math.radians(217.0), 1024, 768, 397.0 / 1024, 397.0 / 1024, 0.5 * 480.0 / 512)
    f0_t, f0 = rounded(S.phantom(g, texture=0.0), torch.float32)
    df0 = f0_t.to(DEV)
    p = L.forward_project(g, G, df0).cpu().double().numpy()
    rng = np.random.default_rng(12)
    pmax = float(np.abs(p).max())
    for iu, iv in zip(rng.integers(0, G.nu, 48), rng.integers(0, G.nv, 48)):
        ref = oracle.project_ray(g, G, f0, int(iu), int(iv))
        assert abs(p[iv, iu] - ref) <= 1e-5 * (abs(ref) + 0.01 * pmax)
    # fused cost of a K = 2 model at this size
    m = S.pca_model(g, 2)
    mean_t, mean = rounded(m.mean, torch.float32)
    U_t, U = rounded(m.U, torch.float32)
    dm = L.DeviceModel(mean_t.to(DEV), U_t.to(DEV))
    w = S.truth_w(m, 2.2)
    # the measurement from the oracle (the projection of the unwarped image)
    y_t, y_np = rounded(oracle.project(g, G, f0), torch.float32)
    y = y_t.to(DEV)
    ctx = L.Context(g, dm, df0)
    J, grad = ctx.cost_grad(y, G, w, 1.0, 0.0)
    ctx.close()
    Jo, go = oracle.cost_grad(g, G, f0, mean, U, w, y_np, 1.0, 0.0)
    assert abs(J - Jo) <= 2e-5 * Jo
    assert rel_l2(grad, go) <= 1e-4


def test_paper_scale_pca():
    L = _L()
    g = S.grid_for("paper")
    d = S.training_dvfs(g, 3)
    print("paper-scale PCA: 9 DVFs", d.shape, flush=True)
    mean, U, sing, wt = L.pca_train(g, torch.from_numpy(d).to(DEV), 3)
    mo, Uo, so, wo = oracle.pca(d, 3)
    assert rel_l2(mean.cpu().numpy(), mo) <= 1e-6
    for k in range(3):
        assert rel_l2(U[k].cpu().numpy(), Uo[k]) <= 2e-5, k
    np.testing.assert_allclose(sing, so, rtol=1e-6)
    np.testing.assert_allclose(wt, wo, rtol=1e-5, atol=1e-6 * np.abs(wo).max())


@pytest.mark.parametrize("angle", [30.0, 85.0])
def test_paper_scale_backprojection(angle):
    """P^T r at paper scale (the backprojection of the paper-order gradient
    and of the autograd gradient in f0) for a seeded residual, element by
    element.  A voxel sums r dt w over the samples whose cell it is a corner
    of.  FP32 sample positions carry an absolute error of up to ~6e-5 voxel
    (q = q_s + t dq cancels terms of ~500 voxels), so each trilinear weight
    is off by up to ~1e-4 in absolute terms, whatever its size; the 8 weights
    of a sample sum to 1 and its corners lie in the 3x3x3 voxels around any
    one of them, so the sum of |r| dt over the samples touching voxel v is at
    most the 3x3x3 box sum of B = P^T |r| around v.  Hence |dg[v]| <=
    1e-4 box27(B)[v] + 1e-5 B[v] (FP32 sums); plus the relative L2 error."""
    L = _L()
    g = S.grid_for("paper")
    G = S.geom_for("paper", math.radians(angle))
    rng = np.random.default_rng(13)
    r_t, r = rounded(rng.standard_normal((G.nv, G.nu)), torch.float32)
    print("backprojection at paper scale, angle", angle, flush=True)
    b = L.backproject_residual(g, G, r_t.to(DEV)).cpu().double().numpy()
    bo = oracle.backproject(g, G, r)
    babs = oracle.backproject(g, G, np.abs(r))
    err = np.abs(b - bo)
    box = np.zeros_like(babs)
    pad = np.pad(babs, 1)
    nz, ny, nx = babs.shape
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                box += pad[dz:dz + nz, dy:dy + ny, dx:dx + nx]
    bound = 1e-4 * box + 1e-5 * babs
    ratio = float(np.max(err / (bound + 1e-300)))
    print("max |dg| / bound = %.3e, max |dg| / P^T|r| = %.3e, rel L2 = %.3e" % (
        ratio, float(np.max(err / (babs + 1e-300))), rel_l2(b, bo)), flush=True)
    assert np.all(err <= bound)
    assert rel_l2(b, bo) <= 1e-5
    assert np.count_nonzero(babs) > 0.3 * babs.size      # the cone covers much of the volume
