"""Mapping loss (eq. 7-9) on the GPU against the float64 oracle, through the
C ABI: the loss terms and the gradient planes per view, ragged and tiny image
sizes, a window-sized view, and the volume term."""
import numpy as np
import pytest
import torch

import scenes
from oracle import loss as oracle_loss

pytestmark = pytest.mark.gpu

# Terms: the loss is a mean of float32 per-pixel values summed in double.
TERM_RTOL = 2e-5
# Gradient: per element |g - g_ref| <= GRAD_TOL * scale + B_FACTOR * fp32 +
# floor, scale and fp32 from oracle_loss.view_grad_bounds (term magnitudes
# and the float32 rounding amplification of the SSIM statistics).  On these
# cases every element is within GRAD_TOL * scale alone (the test prints how
# many fp32 bounds an element needs beyond it: none); the fp32 term covers
# images whose local variance is small against their mean.
GRAD_TOL = 1e-5
B_FACTOR = 4.0


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


class _Cam:
    def __init__(self, W, H):
        self.width, self.height = W, H
        self.fx = self.fy = 100.0
        self.cx, self.cy = W / 2, H / 2
        self.world_to_cam = np.eye(3, 4, dtype=np.float32)


def _view(seed, W, H):
    rng = np.random.default_rng(seed)
    # smooth structure plus noise, like rendered frames against captured ones
    yy, xx = np.mgrid[0:H, 0:W]
    base = 0.5 + 0.3 * np.sin(xx / 7.0 + seed)[None] * np.cos(yy / 5.0)[None] * np.array([1, 0.8, 0.6])[:, None, None]
    x = np.clip(base + rng.normal(0, 0.05, (3, H, W)), 0, 1).astype(np.float32)
    y = np.clip(x + rng.normal(0, 0.08, x.shape), 0, 1).astype(np.float32)
    d = rng.uniform(1, 6, (H, W)).astype(np.float32)
    t = (d + rng.normal(0, 0.3, d.shape)).astype(np.float32)
    t[rng.uniform(size=t.shape) < 0.15] = 0.0
    return x, d, y, t


def _run(views, lam_ssim=0.2, lam_d=1.0):
    from paper_2505_18992_amd import mapping_loss
    dev = "cuda"
    ims = [(torch.from_numpy(x).to(dev), torch.from_numpy(d).to(dev)) for x, d, _, _ in views]
    tgs = [(torch.from_numpy(y).to(dev), torch.from_numpy(t).to(dev)) for _, _, y, t in views]
    cams = [_Cam(v[0].shape[2], v[0].shape[1]) for v in views]
    terms, grads = mapping_loss(ims, tgs, cams, lam_ssim, lam_d)
    torch.cuda.synchronize()
    return terms.cpu().numpy(), [tuple(g.cpu().numpy() for g in gv) for gv in grads]


def _check_view(x, d, y, t, terms, grads, lam_ssim=0.2, lam_d=1.0):
    ref = oracle_loss.view_loss(x, d, y, t, lam_ssim, lam_d)
    for k, name in enumerate(("L_c", "L_ssim", "L_d", "total")):
        assert abs(terms[k] - ref[name]) <= TERM_RTOL * abs(ref[name]) + 1e-9, (name, terms[k], ref[name])
    gx_ref, gd_ref = oracle_loss.view_loss_grad(x, d, y, t, lam_ssim, lam_d)
    scale, fp32 = oracle_loss.view_grad_bounds(x, y, lam_ssim, lam_d)
    gx, gd, ga = grads
    # the L1 kink: pixels where X and Y (or D and T) agree to 1e-6 may take
    # either sign
    kink = np.abs(x.astype(np.float64) - y) < 1e-6
    err = np.abs(gx - gx_ref)
    bound = GRAD_TOL * scale + B_FACTOR * fp32 + 1e-12
    bad = (err > bound) & ~kink
    need = np.maximum(err - GRAD_TOL * scale, 0.0) / (fp32 + 1e-30)
    print("fp32 bounds needed beyond the scale term", float(need[~kink].max()), flush=True)
    assert not bad.any(), (int(bad.sum()), float((err / bound)[~kink].max()))
    dk = (t > 0) & (np.abs(d.astype(np.float64) - t) < 1e-6)
    assert np.all(np.abs(gd - gd_ref)[~dk] <= 1e-6 * np.abs(gd_ref).max() + 1e-12)
    assert np.all(ga == 0.0)
    return float((err / bound)[~kink].max())


def test_loss_ragged_views_match_the_oracle():
    views = [_view(1, 37, 29), _view(2, 70, 45), _view(3, 64, 32)]
    print("case loss ragged", flush=True)
    terms, grads = _run(views)
    for v, (x, d, y, t) in enumerate(views):
        _check_view(x, d, y, t, terms[v], grads[v])


def test_loss_views_smaller_than_the_window():
    views = [_view(4, 7, 9), _view(5, 1, 1), _view(6, 12, 3)]
    print("case loss tiny", flush=True)
    terms, grads = _run(views)
    for v, (x, d, y, t) in enumerate(views):
        _check_view(x, d, y, t, terms[v], grads[v])


def test_loss_weights_and_no_target_depth():
    x, d, y, t = _view(7, 50, 40)
    t[:] = 0.0  # no target depth anywhere: L_d = 0, no depth gradient
    print("case loss weights", flush=True)
    terms, grads = _run([(x, d, y, t)], lam_ssim=0.6, lam_d=0.3)
    assert terms[0][2] == 0.0 and np.all(grads[0][1] == 0.0)
    _check_view(x, d, y, t, terms[0], grads[0], 0.6, 0.3)


def test_loss_identical_images():
    x, d, _, _ = _view(8, 45, 33)
    print("case loss identical", flush=True)
    terms, grads = _run([(x, d, x.copy(), d.copy())])
    assert abs(terms[0][3]) < 1e-6  # SSIM = 1, L1 = 0
    assert np.abs(grads[0][0]).max() < 1e-6 and np.abs(grads[0][1]).max() == 0.0


def test_loss_at_workload_size():
    # one 1200x680 view: rendered frame of the corridor scene against a
    # perturbed copy of itself
    from paper_2505_18992_amd import render
    sc = scenes.make_c4(n=200_000, views=1, sizes=(1200, 680))
    g = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in sc.sets[0].arrays()]
    outs, saved = render([tuple(g)], sc.cameras, [0], tile=(32, 8))
    saved.close()
    x = outs[0][0].cpu().numpy(); d = outs[0][1].cpu().numpy()
    rng = np.random.default_rng(9)
    y = np.clip(x + rng.normal(0, 0.05, x.shape), 0, 1).astype(np.float32)
    t = np.where(d > 0, d + rng.normal(0, 0.1, d.shape), 0.0).astype(np.float32)
    print("case loss 1200x680", flush=True)
    terms, grads = _run([(x, d, y, t)])
    worst = _check_view(x, d, y, t, terms[0], grads[0])
    print("worst gradient error / bound", worst, flush=True)


def test_volume_loss_matches_closed_form_and_adds():
    from paper_2505_18992_amd import volume_loss
    rng = np.random.default_rng(10)
    sets, grads, base = [], [], []
    for n in (1000, 1, 0):
        arrs = [rng.normal(0, 1, (n, 3)), rng.normal(-3, 0.5, (n, 3)), rng.normal(0, 1, (n, 4)),
                rng.uniform(0, 1, (n,)), rng.uniform(0, 1, (n, 3))]
        sets.append(tuple(torch.from_numpy(a.astype(np.float32)).cuda() for a in arrs))
        g0 = rng.normal(0, 1e-3, (n, 3)).astype(np.float32)
        base.append(g0)
        grads.append(tuple(torch.zeros_like(t) for t in sets[-1][:1]) + (torch.from_numpy(g0).cuda(),))
    print("case volume", flush=True)
    out = volume_loss(sets, grads, 0.001).cpu().numpy()
    for s in range(3):
        ls = sets[s][1].cpu().numpy()
        val, gref = oracle_loss.volume_loss(ls, 0.001)
        assert abs(out[s] - val) <= 1e-6 * abs(val) + 1e-12
        got = grads[s][1].cpu().numpy()
        assert np.allclose(got, base[s] + gref, rtol=1e-5, atol=1e-12)
