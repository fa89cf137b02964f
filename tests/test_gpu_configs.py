"""Parity at the workload sizes: the room frame (200k Gaussians, 640x480),
the anchor decode at 50k anchors, one 1200x680 keyframe of the 1M-Gaussian
corridor in the batched launch configuration the benchmark times, and one
view of the 6M-Gaussian street.  Forward images are compared in full;
gradients on three seeded 128x128 crops (the other pixels' upstream weights
are zero on both sides)."""
import numpy as np
import pytest
import torch

import oracle
import scenes
from gpu_util import MARGINS, assert_grads, assert_images, assert_mask_fraction, masked_weights, np_, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _crop_mask(H, W, seed, n=3, size=128):
    rng = np.random.default_rng(seed)
    keep = np.zeros((H, W), bool)
    for _ in range(n):
        x0 = int(rng.integers(0, max(W - size, 0) + 1)); y0 = int(rng.integers(0, max(H - size, 0) + 1))
        keep[y0:y0 + size, x0:x0 + size] = True
    return keep


def _check_view(outs_v, g, cam, workload):
    ref = oracle.render(g, cam, margins=MARGINS)
    mask = ref["flags"]
    errs = assert_images(outs_v, ref, mask)
    frac = assert_mask_fraction(mask, workload)
    print("image errors", {k: f"{v:.2e}" for k, v in errs.items()}, f"masked {frac:.3%}", flush=True)
    return ref, mask


def _crop_weights(sc, v, mask, seed):
    cam = sc.cameras[v]
    keep = _crop_mask(cam.height, cam.width, seed)
    w = masked_weights(sc.weights[v], mask | ~keep)
    return w


def test_c2_room_frame():
    from paper_2505_18992_amd import render, render_backward
    sc = scenes.make_c2()
    g, cam = sc.sets[0], sc.cameras[0]
    print("case c2 full", flush=True)
    sets = [to_dev(g.arrays())]
    outs, saved = render(sets, [cam])
    ref, mask = _check_view(outs[0], g, cam, "c2")
    saved.close()
    w = _crop_weights(sc, 0, mask, 11)
    outs, saved = render(sets, [cam])
    grads, d_pose = render_backward(saved, [to_dev(w)])
    saved.close()
    G, S = oracle.grad(g, cam, *[x.astype(np.float64) for x in w])
    got = dict(zip(["means", "log_scales", "quats", "opacities", "colors"], [np_(t) for t in grads[0]]))
    got["pose"] = np_(d_pose)[0]
    print("grad report", assert_grads(got, G, S), flush=True)


def test_c4_keyframe_in_batched_launch():
    """The benchmark's launch: 8 keyframes at 1200x680 of the 1M-Gaussian
    corridor in one call; keyframes 0 and 5 are checked."""
    from paper_2505_18992_amd import render, render_backward
    sc = scenes.make_c4(sizes=(1200, 680))
    g = sc.sets[0]
    print("case c4-1200 batched", flush=True)
    sets = [to_dev(g.arrays())]
    ws = []
    refs = {}
    for v in (0, 5):
        ref = oracle.render(g, sc.cameras[v], margins=MARGINS)
        refs[v] = ref
    for v in range(8):
        if v in refs:
            ws.append(_crop_weights(sc, v, refs[v]["flags"], 40 + v))
        else:
            ws.append(tuple(np.zeros_like(a) for a in sc.weights[v]))
    outs, saved = render(sets, sc.cameras, sc.view_set)
    for v in (0, 5):
        errs = assert_images(outs[v], refs[v], refs[v]["flags"])
        frac = assert_mask_fraction(refs[v]["flags"], "c4")
        print(f"view {v} image errors", {k: f"{e:.2e}" for k, e in errs.items()}, f"masked {frac:.3%}", flush=True)
    grads, d_pose = render_backward(saved, [to_dev(w) for w in ws])
    saved.close()
    got = dict(zip(["means", "log_scales", "quats", "opacities", "colors"], [np_(t) for t in grads[0]]))
    G0, S0 = oracle.grad(g, sc.cameras[0], *[x.astype(np.float64) for x in ws[0]])
    G5, S5 = oracle.grad(g, sc.cameras[5], *[x.astype(np.float64) for x in ws[5]])
    G = {k: G0[k] + G5[k] for k in G0 if k != "pose"}
    S = {k: S0[k] + S5[k] for k in S0 if k != "pose"}
    print("grad report", assert_grads(got, G, S), flush=True)
    assert_grads({"pose": np_(d_pose)[0]}, {"pose": G0["pose"]}, S0)
    assert_grads({"pose": np_(d_pose)[5]}, {"pose": G5["pose"]}, S5)


def test_c5_street_view():
    from paper_2505_18992_amd import render, render_backward
    sc = scenes.make_c5()
    v = 9
    s = sc.view_set[v]
    g, cam = sc.sets[s], sc.cameras[v]
    print("case c5 view 9", flush=True)
    sets = [to_dev(x.arrays()) for x in sc.sets]
    outs, saved = render(sets, sc.cameras, sc.view_set)
    ref, mask = _check_view(outs[v], g, cam, "c5")
    w = [tuple(np.zeros_like(a) for a in ws) for ws in sc.weights]
    w[v] = _crop_weights(sc, v, mask, 77)
    grads, d_pose = render_backward(saved, [to_dev(x) for x in w])
    saved.close()
    G, S = oracle.grad(g, cam, *[x.astype(np.float64) for x in w[v]])
    got = dict(zip(["means", "log_scales", "quats", "opacities", "colors"], [np_(t) for t in grads[s]]))
    got["pose"] = np_(d_pose)[v]
    print("grad report", assert_grads(got, G, S), flush=True)
    # the oracle's own float32 evaluation against FP64 on the same crops: how
    # much of the gate an FP32 forward of the definition uses by itself
    G32, _ = oracle.grad(g, cam, *[x.astype(np.float64) for x in w[v]], fp32=True)
    print("oracle fp32 report", assert_grads({k: G32[k] for k in got}, G, S), flush=True)


def test_c3_decode_full_size():
    from oracle import decode as odec
    from paper_2505_18992_amd import decode_backward, decode_forward
    sc = scenes.make_c3()
    a, d = sc.anchors, sc.decoder
    cam = np.array([1.0, 2.0, 1.5], np.float32)
    print("case c3 decode 50k", flush=True)
    anchors = to_dev((a.xyz, a.feat, a.scale, a.offsets))
    mlp = tuple([torch.from_numpy(x).cuda() for x in lst] for lst in (d.W1, d.b1, d.W2, d.b2))
    got = [np_(t) for t in decode_forward(anchors, mlp, cam)]
    exp = [t.numpy() for t in odec.decode_forward(a.xyz, a.feat, a.scale, a.offsets, d.W1, d.b1, d.W2, d.b2,
                                                  cam.astype(np.float64))]
    for name, g_, e_ in zip(["means", "log_scales", "quats", "opacities", "colors"], got, exp):
        # a normalised quaternion's components err relative to the unit norm
        np.testing.assert_allclose(g_, e_, rtol=1e-5, atol=1e-5 if name == "quats" else 1e-6, err_msg=name)
    rng = np.random.default_rng(2)
    up = [rng.standard_normal(e_.shape).astype(np.float32) for e_ in exp]
    # anchors with a ReLU pre-activation within rounding of zero get no upstream
    flags = odec.relu_near_ties(a.xyz, a.feat, a.scale, a.offsets, d.W1, d.b1, d.W2, d.b2, cam.astype(np.float64))
    rows = np.repeat(flags, a.k)
    for u in up:
        u[rows] = 0.0
    print("relu near-tie anchors", int(flags.sum()), flush=True)
    d_feat, d_scale, d_off, (dW1, db1, dW2, db2) = decode_backward(anchors, mlp, cam, to_dev(up))
    G = odec.decode_backward(a.xyz, a.feat, a.scale, a.offsets, d.W1, d.b1, d.W2, d.b2, cam.astype(np.float64), up)
    pairs = [("feat", d_feat, G["feat"]), ("scale", d_scale, G["scale"]), ("offsets", d_off, G["offsets"])]
    for h in range(3):
        pairs += [(f"W1[{h}]", dW1[h], G["W1"][h]), (f"b1[{h}]", db1[h], G["b1"][h]),
                  (f"W2[{h}]", dW2[h], G["W2"][h]), (f"b2[{h}]", db2[h], G["b2"][h])]
    for name, g_, e_ in pairs:
        g_ = np_(g_).astype(np.float64)
        nrm = np.linalg.norm(g_ - e_) / np.linalg.norm(e_)
        assert nrm <= 1e-5, (name, nrm)
        assert np.max(np.abs(g_ - e_)) <= 1e-4 * np.abs(e_).max() + 1e-7, (name, np.max(np.abs(g_ - e_)))


def _window_vs_oracle(sc, check_views, tile, persistent, seed):
    """A RenderWindow (graph-captured, every view in one launch per part)
    against the oracle on the checked views: images in full, gradients on
    three 128x128 crops of each checked view (the other views' upstream
    weights are zero), the pose of each checked view; and a second replay
    equal to the first (forward bit for bit)."""
    from paper_2505_18992_amd import RenderWindow
    g = sc.sets[0]
    sets = [to_dev(g.arrays())]
    refs = {v: oracle.render(g, sc.cameras[v], margins=MARGINS) for v in check_views}
    win = RenderWindow(sets, sc.cameras, sc.view_set, tile=tile, persistent=persistent)
    cfg = win.config()
    print("window config", cfg, flush=True)
    ws = {}
    for v in range(len(sc.cameras)):
        if v in refs:
            ws[v] = _crop_weights(sc, v, refs[v]["flags"], seed + v)
            for dst, src in zip(win.grad_out[v], to_dev(ws[v])):
                dst.copy_(src)
        else:
            for dst in win.grad_out[v]:
                dst.zero_()
    win.run()
    torch.cuda.synchronize()
    first = [tuple(t.clone() for t in win.outputs[v]) for v in check_views]
    for v in check_views:
        errs = assert_images(win.outputs[v], refs[v], refs[v]["flags"])
        frac = assert_mask_fraction(refs[v]["flags"], "c4")
        print(f"view {v} ({sc.cameras[v].width}x{sc.cameras[v].height}) image errors",
              {k: f"{e:.2e}" for k, e in errs.items()}, f"masked {frac:.3%}", flush=True)
    GS = {v: oracle.grad(g, sc.cameras[v], *[x.astype(np.float64) for x in ws[v]]) for v in check_views}
    keys = ["means", "log_scales", "quats", "opacities", "colors"]
    G = {k: sum(GS[v][0][k] for v in check_views) for k in keys}
    S = {k: sum(GS[v][1][k] for v in check_views) for k in keys}
    S.update({k + "_fp32": sum(GS[v][1][k + "_fp32"] for v in check_views) for k in keys})
    got = dict(zip(keys, [np_(t) for t in win.grads[0]]))
    print("grad report", assert_grads(got, G, S), flush=True)
    for v in check_views:
        assert_grads({"pose": np_(win.d_pose)[v]}, {"pose": GS[v][0]["pose"]}, GS[v][1])
    win.run()
    torch.cuda.synchronize()
    for v, f in zip(check_views, first):
        for a, b in zip(win.outputs[v], f):
            assert torch.equal(a, b)
    win.close()


def test_c4_bench_window_matches_oracle():
    """The benchmark's configuration exactly: 8 keyframes at 1200x680 of the
    1M-Gaussian corridor in a graph-captured window with 32x8 tiles and one
    compositing workgroup per tile."""
    sc = scenes.make_c4(sizes=(1200, 680))
    print("case c4-1200 bench window", flush=True)
    _window_vs_oracle(sc, (0, 5), (32, 8), 0, 60)


def test_c4_mixed_window_matches_oracle():
    """The corridor keyframes at their mixed resolutions (640x480, 960x540,
    1200x680), tile shape and compositing mode picked by the window's
    search; a view of each size is checked."""
    sc = scenes.make_c4()
    sizes = [(c.width, c.height) for c in sc.cameras]
    print("case c4 mixed window", sizes, flush=True)
    first = {}
    for v, s in enumerate(sizes):
        first.setdefault(s, v)
    views = tuple(sorted(first.values()))
    assert len(views) == 3
    _window_vs_oracle(sc, views, None, -1, 70)
