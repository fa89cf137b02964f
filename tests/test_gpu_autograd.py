"""The torch.autograd.Functions of the render and the decode on the GPU:
gradients through autograd against the FP64 oracle, a float32 central
difference smoke of the GPU forward, and the decode -> render -> loss ->
backward chain of the anchor workload at its full size (50 k anchors,
1200x680)."""
import numpy as np
import pytest
import torch

import oracle
import scenes
from gpu_util import (MARGINS, assert_grads, assert_images, assert_mask_fraction, masked_weights, np_, to_dev)
from oracle import decode as odec

pytestmark = pytest.mark.gpu

KEYS = ["means", "log_scales", "quats", "opacities", "colors"]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _leaves(g):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda().requires_grad_(True) for a in g.arrays()]


def _second_view(cam):
    """The C1 camera turned by a few degrees and moved by a few centimetres."""
    from scipy.spatial.transform import Rotation
    c = cam.copy()
    R = Rotation.from_rotvec([0.05, -0.08, 0.03]).as_matrix()
    c.world_to_cam = np.concatenate([R, np.array([[0.1], [-0.05], [0.2]])], axis=1).astype(np.float32)
    return c


def test_render_views_autograd_matches_oracle():
    """render_views over one set and two views: every leaf's .grad (the five
    Gaussian tensors and the [2, 6] pose increment) against the oracle."""
    from paper_2505_18992_amd import render_views
    sc = scenes.make_c1()
    g, cam0 = sc.sets[0], sc.cameras[0]
    cams = [cam0, _second_view(cam0)]
    print("case render_views c1 x2", flush=True)
    weights = scenes.upstream_weights(111, cams)
    refs = [oracle.render(g, c, margins=MARGINS) for c in cams]
    assert refs[1]["n_blend"].sum() > 10_000, "the second view must see the scene"
    ws = [masked_weights(w, r["flags"]) for w, r in zip(weights, refs)]
    leaves = _leaves(g)
    pose = torch.zeros((2, 6), dtype=torch.float32, device="cuda", requires_grad=True)
    outs = render_views([tuple(leaves)], cams, pose_delta=pose)
    for v in range(2):
        assert_images(outs[v], refs[v], refs[v]["flags"])
    loss = sum((o * torch.from_numpy(w).cuda()).sum() for v in range(2) for o, w in zip(outs[v], ws[v]))
    loss.backward()
    Gs, Ss = zip(*[oracle.grad(g, c, *[x.astype(np.float64) for x in w]) for c, w in zip(cams, ws)])
    G = {k: Gs[0][k] + Gs[1][k] for k in KEYS}
    S = {k: Ss[0][k] + Ss[1][k] for k in KEYS}
    S.update({k + "_fp32": Ss[0][k + "_fp32"] + Ss[1][k + "_fp32"] for k in KEYS})
    got = {k: np_(t.grad) for k, t in zip(KEYS, leaves)}
    print("grad report", assert_grads(got, G, S), flush=True)
    for v in range(2):
        assert_grads({"pose": np_(pose.grad)[v]}, {"pose": Gs[v]["pose"]}, Ss[v])


def test_render_views_central_differences_smoke():
    """float32 central differences of the GPU forward against autograd for
    a few parameters of the best-covered Gaussians.  Pixels near a cutoff
    (margins 5e-3, wider than any step below moves alpha) carry no weight,
    so no step crosses a cutoff; the loss is summed in float64 over the
    bitwise difference of the two renders."""
    from paper_2505_18992_amd import render, render_views
    sc = scenes.make_c1(n=300, width=64, height=48)
    g, cam = sc.sets[0], sc.cameras[0]
    print("case render_views fd smoke", flush=True)
    ref = oracle.render(g, cam, margins=(5e-3, 5e-3, 5e-3))
    w = [torch.from_numpy(x).cuda().double() for x in masked_weights(sc.weights[0], ref["flags"])]
    leaves = _leaves(g)
    outs = render_views([tuple(leaves)], [cam])[0]
    loss = sum((o.double() * wi).sum() for o, wi in zip(outs, w))
    loss.backward()
    # the Gaussians with the largest colour-gradient magnitude are the best covered
    cover = np.abs(np_(leaves[4].grad)).sum(1)
    top = np.argsort(-cover)[:3]
    base = [np.ascontiguousarray(a) for a in g.arrays()]
    checks = 0
    for i in top:
        for name, col, step in (("means", 0, 2e-5), ("means", 2, 2e-5), ("log_scales", 1, 1e-4),
                                ("quats", 2, 1e-4), ("opacities", None, 2e-4), ("colors", 1, 1e-2)):
            k = KEYS.index(name)
            idx = (i,) if col is None else (i, col)
            grad = float(np_(leaves[k].grad)[idx])
            planes = []
            for sgn in (1.0, -1.0):
                arrs = [a.copy() for a in base]
                arrs[k][idx] += np.float32(sgn * step)
                o, _ = render([to_dev(arrs)], [cam], keep=False)
                planes.append(o[0])
            h = float(np.float32(base[k][idx] + np.float32(step)) - np.float32(base[k][idx] - np.float32(step)))
            dL = sum(((p - m).double() * wi).sum() for p, m, wi in zip(planes[0], planes[1], w)).item()
            fd = dL / h
            tol = 2e-2 * abs(grad) + 1e-3 * float(np.abs(np_(leaves[k].grad)).max())
            print(f"  {name}[{idx}] autograd {grad:+.6e} fd {fd:+.6e}", flush=True)
            assert abs(fd - grad) <= tol, (name, idx, grad, fd)
            checks += 1
    assert checks == 18


def _dev_decoder(d):
    return tuple([torch.from_numpy(x).cuda().requires_grad_(True) for x in lst] for lst in (d.W1, d.b1, d.W2, d.b2))


def _untie(up, a, d, cam):
    flags = odec.relu_near_ties(a.xyz, a.feat, a.scale, a.offsets, d.W1, d.b1, d.W2, d.b2, cam.astype(np.float64))
    keep = torch.from_numpy(~np.repeat(flags, a.k)).cuda()
    return [u * (keep.view(-1, *([1] * (u.dim() - 1)))) for u in up], int(flags.sum())


DEC_NAMES = ["feat", "scale", "offsets"] + [f"{p}[{h}]" for p in ("W1", "b1", "W2", "b2") for h in range(3)]


def _decode_grads_vs_oracle(a, d, centre, leaves_anchor, mlp, up, tol=1e-5):
    G = odec.decode_backward(a.xyz, a.feat, a.scale, a.offsets, d.W1, d.b1, d.W2, d.b2, centre.astype(np.float64),
                             [np_(u).astype(np.float64) for u in up])
    exp = [G["feat"], G["scale"], G["offsets"]] + [G[p][h] for p in ("W1", "b1", "W2", "b2") for h in range(3)]
    got = list(leaves_anchor) + [t for lst in mlp for t in lst]
    worst = 0.0
    for name, t, e in zip(DEC_NAMES, got, exp):
        gg = np_(t.grad).astype(np.float64)
        nrm = np.linalg.norm(gg - e) / max(np.linalg.norm(e), 1e-30)
        worst = max(worst, nrm)
        assert nrm <= tol, (name, nrm)
        assert np.max(np.abs(gg - e)) <= 1e-4 * np.abs(e).max() + 1e-7, (name, np.max(np.abs(gg - e)))
    return worst


def test_decode_fn_matches_oracle():
    """DecodeFn (autograd): outputs and all 15 gradients against the FP64
    torch-autograd oracle of eq. 1-5."""
    from paper_2505_18992_amd import decode
    rng = np.random.default_rng(3)
    a = scenes.make_anchors(rng, 2000, 10)
    d = scenes.make_decoder(rng, 64, 10)
    centre = np.array([5.0, 3.0, 2.5], np.float32)
    print("case DecodeFn 2000 anchors", flush=True)
    xyz = torch.from_numpy(a.xyz).cuda()
    leaves = [torch.from_numpy(x).cuda().requires_grad_(True) for x in (a.feat, a.scale, a.offsets)]
    mlp = _dev_decoder(d)
    outs = decode((xyz, *leaves), mlp, centre)
    exp = [t.numpy() for t in odec.decode_forward(a.xyz, a.feat, a.scale, a.offsets, d.W1, d.b1, d.W2, d.b2,
                                                  centre.astype(np.float64))]
    for name, o, e in zip(KEYS, outs, exp):
        np.testing.assert_allclose(np_(o), e, rtol=1e-5, atol=1e-5 if name == "quats" else 1e-6, err_msg=name)
    up = [torch.from_numpy(np.random.default_rng(4 + j).standard_normal(tuple(o.shape)).astype(np.float32)).cuda()
          for j, o in enumerate(outs)]
    up, n_ties = _untie(up, a, d, centre)
    torch.autograd.backward(outs, up)
    print("relu near-tie anchors", n_ties, "worst norm-wise", _decode_grads_vs_oracle(a, d, centre, leaves, mlp, up),
          flush=True)


@pytest.mark.parametrize("m,img", [(4000, (320, 180)), (50_000, (1200, 680))])
def test_c3_decode_render_backward(m, img):
    """The anchor workload end to end: anchors decode to neural Gaussians,
    rendered, loss gradients on three 128x128 crops, backward through the
    render and the decode (both autograd); at a small size and at the
    workload's (50 k anchors to 500 k Gaussians, 1200x680).

    The render is checked against the oracle fed the GPU's own FP32 decoded
    Gaussians (so the standard render gates apply), and the decode backward
    against the oracle's on the same upstream gradients, for all 15 tensors."""
    from paper_2505_18992_amd import decode, render_views
    sc = scenes.make_c3(m=m, img=img)
    a, d, cam = sc.anchors, sc.decoder, sc.cameras[0]
    R = cam.world_to_cam[:, :3].astype(np.float64)
    centre = (-R.T @ cam.world_to_cam[:, 3].astype(np.float64)).astype(np.float32)
    print(f"case c3 end-to-end {m} anchors {img}", flush=True)
    xyz = torch.from_numpy(a.xyz).cuda()
    leaves = [torch.from_numpy(x).cuda().requires_grad_(True) for x in (a.feat, a.scale, a.offsets)]
    mlp = _dev_decoder(d)
    decoded = decode((xyz, *leaves), mlp, centre)
    gpu_g = scenes.GaussianSet(*[np_(t) for t in decoded])
    ref = oracle.render(gpu_g, cam, margins=MARGINS)
    mask = ref["flags"]
    keep = np.zeros((cam.height, cam.width), bool)
    rng = np.random.default_rng(303)
    for _ in range(3):
        x0, y0 = int(rng.integers(0, cam.width - 128)), int(rng.integers(0, cam.height - 128))
        keep[y0:y0 + 128, x0:x0 + 128] = True
    w = masked_weights(sc.weights[0], mask | ~keep)
    # the render's leaves: detached copies of the decoded Gaussians
    rleaves = [t.detach().clone().requires_grad_(True) for t in decoded]
    outs = render_views([tuple(rleaves)], [cam])[0]
    errs = assert_images(outs, ref, mask)
    frac = assert_mask_fraction(mask, "c3")
    print("image errors", {k: f"{e:.2e}" for k, e in errs.items()}, f"masked {frac:.3%}", flush=True)
    loss = sum((o * torch.from_numpy(x).cuda()).sum() for o, x in zip(outs, w))
    loss.backward()
    G, S = oracle.grad(gpu_g, cam, *[x.astype(np.float64) for x in w])
    got = {k: np_(t.grad) for k, t in zip(KEYS, rleaves)}
    print("render grad report", assert_grads(got, G, S), flush=True)
    up, n_ties = _untie([t.grad for t in rleaves], a, d, centre)
    torch.autograd.backward(decoded, up)
    print("relu near-tie anchors", n_ties, "decode worst norm-wise",
          _decode_grads_vs_oracle(a, d, centre, leaves, mlp, up), flush=True)
