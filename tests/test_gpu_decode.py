"""GPU parity of the anchor decode (Section III-A, eq. 1-5) against the FP64
oracle (its autograd Function and the chain through the render are in
test_gpu_autograd.py)."""
import numpy as np
import pytest
import torch

import scenes
from gpu_util import np_, to_dev
from oracle import decode as odec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _case(seed, m, k, width):
    rng = np.random.default_rng(seed)
    # the scene's surfaces hold about 40 000 voxels of 10 cm: finer for more anchors
    a = scenes.make_anchors(rng, m, k, voxel=0.1 if m <= 30_000 else 0.03)
    d = scenes.make_decoder(rng, width, k)
    cam = np.array([6.0, 4.0, 2.0]) + rng.normal(0, 1.0, 3)
    return a, d, cam.astype(np.float32)


def _dev_inputs(a, d):
    anchors = to_dev((a.xyz, a.feat, a.scale, a.offsets))
    mlp = tuple([torch.from_numpy(x).cuda() for x in lst] for lst in (d.W1, d.b1, d.W2, d.b2))
    return anchors, mlp


def _untie(up, a, d, cam):
    """Zero the upstream rows of anchors whose ReLU decision is a near tie
    (both sides then produce exactly zero for them)."""
    flags = odec.relu_near_ties(a.xyz, a.feat, a.scale, a.offsets, d.W1, d.b1, d.W2, d.b2, cam.astype(np.float64))
    rows = np.repeat(flags, a.k)
    out = []
    for u in up:
        u = np.array(u, np.float32, copy=True)
        u[rows] = 0.0
        out.append(u)
    return out, int(flags.sum())


@pytest.mark.parametrize("m,k,width", [(3000, 10, 64), (1000, 10, 32), (777, 3, 50), (1, 16, 128), (500, 1, 8)])
def test_decode_forward_parity(m, k, width):
    from paper_2505_18992_amd import decode_forward
    print(f"case decode forward m={m} k={k} width={width}", flush=True)
    a, d, cam = _case(m + k, m, k, width)
    anchors, mlp = _dev_inputs(a, d)
    got = [np_(t) for t in decode_forward(anchors, mlp, cam)]
    exp = [t.numpy() for t in odec.decode_forward(a.xyz, a.feat, a.scale, a.offsets, d.W1, d.b1, d.W2, d.b2,
                                                  cam.astype(np.float64))]
    for name, g, e in zip(["means", "log_scales", "quats", "opacities", "colors"], got, exp):
        # a normalised quaternion's components err relative to the unit norm
        np.testing.assert_allclose(g, e, rtol=1e-5, atol=1e-5 if name == "quats" else 1e-6, err_msg=name)


# 140 000 anchors: more blocks of 64 than one launch of the backward takes,
# so the weight gradients add the partial sums of several launches
@pytest.mark.parametrize("m,k,width", [(3000, 10, 64), (1000, 10, 32), (777, 3, 50), (1, 16, 128), (500, 1, 8),
                                       (140_000, 10, 64)])
def test_decode_backward_parity(m, k, width):
    from paper_2505_18992_amd import decode_backward
    print(f"case decode backward m={m} k={k} width={width}", flush=True)
    a, d, cam = _case(7 * m + k, m, k, width)
    anchors, mlp = _dev_inputs(a, d)
    rng = np.random.default_rng(5)
    n = m * k
    up = [rng.standard_normal((n, 3)).astype(np.float32), rng.standard_normal((n, 3)).astype(np.float32),
          rng.standard_normal((n, 4)).astype(np.float32), rng.standard_normal(n).astype(np.float32),
          rng.standard_normal((n, 3)).astype(np.float32)]
    up, n_ties = _untie(up, a, d, cam)
    print("relu near-tie anchors", n_ties, flush=True)
    d_feat, d_scale, d_off, (dW1, db1, dW2, db2) = decode_backward(anchors, mlp, cam, to_dev(up))
    G = odec.decode_backward(a.xyz, a.feat, a.scale, a.offsets, d.W1, d.b1, d.W2, d.b2, cam.astype(np.float64), up)
    pairs = [("feat", d_feat, G["feat"]), ("scale", d_scale, G["scale"]), ("offsets", d_off, G["offsets"])]
    for h in range(3):
        pairs += [(f"W1[{h}]", dW1[h], G["W1"][h]), (f"b1[{h}]", db1[h], G["b1"][h]),
                  (f"W2[{h}]", dW2[h], G["W2"][h]), (f"b2[{h}]", db2[h], G["b2"][h])]
    for name, g, e in pairs:
        g = np_(g).astype(np.float64)
        nrm = np.linalg.norm(g - e) / max(np.linalg.norm(e), 1e-30)
        assert nrm <= 1e-5, (name, nrm)
        # per element against the tensor's largest magnitude (sums of many signed terms)
        assert np.max(np.abs(g - e)) <= 1e-4 * np.abs(e).max() + 1e-7, (name, np.max(np.abs(g - e)))


def test_decode_empty():
    """No anchors: nothing is decoded and every weight and bias gradient comes
    back zero."""
    from paper_2505_18992_amd import decode_backward, decode_forward
    print("case decode empty", flush=True)
    a, d, cam = _case(11, 4, 10, 64)
    anchors, mlp = _dev_inputs(a, d)
    empty = tuple(t[:0] for t in anchors)
    outs = decode_forward(empty, mlp, cam)
    assert all(o.shape[0] == 0 for o in outs)
    d_feat, d_scale, d_off, grads = decode_backward(empty, mlp, cam, [torch.zeros_like(o) for o in outs])
    assert d_feat.shape[0] == 0 and d_scale.shape[0] == 0 and d_off.shape[0] == 0
    for lst in grads:
        for g in lst:
            assert g.numel() > 0 and int(torch.count_nonzero(g)) == 0
