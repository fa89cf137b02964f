"""Anchor -> neural-Gaussian decode in plain PyTorch CPU float64 -- TEST INFRASTRUCTURE.

Section III-A of the paper, written out step by step:

* eq. 1  means of the k Gaussians of an anchor: x_a + O_m * l (elementwise);
* eq. 3  viewing distance delta = |x_a - x_c| and direction d = (x_a - x_c)/delta;
* eq. 2  the input {f, delta, d} goes through three individual LINEAR-ReLU-LINEAR
         heads (opacity, colour, covariance); the input vector is laid out as
         [f (32), d (3), delta (1)];
* opacity is tanh of its head (values <= 0 are the invalid samples the
  renderer culls);
* eq. 4  colour = sigmoid of its head, k x 3;
* eq. 5  scale = sigmoid(head) * l, passed on as a log-scale
         log_sigmoid(head) + log l; rotation = the head's 4-vector normalised
         (norm floored at 1e-12).  The covariance head emits [scale(3) | quat(4)]
         per Gaussian.

The backward is torch autograd of this forward.  The camera centre is a
constant of the decode.
"""
from __future__ import annotations

import torch

__all__ = ["decode_forward", "decode_backward", "relu_near_ties"]


def _t(a):
    return torch.as_tensor(a).to(torch.float64)


def decode_forward(xyz, feat, scale, offsets, W1, b1, W2, b2, cam_center):
    """Returns (means, log_scales, quats, opacities, colors), each flattened over
    (anchor, k) in anchor-major order."""
    xyz, feat, scale, offsets = _t(xyz), _t(feat), _t(scale), _t(offsets)
    W1 = [_t(w) for w in W1]; b1 = [_t(b) for b in b1]
    W2 = [_t(w) for w in W2]; b2 = [_t(b) for b in b2]
    xc = _t(cam_center).reshape(1, 3)
    m, k = offsets.shape[0], offsets.shape[1]
    diff = xyz - xc
    delta = torch.linalg.norm(diff, dim=1, keepdim=True)
    d = diff / delta
    h = torch.cat([feat, d, delta], dim=1)
    y = [torch.relu(h @ W1[j].T + b1[j]) @ W2[j].T + b2[j] for j in range(3)]
    opac = torch.tanh(y[0])
    col = torch.sigmoid(y[1].reshape(m, k, 3))
    cov = y[2].reshape(m, k, 7)
    log_scales = torch.nn.functional.logsigmoid(cov[..., :3]) + torch.log(scale)[:, None, :]
    yq = cov[..., 3:]
    quats = yq / torch.clamp(torch.linalg.norm(yq, dim=-1, keepdim=True), min=1e-12)
    means = xyz[:, None, :] + offsets * scale[:, None, :]
    return (means.reshape(m * k, 3), log_scales.reshape(m * k, 3), quats.reshape(m * k, 4),
            opac.reshape(m * k), col.reshape(m * k, 3))


def decode_backward(xyz, feat, scale, offsets, W1, b1, W2, b2, cam_center, upstream):
    """Gradient of sum(upstream . outputs) w.r.t. feat, scale, offsets and the
    weights.  ``upstream`` = (g_means, g_log_scales, g_quats, g_opac, g_colors).
    Returns a dict of float64 numpy arrays."""
    feat = _t(feat).requires_grad_(True)
    scale = _t(scale).requires_grad_(True)
    offsets = _t(offsets).requires_grad_(True)
    W1 = [_t(w).requires_grad_(True) for w in W1]
    b1 = [_t(b).requires_grad_(True) for b in b1]
    W2 = [_t(w).requires_grad_(True) for w in W2]
    b2 = [_t(b).requires_grad_(True) for b in b2]
    outs = decode_forward(xyz, feat, scale, offsets, W1, b1, W2, b2, cam_center)
    loss = sum((o * _t(g).reshape(o.shape)).sum() for o, g in zip(outs, upstream))
    loss.backward()
    n = lambda t: t.grad.detach().numpy().copy()
    return dict(feat=n(feat), scale=n(scale), offsets=n(offsets),
                W1=[n(w) for w in W1], b1=[n(b) for b in b1],
                W2=[n(w) for w in W2], b2=[n(b) for b in b2])


def relu_near_ties(xyz, feat, scale, offsets, W1, b1, W2, b2, cam_center, margin=1e-5):
    """Anchors with a hidden pre-activation within ``margin`` (relative to the
    sum of the magnitudes of its terms) of zero: there a float32 evaluation
    may take the other side of the ReLU, whose derivative jumps."""
    xyz, feat = _t(xyz), _t(feat)
    xc = _t(cam_center).reshape(1, 3)
    diff = xyz - xc
    delta = torch.linalg.norm(diff, dim=1, keepdim=True)
    h = torch.cat([feat, diff / delta, delta], dim=1)
    flag = torch.zeros(h.shape[0], dtype=torch.bool)
    for j in range(3):
        W, b = _t(W1[j]), _t(b1[j])
        pre = h @ W.T + b
        mag = h.abs() @ W.abs().T + b.abs()
        flag |= (pre.abs() <= margin * mag).any(dim=1)
    return flag.numpy()
