"""Pins of the decode oracle (Section III-A, eq. 1-5) against closed forms
and central differences (CPU only)."""
import math

import numpy as np
import pytest

import scenes
from oracle import decode as dec


def _small(seed=0, m=6, k=3, width=8):
    rng = np.random.default_rng(seed)
    a = scenes.make_anchors(rng, m, k, size=(2.0, 2.0, 1.0))
    d = scenes.make_decoder(rng, width, k)
    return a, d, np.array([0.3, -0.4, 0.5])


def _zero_w2(d):
    return [np.zeros_like(w) for w in d.W2]


def test_means_are_anchor_plus_scaled_offsets():
    a, d, xc = _small()
    out = dec.decode_forward(a.xyz, a.feat, a.scale, a.offsets, d.W1, d.b1, d.W2, d.b2, xc)
    exp = (a.xyz.astype(np.float64)[:, None, :]
           + a.offsets.astype(np.float64) * a.scale.astype(np.float64)[:, None, :]).reshape(-1, 3)
    np.testing.assert_allclose(out[0].numpy(), exp, rtol=0, atol=1e-15)


def test_heads_with_zero_output_weights_give_activated_biases():
    a, d, xc = _small(1)
    k = d.k
    rng = np.random.default_rng(3)
    b2 = [rng.normal(size=k), rng.normal(size=3 * k), rng.normal(size=7 * k)]
    out = dec.decode_forward(a.xyz, a.feat, a.scale, a.offsets, d.W1, d.b1, _zero_w2(d), b2, xc)
    means, ls, q, o, c = (t.numpy() for t in out)
    m = a.m
    np.testing.assert_allclose(o.reshape(m, k), np.tile(np.tanh(b2[0]), (m, 1)), rtol=1e-15)
    np.testing.assert_allclose(c.reshape(m, k, 3), np.tile(1 / (1 + np.exp(-b2[1].reshape(k, 3))), (m, 1, 1)),
                               rtol=1e-14)
    cov = b2[2].reshape(k, 7)
    sig = 1 / (1 + np.exp(-cov[:, :3]))
    exp_s = sig[None] * a.scale.astype(np.float64)[:, None, :]       # eq. 5: sigmoid(F_s) * s_v
    np.testing.assert_allclose(np.exp(ls.reshape(m, k, 3)), exp_s, rtol=1e-14)
    qn = cov[:, 3:] / np.linalg.norm(cov[:, 3:], axis=1, keepdims=True)
    np.testing.assert_allclose(q.reshape(m, k, 4), np.tile(qn, (m, 1, 1)), rtol=1e-14)


def test_input_layout_distance_and_direction():
    """With the first layer picking single inputs, the heads expose the
    viewing distance (input 35) and direction (inputs 32-34) of eq. 3."""
    a, d, xc = _small(2, width=8)
    k = d.k
    W1 = [np.zeros_like(w) for w in d.W1]
    b1 = [np.zeros_like(b) for b in d.b1]
    W2 = _zero_w2(d)
    b2 = [np.zeros_like(b) for b in d.b2]
    # opacity head: hidden 0 = relu(delta); output m = hidden 0 * 0.125
    W1[0][0, 35] = 1.0
    W2[0][:, 0] = 0.125
    # colour head: hidden j = relu(d_j + 1); output (m, j) = hidden j - 1 = d_j
    for j in range(3):
        W1[1][j, 32 + j] = 1.0
        b1[1][j] = 1.0
        W2[1][np.arange(k) * 3 + j, j] = 1.0
        b2[1][np.arange(k) * 3 + j] = -1.0
    out = dec.decode_forward(a.xyz, a.feat, a.scale, a.offsets, W1, b1, W2, b2, xc)
    diff = a.xyz.astype(np.float64) - xc
    delta = np.linalg.norm(diff, axis=1)
    np.testing.assert_allclose(out[3].numpy().reshape(-1, k), np.tanh(0.125 * delta)[:, None].repeat(k, 1), rtol=1e-14)
    dirn = diff / delta[:, None]
    col = out[4].numpy().reshape(-1, k, 3)
    np.testing.assert_allclose(col, np.broadcast_to(1 / (1 + np.exp(-dirn[:, None, :])), col.shape), rtol=1e-14)


def test_zero_quaternion_head_is_floored():
    a, d, xc = _small(4)
    b2 = [b.copy() for b in d.b2]
    b2[2][:] = 0.0
    out = dec.decode_forward(a.xyz, a.feat, a.scale, a.offsets, d.W1, d.b1, _zero_w2(d), b2, xc)
    assert np.all(out[2].numpy() == 0.0)


def test_decode_backward_matches_central_differences():
    a, d, xc = _small(5, m=3, k=2, width=5)
    rng = np.random.default_rng(9)
    n = a.m * a.k
    up = [rng.normal(size=(n, 3)), rng.normal(size=(n, 3)), rng.normal(size=(n, 4)), rng.normal(size=n),
          rng.normal(size=(n, 3))]
    G = dec.decode_backward(a.xyz, a.feat, a.scale, a.offsets, d.W1, d.b1, d.W2, d.b2, xc, up)
    f64 = lambda x: x.astype(np.float64)
    P = dict(feat=f64(a.feat), scale=f64(a.scale), offsets=f64(a.offsets),
             W1=[f64(w) for w in d.W1], b1=[f64(b) for b in d.b1], W2=[f64(w) for w in d.W2],
             b2=[f64(b) for b in d.b2])

    def loss():
        out = dec.decode_forward(a.xyz, P["feat"], P["scale"], P["offsets"], P["W1"], P["b1"], P["W2"], P["b2"], xc)
        return sum(float((o.numpy() * u.reshape(o.shape)).sum()) for o, u in zip(out, up))

    def check(arr, garr, count=6):
        r = np.random.default_rng(arr.size)
        for flat in r.choice(arr.size, size=min(count, arr.size), replace=False):
            idx = np.unravel_index(flat, arr.shape)
            old = arr[idx]
            h = 1e-6 * max(1.0, abs(old))
            arr[idx] = old + h; lp = loss()
            arr[idx] = old - h; lm = loss()
            arr[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - garr[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, garr[idx])

    check(P["feat"], G["feat"])
    check(P["scale"], G["scale"])
    check(P["offsets"], G["offsets"])
    for j in range(3):
        check(P["W1"][j], G["W1"][j]); check(P["b1"][j], G["b1"][j])
        check(P["W2"][j], G["W2"][j]); check(P["b2"][j], G["b2"][j])


def test_relu_clamps_negative_preactivations():
    """The hidden layers of eq. 2 are ReLU: a unit fed -delta (negative for
    every anchor) contributes nothing and receives no gradient, and a unit
    fed delta - c is max(delta - c, 0), zero exactly on the anchors nearer
    than c.  Expected values are evaluated here in NumPy from eq. 3."""
    a, d, xc = _small(6, m=12, k=3, width=8)
    k = d.k
    W1 = [np.zeros_like(w) for w in d.W1]
    b1 = [np.zeros_like(b) for b in d.b1]
    W2 = _zero_w2(d)
    b2 = [np.zeros_like(b) for b in d.b2]
    diff = a.xyz.astype(np.float64) - xc
    delta = np.linalg.norm(diff, axis=1)
    c = float(np.float32(np.median(delta)))  # the bias array is float32
    assert (delta < c).sum() >= 3 and (delta > c).sum() >= 3
    # opacity head: hidden 0 = relu(-delta) = 0, hidden 1 = relu(delta - c)
    W1[0][0, 35] = -1.0
    W1[0][1, 35] = 1.0
    b1[0][1] = -c
    W2[0][:, 0] = 1.0
    W2[0][:, 1] = 0.5
    b2[0][:] = 0.25
    out = dec.decode_forward(a.xyz, a.feat, a.scale, a.offsets, W1, b1, W2, b2, xc)
    y = 0.25 + 0.5 * np.maximum(delta - c, 0.0)
    np.testing.assert_allclose(out[3].numpy().reshape(-1, k), np.tanh(y)[:, None].repeat(k, 1), rtol=1e-14)
    # gradients of sum(g * opacity): unit 0 is dead, unit 1 lives on delta > c
    rng = np.random.default_rng(12)
    n = a.m * k
    g_o = rng.normal(size=n)
    up = [np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 4)), g_o, np.zeros((n, 3))]
    G = dec.decode_backward(a.xyz, a.feat, a.scale, a.offsets, W1, b1, W2, b2, xc, up)
    dy = (g_o.reshape(-1, k) * (1.0 - np.tanh(y)[:, None] ** 2))    # d loss / d head output [m, k]
    live = delta > c
    assert np.all(G["W1"][0][0] == 0.0) and G["b1"][0][0] == 0.0 and np.all(G["W2"][0][:, 0] == 0.0)
    np.testing.assert_allclose(G["W2"][0][:, 1], (dy * np.maximum(delta - c, 0.0)[:, None]).sum(0), rtol=1e-12)
    np.testing.assert_allclose(G["b1"][0][1], 0.5 * dy[live].sum(), rtol=1e-12)
    np.testing.assert_allclose(G["W1"][0][1, 35], 0.5 * (dy[live] * delta[live, None]).sum(), rtol=1e-12)
    np.testing.assert_allclose(G["b2"][0], dy.sum(0), rtol=1e-12)
