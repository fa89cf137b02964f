"""Pins of the oracle's integer binning (CPU only): brute-force tile/box
overlap, a library lexicographic sort and a linear scan for the ranges."""
import numpy as np
import pytest

import oracle


def _random_inputs(rng, n, W, H):
    u = rng.uniform(-20, W + 20, n).astype(np.float32)
    v = rng.uniform(-20, H + 20, n).astype(np.float32)
    hx = rng.uniform(0.1, 30, n).astype(np.float32)
    hy = rng.uniform(0.1, 30, n).astype(np.float32)
    z = rng.uniform(0.3, 5.0, n).astype(np.float32)
    z[::7] = z[0]  # equal depths: ties broken by index
    valid = rng.uniform(size=n) < 0.85
    return valid, u, v, hx, hy, z.view(np.uint32)


def _brute(valid, u, v, hx, hy, zb, W, H, tw, th, tile_base, index_base):
    tiles_x, tiles_y = -(-W // tw), -(-H // th)
    px = np.arange(W) + 0.5
    py = np.arange(H) + 0.5
    trip = []
    for i in range(len(u)):
        if not valid[i]:
            continue
        # a pixel belongs to the padded box if its centre lies in
        # [u - hx - 1, u + hx + 1] x [v - hy - 1, v + hy + 1]
        inx = (px >= np.float64(u[i]) - hx[i] - 1) & (px <= np.float64(u[i]) + hx[i] + 1)
        iny = (py >= np.float64(v[i]) - hy[i] - 1) & (py <= np.float64(v[i]) + hy[i] + 1)
        for ty in range(tiles_y):
            for tx in range(tiles_x):
                if inx[tx * tw:(tx + 1) * tw].any() and iny[ty * th:(ty + 1) * th].any():
                    trip.append((tile_base + ty * tiles_x + tx, int(zb[i]), index_base + i))
    trip.sort()
    keys = np.array([(t << 32) | z for t, z, _ in trip], np.uint64)
    vals = np.array([i for _, _, i in trip], np.uint32)
    ranges = np.zeros((tiles_x * tiles_y, 2), np.uint32)
    for k, (t, _, _) in enumerate(trip):
        tl = t - tile_base
        if k == 0 or trip[k - 1][0] != t:
            ranges[tl, 0] = k
        ranges[tl, 1] = k + 1
    return keys, vals, ranges


@pytest.mark.parametrize("seed,W,H,tw,th", [(0, 64, 48, 16, 16), (1, 70, 37, 16, 16), (2, 50, 50, 8, 8),
                                             (3, 33, 65, 16, 8), (4, 1, 1, 16, 16)])
def test_binning_matches_brute_force(seed, W, H, tw, th):
    rng = np.random.default_rng(seed)
    args = _random_inputs(rng, 60, W, H)
    keys, vals, ranges = oracle.binning(*args, W, H, tw, th, tile_base=17, index_base=5)
    bk, bv, br = _brute(*args, W, H, tw, th, 17, 5)
    assert np.array_equal(keys, bk)
    assert np.array_equal(vals, bv)
    assert np.array_equal(ranges, br)


def test_binning_empty():
    e = np.zeros(0, np.float32)
    keys, vals, ranges = oracle.binning(np.zeros(0, bool), e, e, e, e, np.zeros(0, np.uint32), 32, 32, 16, 16)
    assert keys.size == 0 and vals.size == 0 and not ranges.any()
