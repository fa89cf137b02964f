"""GPU parity of the render path against the FP64 oracle (through the C ABI).

Gates (FP32 kernels vs FP64 oracle):
* projected centres and depth bits: bit-exact against the oracle's FP32
  values; conic and box extents to a relative 1e-5 of their scale;
* binning: keys, sorted values and tile ranges bit-exact against the oracle's
  integer binning fed the kernel's own per-Gaussian floats;
* images: norm-wise relative 1e-5 per plane over pixels away from a cutoff;
* gradients: per element within 1e-4 of the summation error scale.
"""
import numpy as np
import pytest
import torch

import oracle
import scenes
from gpu_util import (MARGINS, assert_grads, assert_images, assert_mask_fraction, masked_weights, np_,
                      oracle_reference, to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_18992_amd import _lib
    _lib.load()


def _render(sc, tile=(16, 16), views=None, cap=0, lds_batch=0, grid_ctas=0):
    from paper_2505_18992_amd import render
    sets = [to_dev(g.arrays()) for g in sc.sets]
    cams = sc.cameras if views is None else [sc.cameras[v] for v in views]
    vset = sc.view_set if views is None else [sc.view_set[v] for v in views]
    outs, saved = render(sets, cams, vset, tile=tile, pair_capacity=cap, lds_batch=lds_batch, grid_ctas=grid_ctas)
    torch.cuda.synchronize()
    return sets, outs, saved


def test_c1_projection_parity():
    from paper_2505_18992_amd import _lib
    sc = scenes.make_c1()
    g, cam = sc.sets[0], sc.cameras[0]
    print("case c1 projection", flush=True)
    _, outs, saved = _render(sc)
    proj = np_(saved.export(_lib.BUF_PROJ)).reshape(-1, 12)
    ext = np_(saved.export(_lib.BUF_EXTENT)).reshape(-1, 2)
    count = np_(saved.export(_lib.BUF_COUNT, torch.int32)).view(np.uint32)
    saved.close()
    p = oracle.project(g, cam)
    vis = count > 0
    assert np.array_equal(vis, p["valid"]), f"visibility differs at {np.nonzero(vis != p['valid'])[0][:10]}"
    assert vis.sum() > 500
    u, v, z = proj[vis, 0], proj[vis, 1], proj[vis, 2]
    assert np.array_equal(u.view(np.uint32), p["u32"][vis].view(np.uint32))
    assert np.array_equal(v.view(np.uint32), p["v32"][vis].view(np.uint32))
    assert np.array_equal(z.view(np.uint32), p["z32"][vis].view(np.uint32))
    qs = np.abs(p["Qa"][vis]) + np.abs(p["Qc"][vis])
    for k, col in (("Qa", 4), ("Qb", 5), ("Qc", 6)):
        err = np.abs(proj[vis, col] - p[k][vis]) / qs
        assert err.max() < 1e-5, (k, err.max())
    np.testing.assert_allclose(ext[vis, 0], p["hx"][vis], rtol=1e-5)
    np.testing.assert_allclose(ext[vis, 1], p["hy"][vis], rtol=1e-5)


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (16, 8), (32, 8)])
def test_c1_binning_bit_exact(tile):
    from paper_2505_18992_amd import _lib
    sc = scenes.make_c1()
    cam = sc.cameras[0]
    print(f"case c1 binning tile={tile}", flush=True)
    _, outs, saved = _render(sc, tile=tile)
    st = saved.stats()
    P = st["n_pairs"]
    proj = np_(saved.export(_lib.BUF_PROJ)).reshape(-1, 12)
    ext = np_(saved.export(_lib.BUF_EXTENT)).reshape(-1, 2)
    count = np_(saved.export(_lib.BUF_COUNT, torch.int32)).view(np.uint32)
    keys = np_(saved.export(_lib.BUF_KEYS, torch.int64)).view(np.uint64)[:P]
    vals = np_(saved.export(_lib.BUF_VALUES, torch.int32)).view(np.uint32)[:P]
    ranges = np_(saved.export(_lib.BUF_RANGES, torch.int32)).view(np.uint32).reshape(-1, 2)
    saved.close()
    ok = count > 0
    valid = ok.copy()
    # culled records carry no box: the oracle sees them as invalid
    ek, ev, er = oracle.binning(valid, proj[:, 0], proj[:, 1], np.where(ok, ext[:, 0], 0),
                                np.where(ok, ext[:, 1], 0), proj[:, 2].view(np.uint32), cam.width, cam.height, *tile)
    assert P == len(ek) and st["overflow"] == 0
    assert np.array_equal(keys, ek)
    assert np.array_equal(vals, ev)
    assert np.array_equal(ranges, er)


@pytest.mark.parametrize("tile", [(8, 8), (32, 8)])
def test_wide_footprint_binning_bit_exact(tile):
    """Records whose tile rectangles are tens to thousands of tiles (up to the
    whole 1200x680 view: 150 x 85 tiles of 8x8) are emitted by a whole
    wavefront, each tile's row from a float reciprocal; keys, values and
    ranges stay bit-exact against the oracle's binning."""
    from paper_2505_18992_amd import _lib
    sc = scenes.make_c1(seed=7, n=400, width=1200, height=680)
    g, cam = sc.sets[0], sc.cameras[0]
    rng = np.random.default_rng(17)
    big = rng.choice(g.n, 80, replace=False)
    # footprints from about ten pixels to beyond the view (f = 100, z in [2, 6])
    g.log_scales[big] += rng.uniform(1.0, 5.5, (80, 1)).astype(np.float32)
    print(f"case wide-footprint binning tile={tile}", flush=True)
    _, outs, saved = _render(sc, tile=tile)
    st = saved.stats()
    P = st["n_pairs"]
    proj = np_(saved.export(_lib.BUF_PROJ)).reshape(-1, 12)
    ext = np_(saved.export(_lib.BUF_EXTENT)).reshape(-1, 2)
    count = np_(saved.export(_lib.BUF_COUNT, torch.int32)).view(np.uint32)
    keys = np_(saved.export(_lib.BUF_KEYS, torch.int64)).view(np.uint64)[:P]
    vals = np_(saved.export(_lib.BUF_VALUES, torch.int32)).view(np.uint32)[:P]
    ranges = np_(saved.export(_lib.BUF_RANGES, torch.int32)).view(np.uint32).reshape(-1, 2)
    saved.close()
    ok = count > 0
    # the case reaches the wide rectangles it is about
    assert count[big[ok[big]]].max() > 2000 and int((count > 8).sum()) >= 40, (count[big].max(), (count > 8).sum())
    ek, ev, er = oracle.binning(ok.copy(), proj[:, 0], proj[:, 1], np.where(ok, ext[:, 0], 0),
                                np.where(ok, ext[:, 1], 0), proj[:, 2].view(np.uint32), cam.width, cam.height, *tile)
    assert P == len(ek) and st["overflow"] == 0
    assert np.array_equal(keys, ek)
    assert np.array_equal(vals, ev)
    assert np.array_equal(ranges, er)


@pytest.mark.parametrize("tile", [(32, 8), (16, 16)])
def test_c4_binning_bit_exact(tile):
    """The benchmark's binning: 8 keyframes at 1200x680 of the 1M-Gaussian
    corridor in one call (8 M records, about 12 M pairs), every key, value
    and tile range against the oracle's binning of each view, concatenated
    in view order (views own consecutive record and tile ranges)."""
    from paper_2505_18992_amd import _lib
    sc = scenes.make_c4(sizes=(1200, 680))
    print(f"case c4-1200 binning tile={tile}", flush=True)
    _, outs, saved = _render(sc, tile=tile)
    st = saved.stats()
    P = st["n_pairs"]
    proj = np_(saved.export(_lib.BUF_PROJ)).reshape(-1, 12)
    ext = np_(saved.export(_lib.BUF_EXTENT)).reshape(-1, 2)
    count = np_(saved.export(_lib.BUF_COUNT, torch.int32)).view(np.uint32)
    keys = np_(saved.export(_lib.BUF_KEYS, torch.int64)).view(np.uint64)[:P]
    vals = np_(saved.export(_lib.BUF_VALUES, torch.int32)).view(np.uint32)[:P]
    ranges = np_(saved.export(_lib.BUF_RANGES, torch.int32)).view(np.uint32).reshape(-1, 2)
    saved.close()
    assert st["overflow"] == 0
    n = sc.sets[0].means.shape[0]
    tw, th = tile
    rec = tb = pos = 0
    ek, ev, er = [], [], []
    for cam in sc.cameras:
        s = slice(rec, rec + n)
        ok = count[s] > 0
        k, v, r = oracle.binning(ok, proj[s, 0], proj[s, 1], np.where(ok, ext[s, 0], 0), np.where(ok, ext[s, 1], 0),
                                 proj[s, 2].view(np.uint32), cam.width, cam.height, tw, th, tile_base=tb,
                                 index_base=rec, cap=4 * int(count[s].sum()) + 1)
        ek.append(k); ev.append(v)
        er.append(np.where(r[:, 1:2] > 0, r + np.uint32(pos), 0).astype(np.uint32))
        rec += n
        tb += r.shape[0]
        pos += len(k)
    assert P == pos and ranges.shape[0] == tb
    assert np.array_equal(keys, np.concatenate(ek))
    assert np.array_equal(vals, np.concatenate(ev))
    assert np.array_equal(ranges, np.concatenate(er))


def test_c1_forward_parity():
    sc = scenes.make_c1()
    g, cam = sc.sets[0], sc.cameras[0]
    print("case c1 forward", flush=True)
    _, outs, saved = _render(sc)
    st = saved.stats()
    saved.close()
    ref, mask, _ = oracle_reference(g, cam)
    errs = assert_images(outs[0], ref, mask)
    frac = assert_mask_fraction(mask, "c1")
    print("c1 image errors", errs, f"masked {frac:.3%}", flush=True)
    # blends agree exactly on unmasked pixels
    assert abs(st["n_blended"] - int(ref["n_blend"].sum())) <= int(ref["n_blend"][mask].sum()) + 0


@pytest.fixture(scope="module")
def c1_backward_ref():
    sc = scenes.make_c1()
    _, _, (w, G, S) = oracle_reference(sc.sets[0], sc.cameras[0], sc.weights[0])
    return sc, w, G, S


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (16, 8), (32, 8)])
def test_c1_backward_parity(tile, c1_backward_ref):
    # every tile shape: 1, 2 or 4 wavefronts per tile and 1, 2 or 4 words of
    # forward hit bits per wavefront and batch
    from paper_2505_18992_amd import render_backward
    sc, w, G, S = c1_backward_ref
    print(f"case c1 backward tile={tile}", flush=True)
    _, outs, saved = _render(sc, tile=tile)
    grads, d_pose = render_backward(saved, [to_dev(w)])
    saved.close()
    got = dict(zip(["means", "log_scales", "quats", "opacities", "colors"], [np_(t) for t in grads[0]]))
    got["pose"] = np_(d_pose)[0]
    rep = assert_grads(got, G, S)
    print("c1 grad errors", rep, flush=True)


# every built (tile shape, LDS batch) pair: batches of half, once and twice
# the tile's pixels (multiples of 64), so a batch's hit masks take one to
# eight words per wavefront and a thread stages zero to two entries
BATCHES = [((16, 16), 128), ((16, 16), 512), ((16, 8), 64), ((16, 8), 256), ((8, 8), 128), ((32, 8), 128),
           ((32, 8), 512)]


@pytest.mark.parametrize("tile,nb", BATCHES)
def test_c1_backward_parity_per_lds_batch(tile, nb, c1_backward_ref):
    from paper_2505_18992_amd import render_backward
    sc, w, G, S = c1_backward_ref
    print(f"case c1 backward tile={tile} lds_batch={nb}", flush=True)
    _, outs, saved = _render(sc, tile=tile, lds_batch=nb)
    assert saved.stats()["lds_batch"] == nb
    grads, d_pose = render_backward(saved, [to_dev(w)])
    saved.close()
    got = dict(zip(["means", "log_scales", "quats", "opacities", "colors"], [np_(t) for t in grads[0]]))
    got["pose"] = np_(d_pose)[0]
    print("c1 grad errors", assert_grads(got, G, S), flush=True)


@pytest.mark.parametrize("tile,nb,grid", [((16, 16), 512, 0), ((32, 8), 128, 512), ((16, 8), 64, 1024),
                                          ((8, 8), 128, 256)])
def test_forward_is_batch_and_grid_invariant(tile, nb, grid):
    """The forward is bit-identical for every LDS batch and compositing grid
    (a 200x150 view of the room scene: lists longer than one batch)."""
    sc = scenes.make_c2(n=50_000)
    sc.cameras[0] = sc.cameras[0].copy()
    cam = sc.cameras[0]
    cam.width, cam.height, cam.cx, cam.cy = 200, 150, 100.0, 75.0
    cam.fx = cam.fy = 164.0
    print(f"case forward invariance tile={tile} lds_batch={nb} grid={grid}", flush=True)
    _, a, s1 = _render(sc)
    _, b, s2 = _render(sc, tile=tile, lds_batch=nb, grid_ctas=grid)
    st = s2.stats()
    s1.close(); s2.close()
    assert st["n_pairs"] > 20 * nb  # several batches per tile on average
    for x, y in zip(a[0], b[0]):
        assert torch.equal(x, y)


@pytest.mark.parametrize("tile", [(8, 8), (16, 8), (32, 8)])
def test_forward_is_tile_size_invariant(tile):
    sc = scenes.make_c1()
    print(f"case c1 tile invariance {tile}", flush=True)
    _, a, s1 = _render(sc)
    _, b, s2 = _render(sc, tile=tile)
    s1.close(); s2.close()
    for x, y in zip(a[0], b[0]):
        assert torch.equal(x, y)


def test_forward_deterministic():
    sc = scenes.make_c2(n=50_000)
    print("case c2-50k determinism", flush=True)
    _, a, s1 = _render(sc)
    _, b, s2 = _render(sc)
    from paper_2505_18992_amd import _lib
    k1 = s1.export(_lib.BUF_VALUES, torch.int32)
    k2 = s2.export(_lib.BUF_VALUES, torch.int32)
    s1.close(); s2.close()
    assert torch.equal(k1, k2)
    for x, y in zip(a[0], b[0]):
        assert torch.equal(x, y)


def test_forward_without_work_counters():
    """skip_counts: the same images bit for bit, evaluation and blend counts
    reported as zero, the pair list and backward unchanged."""
    from paper_2505_18992_amd import render, render_backward
    sc = scenes.make_c1()
    print("case c1 forward without counters", flush=True)
    sets = [to_dev(g.arrays()) for g in sc.sets]
    outs = []
    for count in (True, False):
        o, saved = render(sets, sc.cameras, tile=(32, 8), count=count)
        st = saved.stats()
        grads, d_pose = render_backward(saved, [to_dev(sc.weights[0])])
        saved.close()
        outs.append((o[0], st, grads[0]))
    (a, sa, ga), (b, sb, gb) = outs
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    assert sa["n_blended"] > 0 and sb["n_blended"] == 0 and sb["n_evaluated"] == 0
    assert sa["n_pairs"] == sb["n_pairs"] and sa["n_bwd_steps"] == sb["n_bwd_steps"]
    for x, y in zip(ga, gb):
        assert torch.allclose(x, y, rtol=1e-5, atol=1e-6 * float(x.abs().max()))
