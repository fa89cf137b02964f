"""Edge cases, argument validation, capacity overflow and batching of the
GPU render path (through the C ABI)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import scenes
from gpu_util import assert_grads, assert_images, np_, oracle_reference, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _gs(means, ls, quats, opac, cols):
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return scenes.GaussianSet(f(means), f(ls), f(quats), f(opac), f(cols))


def test_empty_set_renders_background_and_zero_gradients():
    from paper_2505_18992_amd import render, render_backward
    cam = scenes.identity_camera(40, 30, 50.0, 50.0, 20.0, 15.0)
    e = torch.zeros((0, 3), device="cuda")
    s = (e, e.clone(), torch.zeros((0, 4), device="cuda"), torch.zeros((0,), device="cuda"), e.clone())
    outs, saved = render([s], [cam])
    for t in outs[0]:
        assert torch.count_nonzero(t) == 0
    w = scenes.upstream_weights(1, [cam])[0]
    grads, d_pose = render_backward(saved, [to_dev(w)])
    st = saved.stats()
    saved.close()
    assert st["n_pairs"] == 0 and st["n_blended"] == 0
    assert all(t.numel() == 0 for t in grads[0])
    assert torch.count_nonzero(d_pose) == 0


def test_all_culled():
    from paper_2505_18992_amd import render
    sc = scenes.make_c1(n=200)
    g = sc.sets[0]
    g.means[:, 2] = -1.0  # behind the camera
    outs, saved = render([to_dev(g.arrays())], sc.cameras)
    st = saved.stats()
    saved.close()
    assert st["n_pairs"] == 0
    for t in outs[0]:
        assert torch.count_nonzero(t) == 0


def test_degenerate_gaussians_are_culled_like_the_oracle():
    from paper_2505_18992_amd import render, render_backward
    sc = scenes.make_c1(n=400, width=37, height=23)   # ragged: not a multiple of the tile size
    sc.cameras[0].cx, sc.cameras[0].cy = 18.5, 11.5
    sc.cameras[0].fx = sc.cameras[0].fy = 30.0
    g = sc.sets[0]
    g.quats[0:10] = 0.0                       # zero quaternion
    g.opacities[10:20] = 1.0 / 255.0          # at the opacity cutoff
    g.opacities[20:25] = 0.0
    g.means[25:30, 2] = 0.2                   # at the near plane
    g.means[30:35, 2] = 0.15                  # in front of the near plane
    g.log_scales[35:40] = -30.0               # vanishing scale: only the 0.3 px dilation remains
    g.log_scales[40:42] = 8.0                 # huge (kilometres)
    w = scenes.upstream_weights(3, sc.cameras)[0]
    ref, mask, (wm, G, S) = oracle_reference(g, sc.cameras[0], w)
    outs, saved = render([to_dev(g.arrays())], sc.cameras)
    assert_images(outs[0], ref, mask)
    grads, d_pose = render_backward(saved, [to_dev(wm)])
    saved.close()
    got = dict(zip(["means", "log_scales", "quats", "opacities", "colors"], [np_(t) for t in grads[0]]))
    got["pose"] = np_(d_pose)[0]
    assert_grads(got, G, S)
    for k in got:
        assert np.all(np.isfinite(got[k]))


def test_capacity_overflow_is_reported():
    from paper_2505_18992_amd import _lib, render
    sc = scenes.make_c1()
    outs, saved = render([to_dev(sc.sets[0].arrays())], sc.cameras, pair_capacity=100)
    st = saved.stats()
    saved.close()
    assert st["overflow"] == 1 and st["n_pairs"] > 100 and st["pair_capacity"] == 100
    # a larger capacity on the same context works again
    outs2, saved2 = render([to_dev(sc.sets[0].arrays())], sc.cameras, pair_capacity=st["n_pairs"])
    st2 = saved2.stats()
    saved2.close()
    assert st2["overflow"] == 0


def test_invalid_arguments_are_rejected():
    from paper_2505_18992_amd import _lib, camera_struct, get_context, render
    from paper_2505_18992_amd._lib import VpgsError
    sc = scenes.make_c1(n=50)
    t = to_dev(sc.sets[0].arrays())
    cam = sc.cameras[0]
    bad = cam.copy(); bad.width = 0
    with pytest.raises(VpgsError) as e:
        render([t], [bad])
    assert e.value.status == _lib.VPGS_EINVAL
    bad = cam.copy(); bad.fx = float("nan")
    with pytest.raises(VpgsError):
        render([t], [bad])
    bad = cam.copy(); bad.world_to_cam = bad.world_to_cam.copy(); bad.world_to_cam[0, 3] = float("inf")
    with pytest.raises(VpgsError):
        render([t], [bad])
    with pytest.raises(VpgsError) as e:
        render([t], [cam], tile=(12, 12))
    assert e.value.status == _lib.VPGS_EUNSUPPORTED
    for nb in (96, 1024, 32):  # not a multiple of 64, or not half/once/twice 256 pixels
        with pytest.raises(VpgsError) as e:
            render([t], [cam], tile=(16, 16), lds_batch=nb)
        assert e.value.status == _lib.VPGS_EUNSUPPORTED
    with pytest.raises(VpgsError) as e:
        render([t], [cam], grid_ctas=-1)
    assert e.value.status == _lib.VPGS_EINVAL
    with pytest.raises(VpgsError):
        render([t], [cam], view_set=[1])
    # misaligned quaternions
    q = torch.zeros(51 * 4 + 1, device="cuda")[1:].view(51, 4)[:50]
    with pytest.raises(VpgsError):
        render([(t[0], t[1], q, t[3], t[4])], [cam])
    # NULL planes straight through the ABI
    L = _lib.load()
    ctx = get_context()
    gs = (_lib.Gaussians * 1)()
    gs[0].n = 50
    cams = (_lib.Camera * 1)(camera_struct(cam))
    ims = (_lib.Images * 1)()
    vs = (ctypes.c_int32 * 1)(0)
    assert L.vpgs_render_forward(ctx.handle, 1, gs, 1, vs, cams, ims, None, None, None) == _lib.VPGS_EINVAL
    gs[0].n = -1
    assert L.vpgs_render_forward(ctx.handle, 1, gs, 1, vs, cams, ims, None, None, None) == _lib.VPGS_EINVAL
    assert b"n = -1" in L.vpgs_last_error(ctx.handle)


def test_batched_views_equal_per_view_calls():
    """Views of mixed resolution rendered in one call equal one-view calls bit
    for bit; the set gradient is the sum of the per-view gradients."""
    from paper_2505_18992_amd import render, render_backward
    sc = scenes.make_c4(n=30_000, views=5)
    sets = [to_dev(g.arrays()) for g in sc.sets]
    gw = [to_dev(w) for w in sc.weights]
    outs, saved = render(sets, sc.cameras, sc.view_set)
    grads, d_pose = render_backward(saved, gw)
    saved.close()
    acc = [torch.zeros_like(t) for t in grads[0]]
    for v, cam in enumerate(sc.cameras):
        o1, s1 = render(sets, [cam], [0])
        for a, b in zip(outs[v], o1[0]):
            assert torch.equal(a, b)
        g1, p1 = render_backward(s1, [gw[v]])
        s1.close()
        for k in range(5):
            acc[k] += g1[0][k]
        torch.testing.assert_close(d_pose[v], p1[0], rtol=1e-4, atol=1e-3 * float(p1.abs().max()) + 1e-6)
    for k in range(5):
        scale = float(acc[k].abs().max()) + 1e-12
        assert float((grads[0][k] - acc[k]).abs().max()) <= 1e-4 * scale


def test_multiple_sets_in_one_call():
    from paper_2505_18992_amd import render, render_backward
    sc = scenes.make_c5(n_per=20_000, views_per=2)
    sets = [to_dev(g.arrays()) for g in sc.sets]
    gw = [to_dev(w) for w in sc.weights]
    outs, saved = render(sets, sc.cameras, sc.view_set)
    grads, _ = render_backward(saved, gw)
    saved.close()
    for v in (0, 5):
        s = sc.view_set[v]
        o1, s1 = render([sets[s]], [sc.cameras[v]])
        s1.close()
        for a, b in zip(outs[v], o1[0]):
            assert torch.equal(a, b)
    # view 2 against the oracle (its own set)
    v = 2
    g, cam = sc.sets[sc.view_set[v]], sc.cameras[v]
    ref, mask, _ = oracle_reference(g, cam)
    assert_images(outs[v], ref, mask)


def test_workspace_comes_from_the_torch_allocator():
    """The default context hands the library torch's caching allocator
    (vpgs_create's callbacks): the workspace of a render is held as torch
    blocks, and a context on hipMalloc renders the same images bit for bit."""
    from paper_2505_18992_amd import render
    from paper_2505_18992_amd.render import Context
    sc = scenes.make_c1()
    print("case torch-backed workspace", flush=True)
    ctx = Context(0)
    outs, saved = render([to_dev(sc.sets[0].arrays())], sc.cameras, ctx=ctx)
    saved.close()
    held = ctx.workspace.bytes_held()
    assert held > 0 and all(t.is_cuda for t in ctx.workspace.blocks.values())
    hip_ctx = Context(0, torch_workspace=False)
    assert hip_ctx.workspace is None
    outs2, saved2 = render([to_dev(sc.sets[0].arrays())], sc.cameras, ctx=hip_ctx)
    saved2.close()
    for a, b in zip(outs[0], outs2[0]):
        assert torch.equal(a, b)
    ctx.close()
    assert ctx.workspace.bytes_held() == 0  # every block was handed back
    hip_ctx.close()


def test_workspace_allocator_failure_is_reported():
    """An allocator callback that returns NULL makes the call fail with
    VPGS_ENOMEM and nothing enqueued; the context stays usable once the
    allocator succeeds again."""
    from paper_2505_18992_amd import render
    from paper_2505_18992_amd._lib import VpgsError
    from paper_2505_18992_amd.render import Context
    sc = scenes.make_c1(n=100)
    print("case allocator failure", flush=True)
    ctx = Context(0)
    real = ctx.workspace._alloc
    ctx.workspace._alloc = lambda n, u: None
    with pytest.raises(VpgsError) as e:
        render([to_dev(sc.sets[0].arrays())], sc.cameras, ctx=ctx)
    assert e.value.status == -2  # VPGS_ENOMEM
    ctx.workspace._alloc = real
    outs, saved = render([to_dev(sc.sets[0].arrays())], sc.cameras, ctx=ctx)
    saved.close()
    assert torch.count_nonzero(outs[0][2]) > 0
    ctx.close()
