"""The seeded input generators: determinism and the distributions the
workloads state (CPU only)."""
import numpy as np

import scenes


def test_c1_is_deterministic_and_matches_its_recipe():
    a = scenes.make_c1()
    b = scenes.make_c1()
    for x, y in zip(a.sets[0].arrays(), b.sets[0].arrays()):
        assert x.dtype == np.float32 and np.array_equal(x, y)
    g = a.sets[0]
    assert g.n == 1000
    assert np.all(np.abs(g.means[:, :2]) <= 1) and np.all((g.means[:, 2] >= 2) & (g.means[:, 2] <= 6))
    assert abs(g.log_scales.mean() + 3) < 0.05 and abs(g.log_scales.std() - 0.5) < 0.03
    np.testing.assert_allclose(np.linalg.norm(g.quats, axis=1), 1, rtol=1e-6)
    assert abs(g.opacities.mean() - 0.5) < 0.03
    cam = a.cameras[0]
    assert (cam.width, cam.height, cam.fx, cam.cx, cam.cy) == (128, 96, 100.0, 64.0, 48.0)
    assert np.array_equal(cam.world_to_cam, np.eye(3, 4, dtype=np.float32))
    gr, gd, ga = a.weights[0]
    assert gr.shape == (3, 96, 128) and abs(gr.std() - 1) < 0.02


def test_c2_room():
    sc = scenes.make_c2(n=20000)
    g = sc.sets[0]
    inside = np.all((g.means >= -1e-4) & (g.means <= np.array([6, 5, 3]) + 1e-4), axis=1)
    assert inside.mean() > 0.97   # the six faces bound the room; a few rectangles poke through
    assert abs(g.log_scales.mean() + 4) < 0.05
    cam = sc.cameras[0]
    R = cam.world_to_cam[:, :3].astype(np.float64)
    np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-6)
    centre = -R.T @ cam.world_to_cam[:, 3]
    assert np.all(centre > 0.49) and np.all(centre < np.array([5.51, 4.51, 2.51]))


def test_c3_anchors_unique_voxels():
    sc = scenes.make_c3(m=2000)
    a = sc.anchors
    keys = np.floor(a.xyz / 0.1 + 1e-3).astype(np.int64)
    assert np.unique(keys, axis=0).shape[0] == 2000
    assert a.offsets.shape == (2000, 10, 3) and a.feat.shape == (2000, 32)
    assert sc.decoder.width == 64 and sc.decoder.W2[2].shape == (70, 64)


def test_c4_c5_shapes():
    sc = scenes.make_c4(n=5000, weights=False)
    assert len(sc.cameras) == 8 and all((c.width, c.height) in scenes.C4_SIZES for c in sc.cameras)
    sc5 = scenes.make_c5(n_per=3000, weights=False)
    assert len(sc5.sets) == 4 and len(sc5.cameras) == 16 and sc5.view_set == [j for j in range(4) for _ in range(4)]
    assert all((c.width, c.height, c.fx) == (1242, 375, 720.0) for c in sc5.cameras)
