"""GPU parity of the voxel map and the frame-to-map registration (eq. 10-12)
against the oracle, through the C ABI.

Gates: downsampled indices, occupied-voxel counts, correspondences and
their squared distances bit-exact (FP32 decisions in the same operation
order on both sides); the Gauss-Newton terms within 1e-5 of the sum of
their terms' magnitudes (FP32 terms and workgroup sums, FP64 across
workgroups), the count exact; the registered pose within 1e-6 (rotation)
and 1e-5 m of the oracle's, with the same number of steps.
"""
import numpy as np
import pytest
import torch

import scenes
from oracle import icp

pytestmark = pytest.mark.gpu

TAU, SIGMA, VOXEL, CAP = 3.0, 1.0, 1.0, 20


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_18992_amd import _lib
    _lib.load()


@pytest.fixture(scope="module")
def street():
    sc = scenes.make_street_scan(n_map=300_000)
    return sc, icp.VoxelMap(sc.map_points, VOXEL, CAP)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def _source(sc):
    a = icp.downsample(sc.scan, 0.5 * VOXEL)
    b = a[icp.downsample(sc.scan[a], 1.5 * VOXEL)]
    return sc.scan[b]


@pytest.mark.parametrize("voxel", [0.5, 1.5, 0.07])
def test_downsample_bit_exact(street, voxel):
    from paper_2505_18992_amd import voxel_downsample
    sc, _ = street
    print(f"case downsample voxel={voxel}", flush=True)
    got = voxel_downsample(_dev(sc.scan), voxel).cpu().numpy()
    assert np.array_equal(got, icp.downsample(sc.scan, voxel))


def test_downsample_edges():
    from paper_2505_18992_amd import voxel_downsample
    one = np.array([[0.3, -0.2, 5.0]], np.float32)
    assert voxel_downsample(_dev(one), 1.0).tolist() == [0]
    same = np.tile(np.float32([[1.2, 1.3, 1.4]]), (1000, 1))
    assert voxel_downsample(_dev(same), 0.1).tolist() == [0]
    assert voxel_downsample(torch.zeros((0, 3), device="cuda"), 1.0).numel() == 0


def test_map_and_correspondences_bit_exact(street):
    from paper_2505_18992_amd import VoxelMap, icp_correspond
    sc, vm = street
    print("case voxel map 300k + correspondences", flush=True)
    gm = VoxelMap(_dev(sc.map_points), VOXEL, CAP)
    n, nvox = gm.info()
    assert n == sc.map_points.shape[0] and nvox == len(vm.cells)
    rng = np.random.default_rng(3)
    src = sc.scan[rng.choice(sc.scan.shape[0], 6000, replace=False)]
    for pose in (sc.pose_gt, sc.pose_init):
        nn, d2 = icp_correspond(gm, _dev(src), pose, TAU)
        enn, ed2 = icp.correspond(vm, icp.transform32(src, pose), TAU)
        assert np.array_equal(nn.cpu().numpy(), enn)
        assert np.array_equal(d2.cpu().numpy().view(np.uint32), ed2.view(np.uint32))
        assert (enn >= 0).mean() > 0.5
    gm.close()


def test_lane_group_widths_agree(street):
    # few queries search a voxel per lane, many search all 27 in one lane:
    # 20 k queries (8 lanes each) against the oracle; 131 k (4 lanes) and
    # 392 k (1 lane) against the same queries taken 10 k at a time (32 lanes)
    from paper_2505_18992_amd import VoxelMap, icp_correspond
    sc, vm = street
    print("case lane-group widths", flush=True)
    gm = VoxelMap(_dev(sc.map_points), VOXEL, CAP)
    rng = np.random.default_rng(5)
    src = sc.scan[rng.choice(sc.scan.shape[0], 20000, replace=False)]
    nn, d2 = icp_correspond(gm, _dev(src), sc.pose_init, TAU)
    enn, ed2 = icp.correspond(vm, icp.transform32(src, sc.pose_init), TAU)
    assert np.array_equal(nn.cpu().numpy(), enn) and np.array_equal(d2.cpu().numpy(), ed2)
    for big in (sc.scan, np.concatenate([sc.scan, sc.scan + 0.01, sc.scan - 0.02])):
        nn, d2 = icp_correspond(gm, _dev(big), sc.pose_init, TAU)
        parts = [icp_correspond(gm, _dev(big[k:k + 10000]), sc.pose_init, TAU) for k in range(0, len(big), 10000)]
        assert torch.equal(nn, torch.cat([p[0] for p in parts])) and torch.equal(d2, torch.cat([p[1] for p in parts]))
    gm.close()


def test_correspondence_ties_bit_exact():
    # dyadic map and query coordinates make many squared distances exactly
    # equal: the nearest point is then the lowest index, within a voxel's
    # run (runs of 3, 5, 7 and 20 points, the last capped) and across
    # neighbouring voxels; duplicated points (higher indices) never win
    from paper_2505_18992_amd import VoxelMap, icp_correspond
    print("case correspondence ties", flush=True)
    g = np.arange(0.0, 2.0, 0.25, dtype=np.float32)
    lattice = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    rng = np.random.default_rng(11)
    keep = np.concatenate([lattice[:: 7], lattice[3::11], lattice[rng.choice(len(lattice), 60, replace=False)]])
    pts = np.concatenate([keep, keep[::-1][:40], lattice[lattice[:, 0] >= 1.5]])  # duplicates come later
    q = np.arange(-0.75, 2.75, 0.125, dtype=np.float32)
    qs = np.stack(np.meshgrid(q, q, q, indexing="ij"), -1).reshape(-1, 3)
    for cap in (3, 5, 7, 20):
        vm = icp.VoxelMap(pts, VOXEL, cap)
        gm = VoxelMap(_dev(pts), VOXEL, cap)
        assert gm.info() == (pts.shape[0], len(vm.cells))
        nn, d2 = icp_correspond(gm, _dev(qs), np.eye(3, 4), TAU)
        enn, ed2 = icp.correspond(vm, icp.transform32(qs, np.eye(3, 4)), TAU)
        assert np.array_equal(nn.cpu().numpy(), enn), f"cap {cap}"
        assert np.array_equal(d2.cpu().numpy().view(np.uint32), ed2.view(np.uint32)), f"cap {cap}"
        # fewer queries (a voxel per lane) and the same queries many times
        # over (four lanes per query) give the same answers
        ns, ds = icp_correspond(gm, _dev(qs[:9000]), np.eye(3, 4), TAU)
        assert np.array_equal(ns.cpu().numpy(), enn[:9000]) and np.array_equal(ds.cpu().numpy(), ed2[:9000])
        big = np.tile(qs, (7, 1))
        nb, db = icp_correspond(gm, _dev(big), np.eye(3, 4), TAU)
        assert np.array_equal(nb.cpu().numpy(), np.tile(enn, 7)) and np.array_equal(db.cpu().numpy(), np.tile(ed2, 7))
        gm.close()


@pytest.mark.parametrize("n", [1000, 1025, 65536, 65537, 1048577])
def test_map_sizes_across_sort_paths(n):
    # the map build sorts n voxel keys: sizes on both sides of the sort's
    # switches (one workgroup, 64 workgroups with the digit offsets formed in
    # the scatter, more with the offsets kernel, and above 1 M keys the
    # larger workgroups); a dense cluster makes long runs of one key and
    # capped voxels
    from paper_2505_18992_amd import VoxelMap, icp_correspond
    print(f"case map size {n}", flush=True)
    rng = np.random.default_rng(n)
    k = n // 4
    pts = np.concatenate([rng.uniform(-30, 30, (n - k, 3)), rng.normal(0, 0.6, (k, 3))]).astype(np.float32)
    rng.shuffle(pts)
    vm = icp.VoxelMap(pts, VOXEL, CAP)
    gm = VoxelMap(_dev(pts), VOXEL, CAP)
    assert gm.info() == (n, len(vm.cells))
    q = rng.uniform(-31, 31, (3000, 3)).astype(np.float32)
    q[:1000] = rng.normal(0, 0.8, (1000, 3))
    nn, d2 = icp_correspond(gm, _dev(q), np.eye(3, 4), TAU)
    enn, ed2 = icp.correspond(vm, icp.transform32(q, np.eye(3, 4)), TAU)
    assert np.array_equal(nn.cpu().numpy(), enn)
    assert np.array_equal(d2.cpu().numpy().view(np.uint32), ed2.view(np.uint32))
    gm.close()


def test_cap_and_empty_map():
    from paper_2505_18992_amd import VoxelMap, icp_correspond
    m = np.array([[0.1, 0.1, 0.1], [0.5, 0.5, 0.5], [0.9, 0.2, 0.3]], np.float32)
    gm = VoxelMap(_dev(m), 1.0, 1)
    nn, _ = icp_correspond(gm, _dev(np.array([[0.49, 0.5, 0.5]], np.float32)), np.eye(3, 4), 2.0)
    assert nn.tolist() == [0]
    gm.close()
    em = VoxelMap(torch.zeros((0, 3), device="cuda"), 1.0, 5)
    nn, d2 = icp_correspond(em, _dev(m), np.eye(3, 4), 2.0)
    assert nn.tolist() == [-1, -1, -1] and bool(torch.isinf(d2).all())
    assert em.info() == (0, 0)
    em.close()


def _scales(p, m, sigma):
    """Sum of the magnitudes of each Gauss-Newton term (float64)."""
    r = p - m
    w = icp.gm_weight(np.einsum("ij,ij->i", r, r), sigma)
    sH, sg = np.zeros(21), np.zeros(6)
    for i in range(p.shape[0]):
        J = np.abs(np.concatenate([np.eye(3), -icp._skew(p[i])], axis=1))
        H = w[i] * J.T @ J
        sH += H[np.triu_indices(6)]
        sg += w[i] * J.T @ np.abs(r[i])
    return sH, sg


def test_linearize_terms(street):
    from paper_2505_18992_amd import VoxelMap, icp_linearize
    sc, vm = street
    print("case linearize", flush=True)
    gm = VoxelMap(_dev(sc.map_points), VOXEL, CAP)
    rng = np.random.default_rng(4)
    src = sc.scan[rng.choice(sc.scan.shape[0], 3000, replace=False)]
    got = icp_linearize(gm, _dev(src), sc.pose_init, TAU, SIGMA).cpu().numpy()
    q = icp.transform32(src, sc.pose_init)
    nn, _ = icp.correspond(vm, q, TAU)
    ok = nn >= 0
    p64, m64 = q[ok].astype(np.float64), vm.points[nn[ok]].astype(np.float64)
    H, g, cnt, rho = icp.normal_equations(p64, m64, SIGMA)
    sH, sg = _scales(p64, m64, SIGMA)
    assert got[27] == cnt
    assert np.all(np.abs(got[:21] - H[np.triu_indices(6)]) <= 1e-5 * sH)
    assert np.all(np.abs(got[21:27] - g) <= 1e-5 * sg)
    assert abs(got[28] - rho) <= 1e-5 * rho
    gm.close()


def _rot_err(A, B):
    R = A[:, :3] @ B[:, :3].T
    return float(np.arccos(np.clip((np.trace(R) - 1) / 2, -1, 1)))


def test_register_matches_oracle(street):
    from paper_2505_18992_amd import VoxelMap, icp_register
    sc, vm = street
    print("case register (double-downsampled scan)", flush=True)
    gm = VoxelMap(_dev(sc.map_points), VOXEL, CAP)
    src = _source(sc)
    pose, res = icp_register(gm, _dev(src), sc.pose_init, None, TAU, SIGMA, 100, 1e-4)
    ref = icp.register(vm, src, sc.pose_init, TAU, SIGMA, 100, 1e-4)
    assert res["converged"] == ref["converged"] == 1 and res["degenerate"] == 0
    assert res["iterations"] == ref["iterations"] and res["count"] == ref["count"]
    assert _rot_err(pose, ref["pose"]) < 1e-6 and np.abs(pose[:, 3] - ref["pose"][:, 3]).max() < 1e-5
    # and it moves the 2 degree / 0.58 m initial error to a few hundredths of
    # either (514 points after double downsampling, 20 points per voxel)
    assert _rot_err(sc.pose_init, sc.pose_gt) > 0.03
    assert _rot_err(pose, sc.pose_gt) < 5e-3 and np.abs(pose[:, 3] - sc.pose_gt[:, 3]).max() < 0.05
    # eq. 10: prev * pred composes on the host
    prev = np.concatenate([np.eye(3), np.array([[0.5], [-0.25], [0.125]])], axis=1)  # exact sums
    pred = sc.pose_init.copy()
    pred[:, 3] -= prev[:, 3]
    p2, r2 = icp_register(gm, _dev(src), prev, pred, TAU, SIGMA, 100, 1e-4)
    assert r2["iterations"] == res["iterations"] and np.abs(p2 - pose).max() < 1e-9
    gm.close()


def test_register_degenerate_and_limits(street):
    from paper_2505_18992_amd import VoxelMap, icp_register
    sc, _ = street
    gm = VoxelMap(_dev(sc.map_points[:1000]), VOXEL, CAP)
    far = _dev(np.full((50, 3), 1000.0, np.float32))  # nothing within tau
    pose, res = icp_register(gm, far, np.eye(3, 4), None, TAU, SIGMA, 20, 1e-4)
    assert res["degenerate"] == 1 and res["iterations"] == 0 and np.array_equal(pose, np.eye(3, 4))
    src = _dev(_source(sc))
    pose, res = icp_register(gm, src, sc.pose_init, None, TAU, SIGMA, 0, 1e-4)
    assert res["iterations"] == 0 and np.array_equal(pose, sc.pose_init)
    gm.close()


def test_invalid_arguments():
    from paper_2505_18992_amd import _lib, get_context
    L, ctx = _lib.load(), get_context()
    import ctypes
    h = ctypes.c_void_p()
    pts = torch.zeros((4, 3), device="cuda")
    assert L.vpgs_voxel_map_create(ctx.handle, pts.data_ptr(), 4, 0.0, 5, ctypes.byref(h), None) == _lib.VPGS_EINVAL
    assert L.vpgs_voxel_map_create(ctx.handle, pts.data_ptr(), 4, 1.0, 0, ctypes.byref(h), None) == _lib.VPGS_EINVAL
    assert L.vpgs_voxel_downsample(ctx.handle, pts.data_ptr(), 4, -1.0, None, None, None) == _lib.VPGS_EINVAL
