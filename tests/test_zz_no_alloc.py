"""The allocation-free linearisation (vpgs_icp_linearize_noalloc) against
vpgs_icp_linearize, through the C ABI: the same kernels on a static
per-device scratch array instead of the context's workspace, so the terms
agree bit for bit.  Two calls in a row, the second with fewer source points
(fewer workgroup rows than the first left in the scratch), and an empty
source."""
import numpy as np
import pytest
import torch

import scenes

pytestmark = pytest.mark.gpu

TAU, SIGMA, VOXEL, CAP = 3.0, 1.0, 1.0, 20


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def test_noalloc_linearize_equals_the_allocating_entry_point():
    from paper_2505_18992_amd import VoxelMap, icp_linearize, icp_linearize_noalloc
    sc = scenes.make_street_scan(n_map=300_000)
    gm = VoxelMap(_dev(sc.map_points), VOXEL, CAP)
    rng = np.random.default_rng(8)
    out = torch.empty((29,), dtype=torch.float64, device="cuda")
    # 120 k points: 512 workgroups, every row of the scratch; then 2 000
    # points (250 rows) and none (one row of zeros), after the larger call
    for n in (120_000, 2_000, 0):
        print(f"case noalloc linearize n={n}", flush=True)
        src = _dev(sc.scan[rng.choice(sc.scan.shape[0], n, replace=False)] if n else np.zeros((0, 3)))
        ref = icp_linearize(gm, src, sc.pose_init, TAU, SIGMA)
        out.fill_(np.nan)
        got = icp_linearize_noalloc(gm, src, sc.pose_init, TAU, SIGMA, out)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (n, (got - ref).abs().max().item())
        if n:
            assert got[27].item() > 0.5 * n  # most points found a neighbour
        else:
            assert int(torch.count_nonzero(got)) == 0
    gm.close()


def test_noalloc_linearize_rejects_bad_arguments():
    from paper_2505_18992_amd import VoxelMap, icp_linearize_noalloc
    from paper_2505_18992_amd._lib import VpgsError
    sc = scenes.make_street_scan(n_map=20_000)
    gm = VoxelMap(_dev(sc.map_points), VOXEL, CAP)
    out = torch.empty((29,), dtype=torch.float64, device="cuda")
    src = _dev(sc.scan[:100])
    with pytest.raises(VpgsError):
        icp_linearize_noalloc(gm, src, sc.pose_init, -1.0, SIGMA, out)
    bad = np.array(sc.pose_init, np.float64).copy()
    bad[0, 0] = np.inf
    with pytest.raises(VpgsError):
        icp_linearize_noalloc(gm, src, bad, TAU, SIGMA, out)
    gm.close()
