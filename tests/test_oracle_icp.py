"""Pins of the voxel-map registration oracle (eq. 10-12) on the CPU:
downsampling and the per-voxel point lists against numpy.unique, the voxel
nearest neighbour against a k-d tree within one voxel, the kernel weight
against the derivative of rho, the linear system against central
differences of the robust cost and against the Kabsch rotation in the
least-squares limit, the SE(3) exponential against the matrix exponential,
and the recovery of a known motion."""
import math

import numpy as np
import pytest
import scipy.linalg
from scipy.spatial import cKDTree

import scenes
from oracle import icp


def _cloud(seed, n=3000, extent=6.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(-extent, extent, (n, 3)).astype(np.float32)


def test_downsample_keeps_first_point_of_each_voxel():
    p = _cloud(1, 5000)
    keep = icp.downsample(p, 0.7)
    _, first = np.unique(icp.voxel_coords(p, 0.7), axis=0, return_index=True)
    assert np.array_equal(keep, np.sort(first))


def test_voxel_map_lists_first_points_in_index_order():
    p = _cloud(2, 4000, extent=2.0)
    vm = icp.VoxelMap(p, 0.5, 5)
    keys, inv = np.unique(icp.voxel_coords(p, 0.5), axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    assert len(vm.cells) == keys.shape[0]
    for k in range(keys.shape[0]):
        members = np.nonzero(inv == k)[0]  # ascending
        assert vm.cells[tuple(keys[k])] == members[:5].tolist()
    assert max(len(v) for v in vm.cells.values()) == 5  # the cap is reached


def test_voxel_nearest_neighbour_equals_kdtree_within_a_voxel():
    m = _cloud(3, 800, extent=5.0)
    v = 1.0
    vm = icp.VoxelMap(m, v, 10 ** 6)  # no cap: every point is kept
    q = _cloud(4, 3000, extent=5.0)
    tau = 0.9 * v
    nn, d2 = icp.correspond(vm, q, tau)
    dist, idx = cKDTree(m.astype(np.float64)).query(q.astype(np.float64), k=2)
    exact = dist[:, 0] < tau
    clear = (dist[:, 1] - dist[:, 0]) > 1e-5
    close = np.abs(dist[:, 0] - tau) < 1e-5
    sel = clear & ~close
    assert np.array_equal(nn[sel] >= 0, exact[sel])
    assert np.array_equal(nn[sel & exact], idx[sel & exact, 0])
    assert np.allclose(np.sqrt(d2[sel & exact].astype(np.float64)), dist[sel & exact, 0], rtol=1e-5)
    assert (sel & exact).sum() > 1000 and (sel & ~exact).sum() > 100


def test_voxel_cap_limits_candidates():
    # two points in one voxel, a cap of one: only the first is ever matched
    m = np.array([[0.1, 0.1, 0.1], [0.5, 0.5, 0.5]], np.float32)
    vm = icp.VoxelMap(m, 1.0, 1)
    nn, _ = icp.correspond(vm, np.array([[0.49, 0.5, 0.5]], np.float32), 2.0)
    assert nn.tolist() == [0]


def test_weight_is_derivative_of_rho_over_e():
    sigma = 0.6
    for e in (0.01, 0.1, 0.3, 1.0, 3.0):
        h = 1e-6
        d = (icp.gm_rho((e + h) ** 2, sigma) - icp.gm_rho((e - h) ** 2, sigma)) / (2 * h)
        assert math.isclose(icp.gm_weight(e * e, sigma), d / e, rel_tol=1e-7)
    assert icp.gm_rho(0.0, sigma) == 0.0 and abs(icp.gm_rho(1e12, sigma) - 0.5) < 1e-9


def _pairs(seed, n=200):
    rng = np.random.default_rng(seed)
    p = rng.uniform(-3, 3, (n, 3))
    m = p + rng.normal(0, 0.2, p.shape)
    return p, m


def test_gradient_matches_central_differences_of_the_robust_cost():
    p, m = _pairs(5)
    sigma = 0.5
    H, g, n, rho = icp.normal_equations(p, m, sigma)

    def cost(xi):
        T = icp.se3_exp(xi)
        q = p @ T[:, :3].T + T[:, 3]
        r = q - m
        return icp.gm_rho(np.einsum("ij,ij->i", r, r), sigma).sum()
    assert math.isclose(cost(np.zeros(6)), rho, rel_tol=1e-12)
    for k in range(6):
        e = np.zeros(6)
        e[k] = 1e-6
        fd = (cost(e) - cost(-e)) / 2e-6
        assert abs(fd - g[k]) < 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])
    assert np.allclose(H, H.T) and np.linalg.eigvalsh(H).min() > 0


def test_least_squares_limit_reaches_the_kabsch_solution():
    # kappa >> e^2 makes every weight ~1/kappa: Gauss-Newton on fixed pairs
    # converges to the rigid least-squares fit (Kabsch, by SVD)
    p, m = _pairs(6)
    T = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)
    for _ in range(30):
        q = p @ T[:, :3].T + T[:, 3]
        H, g, _, _ = icp.normal_equations(q, m, 1e9)
        T = icp._compose(icp.se3_exp(-np.linalg.solve(H, g)), T)
    pc, mc = p - p.mean(0), m - m.mean(0)
    U, _, Vt = np.linalg.svd(mc.T @ pc)
    D = np.diag([1, 1, np.sign(np.linalg.det(U @ Vt))])
    R = U @ D @ Vt
    t = m.mean(0) - R @ p.mean(0)
    assert np.allclose(T[:, :3], R, atol=1e-9) and np.allclose(T[:, 3], t, atol=1e-9)


@pytest.mark.parametrize("xi", [[0.3, -0.2, 0.1, 0.2, -0.1, 0.4], [1.0, 2.0, 3.0, 0.0, 0.0, 0.0],
                                [0.1, 0.0, 0.0, 1e-10, 0.0, 0.0]])
def test_se3_exp_equals_matrix_exponential(xi):
    rho, phi = np.array(xi[:3]), np.array(xi[3:])
    tw = np.zeros((4, 4))
    tw[:3, :3] = icp._skew(phi)
    tw[:3, 3] = rho
    E = scipy.linalg.expm(tw)
    assert np.allclose(icp.se3_exp(xi), E[:3, :], atol=1e-12)


def test_register_recovers_a_known_motion():
    # points on the street's surfaces with no noise, scan = map subset moved;
    # no cap, so every scan point's own map point is a candidate
    sc = scenes.make_street_scan(n_map=60_000, noise=0.0)
    vm = icp.VoxelMap(sc.map_points, 1.0, 1000)
    rng = np.random.default_rng(7)
    sel = rng.choice(sc.map_points.shape[0], 3000, replace=False)
    true = icp.se3_exp([0.2, -0.1, 0.05, 0.0, 0.0, 0.02])
    inv_R = true[:, :3].T
    src = ((sc.map_points[sel].astype(np.float64) - true[:, 3]) @ inv_R.T).astype(np.float32)
    out = icp.register(vm, src, np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1), tau=1.0, sigma=0.3,
                       max_iter=100, eps=1e-6)
    assert out["converged"] and out["count"] == 3000
    assert np.allclose(out["pose"][:, :3], true[:, :3], atol=1e-6)
    assert np.allclose(out["pose"][:, 3], true[:, 3], atol=2e-5)
