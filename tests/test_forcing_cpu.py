"""Host logic of the optimal-forcing driver on an affine map with a known
answer (no GPU): Nelder-Mead on |y - (a - B^T F)| reaches the least-squares
solution, which for an invertible 3 x 3 B matches y exactly."""
import numpy as np

from paper_1808_10580_amd import forcing


def test_nelder_mead_reaches_the_least_squares_optimum():
    rng = np.random.default_rng(4)
    B = rng.uniform(0.05, 0.3, (3, 3))
    F_true = np.array([2.0, -1.5, 3.0])
    a = rng.uniform(0.3, 0.9, 3)
    y = a - B.T @ F_true
    res = forcing.optimal_forcing(a, B, y)
    assert np.allclose(res["F_ls"], F_true, atol=1e-9)
    assert np.allclose(res["F_nm"], F_true, atol=1e-6)
    assert res["cost_nm"] < 1e-8


def test_overdetermined_map_gives_the_least_squares_residual():
    rng = np.random.default_rng(5)
    B = rng.uniform(0.05, 0.3, (2, 5))  # 2 sources, 5 observations
    a, y = rng.uniform(0, 1, 5), np.zeros(5)
    res = forcing.optimal_forcing(a, B, y)
    assert abs(res["cost_nm"] - res["cost_ls"]) < 1e-7
    # the least-squares residual is orthogonal to the columns of B^T
    r = y - (a - B.T @ res["F_ls"])
    assert np.max(np.abs(B @ r)) < 1e-10
