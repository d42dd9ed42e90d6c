"""Pins of the oracle's finite-difference Jacobian of G (common random
numbers, central differences).

  J1  directional consistency: J d matches the central difference of G along
      a random direction d, to O(h^2) (a transposed, mis-signed or mis-scaled
      assembly fails);
  J2  convergence: J(h) - J(h/2) shrinks like h^2 (CRN makes G smooth in u);
  J3  zero sensitivity where it must vanish: with theta0 depending on x only
      and the single mode k = (1, 0) (a flow along y), G does not depend on u
      on common random numbers, so J is exactly zero; the mode k = (0, 1)
      (a flow along x) gives a non-zero J.
"""
import numpy as np

import workloads as W


def _small():
    wl = W.time_small()
    return wl.modes, wl.u, wl.theta0, wl.obs[:3], wl.kappa, 0.02, wl.dt, 200, wl.seed


def test_J1_directional_consistency(orc):
    modes, u, th, obs, kappa, T, dt, Np, seed = _small()
    h = 1e-4
    J = orc.jacobian_time(modes, u, th, obs, kappa, T, dt, Np, seed, h)
    d = np.random.default_rng(3).standard_normal(u.size)
    d /= np.linalg.norm(d)
    gp, _ = orc.observe_time(modes, u + h * d, th, obs, kappa, T, dt, Np, seed)
    gm, _ = orc.observe_time(modes, u - h * d, th, obs, kappa, T, dt, Np, seed)
    dd = (gp - gm) / (2 * h)
    assert np.max(np.abs(J @ d - dd)) <= 1e-5 * max(1.0, np.max(np.abs(dd)))
    assert np.max(np.abs(dd)) > 1e-3  # the test has power


def test_J2_second_order_convergence(orc):
    modes, u, th, obs, kappa, T, dt, Np, seed = _small()
    J1 = orc.jacobian_time(modes, u, th, obs, kappa, T, dt, Np, seed, 4e-3)
    J2 = orc.jacobian_time(modes, u, th, obs, kappa, T, dt, Np, seed, 2e-3)
    J3 = orc.jacobian_time(modes, u, th, obs, kappa, T, dt, Np, seed, 1e-3)
    e1, e2 = np.max(np.abs(J1 - J2)), np.max(np.abs(J2 - J3))
    assert e2 < 0.4 * e1, (e1, e2)  # ~1/4 for a second-order difference


def test_J3_flow_along_level_sets_has_no_effect(orc):
    th = W.fld("fourier", [1, 0, 0, 1])   # sin 2 pi x: depends on x only
    obs = np.array([[0.1, 0.3], [0.6, 0.8]])
    # k = (1, 0) alone gives v = (0, v_y(x)): x diffuses freely whatever u is,
    # so on common random numbers G does not depend on u at all
    modes = np.array([[1, 0]], dtype=np.int32)
    J = orc.jacobian_time(modes, np.array([0.3, -0.1]), th, obs, 0.02, 0.05, 1e-3, 100, 4, 1e-3)
    assert np.all(J == 0.0)
    # k = (0, 1) alone gives v = (v_x(y), 0): it moves x, so G does depend on u
    modes = np.array([[0, 1]], dtype=np.int32)
    J = orc.jacobian_time(modes, np.array([0.2, 0.25]), th, obs, 0.02, 0.05, 1e-3, 100, 4, 1e-3)
    assert np.min(np.abs(J)) > 1e-3
