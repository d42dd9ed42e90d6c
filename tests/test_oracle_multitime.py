"""Pins of the oracle's multi-time observation (Algorithm 1 run once per
observation time t_k = n_k dt and point x_j, with step dt).

  M1  n_k = 0 reads theta0 at the start point: mean theta0(x_j), variance 0
      (to the rounding of the sum).
  M2  constant drift c, periodised Gaussian theta0: at every t_k the mean
      matches the closed form (the Gaussian spread by 2 kappa t_k and moved by
      c t_k; Euler-Maruyama is exact in law here), so a wrong time index, step
      size or drift sign fails.
  M3  heat (v = 0, theta0 = sin sin): every t_k decays as exp(-8 pi^2 kappa t_k).
  M4  with dt a power of two, T = n dt divides back to dt exactly, so the read
      at n equals a plain Algorithm 1 run to T bit for bit.
"""
import math

import numpy as np

import workloads as W
from tests.test_oracle_closed_forms import _periodic_gauss_conv, _z


def test_M1_zero_steps_reads_theta0(orc):
    modes = W.torus_modes(2)
    rng = np.random.default_rng(11)
    u = W.draw_prior(modes, rng)
    obs = rng.random((5, 2))
    th = W.fld("sinsin", [1.0])
    m, v = orc.observe_time_multi(modes, u, th, obs, 0.05, [0, 3], 1e-3, 64, seed=2)
    ref = np.sin(2 * np.pi * obs[:, 0]) * np.sin(2 * np.pi * obs[:, 1])
    # the mean of 64 equal values carries only the summation's rounding
    assert np.allclose(m[0], ref, rtol=1e-14, atol=1e-15)
    assert np.all(v[0] < 1e-28)
    assert not np.array_equal(m[1], ref)


def test_M2_constant_drift_at_several_times(orc):
    m0 = np.array([0.3, 0.6])
    s = 0.1
    c = np.array([0.7, -1.3])
    kappa, dt, Np = 0.01, 1e-2, 20000
    steps = [10, 25, 50]
    obs = np.array([[0.37, 0.47], [0.48, 0.28], [0.65, 0.95], [0.1, 0.2]])
    theta0 = W.fld("gauss_periodic", [m0[0], m0[1], s, 1.0])
    modes = W.torus_modes(1)
    u = np.zeros(2 * len(modes))
    mm, vv = orc.observe_time_multi(modes, u, theta0, obs, kappa, steps, dt, Np, seed=6, v0=c)
    for k, n in enumerate(steps):
        t = n * dt
        ref = np.array([_periodic_gauss_conv(x, c, m0, s, kappa, t) for x in obs])
        assert ref.max() > 0.3, (t, ref)  # the test has power at every time
        z, _ = _z(mm[k], vv[k], Np, ref)
        assert np.all(z < 4.5), (t, mm[k], ref, z)


def test_M3_heat_decay_at_several_times(orc):
    rng = np.random.default_rng(12)
    modes = W.torus_modes(2)
    u = np.zeros(2 * len(modes))
    obs = rng.random((4, 2))
    kappa, dt, Np = 0.05, 1e-3, 20000
    steps = [20, 60, 100]
    m, v = orc.observe_time_multi(modes, u, W.fld("sinsin", [1.0]), obs, kappa, steps, dt, Np, seed=5)
    base = np.sin(2 * np.pi * obs[:, 0]) * np.sin(2 * np.pi * obs[:, 1])
    for k, n in enumerate(steps):
        z, _ = _z(m[k], v[k], Np, math.exp(-8 * math.pi**2 * kappa * n * dt) * base)
        assert np.all(z < 4.5), (n, z)


def test_M4_last_read_equals_a_plain_run(orc):
    wl = W.time_small()
    dt = 2.0 ** -10
    steps = [7, 40, 102]
    m, v = orc.observe_time_multi(wl.modes, wl.u, wl.theta0, wl.obs, wl.kappa, steps, dt, 300, wl.seed)
    for k, n in enumerate(steps):
        m1, v1 = orc.observe_time(wl.modes, wl.u, wl.theta0, wl.obs, wl.kappa, n * dt, dt, 300, wl.seed)
        assert np.array_equal(m[k], m1) and np.array_equal(v[k], v1)
