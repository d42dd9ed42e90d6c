"""Pins of the oracle's two algorithms against results the mathematics fixes.

Time problem (Algorithm 1, Theorem 3.1):
  T1  v = 0, theta0 = sin 2pi x sin 2pi y:  theta(T,x) = exp(-8 pi^2 kappa T) theta0(x).
  T2  constant drift c, periodised Gaussian theta0 (width s, centre m):
      theta(T,x) = sum_n s^2/(s^2+2 kappa T) exp(-|x - cT - m - n|^2 / (2(s^2+2 kappa T))).
  T3  one shear mode k = (1,0) with any (a,b), theta0 = sin 2pi x:
      theta(T,x) = exp(-4 pi^2 kappa T) sin 2pi x  (the drift is orthogonal to k).
  In all three Euler-Maruyama is exact in law, so only Monte Carlo error remains.
  PDE  a general Fourier field: the particle mean agrees with an independent
       pseudo-spectral solve of eq. adr (tests/pde_reference.py).

Dirichlet problem (Algorithm 2, Theorem 3.2) on the unit disk:
  D1  v = 0, f = 0, g = cos 3 phi:          theta = r^3 cos 3 phi.
  D2  v = 0, f = -1 (payoff g + tau):        theta = r^3 cos 3 phi + (1 - r^2)/(4 kappa),
      and the mean exit time is (1 - r^2)/(4 kappa).
  D3  psi = a0 (1-r^2)^2 (k = 0 only): a purely azimuthal drift leaves |X|^2
      unchanged in law, so E tau = (1 - r^2)/(4 kappa) still holds.
  D4  constant drift c, f = 0, g = exp(c.x/kappa): theta = exp(c.x/kappa).
  Discrete monitoring of the exit overshoots the boundary by O(sqrt(dt)).  The
  expected exit statistics are compared with the continuity-corrected radius
  R = 1 + 0.5826 sqrt(2 kappa dt) (Broadie, Glasserman and Kou, 1997) and the
  tolerance carries a bias allowance of the same order.
"""
import math

import numpy as np
import pytest

import workloads as W
from tests import pde_reference as PDE

BETA_BGK = 0.5826


def _z(mean, var, n, ref):
    se = np.sqrt(var / n)
    return np.abs(mean - ref) / se, se


def test_T1_heat_on_torus(orc):
    rng = np.random.default_rng(1)
    modes = W.torus_modes(2)
    u = np.zeros(2 * len(modes))
    obs = rng.random((6, 2))
    kappa, T, dt, Np = 0.05, 0.1, 1e-3, 20000
    m, v = orc.observe_time(modes, u, W.fld("sinsin", [1.0]), obs, kappa, T, dt, Np, seed=5)
    ref = math.exp(-8 * math.pi**2 * kappa * T) * np.sin(2 * np.pi * obs[:, 0]) * np.sin(2 * np.pi * obs[:, 1])
    z, _ = _z(m, v, Np, ref)
    assert np.all(z < 4.5), z


def _periodic_gauss_conv(x, c, m, s, kappa, T):
    s2 = s * s + 2 * kappa * T
    out = 0.0
    for nx in range(-3, 4):
        for ny in range(-3, 4):
            d = np.array([x[0] - c[0] * T - m[0] - nx, x[1] - c[1] * T - m[1] - ny])
            out += s * s / s2 * np.exp(-(d @ d) / (2 * s2))
    return out


def test_T2_constant_drift_gaussian(orc):
    rng = np.random.default_rng(2)
    m0 = np.array([0.3, 0.6])
    s = 0.1
    c = np.array([0.7, -1.3])
    kappa, T, dt, Np = 0.01, 0.5, 1e-2, 20000
    obs = np.array([[0.65, 0.95], [0.72, 0.02], [0.55, 0.9], [0.1, 0.2]])
    theta0 = W.fld("gauss_periodic", [m0[0], m0[1], s, 1.0])
    modes = W.torus_modes(1)
    u = np.zeros(2 * len(modes))
    mm, v = orc.observe_time(modes, u, theta0, obs, kappa, T, dt, Np, seed=6, v0=c)
    ref = np.array([_periodic_gauss_conv(x, c, m0, s, kappa, T) for x in obs])
    # the mean is sizeable at some points, so the test has power there
    assert ref.max() > 0.3
    z, _ = _z(mm, v, Np, ref)
    assert np.all(z < 4.5), (mm, ref, z)


def test_T3_single_shear_mode(orc):
    modes = np.array([[1, 0]], dtype=np.int32)
    u = np.array([0.8, -0.5])
    rng = np.random.default_rng(3)
    obs = rng.random((5, 2))
    kappa, T, dt, Np = 0.02, 0.5, 1e-2, 20000
    m, v = orc.observe_time(modes, u, W.fld("fourier", [1, 0, 0, 1]), obs, kappa, T, dt, Np, seed=7)
    ref = math.exp(-4 * math.pi**2 * kappa * T) * np.sin(2 * np.pi * obs[:, 0])
    z, _ = _z(m, v, Np, ref)
    assert np.all(z < 4.5), z
    # a theta0 that depends on y does feel the drift: the same mode moves it
    m2, _ = orc.observe_time(modes, u, W.fld("fourier", [0, 1, 0, 1]), obs, kappa, T, dt, 4000, seed=7)
    ref_nodrift = math.exp(-4 * math.pi**2 * kappa * T) * np.sin(2 * np.pi * obs[:, 1])
    assert np.max(np.abs(m2 - ref_nodrift)) > 0.05


@pytest.mark.slow
def test_time_problem_matches_spectral_pde_solve(orc):
    wl = W.time_small()
    kappa, T = wl.kappa, wl.T
    h, k = PDE.solve(wl.modes, wl.u, lambda X, Y: np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y),
                     kappa, T, N=64, dt=1e-4)
    ref = PDE.evaluate(h, k, wl.obs)
    # Euler-Maruyama has weak order one: Richardson-extrapolate the particle
    # mean from dt and dt/2 to cancel the O(dt) bias (large for this flow).
    Np = 20000
    m1, v1 = orc.observe_time(wl.modes, wl.u, wl.theta0, wl.obs, kappa, T, 1e-4, Np, seed=11)
    m2, v2 = orc.observe_time(wl.modes, wl.u, wl.theta0, wl.obs, kappa, T, 5e-5, Np, seed=12)
    m = 2 * m2 - m1
    se = np.sqrt((4 * v2 + v1) / Np)
    z = np.abs(m - ref) / se
    assert np.all(z < 4.5), (m, ref, z)
    # the flow matters at these points: the v = 0 answer is many SEs away
    heat = math.exp(-8 * math.pi**2 * kappa * T) * np.sin(2 * np.pi * wl.obs[:, 0]) * np.sin(2 * np.pi * wl.obs[:, 1])
    assert np.max(np.abs(ref - heat) / se) > 20
    # and the reversed drift is rejected
    h2, _ = PDE.solve(wl.modes, -wl.u, lambda X, Y: np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y),
                      kappa, T, N=64, dt=1e-4)
    ref_rev = PDE.evaluate(h2, k, wl.obs)
    assert np.max(np.abs(m - ref_rev) / se) > 10


# ---------------------------------------------------------------------------
# Dirichlet problem
# ---------------------------------------------------------------------------

DISK_OBS = np.array([[0.0, 0.0], [0.3, 0.1], [-0.2, 0.5], [0.6, -0.3], [0.1, -0.75]])


def _r_eff(kappa, dt):
    return 1 + BETA_BGK * math.sqrt(2 * kappa * dt)


def test_D1_D2_harmonic_boundary_data_and_exit_time(orc):
    kappa, dt, Np = 0.25, 1e-3, 20000
    empty = np.zeros((0, 2), dtype=np.int32)
    r = orc.observe_dirichlet(empty, np.zeros(0), W.fld("const", [-1.0]), W.fld("cos_m_theta", [3]),
                              DISK_OBS, kappa, dt, Np, seed=21, max_steps=10**6)
    x, y = DISK_OBS[:, 0], DISK_OBS[:, 1]
    rr2 = x * x + y * y
    h = (x**3 - 3 * x * y * y)  # r^3 cos 3 phi
    R = _r_eff(kappa, dt)
    et = (R * R - rr2) / (4 * kappa)
    et0 = (1 - rr2) / (4 * kappa)
    # exit time: BGK-corrected, allowance 25% of the correction
    se_t = np.sqrt(r["tau_var"] / Np)
    assert np.all(np.abs(r["tau_mean"] - et) < 4 * se_t + 0.25 * np.abs(et - et0)), (r["tau_mean"], et)
    # the uncorrected value is measurably different at this dt (the bias is real)
    assert np.mean(r["tau_mean"] - et0) > 0
    # D2 payoff g + tau; D1 then follows by subtracting the exit time path by path
    ref = h / R**3 + et
    se = np.sqrt(r["var"] / Np)
    allow = 0.25 * (np.abs(h - h / R**3) + np.abs(et - et0))
    assert np.all(np.abs(r["mean"] - ref) < 4 * se + allow), (r["mean"], ref)
    assert np.all(r["n_capped"] == 0)


def test_D1_harmonic_only(orc):
    kappa, dt, Np = 0.25, 1e-3, 20000
    empty = np.zeros((0, 2), dtype=np.int32)
    r = orc.observe_dirichlet(empty, np.zeros(0), W.fld("zero"), W.fld("cos_m_theta", [3]),
                              DISK_OBS, kappa, dt, Np, seed=22, max_steps=10**6)
    x, y = DISK_OBS[:, 0], DISK_OBS[:, 1]
    h = x**3 - 3 * x * y * y
    R = _r_eff(kappa, dt)
    se = np.sqrt(r["var"] / Np)
    assert np.all(np.abs(r["mean"] - h / R**3) < 4 * se + 0.25 * np.abs(h - h / R**3))
    # cos 3 phi on the circle has mean zero from the centre
    assert abs(r["mean"][0]) < 4 * se[0]


def test_D3_azimuthal_drift_keeps_exit_time(orc):
    kappa, dt, Np = 0.25, 1e-3, 20000
    modes = np.array([[0, 0]], dtype=np.int32)
    u = np.array([1.5, 0.0])
    # the field really is azimuthal and non-zero
    V = orc.velocity("disk", modes, u, DISK_OBS[1:])
    assert np.max(np.abs((V * DISK_OBS[1:]).sum(1))) < 1e-12
    assert np.min(np.hypot(V[:, 0], V[:, 1])) > 0.1
    r = orc.observe_dirichlet(modes, u, W.fld("zero"), W.fld("zero"), DISK_OBS, kappa, dt, Np,
                              seed=23, max_steps=10**6)
    rr2 = (DISK_OBS**2).sum(1)
    R = _r_eff(kappa, dt)
    et = (R * R - rr2) / (4 * kappa)
    et0 = (1 - rr2) / (4 * kappa)
    se_t = np.sqrt(r["tau_var"] / Np)
    assert np.all(np.abs(r["tau_mean"] - et) < 4 * se_t + 0.35 * np.abs(et - et0)), (r["tau_mean"], et)


def test_D4_constant_drift_exponential_harmonic(orc):
    kappa, dt, Np = 0.25, 2.5e-4, 20000
    c = np.array([0.15, 0.075])
    empty = np.zeros((0, 2), dtype=np.int32)
    g = W.fld("exp_linear", [c[0] / kappa, c[1] / kappa])
    r = orc.observe_dirichlet(empty, np.zeros(0), W.fld("zero"), g, DISK_OBS, kappa, dt, Np,
                              seed=24, max_steps=10**6, v0=c)
    ref = np.exp(DISK_OBS @ c / kappa)
    se = np.sqrt(r["var"] / Np)
    bias = 2 * BETA_BGK * math.sqrt(2 * kappa * dt) * np.linalg.norm(c / kappa) * np.exp(np.linalg.norm(c) / kappa)
    assert np.all(np.abs(r["mean"] - ref) < 4 * se + bias), (r["mean"], ref)
    # the opposite drift gives a clearly different answer
    r2 = orc.observe_dirichlet(empty, np.zeros(0), W.fld("zero"), g, DISK_OBS, kappa, dt, 4000,
                               seed=24, max_steps=10**6, v0=-c)
    assert np.max(np.abs(r2["mean"] - ref) / (4 * se + bias)) > 3


def test_capped_paths_are_flagged(orc):
    empty = np.zeros((0, 2), dtype=np.int32)
    r = orc.observe_dirichlet(empty, np.zeros(0), W.fld("const", [1.0]), W.fld("const", [5.0]),
                              DISK_OBS[:1], 0.02, 1e-4, 64, seed=25, max_steps=10)
    assert np.all(r["n_capped"] == 64)
    # a capped path has no boundary term: payoff = -int f = -(max_steps * dt)
    assert r["mean"][0] == pytest.approx(-10 * 1e-4)


def test_D5_linear_source(orc):
    """kappa Lap theta = x, theta = 0 on the circle: theta = x (r^2 - 1) / (8 kappa);
    Theorem 3.2 then gives E int_0^tau X_x dt = x (1 - r^2) / (8 kappa)."""
    kappa, dt, Np = 0.25, 1e-3, 20000
    empty = np.zeros((0, 2), dtype=np.int32)
    r = orc.observe_dirichlet(empty, np.zeros(0), W.fld("linear", [1.0, 0.0, 0.0]), W.fld("zero"),
                              DISK_OBS, kappa, dt, Np, seed=26, max_steps=10**6)
    x = DISK_OBS[:, 0]
    rr2 = (DISK_OBS**2).sum(1)
    ref = x * (rr2 - 1) / (8 * kappa)
    R = _r_eff(kappa, dt)
    ref_R = x * (rr2 - R * R) / (8 * kappa)
    se = np.sqrt(r["var"] / Np)
    assert np.all(np.abs(r["mean"] - ref_R) < 4 * se + 0.25 * np.abs(ref - ref_R) + 1e-3), (r["mean"], ref)
    # a sign error in the source term would be many errors away at x = 0.6
    assert abs(r["mean"][3] + ref[3]) > 10 * se[3]
