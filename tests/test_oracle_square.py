"""Pins of the oracle's Algorithm 2 on the unit square (0,1)^2 and of the
affine source decomposition used for the optimal-forcing example.

  S1  v = 0, f = 0, linear g (harmonic): theta = g;
  S2  constant drift c, f = 0, g = exp(c.x / kappa) (the operator's own
      harmonic function): theta = exp(c.x / kappa);
  S3  v = 0, f = -1, g = 0: theta = E tau = sum over odd m, n of
      16 / (pi^4 kappa m n (m^2 + n^2)) sin(m pi x) sin(n pi y);
  S4  G(F) = a - B F holds exactly on common random numbers: a run with the
      combined source equals the decomposition to rounding.
Discrete monitoring overshoots the boundary by O(sqrt(dt)); S1 and S2 carry
an allowance of that size, S3 uses the square enlarged by the continuity
correction 0.5826 sqrt(2 kappa dt) on each side (Broadie, Glasserman, Kou).
"""
import math

import numpy as np

import workloads as W

BETA_BGK = 0.5826
NONE = np.zeros((0, 2), dtype=np.int32)
ZERO = {"kind": "zero", "params": []}


def _run(orc, f, g, obs, kappa, dt, Np, seed, v0=(0.0, 0.0)):
    return orc.observe_dirichlet(NONE, np.zeros(0), f, g, obs, kappa, dt, Np, seed, 10_000_000, v0,
                                 domain="square")


def test_S1_harmonic_linear_boundary_data(orc):
    kappa, dt, Np = 0.1, 1e-4, 4000
    obs = np.array([[0.3, 0.4], [0.7, 0.2], [0.5, 0.85]])
    c = np.array([0.8, -0.5, 0.3])
    r = _run(orc, ZERO, W.fld("linear", c), obs, kappa, dt, Np, 11)
    ref = obs @ c[:2] + c[2]
    allow = 2 * np.abs(c[:2]).sum() * BETA_BGK * math.sqrt(2 * kappa * dt)
    se = np.sqrt(r["var"] / Np)
    assert np.all(np.abs(r["mean"] - ref) <= 4.5 * se + allow), (r["mean"], ref, se, allow)
    assert np.all(r["n_capped"] == 0)


def test_S2_drift_and_its_harmonic_function(orc):
    kappa, dt, Np = 0.1, 1e-4, 4000
    cvec = np.array([0.2, -0.1])
    obs = np.array([[0.3, 0.4], [0.7, 0.2], [0.5, 0.85]])
    r = _run(orc, ZERO, W.fld("exp_linear", cvec / kappa), obs, kappa, dt, Np, 12, v0=tuple(cvec))
    ref = np.exp(obs @ cvec / kappa)
    # |grad g| on the square: |c / kappa| max g, g <= exp(max over corners of c.x / kappa)
    grad = np.linalg.norm(cvec / kappa) * np.exp(max(0.0, cvec[0] / kappa) + max(0.0, cvec[1] / kappa))
    allow = 2 * grad * BETA_BGK * math.sqrt(2 * kappa * dt)
    se = np.sqrt(r["var"] / Np)
    assert np.all(np.abs(r["mean"] - ref) <= 4.5 * se + allow), (r["mean"], ref, se, allow)
    # the reversed drift gives a clearly different answer (sign pin)
    rr = _run(orc, ZERO, W.fld("exp_linear", cvec / kappa), obs, kappa, dt, 1000, 12, v0=tuple(-cvec))
    assert np.max(np.abs(rr["mean"] - ref)) > 4 * (np.max(se) + allow)


def _exit_time_series(x, y, kappa, d):
    L = 1.0 + 2 * d
    xs, ys = (x + d) / L, (y + d) / L
    s = 0.0
    for m in range(1, 200, 2):
        for n in range(1, 200, 2):
            s += 16.0 / (math.pi ** 4 * kappa * m * n * (m * m + n * n)) * math.sin(m * math.pi * xs) * math.sin(
                n * math.pi * ys)
    return s * L * L


def test_S3_mean_exit_time(orc):
    kappa, dt, Np = 0.1, 1e-4, 4000
    obs = np.array([[0.5, 0.5], [0.2, 0.3], [0.8, 0.9]])
    r = _run(orc, W.fld("const", [-1.0]), ZERO, obs, kappa, dt, Np, 13)
    d = BETA_BGK * math.sqrt(2 * kappa * dt)
    ref = np.array([_exit_time_series(x, y, kappa, d) for x, y in obs])
    se = np.sqrt(r["var"] / Np)
    assert np.allclose(r["mean"], r["tau_mean"], rtol=1e-12, atol=1e-14)  # payoff = tau for f = -1, g = 0
    assert np.all(np.abs(r["mean"] - ref) <= 4.5 * se + 0.01 * ref), (r["mean"], ref, se)


def test_S4_affine_source_decomposition(orc):
    wl = W.bvp_square(n_particles=500)
    src = wl.extra["sources"]
    F = np.array([0.7, -1.3, 2.1])
    a, _, B, _ = orc.observe_dirichlet_sources(NONE, np.zeros(0), wl.g, wl.obs, wl.kappa, wl.dt, 500, wl.seed,
                                               wl.max_steps, src, wl.v0)
    f = {"kind": "gauss", "params": [v for (cx, cy, w), fj in zip(src, F) for v in (cx, cy, w, fj)]}
    r = _run(orc, f, wl.g, wl.obs, wl.kappa, wl.dt, 500, wl.seed, v0=wl.v0)
    assert np.max(np.abs(r["mean"] - (a - B @ F))) <= 1e-12
    assert np.all(B > 0)  # positive sources, positive integrals
