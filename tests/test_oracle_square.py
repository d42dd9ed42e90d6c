"""Pins of the oracle's Algorithm 2 on the unit square (0,1)^2 and of the
affine source decomposition used for the optimal-forcing example.

  S1  v = 0, f = 0, linear g (harmonic): theta = g;
  S2  constant drift c, f = 0, g = exp(c.x / kappa) (the operator's own
      harmonic function): theta = exp(c.x / kappa);
  S3  v = 0, f = -1, g = 0: theta = E tau = sum over odd m, n of
      16 / (pi^4 kappa m n (m^2 + n^2)) sin(m pi x) sin(n pi y);
  S4  G(F) = a - B F holds exactly on common random numbers: a run with the
      combined source equals the decomposition to rounding;
  S5  v = 0, g = 0, f = A exp(-w |x - c|^2) (the Gaussian field kind of the
      optimal-forcing example's sources): theta solves kappa Lap theta = f
      with theta = 0 on the boundary, a double sine series whose coefficients
      come from one-dimensional quadratures (the source is separable);
  S6  v = 0, f = 0, g = (cos(pi x / 2) + cos(pi y / 2)) / 2 (the example's
      boundary data, the cosine field kind): theta is the harmonic extension,
      g plus a sine series.
S5 and S6 also check that the tolerance would reject the plausible misreadings
of the two field kinds (the exponent exp(-|x-c|^2 / (2 w)), swapped centre
coordinates, the cosine scale pi x instead of pi x / 2).
Discrete monitoring overshoots the boundary by O(sqrt(dt)); S1 and S2 carry
an allowance of that size, S3 uses the square enlarged by the continuity
correction 0.5826 sqrt(2 kappa dt) on each side (Broadie, Glasserman, Kou).
"""
import math

import numpy as np

import workloads as W
from tests.pde_reference import laplace_square_cos_axes, poisson_square_separable

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


def _gauss_ref(cx, cy, w, A, kappa, obs, d):
    hx = lambda s: np.exp(-w * (s - cx) ** 2)
    hy = lambda s: np.exp(-w * (s - cy) ** 2)
    return np.array([poisson_square_separable(hx, hy, A, kappa, x, y, d) for x, y in obs])


def test_S5_gaussian_source_field(orc):
    kappa, dt, Np = 0.1, 1e-4, 16000
    obs = np.array([[0.4, 0.55], [0.2, 0.3], [0.75, 0.8]])
    d = BETA_BGK * math.sqrt(2 * kappa * dt)  # continuity-corrected square, as in S3
    for (cx, cy, w, A, seed) in [(0.4, 0.55, 4.0, 1.5, 21), (0.6, 0.35, 30.0, 2.0, 22)]:
        r = _run(orc, W.fld("gauss", [cx, cy, w, A]), ZERO, obs, kappa, dt, Np, seed)
        ref = _gauss_ref(cx, cy, w, A, kappa, obs, d)
        se = np.sqrt(r["var"] / Np)
        tol = 4.5 * se + 0.01 * np.abs(ref)
        assert np.all(np.abs(r["mean"] - ref) <= tol), (w, r["mean"], ref, tol)
        assert np.all(r["n_capped"] == 0)
        # power: each misreading moves some observation by more than twice the tolerance
        for wrong in (_gauss_ref(cx, cy, 1.0 / (2.0 * w), A, kappa, obs, d),   # exp(-r^2 / (2 w))
                      _gauss_ref(cy, cx, w, A, kappa, obs, d),                # centre swapped
                      -ref):                                                   # source sign
            assert np.max(np.abs(wrong - ref) / tol) > 2.0


def test_S6_cosine_boundary_data_field(orc):
    kappa, dt, Np = 0.1, 1e-4, 16000
    obs = np.array([[0.4, 0.55], [0.2, 0.3], [0.75, 0.8]])
    A, w = 0.5, math.pi / 2
    r = _run(orc, ZERO, W.fld("cos_axes", [A, w]), obs, kappa, dt, Np, 23)
    ref = np.array([laplace_square_cos_axes(x, y, A, w) for x, y in obs])
    # the series meets the boundary data (away from the corners)
    for (x, y) in [(1e-9, 0.3), (0.6, 1.0 - 1e-9)]:
        assert abs(laplace_square_cos_axes(x, y, A, w) - A * (math.cos(w * x) + math.cos(w * y))) < 2e-3
    grad = A * w * math.sqrt(2.0)  # max |grad g| on the square
    allow = 2 * grad * BETA_BGK * math.sqrt(2 * kappa * dt)
    se = np.sqrt(r["var"] / Np)
    tol = 4.5 * se + allow
    assert np.all(np.abs(r["mean"] - ref) <= tol), (r["mean"], ref, tol)
    for wrong in (np.array([laplace_square_cos_axes(x, y, A, 2 * w) for x, y in obs]),   # cos(pi x)
                  np.array([laplace_square_cos_axes(x, y, 2 * A, w) for x, y in obs])):  # amplitude 1
        assert np.max(np.abs(wrong - ref) / tol) > 2.0
