"""Pins of the oracle's velocity field, wavevector tables and single paths.

- The real stream-function form used everywhere, v = (d psi/dy, -d psi/dx) with
  psi = sum_k a_k cos 2pi k.x + b_k sin 2pi k.x, is checked against the paper's
  complex divergence-free expansion (Section 4.1, eq. v_expand),
      v(x) = sum_{k in Z^2} v_k k_perp/|k| exp(2 pi i k.x),  k_perp = (-k_y, k_x),
  with v_k = -pi |k| (b_k + i a_k) on the half-plane set and the reality
  condition v_{-k} = -conj(v_k) for the mirrored modes.
- Finite differences of the oracle's own psi reproduce v (orientation of the
  perpendicular gradient) and give a zero divergence (eq. adr, div v = 0).
- On the disk, v = grad_perp((1-r^2)^2 psi_F) vanishes on the boundary.
- The mode counts of the paper's examples (Section 4.1: 197, 3,209 and 20,081
  wavevectors for |k|_2 <= 8, 32, 80) are reproduced by the table generator.
- A pure-Python re-derivation of eq. (euler) with its own Philox, Box-Muller and
  the complex velocity reproduces the oracle's paths on tiny inputs.
"""
import math

import numpy as np
import pytest

import workloads as W


def paper_complex_velocity(modes, u, X):
    M = len(modes)
    a, b = u[:M], u[M:]
    V = np.zeros((len(X), 2))
    for m, (kx, ky) in enumerate(modes):
        nk = math.hypot(kx, ky)
        vk = -math.pi * nk * (b[m] + 1j * a[m])
        for sgn, coef in ((1, vk), (-1, -np.conj(vk))):
            k = np.array([sgn * kx, sgn * ky], dtype=float)
            kperp = np.array([-k[1], k[0]])
            e = np.exp(2j * np.pi * (X @ k))
            V += np.real(coef * e)[:, None] * (kperp / nk)[None, :]
    return V


@pytest.mark.parametrize("K", [1, 2, 6])
def test_velocity_matches_paper_complex_expansion(orc, K):
    rng = np.random.default_rng(K)
    modes = W.torus_modes(K)
    u = W.draw_prior(modes, rng)
    X = rng.random((500, 2))
    ref = paper_complex_velocity(modes, u, X)
    got = orc.velocity("torus", modes, u, X)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def _d(fun, X, axis, h):
    e = np.zeros(2)
    e[axis] = h
    return (-fun(X + 2 * e) + 8 * fun(X + e) - 8 * fun(X - e) + fun(X - 2 * e)) / (12 * h)


@pytest.mark.parametrize("domain", ["torus", "disk"])
def test_velocity_is_perpendicular_gradient_of_stream_function(orc, domain):
    rng = np.random.default_rng(5)
    modes = W.torus_modes(6) if domain == "torus" else W.disk_modes()
    u = W.draw_prior(modes, rng)
    if domain == "torus":
        X = rng.random((300, 2))
    else:
        X = W.uniform_disk_points(300, 0.95, rng)
    psi = lambda P: orc.stream(domain, modes, u, P)
    V = orc.velocity(domain, modes, u, X)
    h = 1e-4
    vx = _d(psi, X, 1, h)
    vy = -_d(psi, X, 0, h)
    scale = np.max(np.abs(V))
    assert np.max(np.abs(V[:, 0] - vx)) < 1e-6 * scale
    assert np.max(np.abs(V[:, 1] - vy)) < 1e-6 * scale
    # divergence free
    vxf = lambda P: orc.velocity(domain, modes, u, P)[:, 0]
    vyf = lambda P: orc.velocity(domain, modes, u, P)[:, 1]
    div = _d(vxf, X, 0, h) + _d(vyf, X, 1, h)
    grad_scale = np.max(np.abs(_d(vxf, X, 0, h)))
    assert np.max(np.abs(div)) < 1e-6 * grad_scale


def test_disk_velocity_vanishes_on_boundary(orc):
    rng = np.random.default_rng(9)
    modes = W.disk_modes()
    u = W.draw_prior(modes, rng)
    ph = rng.random(200) * 2 * np.pi
    X = np.stack([np.cos(ph), np.sin(ph)], 1)
    inner = orc.velocity("disk", modes, u, 0.5 * X)
    V = orc.velocity("disk", modes, u, X)
    assert np.max(np.abs(V)) < 1e-12 * np.max(np.abs(inner))


def test_constant_drift_is_added(orc):
    modes = W.torus_modes(1)
    u = np.zeros(2 * len(modes))
    V = orc.velocity("torus", modes, u, np.random.default_rng(0).random((5, 2)), v0=(0.3, -1.5))
    assert np.allclose(V, [[0.3, -1.5]] * 5, atol=0, rtol=0)


def test_mode_tables():
    assert len(W.torus_modes(2)) == 12
    assert len(W.torus_modes(6)) == 84
    assert len(W.disk_modes()) == 32
    # half-plane: no wavevector together with its negative, no k = 0
    for K in (2, 6):
        s = {tuple(k) for k in W.torus_modes(K)}
        assert (0, 0) not in s
        assert all((-a, -b) not in s for a, b in s)
        assert len(s) == ((2 * K + 1) ** 2 - 1) // 2
    # the paper's N_u counts for |k|_2 <= 8, 32, 80 (Examples 1-3)
    assert len(W.l2_ball_modes(8)) == 197
    assert len(W.l2_ball_modes(32)) == 3209
    assert len(W.l2_ball_modes(80)) == 20081


# ---------------------------------------------------------------------------
# Pure-Python brute force of single paths
# ---------------------------------------------------------------------------

def _mulhilo(a, b):
    p = a * b
    return p >> 32, p & 0xFFFFFFFF


def py_philox(ctr, key):
    x = list(ctr)
    k = list(key)
    for _ in range(10):
        h0, l0 = _mulhilo(0xD2511F53, x[0])
        h1, l1 = _mulhilo(0xCD9E8D57, x[2])
        x = [h1 ^ x[1] ^ k[0], l1, h0 ^ x[3] ^ k[1], l0]
        k = [(k[0] + 0x9E3779B9) & 0xFFFFFFFF, (k[1] + 0xBB67AE85) & 0xFFFFFFFF]
    return x


def py_normal(seed, n, i, j):
    w = py_philox([n // 2, i, j, 0], [seed & 0xFFFFFFFF, seed >> 32])
    wa, wb = (w[0], w[1]) if n % 2 == 0 else (w[2], w[3])
    ua = ((wa >> 8) + 1) / 2.0**24
    ub = (wb >> 8) / 2.0**24
    r = math.sqrt(-2 * math.log(ua))
    return r * math.cos(2 * math.pi * ub), r * math.sin(2 * math.pi * ub)


def py_path(modes, u, kappa, dt, seed, i, j, x0, nsteps):
    X = np.array(x0, dtype=float)
    out = [X.copy()]
    for n in range(nsteps):
        v = paper_complex_velocity(modes, u, X[None, :])[0]
        z = py_normal(seed, n, i, j)
        X = X - v * dt + math.sqrt(2 * kappa * dt) * np.array(z)
        X = X - np.floor(X)
        out.append(X.copy())
    return np.array(out)


@pytest.mark.parametrize("K", [1, 2])
def test_paths_match_pure_python_brute_force(orc, K):
    rng = np.random.default_rng(100 + K)
    modes = W.torus_modes(K)
    u = W.draw_prior(modes, rng)
    x0 = rng.random(2)
    for i in range(8):
        ref = py_path(modes, u, 0.05, 1e-3, 77, i, 3, x0, 10)
        got = orc.path("torus", modes, u, 0.05, 1e-3, 77, i, 3, x0, 10)
        d = np.abs(got - ref)
        d = np.minimum(d, 1 - d)  # torus distance
        assert np.max(d) < 1e-13
