"""Independent "solve, then observe" reference for the time-dependent problem.

A pseudo-spectral Fourier-Galerkin solve of the advection-diffusion equation
on the unit torus (Section 4.1, eq. adr):
    d theta/dt = -v . grad theta + kappa Laplacian theta,  theta(0) = theta0,
integrated with classical RK4 and 2/3-rule de-aliasing, then evaluated at
arbitrary points by the trigonometric interpolant.  This is the paper's
two-step comparison method (Section 3.4, Algorithm 3 in spirit) and shares
nothing with the particle oracle; it pins the oracle's drift sign, the
velocity convention and the payoff readout through Theorem 3.1.

The velocity is built here from the paper's complex form (eq. v_expand)
rather than from the oracle.
"""
import math

import numpy as np


def complex_velocity(modes, u, X, Y):
    M = len(modes)
    a, b = u[:M], u[M:]
    vx = np.zeros_like(X)
    vy = np.zeros_like(X)
    for m, (kx, ky) in enumerate(modes):
        nk = math.hypot(kx, ky)
        vk = -math.pi * nk * (b[m] + 1j * a[m])
        ph = 2 * np.pi * (kx * X + ky * Y)
        # v_k k_perp/|k| e^{i ph} + v_{-k} (-k_perp)/|k| e^{-i ph}, v_{-k} = -conj(v_k)
        s = 2 * np.real(vk * np.exp(1j * ph)) / nk
        vx += s * (-ky)
        vy += s * kx
    return vx, vy


def solve(modes, u, theta0_grid_fn, kappa, T, N=96, dt=1e-4):
    x = np.arange(N) / N
    X, Y = np.meshgrid(x, x, indexing="ij")
    vx, vy = complex_velocity(modes, u, X, Y)
    k = np.fft.fftfreq(N, 1.0 / N)
    KX, KY = np.meshgrid(k, k, indexing="ij")
    dealias = ((np.abs(KX) < N / 3) & (np.abs(KY) < N / 3)).astype(float)
    lap = -4 * np.pi**2 * (KX**2 + KY**2)
    ikx = 2j * np.pi * KX
    iky = 2j * np.pi * KY

    def rhs(h):
        tx = np.fft.ifft2(ikx * h).real
        ty = np.fft.ifft2(iky * h).real
        adv = -(vx * tx + vy * ty)
        return dealias * np.fft.fft2(adv) + kappa * lap * h

    h = np.fft.fft2(theta0_grid_fn(X, Y))
    nsteps = int(round(T / dt))
    for _ in range(nsteps):
        k1 = rhs(h)
        k2 = rhs(h + 0.5 * dt * k1)
        k3 = rhs(h + 0.5 * dt * k2)
        k4 = rhs(h + dt * k3)
        h = h + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return h, k


def evaluate(h, k, pts):
    N = h.shape[0]
    c = h / (N * N)
    out = []
    for px, py in pts:
        ex = np.exp(2j * np.pi * k * px)
        ey = np.exp(2j * np.pi * k * py)
        out.append(np.real(ex @ c @ ey))
    return np.array(out)


# ---------------------------------------------------------------------------
# Elliptic problems on a square (Theorem 3.2 with v = 0): double sine series.
# ---------------------------------------------------------------------------

def sine_coeffs(h, a, b, nmax, nq=600):
    """c_m = (2/L) int_a^b h(s) sin(m pi (s - a) / L) ds, m = 1..nmax
    (Gauss-Legendre quadrature, L = b - a)."""
    L = b - a
    t, w = np.polynomial.legendre.leggauss(nq)
    s = a + (t + 1.0) * L / 2.0
    w = w * L / 2.0
    m = np.arange(1, nmax + 1)
    S = np.sin(np.outer(m, np.pi * (s - a) / L))
    return (2.0 / L) * (S * (w * h(s))).sum(axis=1)


def poisson_square_separable(hx, hy, amp, kappa, x, y, d=0.0, nmax=200):
    """theta with kappa Lap theta = amp hx(x) hy(y) on [-d, 1+d]^2 and theta = 0
    on its boundary.  Each sine mode sin(m pi (x+d)/L) sin(n pi (y+d)/L) is an
    eigenfunction of the Laplacian with eigenvalue -(pi/L)^2 (m^2 + n^2), so
    theta_mn = -amp hx_m hy_n / (kappa (pi/L)^2 (m^2 + n^2))."""
    a, b = -d, 1.0 + d
    L = b - a
    cx = sine_coeffs(hx, a, b, nmax)
    cy = sine_coeffs(hy, a, b, nmax)
    m = np.arange(1, nmax + 1)
    lam = (np.pi / L) ** 2 * (m[:, None] ** 2 + m[None, :] ** 2)
    C = -amp * np.outer(cx, cy) / (kappa * lam)
    sx = np.sin(m * np.pi * (x - a) / L)
    sy = np.sin(m * np.pi * (y - a) / L)
    return float(sx @ C @ sy)


def laplace_square_cos_axes(x, y, A, w, nmax=200):
    """Harmonic theta on the unit square with theta = A (cos(w x) + cos(w y))
    on its boundary.  g = A (cos w x + cos w y) itself satisfies Lap g = -w^2 g,
    so theta = g + r with Lap r = w^2 g and r = 0 on the boundary, a Poisson
    problem with two separable sources."""
    one = lambda s: np.ones_like(s)
    cosw = lambda s: np.cos(w * s)
    r = (poisson_square_separable(cosw, one, A * w * w, 1.0, x, y, 0.0, nmax)
         + poisson_square_separable(one, cosw, A * w * w, 1.0, x, y, 0.0, nmax))
    return A * (math.cos(w * x) + math.cos(w * y)) + r
