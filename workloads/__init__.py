"""Seeded synthetic inputs shared by the CPU oracle tests and the GPU path.

This module only builds initial data (numpy float64 arrays) and problem
descriptions.  It holds none of the scheme's arithmetic: no fluxes, no
reconstruction, no time stepping.  Random numbers come from numpy's PCG64
(``numpy.random.default_rng(seed)``).

Grid convention (Sec. 2.1, Eq. 1DHCL): nodes x_j = x_L + (j-1) h, h = (x_R-x_L)/N.
A periodic line keeps the N nodes x_1..x_N (x_{N+1} is x_1 again); an outflow
line uses the same N nodes.

Conserved Euler variables are (rho, rho*u, [rho*v,] rho*e) with the specific
total energy e = p/(rho (gamma-1)) + |u|^2/2 (Sec. 4.3, 4.4); arrays are laid
out [variable][y][x], x fastest.
"""
import math

import numpy as np

GAMMA = 1.4


def nodes(x_left, x_right, n):
    """x_j = x_L + (j-1) h, j = 1..n, h = (x_R - x_L)/n."""
    h = (x_right - x_left) / n
    return x_left + h * np.arange(n, dtype=np.float64), h


def conserved_1d(rho, u, p, gamma=GAMMA):
    rho = np.asarray(rho, np.float64)
    u = np.asarray(u, np.float64)
    p = np.asarray(p, np.float64)
    E = p / (gamma - 1.0) + 0.5 * rho * u * u
    return np.ascontiguousarray(np.stack([rho, rho * u, E]))


def conserved_2d(rho, u, v, p, gamma=GAMMA):
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.ascontiguousarray(np.stack([rho, rho * u, rho * v, E]).astype(np.float64))


# --------------------------------------------------------------------------
# Scalar problems
# --------------------------------------------------------------------------

def sin_power(alpha, lam=1.0, n=100):
    """u0 = lam * sin^alpha(pi x) on [-1, 1], periodic (Sec. 4.1, convergence test)."""
    x, h = nodes(-1.0, 1.0, n)
    return x, h, lam * np.sin(np.pi * x) ** alpha


def burgers_sin3(lam=1.0, n=64):
    """u0 = lam * (1 + 0.5 sin^3(pi x)) on [0, 2], periodic (Sec. 4.2)."""
    x, h = nodes(0.0, 2.0, n)
    return x, h, lam * (1.0 + 0.5 * np.sin(np.pi * x) ** 3)


def advection_sines_step(seed, n=200):
    """Sum of three seeded sines plus one seeded step on [-1, 1], periodic.

    u0 = sum_i A_i sin(pi k_i x + phi_i) + H * 1[a <= x < b] with k_i in {1..4},
    A_i ~ U(0.2, 1), phi_i ~ U(0, 2 pi), H ~ U(0.5, 1), a < b ~ U(-1, 1), b-a >= 0.1.
    """
    rng = np.random.default_rng(seed)
    k = rng.integers(1, 5, size=3)
    A = rng.uniform(0.2, 1.0, size=3)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=3)
    H = rng.uniform(0.5, 1.0)
    while True:
        a, b = np.sort(rng.uniform(-1.0, 1.0, size=2))
        if b - a >= 0.1:
            break
    x, h = nodes(-1.0, 1.0, n)
    u = sum(A[i] * np.sin(np.pi * k[i] * x + phi[i]) for i in range(3))
    u = u + H * ((x >= a) & (x < b))
    return x, h, np.ascontiguousarray(u)


def smooth_sines(seed, x, period, nterms=3, kmax=4):
    """Seeded sum of `nterms` sines periodic on `period`, scaled to max |s| = 1."""
    rng = np.random.default_rng(seed)
    k = rng.integers(1, kmax + 1, size=nterms)
    A = rng.uniform(0.2, 1.0, size=nterms)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=nterms)
    s = sum(A[i] * np.sin(2.0 * np.pi * k[i] * x / period + phi[i]) for i in range(nterms))
    return s / np.max(np.abs(s))


# --------------------------------------------------------------------------
# 1D Euler
# --------------------------------------------------------------------------

def euler1d_lax(n=200):
    """Lax shock tube on [0, 2], step at x = 1, outflow (Sec. 4.3)."""
    x, h = nodes(0.0, 2.0, n)
    left = x < 1.0
    rho = np.where(left, 0.445, 0.5)
    u = np.where(left, 0.698, 0.0)
    p = np.where(left, 3.528, 0.571)
    return x, h, conserved_1d(rho, u, p)


def euler1d_riemann_perturbed(seed, n=4096, gamma=GAMMA):
    """Seeded Riemann step with a multiplicative density wave on the right.

    Domain [0, 2], step at x = 1, outflow.  rho_L, p_L, rho_R, p_R ~ U(0.1, 1),
    u = 0, and on the right rho = rho_R (1 + 0.2 sin(k x)) with k in {3..8}.
    """
    rng = np.random.default_rng(seed)
    rho_l, p_l, rho_r, p_r = rng.uniform(0.1, 1.0, size=4)
    k = int(rng.integers(3, 9))
    x, h = nodes(0.0, 2.0, n)
    left = x < 1.0
    rho = np.where(left, rho_l, rho_r * (1.0 + 0.2 * np.sin(k * x)))
    p = np.where(left, p_l, p_r)
    u = np.zeros_like(x)
    return x, h, conserved_1d(rho, u, p, gamma)


def euler1d_smooth_periodic(seed, n=8192, gamma=GAMMA):
    """Smooth periodic state on [0, 1]: rho = 1 + 0.1 s1, u = 0, p = 1 + 0.1 s2."""
    x, h = nodes(0.0, 1.0, n)
    s1 = smooth_sines(seed * 2 + 0, x, 1.0)
    s2 = smooth_sines(seed * 2 + 1, x, 1.0)
    rho = 1.0 + 0.1 * s1
    p = 1.0 + 0.1 * s2
    return x, h, conserved_1d(rho, np.zeros_like(x), p, gamma)


def density_target(seed, n=8192):
    """Seeded smooth density target on [0, 1] for the adjoint loss."""
    x, _ = nodes(0.0, 1.0, n)
    return 1.0 + 0.1 * smooth_sines(seed + 1000, x, 1.0)


def batched_problems(seed, nprob=4096, nmin=256, nmax=16384, orders=(7, 9, 13, 17)):
    """Seeded list of independent 1D Euler problems of uneven sizes and orders.

    Returns a list of dicts {n, order, h, U}; each problem's data follows
    euler1d_riemann_perturbed with its own child seed.
    """
    ss = np.random.SeedSequence(seed)
    children = ss.spawn(nprob)
    out = []
    for child in children:
        rng = np.random.default_rng(child)
        n = int(rng.integers(nmin, nmax + 1))
        order = int(orders[int(rng.integers(0, len(orders)))])
        sub = int(rng.integers(0, 2**31 - 1))
        _, h, U = euler1d_riemann_perturbed(sub, n)
        out.append({"n": n, "order": order, "h": h, "U": U})
    return out


def batched_problems_2d(seed, nprob=256, nmin=32, nmax=192, orders=(7, 9, 13, 17)):
    """Seeded list of independent 2D Euler problems of uneven sizes and orders.

    Returns a list of dicts {nx, ny, order, hx, hy, U}; each problem's data
    follows euler2d_quadrants_vortices with its own child seed.
    """
    ss = np.random.SeedSequence(seed)
    out = []
    for child in ss.spawn(nprob):
        rng = np.random.default_rng(child)
        nx = int(rng.integers(nmin, nmax + 1))
        ny = int(rng.integers(nmin, nmax + 1))
        order = int(orders[int(rng.integers(0, len(orders)))])
        sub = int(rng.integers(0, 2**31 - 1))
        (x, y, hx, hy), U = euler2d_quadrants_vortices(sub, nx, ny)
        out.append({"nx": nx, "ny": ny, "order": order, "hx": hx, "hy": hy, "U": U})
    return out


# --------------------------------------------------------------------------
# 2D Euler
# --------------------------------------------------------------------------

RP_CONFIGS = {
    # (rho, u, v, p) in the quadrants [-1,0]x[-1,0], [-1,0]x[0,1], [0,1]x[0,1],
    # [0,1]x[-1,0] (Sec. 4.4.1, first and second configurations).
    1: ((0.138, 1.206, 1.206, 0.029), (0.5323, 1.206, 0.0, 0.3),
        (1.5, 0.0, 0.0, 1.5), (0.5323, 0.0, 1.206, 0.3)),
    2: ((1.0, -0.75, 0.5, 1.0), (2.0, 0.75, 0.5, 1.0),
        (1.0, 0.75, -0.5, 1.0), (3.0, -0.75, -0.5, 1.0)),
}


def _quadrant_fields(X, Y, states):
    q_ll = (X < 0) & (Y < 0)
    q_lu = (X < 0) & (Y >= 0)
    q_uu = (X >= 0) & (Y >= 0)
    q_ul = (X >= 0) & (Y < 0)
    out = []
    for var in range(4):
        f = np.zeros_like(X)
        for mask, st in zip((q_ll, q_lu, q_uu, q_ul), states):
            f = np.where(mask, st[var], f)
        out.append(f)
    return out


def euler2d_riemann(config, nx=128, ny=None, gamma=GAMMA):
    """Four-quadrant Riemann problem on [-1, 1]^2 (Sec. 4.4.1)."""
    ny = nx if ny is None else ny
    x, hx = nodes(-1.0, 1.0, nx)
    y, hy = nodes(-1.0, 1.0, ny)
    X, Y = np.meshgrid(x, y)
    rho, u, v, p = _quadrant_fields(X, Y, RP_CONFIGS[config])
    return (x, y, hx, hy), conserved_2d(rho, u, v, p, gamma)


def euler2d_quadrants_vortices(seed, nx=2048, ny=None, nvort=8, gamma=GAMMA):
    """Seeded four-quadrant states plus isentropic vortices on [-1, 1]^2.

    Quadrants split at (0, 0): rho, p ~ U(0.1, 1.5), u, v ~ U(-0.8, 0.8).
    Each vortex (strength eps ~ U(1, 5), radius R ~ U(0.05, 0.15), centre
    ~ U(-0.8, 0.8)^2) adds the velocity sqrt(T) eps/(2 pi) e^{(1-s^2)/2} (-dy, dx)/R
    and multiplies T = p/rho by 1 - (gamma-1) eps^2 e^{1-s^2} / (8 gamma pi^2)
    with s = r/R; rho and p follow isentropically (rho ~ T^{1/(gamma-1)}).
    The factor stays >= 0.75 for eps <= 5, so rho, p > 0.
    """
    ny = nx if ny is None else ny
    rng = np.random.default_rng(seed)
    states = [tuple(rng.uniform(0.1, 1.5, size=1)) + tuple(rng.uniform(-0.8, 0.8, size=2))
              + tuple(rng.uniform(0.1, 1.5, size=1)) for _ in range(4)]
    vort = [(rng.uniform(1.0, 5.0), rng.uniform(0.05, 0.15), rng.uniform(-0.8, 0.8),
             rng.uniform(-0.8, 0.8)) for _ in range(nvort)]
    x, hx = nodes(-1.0, 1.0, nx)
    y, hy = nodes(-1.0, 1.0, ny)
    X, Y = np.meshgrid(x, y)
    rho, u, v, p = _quadrant_fields(X, Y, states)
    T = p / rho
    ratio = np.ones_like(X)
    du = np.zeros_like(X)
    dv = np.zeros_like(X)
    for eps, R, xc, yc in vort:
        dx = (X - xc) / R
        dy = (Y - yc) / R
        s2 = dx * dx + dy * dy
        amp = eps / (2.0 * math.pi) * np.exp(0.5 * (1.0 - s2)) * np.sqrt(T)
        du += -amp * dy
        dv += amp * dx
        ratio *= 1.0 - (gamma - 1.0) * eps * eps * np.exp(1.0 - s2) / (8.0 * gamma * math.pi ** 2)
    rho = rho * ratio ** (1.0 / (gamma - 1.0))
    p = p * ratio ** (gamma / (gamma - 1.0))
    u = u + du
    v = v + dv
    return (x, y, hx, hy), conserved_2d(rho, u, v, p, gamma)


def euler2d_rayleigh_taylor(nx=64, ny=256, gamma=5.0 / 3.0):
    """Rayleigh-Taylor initial data on [0, 0.25] x [0, 1] (Sec. 4.4): heavy
    fluid (rho = 2, p = 2y + 1) below y = 1/2, light (rho = 1, p = y + 3/2)
    above, u = 0, v = -0.025 c cos(8 pi x) with c the local sound speed.
    In hydrostatic balance with the source [0, 0, rho, rho v] (g = 1).
    Returns ((x, y, hx, hy), U)."""
    x, hx = nodes(0.0, 0.25, nx)
    y, hy = nodes(0.0, 1.0, ny)
    X, Y = np.meshgrid(x, y)
    low = Y < 0.5
    rho = np.where(low, 2.0, 1.0)
    p = np.where(low, 2.0 * Y + 1.0, Y + 1.5)
    c = np.sqrt(gamma * p / rho)
    v = -0.025 * c * np.cos(8.0 * math.pi * X)
    return (x, y, hx, hy), conserved_2d(rho, np.zeros_like(X), v, p, gamma)
