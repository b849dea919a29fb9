"""The step kernel evaluates both collisions in closed form rather than as the
paper's cascade of moment changes (Secs. 4 and 5).  These CPU tests restate the
two closed forms in numpy and compare them with the oracle's step-by-step
cascade on random nodes: the identities the kernel rests on, checked without a
GPU.

- Phase field (rates 1 above first order): every central moment of order >= 2
  at its equilibrium, the two first-order central moments relaxed, so
  f~ = phi W(ex) W(ey) + a D(ex) V(ey) + b V(ex) D(ey).
- Hydrodynamics (rates 1 except the two shear rates): post-collision raw moments
  that depend on the incoming gbar only through pbar, j and the shear
  non-equilibria N, X, each times (1 - omega); the printed closed forms of the
  moment changes, and the solve of the conditions they come from (the collision
  of the cascaded pair) as those moments plus force terms."""
import numpy as np

import oracle

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def _axis(u):
    """Three-velocity weights at e = -1, 0, +1: W (mean u, central second moment
    1/3), D (moments 0, 1, 2u), V (mean u, central second moment 0)."""
    W = {-1: (1 / 3 + u * u - u) / 2, 0: 2 / 3 - u * u, 1: (1 / 3 + u * u + u) / 2}
    D = {-1: u - 0.5, 0: -2 * u, 1: u + 0.5}
    V = {-1: (u * u - u) / 2, 0: 1 - u * u, 1: (u * u + u) / 2}
    return W, D, V


def ace_closed(f, ux, uy, M, th, nx, ny, om):
    phi = f.sum()
    k10, k01 = (f * EX).sum(), (f * EY).sum()
    a = k10 + om * (phi * ux + M * th * nx - k10) - ux * phi
    b = k01 + om * (phi * uy + M * th * ny - k01) - uy * phi
    (Wx, Dx, Vx), (Wy, Dy, Vy) = _axis(ux), _axis(uy)
    return np.array([phi * Wx[i] * Wy[j] + a * Dx[i] * Vy[j] + b * Vx[i] * Dy[j]
                     for i, j in zip(EX, EY)])


def _from_raw(m):
    """D2Q9 distribution with raw moments m = (m00, m10, m01, m20, m02, m11, m21, m12, m22)."""
    m00, m10, m01, m20, m02, m11, m21, m12, m22 = m
    return np.array([m00 - m20 - m02 + m22,
                     (m10 + m20 - m12 - m22) / 2, (m01 + m02 - m21 - m22) / 2,
                     (-m10 + m20 + m12 - m22) / 2, (-m01 + m02 + m21 - m22) / 2,
                     (m11 + m21 + m12 + m22) / 4, (-m11 + m21 - m12 + m22) / 4,
                     (m11 - m21 - m12 + m22) / 4, (-m11 - m21 + m12 + m22) / 4])


def hydro_closed(g, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, om):
    c2 = 1 / 3
    pbar = p - 0.5 * (Fpx * ux + Fpy * uy)
    jx, jy = (g * EX).sum(), (g * EY).sum()
    e20, e02, e11 = (g * EX ** 2).sum(), (g * EY ** 2).sum(), (g * EX * EY).sum()
    G = Fpx * ux + Fpy * uy
    Sx, Sy = Ftx + Fpx, Fty + Fpy
    s20, s02, s11 = 2 * c2 * Sx * ux + c2 * G, 2 * c2 * Sy * uy + c2 * G, c2 * (Sx * uy + Sy * ux)
    N = (e20 - e02) - c2 * rho * (ux ** 2 - uy ** 2)
    X = e11 - c2 * rho * ux * uy
    nn, xx = (1 - om) * N, (1 - om) * X
    hw = 1 - om / 2
    T = 2 * c2 * p + c2 * rho * (ux ** 2 + uy ** 2) + 4 / 3 * G + c2 * (Ftx * ux + Fty * uy)
    Dd = c2 * rho * (ux ** 2 - uy ** 2) + nn + hw * (s20 - s02)
    m = [pbar + G, jx + c2 * Ftx, jy + c2 * Fty, (T + Dd) / 2, (T - Dd) / 2,
         c2 * rho * ux * uy + xx + hw * s11,
         c2 * rho * uy * (c2 + ux ** 2) + Fty / 9 + uy * nn / 2 + 2 * ux * xx,
         c2 * rho * ux * (c2 + uy ** 2) + Ftx / 9 - ux * nn / 2 + 2 * uy * xx,
         p / 9 + rho * (ux ** 2 + uy ** 2) / 9 + rho * ux ** 2 * uy ** 2 / 3 + 2 * G / 9
         - (ux ** 2 - uy ** 2) * nn / 2 + 4 * ux * uy * xx]
    return _from_raw(m)


def test_phase_field_closed_form_equals_cascade():
    rng = np.random.default_rng(11)
    worst = 0.0
    for _ in range(500):
        f = rng.uniform(-0.05, 0.5, 9)
        ux, uy = rng.uniform(-0.15, 0.15, 2)
        M, th, ang, om = rng.uniform(0, 0.1), rng.uniform(0, 1), rng.uniform(0, 2 * np.pi), rng.uniform(0.3, 1.95)
        ref = oracle.ace_collide(f, f.sum(), ux, uy, M, th, np.cos(ang), np.sin(ang), [1.0, om, om] + [1.0] * 6)
        got = ace_closed(f, ux, uy, M, th, np.cos(ang), np.sin(ang), om)
        worst = max(worst, np.abs(ref - got).max())
    assert worst <= 1e-14


def test_hydrodynamic_closed_form_equals_cascade():
    """The kernel's closed form of the printed moment changes (the printed option)
    against the oracle's printed cascade: random pre-collision gbar, u, rho up to
    1000 and forces, with p = pbar + F_p.u / 2 as the step computes it; the closed
    form takes pbar back from p."""
    rng = np.random.default_rng(12)
    worst = 0.0
    for _ in range(500):
        rho = float(np.exp(rng.uniform(0, np.log(1000))))
        g = rng.normal(scale=0.05, size=9)
        ux, uy = rng.uniform(-0.1, 0.1, 2)
        Ftx, Fty, Fpx, Fpy = rng.normal(scale=1e-3, size=4)
        p = g.sum() + 0.5 * (Fpx * ux + Fpy * uy)  # p = pbar + F_p.u / 2, pbar = sum gbar
        om = rng.uniform(0.3, 1.95)
        rates = [1.0] * 4 + [om, om] + [1.0] * 3
        ref = oracle.hydro_collide_study(g, p, rho, p - rho / 3, ux, uy, Ftx, Fty, Fpx, Fpy, rates,
                                         q8_printed=True)
        got = hydro_closed(g, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, om)
        worst = max(worst, np.abs(ref - got).max() / max(1.0, np.abs(ref).max()))
    assert worst <= 1e-12


def hydro_solved_closed(g, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, om):
    """The kernel's closed form of the collision (h_3..h_8 solve the relaxation
    conditions as stated): the printed form's raw moments with the shear
    non-equilibria taken about u (N', X') and without the pure force terms
    (2/3) G, c^4 F_ty, c^4 F_tx and 2 c^4 G."""
    c2 = 1 / 3
    pbar = p - 0.5 * (Fpx * ux + Fpy * uy)
    jx, jy = (g * EX).sum(), (g * EY).sum()
    e20, e02, e11 = (g * EX ** 2).sum(), (g * EY ** 2).sum(), (g * EX * EY).sum()
    G = Fpx * ux + Fpy * uy
    Sx, Sy = Ftx + Fpx, Fty + Fpy
    s20, s02, s11 = 2 * c2 * Sx * ux + c2 * G, 2 * c2 * Sy * uy + c2 * G, c2 * (Sx * uy + Sy * ux)
    N = (e20 - e02) - c2 * rho * (ux ** 2 - uy ** 2) + c2 * (Ftx * ux - Fty * uy) - (ux ** 2 - uy ** 2) * G / 2
    X = e11 - c2 * rho * ux * uy + c2 * (Ftx * uy + Fty * ux) / 2 - ux * uy * G / 2
    nn, xx = (1 - om) * N, (1 - om) * X
    hw = 1 - om / 2
    T = 2 * c2 * p + c2 * rho * (ux ** 2 + uy ** 2) + 2 / 3 * G + c2 * (Ftx * ux + Fty * uy)
    Dd = c2 * rho * (ux ** 2 - uy ** 2) + nn + hw * (s20 - s02)
    m = [pbar + G, jx + c2 * Ftx, jy + c2 * Fty, (T + Dd) / 2, (T - Dd) / 2,
         c2 * rho * ux * uy + xx + hw * s11,
         c2 * rho * uy * (c2 + ux ** 2) + uy * nn / 2 + 2 * ux * xx,
         c2 * rho * ux * (c2 + uy ** 2) - ux * nn / 2 + 2 * uy * xx,
         p / 9 + rho * (ux ** 2 + uy ** 2) / 9 + rho * ux ** 2 * uy ** 2 / 3
         - (ux ** 2 - uy ** 2) * nn / 2 + 4 * ux * uy * xx]
    return _from_raw(m)


def test_hydrodynamic_solved_closed_form_equals_numerical_solve():
    """The kernel's closed form of the collision against the oracle's numerical
    solve of the relaxation conditions (itself pinned to the brute-force solve):
    random gbar, rho up to 1000 and forces, with u and p as the step
    computes them from gbar (u = (j + c^2 F_t / 2) / (rho c^2), p = pbar + F_p.u / 2)."""
    rng = np.random.default_rng(13)
    worst = 0.0
    for _ in range(500):
        rho = float(np.exp(rng.uniform(0, np.log(1000))))
        g = rng.normal(scale=0.05, size=9)
        Ftx, Fty, Fpx, Fpy = rng.normal(scale=1e-3, size=4)
        ux = ((g * EX).sum() + Ftx / 6) / (rho / 3)
        uy = ((g * EY).sum() + Fty / 6) / (rho / 3)
        if max(abs(ux), abs(uy)) > 0.2:
            continue
        p = g.sum() + 0.5 * (Fpx * ux + Fpy * uy)
        om = rng.uniform(0.3, 1.95)
        rates = [1.0] * 4 + [om, om] + [1.0] * 3
        ref = oracle.hydro_collide(g, p, rho, p - rho / 3, ux, uy, Ftx, Fty, Fpx, Fpy, rates)
        got = hydro_solved_closed(g, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, om)
        worst = max(worst, np.abs(ref - got).max() / max(1.0, np.abs(ref).max()))
    assert worst <= 1e-12, worst
