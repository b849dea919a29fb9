"""Pins of the oracle's per-node collision operators (Secs. 4 and 5).

Expected values come from tests/bruteforce.py: Gauss-Hermite moments of the
Maxwellian and of the sources as defined in Sec. 3, and numerical solves of the
relaxation conditions of Secs. 4-5.  A dropped term, a wrong sign or index in
any closed form of the oracle fails one of these.
"""
import numpy as np
import pytest

import bruteforce as bf
import oracle

NORMS = np.array([9, 6, 6, 36, 4, 4, 12, 12, 36], dtype=float)


def test_basis_orthogonal_with_norms():
    K = bf.basis_K()
    G = K.T @ K
    assert np.allclose(G, np.diag(NORMS), atol=0, rtol=0)


def _rand_hydro(rng, scale_u=0.1, scale_f=0.02):
    gbar = rng.normal(size=9) * 0.1
    p = float(rng.normal() * 0.1)
    rho = float(np.exp(rng.uniform(0, np.log(1000))))
    ux, uy = rng.normal(size=2) * scale_u
    Ftx, Fty, Fpx, Fpy = rng.normal(size=4) * scale_f
    om = rng.uniform(0.2, 1.95, size=9)
    return gbar, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, om


def test_hydro_matches_central_moment_solve():
    """The collision (h_3..h_8 solved from the relaxation conditions of Sec. 4 with
    gbar's own central moments, h_0..h_2 carried into them, plus delta g^s)
    equals the brute-force solve of the same conditions, whose equilibrium and
    source moments come from quadrature of their definitions."""
    rng = np.random.default_rng(11)
    worst = 0.0
    for _ in range(400):
        gbar, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, om = _rand_hydro(rng)
        got = oracle.hydro_collide(gbar, p, rho, p - rho / 3, ux, uy, Ftx, Fty, Fpx, Fpy, om)
        exp = bf.hydro_expected(gbar, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, om, reading_B=False)
        worst = max(worst, np.abs(got - exp).max() / max(1.0, np.abs(exp).max()))
    assert worst <= 1e-12, worst


def test_printed_forms_match_central_moment_solve_reading_B():
    """The printed h_0..h_8 (kept as a study switch) + delta g^s equal the
    numerical solution of the relaxation conditions when the 0th/1st raw moments
    are (p, rho c^2 u) and h_0..h_2 are not carried into the higher moments
    (reading B): that is what the closed forms leave out."""
    rng = np.random.default_rng(11)
    worst = 0.0
    for _ in range(400):
        gbar, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, om = _rand_hydro(rng)
        got = oracle.hydro_collide_study(gbar, p, rho, p - rho / 3, ux, uy, Ftx, Fty, Fpx, Fpy, om,
                                         q8_printed=True)
        exp = bf.hydro_expected(gbar, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, om)
        worst = max(worst, np.abs(got - exp).max() / max(1.0, np.abs(exp).max()))
    assert worst <= 1e-13


def test_hydro_exact_without_sources():
    """With F_t = F_p = 0 and (p, u) taken from gbar itself, the collision and the
    printed forms both are the exact central-moment relaxation."""
    rng = np.random.default_rng(12)
    for _ in range(200):
        gbar, _, rho, *_rest = _rand_hydro(rng)
        om = rng.uniform(0.2, 1.95, size=9)
        p = gbar.sum()
        ux, uy = gbar @ bf.EX / (rho / 3), gbar @ bf.EY / (rho / 3)
        got = oracle.hydro_collide(gbar, p, rho, p - rho / 3, ux, uy, 0, 0, 0, 0, om)
        printed = oracle.hydro_collide_study(gbar, p, rho, p - rho / 3, ux, uy, 0, 0, 0, 0, om, q8_printed=True)
        exp = bf.hydro_expected(gbar, p, rho, ux, uy, 0, 0, 0, 0, om, reading_B=False)
        assert np.abs(got - exp).max() <= 1e-13 * max(1.0, np.abs(exp).max())
        assert np.abs(printed - exp).max() <= 1e-13 * max(1.0, np.abs(exp).max())


def test_hydro_collision_invariants():
    """sum(g~ - g) = F_p.u and sum(g~ - g) e = c^2 F_t, for any omega."""
    rng = np.random.default_rng(13)
    for _ in range(200):
        gbar, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, om = _rand_hydro(rng)
        d = oracle.hydro_collide(gbar, p, rho, p - rho / 3, ux, uy, Ftx, Fty, Fpx, Fpy, om) - gbar
        assert abs(d.sum() - (Fpx * ux + Fpy * uy)) <= 1e-14
        assert abs(d @ bf.EX - Ftx / 3) <= 1e-14
        assert abs(d @ bf.EY - Fty / 3) <= 1e-14


def test_hydro_equilibrium_is_fixed_point():
    """A distribution whose central moments equal the matched equilibria (with no
    sources) is left unchanged by the collision."""
    rng = np.random.default_rng(14)
    for _ in range(50):
        p = float(rng.normal() * 0.01)
        rho = float(rng.uniform(1, 1000))
        ux, uy = rng.normal(size=2) * 0.05
        eq = np.array([bf.geq_central(p, rho, ux, uy, m, n) for (m, n) in bf.MN])
        geq = np.linalg.solve(bf.central_matrix(ux, uy), eq)
        om = rng.uniform(0.2, 1.95, size=9)
        got = oracle.hydro_collide(geq, p, rho, p - rho / 3, ux, uy, 0, 0, 0, 0, om)
        assert np.abs(got - geq).max() <= 1e-12 * max(1.0, np.abs(geq).max())


def _rand_ace(rng):
    f = rng.uniform(0, 0.3, size=9)
    ux, uy = rng.normal(size=2) * 0.1
    M = float(rng.uniform(0.005, 0.1))
    theta = float(rng.uniform(0, 0.3))
    n = rng.normal(size=2)
    n /= np.linalg.norm(n)
    om = rng.uniform(0.2, 1.95, size=9)
    return f, ux, uy, M, theta, n, om


def test_ace_matches_central_moment_solve():
    """Printed g_0..g_8 (g_7 read with u_x) equal the exact relaxation of all nine
    central moments to the equilibria with the sharpening flux M theta n."""
    rng = np.random.default_rng(21)
    for _ in range(400):
        f, ux, uy, M, th, n, om = _rand_ace(rng)
        got = oracle.ace_collide(f, f.sum(), ux, uy, M, th, n[0], n[1], om)
        exp = bf.ace_expected(f, ux, uy, M, th, n[0], n[1], om)
        assert np.abs(got - exp).max() <= 1e-13 * max(1.0, np.abs(exp).max())


def test_ace_invariants():
    rng = np.random.default_rng(22)
    for _ in range(200):
        f, ux, uy, M, th, n, om = _rand_ace(rng)
        phi = f.sum()
        d = oracle.ace_collide(f, phi, ux, uy, M, th, n[0], n[1], om) - f
        assert abs(d.sum()) <= 1e-14
        k10 = f @ bf.EX
        assert abs(d @ bf.EX - om[1] * (phi * ux + M * th * n[0] - k10)) <= 1e-14


def test_printed_m8_coefficient_is_inconsistent():
    """Documents the reading of the m^s'_8 coefficient: <K_8|S> has +4 sigma'_00.
    The brute force derives it from K_8 itself; -8 would not project onto K_8."""
    K = bf.basis_K()
    Mr = bf.raw_matrix()
    # coefficients of <K_8|S> on the raw moments: K_8 = M^T c  ->  c = M^{-T} K_8
    c = np.linalg.solve(Mr.T, K[:, 8])
    idx = bf.IDX
    assert np.isclose(c[idx[(0, 0)]], 4.0)
    assert np.isclose(c[idx[(2, 0)]], -6.0) and np.isclose(c[idx[(0, 2)]], -6.0)
    assert np.isclose(c[idx[(2, 2)]], 9.0)
