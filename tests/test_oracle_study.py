"""Pins of the oracle's study switches (CPU): other readings of three passages,
kept to measure their effect.  Off by default; the GPU path follows the
default readings (and offers the printed forms as the "printed" collision).

  q8_printed the printed closed forms of h_3..h_8 instead of the solve of the
             relaxation conditions: equal to the brute-force solve under reading
             B (test_oracle_collision.py); without forces the two coincide, with
             forces they differ.
  q6_minus8  the printed -8 in m^s'_8: changes only the K_8 component of the
             source, by (1 - omega_8 / 2) (-12) sigma'_00 K_8 / |K_8|^2.
  q11_lagged the pressure gradient of F_p from the previous step's p: the first
             step equals the default (no previous p yet) and later steps differ.
"""
import numpy as np

import bruteforce as bf
import oracle
from paper_1909_04166_amd import workloads as W

from test_oracle_collision import _rand_hydro


def test_q8_printed_differs_only_through_the_sources():
    """Without forces (and gbar carrying p, rho c^2 u as its own moments) the
    printed forms are the solve of the conditions; with forces they differ."""
    rng = np.random.default_rng(22)
    for _ in range(50):
        gbar, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, om = _rand_hydro(rng)
        g2 = gbar.copy()
        g2[0] += p - g2.sum()
        jx = rho / 3 * ux - (g2[1] - g2[3] + g2[5] - g2[6] - g2[7] + g2[8])
        jy = rho / 3 * uy - (g2[2] - g2[4] + g2[5] + g2[6] - g2[7] - g2[8])
        g2[1] += jx / 2; g2[3] -= jx / 2
        g2[2] += jy / 2; g2[4] -= jy / 2
        a = oracle.hydro_collide_study(g2, p, rho, p - rho / 3, ux, uy, 0, 0, 0, 0, om, q8_printed=True)
        b = oracle.hydro_collide(g2, p, rho, p - rho / 3, ux, uy, 0, 0, 0, 0, om)
        assert np.abs(a - b).max() <= 1e-13 * max(1.0, np.abs(b).max())
    gbar, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, om = _rand_hydro(rng)
    a = oracle.hydro_collide_study(gbar, p, rho, p - rho / 3, ux, uy, Ftx, Fty, Fpx, Fpy, om, q8_printed=True)
    b = oracle.hydro_collide(gbar, p, rho, p - rho / 3, ux, uy, Ftx, Fty, Fpx, Fpy, om)
    assert np.abs(a - b).max() > 1e-8


def test_q6_minus8_changes_only_the_K8_component():
    rng = np.random.default_rng(23)
    K = bf.basis_K()
    for printed in (False, True):
        for _ in range(100):
            gbar, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, om = _rand_hydro(rng)
            a = oracle.hydro_collide_study(gbar, p, rho, p - rho / 3, ux, uy, Ftx, Fty, Fpx, Fpy, om,
                                           q6_minus8=True, q8_printed=printed)
            b = oracle.hydro_collide_study(gbar, p, rho, p - rho / 3, ux, uy, Ftx, Fty, Fpx, Fpy, om,
                                           q8_printed=printed)
            s00 = Fpx * ux + Fpy * uy  # sigma'_00 = F_p . u
            expect = (1 - om[8] / 2) * (-8.0 - 4.0) * s00 * K[:, 8] / 36.0
            assert np.abs((a - b) - expect).max() <= 1e-14 * max(1.0, np.abs(b).max())


def test_q11_lagged_first_step_equal_then_differs():
    case, phi0 = W.droplet(48, 10.0, W=5.0, ratio=100.0)
    a = oracle.Oracle(case, phi0)
    b = oracle.Oracle(dict(case, oracle_q11_lagged=True), phi0)
    a.step(1)
    b.step(1)
    fa, ga = a.get_dist()
    fb, gb = b.get_dist()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    a.step(5)
    b.step(5)
    assert np.abs(a.get_dist()[1] - b.get_dist()[1]).max() > 1e-12


def test_printed_collision_name_selects_the_switch():
    case, phi0 = W.droplet(32, 8.0, W=5.0, ratio=100.0)
    assert oracle.params_from_case(dict(case, collision="printed")).q8_printed == 1
    assert oracle.params_from_case(case).q8_printed == 0
