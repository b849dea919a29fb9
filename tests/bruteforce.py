"""Independent brute-force derivations used to pin the oracle's closed forms.

Nothing here retypes the paper's closed-form results.  The continuous moments
come from Gauss-Hermite quadrature of the Maxwellian and source terms as
*defined* in Sec. 3 (Eqs. Maxwelldistribution, modifiedeqm, sourcetotalforce,
sourcenetgradientpressureforce); the discrete collision results come from
numerically solving the central-moment relaxation conditions stated in Secs. 4
and 5 with numpy.linalg.solve.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial.hermite_e import hermegauss

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)
CS2 = 1.0 / 3.0

# the nine moment orders supported by D2Q9, in the order used below
MN = [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)]
IDX = {mn: k for k, mn in enumerate(MN)}


def basis_K() -> np.ndarray:
    """Columns K_0..K_8 of the orthogonal basis built from e_x, e_y (Sec. 4)."""
    one = np.ones(9)
    ex, ey = EX, EY
    cols = [one, ex, ey, 3 * (ex**2 + ey**2) - 4 * one, ex**2 - ey**2, ex * ey,
            -3 * ex**2 * ey + 2 * ey, -3 * ex * ey**2 + 2 * ex,
            9 * ex**2 * ey**2 - 6 * (ex**2 + ey**2) + 4 * one]
    return np.stack(cols, axis=1)


def raw_matrix() -> np.ndarray:
    """Rows e_x^m e_y^n: maps a distribution to its nine raw moments."""
    return np.stack([EX**m * EY**n for (m, n) in MN], axis=0)


def central_matrix(ux: float, uy: float) -> np.ndarray:
    """Rows (e_x - u_x)^m (e_y - u_y)^n: maps a distribution to its central moments."""
    return np.stack([(EX - ux) ** m * (EY - uy) ** n for (m, n) in MN], axis=0)


# ---------------------------------------------------------- continuous moments

_XI, _WQ = hermegauss(16)  # exact for polynomials of degree <= 31 against exp(-x^2/2)


def _gauss2(fun, ux, uy, c2):
    """Integral over R^2 of fun(xi_x, xi_y) * N(xi; u, c2 I) (unit-mass Gaussian)."""
    c = np.sqrt(c2)
    X = ux + c * _XI[:, None]
    Y = uy + c * _XI[None, :]
    W = (_WQ[:, None] * _WQ[None, :]) / (2 * np.pi)
    return float(np.sum(W * fun(X, Y)))


def maxwell_central(rho, ux, uy, m, n, c2=CS2, at_rest=False):
    """Central moment about u of f^M(rho, u) (or of f^M(rho, 0) if at_rest),
    the Maxwellian of Eq. Maxwelldistribution."""
    cx, cy = (0.0, 0.0) if at_rest else (ux, uy)
    return rho * _gauss2(lambda X, Y: (X - ux) ** m * (Y - uy) ** n, cx, cy, c2)


def geq_central(p, rho, ux, uy, m, n):
    """Central moments of g^eq = c^2 f^M(rho,u) + psi f^M(rho,0)/rho (Eq. modifiedeqm)."""
    psi = p - rho * CS2
    return CS2 * maxwell_central(rho, ux, uy, m, n) + psi * maxwell_central(1.0, ux, uy, m, n, at_rest=True)


def source_central(rho, ux, uy, Ftx, Fty, Fpx, Fpy, m, n):
    """Central moments of S = S^t + S^p (Eqs. sourcetotalforce, sourcenetgradientpressureforce)."""
    def St(X, Y):
        return ((X - ux) * Ftx + (Y - uy) * Fty) * (X - ux) ** m * (Y - uy) ** n

    c = np.sqrt(CS2)
    gt = _gauss2(St, ux, uy, CS2)  # f^M(rho,u)/rho is a unit-mass Gaussian at u
    # S^p = (xi - u).F_p [f^M(rho,u) - f^M(rho,0)]/rho
    gp = _gauss2(lambda X, Y: ((X - ux) * Fpx + (Y - uy) * Fpy) * (X - ux) ** m * (Y - uy) ** n, ux, uy, CS2) \
        - _gauss2(lambda X, Y: ((X - ux) * Fpx + (Y - uy) * Fpy) * (X - ux) ** m * (Y - uy) ** n, 0.0, 0.0, CS2)
    del c
    return gt, gp


def source_raw_moments(rho, ux, uy, Ftx, Fty, Fpx, Fpy):
    """Raw source moments sigma'_mn: continuous central moments of the two sources,
    those above second order dealiased to zero, binomially transformed to raw
    moments, whose third and fourth orders are then also set to zero."""
    cen = np.zeros(9)
    for (m, n), k in IDX.items():
        if m + n <= 2:
            gt, gp = source_central(rho, ux, uy, Ftx, Fty, Fpx, Fpy, m, n)
            cen[k] = gt + gp
    # central -> raw via a distribution that has these central moments
    S = np.linalg.solve(central_matrix(ux, uy), cen)
    raw = raw_matrix() @ S
    for mn in [(2, 1), (1, 2), (2, 2)]:
        raw[IDX[mn]] = 0.0
    return raw


# ------------------------------------------------------------ collision solves

def _higher_rows(C: np.ndarray) -> np.ndarray:
    """Rows of the six non-conserved relaxation conditions: trace 20+02,
    difference 20-02, 11, 21, 12, 22."""
    return np.stack([C[IDX[(2, 0)]] + C[IDX[(0, 2)]], C[IDX[(2, 0)]] - C[IDX[(0, 2)]],
                     C[IDX[(1, 1)]], C[IDX[(2, 1)]], C[IDX[(1, 2)]], C[IDX[(2, 2)]]])


def _higher_vals(v: np.ndarray) -> np.ndarray:
    return np.array([v[IDX[(2, 0)]] + v[IDX[(0, 2)]], v[IDX[(2, 0)]] - v[IDX[(0, 2)]],
                     v[IDX[(1, 1)]], v[IDX[(2, 1)]], v[IDX[(1, 2)]], v[IDX[(2, 2)]]])


def hydro_expected(gbar, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, om, reading_B=True):
    """Post-collision gbar from the conditions of Sec. 4 solved numerically.

    * 0th/1st-order changes: sum (K h) = (w0/2) sigma'_00, sum (K h) e = (w/2) sigma'_10/01.
    * higher orders: the central moments of the change equal
      omega (eta^eq - eta_bar) with eta^eq from Gauss-Hermite quadrature.
      reading_B: the 0th/1st raw moments of gbar entering eta_bar are replaced by
      (p, rho c^2 u), and only K_3..K_8 carry the higher-order relaxation.
    * delta g^s = (K^T)^{-1} (I - Lambda/2) K^T S with S the distribution that
      has the raw moments sigma'.
    """
    K = basis_K()
    Mr = raw_matrix()
    C = central_matrix(ux, uy)
    om = np.asarray(om, dtype=np.float64)
    sig = source_raw_moments(rho, ux, uy, Ftx, Fty, Fpx, Fpy)
    S = np.linalg.solve(Mr, sig)
    dgs = np.linalg.solve(K.T, (1.0 - 0.5 * om) * (K.T @ S))

    raw = Mr @ np.asarray(gbar, dtype=np.float64)
    if reading_B:
        raw = raw.copy()
        raw[IDX[(0, 0)]] = p
        raw[IDX[(1, 0)]] = rho * CS2 * ux
        raw[IDX[(0, 1)]] = rho * CS2 * uy
    gB = np.linalg.solve(Mr, raw)
    eta = C @ gB
    eq = np.array([geq_central(p, rho, ux, uy, m, n) for (m, n) in MN])
    rates = np.array([om[3], om[4], om[5], om[6], om[7], om[8]])
    target = rates * (_higher_vals(eq) - _higher_vals(eta))

    h = np.zeros(9)
    h[0] = 0.5 * om[0] * sig[IDX[(0, 0)]] / 9.0
    h[1] = 0.5 * om[1] * sig[IDX[(1, 0)]] / 6.0
    h[2] = 0.5 * om[2] * sig[IDX[(0, 1)]] / 6.0
    A = _higher_rows(C) @ K[:, 3:]
    if reading_B:
        h[3:] = np.linalg.solve(A, target)
    else:
        rhs = target - _higher_rows(C) @ (K[:, :3] @ h[:3])
        h[3:] = np.linalg.solve(A, rhs)
    return np.asarray(gbar) + K @ h + dgs


def ace_expected(f, ux, uy, M, theta, nx, ny, om):
    """Post-collision f from the central-moment relaxation conditions of Sec. 5
    solved numerically: zeroth moment conserved; first-order central moments
    relax to M theta n; higher ones to the central moments of the Gaussian with
    mass phi (computed by quadrature)."""
    K = basis_K()
    C = central_matrix(ux, uy)
    f = np.asarray(f, dtype=np.float64)
    om = np.asarray(om, dtype=np.float64)
    phi = f.sum()
    kap = C @ f
    eq = np.array([maxwell_central(phi, ux, uy, m, n) for (m, n) in MN])
    eq[IDX[(1, 0)]] = M * theta * nx
    eq[IDX[(0, 1)]] = M * theta * ny
    rows = [C[IDX[(0, 0)]], C[IDX[(1, 0)]], C[IDX[(0, 1)]]] + list(_higher_rows(C))
    rhs = [0.0, om[1] * (eq[IDX[(1, 0)]] - kap[IDX[(1, 0)]]),
           om[2] * (eq[IDX[(0, 1)]] - kap[IDX[(0, 1)]])]
    rates = np.array([om[3], om[4], om[5], om[6], om[7], om[8]])
    rhs += list(rates * (_higher_vals(eq) - _higher_vals(kap)))
    A = np.stack(rows) @ K
    gh = np.linalg.solve(A, np.array(rhs))
    return f + K @ gh
