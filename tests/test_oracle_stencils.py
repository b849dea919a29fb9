"""Pins of the isotropic D2Q9 finite-difference stencils used for grad phi,
div n, grad p and lap phi (Sec. 4, text after Eq. fluidviscosity)."""
import numpy as np

import bruteforce as bf
import oracle


def _samples(fun, x0=0.3, y0=-0.7):
    return np.array([fun(x0 + ex, y0 + ey) for ex, ey in zip(bf.EX, bf.EY)])


def test_gradient_exact_on_quadratics():
    rng = np.random.default_rng(1)
    for _ in range(50):
        a, b, c, d, e, f = rng.normal(size=6)
        fun = lambda x, y: a + b * x + c * y + d * x * x + e * x * y + f * y * y
        x0, y0 = 0.3, -0.7
        gx, gy = oracle.grad9(_samples(fun, x0, y0))
        assert abs(gx - (b + 2 * d * x0 + e * y0)) < 1e-13
        assert abs(gy - (c + e * x0 + 2 * f * y0)) < 1e-13


def test_laplacian_exact_on_quadratics():
    rng = np.random.default_rng(2)
    for _ in range(50):
        a, b, c, d, e, f = rng.normal(size=6)
        fun = lambda x, y: a + b * x + c * y + d * x * x + e * x * y + f * y * y
        assert abs(oracle.lap9(_samples(fun)) - 2 * (d + f)) < 1e-13


def test_gradient_rotation_covariance():
    """Rotating the samples by 90 degrees rotates the gradient exactly."""
    rng = np.random.default_rng(3)
    # direction a -> direction of the velocity rotated by +90 degrees: (ex, ey) -> (-ey, ex)
    rot = [next(b for b in range(9) if bf.EX[b] == -bf.EY[a] and bf.EY[b] == bf.EX[a]) for a in range(9)]
    for _ in range(50):
        q = rng.normal(size=9)
        qr = np.empty(9)
        for a in range(9):
            qr[rot[a]] = q[a]
        gx, gy = oracle.grad9(q)
        rx, ry = oracle.grad9(qr)
        assert abs(rx + gy) < 1e-14 and abs(ry - gx) < 1e-14
        assert abs(oracle.lap9(q) - oracle.lap9(qr)) < 1e-14


def test_divergence_of_normal_is_circle_curvature():
    """div n on a tanh droplet (phi = 1 inside, so n = grad phi / |grad phi| points
    inward and div n = -1/r): at every interface node (0.25 < phi < 0.75) of
    R = 12, 25, 40 drops, div n * r = -1 within 1%."""
    from paper_1909_04166_amd import workloads as W
    for R in (12.0, 25.0, 40.0):
        case, phi0 = W.droplet(128, R, W=4.0)
        divn = oracle.Oracle(case, phi0).coupling()["divn"]
        y, x = np.mgrid[0:128, 0:128].astype(float)
        r = np.hypot(x - 64, y - 64)
        band = (phi0 > 0.25) & (phi0 < 0.75)
        assert band.sum() > 100
        assert np.abs(divn[band] * r[band] + 1).max() <= 0.01
