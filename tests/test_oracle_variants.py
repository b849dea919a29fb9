"""Pins of the oracle's option paths against what the mathematics fixes:

- SRT collisions (comparison model of Sec. 7): moment identities of a BGK step
  toward a second-order Hermite equilibrium, exact agreement with the cascaded
  collision where the two must coincide, and the textbook shear-wave viscosity;
- free-slip walls: a slip channel is the lower half of a periodic channel of twice
  the height holding the mirror image (method of images), and a uniform plug flow
  is unaffected by the walls;
- Langmuir surface tension (Eq. Langmuirisotherm): a uniform concentration
  reduces to a constant sigma, and the Marangoni force on a vertical interface is
  |grad phi|^2 d kappa~/dy, checked against a finite difference of kappa~(psi(y));
- ACE only under an imposed velocity (Sec. 6.1): with u = 0 it reproduces the
  coupled step of a fluid at rest, and a small sine wave in phi is advected at the
  imposed velocity and decays at the mobility (textbook advection-diffusion).
CPU only, a few seconds each."""
import numpy as np
import pytest

import oracle
from paper_1909_04166_amd import workloads as W

C2 = 1.0 / 3.0
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
WT = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
POW = [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)]


def moments(v):
    """Raw moments m_mn = sum_a v_a ex^m ey^n in the order of POW."""
    return np.array([np.sum(v * EX ** m * EY ** n) for m, n in POW])


def zero_first_moments(v):
    """Shifts weight between opposite axis directions so that sum v e = 0."""
    jx, jy = np.sum(v * EX), np.sum(v * EY)
    v = v.copy()
    v[1] -= jx / 2; v[3] += jx / 2
    v[2] -= jy / 2; v[4] += jy / 2
    return v


def consistent_hydro_inputs(rng, forces=True):
    """Pre-collision gbar and the macroscopic values the step derives from it
    (u from the first moment with the half-force shift, p = sum gbar + F_p.u / 2)."""
    g = rng.normal(size=9) * 0.1
    rho = 1.0 + 5.0 * rng.random()
    Ft = rng.normal(size=2) * 0.01 if forces else np.zeros(2)
    Fp = rng.normal(size=2) * 0.01 if forces else np.zeros(2)
    ux = (np.sum(g * EX) + 0.5 * C2 * Ft[0]) / (rho * C2)
    uy = (np.sum(g * EY) + 0.5 * C2 * Ft[1]) / (rho * C2)
    p = g.sum() + 0.5 * (Fp[0] * ux + Fp[1] * uy)
    return g, p, rho, ux, uy, Ft, Fp


# ------------------------------------------------------------------ SRT per node

def test_srt_hydro_agrees_with_cascaded_to_second_order_without_forces():
    """Without forces both collisions relax the zeroth to second raw moments to
    p, rho c^2 u, p c^2 I + rho c^2 u u; with every cascaded rate set to the SRT
    rate they must agree on those six moments (they differ at third order)."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        g, p, rho, ux, uy, Ft, Fp = consistent_hydro_inputs(rng, forces=False)
        om = rng.uniform(0.3, 1.9)
        a = oracle.hydro_collide(g, p, rho, p - rho * C2, ux, uy, 0, 0, 0, 0, [om] * 9)
        b = oracle.hydro_srt(g, p, rho, ux, uy, 0, 0, 0, 0, om)
        ma, mb = moments(a), moments(b)
        assert np.abs(ma[:6] - mb[:6]).max() <= 1e-15
        assert np.abs(ma[6:] - mb[6:]).max() > 1e-6  # the models are not the same


def test_srt_equals_cascaded_at_rest_with_unit_rates():
    """At u = 0, no force and unit rates both collisions return their equilibrium,
    whose nine moments coincide (p, 0, 0, p c^2, p c^2, 0, 0, 0, p c^4); likewise
    for the phase field at theta = 0."""
    rng = np.random.default_rng(12)
    for _ in range(10):
        g = zero_first_moments(rng.normal(size=9) * 0.1)
        rho = 1.0 + rng.random()
        p = g.sum()
        a = oracle.hydro_collide(g, p, rho, p - rho * C2, 0, 0, 0, 0, 0, 0, [1.0] * 9)
        b = oracle.hydro_srt(g, p, rho, 0, 0, 0, 0, 0, 0, 1.0)
        assert np.abs(a - b).max() <= 1e-15
        f = zero_first_moments(rng.random(9) * 0.1)
        a = oracle.ace_collide(f, f.sum(), 0, 0, 0.05, 0.0, 0.6, 0.8, [1.0] * 9)
        b = oracle.ace_srt(f, f.sum(), 0, 0, 0.05, 0.0, 0.6, 0.8, 1.0)
        assert np.abs(a - b).max() <= 1e-15


def test_srt_hydro_moment_identities_with_forces():
    """Every post-collision raw moment of the hydrodynamic SRT equals
    (1 - om) m + om m_eq + (1 - om/2) m_S with the D2Q9 Hermite-2 closures
    m_eq = (p, rho c^2 u, p c^2 + rho c^2 u u, rho c^4 u_y, rho c^4 u_x, c^4 (p + rho u^2))
    and the source moments of the step (zeroth F_p.u, first c^2 F_t, second
    sigma'_20, sigma'_02, sigma'_11, third c^2 sigma'_01, c^2 sigma'_10, fourth
    (3 (sigma'_20 + sigma'_02) - sigma'_00) / 9).  The zeroth and first
    identities are the invariants sum (g~ - g) = F_p . u, sum (g~ - g) e = c^2 F_t."""
    rng = np.random.default_rng(13)
    for _ in range(20):
        g, p, rho, ux, uy, Ft, Fp = consistent_hydro_inputs(rng)
        om = rng.uniform(0.3, 1.9)
        out = oracle.hydro_srt(g, p, rho, ux, uy, *Ft, *Fp, om)
        Gam = Fp[0] * ux + Fp[1] * uy
        s20 = 2 * C2 * (Ft[0] + Fp[0]) * ux + C2 * Gam
        s02 = 2 * C2 * (Ft[1] + Fp[1]) * uy + C2 * Gam
        s11 = C2 * (Ft[0] * uy + Ft[1] * ux) + C2 * (Fp[0] * uy + Fp[1] * ux)
        c4 = C2 * C2
        meq = np.array([p, rho * C2 * ux, rho * C2 * uy, p * C2 + rho * C2 * ux * ux,
                        p * C2 + rho * C2 * uy * uy, rho * C2 * ux * uy, rho * c4 * uy,
                        rho * c4 * ux, c4 * (p + rho * (ux * ux + uy * uy))])
        mS = np.array([Gam, C2 * Ft[0], C2 * Ft[1], s20, s02, s11, C2 * C2 * Ft[1],
                       C2 * C2 * Ft[0], (3 * (s20 + s02) - Gam) / 9.0])
        expect = (1 - om) * moments(g) + om * meq + (1 - 0.5 * om) * mS
        assert np.abs(moments(out) - expect).max() <= 1e-15
        d = out - g
        assert abs(d.sum() - Gam) <= 1e-15
        assert abs(np.sum(d * EX) - C2 * Ft[0]) <= 1e-15
        assert abs(np.sum(d * EY) - C2 * Ft[1]) <= 1e-15


def test_srt_ace_moment_identities():
    """Phase-field SRT: phi is conserved, and the other raw moments relax at one
    rate to (phi u + M theta n, c^2 phi I + phi u u, c^2 (phi u_y + M theta n_y),
    c^2 (phi u_x + M theta n_x), c^4 phi (1 + 3 u^2))."""
    rng = np.random.default_rng(14)
    for _ in range(20):
        f = rng.random(9) * 0.1
        phi = f.sum()
        ux, uy = rng.normal(size=2) * 0.05
        M, th = 0.05, rng.random()
        ang = rng.uniform(0, 2 * np.pi)
        nx, ny = np.cos(ang), np.sin(ang)
        om = rng.uniform(0.3, 1.9)
        out = oracle.ace_srt(f, phi, ux, uy, M, th, nx, ny, om)
        jx, jy = phi * ux + M * th * nx, phi * uy + M * th * ny
        meq = np.array([phi, jx, jy, C2 * phi + phi * ux * ux, C2 * phi + phi * uy * uy,
                        phi * ux * uy, C2 * jy, C2 * jx, C2 * C2 * phi * (1 + 3 * (ux * ux + uy * uy))])
        expect = (1 - om) * moments(f) + om * meq
        assert np.abs(moments(out) - expect).max() <= 1e-15
        assert abs(out.sum() - phi) <= 1e-15


@pytest.mark.parametrize("collision", ["cascaded", "srt"])
def test_shear_wave_viscosity_both_models(collision):
    """Single phase: a shear wave decays as exp(-nu k^2 t) with
    nu = c^2 (1/omega - 1/2) under either collision model."""
    nu = 0.05
    case, phi0 = W.uniform_phase(4, 64, 1.0, nu_A=nu, nu_B=nu, collision=collision)
    o = oracle.Oracle(case, phi0)
    f, _ = o.get_dist()
    y = np.arange(64)
    ux = 1e-3 * np.sin(2 * np.pi * y / 64)[:, None] * np.ones((1, 4))
    o.set_dist(f, WT[:, None, None] * EX[:, None, None] * ux[None], 0)
    amps = []
    for t in (200, 1200):
        o.step(t - o.t)
        u = o.fields()[2][:, 0]
        amps.append((u * np.sin(2 * np.pi * y / 64)).sum() * 2 / 64)
    k = 2 * np.pi / 64
    assert abs(np.log(amps[0] / amps[1]) / (k * k * 1000) / nu - 1) <= 5e-3


def test_srt_laplace_law():
    """The SRT pair keeps the force balance of a static drop (Laplace-Young,
    Sec. 6.2) at a moderate density ratio."""
    case, phi0 = W.droplet(64, 14.0, W=4.0, ratio=10.0, sigma=0.01)
    case["collision"] = "srt"
    o = oracle.Oracle(case, phi0)
    o.step(3000)
    d = o.diagnostics()
    assert d["nan_flag"] == 0
    assert abs(d["dp_laplace"] * d["r_eff"] / 0.01 - 1.0) <= 0.1


# ------------------------------------------------------------------ free slip

def test_slip_channel_is_half_of_mirrored_periodic_channel():
    """Method of images: halfway specular walls at y = -1/2 and ny - 1/2 give the
    same state as a periodic channel of height 2 ny whose upper half holds the
    mirror image (no body force, so the image problem is itself symmetric)."""
    nx, ny = 48, 40
    case, phi0 = W.droplet(nx, 9.0, ny=ny, ratio=20.0, sigma=0.01)
    case["bc_y"] = "slip"
    y, x = np.mgrid[0:ny, 0:nx]
    phi0 = W.tanh_profile(9.0 - np.hypot(x - 20.3, y - 12.6), 4.0)  # off-centre, near the bottom
    big = dict(case, ny=2 * ny, bc_y="periodic")
    phi_big = np.concatenate([phi0, phi0[::-1]], axis=0)
    a = oracle.Oracle(case, phi0)
    b = oracle.Oracle(big, phi_big)
    a.step(80)
    b.step(80)
    fa, ga = a.get_dist()
    fb, gb = b.get_dist()
    assert np.abs(fb[:, :ny] - fa).max() <= 1e-13
    assert np.abs(gb[:, :ny] - ga).max() <= 1e-13
    # the image half is the mirror of the lower half: direction a <-> its y-mirror
    mir = [0, 1, 4, 3, 2, 8, 7, 6, 5]
    assert np.abs(fb[mir, ny:][:, ::-1] - fa).max() <= 1e-13
    pa, pb = a.fields(), b.fields()
    assert np.abs(pb[3][:ny]).max() > 1e-6  # the drop moves (the test is not vacuous)
    for u, v in zip(pa, pb):
        assert np.abs(v[:ny] - u).max() <= 1e-12


def test_slip_walls_leave_plug_flow_free():
    """A uniform fluid under a uniform body force between free-slip walls
    accelerates as in a periodic box, u(t) = g (t + 1/2) at every node; halfway
    bounce-back walls instead hold the wall layers back."""
    gx = 1e-5
    case, phi0 = W.uniform_phase(8, 12, 1.0, rho_A=2.0, rho_B=2.0, gx=gx, force_ref="none",
                                 bc_y="slip")
    o = oracle.Oracle(case, phi0)
    o.step(60)
    ux = o.fields()[2]
    assert np.allclose(ux, gx * 60.5, rtol=1e-12, atol=0)
    case["bc_y"] = "wall"
    o = oracle.Oracle(case, phi0)
    o.step(60)
    ux = o.fields()[2]
    assert ux[0, 0] < 0.9 * gx * 60.5


# ------------------------------------------------------------------ Langmuir

def test_langmuir_uniform_concentration_is_constant_sigma():
    """psi = a everywhere: kappa~ = 1.5 W sigma0 (1 + beta ln(1 - a)) is constant and
    the run equals the linear law with sigma = sigma0 (1 + beta ln(1 - a))."""
    a, beta = 0.3, 0.8
    case, phi0 = W.droplet(48, 10.0, ratio=10.0, sigma=0.01)
    lang = dict(case, surf="langmuir", beta=beta, psi_a=a, psi_G=0.0)
    lin = dict(case, sigma0=0.01 * (1 + beta * np.log(1 - a)))
    o1, o2 = oracle.Oracle(lang, phi0), oracle.Oracle(lin, phi0)
    o1.step(40)
    o2.step(40)
    for u, v in zip(o1.fields(), o2.fields()):
        assert np.abs(u - v).max() <= 1e-13 * max(1.0, np.abs(v).max())


def test_langmuir_marangoni_force_on_vertical_interface():
    """On a vertical flat interface (n = (+-1, 0), div n = 0) the surface-tension
    force is purely tangential: F_y = |grad phi|^2 d kappa~/dy.  d kappa~/dy is
    checked against a central difference of kappa~(psi(y)) = 1.5 W sigma0 (1 + beta
    ln(1 - psi)), psi = psi_a + psi_G y."""
    nx, ny, Wd = 32, 24, 4.0
    s0, beta, pa, pG = 0.01, 2.44, 0.05, 2e-3
    case = W.base_case(nx, ny, bc_y="wall", rho_A=3.0, rho_B=1.0, sigma0=s0, W=Wd,
                       surf="langmuir", beta=beta, psi_a=pa, psi_G=pG)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    phi0 = W.tanh_profile(8.0 - np.abs(x - 15.5), Wd)  # strip of phase A, two interfaces
    o = oracle.Oracle(case, phi0)
    c = o.coupling()
    m2 = c["dphix"] ** 2 + c["dphiy"] ** 2

    def kt(yy):
        return 1.5 * Wd * s0 * (1 + beta * np.log(1 - (pa + pG * yy)))

    h = 1e-3
    dk = (kt(y + h) - kt(y - h)) / (2 * h)
    sel = m2 > 1e-4
    assert sel.sum() > 100
    assert np.abs(c["Fty"][sel] / (m2[sel] * dk[sel]) - 1).max() <= 1e-6
    # no normal force on the interface (div n = 0 there; n flips sign only where
    # |grad phi|^2 is negligible)
    assert np.abs(c["Ftx"][sel]).max() <= 1e-12 * np.abs(c["Fty"]).max()


# ------------------------------------------------------------------ ACE only

def test_imposed_zero_velocity_matches_coupled_step_at_rest():
    """With sigma = 0 and no gravity the coupled fluid stays at rest, so its phase
    field evolves as the ACE at u = 0; the ACE-only mode with an imposed u = 0
    gives the same distributions to round-off."""
    case, phi0 = W.droplet(40, 9.0, ratio=100.0, sigma=0.0)
    a = oracle.Oracle(case, phi0)
    b = oracle.Oracle(dict(case, flow="imposed"), phi0)
    b.set_velocity(np.zeros((40, 40)), np.zeros((40, 40)))
    a.step(100)
    b.step(100)
    # at rest up to the rounding of c^6 rho + psi c^4 = 0 in the fourth-order equilibrium
    assert np.abs(a.fields()[2]).max() <= 1e-15
    assert np.abs(a.get_dist()[0] - b.get_dist()[0]).max() <= 1e-15
    phi, p, ux, uy = b.fields()
    assert np.abs(p).max() == 0.0


@pytest.mark.parametrize("collision", ["cascaded", "srt"])
def test_imposed_velocity_advection_diffusion(collision):
    """Textbook special case of the ACE under an imposed uniform velocity: with
    theta negligible (W = 1e6) a small sine wave phi = 1/2 + A sin(k . x) moves at u
    and decays as exp(-M |k|^2 t) (M = c^2 (1/omega_phi - 1/2))."""
    n, M = 32, 0.05
    U = np.array([0.05, -0.03])
    case = W.base_case(n, n, flow="imposed", W=1e6, M=M, collision=collision)
    x, y = np.mgrid[0:n, 0:n].astype(float)[::-1]  # x varies along axis 1
    kv = 2 * np.pi * np.array([1.0, 1.0]) / n
    A = 1e-2
    phi0 = 0.5 + A * np.sin(kv[0] * x + kv[1] * y)
    o = oracle.Oracle(case, phi0)
    o.set_velocity(np.full((n, n), U[0]), np.full((n, n), U[1]))
    t = 300
    o.step(t)
    phi = o.fields()[0] - 0.5
    z = (phi * np.exp(-1j * (kv[0] * x + kv[1] * y))).sum() * 2 / (n * n)  # = A e^{-rate t} e^{-i k.U t} / i
    amp = abs(z)
    phase = np.angle(z * 1j)
    k2 = kv @ kv
    assert abs(np.log(A / amp) / (k2 * t) / M - 1) <= 0.03
    expect = -(kv @ U) * t
    assert abs(np.angle(np.exp(1j * (phase - expect)))) <= 0.01


# ------------------------------------------------------------------ walls in x

def _transpose_case(case):
    t = dict(case, nx=case["ny"], ny=case["nx"], bc_x=case["bc_y"], bc_y=case["bc_x"],
             gx=case["gy"], gy=case["gx"])
    return t


@pytest.mark.parametrize("bcx,bcy", [("periodic", "wall"), ("periodic", "slip"), ("slip", "wall"),
                                     ("wall", "slip")])
def test_walls_in_x_equal_transposed_walls_in_y(bcx, bcy):
    """Rotating the lattice by a quarter turn (x <-> y, walls and body force with
    it) maps the step onto itself: the x-wall paths reproduce the pinned y-wall
    paths, to round-off, including the corners when both directions have walls."""
    nx, ny = 40, 56
    case = W.base_case(nx, ny, bc_x=bcx, bc_y=bcy, rho_A=10.0, rho_B=1.0, sigma0=0.01,
                       gy=-1e-5, force_ref="mean")
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    phi0 = W.tanh_profile(11.0 - np.hypot(x - 14.2, y - 13.7), 4.0)
    a = oracle.Oracle(case, phi0)
    b = oracle.Oracle(_transpose_case(case), phi0.T.copy())
    a.step(60)
    b.step(60)
    pa, pb = a.fields(), b.fields()
    assert np.abs(pa[3]).max() > 1e-6  # flow develops (not vacuous)
    assert np.abs(pb[0] - pa[0].T).max() <= 1e-12
    assert np.abs(pb[1] - pa[1].T).max() <= 1e-12 * max(1.0, np.abs(pa[1]).max())
    assert np.abs(pb[2] - pa[3].T).max() <= 1e-12
    assert np.abs(pb[3] - pa[2].T).max() <= 1e-12


@pytest.mark.parametrize("bcy", ["wall", "slip"])
def test_slip_in_x_is_half_of_mirrored_periodic_domain(bcy):
    """Method of images in x: specular walls at x = -1/2 and nx - 1/2 equal the left
    half of a periodic domain of width 2 nx holding the mirror image.  With walls
    in y as well this fixes the corner rule (the image problem reflects twice)."""
    nx, ny = 36, 48
    case = W.base_case(nx, ny, bc_x="slip", bc_y=bcy, rho_A=10.0, rho_B=1.0, sigma0=0.01,
                       gy=-1e-5, force_ref="mean")
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    phi0 = W.tanh_profile(10.0 - np.hypot(x - 9.3, y - 12.1), 4.0)  # near the corner
    big = dict(case, nx=2 * nx, bc_x="periodic")
    a = oracle.Oracle(case, phi0)
    b = oracle.Oracle(big, np.concatenate([phi0, phi0[:, ::-1]], axis=1))
    a.step(80)
    b.step(80)
    fa, ga = a.get_dist()
    fb, gb = b.get_dist()
    assert np.abs(fb[:, :, :nx] - fa).max() <= 1e-13
    assert np.abs(gb[:, :, :nx] - ga).max() <= 1e-13
    mirx = [0, 3, 2, 1, 4, 6, 5, 8, 7]
    assert np.abs(fb[mirx][:, :, nx:][:, :, ::-1] - fa).max() <= 1e-13
    assert np.abs(a.fields()[2]).max() > 1e-6
