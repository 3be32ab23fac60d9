"""Pins of the oracle's background (Sec. 2.2 Eq. 1), its step-in-a time
mapping (Sec. 2.3, Eq. 13 as the first-order limit) and its KDK integrator
(Sec. 2.3 Eqs. 9-11 with the acceleration of Eq. 8) to closed forms."""
import math

import numpy as np
import pytest

import oracle
from helpers import kepler_position, lattice_ball

KMS = 1.0e3 * (365.25 * 86400.0 * 1e9) / (149597870700.0 * 648000.0 / math.pi * 1e6)


def test_unit_constants():
    # G in Mpc^3/(Msun Gyr^2) from CODATA G and the IAU solar mass
    G_si, msun = 6.67430e-11, 1.988409870698051e30
    mpc, gyr = 149597870700.0 * 648000.0 / math.pi * 1e6, 365.25 * 86400 * 1e9
    assert oracle.G() == pytest.approx(G_si * msun * gyr ** 2 / mpc ** 3, rel=1e-4)
    assert oracle.kms_to_mpc_per_gyr() == pytest.approx(1.0227121650457e-3, rel=1e-12)


def test_hubble_today_and_components():
    c = oracle.Cosmology(H0=67.74, omega_m=0.3089, omega_l=0.6911)
    assert oracle.hubble(1.0, c) == pytest.approx(67.74 * KMS, rel=1e-14)
    eds = oracle.Cosmology(H0=70.0, omega_m=1.0, omega_l=0.0)
    for a in (0.02, 0.5, 2.0):
        assert oracle.hubble(a, eds) == pytest.approx(70 * KMS * a ** -1.5, rel=1e-14)


def _t_flat_lcdm(a, H0, om, ol):
    return 2.0 / (3.0 * H0 * math.sqrt(ol)) * math.asinh(math.sqrt(ol / om) * a ** 1.5)


@pytest.mark.parametrize("a,da", [(0.02, 0.98), (0.02, 0.0002), (0.3, 0.05),
                                  (0.9, -0.4), (0.1, 1e-7)])
def test_dt_flat_lcdm_closed_form(a, da):
    H0, om, ol = 67.74 * KMS, 0.3089, 0.6911
    c = oracle.Cosmology(H0=67.74, omega_m=om, omega_l=ol)
    ref = _t_flat_lcdm(a + da, H0, om, ol) - _t_flat_lcdm(a, H0, om, ol)
    assert oracle.dt(a, da, c) == pytest.approx(ref, rel=1e-12)


def test_dt_eds_and_radiation_closed_forms():
    H0 = 70 * KMS
    eds = oracle.Cosmology(H0=70.0, omega_m=1.0, omega_l=0.0)
    for a, da in [(0.02, 0.03), (0.1, 0.9)]:
        ref = 2.0 / (3.0 * H0) * ((a + da) ** 1.5 - a ** 1.5)
        assert oracle.dt(a, da, eds) == pytest.approx(ref, rel=1e-13)
    rad = oracle.Cosmology(H0=70.0, omega_m=0.0, omega_l=0.0, omega_r=1.0)
    for a, da in [(0.02, 0.03), (0.1, 0.9)]:
        ref = ((a + da) ** 2 - a ** 2) / (2.0 * H0)
        assert oracle.dt(a, da, rad) == pytest.approx(ref, rel=1e-13)
    # open, matter + curvature: t(a) = (sqrt(a(a+q)) - q asinh sqrt(a/q))/(H0 sqrt(Ok))
    # with q = Om/Ok
    om, ok = 0.3, 0.7
    opn = oracle.Cosmology(H0=70.0, omega_m=om, omega_l=0.0)
    q = om / ok

    def t(a):
        return (math.sqrt(a * (a + q)) - q * math.asinh(math.sqrt(a / q))) / (H0 * math.sqrt(ok))

    for a, da in [(0.05, 0.5), (0.5, 0.4)]:
        assert oracle.dt(a, da, opn) == pytest.approx(t(a + da) - t(a), rel=1e-12)


def test_dt_first_order_limit_is_eq13():
    c = oracle.Cosmology(H0=70.0, omega_m=0.3, omega_l=0.7)
    a = 0.04
    eq13 = lambda da: da / (a * oracle.hubble(a, c))
    e1 = abs(oracle.dt(a, 1e-3, c) / eq13(1e-3) - 1)
    e2 = abs(oracle.dt(a, 5e-4, c) / eq13(5e-4) - 1)
    assert e1 < 0.05 and e2 / e1 == pytest.approx(0.5, rel=0.02)


# ---------------- KDK in the Newtonian test mode ----------------

def _kepler_setup(ecc, G=1.0):
    # two bodies, total mass 1, relative orbit semi-major axis 1, starting at
    # pericentre; zero softening
    m1, m2 = 0.75, 0.25
    rp = 1.0 - ecc
    vp = math.sqrt(G * (1.0 + ecc) / rp)
    rel_x, rel_v = np.array([rp, 0, 0]), np.array([0, vp, 0])
    pos = np.stack([-m2 * rel_x, m1 * rel_x], axis=1)
    vel = np.stack([-m2 * rel_v, m1 * rel_v], axis=1)
    return (np.ascontiguousarray(pos), np.ascontiguousarray(vel),
            np.array([m1, m2]), np.zeros(2))


def _energy(pos, vel, mass, soft, G):
    kin = 0.5 * np.sum(mass * np.sum(vel * vel, axis=0))
    pot = 0.5 * G * np.dot(mass, oracle.potential(pos, mass, soft))
    return kin + pot


def _kepler_run(ecc, nsteps, T):
    c = oracle.Cosmology(G=1.0, newtonian_test=True)
    pos, vel, mass, soft = _kepler_setup(ecc)
    grid = np.linspace(0.0, T, nsteps + 1)
    p, v, _ = oracle.run(pos, vel, mass, soft, grid, c)
    return p[:, 1] - p[:, 0], (pos, vel, mass, soft, c)


def test_kepler_second_order_convergence():
    ecc, T = 0.5, 2.0
    exact = kepler_position(T, 1.0, ecc, 1.0)
    errs = [np.linalg.norm(_kepler_run(ecc, n, T)[0] - exact) for n in (400, 800, 1600)]
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.1)
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.1)


def test_kepler_energy_bounded_and_period():
    ecc = 0.3
    c = oracle.Cosmology(G=1.0, newtonian_test=True)
    pos, vel, mass, soft = _kepler_setup(ecc)
    e0 = _energy(pos, vel, mass, soft, 1.0)
    period = 2.0 * math.pi            # a = 1, G M = 1
    steps_per_orbit = 400
    S = oracle.forces(pos, mass, soft)
    p, v = pos.copy(), vel.copy()
    dt = period / steps_per_orbit
    devs = []
    for k in range(10 * steps_per_orbit):
        oracle.kdk_step(p, v, mass, soft, S, k * dt, dt, c)
        if (k + 1) % 50 == 0:
            devs.append(abs(_energy(p, v, mass, soft, 1.0) / e0 - 1.0))
        if k + 1 == steps_per_orbit:
            rel = p[:, 1] - p[:, 0]
            assert np.linalg.norm(rel - [1.0 - ecc, 0, 0]) < 5e-3  # O(dt^2) phase error
    devs = np.array(devs)
    assert devs.max() < 1e-3
    # no secular drift: last orbit's max deviation ~ first orbit's
    n_per = steps_per_orbit // 50
    assert devs[-n_per:].max() < 1.5 * devs[:n_per].max() + 1e-12
    # momentum exactly balanced by Newton's third law
    assert np.abs((mass * v).sum(axis=1)).max() < 1e-15


def test_time_reversibility():
    c = oracle.Cosmology(G=1.0, newtonian_test=True)
    pos, vel, mass, soft = _kepler_setup(0.6)
    S = oracle.forces(pos, mass, soft)
    p, v = pos.copy(), vel.copy()
    for k in range(300):
        oracle.kdk_step(p, v, mass, soft, S, 0.0, 0.01, c)
    for k in range(300):
        oracle.kdk_step(p, v, mass, soft, S, 0.0, -0.01, c)
    np.testing.assert_allclose(p, pos, atol=1e-12)
    np.testing.assert_allclose(v, vel, atol=1e-12)


# ---------------- comoving spherical mode ----------------

def test_eds_lone_particle_closed_form():
    # One particle, no other mass, Omega_m = 1: Eq. 8 reduces to
    # x'' + (4/3t) x' - (2/9t^2) x = 0 with solution x1 [2/3 (a/a1)^(1/2)
    # + 1/3 (a/a1)^-1] from rest at a1.  Pins the drag term, the radial term
    # with its a^-3 and the a -> t mapping.
    c = oracle.Cosmology(H0=70.0, omega_m=1.0, omega_l=0.0)
    x1 = np.array([[3.0], [-1.0], [2.0]])
    a1, a2 = 0.02, 0.2

    def run(ns):
        grid = a1 * (a2 / a1) ** (np.arange(ns + 1) / ns)
        p, v, _ = oracle.run(x1, np.zeros((3, 1)), np.ones(1), np.zeros(1), grid, c)
        return p[:, 0]

    exact = x1[:, 0] * (2.0 / 3.0 * math.sqrt(a2 / a1) + 1.0 / 3.0 * (a1 / a2))
    e1 = np.linalg.norm(run(200) - exact) / np.linalg.norm(exact)
    e2 = np.linalg.norm(run(400) - exact) / np.linalg.norm(exact)
    assert e1 < 1e-4
    assert e1 / e2 == pytest.approx(4.0, rel=0.1)


def test_uniform_ball_stays_at_rest():
    # A uniform comoving ball of the mean density at rest: pair gravity and
    # the radial term cancel at every a (Q: radial term read with a^-3).
    om, H0 = 0.3089, 67.74
    c = oracle.Cosmology(H0=H0, omega_m=om, omega_l=1 - om)
    h0 = H0 * oracle.kms_to_mpc_per_gyr()
    rho_bar = om * 3 * h0 ** 2 / (8 * math.pi * oracle.G())
    cell = 2.0
    pos = lattice_ball(12.0, cell)
    n = pos.shape[1]
    mass = np.full(n, rho_bar * cell ** 3)
    soft = np.full(n, 0.2 * cell)
    r = np.linalg.norm(pos, axis=0)
    inner = (r > 0.5 * cell) & (r < 0.5 * 12.0 * cell)
    for a in (0.05, 0.5, 1.0):
        S = oracle.forces(pos, mass, soft)
        p, v = pos.copy(), np.zeros_like(pos)
        da = 0.05 * a
        oracle.kdk_step(p, v, mass, soft, S, a, da, c)
        moved = np.linalg.norm(p - pos, axis=0)[inner]
        # what the radial term alone would do over the step
        dt = oracle.dt(a, da, c)
        radial_only = 0.5 * om * h0 ** 2 / a ** 3 * r[inner] * dt ** 2
        assert np.median(moved / radial_only) < 0.02
