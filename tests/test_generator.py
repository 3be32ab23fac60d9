"""Pins of the seeded input generator (the synthetic stand-in for the
paper's compactified initial loads, Sec. 3): the projection, the mass and
softening laws, the velocities.  The generator holds no pair-sum, kick,
drift or time-step arithmetic."""
import math

import numpy as np
import pytest
from scipy import stats

import synth

C = synth.Cosmo(H0=67.74, omega_m=0.3089, omega_l=0.6911)


def _set(sigma=0.01, zeldovich=True, n=20000, seed=123):
    return synth.make_set(n, 100.0, 1000.0, C, sigma, seed, 0.05, 1.0, 10,
                          zeldovich=zeldovich)


def test_compact_angle_follows_the_s3_law():
    # uniform on S^3: the polar angle omega has CDF (2w - sin 2w) / (2 pi)
    # (Eq. 18's volume element); r = D tan(omega / 2) (Eq. 15); truncated at
    # r_max, so the CDF is renormalised to omega_max
    ps = _set(sigma=0.0, zeldovich=False)
    r = np.linalg.norm(ps.pos, axis=0)
    w = 2.0 * np.arctan(r / 100.0)
    wmax = 2.0 * math.atan(1000.0 / 100.0)
    cdf = lambda x: (2 * x - np.sin(2 * x)) / (2 * wmax - math.sin(2 * wmax))
    assert stats.kstest(w, cdf).pvalue > 1e-3
    assert r.max() <= 1000.0


def test_mass_and_softening_laws():
    ps = _set(sigma=0.0, zeldovich=False)
    h0 = C.H0 * synth.KMS_TO_MPC_PER_GYR
    rho_bar = C.omega_m * 3 * h0 * h0 / (8 * math.pi * synth.G_MPC3_MSUN_GYR2)
    # total mass of a sphere of r_max at the mean density (Eq. 25)
    assert ps.mass.sum() == pytest.approx(rho_bar * 4 / 3 * math.pi * 1000.0 ** 3, rel=1e-12)
    # m proportional to (1 + r^2/D^2)^3
    r = np.linalg.norm(ps.pos, axis=0)
    ratio = ps.mass / (1 + (r / 100.0) ** 2) ** 3
    assert np.ptp(ratio) <= 1e-12 * ratio.mean()
    # h = 0.05 (m / rho_bar)^(1/3), so h / h_min = (m / m_min)^(1/3) (Eq. 7)
    np.testing.assert_allclose(ps.soft, 0.05 * np.cbrt(ps.mass / rho_bar), rtol=1e-14)


def test_zeldovich_velocities_follow_the_displacements():
    a = _set(sigma=0.01, zeldovich=True)
    b = _set(sigma=0.0, zeldovich=False)          # same seed, undisplaced
    psi = a.pos - b.pos
    spacing = np.cbrt(a.mass / (a.mass.sum() / (4 / 3 * math.pi * 1000.0 ** 3)))
    assert np.std(psi / spacing) == pytest.approx(0.01, rel=0.02)
    # v = f(a0) H(a0) psi, one factor for every particle; psi recovered as
    # (X + psi) - X carries the rounding of X + psi, eps |X|
    H = C.H0 * synth.KMS_TO_MPC_PER_GYR * math.sqrt(C.omega_m / 0.05 ** 3 + C.omega_l)
    fac = synth.growth_rate(0.05, C) * H
    bound = 4 * np.finfo(float).eps * np.abs(b.pos) * fac + 1e-15 * np.abs(a.vel)
    assert np.all(np.abs(a.vel - fac * psi) <= bound)


def test_growth_rate_limits():
    eds = synth.Cosmo(H0=70.0, omega_m=1.0, omega_l=0.0)
    assert synth.growth_rate(0.3, eds) == pytest.approx(1.0, rel=1e-10)
    # Lambda-CDM today: f close to Omega_m^0.55 (a well-known fit, ~1%)
    assert synth.growth_rate(1.0, C) == pytest.approx(C.omega_m ** 0.55, rel=0.01)


def test_seeded_and_member_distinct():
    a, b = synth.config(1, n=500), synth.config(1, n=500)
    assert np.array_equal(a.pos, b.pos) and np.array_equal(a.mass, b.mass)
    c = synth.config(1, n=500, member=1)
    assert not np.array_equal(a.pos, c.pos)
