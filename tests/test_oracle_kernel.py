"""Pins of the oracle's softening kernel (Sec. 2.2, Eq. 4) to mathematics the
oracle does not contain: the enclosed mass of the textbook cubic-spline
density, hand-derived exact values, and continuity/smoothness."""
import math

import numpy as np
import pytest

import oracle
from helpers import load_m4_golden, m4_force, m4_potential

H_VALUES = [0.37, 1.0, 2.5e-3, 41.0]


@pytest.mark.parametrize("h", H_VALUES)
def test_force_equals_m4_enclosed_mass(h):
    # r^2 F(r, h) must be the mass of the M4 spline inside r (Eq. 4 cites
    # that kernel): checks every coefficient and sign of both branches.
    for u in np.linspace(1e-3, 0.999, 97):
        r = u * h
        ref = m4_force(r, h)
        got = oracle.kernel_F(r, h)
        assert got == pytest.approx(ref, rel=2e-12, abs=0.0), (u, got, ref)


def test_golden_points():
    for u, h2f, hphi in load_m4_golden():
        for h in (1.0, 0.125, 3.0):
            r = float(u) * h
            if r > 0:
                got = oracle.kernel_F(r, h) * h * h
                assert got == pytest.approx(float(h2f), rel=1e-14), (u, h)
            if hphi is not None:
                got = oracle.kernel_phi(r, h) * h
                assert got == pytest.approx(float(hphi), rel=1e-14), (u, h)


@pytest.mark.parametrize("h", [1.0, 0.3])
def test_newtonian_beyond_support(h):
    for r in [h, 1.0000001 * h, 2 * h, 17.3 * h, 1e4 * h]:
        assert oracle.kernel_F(r, h) == 1.0 / (r * r)
        assert oracle.kernel_phi(r, h) == -1.0 / r
    # zero softening: pure 1/r^2 at every r > 0
    for r in [1e-6, 0.01, 3.0]:
        assert oracle.kernel_F(r, 0.0) == 1.0 / (r * r)


@pytest.mark.parametrize("h", [1.0, 0.7])
def test_continuity_and_slope_at_joins(h):
    # value and slope continuous at u = 1/2 and u = 1 (C^1 kernel)
    for uj in (0.5, 1.0):
        e = 1e-7
        lo, hi = (uj - e) * h, (uj + e) * h
        assert oracle.kernel_F(lo, h) == pytest.approx(oracle.kernel_F(hi, h),
                                                       rel=1e-6)
        d = 1e-5 * h
        sl = (oracle.kernel_F(uj * h - d, h) - oracle.kernel_F(uj * h - 2 * d, h)) / d
        sr = (oracle.kernel_F(uj * h + 2 * d, h) - oracle.kernel_F(uj * h + d, h)) / d
        assert sl == pytest.approx(sr, rel=1e-3)
    # slopes from the M4 enclosed mass: dF/dr at u=1/2 is -32/15 h^-3,
    # at u=1 it is -2 h^-3 (that of 1/r^2)
    d = 1e-6 * h
    s_half = (oracle.kernel_F(0.5 * h + d, h) - oracle.kernel_F(0.5 * h - d, h)) / (2 * d)
    assert s_half * h ** 3 == pytest.approx(-32.0 / 15.0, rel=1e-6)
    s_one = (oracle.kernel_F(h + d, h) - oracle.kernel_F(h - d, h)) / (2 * d)
    assert s_one * h ** 3 == pytest.approx(-2.0, rel=1e-5)


def test_small_r_limit():
    # F/r -> 32 / (3 h^3) as r -> 0 (uniform central density 8/(pi h^3))
    for h in (1.0, 0.25):
        for u in (1e-4, 1e-6):
            r = u * h
            assert oracle.kernel_F(r, h) / r * h ** 3 == pytest.approx(
                32.0 / 3.0, rel=1e-3)


@pytest.mark.parametrize("h", [1.0, 0.3])
def test_potential_is_integral_of_force(h):
    # phi(r) = -int_r^inf F from the independent M4 quadrature
    for u in np.linspace(0.0, 0.999, 41):
        r = u * h
        ref = m4_potential(r, h)
        assert oracle.kernel_phi(r, h) == pytest.approx(ref, rel=1e-11)


def test_potential_derivative_is_force():
    h = 1.3
    for u in np.linspace(0.05, 1.4, 40):
        r = u * h
        d = 1e-6 * r
        dphi = (oracle.kernel_phi(r + d, h) - oracle.kernel_phi(r - d, h)) / (2 * d)
        assert dphi == pytest.approx(oracle.kernel_F(r, h), rel=1e-6)
