"""Pins of the periodic pair sum (Sec. 2.2, Eqs. 2 and 5) and the periodic
equations of motion."""
import itertools
import math

import numpy as np
import pytest

import oracle

L = 10.0


def _lattice(k):
    g = (np.arange(k) + 0.5) * (L / k)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return np.ascontiguousarray(np.stack([X.ravel(), Y.ravel(), Z.ravel()]))


@pytest.mark.parametrize("images", [1, 2])
def test_lattice_feels_no_force(images):
    # a simple cubic lattice filling the box is symmetric about every one
    # of its points, in both image rules (k odd: no pair at exactly L/2)
    pos = _lattice(5)
    n = pos.shape[1]
    mass, soft = np.full(n, 2.0), np.full(n, 0.05)
    S = oracle.forces_periodic(pos, mass, soft, L, images)
    scale = 2.0 / (L / 5) ** 2            # one neighbour's pull
    assert np.abs(S).max() < 1e-12 * scale


def test_nearest_image_two_body_closed_form():
    pos = np.array([[0.1 * L, 0.9 * L], [0.5, 0.5], [0.5, 0.5]])
    mass, soft = np.array([1.0, 3.0]), np.full(2, 0.01)
    S = oracle.forces_periodic(pos, mass, soft, L, 1)
    # nearest image of particle 2 seen from 1 is at -0.2 L along x
    assert S[0, 0] == pytest.approx(-3.0 / (0.2 * L) ** 2, rel=1e-14)
    assert S[0, 1] == pytest.approx(+1.0 / (0.2 * L) ** 2, rel=1e-14)
    assert np.all(S[1:] == 0.0)


def test_image_sum_against_brute_force():
    # raw displacements (no nearest-image step), every n in [-6, 6]^3, the
    # cut |x_j + n L - x_i| < 2.6 L, Newtonian pairs (h small): an
    # enumeration independent of the oracle's
    rng = np.random.default_rng(4)
    pos = rng.uniform(0, L, (3, 3)) + np.array([[0.0], [L], [-2 * L]])
    mass, soft = np.array([1.0, 2.0, 3.0]), np.full(3, 1e-4)
    S = oracle.forces_periodic(pos, mass, soft, L, 2)
    ns = np.array(list(itertools.product(range(-6, 7), repeat=3)), dtype=float).T
    for i in range(3):
        want = np.zeros(3)
        for j in range(3):
            if j == i:
                continue
            e = (pos[:, j] - pos[:, i])[:, None] + L * ns
            r = np.sqrt((e * e).sum(0))
            keep = r < 2.6 * L
            want += (mass[j] * e[:, keep] / r[keep] ** 3).sum(1)
        assert S[:, i] == pytest.approx(want, rel=1e-13, abs=1e-15 * np.abs(want).max())


@pytest.mark.parametrize("images", [1, 2])
def test_box_shifts_and_third_law(images):
    rng = np.random.default_rng(7)
    n = 60
    pos = rng.uniform(0, L, (3, n))
    mass, soft = rng.uniform(1, 3, n), rng.uniform(0.05, 0.3, n)
    S = oracle.forces_periodic(pos, mass, soft, L, images)
    shifted = pos + L * rng.integers(-2, 3, (3, n))
    S2 = oracle.forces_periodic(shifted, mass, soft, L, images)
    np.testing.assert_allclose(S2, S, rtol=1e-11, atol=1e-12 * np.abs(S).max())
    net = np.abs((mass * S).sum(1)).max()
    assert net < 1e-13 * (mass * np.abs(S)).sum(1).max()


def test_lattice_at_rest_stays_at_rest_under_eq2():
    # Eq. 2 has no radial term: the force-free lattice does not move, where
    # the spherical equations (Eq. 8) would push it outwards
    pos = _lattice(5)
    n = pos.shape[1]
    mass, soft = np.full(n, 1e12), np.full(n, 0.05)
    c = oracle.Cosmology(H0=70.0, omega_m=0.3, omega_l=0.7, images=2, box_L=L)
    S = oracle.forces_periodic(pos, mass, soft, L, 2)
    p, v = pos.copy(), np.zeros_like(pos)
    oracle.kdk_step(p, v, mass, soft, S, 0.5, 0.05, c)
    assert np.abs(p - pos).max() < 1e-12 * L
    c8 = oracle.Cosmology(H0=70.0, omega_m=0.3, omega_l=0.7)
    p8, v8 = pos.copy(), np.zeros_like(pos)
    oracle.kdk_step(p8, v8, mass, soft, np.zeros_like(S), 0.5, 0.05, c8)
    assert np.abs(p8 - pos).max() > 1e-6 * L
