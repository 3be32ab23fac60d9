"""Pins of reversed gravity, the glass relaxation of Sec. 3 (integrate
Eq. 8 with G -> -G until the particles settle)."""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
import synth
from helpers import lattice_ball


def nn_cv(pos, radius, inner=0.8):
    """Coefficient of variation of nearest-neighbour distances of the
    particles within inner * radius (about 0.36 for Poisson points)."""
    d, _ = cKDTree(pos.T).query(pos.T, k=2)
    keep = np.linalg.norm(pos, axis=0) < inner * radius
    dd = d[keep, 1]
    return dd.std() / dd.mean()


def _cosmo(rev):
    return oracle.Cosmology(H0=67.74, omega_m=0.3089, omega_l=0.6911,
                            reversed_gravity=rev)


def test_uniform_ball_at_rest_stays_at_rest_reversed():
    # both the pair term and the radial term flip, so they still cancel
    c = _cosmo(True)
    h0 = 67.74 * oracle.kms_to_mpc_per_gyr()
    rho_bar = 0.3089 * 3 * h0 ** 2 / (8 * math.pi * oracle.G())
    cell = 2.0
    pos = lattice_ball(12.0, cell)
    n = pos.shape[1]
    mass = np.full(n, rho_bar * cell ** 3)
    soft = np.full(n, 0.2 * cell)
    r = np.linalg.norm(pos, axis=0)
    inner = (r > 0.5 * cell) & (r < 6.0 * cell)
    for a in (0.05, 1.0):
        S = oracle.forces(pos, mass, soft)
        p, v = pos.copy(), np.zeros_like(pos)
        oracle.kdk_step(p, v, mass, soft, S, a, 0.05 * a, c)
        moved = np.linalg.norm(p - pos, axis=0)[inner]
        radial_only = 0.5 * 0.3089 * h0 ** 2 / a ** 3 * r[inner] * \
            oracle.dt(a, 0.05 * a, c) ** 2
        assert np.median(moved / radial_only) < 0.02


def test_reversed_potential_energy_flips_sign_exactly():
    ps = synth.config(1, n=300)
    rng = np.random.default_rng(2)
    vel = rng.normal(0, 2.0, ps.pos.shape)
    e = oracle.energy(ps.pos, vel, ps.mass, ps.soft, 0.4, _cosmo(False))
    r = oracle.energy(ps.pos, vel, ps.mass, ps.soft, 0.4, _cosmo(True))
    assert r["K"] == e["K"]
    assert r["U_pair"] == -e["U_pair"] and r["U_radial"] == -e["U_radial"]
    assert r["W"] == -e["W"]


def test_reversed_two_body_repels_and_conserves_energy():
    c = oracle.Cosmology(G=1.0, newtonian_test=True, reversed_gravity=True)
    pos = np.array([[-0.5, 0.5], [0.0, 0.0], [0.0, 0.0]])
    vel = np.zeros((3, 2))
    mass, soft = np.array([1.0, 1.0]), np.full(2, 1e-3)
    e0 = oracle.energy(pos, vel, mass, soft, 1.0, c)
    assert e0["W"] == pytest.approx(+1.0, rel=1e-12)   # +G m1 m2 / r
    S = oracle.forces(pos, mass, soft)
    p, v = pos.copy(), vel.copy()
    for _ in range(400):
        oracle.kdk_step(p, v, mass, soft, S, 0.0, 0.005, c)
    assert p[0, 1] - p[0, 0] > 1.5                      # moved apart
    e1 = oracle.energy(p, v, mass, soft, 1.0, c)
    assert e1["K"] + e1["W"] == pytest.approx(e0["K"] + e0["W"], rel=1e-5)


def test_poisson_ball_relaxes_into_a_glass():
    ps = synth.poisson_ball(1000, 100.0, synth.Cosmo(67.74, 0.3089, 0.6911),
                            seed=21)
    cv0 = nn_cv(ps.pos, 100.0)
    p, v, _ = oracle.run(ps.pos, ps.vel, ps.mass, ps.soft, ps.a_grid(),
                         _cosmo(True))
    cv1 = nn_cv(p, 100.0)
    rms0 = np.sqrt(np.mean(np.sum(ps.pos ** 2, 0)))
    rms1 = np.sqrt(np.mean(np.sum(p ** 2, 0)))
    assert cv0 > 0.3            # Poisson
    assert cv1 < 0.15           # glass: nearly uniform nearest-neighbour spacing
    assert rms1 == pytest.approx(rms0, rel=0.02)   # still a uniform ball
    # ordinary gravity from the same start clusters instead
    pg, _, _ = oracle.run(ps.pos, ps.vel, ps.mass, ps.soft, ps.a_grid(),
                          _cosmo(False))
    assert nn_cv(pg, 100.0) > cv0
