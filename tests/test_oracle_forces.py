"""Pins of the oracle's pair sum S_i (Sec. 2.2, Eq. 8 first term with Eq. 3)
to closed forms, brute force with an independent kernel, invariances and
potential theory."""
import math

import numpy as np
import pytest

import oracle
import synth
from helpers import (brute_pair_sum, fibonacci_sphere, lattice_ball,
                     m4_force)


def _rel(a, b):
    return np.linalg.norm(a - b, axis=0) / np.maximum(
        np.linalg.norm(b, axis=0), 1e-300)


def test_two_body_closed_form_newtonian():
    # separation beyond h_i + h_j: |S| = m_j / r^2, pointing at j
    pos = np.array([[0.0, 3.0], [0.0, 4.0], [0.0, 0.0]])
    mass = np.array([2.0, 7.0])
    soft = np.array([0.5, 1.5])      # h = 2 < r = 5
    S = oracle.forces(pos, mass, soft)
    np.testing.assert_allclose(S[:, 0], 7.0 / 25.0 * np.array([0.6, 0.8, 0.0]),
                               rtol=1e-15)
    np.testing.assert_allclose(S[:, 1], -2.0 / 25.0 * np.array([0.6, 0.8, 0.0]),
                               rtol=1e-15)


@pytest.mark.parametrize("r", [0.1, 0.6, 1.0, 1.7, 1.999])
def test_two_body_softened_uses_sum_of_softenings(r):
    # support h = h_i + h_j = 2; magnitude from the M4 enclosed mass
    pos = np.array([[0.0, r], [0.0, 0.0], [0.0, 0.0]])
    mass = np.array([1.0, 3.0])
    soft = np.array([0.25, 1.75])
    S = oracle.forces(pos, mass, soft)
    assert S[0, 0] == pytest.approx(3.0 * m4_force(r, 2.0), rel=1e-12)
    assert S[0, 1] == pytest.approx(-1.0 * m4_force(r, 2.0), rel=1e-12)
    assert S[1, 0] == 0.0 and S[2, 0] == 0.0


def test_single_particle_and_coincident_pairs():
    S = oracle.forces(np.zeros((3, 1)), np.ones(1), np.ones(1))
    assert np.all(S == 0.0)
    # coincident particles contribute nothing, also with zero softening
    pos = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    S = oracle.forces(pos, np.array([1.0, 2.0, 4.0]), np.zeros(3))
    np.testing.assert_allclose(S[:, 0], [4.0, 0, 0], rtol=1e-15)
    np.testing.assert_allclose(S[:, 2], [-3.0, 0, 0], rtol=1e-15)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_brute_force_small_n(seed):
    # N <= 8, mixed softened / unsoftened pairs, one zero softening, one
    # coincident pair: compare with an fsum loop over the M4 quadrature kernel
    rng = np.random.default_rng(seed)
    n = 8
    pos = rng.uniform(-1.0, 1.0, (3, n))
    pos[:, 5] = pos[:, 2]
    mass = rng.uniform(0.1, 3.0, n)
    soft = rng.uniform(0.05, 0.8, n)
    soft[1] = 0.0
    S = oracle.forces(pos, mass, soft)
    for i in range(n):
        ref = brute_pair_sum(pos, mass, soft, i)
        np.testing.assert_allclose(S[:, i], ref, rtol=1e-11,
                                   atol=1e-12 * np.abs(ref).max())


def test_subset_rows_match_full():
    ps = synth.config(1, n=512)
    S = oracle.forces(ps.pos, ps.mass, ps.soft)
    idx = np.array([511, 0, 17, 17, 300])
    Ss = oracle.forces(ps.pos, ps.mass, ps.soft, idx=idx)
    np.testing.assert_array_equal(Ss, S[:, idx])


def _clustered(n, seed):
    # a dense clump inside a wider cloud: many softened pairs
    rng = np.random.default_rng(seed)
    pos = np.concatenate([rng.normal(0, 0.05, (3, n // 2)),
                          rng.normal(0, 2.0, (3, n - n // 2))], axis=1)
    mass = rng.uniform(0.5, 5.0, n)
    soft = rng.uniform(0.01, 0.2, n)
    return np.ascontiguousarray(pos), mass, soft


@pytest.mark.parametrize("kind", ["config1", "clustered"])
def test_newtons_third_law(kind):
    if kind == "config1":
        ps = synth.config(1, n=1024)
        pos, mass, soft = ps.pos, ps.mass, ps.soft
    else:
        pos, mass, soft = _clustered(600, 5)
    S = oracle.forces(pos, mass, soft)
    net = np.abs((mass * S).sum(axis=1)).max()
    scale = (mass * np.linalg.norm(S, axis=0)).sum()
    assert net / scale < 1e-14


def test_translation_invariance_exact():
    # positions on a 2^-12 grid, shifted by 2^10: every difference is exact
    rng = np.random.default_rng(7)
    n = 300
    pos = np.round(rng.uniform(-4, 4, (3, n)) * 4096) / 4096
    mass = rng.uniform(1, 2, n)
    soft = rng.uniform(0.05, 0.4, n)
    S0 = oracle.forces(pos, mass, soft)
    S1 = oracle.forces(pos + 1024.0, mass, soft)
    np.testing.assert_array_equal(S0, S1)


def test_power_of_two_scaling_exact():
    pos, mass, soft = _clustered(300, 9)
    S0 = oracle.forces(pos, mass, soft)
    S1 = oracle.forces(pos * 4.0, mass * 8.0, soft * 4.0)
    # S scales as m / L^2: 8 / 16
    np.testing.assert_array_equal(S1, S0 * 0.5)


def test_permutation_equivariance():
    pos, mass, soft = _clustered(257, 11)
    perm = np.random.default_rng(3).permutation(257)
    S0 = oracle.forces(pos, mass, soft)
    S1 = oracle.forces(pos[:, perm], mass[perm], soft[perm])
    np.testing.assert_allclose(S1, S0[:, perm], rtol=1e-13,
                               atol=1e-15 * np.abs(S0).max())


def test_linearity_in_mass():
    pos, mass, soft = _clustered(200, 13)
    m2 = np.random.default_rng(4).uniform(0, 1, 200)
    Sa = oracle.forces(pos, mass, soft)
    Sb = oracle.forces(pos, m2, soft)
    Sab = oracle.forces(pos, mass + m2, soft)
    np.testing.assert_allclose(Sab, Sa + Sb, rtol=1e-12,
                               atol=1e-14 * np.abs(Sab).max())


def test_shell_theorem():
    # equal masses on a Fibonacci sphere (radius 1, total mass 1); massless
    # probes inside feel ~0, probes outside feel 1/r^2 towards the centre.
    m = 4000
    shell = fibonacci_sphere(m, 1.0)
    probes_in = np.array([[0.0, 0.3, 0.0, -0.2], [0.0, 0.0, 0.4, 0.1],
                          [0.0, 0.1, -0.3, 0.25]])
    dirs = fibonacci_sphere(5, 1.0)
    probes_out = np.concatenate([dirs * 2.5, dirs * 7.0], axis=1)
    pos = np.concatenate([shell, probes_in, probes_out], axis=1)
    n = pos.shape[1]
    mass = np.concatenate([np.full(m, 1.0 / m), np.zeros(n - m)])
    soft = np.zeros(n)
    idx = np.arange(m, n)
    S = oracle.forces(pos, mass, soft, idx=idx)
    k = probes_in.shape[1]
    # inside: residual far below the 1/R^2 = 1 scale of one wrong term
    assert np.linalg.norm(S[:, :k], axis=0).max() < 2e-3
    r = np.linalg.norm(probes_out, axis=0)
    expect = -probes_out / r ** 3
    assert _rel(S[:, k:], expect).max() < 1e-4


def test_uniform_ball_interior_field():
    # equal-mass lattice ball, density 1 per cell: interior S ~ -(4 pi/3) x
    pos = lattice_ball(14.0)
    n = pos.shape[1]
    mass = np.ones(n)
    soft = np.full(n, 0.3)
    r = np.linalg.norm(pos, axis=0)
    idx = np.nonzero((r > 2.0) & (r < 7.0))[0]
    S = oracle.forces(pos, mass, soft, idx=idx)
    expect = -(4.0 * math.pi / 3.0) * pos[:, idx]
    err = _rel(S, expect)
    assert np.median(err) < 5e-3
    assert err.max() < 3e-2


def test_potential_gradient_is_force():
    # d/dx_i of U = 1/2 sum_ij m_i m_j phi_ij equals -m_i S_i
    pos, mass, soft = _clustered(60, 21)
    S = oracle.forces(pos, mass, soft)

    def U(p):
        return 0.5 * float(np.dot(mass, oracle.potential(p, mass, soft)))

    for i in (0, 7, 45):
        for d in range(3):
            e = 1e-6
            pp = pos.copy(); pp[d, i] += e
            pm = pos.copy(); pm[d, i] -= e
            g = (U(pp) - U(pm)) / (2 * e)
            assert g == pytest.approx(-mass[i] * S[d, i], rel=2e-5,
                                      abs=1e-7 * np.abs(mass * S).max())


def test_kappa_reported():
    ps = synth.config(1, n=256)
    S, kap = oracle.forces(ps.pos, ps.mass, ps.soft, want_kappa=True)
    assert np.all(kap >= 1.0 - 1e-12)


def test_kappa_closed_form():
    # kappa_i = |(sum_j |t_jx|, sum_j |t_jy|, sum_j |t_jz|)| / |S_i| with
    # t_j = m_j (x_j - x_i) / r^3 (Newtonian pairs).  Particle 0 at the
    # origin, unit masses at (3, 0, 0), (0, 4, 0) and (-1, 0, 0):
    # t = (1/9, 0, 0), (0, 1/16, 0), (-1, 0, 0), so S = (-8/9, 1/16, 0) and
    # the absolute sums are (10/9, 1/16, 0).  Summing norms of the terms
    # instead (1/9 + 1/16 + 1), or dropping the absolute value, gives other
    # numbers.
    pos = np.array([[0.0, 3.0, 0.0, -1.0], [0.0, 0.0, 4.0, 0.0],
                    [0.0, 0.0, 0.0, 0.0]])
    mass = np.ones(4)
    soft = np.full(4, 1e-3)
    S, kap = oracle.forces(pos, mass, soft, idx=np.array([0]), want_kappa=True)
    np.testing.assert_allclose(S[:, 0], [-8.0 / 9.0, 1.0 / 16.0, 0.0], rtol=1e-15)
    expected = math.hypot(10.0 / 9.0, 1.0 / 16.0) / math.hypot(8.0 / 9.0, 1.0 / 16.0)
    assert kap[0] == pytest.approx(expected, rel=1e-14)
    # terms of one sign per component: kappa = 1 exactly
    S, kap = oracle.forces(pos[:, :3], mass[:3], soft[:3], idx=np.array([0]),
                           want_kappa=True)
    assert kap[0] == pytest.approx(1.0, rel=1e-15)
    # midway between two equal masses the pulls cancel: S = 0, kappa = inf
    pos2 = np.array([[-2.0, 0.0, 2.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    S, kap = oracle.forces(pos2, np.ones(3), np.full(3, 1e-3),
                           idx=np.array([1]), want_kappa=True)
    assert np.all(S[:, 0] == 0.0) and math.isinf(kap[0])
