"""Pins of the oracle's comoving energies (derived from Sec. 2.2 Eq. 8; the
paper gives no energy diagnostic): the gradient of U_c is the force of
Eq. 8, the Layzer-Irvine residual vanishes at second order, and the
Newtonian limit conserves K + W."""
import math

import numpy as np
import pytest

import oracle
import synth

COS = oracle.Cosmology(H0=70.0, omega_m=0.3, omega_l=0.7)


def _cloud(n, seed):
    rng = np.random.default_rng(seed)
    pos = np.ascontiguousarray(rng.normal(0.0, 3.0, (3, n)))
    vel = np.ascontiguousarray(rng.normal(0.0, 5.0, (3, n)))
    mass = rng.uniform(1e11, 4e11, n)
    soft = rng.uniform(0.05, 0.3, n)
    return pos, vel, mass, soft


def test_gradient_of_potential_energy_is_eq8_force():
    # -dU_c/dx_i = m_i (G S_i + (Omega_m H0^2 / 2) x_i)
    pos, vel, mass, soft = _cloud(40, 1)
    S = oracle.forces(pos, mass, soft)
    h0 = 70.0 * oracle.kms_to_mpc_per_gyr()
    G = oracle.G()
    a = 0.5

    def U(p):
        e = oracle.energy(p, vel, mass, soft, a, COS)
        return e["U_pair"] + e["U_radial"]

    for i in (0, 13, 39):
        for d in range(3):
            eps = 1e-5
            pp = pos.copy(); pp[d, i] += eps
            pm = pos.copy(); pm[d, i] -= eps
            g = -(U(pp) - U(pm)) / (2 * eps)
            want = mass[i] * (G * S[d, i] + 0.5 * 0.3 * h0 ** 2 * pos[d, i])
            assert g == pytest.approx(want, rel=2e-5, abs=1e-6 * abs(want) + 1e-30)


def test_kinetic_and_radial_closed_forms():
    pos, vel, mass, soft = _cloud(50, 2)
    a = 0.3
    e = oracle.energy(pos, vel, mass, soft, a, COS)
    h0 = 70.0 * oracle.kms_to_mpc_per_gyr()
    assert e["K"] == pytest.approx(0.5 * a * a * np.sum(mass * np.sum(vel ** 2, 0)), rel=1e-14)
    assert e["U_radial"] == pytest.approx(-0.25 * 0.3 * h0 ** 2 * np.sum(mass * np.sum(pos ** 2, 0)), rel=1e-14)
    assert e["W"] == pytest.approx((e["U_pair"] + e["U_radial"]) / a, rel=1e-14)
    np.testing.assert_allclose(e["P"], a * a * (mass * vel).sum(axis=1), rtol=1e-13)


def _li_residual(nsteps, form="t"):
    ps = synth.config(1, n=256)
    rng = np.random.default_rng(3)
    vel = np.ascontiguousarray(rng.normal(0.0, 2.0, ps.pos.shape))
    a0, a1 = 0.05, 0.06
    grid = a0 * (a1 / a0) ** (np.arange(nsteps + 1) / nsteps)
    p, v = ps.pos.copy(), vel.copy()
    S = oracle.forces(p, ps.mass, ps.soft)
    es = [oracle.energy(p, v, ps.mass, ps.soft, grid[0], COS)]
    for k in range(nsteps):
        oracle.kdk_step(p, v, ps.mass, ps.soft, S, grid[k], grid[k + 1] - grid[k], COS)
        es.append(oracle.energy(p, v, ps.mass, ps.soft, grid[k + 1], COS))
    scale = max(abs(e["W"]) for e in es)
    if form == "t":
        R = oracle.layzer_irvine(es, grid, COS)
    else:
        # the same law in the scale factor, d[a (K + W)]/da = -K (multiply
        # d(K+W)/dt = -H (2K + W) by a and use da/dt = a H); the integral of
        # K by the trapezoid rule over the steps
        R, acc = [0.0], 0.0
        for k in range(1, len(es)):
            acc += 0.5 * (es[k - 1]["K"] + es[k]["K"]) * (grid[k] - grid[k - 1])
            R.append(grid[k] * (es[k]["K"] + es[k]["W"])
                     - grid[0] * (es[0]["K"] + es[0]["W"]) + acc)
        scale = max(abs(grid[k] * es[k]["W"] - grid[0] * es[0]["W"])
                    for k in range(len(es)))
    return np.abs(R).max() / scale


def test_layzer_irvine_second_order():
    # |R|/|W| of the sparse 256-particle set: 1.6e-2 at 20 steps, 3.8e-3
    # at 40; a wrong sign or factor in K, W or the drag breaks the ratio 4
    r1, r2 = _li_residual(20), _li_residual(40)
    assert r1 < 5e-2
    assert r1 / r2 == pytest.approx(4.0, rel=0.25)


def test_layzer_irvine_scale_factor_form_second_order():
    # relative to the change of U_c = a W over the run
    r1, r2 = _li_residual(20, "a"), _li_residual(40, "a")
    assert r1 < 5e-2
    assert r1 / r2 == pytest.approx(4.0, rel=0.25)


def test_newtonian_limit_conserves_energy():
    c = oracle.Cosmology(G=1.0, newtonian_test=True)
    pos = np.array([[-0.25, 0.75], [0.0, 0.0], [0.0, 0.0]])
    vel = np.array([[0.0, 0.0], [-0.25, 0.75], [0.0, 0.0]])
    mass, soft = np.array([0.75, 0.25]), np.zeros(2)
    e0 = oracle.energy(pos, vel, mass, soft, 1.0, c)
    # two-body closed form: K = 1/2 sum m v^2, W = -G m1 m2 / r
    assert e0["K"] == pytest.approx(0.5 * (0.75 * 0.0625 + 0.25 * 0.5625), rel=1e-15)
    assert e0["W"] == pytest.approx(-0.75 * 0.25, rel=1e-15)
    S = oracle.forces(pos, mass, soft)
    p, v = pos.copy(), vel.copy()
    for k in range(2000):
        oracle.kdk_step(p, v, mass, soft, S, 0.0, 2 * math.pi / 500, c)
    e1 = oracle.energy(p, v, mass, soft, 1.0, c)
    assert (e1["K"] + e1["W"]) == pytest.approx(e0["K"] + e0["W"], rel=1e-4)
