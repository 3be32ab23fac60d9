"""GPU parity of the adaptive step of Eq. 12 (steps_adaptive_dt,
steps_run_adaptive) against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import clustered, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def st():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1811_05903_amd as m
    m.load()
    return m


def _cosmos(st, c, newtonian=False):
    return (oracle.Cosmology(c.H0, c.omega_m, c.omega_l, c.omega_r,
                             G=1.0 if newtonian else None, newtonian_test=newtonian),
            st.Cosmology(c.H0, c.omega_m, c.omega_l, c.omega_r,
                         G=1.0 if newtonian else 0.0, newtonian_test=newtonian))


@pytest.mark.parametrize("newtonian", [False, True])
@pytest.mark.parametrize("eps,dt_max", [(1e-2, 1e3), (1e-4, 1e3), (1e-2, 1e-3)])
def test_adaptive_dt_parity(st, newtonian, eps, dt_max):
    ps = synth.config(2, n=3000)
    pos, mass, soft = clustered(3000, 51, 0.0)
    pos = pos * 50.0
    rng = np.random.default_rng(8)
    vel = np.ascontiguousarray(rng.normal(0.0, 5.0, pos.shape))
    mass = mass * 1e11
    oc, gc = _cosmos(st, ps.cosmo, newtonian)
    S = oracle.forces(pos, mass, soft)
    want = oracle.adaptive_dt(pos, vel, soft, S, 0.4, oc, eps, dt_max)
    acc = st.steps_forces(dev(pos), dev(mass), dev(soft))
    got = st.steps_adaptive_dt(dev(pos), dev(vel), dev(soft), acc, 0.4, gc, eps, dt_max)
    assert got[0] == pytest.approx(want[0], rel=1e-13)
    assert got[1] == pytest.approx(want[1], rel=1e-12)


def test_run_adaptive_matches_oracle(st):
    ps = synth.config(1, n=1024)
    oc, gc = _cosmos(st, ps.cosmo)
    po, vo, So, grid = oracle.run_adaptive(ps.pos, ps.vel, ps.mass, ps.soft,
                                           0.02, 0.05, oc, 1e-2, 1.0)
    p, v = dev(ps.pos), dev(ps.vel)
    acc, steps, reached = st.steps_run_adaptive(p, v, dev(ps.mass), dev(ps.soft),
                                                0.02, 0.05, gc, 1e-2, 1.0)
    assert steps == len(grid) - 1 and reached == 0.05
    dx = np.linalg.norm(host(p) - po, axis=0) / ps.soft
    print("adaptive run: %d steps, |dx|/h median %.2e max %.2e"
          % (steps, np.median(dx), dx.max()))
    assert np.median(dx) < 1e-10 and dx.max() < 1e-7
    rel = np.linalg.norm(host(acc) - So, axis=0) / np.linalg.norm(So, axis=0)
    assert np.median(rel) < 1e-10


def test_run_adaptive_cap_and_errors(st):
    import torch
    ps = synth.config(1, n=500)
    _, gc = _cosmos(st, ps.cosmo)
    p, v, m, h = dev(ps.pos), dev(ps.vel), dev(ps.mass), dev(ps.soft)
    _, steps, reached = st.steps_run_adaptive(p, v, m, h, 0.02, 0.05, gc,
                                              1e-2, 1.0, max_steps=7)
    assert steps == 7 and 0.02 < reached < 0.05
    _, steps, reached = st.steps_run_adaptive(p, v, m, h, 0.03, 0.03, gc, 1e-2, 1.0)
    assert steps == 0 and reached == 0.03
    acc = st.steps_forces(p, m, h)
    for bad in [dict(eps=0.0), dict(eps=-1.0), dict(dt_max=0.0),
                dict(eps=float("nan"))]:
        kw = dict(eps=1e-2, dt_max=1.0)
        kw.update(bad)
        with pytest.raises(st.StepsError):
            st.steps_adaptive_dt(p, v, h, acc, 0.03, gc, kw["eps"], kw["dt_max"])
    with pytest.raises(st.StepsError):
        st.steps_run_adaptive(p, v, m, h, 0.05, 0.02, gc, 1e-2, 1.0)
    e = torch.empty((3, 0), dtype=torch.float64, device="cuda")
    z = torch.empty(0, dtype=torch.float64, device="cuda")
    dt, da = st.steps_adaptive_dt(e, e, z, e, 0.03, gc, 1e-2, 0.5)
    assert dt == 0.5 and da > 0.0
    # zero softening: Eq. 12 gives a zero step (the oracle says 0 as well)
    h0 = h.clone()
    h0[5] = 0.0
    with pytest.raises(st.StepsError) as ei:
        st.steps_adaptive_dt(p, v, h0, acc, 0.03, gc, 1e-2, 1.0)
    assert "zero softening" in str(ei.value)
    oc, _ = _cosmos(st, ps.cosmo)
    soft0 = ps.soft.copy()
    soft0[5] = 0.0
    assert oracle.adaptive_dt(host(p), host(v), soft0, host(acc), 0.03, oc, 1e-2, 1.0)[0] == 0.0
