"""GPU path with reversed gravity (the glass relaxation of Sec. 3) against
the oracle, and the glass property at a size the oracle would take long
for."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
import synth
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def st():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1811_05903_amd as m
    m.load()
    return m


def _pair(st, c, rev=True):
    return (oracle.Cosmology(c.H0, c.omega_m, c.omega_l, c.omega_r, reversed_gravity=rev),
            st.Cosmology(c.H0, c.omega_m, c.omega_l, c.omega_r, reversed_gravity=rev))


def nn_cv(pos, radius, inner=0.8):
    d, _ = cKDTree(pos.T).query(pos.T, k=2)
    keep = np.linalg.norm(pos, axis=0) < inner * radius
    return d[keep, 1].std() / d[keep, 1].mean()


def test_reversed_trajectory_and_energy_parity(st):
    ps = synth.poisson_ball(1500, 80.0, synth.Cosmo(67.74, 0.3089, 0.6911), seed=5,
                            nsteps=40)
    grid = ps.a_grid()
    oc, gc = _pair(st, ps.cosmo)
    po, vo, So = oracle.run(ps.pos, ps.vel, ps.mass, ps.soft, grid, oc)
    p, v, m, h = dev(ps.pos), dev(ps.vel), dev(ps.mass), dev(ps.soft)
    st.run(p, v, m, h, grid, gc)
    dx = np.linalg.norm(host(p) - po, axis=0) / ps.soft
    print("reversed gravity, 40 steps: |dx|/h median %.2e max %.2e"
          % (np.median(dx), dx.max()))
    assert np.median(dx) < 1e-10 and dx.max() < 1e-7
    eo = oracle.energy(po, vo, ps.mass, ps.soft, grid[-1], oc)
    eg = st.steps_energy(dev(po), dev(vo), m, h, grid[-1], gc)
    for key in ("K", "W", "U_pair", "U_radial"):
        assert eg[key] == pytest.approx(eo[key], rel=1e-12), key
    assert eo["U_pair"] > 0.0          # repulsive pair energy


def test_glass_forms_on_the_gpu(st):
    R = 150.0
    ps = synth.poisson_ball(32768, R, synth.Cosmo(67.74, 0.3089, 0.6911), seed=6)
    cv0 = nn_cv(ps.pos, R)
    _, gc = _pair(st, ps.cosmo)
    p, v, m, h = dev(ps.pos), dev(ps.vel), dev(ps.mass), dev(ps.soft)
    st.run(p, v, m, h, ps.a_grid(), gc)
    q = host(p)
    cv1 = nn_cv(q, R)
    rms0 = np.sqrt(np.mean(np.sum(ps.pos ** 2, 0)))
    rms1 = np.sqrt(np.mean(np.sum(q ** 2, 0)))
    print("glass N=32768: nearest-neighbour CV %.3f -> %.3f, rms radius %.4f -> %.4f"
          % (cv0, cv1, rms0, rms1))
    assert cv0 > 0.3 and cv1 < 0.15
    assert rms1 == pytest.approx(rms0, rel=0.01)


def test_reversed_gravity_in_the_ensemble(st):
    # two members, one reversed: each matches its own oracle run
    import torch
    c = synth.Cosmo(67.74, 0.3089, 0.6911)
    # the ordinary-gravity member over a short range only: a Poisson ball
    # collapsing from a = 0.01 in 12 steps amplifies rounding-level force
    # differences to ~1e-6 h in a few close pairs
    members = [synth.poisson_ball(700, 60.0, c, seed=11, nsteps=12),
               synth.poisson_ball(900, 70.0, c, seed=12, a0=0.5, a1=0.6, nsteps=12)]
    revs = [True, False]
    offs = np.cumsum([0] + [s.n for s in members])
    cat = lambda k, ax: np.ascontiguousarray(np.concatenate([getattr(s, k) for s in members], axis=ax))
    p, v = dev(cat("pos", 1)), dev(cat("vel", 1))
    acc = torch.zeros_like(p)
    gcs = [st.Cosmology(67.74, 0.3089, 0.6911, reversed_gravity=r) for r in revs]
    status = st.steps_batch_run(p, v, dev(cat("mass", 0)), dev(cat("soft", 0)), acc,
                                offs, gcs, [s.a0 for s in members],
                                [s.a1 for s in members], 12)
    assert status == [0, 0]
    q = host(p)
    for b, (s, r) in enumerate(zip(members, revs)):
        po, _, _ = oracle.run(s.pos, s.vel, s.mass, s.soft, s.a_grid(),
                              oracle.Cosmology(67.74, 0.3089, 0.6911, reversed_gravity=r))
        dx = np.linalg.norm(q[:, offs[b]:offs[b + 1]] - po, axis=0) / s.soft
        assert np.median(dx) < 1e-10 and dx.max() < 1e-7, (b, dx.max())
