"""GPU parity of the periodic pair sum (Sec. 2.2, Eqs. 2 and 5) and the
periodic equations of motion against the oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import dev, host, rel_err

pytestmark = pytest.mark.gpu

L = 50.0


@pytest.fixture(scope="module")
def st():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1811_05903_amd as m
    m.load()
    return m


def _box_set(n, seed):
    # uniform in the box, a dense clump, a coincident pair, and some
    # particles stored one box length outside
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, L, (3, n))
    pos[:, : n // 5] = 20.0 + rng.normal(0, 0.5, (3, n // 5))
    pos[:, 7] = pos[:, 3]
    k = min(40, n // 4)
    pos[:, n // 2: n // 2 + k] += L * rng.integers(-1, 2, (3, k))
    mass = rng.uniform(0.5, 2.0, n)
    soft = rng.uniform(0.02, 0.3, n)
    return np.ascontiguousarray(pos), mass, soft


@pytest.mark.parametrize("images", [1, 2])
@pytest.mark.parametrize("n", [1, 2, 257, 1537])
def test_periodic_forces_parity(st, images, n):
    pos, mass, soft = _box_set(max(n, 8), 3 + n)
    pos, mass, soft = np.ascontiguousarray(pos[:, :n]), mass[:n], soft[:n]
    ref = oracle.forces_periodic(pos, mass, soft, L, images)
    ctx = st.Context(0, precision="fp64")
    ctx.set_periodic(L, images)
    got = host(st.steps_forces(dev(pos), dev(mass), dev(soft), ctx=ctx))
    again = host(st.steps_forces(dev(pos), dev(mass), dev(soft), ctx=ctx))
    ctx.close()
    assert np.array_equal(got, again)
    if n < 2:
        assert np.all(got == 0.0)
        return
    err = rel_err(got, ref)
    print("periodic images=%d n=%d: median %.2e max %.2e" % (images, n, np.median(err), err.max()))
    assert err.max() <= 1e-12


@pytest.mark.parametrize("images", [1, 2])
def test_periodic_far_outside_box(st, images):
    # a third of the particles stored up to three box lengths outside: blocks
    # whose raw displacement range is too wide for the per-block image list
    # wrap each pair instead, next to blocks that take the list
    n = 1100
    pos, mass, soft = _box_set(n, 17)
    rng = np.random.default_rng(18)
    sel = rng.choice(n, n // 3, replace=False)
    pos[:, sel] += L * rng.integers(-3, 4, (3, sel.size))
    pos = np.ascontiguousarray(pos)
    ref = oracle.forces_periodic(pos, mass, soft, L, images)
    ctx = st.Context(0, precision="fp64")
    ctx.set_periodic(L, images)
    got = host(st.steps_forces(dev(pos), dev(mass), dev(soft), ctx=ctx))
    ctx.close()
    err = rel_err(got, ref)
    print("far outside, images=%d: median %.2e max %.2e" % (images, np.median(err), err.max()))
    assert err.max() <= 1e-12


@pytest.mark.parametrize("images,n,rows", [(1, 262144, 256), (2, 65536, 48),
                                           (1, 262144 + 37, 64), (2, 65536 + 37, 32)])
def test_periodic_uniform_box_sampled_rows(st, images, n, rows):
    # the timed periodic workload: uniform particles in a box of side 100,
    # N and image rule as timed (and with a ragged last tile), on
    # seeded-sampled rows
    Lb = 100.0
    rng = np.random.default_rng(40 + images)
    pos = rng.uniform(0, Lb, (3, n))
    mass, soft = rng.uniform(0.5, 2.0, n), np.full(n, 0.02 * Lb / n ** (1 / 3))
    idx = np.sort(np.random.default_rng(900 + images).choice(n, rows, replace=False))
    ref = oracle.forces_periodic(pos, mass, soft, Lb, images, idx=idx)
    print("uniform box images=%d n=%d: %d oracle rows" % (images, n, rows), flush=True)
    ctx = st.Context(0, precision="fp64")
    ctx.set_periodic(Lb, images)
    got = host(st.steps_forces(dev(pos), dev(mass), dev(soft), ctx=ctx))[:, idx]
    ctx.close()
    err = rel_err(got, ref)
    print("uniform box images=%d: median %.2e max %.2e" % (images, np.median(err), err.max()))
    assert err.max() <= 1e-12


@pytest.mark.parametrize("images", [1, 2])
def test_periodic_lattice_is_force_free(st, images):
    k = 5
    g = (np.arange(k) + 0.5) * (L / k)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.ascontiguousarray(np.stack([X.ravel(), Y.ravel(), Z.ravel()]))
    n = pos.shape[1]
    ctx = st.Context(0, precision="fp64")
    ctx.set_periodic(L, images)
    got = host(st.steps_forces(dev(pos), dev(np.full(n, 2.0)), dev(np.full(n, 0.1)), ctx=ctx))
    ctx.close()
    assert np.abs(got).max() < 1e-12 * 2.0 / (L / k) ** 2


def test_periodic_run_matches_oracle(st):
    n = 800
    pos, mass, soft = _box_set(n, 11)
    mass = mass * 1e12
    oc = oracle.Cosmology(H0=70.0, omega_m=0.3, omega_l=0.7, images=2, box_L=L)
    gc = st.Cosmology(70.0, 0.3, 0.7, periodic=True)
    grid = 0.2 * (1.5) ** (np.arange(11) / 10)
    vel = np.zeros_like(pos)
    po, vo, So = oracle.run(pos, vel, mass, soft, grid, oc)
    ctx = st.Context(0, precision="fp64")
    ctx.set_periodic(L, 2)
    p, v, m, h = dev(pos), dev(vel), dev(mass), dev(soft)
    st.run(p, v, m, h, grid, gc, ctx=ctx)
    ctx.close()
    dx = np.linalg.norm(host(p) - po, axis=0) / soft
    print("periodic run: |dx|/h median %.2e max %.2e" % (np.median(dx), dx.max()))
    assert np.median(dx) < 1e-10 and dx.max() < 1e-7


def test_periodic_mode_errors(st):
    import torch
    pos, mass, soft = _box_set(64, 2)
    p, v, m, h = dev(pos), dev(np.zeros_like(pos)), dev(mass), dev(soft)
    ctx = st.Context(0, precision="fp64")
    for L_bad, im in [(0.0, 1), (-1.0, 2), (float("nan"), 1), (10.0, 3)]:
        with pytest.raises(st.StepsError):
            ctx.set_periodic(L_bad, im)
    # periodic equations on an open context
    acc = st.steps_forces(p, m, h, ctx=ctx)
    with pytest.raises(st.StepsError):
        st.steps_step(p, v, m, h, acc, 0.5, 0.01, st.Cosmology(periodic=True), ctx=ctx)
    ctx.set_periodic(L, 2)
    acc = st.steps_forces(p, m, h, ctx=ctx)
    # spherical equations on a periodic context
    with pytest.raises(st.StepsError):
        st.steps_step(p, v, m, h, acc, 0.5, 0.01, st.Cosmology(), ctx=ctx)
    for call in (lambda: st.steps_potential(p, m, h, ctx=ctx),
                 lambda: st.steps_energy(p, v, m, h, 0.5, st.Cosmology(periodic=True), ctx=ctx)):
        with pytest.raises(st.StepsError) as ei:
            call()
        assert ei.value.code == st.STEPS_E_UNSUPPORTED
    ctx.set_precision("mixed")
    with pytest.raises(st.StepsError) as ei:
        st.steps_forces(p, m, h, ctx=ctx)
    assert ei.value.code == st.STEPS_E_UNSUPPORTED
    ctx.set_precision("fp64")
    ctx.set_periodic(0.0, 0)           # back to the open sphere
    st.steps_step(p, v, m, h, st.steps_forces(p, m, h, ctx=ctx), 0.5, 0.01,
                  st.Cosmology(), ctx=ctx)
    ctx.close()
    torch.cuda.synchronize()
