"""Ensemble parity at the size of workload 4: 64 members, N_b drawn from
[8192, 131072], sum N = 4.7e6, mixed precision in the workload (FP64 and
both mixed accumulations here).  At this size the library's work items
cover a member's whole j-range (or a few parts of it), a different layout
from the small test ensembles; every ensemble kernel is forced in turn and
every member is compared with the oracle on 256 seeded-sampled rows: at the
start (a zero-length run returns S of the initial positions) and after three
steps (the oracle's sums at the positions the GPU reached).  The two
smallest members' three-step FP64 trajectories are compared with the
oracle's own integration."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host

pytestmark = pytest.mark.gpu

ROWS = 256
SHAPES_F64 = [(2, 128, 2), (2, 128, 3), (4, 128, 2), (4, 128, 3), (1, 128, 6),
              (1, 256, 30)]
# one-sided (variant 2) and symmetric (variant 10: chunk-pair units of each
# member, one weight per unordered pair) ensemble kernels
SHAPES_MIXED = [(1, 128, 2), (2, 256, 2), (4, 256, 2), (2, 256, 10), (4, 256, 10)]


@pytest.fixture(scope="module")
def st():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1811_05903_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def ens():
    members = synth.ensemble(64, nsteps=100)
    offs = np.cumsum([0] + [m.n for m in members])
    cat = lambda key, axis: np.ascontiguousarray(
        np.concatenate([getattr(m, key) for m in members], axis=axis))
    pos, vel, mass, soft = cat("pos", 1), cat("vel", 1), cat("mass", 0), cat("soft", 0)
    rows = [np.sort(np.random.default_rng(700 + b).choice(m.n, ROWS, replace=False))
            for b, m in enumerate(members)]
    refs = [oracle.forces(m.pos, m.mass, m.soft, idx=r) for m, r in zip(members, rows)]
    print("workload-4 ensemble: %d members, N = %d" % (len(members), offs[-1]),
          flush=True)
    return members, offs, pos, vel, mass, soft, rows, refs


def _cosmos(st, members):
    return [st.Cosmology(m.cosmo.H0, m.cosmo.omega_m, m.cosmo.omega_l)
            for m in members]


def _run(st, ens, ctx, nsteps, a1):
    import torch
    members, offs, pos, vel, mass, soft = ens[:6]
    p, v = dev(pos), dev(vel)
    acc = torch.zeros_like(p)
    status = st.steps_batch_run(p, v, dev(mass), dev(soft), acc, offs,
                                _cosmos(st, members), [m.a0 for m in members],
                                a1, nsteps, flags=st.STEPS_BATCH_GRAPH, ctx=ctx)
    assert status == [0] * len(members)
    return host(p), host(v), host(acc)


def _check(prec, members, offs, acc, rows, refs, label):
    worst_med, worst_max = 0.0, 0.0
    for b, m in enumerate(members):
        got = acc[:, offs[b]:offs[b + 1]][:, rows[b]]
        err = np.linalg.norm(got - refs[b], axis=0) / np.linalg.norm(refs[b], axis=0)
        worst_med = max(worst_med, float(np.median(err)))
        worst_max = max(worst_max, float(err.max()))
        if prec == "fp64":
            assert err.max() <= 1e-12, (label, b, m.n, err.max())
        else:
            assert np.median(err) <= 1e-5 and err.max() <= 1e-3, \
                (label, b, m.n, np.median(err), err.max())
    print("%s: worst member median %.2e, worst max %.2e" % (label, worst_med, worst_max),
          flush=True)


@pytest.mark.parametrize("prec,shape",
                         [("fp64", s) for s in SHAPES_F64] +
                         [(p, s) for p in ("mixed", "kahan") for s in SHAPES_MIXED])
def test_config4_start_forces_every_kernel(st, ens, prec, shape):
    members, offs = ens[0], ens[1]
    rows, refs = ens[6], ens[7]
    print("forcing %s %s" % (prec, shape), flush=True)
    ctx = st.Context(0, precision=prec)
    ctx.set_tile(shape[0], shape[1], 1, shape[2])
    # a1 = a0: the step has dt = 0, so acc = S(initial positions)
    _, _, acc = _run(st, ens, ctx, 1, [m.a0 for m in members])
    tile = st.steps_batch_tile(ctx)
    ctx.close()
    assert (tile["r"], tile["tj"], tile["variant"]) == shape
    _check(prec, members, offs, acc, rows, refs,
           "%s %s (j parts %d)" % (prec, shape, tile["jsplit"]))


def test_config4_layout_has_whole_j_ranges(st, ens):
    # at this size the default mixed shapes need no j-splitting: the work
    # items of r = 1 and r = 2 kernels cover whole member j-ranges
    members = ens[0]
    for shape in SHAPES_MIXED[:2]:
        ctx = st.Context(0, precision="mixed")
        ctx.set_tile(shape[0], shape[1], 1, shape[2])
        _run(st, ens, ctx, 1, [m.a0 for m in members])
        tile = st.steps_batch_tile(ctx)
        ctx.close()
        assert tile["jsplit"] == 1, (shape, tile)


@pytest.mark.parametrize("prec", ["fp64", "mixed", "kahan"])
def test_config4_three_steps(st, ens, prec):
    members, offs = ens[0], ens[1]
    rows = ens[6]
    # the first three steps of each member's 100-step grid a0 -> 1
    a1 = [m.a0 * (m.a1 / m.a0) ** (3.0 / 100.0) for m in members]
    print("three steps, %s" % prec, flush=True)
    ctx = st.Context(0, precision=prec)
    p, v, acc = _run(st, ens, ctx, 3, a1)
    tile = st.steps_batch_tile(ctx)
    ctx.close()
    assert np.isfinite(p).all() and np.isfinite(v).all()
    # forces: the oracle's sums at the positions the GPU reached
    refs = [oracle.forces(p[:, offs[b]:offs[b + 1]], m.mass, m.soft, idx=rows[b])
            for b, m in enumerate(members)]
    _check(prec, members, offs, acc, rows, refs, "%s after 3 steps %s" % (prec, tile))
    if prec != "fp64":
        return
    # trajectories of the two smallest members against the oracle's
    for b in np.argsort([m.n for m in members])[:2]:
        m = members[b]
        g = m.a0 * (a1[b] / m.a0) ** (np.arange(4) / 3.0)
        g[0], g[-1] = m.a0, a1[b]
        oc = oracle.Cosmology(m.cosmo.H0, m.cosmo.omega_m, m.cosmo.omega_l)
        po, vo, _ = oracle.run(m.pos, m.vel, m.mass, m.soft, g, oc)
        sl = slice(offs[b], offs[b + 1])
        dx = np.linalg.norm(p[:, sl] - po, axis=0) / m.soft
        dv = np.linalg.norm(v[:, sl] - vo, axis=0) / np.linalg.norm(vo, axis=0).max()
        print("member %d n=%d: |dx|/h median %.2e max %.2e, |dv| max %.2e"
              % (b, m.n, np.median(dx), dx.max(), dv.max()), flush=True)
        assert np.median(dx) < 1e-10 and dx.max() < 1e-7 and dv.max() < 1e-9
