"""GPU test of the allocation-free entry point steps_forces_noalloc (fixed
device scratch): its output against steps_forces on the same inputs, on
calls in a row with shrinking n (each call reuses the scratch the previous
one left), no change of free device memory across calls, and its argument
errors."""
import numpy as np
import pytest

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


def _rel(a, b):
    return np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)


def test_noalloc_matches_steps_forces_on_calls_in_a_row(st):
    import torch
    # sorted matrix-core shape, then sorted VALU, then unsorted: three
    # layouts of the fixed scratch, each call smaller than the one before
    for k, n in enumerate((262144, 200001, 40000, 5000)):
        ps = synth.config(2, n=n)
        pos, mass, soft = dev(ps.pos), dev(ps.mass), dev(ps.soft)
        print("noalloc call %d: n=%d" % (k, n), flush=True)
        got = torch.full((3, n), np.nan, dtype=torch.float64, device="cuda")
        st.steps_forces_noalloc(pos, mass, soft, got)
        ref = st.steps_forces(pos, mass, soft)
        torch.cuda.synchronize()
        g, r = host(got), host(ref)
        assert np.isfinite(g).all()
        err = _rel(g, r)
        print("n=%d: max rel difference to steps_forces %.2e" % (n, err.max()), flush=True)
        assert err.max() <= 1e-12
        rows = np.sort(np.random.default_rng(k).choice(n, 64, replace=False))
        ora = oracle.forces(ps.pos, ps.mass, ps.soft, idx=rows)
        assert _rel(g[:, rows], ora).max() <= 1e-12


def test_noalloc_allocates_nothing(st):
    import torch
    ps = synth.config(2, n=150000)
    small = 30000
    pos, mass, soft = dev(ps.pos), dev(ps.mass), dev(ps.soft)
    pos_s, mass_s, soft_s = dev(ps.pos[:, :small]), dev(ps.mass[:small]), dev(ps.soft[:small])
    acc = torch.empty((3, ps.n), dtype=torch.float64, device="cuda")
    acc_s = torch.empty((3, small), dtype=torch.float64, device="cuda")
    # first calls of each shape (the runtime sets up code objects and the
    # per-lane spill memory of a kernel on its first launch)
    st.steps_forces_noalloc(pos, mass, soft, acc)
    st.steps_forces_noalloc(pos_s, mass_s, soft_s, acc_s)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(3):
        st.steps_forces_noalloc(pos, mass, soft, acc)
        st.steps_forces_noalloc(pos_s, mass_s, soft_s, acc_s)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
    ref = st.steps_forces(pos_s, mass_s, soft_s)
    assert _rel(host(acc_s), host(ref)).max() <= 1e-12


def test_noalloc_argument_errors(st):
    import torch
    n = 262145
    p = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    m = torch.ones(n, dtype=torch.float64, device="cuda")
    h = torch.ones(n, dtype=torch.float64, device="cuda")
    a = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    with pytest.raises(st.StepsError) as ei:   # above the fixed-scratch limit
        st.steps_forces_noalloc(p, m, h, a)
    assert ei.value.code == st.STEPS_E_INVAL and "allocation-free" in str(ei.value)
    q = torch.zeros((3, 1000), dtype=torch.float64, device="cuda")
    with pytest.raises(st.StepsError):         # acc aliases pos
        st.steps_forces_noalloc(q, m[:1000], h[:1000], q)
    # n = 1: no pair, S = 0
    one = st.steps_forces_noalloc(p[:, :1].contiguous(), m[:1], h[:1],
                                  torch.full((3, 1), 7.0, dtype=torch.float64,
                                             device="cuda"))
    assert np.all(host(one) == 0.0)
    assert np.all(host(a) == 0.0)             # refused calls wrote nothing
