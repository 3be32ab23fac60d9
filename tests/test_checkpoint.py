"""The checkpoint file format round-trips the state and run scalars
exactly (CPU tensors; the GPU resume test checks bitwise continuation)."""
import numpy as np
import pytest

import paper_1811_05903_amd as st
from paper_1811_05903_amd import checkpoint


@pytest.mark.parametrize("cosmo", [
    st.Cosmology(67.74, 0.3089, 0.6911),
    st.Cosmology(70.0, 0.3, 0.7, omega_k=0.0, G=2.5, reversed_gravity=True),
    st.Cosmology(G=1.0, newtonian_test=True),
    st.Cosmology(70.0, 0.3, 0.7, periodic=True),
])
def test_round_trip(tmp_path, cosmo):
    import torch
    rng = np.random.default_rng(1)
    pos, vel, acc = (torch.from_numpy(rng.normal(size=(3, 17))) for _ in range(3))
    path = str(tmp_path / "c.npz")
    checkpoint.save(path, pos, vel, acc, 0.123456789, 42, cosmo, "kahan")
    p, v, a_, a, k, c, prec = checkpoint.load(path, device="cpu")
    for x, y in ((p, pos), (v, vel), (a_, acc)):
        assert torch.equal(x, y)
    assert (a, k, prec) == (0.123456789, 42, "kahan")
    assert c == cosmo
