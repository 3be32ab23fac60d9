"""Helpers for the GPU tests: move seeded numpy inputs to the device and
compare against the oracle.  No arithmetic of the method lives here."""
import numpy as np


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel_err(got, ref):
    """Per-particle |got - ref| / |ref| over columns of (3, n) arrays."""
    num = np.linalg.norm(got - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    out = np.where(den > 0, num / np.where(den > 0, den, 1.0), num)
    return out


def clustered(n, seed, zero_soft_frac=0.0):
    """A dense clump in a wide cloud, with coincident pairs: many softened
    pairs, r = 0 pairs and (optionally) zero softenings."""
    rng = np.random.default_rng(seed)
    pos = np.concatenate([rng.normal(0, 0.05, (3, n // 2)),
                          rng.normal(0, 2.0, (3, n - n // 2))], axis=1)
    if n >= 8:
        pos[:, 3] = pos[:, 1]
        pos[:, n - 1] = pos[:, n - 2]
    mass = rng.uniform(0.5, 5.0, n)
    soft = rng.uniform(0.01, 0.2, n)
    if zero_soft_frac > 0:
        soft[rng.uniform(size=n) < zero_soft_frac] = 0.0
    return np.ascontiguousarray(pos), mass, soft
