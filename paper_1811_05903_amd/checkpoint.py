"""Checkpoint and resume of a run on the GPU path.

The whole state of a run is (pos, vel, S) plus the scale factor reached,
the step index, the cosmology and the precision: S is carried between steps
(each KDK step makes exactly one pair-sum evaluation), so resuming from a
saved S continues the run bit for bit.  Saved as a numpy .npz file, loaded
with allow_pickle=False."""
from __future__ import annotations

import dataclasses

import numpy as np

from . import Cosmology

_FORMAT = 1


def save(path, pos, vel, acc, a: float, step: int, cosmo: Cosmology,
         precision: str = "fp64") -> None:
    """Write the device tensors pos, vel, acc ((3, n) float64) and the run
    scalars to path (.npz)."""
    fields = dataclasses.asdict(cosmo)
    np.savez(path, format=np.int64(_FORMAT),
             pos=pos.detach().cpu().numpy(), vel=vel.detach().cpu().numpy(),
             acc=acc.detach().cpu().numpy(), a=np.float64(a),
             step=np.int64(step), precision=np.array(precision),
             cosmo_keys=np.array(list(fields.keys())),
             cosmo_vals=np.array([np.nan if v is None else float(v)
                                  for v in fields.values()]))


def load(path, device="cuda"):
    """Read a checkpoint; returns (pos, vel, acc, a, step, cosmo, precision)
    with the arrays as float64 tensors on device."""
    import torch
    with np.load(path, allow_pickle=False) as z:
        if int(z["format"]) != _FORMAT:
            raise ValueError("unknown checkpoint format %d" % int(z["format"]))
        arrays = [torch.from_numpy(np.ascontiguousarray(z[k])).to(device)
                  for k in ("pos", "vel", "acc")]
        kw = {}
        for k, v in zip(z["cosmo_keys"].tolist(), z["cosmo_vals"].tolist()):
            if k == "omega_k":
                kw[k] = None if np.isnan(v) else v
            elif k in ("newtonian_test", "reversed_gravity", "periodic"):
                kw[k] = bool(v)
            else:
                kw[k] = v
        return (*arrays, float(z["a"]), int(z["step"]), Cosmology(**kw),
                str(z["precision"]))
