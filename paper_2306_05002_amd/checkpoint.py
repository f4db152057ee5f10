"""Run checkpoints: the state, simulated time, step count and parameters of a
run in one .npz file, and their reload onto the GPU.

The kernels are deterministic and the device time step depends on the state
alone, so a run resumed from a checkpoint continues bit for bit as if it had
not stopped.  The file holds plain arrays (no pickled objects): U as float64
[field][element][node], t and step as scalars, the parameter dictionary and
the mesh description as JSON text.
"""

import json

import numpy as np
import torch


def save(path, U, t, step, params, mesh_desc=None):
    """Write U (device or host float64 tensor), t (float or 1-element tensor),
    step (int), params (the workloads-style parameter dict) and an optional
    mesh description dict to ``path`` (.npz)."""
    tv = float(t.detach().cpu().reshape(-1)[0]) if torch.is_tensor(t) else float(t)
    np.savez(path, U=U.detach().cpu().numpy(), t=np.float64(tv), step=np.int64(step),
             params=np.array(json.dumps(params, sort_keys=True)),
             mesh=np.array(json.dumps(mesh_desc or {}, sort_keys=True, default=list)))


def load(path, device="cuda"):
    """Read a checkpoint written by save(): dict(U (contiguous float64 tensor
    on ``device``), t (1-element float64 tensor on ``device``), step, params,
    mesh)."""
    with np.load(path, allow_pickle=False) as z:
        U = torch.from_numpy(np.ascontiguousarray(z["U"])).to(device)
        t = torch.tensor([float(z["t"])], dtype=torch.float64, device=device)
        out = dict(U=U, t=t, step=int(z["step"]), params=json.loads(str(z["params"])),
                   mesh=json.loads(str(z["mesh"])))
    return out
