"""Checkpoint file round trip on the host (no GPU)."""

import numpy as np
import torch

from paper_2306_05002_amd import checkpoint, workloads


def test_checkpoint_round_trip_host(tmp_path):
    cfg = workloads.config("drop2d", n_elem=(3, 2))
    U = torch.randn(7, 6, 16, dtype=torch.float64, generator=torch.Generator().manual_seed(5))
    path = tmp_path / "c.npz"
    checkpoint.save(path, U, torch.tensor([0.125], dtype=torch.float64), 17, cfg["params"],
                    {"n_elem": list(cfg["n_elem"])})
    ck = checkpoint.load(path, device="cpu")
    assert torch.equal(ck["U"], U)
    assert float(ck["t"]) == 0.125 and ck["step"] == 17
    assert ck["params"]["gamma"] == list(cfg["params"]["gamma"])
    assert ck["mesh"] == {"n_elem": [3, 2]}
    with np.load(path, allow_pickle=False) as z:      # plain arrays only
        assert set(z.files) == {"U", "t", "step", "params", "mesh"}
