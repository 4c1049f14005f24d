"""Helpers for the GPU parity tests (HIP library through its C ABI)."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2406_03121_amd import mess
    return mess


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def zeros(*shape):
    return torch.zeros(*shape, dtype=torch.float64, device="cuda")


def random_density(n, seed=0):
    from mess_inputs.generators import symmetric_density
    return symmetric_density(n, seed)


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    os.sync() if hasattr(os, "sync") else None
