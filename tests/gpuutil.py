"""Helpers shared by the GPU parity tests (test code only)."""
import sys

import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    a = a.astype(np.complex128 if np.iscomplexobj(a) or np.iscomplexobj(b) else np.float64)
    b = b.astype(a.dtype)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def slots_of(gop, keys):
    return np.array([gop.slot(*key) for key in keys], dtype=np.int64)


def state_to_oracle(gop, oop, fields):
    """Gather a GPU field buffer into the oracle's unknown ordering."""
    f = fields.detach().cpu().numpy().astype(np.float64)
    e = f[slots_of(gop, oop.ne.keys)]
    h = f[slots_of(gop, oop.nh.keys)]
    return np.concatenate([e, h])


def oracle_to_state(gop, oop, x, dtype, device="cuda"):
    import torch
    f = np.zeros(gop.field_len)
    f[slots_of(gop, oop.ne.keys)] = x[:oop.Ne]
    f[slots_of(gop, oop.nh.keys)] = x[oop.Ne:]
    return torch.tensor(f, dtype=dtype, device=device)
