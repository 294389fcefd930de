"""Shared helpers for the GPU parity tests (not a test module)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2504_19308_amd", "libamm.so")

# Parity bar for float32 mode: relative Frobenius error against the float64
# oracle on identical decompositions.
TOL_F32 = 1e-5


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def ctx():
    from paper_2504_19308_amd import Context
    return Context(0)


def f32(a):
    """Round to float32 and back: the exact values both sides consume."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def gpu(a):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32))).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel(x, y):
    d = np.linalg.norm(y)
    return float(np.linalg.norm(np.asarray(x) - np.asarray(y)) / (d if d > 0 else 1.0))


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def bf16(x):
    """Round to bfloat16 (nearest, ties to even) through float32, as float64:
    the exact values a bfloat16 operand holds (finite inputs)."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = a.view(np.uint32).astype(np.uint64)
    r = (((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)
