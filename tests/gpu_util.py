"""Helpers shared by the GPU tests (no solver arithmetic here)."""
import sys

import numpy as np
import torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def to_np(t):
    return t.detach().cpu().numpy()


def rel_max(a, b):
    """max |a - b| / max |b|"""
    a, b = np.asarray(a), np.asarray(b)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def rel_l2(a, b):
    a, b = np.asarray(a), np.asarray(b)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def bf16_rne(x):
    """Round positive/negative finite doubles to the nearest bfloat16 value (ties to even),
    computed exactly in FP64 from the binary exponent: 8 significant bits."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)             # x = m 2^e, |m| in [0.5, 1)
    q = np.rint(m * 256.0)         # numpy rint: round half to even
    return np.ldexp(q, e - 8)


def rand_vec(n, seed):
    v = np.random.default_rng(seed).standard_normal((n, n, n))
    v[0] = v[-1] = 0
    v[:, 0] = v[:, -1] = 0
    v[:, :, 0] = v[:, :, -1] = 0
    return v
