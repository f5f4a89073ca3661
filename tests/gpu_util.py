"""Helpers shared by the GPU parity tests (marshalling only, no method arithmetic)."""
import sys

import numpy as np


def device():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch.device("cuda:0")


def make_system(cfg, pos, vel):
    import torch

    from paper_1705_04368_amd import System
    d = device()
    return System(cfg, torch.from_numpy(np.ascontiguousarray(pos, dtype=np.float32)).to(d),
                  torch.from_numpy(np.ascontiguousarray(vel, dtype=np.float32)).to(d))


def unwrapped(state, s):
    """Exact FP64 unwrapped positions ucell * s + off of a GPU state."""
    return state["ucell"].astype(np.float64) * s + state["off"].astype(np.float64)


def wrapped(state, s, mc):
    return np.mod(state["ucell"], mc).astype(np.float64) * s + state["off"].astype(np.float64)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def force_error(acc_gpu, acc_ref):
    """Per-particle |F_gpu - F_ref| / max(|F_ref|, F_rms)."""
    frms = np.sqrt(np.mean(np.sum(acc_ref ** 2, axis=1)))
    den = np.maximum(np.linalg.norm(acc_ref, axis=1), frms)
    return np.linalg.norm(acc_gpu.astype(np.float64) - acc_ref, axis=1) / den
