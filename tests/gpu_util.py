"""Helpers shared by the GPU parity tests (no arithmetic of the method here)."""
import numpy as np
import torch


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def host64(t):
    return t.detach().double().cpu().numpy()


def f32(a):
    """Round a float64 array to float32 and back, so the oracle sees the GPU's inputs."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def max_rel(got, want, floor=0.0):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return float(np.max(np.abs(got - want) / np.maximum(np.abs(want), floor)))
