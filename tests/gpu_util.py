"""Helpers for the GPU parity tests: move seeded inputs to the device, pack /
unpack k-space data, relative errors."""
import numpy as np


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.complex128).ravel()
    b = np.asarray(b, dtype=np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(a, dev="cuda"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def pack(ys_oracle):
    """oracle list of [C][M_p] -> [sum M_p][C] (the library's data layout)"""
    return np.concatenate([np.asarray(y).T for y in ys_oracle], axis=0)


def unpack(y, ks):
    """[sum M_p][C] -> list of [C][M_p]"""
    out, off = [], 0
    for k in ks:
        m = k.shape[0]
        out.append(np.asarray(y[off:off + m]).T)
        off += m
    return out


def say(msg):
    print(msg, flush=True)
