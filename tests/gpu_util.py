"""Helpers shared by the GPU tests (inputs from ``synthetic``, results from
the HIP library through its binding)."""
import numpy as np


def torch():
    import torch as t
    return t


def to_dev(a: np.ndarray, dtype=None):
    t = torch()
    x = t.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        x = x.to(dtype)
    return x.cuda()


def to_np(x) -> np.ndarray:
    return x.detach().cpu().numpy()


def rel_err(a: np.ndarray, b: np.ndarray) -> float:
    """max over columns (last axis) of ||a - b|| / ||b||"""
    L = a.shape[-1]
    d = np.linalg.norm((a - b).reshape(-1, L), axis=0)
    n = np.linalg.norm(b.reshape(-1, L), axis=0)
    return float(np.max(d / n))


def lattice(U, kappa, csw, flags=0):
    from paper_0903_4936_amd import Lattice
    return Lattice(U, kappa, csw, flags=flags)
