"""Helpers shared by the GPU tests: move a workload to the device and compare
GPU results with the CPU reference."""
from __future__ import annotations

import numpy as np
import torch

import paper_1809_04600_amd as P


def device_inputs(x):
    h1 = torch.from_numpy(np.ascontiguousarray(x.h1)).cuda()
    eri = torch.from_numpy(np.ascontiguousarray(x.eri)).cuda()
    dets = P.dets_tensor(x.dets)
    c = torch.from_numpy(np.ascontiguousarray(x.c)).cuda()
    return h1, eri, dets, c


def context(x):
    h1, eri, dets, c = device_inputs(x)
    ctx = P.Context(h1, eri, x.wl.n_alpha, x.wl.n_beta)
    return ctx, dets, c


def sort_keys(keys: np.ndarray, *extra):
    """Lexicographic order on (word3, word2, word1, word0, extra...)."""
    cols = [e for e in reversed(extra)] + [keys[:, 0], keys[:, 1], keys[:, 2], keys[:, 3]]
    return np.lexsort(cols)


def keys_np(t: torch.Tensor) -> np.ndarray:
    return P.dets_numpy(t).reshape(-1, 4)
