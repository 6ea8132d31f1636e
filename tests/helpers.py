"""Shared set-up for the GPU parity tests: seeded inputs from ``workloads``,
expected values from ``oracle`` only."""
from __future__ import annotations

import functools
import sys

import numpy as np

import workloads as wl
from oracle import dirac as od
from oracle import pfe

# a_scale used where running the oracle's power iteration would be slow: any
# positive value is a valid input, both sides receive the same one.
A_SCALE_BOUND = 1.0 / (1.01 * 36.5)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).reshape(-1)) / np.linalg.norm(b.reshape(-1)))


@functools.lru_cache(maxsize=8)
def problem(name: str, exact_scale: bool = True):
    """(workload, links, oracle operator, a_scale, sigma, w, sources)."""
    wk = wl.WORKLOADS[name]
    U = wk.links()
    op = od.Dirac(U, wk.dims, wk.mass, wk.mu, wk.bc_t)
    if exact_scale:
        a = od.a_scale_from_radius(od.spectral_radius(op, wk.power_start(), 100))
    else:
        a = A_SCALE_BOUND
    sig, w = pfe.neuberger(wk.n_shift)
    return wk, U, op, a, sig, w, wk.sources()


def cuda(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()
