"""Shared helpers of the GPU parity tests: oracle tables cached per (kernel, n)."""
from __future__ import annotations

import functools
import math

import numpy as np

from oracle import moments

B = 2
A_DEFAULT = (B + math.sqrt(2) / 2 - 0.5) / 2

# Upper bounds of cond_2(I + kappa^2 A_n M) for the LS workload (contrast 0.5 cut(r), b = 2,
# default a): the oracle's dense SVD gives 8.49 / 8.38 / 8.34 (kappa = 20, n = 16 / 32 / 64),
# 29.1 / 27.7 / 27.4 (kappa = 40), 91 / 110 / 109 (kappa = 80).  Checked at n = 32 by
# tests/test_oracle_smoothing_ls.py.
COND_BOUND = {20.0: 10.0, 40.0: 35.0, 80.0: 150.0}

KERNELS = {
    "laplace": dict(family="log", scale=-1.0 / (2.0 * math.pi)),
    "log": dict(family="log", scale=1.0),
    "pow-1/2": dict(family="power", scale=1.0, gamma=-0.5),
    "pow-1/3": dict(family="power", scale=1.0, gamma=-1.0 / 3.0),
    "helm20": dict(family="helmholtz", scale=1.0, kappa=20.0),
    "helm40": dict(family="helmholtz", scale=1.0, kappa=40.0),
}


def oracle_kernel(name: str) -> moments.Kernel:
    k = KERNELS[name]
    return moments.Kernel(k["family"], k.get("scale", 1.0), k.get("gamma", 0.0), k.get("kappa", 0.0))


@functools.lru_cache(maxsize=32)
def oracle_table(name: str, n: int) -> np.ndarray:
    return moments.ghat_table(oracle_kernel(name), n, B, A_DEFAULT)


def plan_kwargs(name: str) -> dict:
    k = dict(KERNELS[name])
    return k
