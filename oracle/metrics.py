"""Error measures of Section 3 (eqs. rel-err and ord-conv).

Test infrastructure only (see the package header).

rel_linf is eq. rel-err: max |exact - approx| / max |exact| over the grid.
rel_l2 is its L2 analogue ||exact - approx||_2 / ||exact||_2.
noc is eq. ord-conv: log2(eps_n / eps_2n).
"""
from __future__ import annotations

import math

import numpy as np


def rel_linf(approx, exact) -> float:
    approx = np.asarray(approx)
    exact = np.asarray(exact)
    den = np.max(np.abs(exact))
    return float(np.max(np.abs(approx - exact)) / den) if den > 0 else float(np.max(np.abs(approx)))


def rel_l2(approx, exact) -> float:
    approx = np.asarray(approx)
    exact = np.asarray(exact)
    den = np.linalg.norm(exact.ravel())
    return float(np.linalg.norm((approx - exact).ravel()) / den) if den > 0 else float(np.linalg.norm(approx.ravel()))


def noc(eps_n: float, eps_2n: float) -> float:
    return math.log2(eps_n / eps_2n)
