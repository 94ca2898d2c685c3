"""CPU oracle of the unsigned-nibble form with O(N) pre-sums -- TEST
INFRASTRUCTURE ONLY (see the package docstring for who may call it).

The paper's GPUs worked on the stored 4-bit values directly and paid for it
with O(N) extra bookkeeping next to the O(N^2) products (Sec. 2.3, "GPUs";
Table tab:computing lists a "Re-Order and Pre-Sum" task).  Written out: with
u = nibble in [0, 15] and the value x = u - 8 (offset encoding), for the
real and imaginary nibbles uR, uI of inputs i and j,

  Re V_ij = sum (uR_i uR_j + uI_i uI_j) - 8 (SR_i + SI_i + SR_j + SI_j) + 128 T
  Im V_ij = sum (uI_i uR_j - uR_i uI_j) + 8 (SR_i - SI_i) - 8 (SR_j - SI_j)

where SR_i = sum_t uR_i(t) and SI_i = sum_t uI_i(t) are the per-input
pre-sums.  This module computes exactly that: the unsigned products as int64
matrix products, the pre-sums as column sums, and the corrections.
"""
from __future__ import annotations

import numpy as np


def unsigned_nibbles(samples: np.ndarray, n_inputs: int | None = None, re_low: bool = False):
    """(uR, uI) int64 [T][N] in 0..15: the stored nibbles, no offset removed."""
    s = np.asarray(samples, dtype=np.uint8)
    n = s.shape[1] if n_inputs is None else n_inputs
    s = s[:, :n].astype(np.int64)
    hi, lo = s >> 4, s & 15
    return (lo, hi) if re_low else (hi, lo)


def presums(samples: np.ndarray, n_inputs: int | None = None, re_low: bool = False):
    """Per-input sums of the unsigned nibbles over time: (SR, SI) int64 [N]."""
    ur, ui = unsigned_nibbles(samples, n_inputs, re_low)
    return ur.sum(axis=0), ui.sum(axis=0)


def unsigned_products(samples: np.ndarray, n_inputs: int | None = None, re_low: bool = False):
    """(U_re, U_im) int64 [N][N]: sum_t uR_i uR_j + uI_i uI_j and
    sum_t uI_i uR_j - uR_i uI_j."""
    ur, ui = unsigned_nibbles(samples, n_inputs, re_low)
    return ur.T @ ur + ui.T @ ui, ui.T @ ur - ur.T @ ui


def correlate_presum(samples: np.ndarray, n_inputs: int | None = None, re_low: bool = False) -> np.ndarray:
    """V_ij from unsigned products plus pre-sum corrections, int64
    [N(N+1)/2][2], packed upper triangle in the order of oracle.correlate."""
    t = np.asarray(samples).shape[0]
    ure, uim = unsigned_products(samples, n_inputs, re_low)
    sr, si = presums(samples, n_inputs, re_low)
    re = ure - 8 * (sr + si)[:, None] - 8 * (sr + si)[None, :] + 128 * t
    im = uim + 8 * (sr - si)[:, None] - 8 * (sr - si)[None, :]
    iu, ju = np.triu_indices(re.shape[0])
    return np.stack([re[iu, ju], im[iu, ju]], axis=-1)
