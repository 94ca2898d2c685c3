"""CPU oracle for flag-aware correlation and its RFI-excision step -- TEST
INFRASTRUCTURE ONLY (see the package docstring for who may call it).

The paper sets aside flags and metadata beside every block of samples
(Sec. 2.2: 644 B per 4096 B of data; Table tab:data-flow: 4.0 Gb/s of flags
and metadata per node) and runs an "RFI Excision" task on the GPU ahead of
the correlation (Table tab:computing), but says neither how the flags are
laid out nor how RFI is found.  The readings taken here:

* a flag covers one input over a block of ``block_len`` consecutive samples
  (the last block of a call may be shorter): ``flags[b][i]`` nonzero means
  input i is flagged over block b;
* flag-aware correlation integrates V_ij = sum_t w_i(t) w_j(t) x_i(t)
  conj(x_j(t)) with w = 0 over flagged blocks and 1 elsewhere, and counts
  per baseline the samples that entered it, n_ij = sum_t w_i(t) w_j(t), so
  that V_ij / n_ij is the mean visibility over unflagged samples;
* RFI excision flags a block by its spectral kurtosis, the estimator of Nita
  and Gary (2010) applied to the power P = |x|^2 of the M samples of the
  block: with S1 = sum P and S2 = sum P^2,
      SK = (M + 1) / (M - 1) * (M S2 / S1^2 - 1),
  whose expectation is 1 for Gaussian noise.  A block is flagged when
  SK < lo or SK > hi (thresholds given as integer fractions of one common
  denominator) or when S1 = 0 (no power at all); blocks of fewer than two
  samples are never flagged.  The comparison is made exactly, in integers.

Everything here is plain numpy/Python: decoding, sums, comparisons with
Python integers, and the masked correlation through the C oracle.
"""
from __future__ import annotations

import numpy as np

from . import correlate, decode, tri


def n_blocks(n_samples: int, block_len: int) -> int:
    return (n_samples + block_len - 1) // block_len


def block_lengths(n_samples: int, block_len: int) -> np.ndarray:
    nb = n_blocks(n_samples, block_len)
    lens = np.full(nb, block_len, dtype=np.int64)
    if nb:
        lens[-1] = n_samples - (nb - 1) * block_len
    return lens


def sk_value(s1: int, s2: int, m: int):
    """The estimator as an exact fraction (numerator, denominator), or None
    where it is undefined (m < 2 or s1 = 0)."""
    if m < 2 or s1 == 0:
        return None
    return (m + 1) * (m * s2 - s1 * s1), (m - 1) * s1 * s1


def sk_flag(s1: int, s2: int, m: int, lo_num: int, hi_num: int, den: int) -> bool:
    """Flag decision for one block, in exact integer arithmetic."""
    if m < 2:
        return False
    v = sk_value(s1, s2, m)
    if v is None:
        return True
    num, dd = v                       # SK = num / dd, dd > 0
    return num * den < lo_num * dd or num * den > hi_num * dd


def sk_flags(samples: np.ndarray, n_inputs: int | None = None, block_len: int = 256,
             lo_num: int = 625, hi_num: int = 1375, den: int = 1000, re_low: bool = False) -> np.ndarray:
    """RFI flags uint8 [n_blocks][N]: 1 where the block's spectral kurtosis
    lies outside [lo_num / den, hi_num / den] or it carries no power."""
    re, im = decode(samples, n_inputs, re_low)
    p = re * re + im * im                               # int64 [T][N]
    t, n = p.shape
    nb = n_blocks(t, block_len)
    out = np.zeros((nb, n), dtype=np.uint8)
    for b in range(nb):
        blk = p[b * block_len:(b + 1) * block_len]
        m = blk.shape[0]
        s1 = blk.sum(axis=0)
        s2 = (blk * blk).sum(axis=0)
        for i in range(n):
            out[b, i] = sk_flag(int(s1[i]), int(s2[i]), m, lo_num, hi_num, den)
    return out


def mask_samples(samples: np.ndarray, flags: np.ndarray, block_len: int, n_inputs: int | None = None) -> np.ndarray:
    """Copy of [T][N] samples with every flagged (block, input) set to the
    zero sample 0x88 (value 0 + 0j)."""
    s = np.array(samples[:, :(samples.shape[1] if n_inputs is None else n_inputs)], dtype=np.uint8, copy=True)
    t = s.shape[0]
    for b in range(n_blocks(t, block_len)):
        rows = slice(b * block_len, min((b + 1) * block_len, t))
        s[rows, flags[b] != 0] = 0x88
    return s


def correlate_flagged(samples: np.ndarray, flags: np.ndarray, block_len: int,
                      n_inputs: int | None = None, re_low: bool = False):
    """(visibilities int64 [N(N+1)/2][2], counts int64 [N(N+1)/2]) of one
    flag-aware call: the correlation of the masked samples, and per pair the
    number of samples at which neither input is flagged."""
    s = mask_samples(samples, flags, block_len, n_inputs)
    t, n = s.shape
    vis = correlate(s, re_low=re_low)
    w = (np.asarray(flags)[:, :n] == 0).astype(np.int64)   # [nb][N]
    lens = block_lengths(t, block_len)
    full = (w * lens[:, None]).T @ w                        # n_ij = sum_b len_b w_i(b) w_j(b)
    iu, ju = np.triu_indices(n)
    return vis, full[iu, ju]


def counts_python(flags, block_len: int, n_samples: int, n: int) -> list:
    """Per-sample loops for tiny cases: n_ij = #{t : neither flagged at t}."""
    out = []
    for i in range(n):
        for j in range(i, n):
            c = 0
            for t in range(n_samples):
                b = t // block_len
                if not flags[b][i] and not flags[b][j]:
                    c += 1
            out.append(c)
    return out


def tri_count(n: int) -> int:
    return tri(n)
