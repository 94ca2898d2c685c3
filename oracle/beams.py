"""CPU oracle of phased-array beamforming -- TEST INFRASTRUCTURE ONLY (see
the package docstring for who may call it).

The paper's nodes form 10 phased-array beams for pulsar timing from the same
channelised samples (Sec. 2.1; "Pulsar Beamforming" in Table
tab:computing) and export them at 0.25 Gb/s per node (Table tab:data-flow:
4 channels x 10 beams x 390625 samples/s leaves 16 bits per complex beam
sample).  The paper gives neither the weights' precision nor the output
scaling.  The readings taken here:

* beam b at time t is y_b(t) = sum_i w_bi x_i(t), with complex integer
  weights w_bi whose parts lie in [-127, 127] (the phase and gain of input i
  for beam b);
* the exact sums are int32 (|y| <= N * 2 * 8 * 127 fits for N < 2^17);
* the exported form is 8 + 8 bits: each part divided by 2^shift, rounded
  half to even, and clipped to [-127, 127].
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from . import decode


def beamform(samples: np.ndarray, weights: np.ndarray, n_inputs: int | None = None,
             re_low: bool = False) -> np.ndarray:
    """Exact beams int64 [T][B][2] for weights int [B][N][2] (re, im)."""
    xr, xi = decode(samples, n_inputs, re_low)                  # int64 [T][N]
    w = np.asarray(weights, dtype=np.int64)
    wr, wi = w[:, :, 0], w[:, :, 1]                             # [B][N]
    yr = xr @ wr.T - xi @ wi.T                                  # (xr + j xi)(wr + j wi)
    yi = xr @ wi.T + xi @ wr.T
    return np.stack([yr, yi], axis=-1)


def quantize(beams: np.ndarray, shift: int) -> np.ndarray:
    """8-bit parts: round(y / 2^shift) half to even, clipped to [-127, 127]."""
    flat = [max(-127, min(127, round(Fraction(int(v), 1 << shift)))) for v in np.asarray(beams).ravel()]
    return np.array(flat, dtype=np.int8).reshape(np.asarray(beams).shape)


def beamform_python(samples, weights, n_inputs: int | None = None) -> list:
    """Python complex numbers, for tiny inputs: [t][b] -> (re, im)."""
    rows = [list(map(int, r)) for r in np.asarray(samples, dtype=np.uint8)]
    w = np.asarray(weights)
    n = w.shape[1] if n_inputs is None else n_inputs
    out = []
    for r in rows:
        xs = [complex((b >> 4) - 8, (b & 15) - 8) for b in r[:n]]
        out.append([(int(s.real), int(s.imag)) for s in
                    (sum(complex(int(w[bb, i, 0]), int(w[bb, i, 1])) * xs[i] for i in range(n))
                     for bb in range(w.shape[0]))])
    return out
