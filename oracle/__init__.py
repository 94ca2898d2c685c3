"""CPU oracle for the X-engine correlation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never links or calls
it, and it imports nothing from the GPU package.

Three independent ways to get the same integers (Sec. 2.2, "Computational
Requirements": 4+4-bit complex samples, N(N+1)/2 products per sample
including autocorrelations, V_ij = sum_t x_i(t) conj(x_j(t))):

* ``correlate``        the plain C int64 nested loop in ``xcorr_oracle.c``;
* ``correlate_numpy``  decode + one complex128 matrix product X^T conj(X)
                       (exact: every partial sum is an integer far below 2^53);
* ``correlate_python`` Python ``complex`` arithmetic, for tiny inputs.

``oracle.flags`` holds the flag-aware correlation (per-baseline sample
counts) and its RFI-excision step (spectral kurtosis per block);
``oracle.presum`` the unsigned-nibble form with O(N) pre-sums;
``oracle.beams`` phased-array beamforming.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xcorr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None
_DUMMY = np.zeros(1, dtype=np.uint8)


def compile_source(src: str, out: str, native: bool = False) -> str:
    """Compile an oracle C source into a shared library (OpenMP).  The
    shipped build is portable (-O2); ``native`` builds for the host it runs
    on (-O3 -march=native), for timing the oracle there."""
    tmp = out + ".tmp"
    opt = ["-O3", "-march=native"] if native else ["-O2"]
    subprocess.check_call(["gcc", *opt, "-fopenmp", "-shared", "-fPIC", "-o", tmp, src])
    os.replace(tmp, out)
    return out


def build_native(out_dir: str) -> str:
    """The oracle compiled -O3 -march=native into ``out_dir`` (timing only)."""
    return compile_source(_SRC, os.path.join(out_dir, "liboracle_native.so"), native=True)


def build(force: bool = True) -> str:
    """Compile the C oracle next to its source."""
    if force or not os.path.exists(_LIB):
        compile_source(_SRC, _LIB)
    return _LIB


def load_library(path: str):
    """Open a compiled oracle library and declare its signatures."""
    lib = ctypes.CDLL(path)
    lib.xo_correlate.restype = ctypes.c_int
    lib.xo_correlate.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_void_p]
    lib.xo_num_threads.restype = ctypes.c_int
    lib.xo_set_threads.argtypes = [ctypes.c_int]
    lib.xo_set_threads.restype = None
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = load_library(_LIB)
    return _lib


def tri(n: int) -> int:
    """Number of (i <= j) pairs: the N(N+1)/2 of the cost model eta."""
    return n * (n + 1) // 2


def tri_index(i: int, j: int, n: int) -> int:
    """Row-major upper-triangle position of pair (i, j), i <= j."""
    return i * n - i * (i - 1) // 2 + (j - i)


def num_threads() -> int:
    return int(_load().xo_num_threads())


def correlate(samples: np.ndarray, n_inputs: int | None = None, re_low: bool = False,
              full: bool = False, _lib_override=None) -> np.ndarray:
    """C oracle.  ``samples`` is uint8 [T][stride]; the first ``n_inputs``
    columns are the inputs.  Returns int64 [N(N+1)/2, 2] (or [N, N, 2])."""
    samples = np.ascontiguousarray(samples, dtype=np.uint8)
    if samples.ndim != 2:
        raise ValueError("samples must be 2-D [T][stride]")
    t, stride = samples.shape
    n = stride if n_inputs is None else int(n_inputs)
    shape = (n, n, 2) if full else (tri(n), 2)
    out = np.zeros(shape, dtype=np.int64)
    lib = _load() if _lib_override is None else _lib_override
    ptr = samples.ctypes.data if samples.size else _DUMMY.ctypes.data
    rc = lib.xo_correlate(ptr, t, n, stride, int(re_low), int(full), out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected arguments")
    return out


def decode(samples: np.ndarray, n_inputs: int | None = None, re_low: bool = False):
    """Signed (re, im) int64 arrays [T][N] from packed offset-binary bytes."""
    s = np.asarray(samples, dtype=np.uint8)
    n = s.shape[1] if n_inputs is None else n_inputs
    s = s[:, :n].astype(np.int64)
    hi, lo = s >> 4, s & 15
    re, im = (lo, hi) if re_low else (hi, lo)
    return re - 8, im - 8


def correlate_numpy(samples: np.ndarray, n_inputs: int | None = None,
                    re_low: bool = False, full: bool = False) -> np.ndarray:
    """Second oracle: V = X^T conj(X) as one complex128 matrix product."""
    re, im = decode(samples, n_inputs, re_low)
    x = re.astype(np.float64) + 1j * im.astype(np.float64)      # [T][N]
    v = x.T @ np.conj(x)                                          # [N][N]
    if np.abs(v).max(initial=0) >= 2.0 ** 52:
        raise ValueError("too large for an exact float64 product")
    n = v.shape[0]
    if full:
        return np.stack([np.rint(v.real), np.rint(v.imag)], axis=-1).astype(np.int64)
    iu, ju = np.triu_indices(n)                                    # row-major i <= j
    return np.stack([np.rint(v.real[iu, ju]), np.rint(v.imag[iu, ju])], axis=-1).astype(np.int64)


def correlate_python(samples, n_inputs: int | None = None, re_low: bool = False) -> list:
    """Third oracle for tiny inputs: Python complex numbers, one pair at a time."""
    rows = [list(map(int, r)) for r in np.asarray(samples, dtype=np.uint8)]
    n = len(rows[0]) if (n_inputs is None and rows) else (n_inputs or 0)

    def x(b: int) -> complex:
        hi, lo = divmod(b, 16)
        return complex(lo - 8, hi - 8) if re_low else complex(hi - 8, lo - 8)

    out = []
    for i in range(n):
        for j in range(i, n):
            acc = 0j
            for r in rows:
                acc += x(r[i]) * x(r[j]).conjugate()
            out.append((int(acc.real), int(acc.imag)))
    return out
