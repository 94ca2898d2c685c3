"""Full-size parity helpers for the GPU tests: compare a complete output of
the library with the oracle's recorded digest for the same seeded case; on a
mismatch, run the oracle on that case and name the first differing pair."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))

import full_size_cases as fc  # noqa: E402

import oracle  # noqa: E402

_DIGESTS = None


def digests() -> dict:
    global _DIGESTS
    if _DIGESTS is None:
        _DIGESTS = fc.load_digests()
    return _DIGESTS


def first_difference(got: np.ndarray, ref: np.ndarray, n: int) -> str:
    bad = np.flatnonzero((got != ref).any(axis=1))
    if bad.size == 0:
        return "no difference"
    k = int(bad[0])
    # pair (i, j) of packed index k: the last row i that starts at or before k
    i = max(r for r in range(n) if oracle.tri_index(r, r, n) <= k)
    j = i + (k - oracle.tri_index(i, i, n))
    return (f"{bad.size} of {len(ref)} pairs differ; first ({i}, {j}): "
            f"got {got[k].tolist()}, oracle {ref[k].tolist()}")


def assert_matches_oracle_digest(name: str, got, samples: np.ndarray):
    """``got``: the library's int32 [N(N+1)/2][2] output (tensor or array)."""
    if hasattr(got, "cpu"):
        got = got.cpu().numpy()
    got = np.asarray(got)
    want, n, t = digests()[name]
    assert (samples.shape[1], samples.shape[0]) == (n, t), f"{name}: case shape changed"
    if fc.vis_sha256(got) == want:
        return
    ref = oracle.correlate(np.ascontiguousarray(samples))
    raise AssertionError(f"{name}: output differs from the oracle: "
                         f"{first_difference(got.astype(np.int64), ref, n)}")
