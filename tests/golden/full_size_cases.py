"""Full-size parity cases: the seeded inputs of the full-size workloads and
the names under which the oracle's outputs are recorded (as SHA-256 digests)
in ``full_size_sha256.txt``.

Only ``synth`` (seeded generators, none of the correlation arithmetic) and
numpy are used here; the digests are written by ``make_full_size_hashes.py``,
which calls the CPU oracle and nothing else.  GPU tests hash the library's
complete output for the same case and compare; on a mismatch they run the
oracle on that case and report the first differing pair.
"""
from __future__ import annotations

import hashlib
import os

import numpy as np

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
DIGESTS = os.path.join(HERE, "full_size_sha256.txt")

# streaming: device-sourced channels of N=2048, 256-sample frames, an export
# every SERVE_DUMP frames, each channel's source cycling SERVE_SRC_FRAMES
# distinct frames (so the exports cover different, wrapping frame windows)
SERVE_N = 2048
SERVE_FRAME = 256
SERVE_DUMP = 32
SERVE_SRC_FRAMES = 48
SERVE_CHANNELS = 4
SERVE_EXPORTS = 3


def vis_sha256(v) -> str:
    """Digest of a packed upper triangle [N(N+1)/2][2] as little-endian int32."""
    a = np.asarray(v)
    if a.dtype != np.int32:
        if a.size and (a.min() < -2 ** 31 or a.max() >= 2 ** 31):
            raise ValueError("visibilities out of int32 range")
        a = a.astype(np.int32)
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i4").tobytes()).hexdigest()


def channel_n2048():
    """The CHIME-shaped channel, N=2048, T=32768 (seed 2)."""
    return synth.chime_channel(2048, 32768, seed=2)


def channels16():
    """16 channels x N=2048, T uniform in [2048, 16384], 5% flagged (seed 3)."""
    return synth.batched_channels(n_channels=16, n_inputs=2048, seed=3)


def subarrays64():
    """64 sub-arrays, N in {256, 512, 1024, 2048}, T in {4096, 8192, 16384} (seed 4)."""
    return synth.subarray_batch(n_instances=64, seed=4)


def serve_source(c: int) -> np.ndarray:
    """Frames [SERVE_SRC_FRAMES][256][2048] of streaming channel c."""
    return synth.stream_frames(SERVE_N, SERVE_SRC_FRAMES, frame_len=SERVE_FRAME, seed=[50, c])


def serve_window(frames: np.ndarray, m: int) -> np.ndarray:
    """Samples [SERVE_DUMP * 256][N] of export m (frames m*D .. m*D+D-1, cyclic)."""
    f = frames[[(m * SERVE_DUMP + k) % frames.shape[0] for k in range(SERVE_DUMP)]]
    return np.ascontiguousarray(f.reshape(-1, frames.shape[2]))


def cases():
    """(name, samples [T][N]) of every recorded case, generated lazily."""
    yield "channel_n2048_t32768", channel_n2048()
    for k, x in enumerate(channels16()):
        yield f"channels16_c{k}", x
    for k, x in enumerate(subarrays64()):
        yield f"subarrays64_k{k}", x
    for c in range(SERVE_CHANNELS):
        src = serve_source(c)
        for m in range(SERVE_EXPORTS):
            yield f"serve_n2048_c{c}_e{m}", serve_window(src, m)


def load_digests() -> dict:
    out = {}
    with open(DIGESTS) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, digest, n, t = line.split()
            out[name] = (digest, int(n), int(t))
    return out
