"""Seeded synthetic inputs for the X-engine correlation workloads.

This module only draws random numbers and encodes them into the packed
4+4-bit sample format; it holds none of the correlation arithmetic.  It is
the one piece of code shared by the CPU oracle's tests and the HIP path's
tests and benchmark.
"""
from .gen import (  # noqa: F401
    encode, uniform_bytes, chime_channel, gaussian_bytes, flag_inputs,
    batched_channels, subarray_batch, stream_frames, rank1_tone, rfi_channel, beam_weights,
)
