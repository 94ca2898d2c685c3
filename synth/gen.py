"""Seeded generators for the five synthetic workloads.

Sample format (Sec. 2.2, "Computational Requirements": each channelised
sample carries 4 bits of real and 4 bits of imaginary part): one byte per
complex sample, real part in the high nibble, imaginary part in the low
nibble, each stored offset-binary (stored nibble = value + 8).  Arrays are
time-major ``uint8[T][N]`` with the inputs of one time sample contiguous,
the layout the node's CPU hands each GPU after the corner turn (Sec. 2.3).

Value models (the paper has no signal model; these stand in for CHIME's
F-engine output and only need to look like it: a noise-dominated sky with a
weak common component and a few narrow-band tones):

* ``uniform_bytes``   every byte uniform on 0..255 (nibble values -8..7);
* ``chime_channel``   per-input complex Gaussian noise + a common sky signal
  at SNR 0.1 with a geometric phase per input + three tones, scaled by 3,
  rounded half-to-even and clipped to [-7, 7];
* ``gaussian_bytes``  independent complex Gaussian noise scaled by 2.5,
  rounded and clipped to [-7, 7].
"""
from __future__ import annotations

import numpy as np

FLAG_BYTE = 0x88          # value 0 + 0j: how a flagged input is represented
_CHUNK = 4096             # time samples generated per numpy chunk (memory bound)


def encode(q_re: np.ndarray, q_im: np.ndarray) -> np.ndarray:
    """Pack integer parts in [-8, 7] into offset-binary bytes (real high)."""
    q_re = np.asarray(q_re)
    q_im = np.asarray(q_im)
    if q_re.min(initial=0) < -8 or q_re.max(initial=0) > 7 \
            or q_im.min(initial=0) < -8 or q_im.max(initial=0) > 7:
        raise ValueError("sample parts must lie in [-8, 7]")
    return (((q_re + 8).astype(np.uint8) << 4) | (q_im + 8).astype(np.uint8)).astype(np.uint8)


def uniform_bytes(n_inputs: int, n_samples: int, seed=1) -> np.ndarray:
    """Every byte (hence every nibble) uniform: values -8..7 for both parts."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 256, size=(n_samples, n_inputs), dtype=np.uint8)


def _quantise(x: np.ndarray, scale: float) -> tuple[np.ndarray, np.ndarray]:
    re = np.clip(np.rint(scale * x.real), -7, 7).astype(np.int8)
    im = np.clip(np.rint(scale * x.imag), -7, 7).astype(np.int8)
    return re, im


def chime_channel(n_inputs: int, n_samples: int, seed=2, snr: float = 0.1,
                  tone_freqs=(0.0625, 0.19, 0.3125), tone_amp: float = 0.3,
                  scale: float = 3.0) -> np.ndarray:
    """One frequency channel of an N-input array (the N=2048 workload).

    x_i(t) = n_i(t) + s(t) e^{j phi_i} + sum_k A e^{j(2 pi f_k t + theta_ki)},
    n_i ~ CN(0,1), s ~ CN(0, snr), phi_i = 2 pi 0.01 (i mod 256).
    """
    rng = np.random.default_rng(seed)
    phi = 2 * np.pi * 0.01 * (np.arange(n_inputs) % 256)
    geo = np.exp(1j * phi).astype(np.complex64)
    theta = rng.uniform(0, 2 * np.pi, size=(len(tone_freqs), n_inputs))
    tone_phase = np.exp(1j * theta).astype(np.complex64)
    out = np.empty((n_samples, n_inputs), dtype=np.uint8)
    sq = np.float32(np.sqrt(0.5))
    for t0 in range(0, n_samples, _CHUNK):
        tc = min(_CHUNK, n_samples - t0)
        x = (rng.standard_normal((tc, n_inputs), dtype=np.float32)
             + 1j * rng.standard_normal((tc, n_inputs), dtype=np.float32)) * sq
        s = (rng.standard_normal(tc, dtype=np.float32)
             + 1j * rng.standard_normal(tc, dtype=np.float32)) * np.float32(np.sqrt(snr / 2))
        x += s[:, None] * geo[None, :]
        t = np.arange(t0, t0 + tc, dtype=np.float64)
        for k, f in enumerate(tone_freqs):
            osc = (tone_amp * np.exp(1j * 2 * np.pi * f * t)).astype(np.complex64)
            x += osc[:, None] * tone_phase[k][None, :]
        re, im = _quantise(x, scale)
        out[t0:t0 + tc] = encode(re, im)
    return out


def gaussian_bytes(n_inputs: int, n_samples: int, seed=4, scale: float = 2.5) -> np.ndarray:
    """Independent complex Gaussian noise per input, 4-bit quantised."""
    rng = np.random.default_rng(seed)
    out = np.empty((n_samples, n_inputs), dtype=np.uint8)
    sq = np.float32(np.sqrt(0.5))
    for t0 in range(0, n_samples, _CHUNK):
        tc = min(_CHUNK, n_samples - t0)
        x = (rng.standard_normal((tc, n_inputs), dtype=np.float32)
             + 1j * rng.standard_normal((tc, n_inputs), dtype=np.float32)) * sq
        re, im = _quantise(x, scale)
        out[t0:t0 + tc] = encode(re, im)
    return out


def flag_inputs(samples: np.ndarray, n_flag: int, seed) -> np.ndarray:
    """Set ``n_flag`` randomly chosen inputs to the zero sample (in place)."""
    rng = np.random.default_rng(seed)
    idx = rng.choice(samples.shape[1], size=n_flag, replace=False)
    samples[:, idx] = FLAG_BYTE
    return np.sort(idx)


def batched_channels(n_channels: int = 16, n_inputs: int = 2048, t_lo: int = 2048,
                     t_hi: int = 16384, flag_frac: float = 0.05, seed: int = 3):
    """Many frequency channels of one array: uneven T, 5% of inputs flagged."""
    rng = np.random.default_rng(seed)
    ts = rng.integers(t_lo, t_hi + 1, size=n_channels)
    n_flag = int(round(flag_frac * n_inputs))
    chans = []
    for c in range(n_channels):
        x = chime_channel(n_inputs, int(ts[c]), seed=[seed, c])
        flag_inputs(x, n_flag, seed=[seed, c, 1])
        chans.append(x)
    return chans


def subarray_batch(n_instances: int = 64, n_choices=(256, 512, 1024, 2048),
                   t_choices=(4096, 8192, 16384), seed: int = 4):
    """Independent sub-arrays of uneven N and T (4-bit Gaussian data)."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(n_choices, size=n_instances)
    ts = rng.choice(t_choices, size=n_instances)
    return [gaussian_bytes(int(ns[k]), int(ts[k]), seed=[seed, k]) for k in range(n_instances)]


def stream_frames(n_inputs: int, n_frames: int, frame_len: int = 256, seed=5) -> np.ndarray:
    """``n_frames`` consecutive frames of one channel, shape [F][frame_len][N]."""
    x = chime_channel(n_inputs, n_frames * frame_len, seed=seed)
    return x.reshape(n_frames, frame_len, n_inputs)


def rank1_tone(n_inputs: int, n_samples: int, seed=7, quarter_turns: int = 1):
    """Common tone x_i(t) = g_i * j^(k t) with Gaussian-integer gains g_i.

    Gains have parts in [-7, 7]; multiplying by a power of j permutes and
    negates the parts, so every sample stays in [-7, 7].  Returns the packed
    samples and the gains as (re, im) integer arrays.
    """
    rng = np.random.default_rng(seed)
    g_re = rng.integers(-7, 8, size=n_inputs)
    g_im = rng.integers(-7, 8, size=n_inputs)
    t = np.arange(n_samples)
    k = (quarter_turns * t) % 4
    # j^k rotates (a, b) -> (a, b), (-b, a), (-a, -b), (b, -a)
    re = np.where(k[:, None] == 0, g_re, np.where(k[:, None] == 1, -g_im,
                  np.where(k[:, None] == 2, -g_re, g_im)))
    im = np.where(k[:, None] == 0, g_im, np.where(k[:, None] == 1, g_re,
                  np.where(k[:, None] == 2, -g_im, -g_re)))
    return encode(re, im), g_re, g_im


def rfi_channel(n_inputs: int, n_samples: int, seed=6, block_len: int = 256, tone_frac: float = 0.03,
                burst_frac: float = 0.02, broadband_blocks: int = 1) -> np.ndarray:
    """A CHIME-shaped channel with radio-frequency interference injected in
    whole (block, input) cells of ``block_len`` samples:

    * narrow-band carriers: a tone of amplitude 6 turning a quarter cycle
      per sample, (6, 0), (0, 6), (-6, 0), (0, -6), ... -- constant power;
    * impulsive bursts: the cell silenced (zero samples) except four
      samples at -7-7j -- a few strong spikes;
    * broadband bursts: ``broadband_blocks`` whole blocks across every
      input turned into impulsive bursts.

    The rest is ``chime_channel`` data (seed ``seed``)."""
    x = chime_channel(n_inputs, n_samples, seed=seed)
    rng = np.random.default_rng([seed, 99])
    nb = (n_samples + block_len - 1) // block_len
    cells = nb * n_inputs
    pick = rng.permutation(cells)
    n_tone = int(round(tone_frac * cells))
    n_burst = int(round(burst_frac * cells))
    tone = encode(np.array([6, 0, -6, 0]), np.array([0, 6, 0, -6]))
    spike = encode(np.array([-7]), np.array([-7]))[0]
    for k, c in enumerate(pick[:n_tone + n_burst]):
        b, i = divmod(int(c), n_inputs)
        t0, t1 = b * block_len, min((b + 1) * block_len, n_samples)
        if k < n_tone:
            x[t0:t1, i] = tone[(np.arange(t0, t1) % 4)]
        else:
            x[t0:t1, i] = FLAG_BYTE
            where = rng.choice(t1 - t0, size=min(4, t1 - t0), replace=False)
            x[t0 + where, i] = spike
    for b in rng.choice(nb, size=min(broadband_blocks, nb), replace=False):
        t0, t1 = int(b) * block_len, min((int(b) + 1) * block_len, n_samples)
        x[t0:t1, :] = FLAG_BYTE
        for i in range(n_inputs):
            where = rng.choice(t1 - t0, size=min(4, t1 - t0), replace=False)
            x[t0 + where, i] = spike
    return x


def beam_weights(n_beams: int, n_inputs: int, seed=8, amplitude: float = 127.0) -> np.ndarray:
    """Phased-array weights int8 [B][N][2]: beam b steers by a phase ramp
    across the inputs, w_bi = A e^{-j 2 pi (b + 1) 0.37 i / N + j theta_b},
    rounded half to even and clipped to [-127, 127]."""
    rng = np.random.default_rng(seed)
    i = np.arange(n_inputs)
    theta = rng.uniform(0, 2 * np.pi, size=n_beams)
    ph = -2 * np.pi * (np.arange(1, n_beams + 1)[:, None] * 0.37 * i[None, :] / max(n_inputs, 1)) + theta[:, None]
    w = amplitude * np.exp(1j * ph)
    out = np.empty((n_beams, n_inputs, 2), dtype=np.int8)
    out[:, :, 0] = np.clip(np.rint(w.real), -127, 127)
    out[:, :, 1] = np.clip(np.rint(w.imag), -127, 127)
    return out
