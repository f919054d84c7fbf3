"""Seeded synthetic MWA-shaped voltage samples, packed 4+4-bit per byte.

This module is the single input generator shared by the tests, the benchmark
and the checks of the CPU oracle.  It holds no correlation arithmetic and no
decoding: it only draws samples and encodes them.

Signal (per input i, fine channel f, time sample t), as used by every workload:

    re = clip(rint(sigma * n1 + A * cos(2*pi*nu*t + phi_i)), -7, 7)
    im = clip(rint(sigma * n2 + A * sin(2*pi*nu*t + phi_i)), -7, 7)

with n1, n2 ~ N(0, 1), sigma = 2.5, A = 2.0, nu = 1/16 cycles per sample, and
one phase phi_i ~ U[0, 2*pi) per input shared by all channels.  The paper's
samples are 4-bit two's complement real and imaginary parts with the code -8
reserved for invalid data (Appendix A, data-format list); the generator clips
to [-7, 7] so it never emits the invalid code.  The real part is stored in the
high nibble, the imaginary part in the low nibble.

Determinism: every (seed, array, channel) triple has its own counter-based
Philox stream, so any subset of channels can be regenerated independently and
in any order, e.g. to check sampled channels of a multi-gigabyte buffer.
"""

from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

SEED_BASE = 150105992
SIGMA = 2.5
TONE_AMP = 2.0
TONE_NU = 1.0 / 16.0

LAYOUT_TFI = 0  # byte offset (t * F + f) * N + i   (time, channel, input)
LAYOUT_FTI = 1  # byte offset (f * T + t) * N + i   (channel, time, input)

_PHASE_STREAM = 0xFFFFFFFF


def config_seed(k: int) -> int:
    """Seed of workload k (0-based), as used by tests and the benchmark."""
    return SEED_BASE + k


def _rng(seed: int, array: int, stream: int) -> np.random.Generator:
    key = np.array([seed & 0xFFFFFFFFFFFFFFFF, ((array & 0xFFFFFFFF) << 32) | (stream & 0xFFFFFFFF)],
                   dtype=np.uint64)
    return np.random.Generator(np.random.Philox(key=key))


def phases(seed: int, array: int, n_inputs: int) -> np.ndarray:
    """Per-input tone phase in [0, 2*pi), shared by all channels of an array."""
    return _rng(seed, array, _PHASE_STREAM).uniform(0.0, 2.0 * np.pi, size=n_inputs)


def pack(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """Encode integer parts in [-8, 7] as one byte: high nibble re, low nibble im."""
    re = np.asarray(re, dtype=np.int64)
    im = np.asarray(im, dtype=np.int64)
    if re.size and (re.min() < -8 or re.max() > 7 or im.min() < -8 or im.max() > 7):
        raise ValueError("4-bit parts must lie in [-8, 7]")
    return (((re & 0xF) << 4) | (im & 0xF)).astype(np.uint8)


def channel_samples(seed: int, array: int, channel: int, n_inputs: int, n_time: int,
                    phi: np.ndarray | None = None, t0: int = 0) -> np.ndarray:
    """Packed samples of one channel, shape (n_time, n_inputs), uint8.

    ``t0`` only shifts the tone's time origin; the noise stream always starts
    at the beginning of the (seed, array, channel) stream.
    """
    if phi is None:
        phi = phases(seed, array, n_inputs)
    rng = _rng(seed, array, channel)
    noise = rng.standard_normal((n_time, n_inputs, 2), dtype=np.float32)
    # The tone has period 16 samples: tabulate one period per input.
    ang = 2.0 * np.pi * TONE_NU * np.arange(16)[:, None] + phi[None, :]
    cos_t = (TONE_AMP * np.cos(ang)).astype(np.float32)
    sin_t = (TONE_AMP * np.sin(ang)).astype(np.float32)
    idx = (np.arange(n_time) + t0) % 16
    re = noise[:, :, 0]
    im = noise[:, :, 1]
    re *= np.float32(SIGMA)
    im *= np.float32(SIGMA)
    re += cos_t[idx]
    im += sin_t[idx]
    re = np.clip(np.rint(re), -7, 7).astype(np.int8)
    im = np.clip(np.rint(im), -7, 7).astype(np.int8)
    return (((re.astype(np.uint8) & 0xF) << 4) | (im.astype(np.uint8) & 0xF)).astype(np.uint8)


def channel_view(buf: np.ndarray, layout: int, n_inputs: int, n_chan: int, n_time: int,
                 channel: int) -> np.ndarray:
    """(n_time, n_inputs) view of one channel inside a packed buffer."""
    if layout == LAYOUT_TFI:
        return buf.reshape(n_time, n_chan, n_inputs)[:, channel, :]
    if layout == LAYOUT_FTI:
        return buf.reshape(n_chan, n_time, n_inputs)[channel]
    raise ValueError(f"unknown layout {layout}")


def make_input(seed: int, n_inputs: int, n_chan: int, n_time: int, layout: int = LAYOUT_TFI,
               array: int = 0, out: np.ndarray | None = None,
               threads: int | None = None) -> np.ndarray:
    """Whole packed buffer (n_inputs * n_chan * n_time bytes) for one array."""
    size = n_inputs * n_chan * n_time
    if out is None:
        out = np.empty(size, dtype=np.uint8)
    if out.size != size or out.dtype != np.uint8:
        raise ValueError("output buffer has the wrong size or dtype")
    phi = phases(seed, array, n_inputs)

    def one(f: int) -> None:
        channel_view(out, layout, n_inputs, n_chan, n_time, f)[...] = channel_samples(
            seed, array, f, n_inputs, n_time, phi)

    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    if threads <= 1 or n_chan == 1:
        for f in range(n_chan):
            one(f)
    else:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(one, range(n_chan)))
    return out


def lane_payloads(seed: int, n_pfb: int, n_coarse: int, n_time: int) -> list[np.ndarray]:
    """Packet payloads of the 8 * n_pfb PFB lanes (lane of PFB b, fibre n at
    index 8 b + n): n_coarse * 4 * n_time packets of 256 packed samples each,
    seeded noise of RMS 2.5 per part, clipped to [-7, 7]; one Philox stream per
    lane.  Only draws samples; their order inside a lane is the caller's."""
    out = []
    n = n_coarse * 4 * n_time * 256
    for lane in range(8 * n_pfb):
        rng = _rng(seed, 1000 + lane, 0)
        z = rng.standard_normal((n, 2), dtype=np.float32) * np.float32(SIGMA)
        re = np.clip(np.rint(z[:, 0]), -7, 7).astype(np.int8)
        im = np.clip(np.rint(z[:, 1]), -7, 7).astype(np.int8)
        out.append((((re.astype(np.uint8) & 0xF) << 4) | (im.astype(np.uint8) & 0xF)).astype(np.uint8))
    return out


def coarse_samples(seed: int, n_coarse: int, n_inputs: int, n_samples: int, rms: float = 16.0) -> np.ndarray:
    """Complex int8 coarse-channel voltages laid out [c][i][n][re, im]:
    seeded Gaussian noise of the given RMS per part, rounded and clipped to
    [-127, 127]; one Philox stream per (coarse channel, input)."""
    out = np.empty((n_coarse, n_inputs, n_samples, 2), dtype=np.int8)
    for c in range(n_coarse):
        for i in range(n_inputs):
            rng = _rng(seed, 2000 + c, i)
            z = rng.standard_normal((n_samples, 2), dtype=np.float32) * np.float32(rms)
            out[c, i] = np.clip(np.rint(z), -127, 127).astype(np.int8)
    return out.reshape(-1)


def tone_input(gains_re: np.ndarray, gains_im: np.ndarray, n_chan: int, n_time: int,
               layout: int = LAYOUT_TFI) -> np.ndarray:
    """Single injected tone x_i(t) = g_i * j**t, identical in every channel.

    Multiplying a Gaussian integer by j only swaps and negates its parts, so the
    samples stay inside [-7, 7] whenever the gains do.
    """
    g = np.asarray(gains_re, dtype=np.int64) + 1j * np.asarray(gains_im, dtype=np.int64)
    n_inputs = g.size
    rot = np.array([1, 1j, -1, -1j])[np.arange(n_time) % 4]
    x = rot[:, None] * g[None, :]
    ch = pack(np.rint(x.real).astype(np.int64), np.rint(x.imag).astype(np.int64))
    out = np.empty(n_inputs * n_chan * n_time, dtype=np.uint8)
    for f in range(n_chan):
        channel_view(out, layout, n_inputs, n_chan, n_time, f)[...] = ch
    return out
