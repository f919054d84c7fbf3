"""CPU oracle of the fine polyphase filterbank (F-engine) -- TEST
INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this module.  It shares no code, table or constant generator
with the GPU library: the taps and the DFT matrix are generated here from
their definitions.

Sec. 3.2.1 of Ord et al. describes the second (fine) stage as a 12-tap,
128-point, critically sampled polyphase filterbank: a filter-weighted DFT that
splits each 1.28 MHz coarse channel into 128 channels of 10 kHz, whose output
is requantised to the 4+4-bit samples the X-engine takes (Appendix A).  The
paper gives neither the filter nor the quantiser; the definitions below are
this implementation's (parity unpinned against the paper beyond the shape):

  taps   h[m], m = 0 .. 1535:  rint(32767 * w[m] * sinc((m - 767.5) / 128) / max),
         w the Hann window over 1536 points, max the largest |w * sinc|;
  frame  k (0 .. T-1) of input i: samples x[128 (k + j) + p], j = 0..11, p = 0..127;
  FIR    v[p] = sum_j h[128 j + p] * x[128 (k + j) + p]          (int64, complex)
  v8     = clip(floor((v + 2^(s1-1)) / 2^s1), -127, 127)          (real, imaginary)
  DFT    Y[q] = sum_p v8[p] * W[p q mod 128],  W[n] = rint(127 e^(-2 pi i n / 128))
  out    = clip(floor((Y + 2^(s2-1)) / 2^s2), -7, 7)
  channel f = (q + 64) mod 128 (lowest frequency first), written as the
  packed byte (re << 4 | im & 15) at (time k, channel 128 c + f, input i).

Input layout: complex int8 pairs [c][i][n][re, im], n = 0 .. 128 (T + 11) - 1.
"""

from __future__ import annotations

import numpy as np

M = 128
TAPS = 12
L = M * TAPS


def taps() -> np.ndarray:
    """int16 prototype filter of 1536 taps (see the module docstring)."""
    m = np.arange(L, dtype=np.float64)
    w = 0.5 - 0.5 * np.cos(2.0 * np.pi * (m + 0.5) / L)
    proto = w * np.sinc((m - (L - 1) / 2.0) / M)
    return np.rint(32767.0 * proto / np.abs(proto).max()).astype(np.int64)


def twiddles() -> tuple[np.ndarray, np.ndarray]:
    """Real and imaginary parts of W[n] = rint(127 e^{-2 pi i n / 128}), n = 0..127."""
    n = np.arange(M, dtype=np.float64)
    return (np.rint(127.0 * np.cos(2.0 * np.pi * n / M)).astype(np.int64),
            np.rint(-127.0 * np.sin(2.0 * np.pi * n / M)).astype(np.int64))


def round_shift(v: np.ndarray, s: int) -> np.ndarray:
    """floor((v + 2^(s-1)) / 2^s) for s >= 1, v itself for s == 0 (int64)."""
    v = np.asarray(v, dtype=np.int64)
    if s == 0:
        return v
    return (v + (1 << (s - 1))) >> s


def fir(x: np.ndarray, n_frames: int) -> np.ndarray:
    """Filter one input's complex samples x (shape (128 (T+11), 2), int) into
    frames v[k][p] (complex as the last axis), int64, by the definition."""
    h = taps()
    x = np.asarray(x, dtype=np.int64)
    v = np.zeros((n_frames, M, 2), dtype=np.int64)
    for k in range(n_frames):
        for j in range(TAPS):
            seg = x[M * (k + j): M * (k + j + 1)]
            v[k] += h[M * j: M * (j + 1), None] * seg
    return v


def dft(v8: np.ndarray) -> np.ndarray:
    """Y[k][q] = sum_p v8[k][p] W[p q mod 128] (complex as the last axis), int64."""
    wr, wi = twiddles()
    p = np.arange(M)
    idx = np.outer(p, p) % M  # [p, q]
    Wr, Wi = wr[idx], wi[idx]
    vr, vi = v8[..., 0].astype(np.int64), v8[..., 1].astype(np.int64)
    yr = vr @ Wr - vi @ Wi
    yi = vr @ Wi + vi @ Wr
    return np.stack([yr, yi], axis=-1)


def channelise(xin: np.ndarray, n_inputs: int, n_coarse: int, n_frames: int, s1: int, s2: int) -> np.ndarray:
    """The whole F-engine: complex int8 input [c][i][n][2] -> packed TFI bytes
    (n_frames, 128 n_coarse, n_inputs)."""
    ns = M * (n_frames + TAPS - 1)
    x = np.asarray(xin, dtype=np.int8).reshape(n_coarse, n_inputs, ns, 2)
    out = np.zeros((n_frames, M * n_coarse, n_inputs), dtype=np.uint8)
    for c in range(n_coarse):
        for i in range(n_inputs):
            v8 = np.clip(round_shift(fir(x[c, i], n_frames), s1), -127, 127)
            y = np.clip(round_shift(dft(v8), s2), -7, 7)
            q = np.arange(M)
            f = (q + M // 2) % M
            packed = ((y[..., 0] & 0xF) << 4) | (y[..., 1] & 0xF)  # [k, q]
            out[:, M * c + f, i] = packed.astype(np.uint8)
    return out.reshape(-1)
