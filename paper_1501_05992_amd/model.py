"""Counting model of the X-engine: baselines, operations, bytes, real-time factor.

Operation convention: 8 operations per complex multiply-accumulate (4 real
multiplies and 4 real additions), the convention behind the paper's
~8 TFLOPS requirement (Abstract; Sec. 1.1) and its 32 FLOPS per dual-polarisation
baseline and sample (Sec. 3.4.2).
"""

from __future__ import annotations

SAMPLE_RATE_HZ = 10_000  # 10 kHz critically sampled fine channels (Sec. 1.1, Sec. 3.2.1)
OPS_PER_CMAC = 8


def n_baselines(n_inputs: int) -> int:
    """Lower-triangle entries including autocorrelations, N(N+1)/2."""
    return n_inputs * (n_inputs + 1) // 2


def n_station_pol(n_inputs: int) -> int:
    """Visibilities per channel in station/polarisation order (Appendix C):
    S(S+1)/2 station pairs x 4 polarisation products, S = N/2 stations."""
    if n_inputs % 2:
        raise ValueError("station/polarisation order needs an even input count")
    s = n_inputs // 2
    return s * (s + 1) // 2 * 4


def alg_ops(n_inputs: int, n_chan: int, n_time: int) -> int:
    """Algorithmic operations of one pass: 8 per complex MAC over the triangle."""
    return OPS_PER_CMAC * n_baselines(n_inputs) * n_chan * n_time


def input_bytes(n_inputs: int, n_chan: int, n_time: int) -> int:
    """Packed 4+4-bit input: one byte per complex sample."""
    return n_inputs * n_chan * n_time


def acc_bytes(n_inputs: int, n_chan: int) -> int:
    """int32 complex lower-triangle accumulator."""
    return n_chan * n_baselines(n_inputs) * 2 * 4


def station_pol_bytes(n_inputs: int, n_chan: int, bytes_per_part: int = 4) -> int:
    """Paper output format: complex, 4 bytes per part, station/polarisation order."""
    return n_chan * n_station_pol(n_inputs) * 2 * bytes_per_part


def data_seconds(n_time: int) -> float:
    return n_time / SAMPLE_RATE_HZ


def realtime_factor(n_time: int, wall_s: float) -> float:
    """Seconds of data correlated per second of wall time."""
    return data_seconds(n_time) / wall_s


def arithmetic_intensity_paper(m: int, n: int, integ: int) -> float:
    """Sec. 3.4.2: flops per byte of an m x n dual-polarisation tile integrated
    over I samples at 32-bit precision, 32mnI / (16(m+n)I + 64mn)."""
    return 32.0 * m * n * integ / (16.0 * (m + n) * integ + 64.0 * m * n)


def arithmetic_intensity_packed(n_inputs: int, n_time: int) -> float:
    """Same ratio for one whole channel processed as a single tile here:
    algorithmic ops over packed input bytes plus int32 triangle output."""
    ops = alg_ops(n_inputs, 1, n_time)
    return ops / (input_bytes(n_inputs, 1, n_time) + acc_bytes(n_inputs, 1))
