"""Counting model pinned to the paper's printed figures; generator properties."""

import os

import numpy as np
import pytest

from paper_1501_05992_amd import model, synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_figures.txt")


def _figures():
    out = {}
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val = line.split()[:2]
            out[key] = float(val)
    return out


def test_visibility_count_per_channel():
    fig = _figures()
    n = int(fig["inputs"])
    assert n == 2 * int(fig["dual_pol_tiles"])
    assert model.n_station_pol(n) == int(fig["visibilities_per_channel"]) == 33024
    assert model.n_baselines(n) == 32896


def test_output_volume_and_rate():
    fig = _figures()
    n, f = int(fig["inputs"]), int(fig["fine_channels"])
    assert f * fig["channel_width_hz"] == fig["bandwidth_hz"]
    vol = model.station_pol_bytes(n, f)  # complex fp32
    assert vol == 811_597_824
    assert abs(vol / fig["bytes_per_time_unit_approx"] - 1) < 0.02
    assert vol * 8 / 1e9 > fig["gbit_per_s_at_1s_min"]


def test_operation_rate_requirement():
    fig = _figures()
    n, f = int(fig["inputs"]), int(fig["fine_channels"])
    # one second of data at 10 kHz per channel
    ops = model.alg_ops(n, f, model.SAMPLE_RATE_HZ)
    assert abs(ops / 1e12 / fig["tflops_required_approx"] - 1) < 0.02
    # per dual-polarisation baseline and sample: 4 complex MACs = 32 ops
    assert 4 * model.OPS_PER_CMAC == fig["naive_flops"]


def test_arithmetic_intensity_formula():
    fig = _figures()
    ai = model.arithmetic_intensity_paper(1, 1, 1)
    assert ai == pytest.approx(fig["naive_flops"] / (fig["naive_bytes_in"] + fig["naive_bytes_out"]))
    assert round(ai, 2) == fig["naive_ai"]
    # grows with tile size and integration length
    assert model.arithmetic_intensity_paper(8, 8, 100) > model.arithmetic_intensity_paper(2, 2, 100)


def test_chunk_arithmetic():
    fig = _figures()
    assert fig["samples_per_50ms"] == 0.05 * model.SAMPLE_RATE_HZ
    assert fig["packets_per_50ms"] == 96 * fig["samples_per_50ms"]
    assert model.realtime_factor(10_000, 0.01) == pytest.approx(100.0)


def test_generator_range_and_determinism():
    n, fc, tc = 32, 4, 256
    a = synth.make_input(synth.config_seed(1), n, fc, tc, threads=1)
    b = synth.make_input(synth.config_seed(1), n, fc, tc, threads=4)
    assert np.array_equal(a, b)
    hi = (a >> 4).astype(np.int16)
    lo = (a & 0xF).astype(np.int16)
    assert not np.any(hi == 8) and not np.any(lo == 8)  # invalid code never emitted
    # one channel regenerated alone equals its slice of the whole buffer
    for f in (0, 3):
        ch = synth.channel_samples(synth.config_seed(1), 0, f, n, tc)
        assert np.array_equal(synth.channel_view(a, synth.LAYOUT_TFI, n, fc, tc, f), ch)
    c = synth.make_input(synth.config_seed(2), n, fc, tc, threads=1)
    assert not np.array_equal(a, c)


def test_generator_statistics():
    n, tc = 64, 4096
    ch = synth.channel_samples(synth.config_seed(0), 0, 0, n, tc).astype(np.int16)
    hi = np.where((ch >> 4) >= 8, (ch >> 4) - 16, ch >> 4)
    lo = np.where((ch & 0xF) >= 8, (ch & 0xF) - 16, ch & 0xF)
    # noise sigma 2.5 plus a tone of amplitude 2 (power 2 per part), clipped at 7
    rms = np.sqrt((hi.astype(float) ** 2).mean())
    assert 2.6 < rms < 3.3
    assert hi.min() >= -7 and hi.max() <= 7 and lo.min() >= -7 and lo.max() <= 7
    # the tone is common to all inputs up to a phase: its power at nu = 1/16
    x = hi + 1j * lo
    spec = np.abs(np.fft.fft(x, axis=0)) ** 2
    assert np.argmax(spec.mean(axis=1)) == tc // 16
