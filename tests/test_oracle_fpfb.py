"""Pins of the F-engine oracle (oracle/fpfb.py): the taps, the DFT table and
the filterbank against definitions and textbook identities.  The paper gives
no filter or quantiser, so these fix our own definitions, not the paper's."""

import numpy as np

from oracle import fpfb


def test_taps_shape_symmetry_and_flat_branches():
    h = fpfb.taps()
    assert h.size == 1536 and h.max() == 32767
    assert np.array_equal(h, h[::-1])  # linear phase
    # every polyphase branch passes DC with the same gain (within 0.2 %)
    branch = np.array([h[p::128].sum() for p in range(128)])
    assert branch.max() / branch.min() < 1.002


def test_twiddles_match_the_unit_circle():
    wr, wi = fpfb.twiddles()
    w = np.exp(-2j * np.pi * np.arange(128) / 128) * 127
    assert np.max(np.abs(wr - w.real)) <= 0.5 and np.max(np.abs(wi - w.imag)) <= 0.5
    assert (wr[0], wi[0]) == (127, 0) and (wr[32], wi[32]) == (0, -127) and (wr[64], wi[64]) == (-127, 0)


def test_dft_against_numpy_fft():
    rng = np.random.default_rng(1)
    v8 = rng.integers(-127, 128, size=(5, 128, 2))
    y = fpfb.dft(v8)
    ref = np.fft.fft(v8[..., 0] + 1j * v8[..., 1], axis=-1) * 127
    got = y[..., 0] + 1j * y[..., 1]
    # each twiddle is within 0.5 (per part) of 127 e^{...}: |error| <= sum |v8| * 0.5 * sqrt(2) * ...
    bound = np.abs(v8).sum(axis=(-1, -2))[:, None] * 0.5 * np.sqrt(2) * 1.0001
    assert np.all(np.abs(got - ref) <= bound)


def test_filterbank_equals_decimated_long_dft():
    # Textbook identity of the critically sampled PFB: the 128-point DFT of the
    # folded, windowed segment equals the 1536-point DFT of the windowed
    # segment at every 12th bin.
    rng = np.random.default_rng(2)
    T = 3
    x = rng.integers(-100, 101, size=(128 * (T + 11), 2))
    v = fpfb.fir(x, T)
    h = fpfb.taps()
    xc = x[:, 0] + 1j * x[:, 1]
    for k in range(T):
        seg = h * xc[128 * k: 128 * k + 1536]
        want = np.fft.fft(seg)[::12]
        got = np.fft.fft(v[k, :, 0] + 1j * v[k, :, 1])
        assert np.allclose(got, want, rtol=0, atol=1e-6 * np.abs(want).max())


def test_tone_lands_in_its_fine_channel():
    # A complex tone at fine-channel centre q0 (frequency q0 / 128 cycles per
    # sample) comes out in channel (q0 + 64) mod 128, the strongest by far.
    T = 4
    for q0 in (0, 5, 64, 100):
        n = np.arange(128 * (T + 11))
        x = np.stack([np.rint(60 * np.cos(2 * np.pi * q0 * n / 128)),
                      np.rint(60 * np.sin(2 * np.pi * q0 * n / 128))], axis=-1).astype(np.int8)
        out = fpfb.channelise(x.reshape(-1), 1, 1, T, 15, 17).reshape(T, 128, 1)
        re = (out[..., 0].astype(np.int16) >> 4).astype(np.int8)
        re = np.where(re > 7, re - 16, re)
        im = (out[..., 0] & 0xF).astype(np.int8)
        im = np.where(im > 7, im - 16, im)
        power = (re.astype(np.int64) ** 2 + im.astype(np.int64) ** 2).sum(axis=0)
        f0 = (q0 + 64) % 128
        assert power.argmax() == f0 and power[f0] > 0
        assert power[f0] > 20 * np.sort(power)[-2]


def test_round_shift_definition():
    v = np.array([-5, -4, -3, -1, 0, 1, 3, 4, 5])
    assert list(fpfb.round_shift(v, 1)) == [-2, -2, -1, 0, 0, 1, 2, 2, 3]  # floor((v + 1) / 2)
    assert list(fpfb.round_shift(v, 0)) == list(v)
