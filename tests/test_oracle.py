"""Pins of the CPU oracle against things other than itself (no GPU).

Each check is chosen so that a plausible slip in the oracle (a dropped product,
a wrong sign of the imaginary part, swapped i/j, a wrong layout offset, a wrong
nibble) fails at least one of them:
  - the decode table against an independent bit-level decode and the encoder;
  - a hand-worked example that fixes the sign convention x_i * conj(x_j);
  - brute force with Python complex integers on tiny inputs, both layouts;
  - numpy complex128 X @ X^H (exact: every partial sum is an integer < 2**53);
  - the closed form of a single injected tone, V_ij = T g_i conj(g_j);
  - Hermitian symmetry, non-negative real autocorrelations, time linearity,
    permutation equivariance, and the zero contribution of invalid samples.
"""

import itertools

import numpy as np
import pytest

from paper_1501_05992_amd import synth


def _py_decode(b):
    # Independent decode: sign-extend each nibble through an int8 shift.
    hi = int(np.int8(np.uint8(b & 0xF0)) >> 4)
    lo = int(np.int8(np.uint8((b & 0x0F) << 4)) >> 4)
    if hi == -8 or lo == -8:
        return 0, 0, False
    return hi, lo, True


def test_decode_all_256_codes(oracle_lib):
    invalid = 0
    for b in range(256):
        re, im, ok = oracle_lib.decode(b)
        assert (re, im, ok) == _py_decode(b), b
        invalid += not ok
    # 16 codes with a high nibble of 8, 16 with a low nibble of 8, one shared.
    assert invalid == 31


def test_decode_inverts_encoder(oracle_lib):
    for re, im in itertools.product(range(-7, 8), repeat=2):
        b = int(synth.pack(np.array([re]), np.array([im]))[0])
        assert oracle_lib.decode(b) == (re, im, True)
    # the high nibble carries the real part
    assert oracle_lib.decode(0x10) == (1, 0, True)
    assert oracle_lib.decode(0x01) == (0, 1, True)
    assert oracle_lib.decode(0xF0) == (-1, 0, True)


def test_worked_example_sign_convention(oracle_lib):
    # x0 = 1, x1 = j, one sample.  V_10 = x1 * conj(x0) = j -> (0, +1);
    # autocorrelations |x|^2 = 1.
    buf = synth.pack(np.array([1, 0]), np.array([0, 1]))
    v = oracle_lib.xmac(buf, 2, 1, 1)
    assert v[0].tolist() == [[1, 0], [0, 1], [1, 0]]


def _brute(buf, n, f_count, t_count, layout):
    out = np.zeros((f_count, n * (n + 1) // 2, 2), dtype=np.int64)
    for f in range(f_count):
        ch = synth.channel_view(buf, layout, n, f_count, t_count, f)
        x = [[complex(*_py_decode(int(ch[t, i]))[:2]) for i in range(n)] for t in range(t_count)]
        for i in range(n):
            for j in range(i + 1):
                s = sum(x[t][i] * x[t][j].conjugate() for t in range(t_count))
                b = i * (i + 1) // 2 + j
                out[f, b] = (int(s.real), int(s.imag))
    return out


@pytest.mark.parametrize("layout", [synth.LAYOUT_TFI, synth.LAYOUT_FTI])
@pytest.mark.parametrize("n,f_count,t_count", [(1, 1, 1), (2, 3, 4), (5, 2, 3), (8, 3, 4), (7, 1, 2)])
def test_brute_force_tiny(oracle_lib, layout, n, f_count, t_count):
    rng = np.random.default_rng(1000 * n + 10 * f_count + t_count)
    # all 256 byte values may occur, invalid codes included
    buf = rng.integers(0, 256, size=n * f_count * t_count, dtype=np.uint8)
    got = oracle_lib.xmac(buf, n, f_count, t_count, layout)
    assert np.array_equal(got, _brute(buf, n, f_count, t_count, layout))


def test_layouts_agree(oracle_lib):
    n, fc, tc = 16, 3, 40
    ref = synth.make_input(synth.config_seed(0), n, fc, tc, synth.LAYOUT_TFI, threads=1)
    alt = np.empty_like(ref)
    for f in range(fc):
        synth.channel_view(alt, synth.LAYOUT_FTI, n, fc, tc, f)[...] = \
            synth.channel_view(ref, synth.LAYOUT_TFI, n, fc, tc, f)
    assert np.array_equal(oracle_lib.xmac(ref, n, fc, tc, 0), oracle_lib.xmac(alt, n, fc, tc, 1))


def _decoded_complex(ch):
    hi = (ch.astype(np.int16) >> 4) & 0xF
    lo = ch.astype(np.int16) & 0xF
    hi = np.where(hi >= 8, hi - 16, hi)
    lo = np.where(lo >= 8, lo - 16, lo)
    bad = (hi == -8) | (lo == -8)
    return np.where(bad, 0, hi) + 1j * np.where(bad, 0, lo)


def test_numpy_library_gemm_256_inputs(oracle_lib):
    n, fc, tc = 256, 2, 2000
    buf = synth.make_input(synth.config_seed(0), n, fc, tc, threads=2)
    got = oracle_lib.xmac(buf, n, fc, tc)
    ii, jj = np.tril_indices(n)
    b = ii * (ii + 1) // 2 + jj
    for f in range(fc):
        x = _decoded_complex(synth.channel_view(buf, 0, n, fc, tc, f)).T  # (N, T)
        v = x @ x.conj().T
        assert np.array_equal(got[f, b, 0], np.rint(v[ii, jj].real).astype(np.int64))
        assert np.array_equal(got[f, b, 1], np.rint(v[ii, jj].imag).astype(np.int64))


@pytest.mark.parametrize("t_count", [1, 3, 4, 17, 1000])
def test_single_tone_closed_form(oracle_lib, t_count):
    rng = np.random.default_rng(t_count)
    n = 24
    gr = rng.integers(-7, 8, size=n)
    gi = rng.integers(-7, 8, size=n)
    buf = synth.tone_input(gr, gi, 2, t_count)
    got = oracle_lib.xmac(buf, n, 2, t_count)
    g = gr + 1j * gi
    for i in range(n):
        for j in range(i + 1):
            want = t_count * g[i] * np.conj(g[j])
            b = i * (i + 1) // 2 + j
            for f in range(2):
                assert got[f, b, 0] == int(want.real) and got[f, b, 1] == int(want.imag)
    autos = [i * (i + 1) // 2 + i for i in range(n)]
    assert np.array_equal(got[0, autos, 0], t_count * (gr * gr + gi * gi))


def test_hermitian_and_autos(oracle_lib):
    n, fc, tc = 20, 2, 300
    buf = synth.make_input(synth.config_seed(0) + 7, n, fc, tc, threads=1)
    full = oracle_lib.xmac_full(buf, n, fc, tc)
    assert np.array_equal(full[..., 0], np.swapaxes(full[..., 0], 1, 2))
    assert np.array_equal(full[..., 1], -np.swapaxes(full[..., 1], 1, 2))
    d = np.arange(n)
    assert np.all(full[:, d, d, 1] == 0)
    assert np.all(full[:, d, d, 0] >= 0)
    tri = oracle_lib.xmac(buf, n, fc, tc)
    ii, jj = np.tril_indices(n)
    assert np.array_equal(tri, full[:, ii, jj, :])


def test_time_linearity(oracle_lib):
    n, fc, t1, t2 = 12, 3, 37, 51
    a = synth.make_input(5, n, fc, t1, threads=1)
    b = synth.make_input(6, n, fc, t2, threads=1)
    joined = np.concatenate([a, b])  # TFI: time is the slowest index
    va = oracle_lib.xmac(a, n, fc, t1)
    vb = oracle_lib.xmac(b, n, fc, t2)
    assert np.array_equal(oracle_lib.xmac(joined, n, fc, t1 + t2), va + vb)


def test_permutation_equivariance(oracle_lib):
    n, fc, tc = 10, 2, 64
    buf = synth.make_input(11, n, fc, tc, threads=1)
    perm = np.random.default_rng(3).permutation(n)
    pbuf = buf.reshape(tc, fc, n)[:, :, perm].reshape(-1)
    full = oracle_lib.tri_to_full(oracle_lib.xmac(buf, n, fc, tc), n)
    pfull = oracle_lib.tri_to_full(oracle_lib.xmac(pbuf, n, fc, tc), n)
    assert np.array_equal(pfull, full[:, perm][:, :, perm])


def test_invalid_samples_contribute_nothing(oracle_lib):
    n, fc, tc = 6, 1, 9
    buf = synth.make_input(12, n, fc, tc, threads=1)
    bad = buf.copy()
    zero = buf.copy()
    for t, i, code in [(0, 0, 0x80), (3, 2, 0x08), (8, 5, 0x88), (4, 1, 0x8F), (5, 3, 0x78)]:
        bad[t * n + i] = code
        zero[t * n + i] = 0x00
    assert np.array_equal(oracle_lib.xmac(bad, n, fc, tc), oracle_lib.xmac(zero, n, fc, tc))


def test_station_pol_order(oracle_lib):
    n, fc, tc = 8, 2, 30
    buf = synth.make_input(13, n, fc, tc, threads=1)
    full = oracle_lib.xmac_full(buf, n, fc, tc)
    sp = oracle_lib.station_pol(oracle_lib.xmac(buf, n, fc, tc), n)
    s = n // 2
    assert sp.shape == (fc, s * (s + 1) // 2, 2, 2, 2)
    for s1 in range(s):
        for s2 in range(s1 + 1):
            bs = s1 * (s1 + 1) // 2 + s2
            for p1, p2 in itertools.product(range(2), repeat=2):
                assert np.array_equal(sp[:, bs, p1, p2], full[:, 2 * s1 + p1, 2 * s2 + p2])


def test_incoherent_beam_matches_autos(oracle_lib):
    n, fc, tc = 16, 3, 50
    buf = synth.make_input(14, n, fc, tc, threads=1)
    beam = oracle_lib.incoherent_beam(buf, n, fc, tc)
    tri = oracle_lib.xmac(buf, n, fc, tc)
    autos = [i * (i + 1) // 2 + i for i in range(n)]
    assert np.array_equal(beam.sum(axis=1), tri[:, autos, 0].sum(axis=1))
