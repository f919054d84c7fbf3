"""Pins of the PFB packet-order and averaging oracle (oracle/pfb.py)."""

import numpy as np
import pytest

from oracle import pfb as opfb
from paper_1501_05992_amd import synth


def test_antenna_order_matches_printed_sequence():
    # Appendix A prints the order 0, 16, 32, 48, 1, 17, 33, 49, 2, 18, ..., 15, 31, 47, 63
    order = opfb.pfb_antenna_order()
    assert order[:10] == [0, 16, 32, 48, 1, 17, 33, 49, 2, 18]
    assert order[-4:] == [15, 31, 47, 63]
    assert sorted(order) == list(range(64))


def test_channel_groups_match_printed_sequence():
    # fibre 0: 0, 4, 8, 12, 128, 132, 136, 140, ..., 2944, 2948, 2952, 2956; fibre n adds 16 n
    g0 = opfb.fibre_channel_groups(0)
    assert g0[:8] == [0, 4, 8, 12, 128, 132, 136, 140]
    assert g0[-4:] == [2944, 2948, 2952, 2956]
    assert len(g0) == 96
    for n in range(8):
        assert opfb.fibre_channel_groups(n) == [f + 16 * n for f in g0]
    # the 8 fibres, 4 fine channels per group, cover all 3072 channels once
    chans = sorted(f + f2 for n in range(8) for f in opfb.fibre_channel_groups(n) for f2 in range(4))
    assert chans == list(range(3072))


def test_packet_counts():
    # 96 channel groups x 500 samples = 48,000 packets per 50 ms, 960,000 per second (Appendix A)
    groups, t50 = len(opfb.fibre_channel_groups(0)), 500
    assert groups * t50 == 48000
    assert groups * t50 * 20 == 960000
    # 384 fine channels per lane, 4 per packet group
    assert groups * 4 == 384


def _lanes(seed, n_pfb, n_coarse, n_time):
    return synth.lane_payloads(seed, n_pfb, n_coarse, n_time)


def test_ingest_layout_spot_checks():
    # Each lane byte lands at the (time, channel, input) the layout defines.
    n_pfb, n_coarse, T = 2, 1, 3
    lanes = _lanes(5, n_pfb, n_coarse, T)
    cube_p = opfb.ingest(lanes, n_pfb, n_coarse, T, natural=False).reshape(T, 128 * n_coarse, 64 * n_pfb)
    cube_n = opfb.ingest(lanes, n_pfb, n_coarse, T, natural=True).reshape(T, 128 * n_coarse, 64 * n_pfb)
    for (b, n, c, s, t, f2, k) in [(0, 0, 0, 0, 0, 0, 0), (1, 7, 0, 3, 2, 3, 63), (1, 3, 0, 1, 1, 2, 17)]:
        val = lanes[8 * b + n][(((c * 4 + s) * T + t) << 8) + 64 * f2 + k]
        f = 128 * c + 16 * n + 4 * s + f2
        assert cube_p[t, f, 64 * b + k] == val
        assert cube_n[t, f, 64 * b + 16 * (k % 4) + k // 4] == val
    # every lane byte is used exactly once: the buffers hold the same multiset
    allb = np.concatenate(lanes)
    assert np.array_equal(np.bincount(cube_p.reshape(-1), minlength=256), np.bincount(allb, minlength=256))


def test_remap_equals_correlating_in_natural_order(oracle_lib):
    # Correlating the natural-order buffer must equal remapping the products of
    # the packet-order buffer (Appendix C): two independent routes.
    n_pfb, n_coarse, T = 2, 1, 40
    lanes = _lanes(11, n_pfb, n_coarse, T)
    N, F = 64 * n_pfb, 128 * n_coarse
    pkt = opfb.ingest(lanes, n_pfb, n_coarse, T, natural=False)
    nat = opfb.ingest(lanes, n_pfb, n_coarse, T, natural=True)
    chans = [0, 5, 127]
    cube_p = pkt.reshape(T, F, N)
    cube_n = nat.reshape(T, F, N)
    vp = np.stack([oracle_lib.xmac(np.ascontiguousarray(cube_p[:, f, :]), N, 1, T)[0] for f in chans])
    vn = np.stack([oracle_lib.xmac(np.ascontiguousarray(cube_n[:, f, :]), N, 1, T)[0] for f in chans])
    assert np.array_equal(opfb.remap(vp, N), vn)
    # and a remap is not the identity here: some products are conjugated
    assert not np.array_equal(vp, vn)


def test_packet_index_inverts_the_pfb_map():
    for i in range(256):
        p = opfb.packet_index(i)
        assert p // 64 == i // 64
        assert 64 * (p // 64) + opfb.pfb_input_at_position(p % 64) == i


def test_channel_sum_definition():
    rng = np.random.default_rng(3)
    v = rng.integers(-1000, 1000, size=(8, 10, 2))
    s2 = opfb.channel_sum(v, 2)
    assert np.array_equal(s2, v[0::2] + v[1::2])
    s4 = opfb.channel_sum(v, 4)
    assert np.array_equal(s4, v[0::4] + v[1::4] + v[2::4] + v[3::4])
    assert np.array_equal(opfb.channel_sum(v, 1), v)


def test_time_and_frequency_averaging_compose(oracle_lib):
    # 2x2 averaging (Sec. 3.4.3): accumulating two integrations and summing two
    # channels equals summing the four (channel, integration) products.
    N, F, T = 16, 4, 30
    a = synth.make_input(21, N, F, T)
    b = synth.make_input(22, N, F, T)
    va = oracle_lib.xmac(a, N, F, T)
    vb = oracle_lib.xmac(b, N, F, T)
    both = np.concatenate([a.reshape(T, F, N), b.reshape(T, F, N)]).reshape(-1)
    vab = oracle_lib.xmac(both, N, F, 2 * T)
    assert np.array_equal(vab, va + vb)
    assert np.array_equal(opfb.channel_sum(vab, 2), opfb.channel_sum(va, 2) + opfb.channel_sum(vb, 2))
