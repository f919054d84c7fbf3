"""GPU parity of the PFB packet-order ingest, the product remap and the
channel-averaged dump against the CPU oracle (tolerance 0: integer data and
power-of-two float scaling)."""

import numpy as np
import pytest

from oracle import pfb as opfb
from paper_1501_05992_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cx():
    import torch

    from paper_1501_05992_amd import corrx

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    corrx.lib()
    return corrx


def _dev():
    import torch

    return torch.device("cuda:0")


def _lanes_dev(lanes):
    import torch

    return [torch.from_numpy(l).to(_dev()) for l in lanes]


@pytest.mark.parametrize("n_pfb,n_coarse,T", [(1, 1, 37), (4, 1, 16), (2, 2, 9), (3, 1, 5)])
@pytest.mark.parametrize("natural", [False, True])
def test_ingest_matches_oracle(cx, n_pfb, n_coarse, T, natural):
    import torch

    print(f"ingest n_pfb={n_pfb} n_coarse={n_coarse} T={T} natural={natural}", flush=True)
    lanes = synth.lane_payloads(100 + n_pfb, n_pfb, n_coarse, T)
    c = cx.Correlator(64 * n_pfb, 128 * n_coarse, T)
    order = cx.CORRX_ORDER_NATURAL if natural else cx.CORRX_ORDER_PACKET
    got = c.pfb_ingest(_lanes_dev(lanes), order)
    torch.cuda.synchronize()
    want = opfb.ingest(lanes, n_pfb, n_coarse, T, natural)
    assert np.array_equal(got.cpu().numpy(), want)
    c.close()


@pytest.mark.parametrize("N,F", [(64, 3), (256, 2)])
def test_remap_matches_oracle(cx, N, F):
    import torch

    rng = np.random.default_rng(N + F)
    nb = N * (N + 1) // 2
    src = rng.integers(-2**30, 2**30, size=(F, nb, 2), dtype=np.int64).astype(np.int32)
    c = cx.Correlator(N, F, 10)
    got = c.pfb_remap(torch.from_numpy(src).to(_dev()))
    torch.cuda.synchronize()
    want = opfb.remap(src.astype(np.int64), N)
    assert np.array_equal(got.cpu().numpy().astype(np.int64), want)
    c.close()


@pytest.mark.parametrize("engine", ["mfma_i8", "plain"])
def test_packet_order_chain_equals_natural_order(cx, oracle_lib, engine):
    # ingest in packet order -> xmac -> remap  ==  ingest in natural order -> xmac  ==  oracle
    import torch

    n_pfb, n_coarse, T = 4, 1, 300
    N, F = 64 * n_pfb, 128 * n_coarse
    lanes = synth.lane_payloads(7, n_pfb, n_coarse, T)
    ld = _lanes_dev(lanes)
    c = cx.Correlator(N, F, T, cx.CORRX_LAYOUT_TFI, engine)
    x_pkt = c.pfb_ingest(ld, cx.CORRX_ORDER_PACKET)
    x_nat = c.pfb_ingest(ld, cx.CORRX_ORDER_NATURAL)
    a_pkt, a_nat = c.new_acc(_dev()), c.new_acc(_dev())
    c.zero(a_pkt)
    c.xmac(x_pkt, a_pkt)
    c.zero(a_nat)
    c.xmac(x_nat, a_nat)
    a_map = c.pfb_remap(a_pkt)
    torch.cuda.synchronize()
    got_map, got_nat = a_map.cpu().numpy(), a_nat.cpu().numpy()
    assert np.array_equal(got_map, got_nat)
    nat = opfb.ingest(lanes, n_pfb, n_coarse, T, natural=True).reshape(T, F, N)
    for f in (0, 63, 127):
        want = oracle_lib.xmac(np.ascontiguousarray(nat[:, f, :]), N, 1, T)[0]
        assert np.array_equal(got_nat[f].astype(np.int64), want)
    c.close()


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("f_avg", [1, 2, 4])
def test_dump_avg_matches_oracle(cx, oracle_lib, order, f_avg):
    import torch

    N, F, T = 48, 8, 200
    a = synth.make_input(31, N, F, T)
    b = synth.make_input(32, N, F, T)
    c = cx.Correlator(N, F, T)
    acc = c.new_acc(_dev())
    c.zero(acc)
    c.xmac(torch.from_numpy(a).to(_dev()), acc)
    c.xmac(torch.from_numpy(b).to(_dev()), acc)  # two integrations: t_avg = 2
    vi = c.dump_avg(acc, f_avg, 2, order, cx.CORRX_I32)
    vf = c.dump_avg(acc, f_avg, 2, order, cx.CORRX_F32)
    torch.cuda.synchronize()
    vis = oracle_lib.xmac(a, N, F, T) + oracle_lib.xmac(b, N, F, T)
    if order == cx.CORRX_TRI_STATION_POL:
        vis = oracle_lib.station_pol(vis, N)
    want = opfb.channel_sum(vis, f_avg)
    assert np.array_equal(vi.cpu().numpy().astype(np.int64), want.reshape(-1))
    want_f = (want.astype(np.float64) / (2 * f_avg)).astype(np.float32)
    assert np.array_equal(vf.cpu().numpy(), want_f.reshape(-1))
    c.close()


def test_dump_avg_argument_errors(cx):
    import torch

    c = cx.Correlator(16, 12, 10)
    acc = c.new_acc(_dev())
    c.zero(acc)
    dst = torch.empty(c.dump(acc).numel(), dtype=torch.int32, device=_dev())
    for f_avg, t_avg in [(3, 1), (8, 1), (2, 3), (0, 1), (2, 0)]:  # not a power of two / not dividing 12
        with pytest.raises(cx.CorrxError) as e:
            cx.corr_dump_avg(c.h, acc, cx.CORRX_TRI_INPUT, cx.CORRX_I32, f_avg, t_avg, dst)
        assert e.value.status == cx.CORRX_EINVAL
    c.close()


def test_dump_avg_float_bound(cx):
    import torch

    # 98 * samples * f_avg must stay within 2^24 for float32 output
    T = 90000
    c = cx.Correlator(4, 2, T)
    acc = c.new_acc(_dev())
    c.zero(acc)
    c.xmac(torch.zeros(4 * 2 * T, dtype=torch.uint8, device=_dev()), acc)
    dst = torch.empty(c.dump(acc).numel(), dtype=torch.float32, device=_dev())
    cx.corr_dump_avg(c.h, acc, cx.CORRX_TRI_INPUT, cx.CORRX_F32, 1, 1, dst)
    with pytest.raises(cx.CorrxError) as e:
        cx.corr_dump_avg(c.h, acc, cx.CORRX_TRI_INPUT, cx.CORRX_F32, 2, 1, dst)
    assert e.value.status == cx.CORRX_EOVERFLOW
    torch.cuda.synchronize()
    c.close()


def test_pfb_shape_checks(cx):
    import torch

    lanes = [torch.zeros(4 * 10 * 256, dtype=torch.uint8, device=_dev()) for _ in range(8)]
    for n, f, layout in [(60, 128, 0), (64, 100, 0), (64, 128, 1), (320, 128, 0)]:
        c = cx.Correlator(n, f, 10, layout)
        with pytest.raises(cx.CorrxError) as e:
            c.pfb_ingest(lanes * 5, cx.CORRX_ORDER_PACKET,
                         inp=torch.empty(n * f * 10, dtype=torch.uint8, device=_dev()))
        assert e.value.status == cx.CORRX_EUNSUPPORTED
        c.close()
    c = cx.Correlator(60, 2, 10)
    acc = c.new_acc(_dev())
    with pytest.raises(cx.CorrxError) as e:
        c.pfb_remap(acc)
    assert e.value.status == cx.CORRX_EUNSUPPORTED
    c.close()


def test_ingest_single_time_step(cx):
    import torch

    lanes = synth.lane_payloads(9, 2, 1, 1)
    c = cx.Correlator(128, 128, 1)
    for natural in (False, True):
        got = c.pfb_ingest(_lanes_dev(lanes), cx.CORRX_ORDER_NATURAL if natural else cx.CORRX_ORDER_PACKET)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), opfb.ingest(lanes, 2, 1, 1, natural))
    c.close()


def test_remap_ragged_channel_count(cx):
    # 13 channels: the remap handles channels in groups of 8
    import torch

    N, F = 128, 13
    rng = np.random.default_rng(13)
    src = rng.integers(-1000, 1000, size=(F, N * (N + 1) // 2, 2), dtype=np.int64).astype(np.int32)
    c = cx.Correlator(N, F, 10)
    got = c.pfb_remap(torch.from_numpy(src).to(_dev()))
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().astype(np.int64), opfb.remap(src.astype(np.int64), N))
    c.close()


def test_dump_avg_rejects_odd_station_pol_and_overlap(cx):
    import torch

    c = cx.Correlator(15, 4, 10)
    acc = c.new_acc(_dev())
    c.zero(acc)
    dst = torch.empty(4 * 120 * 2, dtype=torch.float32, device=_dev())
    with pytest.raises(cx.CorrxError) as e:
        cx.corr_dump_avg(c.h, acc, cx.CORRX_TRI_STATION_POL, cx.CORRX_F32, 2, 1, dst)
    assert e.value.status == cx.CORRX_EINVAL
    with pytest.raises(cx.CorrxError) as e:  # destination overlapping the accumulator
        cx.corr_dump_avg(c.h, acc, cx.CORRX_TRI_INPUT, cx.CORRX_I32, 2, 1, acc)
    assert e.value.status == cx.CORRX_EINVAL
    c.close()
