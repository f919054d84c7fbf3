"""GPU parity of the fine polyphase filterbank (F-engine) against the CPU
oracle: tables equal, outputs equal byte for byte (integer arithmetic)."""

import numpy as np
import pytest

from oracle import fpfb as ofp
from paper_1501_05992_amd import synth

pytestmark = pytest.mark.gpu

S1, S2 = 13, 15


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


def test_tables_equal_the_oracle_definitions(cx):
    fb = cx.FineFilterbank(64, 1, 4)
    taps, wmat = fb.tables()
    assert np.array_equal(taps.astype(np.int64), ofp.taps())
    wr, wi = ofp.twiddles()
    p = np.arange(128)
    t = np.outer(p, p) % 128  # [q, p] (symmetric)
    want = np.zeros((256, 256), dtype=np.int64)
    want[:128, :128] = wr[t]
    want[:128, 128:] = -wi[t]
    want[128:, :128] = wi[t]
    want[128:, 128:] = wr[t]
    assert np.array_equal(wmat.astype(np.int64), want)
    fb.close()


# 64-input tiles (N = 64, 192) and 128-input tiles (N = 128, 256, 384), each
# with a ragged last tile of frames
@pytest.mark.parametrize("n_inputs,n_coarse,n_frames",
                         [(64, 1, 37), (128, 2, 5), (256, 1, 64), (64, 3, 1), (192, 1, 6), (384, 1, 3)])
def test_filterbank_matches_oracle(cx, n_inputs, n_coarse, n_frames):
    import torch

    print(f"fpfb N={n_inputs} C={n_coarse} T={n_frames}", flush=True)
    fb = cx.FineFilterbank(n_inputs, n_coarse, n_frames)
    x = synth.coarse_samples(40 + n_frames, n_coarse, n_inputs, fb.n_samples)
    got = fb.run(torch.from_numpy(x.view(np.uint8)).to(_dev()), S1, S2)
    torch.cuda.synchronize()
    want = ofp.channelise(x, n_inputs, n_coarse, n_frames, S1, S2)
    g = got.cpu().numpy()
    assert np.array_equal(g, want), f"{np.count_nonzero(g != want)} of {g.size} bytes differ"
    fb.close()


def test_filterbank_feeds_the_xengine(cx, oracle_lib):
    # F-engine -> X-engine on the GPU equals oracle F-engine -> oracle X-engine
    import torch

    N, C, T = 64, 1, 48
    fb = cx.FineFilterbank(N, C, T)
    x = synth.coarse_samples(77, C, N, fb.n_samples)
    fin = fb.run(torch.from_numpy(x.view(np.uint8)).to(_dev()), S1, S2)
    c = cx.Correlator(N, 128 * C, T)
    acc = c.new_acc(_dev())
    c.zero(acc)
    c.xmac(fin, acc)
    torch.cuda.synchronize()
    want_in = ofp.channelise(x, N, C, T, S1, S2)
    want = oracle_lib.xmac(want_in, N, 128 * C, T)
    assert np.array_equal(acc.cpu().numpy().astype(np.int64), want)
    c.close()
    fb.close()


def test_fpfb_argument_errors(cx):
    with pytest.raises(cx.CorrxError) as e:
        cx.FineFilterbank(96, 1, 4)
    assert e.value.status == cx.CORRX_EUNSUPPORTED
    import torch

    fb = cx.FineFilterbank(64, 1, 4)
    x = torch.zeros(2 * 64 * fb.n_samples, dtype=torch.uint8, device=_dev())
    for s1, s2 in [(-1, 3), (3, 31)]:
        with pytest.raises(cx.CorrxError) as e:
            fb.run(x, s1, s2)
        assert e.value.status == cx.CORRX_EINVAL
    fb.close()
