"""corr_xmac_noalloc through the C ABI: the same visibilities as corr_xmac on
a handle of the same shape (bit for bit: integer sums), on two calls in a row
with different shapes, the second smaller, so that the library's per-device
scratch is reused with stale contents; overwrite and accumulate modes; the
scratch limit."""

import numpy as np
import pytest

from paper_1501_05992_amd import synth

pytestmark = pytest.mark.gpu

# (inputs, channels, samples): both split every channel's samples over several
# workgroups, so the partial sums go through the scratch (3 images of
# 16.8 MB, then 3 of 1.3 MB)
SHAPES = [(256, 64, 8000), (200, 8, 3000)]


@pytest.fixture(scope="module")
def cx():
    import torch

    from paper_1501_05992_amd import corrx

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    corrx.lib()
    return corrx


def _with_handle(cx, x, n, fc, tc):
    import torch

    c = cx.Correlator(n, fc, tc, cx.CORRX_LAYOUT_TFI, "mfma_i8")
    acc = c.new_acc(x.device)
    c.zero(acc)
    c.xmac(x, acc)
    torch.cuda.synchronize()
    out = acc.cpu().numpy().copy()
    c.close()
    return out


def test_noalloc_equals_corr_xmac_on_two_calls(cx, oracle_lib):
    import torch

    dev = torch.device("cuda:0")
    for k, (n, fc, tc) in enumerate(SHAPES):
        print(f"corr_xmac_noalloc N={n} F={fc} T={tc}", flush=True)
        host = synth.make_input(7700 + k, n, fc, tc)
        x = torch.from_numpy(host).to(dev)
        want = _with_handle(cx, x, n, fc, tc)
        # stale values: overwrite mode must not read them
        acc = torch.full((fc, n * (n + 1) // 2, 2), 12345, dtype=torch.int32, device=dev)
        cx.corr_xmac_noalloc(x, acc, n, fc, tc, cx.CORRX_LAYOUT_TFI, accumulate=False)
        torch.cuda.synchronize()
        got = acc.cpu().numpy()
        assert np.array_equal(got, want), f"N={n}: {np.count_nonzero(got != want)} elements differ from corr_xmac"
        cx.corr_xmac_noalloc(x, acc, n, fc, tc, cx.CORRX_LAYOUT_TFI, accumulate=True)
        torch.cuda.synchronize()
        assert np.array_equal(acc.cpu().numpy().astype(np.int64), 2 * want.astype(np.int64)), \
            f"N={n}: accumulate mode differs"
        # and one channel against the oracle, independently of corr_xmac
        f = fc - 1
        ch = np.ascontiguousarray(synth.channel_view(host, 0, n, fc, tc, f))
        assert np.array_equal(want[f].astype(np.int64), oracle_lib.xmac(ch, n, 1, tc)[0])
        del x, acc


def test_noalloc_rejects_a_plan_beyond_its_scratch(cx):
    import torch

    # 4096 inputs, one channel, 2^20 + 1 samples: the plan splits time in two
    # (a work unit takes at most 2^20 samples) and needs one 67.1 MB partial
    # image, more than the 64 MiB scratch.  Rejected before anything runs.
    n, fc, tc = 4096, 1, (1 << 20) + 1
    dev = torch.device("cuda:0")
    x = torch.empty(n * fc * tc, dtype=torch.uint8, device=dev)
    acc = torch.empty(fc * n * (n + 1), dtype=torch.int32, device=dev)
    with pytest.raises(cx.CorrxError) as e:
        cx.corr_xmac_noalloc(x, acc, n, fc, tc)
    assert e.value.status == cx.CORRX_ESCRATCH
    del x, acc
