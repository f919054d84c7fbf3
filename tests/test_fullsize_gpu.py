"""GPU parity at the benchmarked sizes, in the benchmark's launch
configuration, on sampled channels that the CPU oracle computes one by one
(tolerance 0: integer sums).

- full band: 256 inputs x 3072 channels x 10000 samples, TFI, for all three
  engines, every channel for the int8 engine, plus the station/polarisation
  float32 dump of the timed step;
- one coarse channel: 256 x 128 x 5000, MFMA and plain;
- the uneven batch: 64/256/512/2048 inputs in one persistent launch;
- the four streaming observations at full channel counts, served together
  under a tight memory budget and alone.
"""

import numpy as np
import pytest

from paper_1501_05992_amd import synth

pytestmark = pytest.mark.gpu

FULL = (256, 3072, 10000)
FULL_CHANNELS = [0, 1, 1000, 2047, 3071]
COARSE = (256, 128, 5000)
COARSE_CHANNELS = [0, 17, 64, 127]
UNEVEN = [(64, 3072, 10000, 0), (256, 768, 5000, 0), (512, 384, 4000, 0), (2048, 128, 2000, 0)]


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


class _Problem:
    """Host input (the benchmark's seed and recipe), its device copy and the
    oracle's visibilities of the sampled channels, computed once."""

    def __init__(self, oracle_lib, shape, seed, channels):
        import torch

        self.n, self.fc, self.tc = shape
        print(f"generating {self.n}x{self.fc}x{self.tc}", flush=True)
        self.host = synth.make_input(seed, self.n, self.fc, self.tc)
        self.x = torch.from_numpy(self.host).to(_dev())
        self.channels = channels
        self.want = {}
        for f in channels:
            ch = np.ascontiguousarray(synth.channel_view(self.host, 0, self.n, self.fc, self.tc, f))
            self.want[f] = oracle_lib.xmac(ch, self.n, 1, self.tc)[0]
        print(f"oracle done for channels {channels}", flush=True)


@pytest.fixture(scope="module")
def full_band(oracle_lib):
    return _Problem(oracle_lib, FULL, synth.config_seed(2), FULL_CHANNELS)


@pytest.fixture(scope="module")
def coarse(oracle_lib):
    return _Problem(oracle_lib, COARSE, synth.config_seed(1), COARSE_CHANNELS)


def _check_sampled(cx, prob, engine):
    import torch

    c = cx.Correlator(prob.n, prob.fc, prob.tc, cx.CORRX_LAYOUT_TFI, engine)
    acc = c.new_acc(_dev())
    c.zero(acc)
    c.xmac(prob.x, acc)
    idx = torch.tensor(prob.channels, device=_dev())
    got = acc.index_select(0, idx).cpu().numpy().astype(np.int64)
    for k, f in enumerate(prob.channels):
        assert np.array_equal(got[k], prob.want[f]), f"{engine}: channel {f} differs"
    return c, acc


@pytest.mark.parametrize("engine", ["mfma_i8", "mfma_f8", "plain"])
def test_full_band_sampled_channels(cx, full_band, engine):
    print(f"full band, engine {engine}", flush=True)
    c, acc = _check_sampled(cx, full_band, engine)
    del acc
    c.close()


def test_full_band_every_channel(cx, oracle_lib, full_band):
    """The int8 engine on the whole full band, every one of the 3072 channels
    against the oracle (about a minute of oracle time on the host's cores),
    compared in blocks of 768 channels."""
    c, acc = _check_sampled(cx, full_band, "mfma_i8")
    got = acc.cpu().numpy()
    del acc
    c.close()
    n, fc, tc = full_band.n, full_band.fc, full_band.tc
    tfi = full_band.host.reshape(tc, fc, n)
    for f0 in range(0, fc, 768):
        f1 = min(fc, f0 + 768)
        sub = np.ascontiguousarray(tfi[:, f0:f1, :]).reshape(-1)
        want = oracle_lib.xmac(sub, n, f1 - f0, tc)
        assert np.array_equal(got[f0:f1].astype(np.int64), want), f"channels {f0}..{f1 - 1} differ"
        print(f"channels {f0}..{f1 - 1} equal the oracle", flush=True)


def test_full_band_step_dump(cx, oracle_lib, full_band):
    # the timed step: zero + xmac + station/polarisation float32 dump
    import torch

    print("full band step with dump", flush=True)
    c, acc = _check_sampled(cx, full_band, "auto")
    order = cx.CORRX_TRI_STATION_POL
    dst = c.dump(acc, order, cx.CORRX_F32)
    per_chan = dst.numel() // full_band.fc
    for f in (0, 3071):
        got = dst[f * per_chan:(f + 1) * per_chan].cpu().numpy()
        want = oracle_lib.station_pol(full_band.want[f][None], full_band.n).reshape(-1)
        assert np.array_equal(got, want.astype(np.float32)), f"dump of channel {f} differs"
    torch.cuda.synchronize()
    del acc, dst
    c.close()


@pytest.mark.parametrize("engine", ["mfma_i8", "plain"])
def test_coarse_channel_sampled_channels(cx, coarse, engine):
    print(f"coarse channel, engine {engine}", flush=True)
    c, acc = _check_sampled(cx, coarse, engine)
    del acc
    c.close()


def test_coarse_channel_every_channel(cx, oracle_lib, coarse):
    """One coarse channel with the int8 engine, which splits each channel's
    samples over two workgroups to give every compute unit work: all 128
    channels against the oracle after one call (accumulator overwritten) and
    after a second (partial sums added on top)."""
    import torch

    n, fc, tc = coarse.n, coarse.fc, coarse.tc
    want = oracle_lib.xmac(coarse.host, n, fc, tc)
    c = cx.Correlator(n, fc, tc, cx.CORRX_LAYOUT_TFI, "mfma_i8")
    acc = c.new_acc(_dev())
    c.zero(acc)
    for calls in (1, 2):
        c.xmac(coarse.x, acc)
        torch.cuda.synchronize()
        got = acc.cpu().numpy().astype(np.int64)
        assert np.array_equal(got, calls * want), f"after {calls} call(s): {np.argwhere(got != calls * want)[:3]}"
        print(f"all {fc} channels equal the oracle after {calls} call(s)", flush=True)
    del acc
    c.close()


@pytest.fixture(scope="module")
def uneven(oracle_lib):
    import torch

    print("generating the uneven batch", flush=True)
    seed = synth.config_seed(3)
    hosts = [synth.make_input(seed, n, f, t, array=k) for k, (n, f, t, lay) in enumerate(UNEVEN)]
    wants = []
    for (n, f, t, lay), h in zip(UNEVEN, hosts):
        ch = np.ascontiguousarray(synth.channel_view(h, lay, n, f, t, f - 1))
        wants.append(oracle_lib.xmac(ch, n, 1, t)[0])
    print("oracle done for the last channel of each array", flush=True)
    return [torch.from_numpy(h).to(_dev()) for h in hosts], wants


@pytest.mark.parametrize("codes", [None, [0x101, 0x103, 0x103, 0x103]])
def test_uneven_batch_full_size(cx, uneven, codes):
    import torch

    print(f"uneven batch, tile codes {codes}", flush=True)
    ins, wants = uneven
    b = cx.Batch(UNEVEN, tile_cfg=codes)
    accs = b.new_accs(_dev())
    b.zero(accs)
    b.xmac(ins, accs)
    torch.cuda.synchronize()
    for (n, f, t, lay), want, acc in zip(UNEVEN, wants, accs):
        assert np.array_equal(acc[f - 1].cpu().numpy().astype(np.int64), want), f"array N={n} differs"
    del accs
    b.close()


STREAMS = [("obs256x3072", 256, 3072), ("obs256x768", 256, 768), ("obs512x384", 512, 384), ("obs128x3072", 128, 3072)]


def test_streaming_full_shapes_mixed_equals_alone(cx, oracle_lib):
    # the four streaming observations at their full channel counts, one
    # 0.5 s integration each, under a budget that holds about two at a time
    import torch

    from paper_1501_05992_amd.service import CHUNK_SAMPLES, CHUNKS_PER_INTEGRATION, GpuBackend, Observation, Service

    t_int = CHUNK_SAMPLES * CHUNKS_PER_INTEGRATION
    items = []
    for k, (name, n, f) in enumerate(STREAMS):
        print(f"generating {name}", flush=True)
        host = synth.make_input(synth.config_seed(4), n, f, t_int, array=k)
        pinned = torch.from_numpy(host).pin_memory()
        per = n * f * CHUNK_SAMPLES
        obs = Observation(name, n, f, 1, lambda c, d=pinned, p=per: d[c * p:(c + 1) * p], arrival_s=0.01 * k)
        items.append((host, obs))

    def serve(subset, budget):
        svc = Service(GpuBackend(), budget)
        for _, o in subset:
            svc.submit(o)
        st = svc.run(paced=False, keep_outputs=True)
        return st, {(r.obs_id, r.index): r.output for r in svc.results}

    need = sorted(GpuBackend().mem_bytes(o) for _, o in items)
    budget = need[-1] + need[-2]
    st, mixed = serve(items, budget)
    print(f"mixed: {st['integrations']} integrations, peak {st['peak_hbm_bytes']} of {budget} bytes", flush=True)
    assert st["integrations"] == len(STREAMS)
    assert st["peak_hbm_bytes"] <= budget
    for host, o in items:
        _, alone = serve([(host, o)], 10 ** 12)
        assert np.array_equal(mixed[(o.obs_id, 0)], alone[(o.obs_id, 0)]), o.obs_id
        out = mixed[(o.obs_id, 0)].reshape(o.n_chan, -1)
        for ch in (0, o.n_chan - 1):
            vis = oracle_lib.xmac(np.ascontiguousarray(synth.channel_view(host, 0, o.n_inputs, o.n_chan, t_int, ch)),
                                  o.n_inputs, 1, t_int)
            want = oracle_lib.station_pol(vis, o.n_inputs).astype(np.float32).reshape(-1)
            assert np.array_equal(out[ch], want), (o.obs_id, ch)
        print(f"{o.obs_id}: alone == mixed, channels 0 and {o.n_chan - 1} match the oracle", flush=True)
