"""Streaming service on the GPU: observations of different shapes served
together with a tight memory budget; every integration equals the same
observation served alone, bit for bit, and matches the oracle."""

import numpy as np
import pytest

from paper_1501_05992_amd import synth

pytestmark = pytest.mark.gpu


def _pinned_obs(name, n, f, n_int, seed, arrival=0.0):
    import torch

    from paper_1501_05992_amd.service import CHUNK_SAMPLES, Observation

    host = synth.make_input(seed, n, f, CHUNK_SAMPLES * 10 * n_int)
    pinned = torch.from_numpy(host).pin_memory()
    per = n * f * CHUNK_SAMPLES
    return host, Observation(name, n, f, n_int, lambda k, d=pinned, p=per: d[k * p:(k + 1) * p], arrival_s=arrival)


SHAPES = [("a", 256, 24, 3), ("b", 64, 40, 2), ("c", 512, 6, 2), ("d", 128, 16, 3)]


def _serve(items, budget, paced=False):
    from paper_1501_05992_amd.service import GpuBackend, Service

    be = GpuBackend()
    svc = Service(be, budget)
    for _, o in items:
        svc.submit(o)
    st = svc.run(paced=paced, keep_outputs=True)
    return st, {(r.obs_id, r.index): r.output for r in svc.results}, be


def test_mixed_equals_alone_and_oracle(oracle_lib):
    import torch

    from paper_1501_05992_amd.service import GpuBackend

    assert torch.cuda.is_available()
    items = [_pinned_obs(nm, n, f, k, 100 + j, arrival=0.01 * j) for j, (nm, n, f, k) in enumerate(SHAPES)]
    be = GpuBackend()
    need = [be.mem_bytes(o) for _, o in items]
    budget = sum(sorted(need)[-2:])  # at most about two at a time
    st, mixed, _ = _serve(items, budget)
    assert st["integrations"] == sum(s[3] for s in SHAPES)
    assert st["peak_hbm_bytes"] <= budget
    assert len(st["admissions"]) == len(SHAPES)
    for j, (host, o) in enumerate(items):
        _, alone, _ = _serve([(host, o)], 10 ** 12)
        for key, v in alone.items():
            assert np.array_equal(mixed[key], v), key
    # one integration of each observation against the oracle (station/pol, float32)
    for host, o in items:
        per = o.n_inputs * o.n_chan * 500 * 10
        vis = oracle_lib.xmac(host[:per], o.n_inputs, o.n_chan, 5000)
        want = oracle_lib.station_pol(vis, o.n_inputs).astype(np.float32).reshape(-1)
        assert np.array_equal(mixed[(o.obs_id, 0)], want)


def test_paced_latency_is_reported():
    items = [_pinned_obs("p", 128, 16, 2, 200)]
    st, _, _ = _serve(items, 10 ** 12, paced=True)
    assert st["integrations"] == 2
    assert 0 < st["latency_p50_ms"] < 500
    assert st["realtime_factor"] <= 1.05
