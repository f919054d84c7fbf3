"""Streaming service logic on the CPU: a fake backend (one simulated device
queue, outputs computed by the oracle) and a simulated clock."""

import numpy as np
import pytest

from paper_1501_05992_amd import model, synth
from paper_1501_05992_amd.service import Observation, Service


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeBackend:
    """Serial simulated device: each chunk costs `chunk_s`, an output copy
    `dump_s`; outputs are the oracle's visibilities of the integration."""

    def __init__(self, clock, oracle, chunk_s=0.002, dump_s=0.001):
        self.clock, self.oracle = clock, oracle
        self.chunk_s, self.dump_s = chunk_s, dump_s
        self.busy_until = 0.0
        self.open_count = 0

    def mem_bytes(self, obs):
        return (model.acc_bytes(obs.n_inputs, obs.n_chan)
                + 2 * model.input_bytes(obs.n_inputs, obs.n_chan, obs.chunk_samples))

    def open(self, obs):
        self.open_count += 1
        return {"obs": obs, "chunks": []}

    def close(self, rt):
        pass

    def submit_chunk(self, rt, k, host_chunk, last):
        start = max(self.clock(), self.busy_until)
        self.busy_until = start + self.chunk_s
        rt["chunks"].append(np.asarray(host_chunk))
        if not last:
            return None
        obs = rt["obs"]
        data = np.concatenate(rt["chunks"])
        rt["chunks"] = []
        vis = self.oracle.xmac(data, obs.n_inputs, obs.n_chan, data.size // (obs.n_inputs * obs.n_chan))
        self.busy_until += self.dump_s
        return (self.busy_until, vis)

    def done(self, rt, token):
        return self.clock() >= token[0]

    def output(self, rt, token):
        return token[1]


def _obs(name, n, f, n_int, seed, arrival=0.0):
    period = 100  # short chunks keep the oracle fast; the schedule is the same
    data = synth.make_input(seed, n, f, period * 10 * n_int, threads=1)
    per = n * f * period
    return Observation(name, n, f, n_int, lambda k, d=data, p=per: d[k * p:(k + 1) * p], arrival_s=arrival,
                       chunk_samples=period)


def test_paced_latency_and_admission(oracle_lib):
    clock = FakeClock()
    be = FakeBackend(clock, oracle_lib)
    obs = [_obs("a", 8, 2, 3, 1), _obs("b", 8, 4, 2, 2), _obs("c", 12, 2, 2, 3)]
    need = [be.mem_bytes(o) for o in obs]
    svc = Service(be, need[0] + need[1], clock=clock, sleep=clock.sleep)  # c must wait
    for o in obs:
        svc.submit(o)
    st = svc.run(paced=True, keep_outputs=True)
    assert st["integrations"] == 7
    order = [name for name, _ in st["admissions"]]
    assert order == ["a", "b", "c"]
    t_c = dict(st["admissions"])["c"]
    # c is admitted only after b (the shorter one) has finished its 2 integrations
    assert t_c >= 2 * 10 * obs[1].chunk_period_s
    assert st["peak_hbm_bytes"] <= need[0] + need[1]
    # every integration's latency covers at least its last chunk and the copy
    assert all(r.latency_s >= be.chunk_s + be.dump_s - 1e-9 for r in svc.results)
    assert st["latency_p99_ms"] >= st["latency_p50_ms"] > 0


def test_paced_release_times(oracle_lib):
    clock = FakeClock()
    be = FakeBackend(clock, oracle_lib)
    o = _obs("a", 8, 2, 2, 4)
    svc = Service(be, 10 ** 9, clock=clock, sleep=clock.sleep)
    svc.submit(o)
    st = svc.run(paced=True)
    # data arrives in real time: the wall time covers the whole observation
    assert st["wall_s"] >= o.n_chunks * o.chunk_period_s
    assert st["realtime_factor"] <= 1.0 + 1e-6
    for r in svc.results:
        assert r.t_last_chunk >= (r.index + 1) * 10 * o.chunk_period_s - 1e-9


def test_alone_equals_mixed(oracle_lib):
    def serve(obs_list, budget):
        clock = FakeClock()
        be = FakeBackend(clock, oracle_lib)
        svc = Service(be, budget, clock=clock, sleep=clock.sleep)
        for o in obs_list:
            svc.submit(o)
        svc.run(paced=False, keep_outputs=True)
        return {(r.obs_id, r.index): r.output for r in svc.results}

    mk = lambda: [_obs("a", 8, 2, 2, 5), _obs("b", 16, 2, 2, 6, arrival=0.01), _obs("c", 8, 3, 1, 7)]
    mixed = serve(mk(), 10 ** 9)
    for o in mk():
        alone = serve([o], 10 ** 9)
        for key, v in alone.items():
            assert np.array_equal(mixed[key], v)


def test_oversized_observation_rejected(oracle_lib):
    clock = FakeClock()
    be = FakeBackend(clock, oracle_lib)
    svc = Service(be, 1000, clock=clock, sleep=clock.sleep)
    with pytest.raises(ValueError):
        svc.submit(_obs("big", 16, 4, 1, 8))


def test_flat_out_is_faster_than_real_time(oracle_lib):
    clock = FakeClock()
    be = FakeBackend(clock, oracle_lib, chunk_s=0.001, dump_s=0.0005)
    svc = Service(be, 10 ** 9, clock=clock, sleep=clock.sleep)
    svc.submit(_obs("a", 8, 2, 3, 9))
    st = svc.run(paced=False)
    assert st["realtime_factor"] > 5
    assert st["input_gbps"] == pytest.approx(st["realtime_factor"] * st["realtime_input_gbps"])
