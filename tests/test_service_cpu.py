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
        if k % rt["obs"].chunks_per_integration == 0:
            rt["chunks"] = []  # corr_zero opens every integration
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


class SlotBackend(FakeBackend):
    """Like FakeBackend, but every output lands in one of ``host_slots`` shared
    host buffers when its copy completes, as the GPU backend's pinned buffers
    do; ``output`` reads the buffer.  A later output landing in a buffer whose
    output has not been collected yet would overwrite it."""

    host_slots = 2

    def open(self, obs):
        rt = super().open(obs)
        rt.update(slots=[None] * self.host_slots, inflight=[], n_out=0)
        return rt

    def submit_chunk(self, rt, k, host_chunk, last):
        tok = super().submit_chunk(rt, k, host_chunk, last)
        if tok is None:
            return None
        slot = rt["n_out"] % self.host_slots
        rt["n_out"] += 1
        tok = (tok[0], slot, tok[1])
        rt["inflight"].append(tok)
        return tok

    def _land(self, rt):
        for tok in list(rt["inflight"]):
            if self.clock() >= tok[0]:
                rt["slots"][tok[1]] = tok[2]
                rt["inflight"].remove(tok)

    def done(self, rt, token):
        self._land(rt)
        return self.clock() >= token[0]

    def output(self, rt, token):
        self._land(rt)
        return rt["slots"][token[1]].copy()


def _expected(oracle_lib, obs_data, n, f, period, n_int):
    per = n * f * period * 10
    return [oracle_lib.xmac(obs_data[k * per:(k + 1) * per], n, f, period * 10) for k in range(n_int)]


def test_outputs_wait_for_free_host_buffers(oracle_lib):
    """Slow output copies (the device lags the host): the service never has
    more integrations awaiting collection than host buffers, and every
    collected output is its own integration's."""
    clock = FakeClock()
    be = SlotBackend(clock, oracle_lib, chunk_s=0.0005, dump_s=0.05)
    period, n, f, n_int = 100, 8, 2, 6
    data = synth.make_input(11, n, f, period * 10 * n_int, threads=1)
    per = n * f * period
    obs = Observation("a", n, f, n_int, lambda k: data[k * per:(k + 1) * per], chunk_samples=period)
    svc = Service(be, 10 ** 9, clock=clock, sleep=clock.sleep)
    svc.submit(obs)
    st = svc.run(paced=False, keep_outputs=True)
    assert st["integrations"] == n_int and st["incomplete"] == 0
    assert 1 <= st["peak_pending"] <= be.host_slots
    want = _expected(oracle_lib, data, n, f, period, n_int)
    got = {r.index: r.output for r in svc.results}
    for k in range(n_int):
        assert np.array_equal(got[k], want[k]), k


def _late_obs(data, n, f, period, n_int, clock, arrival):
    """Chunk k arrives at clock time arrival(k) (inf: never)."""
    per = n * f * period

    def chunk(k):
        return data[k * per:(k + 1) * per] if clock() >= arrival(k) else None

    return Observation("late", n, f, n_int, chunk, chunk_samples=period)


@pytest.mark.parametrize("paced", [True, False])
def test_missing_chunk_drops_its_integration(oracle_lib, paced):
    """A chunk that never arrives: its integration is recorded incomplete with
    no output, nothing of it leaks into the next integration, and the others
    are correct (Sec. 3.3.1: only synchronised data are correlated)."""
    clock = FakeClock()
    be = SlotBackend(clock, oracle_lib)
    period, n, f, n_int = 100, 8, 2, 4
    data = synth.make_input(12, n, f, period * 10 * n_int, threads=1)
    missing = 13  # integration 1, chunk 3
    obs = _late_obs(data, n, f, period, n_int, clock, lambda k: float("inf") if k == missing else 0.0)
    svc = Service(be, 10 ** 9, clock=clock, sleep=clock.sleep, late_s=0.02)
    svc.submit(obs)
    st = svc.run(paced=paced, keep_outputs=True)
    assert st["integrations"] == 3 and st["incomplete"] == 1
    assert st["per_observation"]["late"]["incomplete"] == 1
    want = _expected(oracle_lib, data, n, f, period, n_int)
    by = {r.index: r for r in svc.results}
    assert not by[1].complete and by[1].output is None
    for k in (0, 2, 3):
        assert by[k].complete and np.array_equal(by[k].output, want[k]), k
    # the incomplete integration was declared no earlier than the chunk's deadline
    if paced:
        release = (missing + 1) * obs.chunk_period_s
        assert by[1].t_done >= release + 0.02 - 1e-9


def test_late_chunk_within_deadline_is_used_after_it_is_dropped(oracle_lib):
    """Paced: a chunk arriving 10 ms after its release is waited for (late_s =
    30 ms); one arriving 100 ms late is not, and its integration is dropped
    even though the data turn up afterwards."""
    clock = FakeClock()
    be = SlotBackend(clock, oracle_lib)
    period, n, f, n_int = 100, 8, 2, 3
    data = synth.make_input(13, n, f, period * 10 * n_int, threads=1)
    p = period / model.SAMPLE_RATE_HZ
    late = {4: 0.010, 25: 0.100}  # chunk -> delay after its release time
    obs = _late_obs(data, n, f, period, n_int, clock, lambda k: (k + 1) * p + late.get(k, 0.0))
    svc = Service(be, 10 ** 9, clock=clock, sleep=clock.sleep, late_s=0.030)
    svc.submit(obs)
    st = svc.run(paced=True, keep_outputs=True)
    by = {r.index: r for r in svc.results}
    want = _expected(oracle_lib, data, n, f, period, n_int)
    assert by[0].complete and np.array_equal(by[0].output, want[0])
    assert by[1].complete and np.array_equal(by[1].output, want[1])
    assert not by[2].complete
    assert st["integrations"] == 2 and st["incomplete"] == 1


def test_per_observation_statistics(oracle_lib):
    clock = FakeClock()
    be = FakeBackend(clock, oracle_lib)
    obs = [_obs("a", 8, 2, 3, 21), _obs("b", 8, 4, 2, 22, arrival=0.01)]
    svc = Service(be, 10 ** 9, clock=clock, sleep=clock.sleep)
    for o in obs:
        svc.submit(o)
    st = svc.run(paced=True)
    per = st["per_observation"]
    assert set(per) == {"a", "b"}
    assert per["a"]["integrations"] == 3 and per["b"]["integrations"] == 2
    for o in obs:
        s = per[o.obs_id]
        assert s["data_s"] == pytest.approx(o.n_chunks * o.chunk_period_s)
        # paced: an observation cannot be served faster than its data arrive
        assert 0.5 < s["realtime_factor"] <= 1.0 + 1e-6
        assert s["latency_p99_ms"] >= s["latency_p50_ms"] > 0
