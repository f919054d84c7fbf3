"""Streaming correlation service: 50 ms chunks in, one visibility set per
integration out, several observations sharing one GPU.

The paper's XMAC servers receive data continuously, assemble it into a
device-bound buffer while the previous one is being correlated, accumulate
products on the device and copy each integration back asynchronously
(Sec. 3.4.1, Sec. 3.4.3).  This service does the same for several concurrent
observations on one GPU:

  - every admitted observation owns a copy stream, a compute stream, two
    device staging slots for 50 ms chunks (500 samples at 10 kHz, Appendix A),
    a device-resident accumulator and an output buffer;
  - chunk k: pinned host -> device copy on the copy stream; the compute stream
    waits for it, then corr_xmac accumulates it (corr_zero opens each
    integration); after the last chunk of an integration (10 chunks = 0.5 s,
    Sec. 1.1) corr_dump writes the paper's output format and the copy stream
    brings it back to pinned host memory;
  - admission by device-memory budget, first fit in arrival order: an
    observation that does not fit waits and starts as soon as finishing ones
    free their memory (continuous batching); admitted observations run on
    their own streams, so their kernels overlap on the device;
  - latency of an integration = time its output is back on the host minus the
    submission time of its last chunk; p50/p99 over all complete
    integrations and per observation;
  - real-time factor = input bytes served per second of wall time divided by
    the real-time input rate of the whole mix (every observation streaming at
    once): 1.0 means the mix is kept up with exactly; per observation, its
    data time over the wall time it was active (admission to last output);
  - synchronised data only (Sec. 3.3.1): a chunk that has not arrived by its
    deadline (its release time in paced mode, else the time it was first
    asked for, plus ``late_s``) marks its integration incomplete.  The
    integration's remaining chunks are skipped, nothing of it is dumped, and
    the next integration starts from a zeroed accumulator, so partial data are
    never merged into a complete one; the result is recorded as incomplete.

The device work goes through a backend (``GpuBackend`` for the HIP library on
a GPU); the scheduling, admission and statistics are plain Python and can run
against any backend with the same methods, e.g. a fake one under test.
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import model

CHUNK_SAMPLES = 500           # 50 ms at 10 kHz
CHUNKS_PER_INTEGRATION = 10   # 0.5 s


@dataclass
class Observation:
    """One observation: shape, length, and where its chunks come from.

    ``chunk(k)`` returns chunk k (samples 500k .. 500k+499) as the backend's
    host buffer (pinned memory for the GPU backend), layout (t, f, i), or None
    while the chunk has not arrived yet.
    """

    obs_id: str
    n_inputs: int
    n_chan: int
    n_integrations: int
    chunk: object
    arrival_s: float = 0.0
    chunk_samples: int = CHUNK_SAMPLES
    chunks_per_integration: int = CHUNKS_PER_INTEGRATION

    @property
    def n_chunks(self) -> int:
        return self.n_integrations * self.chunks_per_integration

    @property
    def chunk_period_s(self) -> float:
        return self.chunk_samples / model.SAMPLE_RATE_HZ


@dataclass
class IntegrationResult:
    obs_id: str
    index: int
    t_last_chunk: float
    t_done: float
    output: object = None
    complete: bool = True

    @property
    def latency_s(self) -> float:
        return self.t_done - self.t_last_chunk


@dataclass
class _Active:
    obs: Observation
    rt: object
    t_start: float
    next_chunk: int = 0
    pending: list = field(default_factory=list)  # (integration index, t_last_chunk, token)
    done: int = 0
    t_asked: float | None = None  # when the service first asked for chunk next_chunk


def _percentiles(lat_s: list) -> dict:
    lat = np.array(lat_s) if lat_s else np.zeros(1)
    return {"latency_p50_ms": float(np.percentile(lat, 50) * 1e3),
            "latency_p99_ms": float(np.percentile(lat, 99) * 1e3),
            "latency_max_ms": float(lat.max() * 1e3)}


class Service:
    """Runs observations to completion; see the module docstring.

    ``late_s``: how long after its deadline a chunk is waited for before its
    integration is declared incomplete.  ``progress``: optional callable given
    one line of text after every ``progress_every`` results.
    """

    def __init__(self, backend, hbm_budget_bytes: int, clock=time.perf_counter, sleep=time.sleep,
                 late_s: float = 0.05, progress=None, progress_every: int = 50):
        self.backend = backend
        self.budget = int(hbm_budget_bytes)
        self.clock = clock
        self.sleep = sleep
        self.late_s = float(late_s)
        self.progress = progress
        self.progress_every = int(progress_every)
        # integrations whose outputs may be in flight at once (host output buffers per observation)
        self.max_pending = int(getattr(backend, "host_slots", 2))
        self.queue: list[Observation] = []
        self.active: list[_Active] = []
        self.results: list[IntegrationResult] = []
        self.admit_log: list[tuple[str, float]] = []
        self.in_use = 0
        self.peak_in_use = 0
        self.peak_pending = 0
        self._t_admit: dict[str, float] = {}
        self._t_end: dict[str, float] = {}

    def submit(self, obs: Observation) -> None:
        need = self.backend.mem_bytes(obs)
        if need > self.budget:
            raise ValueError(f"observation {obs.obs_id} needs {need} bytes, more than the whole budget")
        self.queue.append(obs)

    # -- scheduling ------------------------------------------------------------

    def _admit(self, now: float, t0: float) -> None:
        """First fit, in arrival order, among observations that have arrived."""
        for obs in list(self.queue):
            if t0 + obs.arrival_s > now:
                continue
            need = self.backend.mem_bytes(obs)
            if self.in_use + need <= self.budget:
                self.queue.remove(obs)
                rt = self.backend.open(obs)
                self.in_use += need
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                self.active.append(_Active(obs, rt, now))
                self.admit_log.append((obs.obs_id, now - t0))
                self._t_admit[obs.obs_id] = now

    def _drop(self, a: _Active, k: int, now: float) -> None:
        """Chunk k missed its deadline: its integration is incomplete."""
        obs = a.obs
        n_int = k // obs.chunks_per_integration
        self.results.append(IntegrationResult(obs.obs_id, n_int, now, now, None, complete=False))
        a.done += 1
        a.next_chunk = (n_int + 1) * obs.chunks_per_integration
        a.t_asked = None

    def _feed(self, a: _Active, now: float, paced: bool) -> bool:
        """Submit every chunk of `a` that is due; True if anything was submitted or dropped."""
        obs = a.obs
        fed = False
        while a.next_chunk < obs.n_chunks:
            k = a.next_chunk
            release = a.t_start + (k + 1) * obs.chunk_period_s
            if paced and now < release:
                break
            last = (k + 1) % obs.chunks_per_integration == 0
            # An integration's last chunk sends its output to a host buffer:
            # wait while every buffer still holds an uncollected output.
            if last and len(a.pending) >= self.max_pending:
                break
            data = obs.chunk(k)
            if data is None:
                if a.t_asked is None:
                    a.t_asked = now
                deadline = (release if paced else a.t_asked) + self.late_s
                if now < deadline:
                    break
                self._drop(a, k, now)
                fed = True
                continue
            token = self.backend.submit_chunk(a.rt, k, data, last)
            if last:
                a.pending.append((k // obs.chunks_per_integration, self.clock(), token))
                self.peak_pending = max(self.peak_pending, len(a.pending))
            a.next_chunk += 1
            a.t_asked = None
            fed = True
        return fed

    def _collect(self, a: _Active, keep_outputs: bool) -> bool:
        got = False
        while a.pending and self.backend.done(a.rt, a.pending[0][2]):
            idx, t_last, token = a.pending.pop(0)
            t_done = self.clock()
            out = self.backend.output(a.rt, token) if keep_outputs else None
            self.results.append(IntegrationResult(a.obs.obs_id, idx, t_last, t_done, out))
            a.done += 1
            got = True
            if self.progress and len(self.results) % self.progress_every == 0:
                self.progress(f"{len(self.results)} integrations done, last {a.obs.obs_id}[{idx}] "
                              f"{(t_done - t_last) * 1e3:.1f} ms")
        return got

    def run(self, paced: bool = True, keep_outputs: bool = False, poll_s: float = 1e-4) -> dict:
        """Serve every submitted observation; returns the statistics."""
        t0 = self.clock()
        data_s = sum(o.n_chunks * o.chunk_period_s for o in self.queue)
        in_bytes = sum(o.n_chunks * model.input_bytes(o.n_inputs, o.n_chan, o.chunk_samples) for o in self.queue)
        rt_rate = sum(model.input_bytes(o.n_inputs, o.n_chan, o.chunk_samples) / o.chunk_period_s
                      for o in self.queue)
        per_obs = {o.obs_id: o for o in self.queue}
        while self.queue or self.active:
            now = self.clock()
            self._admit(now, t0)
            busy = False
            for a in list(self.active):
                busy |= self._feed(a, now, paced)
                busy |= self._collect(a, keep_outputs)
                if a.done == a.obs.n_integrations:
                    self.backend.close(a.rt)
                    self.in_use -= self.backend.mem_bytes(a.obs)
                    self.active.remove(a)
                    self._t_end[a.obs.obs_id] = self.clock()
                    busy = True
            if not busy:
                self.sleep(poll_s)
        wall = self.clock() - t0
        complete = [r for r in self.results if r.complete]
        stats = {
            "integrations": len(complete),
            "incomplete": len(self.results) - len(complete),
            "wall_s": wall,
            "data_s_all_observations": data_s,
            "input_bytes": in_bytes,
            "input_gbps": in_bytes / wall / 1e9 if wall > 0 else float("inf"),
            "realtime_input_gbps": rt_rate / 1e9,
            "realtime_factor": in_bytes / wall / rt_rate if wall > 0 else float("inf"),
            **_percentiles([r.latency_s for r in complete]),
            "peak_hbm_bytes": self.peak_in_use,
            "peak_pending": self.peak_pending,
            "admissions": list(self.admit_log),
        }
        obs_stats = {}
        for oid, o in per_obs.items():
            rs = [r for r in complete if r.obs_id == oid]
            active = self._t_end.get(oid, t0) - self._t_admit.get(oid, t0)
            obs_data = o.n_chunks * o.chunk_period_s
            obs_stats[oid] = {"integrations": len(rs),
                              "incomplete": sum(1 for r in self.results if r.obs_id == oid and not r.complete),
                              "active_s": active, "data_s": obs_data,
                              "realtime_factor": obs_data / active if active > 0 else float("inf"),
                              **_percentiles([r.latency_s for r in rs])}
        stats["per_observation"] = obs_stats
        return stats


class GpuBackend:
    """The HIP library on cuda:0: one Correlator per observation with its own
    streams, staging slots and output buffers.  ``host_slots`` pinned host
    buffers per observation receive the dumps, so at most that many
    integrations may await collection at once."""

    host_slots = 2

    def __init__(self, engine: str = "mfma_i8", order=None, dtype=None, device: str = "cuda:0"):
        import torch

        from . import corrx

        self.torch, self.corrx = torch, corrx
        self.engine = engine
        self.order = corrx.CORRX_TRI_STATION_POL if order is None else order
        self.dtype = corrx.CORRX_F32 if dtype is None else dtype
        self.device = torch.device(device)

    def _dump_count(self, obs: Observation) -> int:
        n, f = obs.n_inputs, obs.n_chan
        if self.order == self.corrx.CORRX_TRI_STATION_POL:
            return f * model.n_station_pol(n) * 2
        return f * model.n_baselines(n) * 2

    def mem_bytes(self, obs: Observation) -> int:
        return (model.acc_bytes(obs.n_inputs, obs.n_chan) + 4 * self._dump_count(obs)
                + 2 * model.input_bytes(obs.n_inputs, obs.n_chan, obs.chunk_samples))

    def open(self, obs: Observation):
        torch, corrx = self.torch, self.corrx
        rt = type("Runtime", (), {})()
        rt.obs = obs
        rt.corr = corrx.Correlator(obs.n_inputs, obs.n_chan, obs.chunk_samples, corrx.CORRX_LAYOUT_TFI, self.engine)
        rt.copy = torch.cuda.Stream(device=self.device)  # chunks in (host -> device)
        rt.comp = torch.cuda.Stream(device=self.device)
        rt.d2h = torch.cuda.Stream(device=self.device)   # dumps out, so the next chunks need not wait for them
        nbytes = model.input_bytes(obs.n_inputs, obs.n_chan, obs.chunk_samples)
        rt.stage = [torch.empty(nbytes, dtype=torch.uint8, device=self.device) for _ in range(2)]
        rt.stage_free = [None, None]
        rt.acc = rt.corr.new_acc(self.device)
        tdt = torch.float32 if self.dtype == corrx.CORRX_F32 else torch.int32
        rt.dump = torch.empty(self._dump_count(obs), dtype=tdt, device=self.device)
        rt.host = [torch.empty(self._dump_count(obs), dtype=tdt, pin_memory=True) for _ in range(self.host_slots)]
        rt.dump_free = None
        rt.n_out = 0
        return rt

    def close(self, rt) -> None:
        rt.copy.synchronize()
        rt.comp.synchronize()
        rt.d2h.synchronize()
        rt.corr.close()
        rt.stage = rt.acc = rt.dump = rt.host = None

    def submit_chunk(self, rt, k: int, host_chunk, last: bool):
        torch = self.torch
        slot = k % 2
        with torch.cuda.stream(rt.copy):
            if rt.stage_free[slot] is not None:
                rt.copy.wait_event(rt.stage_free[slot])
            rt.stage[slot].copy_(host_chunk, non_blocking=True)
            copied = torch.cuda.Event()
            copied.record(rt.copy)
        rt.comp.wait_event(copied)
        if k % rt.obs.chunks_per_integration == 0:
            rt.corr.zero(rt.acc, rt.comp)
        rt.corr.xmac(rt.stage[slot], rt.acc, rt.comp)
        free = torch.cuda.Event()
        free.record(rt.comp)
        rt.stage_free[slot] = free
        if not last:
            return None
        if rt.dump_free is not None:
            rt.comp.wait_event(rt.dump_free)
        rt.corr.dump(rt.acc, self.order, self.dtype, rt.dump, rt.comp)
        dumped = torch.cuda.Event()
        dumped.record(rt.comp)
        out = rt.host[rt.n_out % self.host_slots]
        rt.n_out += 1
        with torch.cuda.stream(rt.d2h):
            rt.d2h.wait_event(dumped)
            out.copy_(rt.dump, non_blocking=True)
            done = torch.cuda.Event()
            done.record(rt.d2h)
        rt.dump_free = done
        return (done, out)

    def done(self, rt, token) -> bool:
        return token[0].query()

    def output(self, rt, token):
        return token[1].numpy().copy()


def checksum(arr: np.ndarray) -> tuple[int, int]:
    """Order-sensitive integer checksum of an output buffer (bit pattern)."""
    v = np.ascontiguousarray(arr).view(np.uint32).astype(np.uint64)
    w = (np.arange(v.size, dtype=np.uint64) % np.uint64(65521)) + np.uint64(1)
    return int(v.sum() % (1 << 61)), int((v * w).sum() % (1 << 61))
