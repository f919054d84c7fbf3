"""Benchmark of the X-engine on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the full MWA band, 256 inputs (128 dual-polarisation tiles) x 3072
fine channels x 10000 samples (1 s of data at 10 kHz), seeded synthetic
4+4-bit samples, TFI layout, resident in HBM before timing.  One step is the
whole hot path: corr_zero -> corr_xmac (decode + cross-multiply + integrate)
-> corr_dump to the paper's output format (station/polarisation order, complex
float32, Appendix C).  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_INT8_TOPS = 5000.0   # MI355X dense int8 MFMA, published
PEAK_FP8_TFLOPS = 5000.0  # MI355X dense fp8 MFMA, published
PEAK_HBM_GBS = 8000.0

# HBM traffic of the dominant kernel (int8 engine, full band) from two
# rocprofv3 --pmc passes over this script with --copy-probe: FETCH_SIZE and
# WRITE_SIZE per dispatch, each scaled by what the same counter reads for the
# 1 GiB device copy.  It describes the kernel built from the sources hashed
# here and is reported as null once any of them has changed.
KERNEL_SOURCES = ("paper_1501_05992_amd/csrc/xengine_mfma.hip",
                  "paper_1501_05992_amd/csrc/corrx_internal.h",
                  "paper_1501_05992_amd/csrc/api.hip")
TRAFFIC = {
    "sources_sha256": "8a119165a1bb5fa6861bbff44e152699d60968bee6c8624a7b86a197387a6371",
    "read_bytes": 7864783155,   # FETCH_SIZE 3,840,226 KiB x 2.000
    "write_bytes": 844381530,   # WRITE_SIZE 824,591 KiB x 1.000
    "summary": "profiles/xmac_diag_i8_full_band_256x3072x10000_counters.txt",
}


def kernel_sources_sha256() -> str:
    import hashlib

    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_field(n, fc, tc, engine, xmac_ms):
    if TRAFFIC is None or engine not in ("mfma_i8", "auto") or (n, fc, tc) != (256, 3072, 10000):
        return None
    if TRAFFIC["sources_sha256"] != kernel_sources_sha256():
        return None
    total = TRAFFIC["read_bytes"] + TRAFFIC["write_bytes"]
    return {"read_bytes": TRAFFIC["read_bytes"], "write_bytes": TRAFFIC["write_bytes"],
            "bytes": total, "gbs": round(total / (xmac_ms * 1e-3) / 1e9, 1), "summary": TRAFFIC["summary"]}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10, help="untimed steps; the shader clock settles after about five")
    ap.add_argument("--engine", default="mfma_i8")
    ap.add_argument("--n-inputs", type=int, default=256)
    ap.add_argument("--n-chan", type=int, default=3072)
    ap.add_argument("--n-time", type=int, default=10000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the plain-engine and small-config lines")
    ap.add_argument("--cpu-channels", type=int, default=768, help="channels in the oracle's timed sample")
    ap.add_argument("--check-channels", type=int, default=2, help="channels checked against the oracle")
    ap.add_argument("--only", choices=("uneven_batch", "coarse_channel", "ceilings", "streaming"),
                    help="run only this extra workload (for profiling) and print its JSON")
    ap.add_argument("--no-tune", action="store_true",
                    help="uneven batch: built-in tile codes instead of the autotuner's (for profiling)")
    ap.add_argument("--stream-integrations", type=int, default=100,
                    help="paced integrations per observation in the streaming run")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after timing, run one 1 GiB device-to-device copy (calibrates traffic counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this benchmark measures one GPU only (asked for {args.gpus}); the X-engine shards by "
              "channel with no exchange, so N GPUs would each run this same per-GPU workload.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1501_05992_amd import corrx, model, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.only:
        import oracle

        fn = {"uneven_batch": lambda: uneven_batch(corrx, model, synth, torch, dev, oracle, not args.no_tune),
              "coarse_channel": lambda: coarse_channel(corrx, model, synth, torch, dev),
              "ceilings": lambda: ceilings(torch, dev),
              "streaming": lambda: streaming(synth, torch, args.stream_integrations)}[args.only]
        print(json.dumps({args.only: fn()}), flush=True)
        if args.copy_probe:
            copy_probe(torch, dev)
        return
    n, fc, tc = args.n_inputs, args.n_chan, args.n_time
    seed = synth.config_seed(2)
    t_start = time.time()
    log(f"generating {n}x{fc}x{tc} input")
    host = synth.make_input(seed, n, fc, tc)
    t_gen = time.time() - t_start
    x = torch.from_numpy(host).to(dev)
    torch.cuda.synchronize()

    corr = corrx.Correlator(n, fc, tc, corrx.CORRX_LAYOUT_TFI, args.engine)
    acc = corr.new_acc(dev)
    order = corrx.CORRX_TRI_STATION_POL
    dst = torch.empty(corrx.corr_dump_count(corr.h, order), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]

    def step(k=None):
        corr.zero(acc)
        if k is not None:
            ev[k][0].record(stream)
        corr.xmac(x, acc)
        if k is not None:
            ev[k][1].record(stream)
        corr.dump(acc, order, corrx.CORRX_F32, dst)

    log(f"input ready ({t_gen:.1f} s); warmup {args.warmup}, timed {args.steps}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall / args.steps * 1e3
    xmac_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))

    ops = model.alg_ops(n, fc, tc)
    tops = ops / (ms_step * 1e-3) / 1e12
    xmac_tops = ops / (xmac_ms * 1e-3) / 1e12

    # correctness of the timed configuration on sampled channels
    import oracle

    check = []
    rng = np.random.default_rng(0)
    chans = sorted(set([0, fc - 1] + list(rng.integers(0, fc, size=max(0, args.check_channels - 2)))))
    acc_h = acc.cpu().numpy()
    for f in chans[: max(1, args.check_channels)]:
        ch = np.ascontiguousarray(synth.channel_view(host, 0, n, fc, tc, f))
        want = oracle.xmac(ch, n, 1, tc)[0]
        check.append(bool(np.array_equal(acc_h[f].astype(np.int64), want)))

    result = {
        "metric": "X-engine TOPS + x real-time at 256 inputs (MFMA vs plain); p99 integration latency",
        "value": round(tops, 2),
        "unit": "TOPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8" if args.engine in ("mfma_i8", "auto") else ("fp8" if args.engine == "mfma_f8" else "int32"),
        "data": "synthetic",
        "config": {"workload": f"full band: {n} inputs x {fc} channels x {tc} samples (1 s at 10 kHz), "
                               "4+4-bit noise+tone, TFI layout; step = zero + xmac + dump(station-pol f32)",
                   "engine": args.engine, "n_inputs": n, "n_chan": fc, "n_time": tc},
        "xrt": round(model.realtime_factor(tc, ms_step * 1e-3), 1),
        "xmac_ms": round(xmac_ms, 4),
        "xmac_tops": round(xmac_tops, 2),
        "xmac_xrt": round(model.realtime_factor(tc, xmac_ms * 1e-3), 1),
        "parity_sampled_channels": {"channels": [int(c) for c in chans], "bit_exact": all(check)},
        "input_gen_s": round(t_gen, 1),
    }
    peak = PEAK_FP8_TFLOPS if args.engine == "mfma_f8" else PEAK_INT8_TOPS
    result["roofline"] = {
        "bound": "mfma",
        "achieved": round(xmac_tops, 2),
        "peak": peak,
        "unit": "TFLOP/s",
        "op_kind": "algorithmic int8 ops (8 per complex MAC)" if args.engine != "mfma_f8" else
                   "algorithmic fp8 ops (8 per complex MAC)",
        "frac": round(xmac_tops / peak, 4),
        "traffic": None,
        "kernel": "xmac_diag_i8<256,4,true,64>" if args.engine in ("mfma_i8", "auto") else args.engine,
    }

    tf = traffic_field(n, fc, tc, args.engine, xmac_ms)
    if tf is not None:
        result["roofline"]["traffic"] = tf["bytes"]
        result["roofline"]["traffic_detail"] = tf
    log(f"timed: {ms_step:.3f} ms/step, xmac {xmac_ms:.3f} ms; parity {check}")
    if args.copy_probe:
        copy_probe(torch, dev)
    if not args.no_extras:
        result["extras"] = extras(corrx, model, synth, torch, dev, x, host, n, fc, tc, args.stream_integrations)

    del acc, dst
    corr.close()

    if not args.no_cpu_baseline:
        log("timing the oracle on a channel sample")
        result["cpu_baseline"] = cpu_baseline(oracle, model, synth, host, n, fc, tc, args.cpu_channels)

    print(json.dumps(result), flush=True)


def copy_probe(torch, dev):
    """One 1 GiB device-to-device copy: calibrates the HBM traffic counters."""
    a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def time_xmac(corrx, torch, c, x, acc, reps):
    s = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    c.zero(acc)
    c.xmac(x, acc)
    torch.cuda.synchronize()
    for a, b in evs:
        c.zero(acc)
        a.record(s)
        c.xmac(x, acc)
        b.record(s)
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in evs]))


def extras(corrx, model, synth, torch, dev, x, host, n, fc, tc, stream_integrations=100):
    import oracle

    out = {}
    ops = model.alg_ops(n, fc, tc)
    # the full band on the other two engines
    for eng, reps in (("mfma_f8", 10), ("plain", 3)):
        c = corrx.Correlator(n, fc, tc, corrx.CORRX_LAYOUT_TFI, eng)
        acc = c.new_acc(dev)
        ms = time_xmac(corrx, torch, c, x, acc, reps)
        ok = bool(np.array_equal(acc[0].cpu().numpy().astype(np.int64),
                                 oracle.xmac(np.ascontiguousarray(synth.channel_view(host, 0, n, fc, tc, 0)),
                                             n, 1, tc)[0]))
        out[f"full_band_{eng}"] = {"xmac_ms": round(ms, 3), "tops": round(ops / ms / 1e9, 2),
                                   "frac_of_peak": round(ops / ms / 1e9 / PEAK_INT8_TOPS, 4),
                                   "xrt": round(model.realtime_factor(tc, ms * 1e-3), 1),
                                   "channel0_bit_exact": ok}
        c.close()
        del acc
        log(f"full band {eng}: {ms:.3f} ms")
    out["ceilings"] = ceilings(torch, dev)
    out.update(coarse_channel(corrx, model, synth, torch, dev))
    out["uneven_batch"] = uneven_batch(corrx, model, synth, torch, dev, oracle)
    out["pfb_and_output"] = pfb_and_output(corrx, torch, dev, x, n, fc, tc)
    out["fine_pfb"] = fine_pfb(corrx, torch, dev, n, fc // 128)
    out["incoherent_beam"] = incoherent_beam(corrx, synth, torch, dev, oracle, x, host, n, fc, tc)
    out["streaming"] = streaming(synth, torch, stream_integrations)
    return out


def coarse_channel(corrx, model, synth, torch, dev):
    """One coarse channel, the paper's per-GPU unit: 256 inputs x 128 channels
    x 5000 samples, int8 MFMA against the plain vector-ALU engine."""
    out = {}
    n2, f2, t2 = 256, 128, 5000
    h2 = synth.make_input(synth.config_seed(1), n2, f2, t2)
    x2 = torch.from_numpy(h2).to(dev)
    for eng in ("mfma_i8", "plain"):
        c = corrx.Correlator(n2, f2, t2, corrx.CORRX_LAYOUT_TFI, eng)
        acc = c.new_acc(dev)
        ms = time_xmac(corrx, torch, c, x2, acc, 20)
        ops2 = model.alg_ops(n2, f2, t2)
        out[f"coarse_channel_{eng}"] = {"xmac_ms": round(ms, 4), "tops": round(ops2 / ms / 1e9, 2),
                                        "frac_of_peak": round(ops2 / ms / 1e9 / PEAK_INT8_TOPS, 4),
                                        "xrt": round(model.realtime_factor(t2, ms * 1e-3), 1)}
        log(f"coarse channel {eng}: {ms:.4f} ms")
        c.close()
    del x2
    return out


def ceilings(torch, dev, reps=5):
    """Measured issue-rate ceilings of the two engines' instructions, every
    compute unit busy, operands in registers (libceiling.so):
    v_dot4_i32_i8 (plain engine) and v_mfma_i32_32x32x32_i8 (int8 engine),
    with the shader clock each workgroup saw (shader-clock cycles over
    100 MHz constant-clock ticks)."""
    import ctypes

    from paper_1501_05992_amd import build as hip_build

    if not os.path.exists(hip_build.CEILING_LIB):
        raise RuntimeError("libceiling.so is not built: run python -m paper_1501_05992_amd.build")
    lib = ctypes.CDLL(hip_build.CEILING_LIB)
    lib.ceiling_launch.argtypes = [ctypes.c_int] * 4 + [ctypes.c_void_p] * 3
    lib.ceiling_dot4_ops.argtypes = lib.ceiling_mfma_ops.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.ceiling_dot4_ops.restype = lib.ceiling_mfma_ops.restype = ctypes.c_double
    n_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    s = torch.cuda.current_stream()
    out = {}
    for kind, name, seed, blocks, iters, ops_fn, peak in (
            (0, "v_dot4_i32_i8", 1, 8 * n_cu, 20000, lib.ceiling_dot4_ops, None),
            (1, "v_mfma_i32_32x32x32_i8 quiet operands", 0, 4 * n_cu, 10000, lib.ceiling_mfma_ops, PEAK_INT8_TOPS),
            (1, "v_mfma_i32_32x32x32_i8 random operands", 1, 4 * n_cu, 10000, lib.ceiling_mfma_ops, PEAK_INT8_TOPS)):
        res = torch.empty(blocks * 256, dtype=torch.int32, device=dev)
        clk = torch.zeros(blocks * 2, dtype=torch.int64, device=dev)

        def launch():
            if lib.ceiling_launch(kind, blocks, iters, seed, ctypes.c_void_p(res.data_ptr()),
                                  ctypes.c_void_p(clk.data_ptr()), ctypes.c_void_p(s.cuda_stream)) != 0:
                raise RuntimeError(f"ceiling probe {name}: launch failed")

        ms = time_ms(torch, launch, reps)
        c = clk.view(blocks, 2).cpu().numpy().astype(np.float64)
        ghz = float(np.median(c[:, 0] / np.maximum(c[:, 1], 1) * 0.1))
        tops = ops_fn(blocks, iters) / (ms * 1e-3) / 1e12
        out[name] = {"ms": round(ms, 4), "tops": round(tops, 2), "workgroups": blocks, "iters": iters,
                     "shader_ghz": round(ghz, 3)}
        if peak:
            out[name]["frac_of_peak"] = round(tops / peak, 4)
        log(f"ceiling {name}: {tops:.1f} TOPS at {ghz:.2f} GHz")
        del res, clk
    return out


def incoherent_beam(corrx, synth, torch, dev, oracle, x, host, n, fc, tc):
    """Incoherent beam over the full band (HBM-bound: the 7.86 GB input read
    once, one int32 per channel and sample written); channel 0 checked."""
    c = corrx.Correlator(n, fc, tc)
    beam = torch.empty((fc, tc), dtype=torch.int32, device=dev)
    ms = time_ms(torch, lambda: c.beam(x, beam), 5)
    ok = bool(np.array_equal(beam[0].cpu().numpy().astype(np.int64),
                             oracle.incoherent_beam(np.ascontiguousarray(synth.channel_view(host, 0, n, fc, tc, 0)),
                                                    n, 1, tc)[0]))
    nbytes = x.numel() + beam.numel() * 4
    res = {"ms": round(ms, 3), "bytes": nbytes, "gbs": round(nbytes / ms / 1e6, 1),
           "hbm_frac": round(nbytes / ms / 1e6 / PEAK_HBM_GBS, 3), "channel0_bit_exact": ok}
    log(f"incoherent beam: {ms:.3f} ms ({res['gbs']} GB/s)")
    del beam
    c.close()
    return res


def time_ms(torch, fn, reps):
    s = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record(s)
        fn()
        b.record(s)
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in evs]))


def fine_pfb(corrx, torch, dev, n, n_coarse, n_frames=2000, s1=13, s2=15):
    """F-engine at the full band's shape: n inputs x n_coarse coarse channels,
    2000 output frames (0.2 s of data), complex int8 input of RMS 16 drawn on
    the device."""
    fb = corrx.FineFilterbank(n, n_coarse, n_frames)
    g = torch.Generator(device=dev)
    g.manual_seed(1501)
    x = torch.randn(n_coarse * n * fb.n_samples * 2, device=dev, generator=g).mul_(16).round_().clamp_(-127, 127)
    x = x.to(torch.int8).view(torch.uint8)
    out = torch.empty(n_frames * 128 * n_coarse * n, dtype=torch.uint8, device=dev)
    ms = time_ms(torch, lambda: fb.run(x, s1, s2, out), 5)
    data_s = n_frames / 1e4
    in_b, ws_b, out_b = x.numel(), corrx.corr_fpfb_workspace_bytes(fb.h), out.numel()
    dft_ops = 2.0 * 256 * 256 * n_frames * n * n_coarse
    res = {"shape": [n, n_coarse, n_frames], "ms": round(ms, 3), "xrt": round(data_s / (ms * 1e-3), 1),
           "bytes": in_b + 2 * ws_b + out_b, "gbs": round((in_b + 2 * ws_b + out_b) / ms / 1e6, 1),
           "dft_mfma_tops": round(dft_ops / ms / 1e9, 1)}
    log(f"fine PFB: {ms:.3f} ms for {data_s} s of data ({res['xrt']}x real time)")
    del x, out
    fb.close()
    return res


def pfb_and_output(corrx, torch, dev, x, n, fc, tc):
    """Steps on either side of the X-engine at the full band, all HBM-bound:
    PFB packet-order ingest (the 7.86 GB input buffer reused as the 32 lane
    payloads: 32 x 24 coarse x 4 groups x 10000 samples x 256 bytes), the
    product remap to natural order, and the 2x2-averaged paper-format dump."""
    res = {}
    c = corrx.Correlator(n, fc, tc)
    lane_bytes = (fc // 128) * 4 * tc * 256
    lanes = [x[k * lane_bytes:(k + 1) * lane_bytes] for k in range(8 * (n // 64))]
    out = torch.empty_like(x)
    for name, order in (("ingest_natural", corrx.CORRX_ORDER_NATURAL), ("ingest_packet", corrx.CORRX_ORDER_PACKET)):
        ms = time_ms(torch, lambda: corrx.corr_pfb_ingest(c.h, lanes, order, out), 10)
        nbytes = 2 * x.numel()
        res[name] = {"ms": round(ms, 3), "gbs": round(nbytes / ms / 1e6, 1),
                     "hbm_frac": round(nbytes / ms / 1e6 / PEAK_HBM_GBS, 3), "bytes": nbytes}
        log(f"{name}: {ms:.3f} ms, {nbytes / ms / 1e6:.0f} GB/s")
    del out
    acc = c.new_acc(dev)
    c.zero(acc)
    c.xmac(x, acc)
    acc2 = torch.empty_like(acc)
    ms = time_ms(torch, lambda: corrx.corr_pfb_remap(c.h, acc, acc2), 10)
    nbytes = 2 * acc.numel() * 4
    res["remap"] = {"ms": round(ms, 3), "gbs": round(nbytes / ms / 1e6, 1),
                    "hbm_frac": round(nbytes / ms / 1e6 / PEAK_HBM_GBS, 3), "bytes": nbytes}
    log(f"remap: {ms:.3f} ms, {nbytes / ms / 1e6:.0f} GB/s")
    del acc2
    for f_avg in (1, 2):
        cnt = corrx.corr_dump_count(c.h, corrx.CORRX_TRI_STATION_POL) // f_avg
        dst = torch.empty(cnt, dtype=torch.float32, device=dev)
        ms = time_ms(torch, lambda: corrx.corr_dump_avg(c.h, acc, corrx.CORRX_TRI_STATION_POL, corrx.CORRX_F32,
                                                          f_avg, 2 if f_avg == 2 else 1, dst), 10)
        nbytes = acc.numel() * 4 + cnt * 4
        res[f"dump_station_pol_f32_favg{f_avg}"] = {"ms": round(ms, 3), "gbs": round(nbytes / ms / 1e6, 1),
                                                    "hbm_frac": round(nbytes / ms / 1e6 / PEAK_HBM_GBS, 3),
                                                    "bytes": nbytes}
        log(f"dump f_avg {f_avg}: {ms:.3f} ms, {nbytes / ms / 1e6:.0f} GB/s")
        del dst
    del acc
    c.close()
    return res


STREAM = [("obs256x3072", 256, 3072), ("obs256x768", 256, 768), ("obs512x384", 512, 384), ("obs128x3072", 128, 3072)]


def _rounded(d):
    if isinstance(d, dict):
        return {k: _rounded(v) for k, v in d.items() if k != "admissions"}
    return round(d, 3) if isinstance(d, float) else d


def streaming(synth, torch, paced_integrations=100, queued_integrations=8, flat_integrations=6):
    """Four observations fed in 50 ms chunks (500 samples), 0.5 s integrations,
    accumulators on the device.
    Paced: chunks released in real time, all four observations served together
    for paced_integrations integrations each; latency (last chunk released ->
    visibilities in host memory) per integration, p50/p99 per observation.
    Queued: the same, paced, under a device-memory budget that holds only three,
    so the fourth waits for admission.
    Flat out: chunks as fast as the device takes them."""
    from paper_1501_05992_amd.service import CHUNK_SAMPLES, GpuBackend, Observation, Service

    pools = {}
    for k, (name, n, f) in enumerate(STREAM):
        host = synth.make_input(synth.config_seed(4), n, f, 2 * CHUNK_SAMPLES, array=k)
        pools[name] = (torch.from_numpy(host).pin_memory(), n * f * CHUNK_SAMPLES)

    def make(n_int, arrivals):
        obs = []
        for (name, n, f), arr in zip(STREAM, arrivals):
            pin, per = pools[name]
            obs.append(Observation(name, n, f, n_int, lambda k, d=pin, p=per: d[(k % 2) * p:(k % 2 + 1) * p],
                                   arrival_s=arr))
        return obs

    be = GpuBackend()
    need = {o.obs_id: be.mem_bytes(o) for o in make(1, [0, 0, 0, 0])}
    everything = sum(need.values())
    out = {"observations": [list(x) for x in STREAM], "chunk_samples": CHUNK_SAMPLES,
           "integration_samples": 10 * CHUNK_SAMPLES,
           "input_gb_per_data_s": round(sum(model_bytes(n, f) for _, n, f in STREAM) / 1e9, 2)}
    log(f"streaming: paced, all four together, {paced_integrations} integrations each "
        f"(about {paced_integrations * 0.5 + 1:.0f} s)")
    svc = Service(be, everything, progress=log, progress_every=100)
    for o in make(paced_integrations, [0.0, 0.25, 0.5, 0.75]):
        svc.submit(o)
    paced = svc.run(paced=True)
    for oid, st in paced["per_observation"].items():
        log(f"  {oid}: {st['integrations']} integrations, p50 {st['latency_p50_ms']:.2f} ms, "
            f"p99 {st['latency_p99_ms']:.2f} ms, real-time factor {st['realtime_factor']:.3f}")
    out["paced"] = {"hbm_budget_bytes": everything, **_rounded(paced)}
    budget = need["obs256x3072"] + need["obs512x384"] + need["obs256x768"]  # the fourth has to wait
    log(f"streaming: paced under a budget of {budget / 1e9:.2f} GB (three of four), {queued_integrations} each")
    svc = Service(be, budget)
    for o in make(queued_integrations, [0.0, 0.25, 0.5, 0.75]):
        svc.submit(o)
    queued = svc.run(paced=True)
    out["paced_queued"] = {"hbm_budget_bytes": budget, **_rounded(queued)}
    svc = Service(be, everything)
    for o in make(flat_integrations, [0, 0, 0, 0]):
        svc.submit(o)
    flat = svc.run(paced=False)
    log(f"streaming flat out: {flat['realtime_factor']:.2f}x real time")
    out["flat_out"] = _rounded(flat)
    return out


def model_bytes(n, f):
    from paper_1501_05992_amd import model

    return model.input_bytes(n, f, model.SAMPLE_RATE_HZ)


UNEVEN = [(64, 3072, 10000, 0), (256, 768, 5000, 0), (512, 384, 4000, 0), (2048, 128, 2000, 0)]


def uneven_batch(corrx, model, synth, torch, dev, oracle, autotune=True):
    """Arrays of 64/256/512/2048 inputs in one persistent launch, tile codes
    from the autotuner; each array also timed alone through corr_xmac."""
    from paper_1501_05992_amd import tune

    seed = synth.config_seed(3)
    hosts = [synth.make_input(seed, n, f, t, array=k) for k, (n, f, t, lay) in enumerate(UNEVEN)]
    ins = [torch.from_numpy(h).to(dev) for h in hosts]
    probe = corrx.Batch(UNEVEN)
    accs = probe.new_accs(dev)
    probe.close()
    if autotune:
        log("autotuning the uneven batch")
        codes, report = tune.tune_batch(UNEVEN, ins, accs, use_cache=False)
    else:
        codes = [corrx.CORRX_TILE_DEFAULT] * len(UNEVEN)
    b = corrx.Batch(UNEVEN, tile_cfg=codes)
    plan = [b.plan(k) for k in range(len(UNEVEN))]
    b.zero(accs)
    b.xmac(ins, accs)
    torch.cuda.synchronize()
    checks = []
    for (n, f, t, lay), h, acc in zip(UNEVEN, hosts, accs):
        ch = np.ascontiguousarray(synth.channel_view(h, lay, n, f, t, f - 1))
        checks.append(bool(np.array_equal(acc[f - 1].cpu().numpy().astype(np.int64), oracle.xmac(ch, n, 1, t)[0])))
    s = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(10)]
    for e0, e1 in evs:
        b.zero(accs)
        e0.record(s)
        b.xmac(ins, accs)
        e1.record(s)
    torch.cuda.synchronize()
    ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in evs]))
    ops = sum(model.alg_ops(n, f, t) for (n, f, t, lay) in UNEVEN)
    alone = []
    for (n, f, t, lay), xin in zip(UNEVEN, ins):
        c = corrx.Correlator(n, f, t, lay)
        acc = c.new_acc(dev)
        ams = time_xmac(corrx, torch, c, xin, acc, 5)
        alone.append({"n_inputs": n, "n_chan": f, "n_time": t, "xmac_ms": round(ams, 3),
                      "tops": round(model.alg_ops(n, f, t) / ams / 1e9, 1)})
        c.close()
        del acc
    res = {"arrays": [list(d[:3]) for d in UNEVEN], "tile_codes": [hex(c) for c in codes],
           "plan_kind_splits": plan, "items": b.items, "ms": round(ms, 3), "tops": round(ops / ms / 1e9, 1),
           "frac_of_peak": round(ops / ms / 1e9 / PEAK_INT8_TOPS, 4), "alone": alone,
           "alone_sum_ms": round(sum(a["xmac_ms"] for a in alone), 3),
           "sampled_channel_bit_exact": checks}
    b.close()
    log(f"uneven batch: {ms:.3f} ms ({res['tops']} TOPS), alone sum {res['alone_sum_ms']} ms")
    return res


def cpu_baseline(oracle, model, synth, host, n, fc, tc, n_ch):
    threads = os.cpu_count() or 1
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    oracle.set_threads(threads)
    used = oracle.get_threads()
    n_ch = min(n_ch, fc)
    sub = np.ascontiguousarray(host.reshape(tc, fc, n)[:, :n_ch, :]).reshape(-1)
    t0 = time.perf_counter()
    oracle.xmac(sub, n, n_ch, tc)
    dt = time.perf_counter() - t0
    ops = model.alg_ops(n, n_ch, tc)
    return {"value": round(ops / dt / 1e12, 4), "unit": "TOPS", "cores": used, "kind": "oracle",
            "sample": f"{n_ch} of {fc} channels x {tc} samples x {n} inputs (gcc -O2 -fopenmp int64 triple loop, "
                      f"OpenMP over channels), {dt:.1f} s",
            "cpu": cpu_model(), "host_cpus": os.cpu_count(),
            "xrt": round(model.realtime_factor(tc, dt * fc / n_ch), 4)}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
