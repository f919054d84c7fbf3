"""GPU parity: every engine of the C-ABI library against the CPU oracle,
element by element, tolerance 0 (all sums are exact integers)."""

import numpy as np
import pytest

from paper_1501_05992_amd import synth

pytestmark = pytest.mark.gpu

ENGINES = ["plain", "mfma_i8", "mfma_f8"]
ENGINES_ANY_N = ["plain", "mfma_i8"]  # the fp8 engine serves up to 256 inputs


@pytest.fixture(scope="module")
def cx():
    import torch

    from paper_1501_05992_amd import corrx

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    corrx.lib()
    return corrx


def _run(cx, buf, n, fc, tc, layout=0, engine="mfma_i8", calls=1):
    import torch

    dev = torch.device("cuda:0")
    c = cx.Correlator(n, fc, tc, layout, engine)
    x = torch.from_numpy(np.ascontiguousarray(buf)).to(dev)
    acc = c.new_acc(dev)
    c.zero(acc)
    for _ in range(calls):
        c.xmac(x, acc)
    torch.cuda.synchronize()
    out = acc.cpu().numpy().astype(np.int64)
    c.close()
    return out


def _compare(got, want, n, label):
    if np.array_equal(got, want):
        return
    bad = np.argwhere(got != want)
    f, b, part = bad[0]
    i = int((np.sqrt(8 * b + 1) - 1) // 2)
    j = b - i * (i + 1) // 2
    raise AssertionError(f"{label}: {len(bad)} mismatches; first f={f} (i={i}, j={j}) part={part} "
                         f"got {got[f, b, part]} want {want[f, b, part]}")


@pytest.mark.parametrize("engine", ENGINES)
def test_config_plain_tiny(cx, oracle_lib, engine):
    # 256 inputs, 8 channels, 2000 samples (the small configuration)
    n, fc, tc = 256, 8, 2000
    buf = synth.make_input(synth.config_seed(0), n, fc, tc)
    _compare(_run(cx, buf, n, fc, tc, engine=engine), oracle_lib.xmac(buf, n, fc, tc), n, engine)


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("n", [1, 2, 3, 5, 63, 64, 65, 100, 127, 128, 129, 200, 255, 256])
def test_input_counts(cx, oracle_lib, engine, n):
    fc, tc = 3, 97
    buf = synth.make_input(1000 + n, n, fc, tc)
    _compare(_run(cx, buf, n, fc, tc, engine=engine), oracle_lib.xmac(buf, n, fc, tc), n, f"{engine} N={n}")


@pytest.mark.parametrize("engine", ENGINES_ANY_N)
@pytest.mark.parametrize("n", [257, 300, 384, 511, 512, 513, 700, 1024, 2048])
def test_multi_block_input_counts(cx, oracle_lib, engine, n):
    # more than 256 inputs: diagonal blocks plus cross units
    fc, tc = 2, 77
    buf = synth.make_input(8000 + n, n, fc, tc)
    _compare(_run(cx, buf, n, fc, tc, engine=engine), oracle_lib.xmac(buf, n, fc, tc), n, f"{engine} N={n}")


def test_multi_block_split_and_layout(cx, oracle_lib):
    n, fc, tc = 520, 1, 3000
    buf = synth.make_input(8100, n, fc, tc, layout=1)
    _compare(_run(cx, buf, n, fc, tc, layout=1), oracle_lib.xmac(buf, n, fc, tc, 1), n, "N=520 FTI split")


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("tc", [1, 15, 16, 63, 64, 65, 129, 1000, 4097])
def test_ragged_time(cx, oracle_lib, engine, tc):
    n, fc = 256, 2
    buf = synth.make_input(2000 + tc, n, fc, tc)
    _compare(_run(cx, buf, n, fc, tc, engine=engine), oracle_lib.xmac(buf, n, fc, tc), n, f"{engine} T={tc}")


@pytest.mark.parametrize("n,layout", [(64, 0), (40, 1)])
@pytest.mark.parametrize("tc", [1, 127, 128, 129, 1000, 4097])
def test_ragged_time_small_units(cx, oracle_lib, n, layout, tc):
    # 64-input units take 128-sample chunks
    fc = 3
    buf = synth.make_input(2500 + tc, n, fc, tc, layout=layout)
    _compare(_run(cx, buf, n, fc, tc, layout), oracle_lib.xmac(buf, n, fc, tc, layout), n, f"N={n} T={tc}")


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("layout", [0, 1])
def test_layouts(cx, oracle_lib, engine, layout):
    n, fc, tc = 96, 5, 333
    buf = synth.make_input(3000, n, fc, tc, layout=layout)
    _compare(_run(cx, buf, n, fc, tc, layout, engine), oracle_lib.xmac(buf, n, fc, tc, layout), n,
             f"{engine} layout={layout}")


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("n", [7, 128, 256])
def test_invalid_codes_and_extreme_values(cx, oracle_lib, engine, n):
    # every byte value occurs, including the invalid code in either nibble,
    # and long runs of the extreme samples (+-7 +-7j)
    fc, tc = 2, 300
    rng = np.random.default_rng(n)
    buf = rng.integers(0, 256, size=n * fc * tc, dtype=np.uint8)
    buf[: n * 40] = 0x77
    buf[n * 40: n * 80] = 0x99
    buf[n * 80: n * 90] = 0x79
    _compare(_run(cx, buf, n, fc, tc, engine=engine), oracle_lib.xmac(buf, n, fc, tc), n, f"{engine} bytes")


@pytest.mark.parametrize("engine", ENGINES_ANY_N)
@pytest.mark.parametrize("n", [300, 520])
def test_invalid_codes_and_extreme_values_large_arrays(cx, oracle_lib, engine, n):
    # the same byte mix through the cross units (rows and columns of
    # off-diagonal blocks), with a ragged last block
    fc, tc = 2, 200
    rng = np.random.default_rng(n)
    buf = rng.integers(0, 256, size=n * fc * tc, dtype=np.uint8)
    buf[: n * 30] = 0x77
    buf[n * 30: n * 60] = 0x99
    buf[n * 60: n * 70] = 0x79
    buf[n * 70: n * 80] = 0x97
    _compare(_run(cx, buf, n, fc, tc, engine=engine), oracle_lib.xmac(buf, n, fc, tc), n, f"{engine} bytes N={n}")


@pytest.mark.parametrize("engine", ENGINES)
def test_accumulates_across_calls(cx, oracle_lib, engine):
    n, fc, tc = 64, 4, 200
    buf = synth.make_input(4000, n, fc, tc)
    _compare(_run(cx, buf, n, fc, tc, engine=engine, calls=3), 3 * oracle_lib.xmac(buf, n, fc, tc), n,
             f"{engine} x3")


@pytest.mark.parametrize("engine,n", [(e, 256) for e in ENGINES] + [("mfma_i8", 64), ("mfma_i8", 128)])
def test_time_split_path(cx, oracle_lib, engine, n):
    # few channels and many samples: the library splits time across workgroups
    fc, tc = 1, 20000
    buf = synth.make_input(5000 + n, n, fc, tc)
    _compare(_run(cx, buf, n, fc, tc, engine=engine), oracle_lib.xmac(buf, n, fc, tc), n, f"{engine} split")


@pytest.mark.parametrize("n,fc,tc,calls", [(300, 2, 6000, 2), (256, 3, 9000, 3), (64, 1, 50000, 2),
                                           (129, 1, 30000, 1), (1000, 1, 4000, 2), (2048, 1, 1500, 1)])
def test_time_split_partial_sums(cx, oracle_lib, n, fc, tc, calls):
    # time splits of the int8 engine: split 0 writes the accumulator (stored
    # on the first call after zero, added on later calls), the others store
    # partial sums that a second launch adds; diagonal blocks and cross units,
    # ragged last block and ragged last split
    buf = synth.make_input(5200 + n, n, fc, tc)
    _compare(_run(cx, buf, n, fc, tc, calls=calls), calls * oracle_lib.xmac(buf, n, fc, tc), n,
             f"N={n} F={fc} T={tc} x{calls}")


@pytest.mark.parametrize("n,fc,tc,calls", [(160, 1030, 200, 1), (256, 1024, 130, 2), (131, 1024, 70, 1)])
def test_many_channels_every_channel(cx, oracle_lib, n, fc, tc, calls):
    # four or more rounds of units per compute unit, channel counts that do
    # not divide evenly among them; every channel checked, also on top of an
    # earlier call (read-modify-write) and for an unaligned input count
    buf = synth.make_input(5500 + n, n, fc, tc)
    _compare(_run(cx, buf, n, fc, tc, calls=calls), calls * oracle_lib.xmac(buf, n, fc, tc), n,
             f"N={n} F={fc} T={tc} x{calls}")


def test_single_tone_closed_form(cx):
    n, fc, tc = 256, 2, 1000
    rng = np.random.default_rng(9)
    gr = rng.integers(-7, 8, size=n)
    gi = rng.integers(-7, 8, size=n)
    buf = synth.tone_input(gr, gi, fc, tc)
    got = _run(cx, buf, n, fc, tc)
    g = gr + 1j * gi
    ii, jj = np.tril_indices(n)
    want = tc * g[ii] * np.conj(g[jj])
    for f in range(fc):
        assert np.array_equal(got[f, :, 0], np.rint(want.real).astype(np.int64))
        assert np.array_equal(got[f, :, 1], np.rint(want.imag).astype(np.int64))


def test_dump_orders_and_types(cx, oracle_lib):
    import torch

    n, fc, tc = 64, 3, 150
    buf = synth.make_input(6000, n, fc, tc)
    want = oracle_lib.xmac(buf, n, fc, tc)
    c = cx.Correlator(n, fc, tc)
    x = torch.from_numpy(buf).cuda()
    acc = c.new_acc()
    c.zero(acc)
    c.xmac(x, acc)
    tri_i = c.dump(acc, cx.CORRX_TRI_INPUT, cx.CORRX_I32).cpu().numpy()
    tri_f = c.dump(acc, cx.CORRX_TRI_INPUT, cx.CORRX_F32).cpu().numpy()
    sp_i = c.dump(acc, cx.CORRX_TRI_STATION_POL, cx.CORRX_I32).cpu().numpy()
    sp_f = c.dump(acc, cx.CORRX_TRI_STATION_POL, cx.CORRX_F32).cpu().numpy()
    assert np.array_equal(tri_i.reshape(want.shape), want)
    assert np.array_equal(tri_f.reshape(want.shape), want.astype(np.float32))
    sp = oracle_lib.station_pol(want, n)
    assert sp_i.size == fc * (n // 2) * (n // 2 + 1) // 2 * 8
    assert np.array_equal(sp_i.reshape(sp.shape), sp)
    assert np.array_equal(sp_f.reshape(sp.shape), sp.astype(np.float32))
    c.close()


def test_zero_resets_and_overflow_guard(cx):
    import torch

    c = cx.Correlator(8, 1, 5_000_000)
    x = torch.zeros(8 * 5_000_000, dtype=torch.uint8, device="cuda")
    acc = c.new_acc()
    c.zero(acc)
    for _ in range(4):
        c.xmac(x, acc)
    with pytest.raises(cx.CorrxError) as e:
        c.xmac(x, acc)
    assert e.value.status == cx.CORRX_EOVERFLOW
    with pytest.raises(cx.CorrxError):
        c.dump(acc, cx.CORRX_TRI_INPUT, cx.CORRX_F32)
    c.zero(acc)
    assert c.samples == 0
    c.xmac(x, acc)
    torch.cuda.synchronize()
    assert int(acc.abs().sum()) == 0
    c.close()


def test_batch_overflow_guard(cx):
    """The batch counts samples per array since corr_batch_zero and refuses a
    call that could wrap an int32 accumulator, before enqueuing anything."""
    import torch

    descs = [(4, 1, 5_000_000, 0), (8, 2, 1000, 0)]
    b = cx.Batch(descs)
    ins = [torch.zeros(n * f * t, dtype=torch.uint8, device="cuda") for (n, f, t, lay) in descs]
    accs = b.new_accs()
    b.zero(accs)
    for k in range(4):
        b.xmac(ins, accs)
        assert b.samples(0) == 5_000_000 * (k + 1) and b.samples(1) == 1000 * (k + 1)
    with pytest.raises(cx.CorrxError) as e:
        b.xmac(ins, accs)  # 25,000,000 > 21,913,098 samples for array 0
    assert e.value.status == cx.CORRX_EOVERFLOW
    assert b.samples(0) == 20_000_000
    b.zero(accs)
    assert b.samples(0) == 0 and b.samples(1) == 0
    b.xmac(ins, accs)
    torch.cuda.synchronize()
    assert all(int(a.abs().sum()) == 0 for a in accs)
    b.close()


# 16-lane rows with a 64 x 64 tile transpose (TFI) or direct rows (FTI) when
# N % 16 == 0; one thread per row otherwise.  Shapes cover whole and ragged
# tiles, N below, at and above 256, and invalid codes.
@pytest.mark.parametrize("n,fc,tc,layout", [(256, 4, 500, 0), (256, 64, 128, 0), (48, 70, 65, 0), (512, 3, 130, 0),
                                            (256, 5, 77, 1), (320, 2, 40, 1), (7, 3, 50, 0), (100, 2, 33, 1)])
def test_beam(cx, oracle_lib, n, fc, tc, layout):
    import torch

    buf = synth.make_input(7000 + n, n, fc, tc, layout=layout)
    buf[:100] = 0x88
    buf[1000:1040] = 0x80  # invalid real part: contributes nothing
    c = cx.Correlator(n, fc, tc, layout)
    out = c.beam(torch.from_numpy(buf).cuda()).cpu().numpy()
    assert np.array_equal(out.astype(np.int64), oracle_lib.incoherent_beam(buf, n, fc, tc, layout))
    c.close()


BATCH = [(64, 6, 300, 0), (256, 3, 200, 0), (512, 2, 150, 0), (1024, 1, 70, 1), (128, 5, 333, 1), (100, 3, 90, 0)]


def _batch_inputs(descs):
    return [synth.make_input(9000 + k, n, f, t, layout=lay) for k, (n, f, t, lay) in enumerate(descs)]


@pytest.mark.parametrize("tile_cfg", [None, "unit256", "splits"])
def test_batch_uneven_arrays(cx, oracle_lib, tile_cfg):
    import torch

    descs = BATCH
    bufs = _batch_inputs(descs)
    cfg = None
    if tile_cfg == "unit256":
        cfg = [cx.CORRX_TILE_UNIT256] * len(descs)
    elif tile_cfg == "splits":
        cfg = [cx.CORRX_TILE_DEFAULT | (3 << 8)] * len(descs)
    b = cx.Batch(descs, tile_cfg=cfg)
    assert b.items > 0
    ins = [torch.from_numpy(x).cuda() for x in bufs]
    accs = [a.fill_(7) for a in b.new_accs()]
    b.zero(accs)
    b.xmac(ins, accs)  # writes
    b.xmac(ins, accs)  # accumulates
    torch.cuda.synchronize()
    for (n, f, t, lay), x, acc in zip(descs, bufs, accs):
        _compare(acc.cpu().numpy().astype(np.int64), 2 * oracle_lib.xmac(x, n, f, t, lay), n, f"batch N={n}")
    b.close()


def test_batch_small_units_ragged_time(cx, oracle_lib):
    # the batch's 64-input units take 256-sample chunks: lengths around it
    import torch

    descs = [(64, 3, 1, 0), (64, 4, 255, 1), (48, 2, 256, 0), (64, 3, 257, 0), (32, 5, 600, 1)]
    bufs = _batch_inputs(descs)
    b = cx.Batch(descs, tile_cfg=[cx.CORRX_TILE_UNIT64 | (1 << 8)] * len(descs))
    accs = b.new_accs()
    b.zero(accs)
    b.xmac([torch.from_numpy(x).cuda() for x in bufs], accs)
    torch.cuda.synchronize()
    for (n, f, t, lay), x, acc in zip(descs, bufs, accs):
        _compare(acc.cpu().numpy().astype(np.int64), oracle_lib.xmac(x, n, f, t, lay), n, f"batch N={n} T={t}")
    b.close()


def test_batch_matches_single_calls(cx):
    import torch

    descs = [(64, 9, 500, 0), (256, 4, 1000, 0), (512, 2, 600, 0)]
    bufs = _batch_inputs(descs)
    ins = [torch.from_numpy(x).cuda() for x in bufs]
    b = cx.Batch(descs)
    accs = b.new_accs()
    b.xmac(ins, accs)
    for (n, f, t, lay), x, acc in zip(descs, ins, accs):
        c = cx.Correlator(n, f, t, lay)
        ref = c.new_acc()
        c.zero(ref)
        c.xmac(x, ref)
        torch.cuda.synchronize()
        assert torch.equal(ref, acc)
        c.close()
    b.close()


def test_batch_rejects_unaligned_inputs(cx):
    with pytest.raises(cx.CorrxError) as e:
        cx.Batch([(66, 2, 10, 0)])
    assert e.value.status == cx.CORRX_EUNSUPPORTED
    with pytest.raises(cx.CorrxError):
        cx.Batch([(256, 2, 10, 0)], tile_cfg=[cx.CORRX_TILE_UNIT64])


@pytest.mark.parametrize("tc", [131072, 131073, 171197])
def test_fp8_exact_at_the_fp32_bound(cx, oracle_lib, tc):
    # every sample 7+7j: |G| grows by 98 per sample, the largest possible, so
    # fp32 partial sums reach 98 * 2^17 within one work unit
    n, fc = 32, 1
    buf = np.full(n * fc * tc, 0x77, dtype=np.uint8)
    got = _run(cx, buf, n, fc, tc, engine="mfma_f8")
    want = oracle_lib.xmac(buf[: n * 1000], n, fc, 1000) * tc // 1000
    _compare(got, want, n, f"fp8 T={tc}")


def test_fp8_rejects_large_arrays(cx):
    c = cx.Correlator(300, 1, 10, engine="mfma_f8")
    import torch

    x = torch.zeros(3000, dtype=torch.uint8, device="cuda")
    acc = c.new_acc()
    with pytest.raises(cx.CorrxError) as e:
        c.xmac(x, acc)
    assert e.value.status == cx.CORRX_EUNSUPPORTED
    c.close()


def test_binding_rejects_host_short_and_strided_buffers(cx):
    # the library takes plain device pointers; the binding checks tensors first
    import torch

    c = cx.Correlator(64, 2, 10)
    acc = c.new_acc()
    x = torch.zeros(64 * 2 * 10, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        c.xmac(x.cpu(), acc)  # host memory
    with pytest.raises(ValueError):
        c.xmac(x[:-1], acc)  # one byte short
    with pytest.raises(ValueError):
        c.xmac(x, acc[:, :-1])  # short accumulator
    with pytest.raises(ValueError):
        c.zero(torch.zeros((acc.shape[1], 2, 2), dtype=torch.int32, device="cuda").transpose(0, 1))  # strided
    with pytest.raises(ValueError):
        c.dump(acc, cx.CORRX_TRI_INPUT, cx.CORRX_I32, dst=torch.empty(10, dtype=torch.int32, device="cuda"))
    c.zero(acc)
    c.xmac(x, acc)
    torch.cuda.synchronize()
    assert int(acc.abs().sum()) == 0  # byte 0x00 is the sample 0 + 0j
    c.close()


def test_graph_capture_of_a_step(cx, oracle_lib):
    # zero + xmac + dump captured once and replayed: every replay equals the
    # eager result, with other device work and synchronisation in between
    import torch

    n, fc, tc = 128, 6, 700
    buf = synth.make_input(4242, n, fc, tc)
    x = torch.from_numpy(buf).cuda()
    c = cx.Correlator(n, fc, tc)
    acc = c.new_acc()
    dst = torch.empty(cx.corr_dump_count(c.h, cx.CORRX_TRI_STATION_POL), dtype=torch.float32, device="cuda")
    c.zero(acc)
    c.xmac(x, acc)
    c.dump(acc, cx.CORRX_TRI_STATION_POL, cx.CORRX_F32, dst)
    torch.cuda.synchronize()
    eager = dst.clone()
    want = oracle_lib.station_pol(oracle_lib.xmac(buf, n, fc, tc), n).astype(np.float32).reshape(-1)
    assert np.array_equal(eager.cpu().numpy(), want)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            c.zero(acc)
            c.xmac(x, acc)
            c.dump(acc, cx.CORRX_TRI_STATION_POL, cx.CORRX_F32, dst)
    torch.cuda.current_stream().wait_stream(s)
    for r in range(4):
        dst.fill_(-1.0)
        acc.fill_(123)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(dst, eager), f"replay {r}"
    del g
    c.close()


_RNG_CASES = np.random.default_rng(1501).integers(0, 2**31, size=16)


@pytest.mark.parametrize("case", range(16))
def test_random_shapes(cx, oracle_lib, case):
    # seeded random shapes, layouts and engines, element by element
    rng = np.random.default_rng(int(_RNG_CASES[case]))
    engine = ["mfma_i8", "plain", "mfma_f8"][case % 3]
    n = int(rng.integers(1, 257 if engine == "mfma_f8" else 401))
    fc, tc, layout = int(rng.integers(1, 4)), int(rng.integers(1, 2001)), int(rng.integers(0, 2))
    print(f"random case {case}: N={n} F={fc} T={tc} layout={layout} {engine}", flush=True)
    buf = synth.make_input(600 + case, n, fc, tc, layout=layout)
    if case % 4 == 1:  # some invalid codes
        buf[rng.integers(0, buf.size, size=max(1, buf.size // 500))] = 0x83
    _compare(_run(cx, buf, n, fc, tc, layout, engine), oracle_lib.xmac(buf, n, fc, tc, layout), n,
             f"case {case} N={n} F={fc} T={tc} layout={layout} {engine}")


def _batch_chunks(cx, unit, n):
    # chunk lengths the batch kernels have for a unit
    if unit == cx.CORRX_TILE_UNIT64 or (unit == cx.CORRX_TILE_DEFAULT and n <= 64):
        return [0, 128, 256]
    if unit == cx.CORRX_TILE_UNIT128 or (unit == cx.CORRX_TILE_DEFAULT and n <= 128):
        return [0, 64, 128]
    return [0, 64]


@pytest.mark.parametrize("case", range(8))
def test_random_batches(cx, oracle_lib, case):
    # seeded random uneven batches with random valid tile codes (unit, time
    # splits, chunk length)
    import torch

    rng = np.random.default_rng(7000 + case)
    descs, codes = [], []
    for _ in range(int(rng.integers(2, 6))):
        n = 4 * int(rng.integers(1, 151))
        descs.append((n, int(rng.integers(1, 5)), int(rng.integers(1, 1501)), int(rng.integers(0, 2))))
        units = [cx.CORRX_TILE_DEFAULT, cx.CORRX_TILE_UNIT256]
        if n <= 128:
            units.append(cx.CORRX_TILE_UNIT128)
        if n <= 64:
            units.append(cx.CORRX_TILE_UNIT64)
        unit = int(rng.choice(units))
        codes.append(cx.tile_code(unit, int(rng.choice([0, 1, 2, 4])), int(rng.choice(_batch_chunks(cx, unit, n)))))
    print(f"random batch {case}: {descs} codes {[hex(c) for c in codes]}", flush=True)
    bufs = [synth.make_input(7100 + 10 * case + k, n, f, t, layout=lay) for k, (n, f, t, lay) in enumerate(descs)]
    b = cx.Batch(descs, tile_cfg=codes)
    accs = b.new_accs()
    b.zero(accs)
    b.xmac([torch.from_numpy(x).cuda() for x in bufs], accs)
    torch.cuda.synchronize()
    for (n, f, t, lay), x, acc in zip(descs, bufs, accs):
        _compare(acc.cpu().numpy().astype(np.int64), oracle_lib.xmac(x, n, f, t, lay), n, f"batch {case} N={n}")
    b.close()


@pytest.mark.parametrize("n", [40, 64, 120, 200, 256, 300])
def test_set_tile_every_candidate(cx, oracle_lib, n):
    # corr_xmac under every tile code the tuner may pick (unit, time splits,
    # chunk length), T ragged for every chunk length, twice in a row
    import torch

    from paper_1501_05992_amd import tune

    fc, tc = 3, 700
    buf = synth.make_input(9300 + n, n, fc, tc)
    want = oracle_lib.xmac(buf, n, fc, tc)
    x = torch.from_numpy(buf).cuda()
    codes = tune.candidates(n, "xmac")
    print(f"N={n}: {len(codes)} codes", flush=True)
    for code in codes:
        c = cx.Correlator(n, fc, tc, 0, "mfma_i8")
        c.set_tile(code)
        acc = c.new_acc()
        c.zero(acc)
        c.xmac(x, acc)
        c.xmac(x, acc)
        torch.cuda.synchronize()
        _compare(acc.cpu().numpy().astype(np.int64), 2 * want, n, f"N={n} code {code:#x}")
        c.close()


def test_set_tile_rejects(cx):
    c = cx.Correlator(100, 2, 100, 0, "mfma_i8")
    with pytest.raises(cx.CorrxError) as e:
        c.set_tile(cx.CORRX_TILE_UNIT64)  # 64-input unit cannot hold 100 inputs
    assert e.value.status == cx.CORRX_EINVAL
    with pytest.raises(cx.CorrxError) as e:
        c.set_tile(cx.tile_code(cx.CORRX_TILE_UNIT256, 0, 128))  # no 128-sample chunk for 256-input units
    assert e.value.status == cx.CORRX_EUNSUPPORTED
    with pytest.raises(cx.CorrxError) as e:
        c.set_tile(1 << 28)
    assert e.value.status == cx.CORRX_EINVAL
    c.close()
