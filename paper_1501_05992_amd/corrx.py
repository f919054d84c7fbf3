"""ctypes binding of libcorrx.so (include/corrx.h), same names as the C ABI.

Argument marshalling only: every step of the correlation runs in the HIP
library.  PyTorch supplies device memory and streams; it is imported before
the library is loaded so that both use the one HIP runtime PyTorch brought
into the process.  There is no fallback: without the built library on a
gfx950 device every call raises.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

import torch  # noqa: F401  (loads the HIP runtime first; see module docstring)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcorrx.so")

CORRX_OK = 0
CORRX_EINVAL = -1
CORRX_ENOMEM = -2
CORRX_EDEVICE = -3
CORRX_EUNSUPPORTED = -4
CORRX_EOVERFLOW = -5
CORRX_ESCRATCH = -6
CORRX_NOALLOC_SCRATCH_BYTES = 64 << 20

CORRX_LAYOUT_TFI = 0
CORRX_LAYOUT_FTI = 1
CORRX_TRI_INPUT = 0
CORRX_TRI_STATION_POL = 1
CORRX_I32 = 0
CORRX_F32 = 1
CORRX_ENGINE_AUTO = 0
CORRX_ENGINE_PLAIN = 1
CORRX_ENGINE_MFMA_I8 = 2
CORRX_ENGINE_MFMA_F8 = 3
CORRX_TILE_DEFAULT = 0
CORRX_TILE_UNIT64 = 1
CORRX_TILE_UNIT128 = 2
CORRX_TILE_UNIT256 = 3
CORRX_ORDER_PACKET = 0
CORRX_ORDER_NATURAL = 1

ENGINES = {"auto": CORRX_ENGINE_AUTO, "plain": CORRX_ENGINE_PLAIN,
           "mfma_i8": CORRX_ENGINE_MFMA_I8, "mfma_f8": CORRX_ENGINE_MFMA_F8}

# Exported symbols, in header order.
SYMBOLS = ("corr_abi_version", "corr_strerror", "corr_create", "corr_destroy", "corr_set_engine",
           "corr_set_tile", "corr_get_engine", "corr_acc_bytes", "corr_dump_count", "corr_zero", "corr_xmac",
           "corr_xmac_noalloc", "corr_dump", "corr_dump_avg", "corr_pfb_ingest", "corr_pfb_remap", "corr_fpfb_create",
           "corr_fpfb_destroy", "corr_fpfb_workspace_bytes", "corr_fpfb_tables", "corr_fpfb", "corr_samples",
           "corr_beam", "corr_batch_create", "corr_batch_destroy",
           "corr_batch_items", "corr_batch_plan", "corr_batch_zero", "corr_batch_xmac", "corr_batch_samples")


class CorrxError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {corr_strerror(status)} ({status})")


class corrx_desc(ctypes.Structure):
    _fields_ = [("n_inputs", ctypes.c_int), ("n_chan", ctypes.c_int),
                ("n_time", ctypes.c_int), ("layout", ctypes.c_int)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libcorrx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1501_05992_amd.build` or __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, sz, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_int64
        sig = {
            "corr_abi_version": ([], i),
            "corr_strerror": ([i], ctypes.c_char_p),
            "corr_create": ([i, i, i, i, ctypes.POINTER(vp)], i),
            "corr_destroy": ([vp], i),
            "corr_set_engine": ([vp, i], i),
            "corr_set_tile": ([vp, i], i),
            "corr_get_engine": ([vp], i),
            "corr_acc_bytes": ([vp], sz),
            "corr_dump_count": ([vp, i], sz),
            "corr_zero": ([vp, vp, vp], i),
            "corr_xmac": ([vp, vp, vp, vp], i),
            "corr_xmac_noalloc": ([vp, vp, i, i, i, i, i, vp], i),
            "corr_dump": ([vp, vp, i, i, vp, vp], i),
            "corr_dump_avg": ([vp, vp, i, i, i, i, vp, vp], i),
            "corr_pfb_ingest": ([vp, ctypes.POINTER(vp), i, vp, vp], i),
            "corr_pfb_remap": ([vp, vp, vp, vp], i),
            "corr_fpfb_create": ([i, i, i, ctypes.POINTER(vp)], i),
            "corr_fpfb_destroy": ([vp], i),
            "corr_fpfb_workspace_bytes": ([vp], sz),
            "corr_fpfb_tables": ([vp, ctypes.POINTER(ctypes.c_int16), ctypes.POINTER(ctypes.c_int8)], i),
            "corr_fpfb": ([vp, vp, i, i, vp, vp, vp], i),
            "corr_samples": ([vp], i64),
            "corr_beam": ([vp, vp, vp, vp], i),
            "corr_batch_create": ([ctypes.POINTER(corrx_desc), i, i, ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(vp)], i),
            "corr_batch_destroy": ([vp], i),
            "corr_batch_items": ([vp], i64),
            "corr_batch_plan": ([vp, i, ctypes.POINTER(i), ctypes.POINTER(i)], i),
            "corr_batch_zero": ([vp, ctypes.POINTER(vp), vp], i),
            "corr_batch_xmac": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp], i),
            "corr_batch_samples": ([vp, i], i64),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        if L.corr_abi_version() != 1:
            raise RuntimeError("libcorrx.so ABI version does not match the binding")
        _lib = L
    return _lib


def corr_strerror(status: int) -> str:
    return lib().corr_strerror(int(status)).decode()


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise CorrxError(rc, what)
    return rc


def _ptr(t, nbytes: int | None = None, what: str = "buffer") -> int | None:
    """Device address of a tensor; a raw integer address passes through.

    The library takes plain pointers and cannot check them, so a tensor must
    be on a GPU, contiguous, and (when nbytes is given) at least nbytes long;
    anything else raises ValueError before the call.
    """
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError(f"{what}: a GPU tensor is required, got one on {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: the tensor must be contiguous")
    have = t.numel() * t.element_size()
    if nbytes is not None and have < nbytes:
        raise ValueError(f"{what}: {have} bytes, at least {nbytes} needed")
    return t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---- flat C-ABI names ---------------------------------------------------------

def corr_create(n_inputs: int, n_chan: int, n_time: int, layout: int = CORRX_LAYOUT_TFI) -> int:
    h = ctypes.c_void_p()
    _check(lib().corr_create(n_inputs, n_chan, n_time, layout, ctypes.byref(h)), "corr_create")
    return h.value


def corr_destroy(h: int) -> None:
    _check(lib().corr_destroy(h), "corr_destroy")


def corr_set_engine(h: int, engine: int) -> None:
    _check(lib().corr_set_engine(h, engine), "corr_set_engine")


def corr_set_tile(h: int, tile_cfg: int) -> None:
    _check(lib().corr_set_tile(h, tile_cfg), "corr_set_tile")


def tile_code(unit: int = CORRX_TILE_DEFAULT, splits: int = 0, chunk: int = 0) -> int:
    """Tile code from a unit (CORRX_TILE_*), time splits (0: automatic) and
    chunk length in samples (0: the unit's default, else 64, 128 or 256)."""
    k = {0: 0, 64: 1, 128: 2, 256: 3}[chunk]
    return unit | (splits << 8) | (k << 24)


def corr_get_engine(h: int) -> int:
    return _check(lib().corr_get_engine(h), "corr_get_engine")


def corr_acc_bytes(h: int) -> int:
    return int(lib().corr_acc_bytes(h))


def corr_dump_count(h: int, order: int) -> int:
    return int(lib().corr_dump_count(h, order))


def corr_samples(h: int) -> int:
    return int(lib().corr_samples(h))


def corr_zero(h: int, acc, stream=None) -> None:
    _check(lib().corr_zero(h, _ptr(acc, corr_acc_bytes(h), "acc"), _stream(stream)), "corr_zero")


def corr_xmac(h: int, inp, acc, stream=None) -> None:
    _check(lib().corr_xmac(h, _ptr(inp, what="input"), _ptr(acc, corr_acc_bytes(h), "acc"), _stream(stream)),
           "corr_xmac")


def corr_xmac_noalloc(inp, acc, n_inputs: int, n_chan: int, n_time: int, layout: int = CORRX_LAYOUT_TFI,
                      accumulate: bool = False, stream=None) -> None:
    """corr_xmac without a handle or any allocation (int8 engine; time-split
    partial sums in the library's per-device scratch)."""
    acc_bytes = n_chan * (n_inputs * (n_inputs + 1) // 2) * 2 * 4
    _check(lib().corr_xmac_noalloc(_ptr(inp, n_inputs * n_chan * n_time, "input"), _ptr(acc, acc_bytes, "acc"),
                                   n_inputs, n_chan, n_time, layout, int(bool(accumulate)), _stream(stream)),
           "corr_xmac_noalloc")


def corr_dump(h: int, acc, order: int, dtype: int, dst, stream=None) -> None:
    n = corr_dump_count(h, order)
    _check(lib().corr_dump(h, _ptr(acc, corr_acc_bytes(h), "acc"), order, dtype,
                           _ptr(dst, 4 * n if n > 0 else None, "dst"), _stream(stream)), "corr_dump")


def corr_dump_avg(h: int, acc, order: int, dtype: int, f_avg: int, t_avg: int, dst, stream=None) -> None:
    _check(lib().corr_dump_avg(h, _ptr(acc, corr_acc_bytes(h), "acc"), order, dtype, f_avg, t_avg,
                               _ptr(dst, what="dst"), _stream(stream)), "corr_dump_avg")


def corr_pfb_ingest(h: int, lanes, order: int, inp, stream=None) -> None:
    n = len(lanes)
    pl = (ctypes.c_void_p * n)(*[_ptr(x, what="lane") for x in lanes])
    _check(lib().corr_pfb_ingest(h, pl, order, _ptr(inp, what="input"), _stream(stream)), "corr_pfb_ingest")


def corr_pfb_remap(h: int, acc_pkt, acc_nat, stream=None) -> None:
    nb = corr_acc_bytes(h)
    _check(lib().corr_pfb_remap(h, _ptr(acc_pkt, nb, "acc_pkt"), _ptr(acc_nat, nb, "acc_nat"), _stream(stream)),
           "corr_pfb_remap")


def corr_fpfb_create(n_inputs: int, n_coarse: int, n_frames: int) -> int:
    h = ctypes.c_void_p()
    _check(lib().corr_fpfb_create(n_inputs, n_coarse, n_frames, ctypes.byref(h)), "corr_fpfb_create")
    return h.value


def corr_fpfb_destroy(h: int) -> None:
    _check(lib().corr_fpfb_destroy(h), "corr_fpfb_destroy")


def corr_fpfb_workspace_bytes(h: int) -> int:
    return int(lib().corr_fpfb_workspace_bytes(h))


def corr_fpfb_tables(h: int):
    taps = np.zeros(1536, dtype=np.int16)
    wmat = np.zeros(256 * 256, dtype=np.int8)
    _check(lib().corr_fpfb_tables(h, taps.ctypes.data_as(ctypes.POINTER(ctypes.c_int16)),
                                  wmat.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))), "corr_fpfb_tables")
    return taps, wmat.reshape(256, 256)


def corr_fpfb(h: int, inp, s1: int, s2: int, work, out, stream=None) -> None:
    _check(lib().corr_fpfb(h, _ptr(inp, what="input"), s1, s2, _ptr(work, corr_fpfb_workspace_bytes(h), "work"),
                           _ptr(out, what="out"), _stream(stream)), "corr_fpfb")


def corr_beam(h: int, inp, out, stream=None) -> None:
    _check(lib().corr_beam(h, _ptr(inp, what="input"), _ptr(out, what="out"), _stream(stream)), "corr_beam")


def corr_batch_create(descs, engine: int = CORRX_ENGINE_AUTO, tile_cfg=None) -> int:
    n = len(descs)
    arr = (corrx_desc * n)(*[corrx_desc(*d) for d in descs])
    cfg = None
    if tile_cfg is not None:
        cfg = (ctypes.c_int * n)(*[int(c) for c in tile_cfg])
    h = ctypes.c_void_p()
    _check(lib().corr_batch_create(arr, n, engine, cfg, ctypes.byref(h)), "corr_batch_create")
    return h.value


def corr_batch_destroy(b: int) -> None:
    _check(lib().corr_batch_destroy(b), "corr_batch_destroy")


def corr_batch_items(b: int) -> int:
    return int(_check(lib().corr_batch_items(b), "corr_batch_items"))


def corr_batch_plan(b: int, array: int) -> tuple[int, int]:
    kind, splits = ctypes.c_int(), ctypes.c_int()
    _check(lib().corr_batch_plan(b, array, ctypes.byref(kind), ctypes.byref(splits)), "corr_batch_plan")
    return kind.value, splits.value


def corr_batch_zero(b: int, accs, stream=None) -> None:
    n = len(accs)
    pacc = (ctypes.c_void_p * n)(*[_ptr(x, what="acc") for x in accs])
    _check(lib().corr_batch_zero(b, pacc, _stream(stream)), "corr_batch_zero")


def corr_batch_xmac(b: int, ins, accs, stream=None) -> None:
    n = len(ins)
    pin = (ctypes.c_void_p * n)(*[_ptr(x, what="input") for x in ins])
    pacc = (ctypes.c_void_p * n)(*[_ptr(x, what="acc") for x in accs])
    _check(lib().corr_batch_xmac(b, pin, pacc, _stream(stream)), "corr_batch_xmac")


def corr_batch_samples(b: int, array: int) -> int:
    return int(_check(lib().corr_batch_samples(b, array), "corr_batch_samples"))


# ---- convenience wrapper --------------------------------------------------------

class Correlator:
    """One correlator handle: shape fixed at creation (corr_create)."""

    def __init__(self, n_inputs: int, n_chan: int, n_time: int, layout: int = CORRX_LAYOUT_TFI,
                 engine: int | str = CORRX_ENGINE_AUTO):
        self.n_inputs, self.n_chan, self.n_time, self.layout = n_inputs, n_chan, n_time, layout
        self.h = corr_create(n_inputs, n_chan, n_time, layout)
        if isinstance(engine, str):
            engine = ENGINES[engine]
        corr_set_engine(self.h, engine)

    def close(self) -> None:
        if self.h:
            corr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def engine(self) -> int:
        return corr_get_engine(self.h)

    def set_engine(self, engine: int | str) -> None:
        corr_set_engine(self.h, ENGINES[engine] if isinstance(engine, str) else engine)

    def set_tile(self, tile_cfg: int) -> None:
        corr_set_tile(self.h, tile_cfg)

    def new_acc(self, device="cuda") -> torch.Tensor:
        nb = self.n_inputs * (self.n_inputs + 1) // 2
        return torch.zeros((self.n_chan, nb, 2), dtype=torch.int32, device=device)

    def zero(self, acc, stream=None) -> None:
        corr_zero(self.h, acc, stream)

    def xmac(self, inp, acc, stream=None) -> None:
        _ptr(inp, self.n_inputs * self.n_chan * self.n_time, "input")
        corr_xmac(self.h, inp, acc, stream)

    def dump(self, acc, order: int = CORRX_TRI_INPUT, dtype: int = CORRX_I32, dst=None, stream=None):
        n = corr_dump_count(self.h, order)
        if dst is None:
            dst = torch.empty(n, dtype=torch.int32 if dtype == CORRX_I32 else torch.float32,
                              device=acc.device)
        corr_dump(self.h, acc, order, dtype, dst, stream)
        return dst

    def dump_avg(self, acc, f_avg: int, t_avg: int = 1, order: int = CORRX_TRI_STATION_POL,
                 dtype: int = CORRX_F32, dst=None, stream=None):
        n = corr_dump_count(self.h, order) // f_avg
        if dst is None:
            dst = torch.empty(n, dtype=torch.int32 if dtype == CORRX_I32 else torch.float32,
                              device=acc.device)
        corr_dump_avg(self.h, acc, order, dtype, f_avg, t_avg, dst, stream)
        return dst

    def pfb_ingest(self, lanes, order: int = CORRX_ORDER_NATURAL, inp=None, stream=None):
        if self.n_chan % 128 == 0:
            for x in lanes:
                _ptr(x, (self.n_chan // 128) * 4 * self.n_time * 256, "lane")
        if inp is None:
            inp = torch.empty(self.n_time * self.n_chan * self.n_inputs, dtype=torch.uint8,
                              device=lanes[0].device)
        corr_pfb_ingest(self.h, lanes, order, inp, stream)
        return inp

    def pfb_remap(self, acc_pkt, acc_nat=None, stream=None):
        if acc_nat is None:
            acc_nat = torch.empty_like(acc_pkt)
        corr_pfb_remap(self.h, acc_pkt, acc_nat, stream)
        return acc_nat

    def beam(self, inp, out=None, stream=None):
        if out is None:
            out = torch.empty((self.n_chan, self.n_time), dtype=torch.int32, device=inp.device)
        _ptr(inp, self.n_inputs * self.n_chan * self.n_time, "input")
        _ptr(out, 4 * self.n_chan * self.n_time, "out")
        corr_beam(self.h, inp, out, stream)
        return out

    @property
    def samples(self) -> int:
        return corr_samples(self.h)


class FineFilterbank:
    """The F-engine stage: complex int8 coarse-channel samples [c][i][n] to the
    packed 4+4-bit TFI input of the X-engine (corr_fpfb)."""

    def __init__(self, n_inputs: int, n_coarse: int, n_frames: int):
        self.n_inputs, self.n_coarse, self.n_frames = n_inputs, n_coarse, n_frames
        self.h = corr_fpfb_create(n_inputs, n_coarse, n_frames)
        self._work = None

    def close(self) -> None:
        if self.h:
            corr_fpfb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_samples(self) -> int:
        """Complex input samples per (coarse channel, input)."""
        return 128 * (self.n_frames + 11)

    def tables(self):
        return corr_fpfb_tables(self.h)

    def run(self, inp, s1: int, s2: int, out=None, stream=None):
        dev = inp.device
        if self._work is None or self._work.device != dev:
            self._work = torch.empty(corr_fpfb_workspace_bytes(self.h), dtype=torch.uint8, device=dev)
        if out is None:
            out = torch.empty(self.n_frames * 128 * self.n_coarse * self.n_inputs, dtype=torch.uint8, device=dev)
        _ptr(inp, 2 * self.n_inputs * self.n_coarse * self.n_samples, "input")
        _ptr(out, self.n_frames * 128 * self.n_coarse * self.n_inputs, "out")
        corr_fpfb(self.h, inp, s1, s2, self._work, out, stream)
        return out


class Batch:
    """Arrays of uneven shapes correlated by one persistent launch."""

    def __init__(self, descs, engine: int = CORRX_ENGINE_AUTO, tile_cfg=None):
        self.descs = [tuple(d) for d in descs]
        self.h = corr_batch_create(self.descs, engine, tile_cfg)

    def close(self) -> None:
        if self.h:
            corr_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def items(self) -> int:
        return corr_batch_items(self.h)

    def plan(self, array: int) -> tuple[int, int]:
        return corr_batch_plan(self.h, array)

    def samples(self, array: int) -> int:
        return corr_batch_samples(self.h, array)

    def new_accs(self, device="cuda"):
        return [torch.zeros((f, n * (n + 1) // 2, 2), dtype=torch.int32, device=device)
                for (n, f, t, lay) in self.descs]

    def _check_accs(self, accs) -> None:
        if len(accs) != len(self.descs):
            raise ValueError(f"{len(accs)} accumulators for {len(self.descs)} arrays")
        for (n, f, t, lay), a in zip(self.descs, accs):
            _ptr(a, 8 * f * (n * (n + 1) // 2), "acc")

    def zero(self, accs, stream=None) -> None:
        self._check_accs(accs)
        corr_batch_zero(self.h, accs, stream)

    def xmac(self, ins, accs, stream=None) -> None:
        self._check_accs(accs)
        if len(ins) != len(self.descs):
            raise ValueError(f"{len(ins)} inputs for {len(self.descs)} arrays")
        for (n, f, t, lay), x in zip(self.descs, ins):
            _ptr(x, n * f * t, "input")
        corr_batch_xmac(self.h, ins, accs, stream)
