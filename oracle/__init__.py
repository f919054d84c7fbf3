"""CPU oracle for the X-engine -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The GPU library never calls it and shares no code
with it.

``oracle.c`` holds the plain int64 triple loop (lower triangle of
V_f = sum_t x(t) x(t)^H per channel, Sec. 2 eq. (3) with the conjugate read on
the second factor, Appendix C "GPU Output" for the packed triangle).  This
module builds and loads it with gcc, and adds the output orderings of
Appendix C as direct numpy index definitions.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc -O2 -fopenmp into liboracle.so (in place)."""
    global _lib
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
                        "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        for name in ("oracle_xmac", "oracle_xmac_full", "oracle_incoherent_beam"):
            fn = getattr(L, name)
            fn.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, i64p]
            fn.restype = ctypes.c_int
        L.oracle_decode.argtypes = [ctypes.c_uint8, i32p, i32p]
        L.oracle_decode.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        L.oracle_get_threads.argtypes = []
        L.oracle_get_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def n_baselines(n_inputs: int) -> int:
    return n_inputs * (n_inputs + 1) // 2


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(lib().oracle_get_threads())


def decode(byte: int) -> tuple[int, int, bool]:
    re = ctypes.c_int32()
    im = ctypes.c_int32()
    ok = lib().oracle_decode(ctypes.c_uint8(byte), ctypes.byref(re), ctypes.byref(im))
    return re.value, im.value, bool(ok)


def _u8(buf: np.ndarray):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    return buf, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def xmac(buf: np.ndarray, n_inputs: int, n_chan: int, n_time: int, layout: int = 0) -> np.ndarray:
    """Lower-triangle visibilities, int64 array of shape (n_chan, N(N+1)/2, 2)."""
    buf, p = _u8(buf)
    if buf.size != n_inputs * n_chan * n_time:
        raise ValueError("input size does not match the shape")
    out = np.empty((n_chan, n_baselines(n_inputs), 2), dtype=np.int64)
    rc = lib().oracle_xmac(p, n_inputs, n_chan, n_time, layout,
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc:
        raise RuntimeError(f"oracle_xmac failed ({rc})")
    return out


def xmac_full(buf: np.ndarray, n_inputs: int, n_chan: int, n_time: int, layout: int = 0) -> np.ndarray:
    """Every ordered pair, int64 array of shape (n_chan, N, N, 2)."""
    buf, p = _u8(buf)
    if buf.size != n_inputs * n_chan * n_time:
        raise ValueError("input size does not match the shape")
    out = np.empty((n_chan, n_inputs, n_inputs, 2), dtype=np.int64)
    rc = lib().oracle_xmac_full(p, n_inputs, n_chan, n_time, layout,
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc:
        raise RuntimeError(f"oracle_xmac_full failed ({rc})")
    return out


def incoherent_beam(buf: np.ndarray, n_inputs: int, n_chan: int, n_time: int, layout: int = 0) -> np.ndarray:
    """Per channel and sample, sum_i |x_i|^2; int64 array (n_chan, n_time)."""
    buf, p = _u8(buf)
    out = np.empty((n_chan, n_time), dtype=np.int64)
    rc = lib().oracle_incoherent_beam(p, n_inputs, n_chan, n_time, layout,
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc:
        raise RuntimeError(f"oracle_incoherent_beam failed ({rc})")
    return out


def tri_to_full(tri: np.ndarray, n_inputs: int) -> np.ndarray:
    """Complex (n_chan, N, N) matrix from a lower triangle, using V_ji = conj(V_ij)."""
    n_chan = tri.shape[0]
    v = tri[..., 0].astype(np.complex128) + 1j * tri[..., 1].astype(np.complex128)
    full = np.zeros((n_chan, n_inputs, n_inputs), dtype=np.complex128)
    ii, jj = np.tril_indices(n_inputs)
    b = ii * (ii + 1) // 2 + jj
    full[:, ii, jj] = v[:, b]
    full[:, jj, ii] = np.conj(v[:, b])
    return full


def station_pol(tri: np.ndarray, n_inputs: int) -> np.ndarray:
    """Appendix C "GPU Output" order: channel, station s1, station s2 <= s1,
    polarisation p1, polarisation p2, re/im.  Input index i = 2*s + p.

    Returns int64 (n_chan, S(S+1)/2, 2, 2, 2).  Within a station pair, the
    element V[2*s1+p1][2*s2+p2] lies in the upper triangle only for s1 == s2,
    p1 = 0, p2 = 1; it is the conjugate of V[2*s1+1][2*s1].
    """
    if n_inputs % 2:
        raise ValueError("station/polarisation order needs an even input count")
    n_st = n_inputs // 2
    out = np.empty((tri.shape[0], n_baselines(n_st), 2, 2, 2), dtype=np.int64)
    for s1 in range(n_st):
        for s2 in range(s1 + 1):
            bs = s1 * (s1 + 1) // 2 + s2
            for p1 in range(2):
                for p2 in range(2):
                    i, j = 2 * s1 + p1, 2 * s2 + p2
                    if i >= j:
                        b = i * (i + 1) // 2 + j
                        out[:, bs, p1, p2, 0] = tri[:, b, 0]
                        out[:, bs, p1, p2, 1] = tri[:, b, 1]
                    else:
                        b = j * (j + 1) // 2 + i
                        out[:, bs, p1, p2, 0] = tri[:, b, 0]
                        out[:, bs, p1, p2, 1] = -tri[:, b, 1]
    return out
