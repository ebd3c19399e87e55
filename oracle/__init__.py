"""ctypes binding of the plain CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It shares no code with the GPU library;
both read the same archive byte format and nothing else.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["common.c", "ans.c", "encode.c", "decode.c"]

OK, E_ARG, E_RANGE, E_CORRUPT, E_NOSPACE, E_NOMEM = 0, -1, -2, -3, -4, -7
MODE_AUTO, MODE_RANS, MODE_RAW = 0, 1, 2
WIDE_OFFSETS = 4  # flags bit: 8-byte offsets at any size


CFLAGS = ["-O2", "-std=c11", "-Wall", "-Wextra", "-fopenmp", "-shared", "-fPIC"]


def build(force: bool = False) -> str:
    """Compiles liboracle.so from the C sources beside this file."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    if not force and os.path.exists(_LIB_PATH):
        t = os.path.getmtime(_LIB_PATH)
        if all(os.path.getmtime(s) <= t for s in srcs + [os.path.join(_HERE, "oracle.h"),
                                                         os.path.join(_HERE, "internal.h")]):
            return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc"] + CFLAGS + ["-o", tmp] + srcs)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class OracleError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [(n, C.c_uint32) for n in ("block_size", "interleave", "min_match", "hash_len",
                                          "max_chain", "max_level", "flags")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        u8p, u16p, u32p, u64p = (C.POINTER(C.c_uint8), C.POINTER(C.c_uint16),
                                 C.POINTER(C.c_uint32), C.POINTER(C.c_uint64))
        L.orc_last_error.restype = C.c_char_p
        L.orc_fnv1a64.restype = C.c_uint64
        L.orc_fnv1a64.argtypes = [C.c_void_p, C.c_uint64]
        L.orc_normalize.argtypes = [u64p, u16p]
        L.orc_rans_encode.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, u16p, C.c_void_p,
                                      C.c_uint32, u32p]
        L.orc_rans_decode.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, u16p,
                                      C.c_void_p]
        L.orc_encode_bound.argtypes = [C.c_uint64, C.POINTER(Params), u64p]
        L.orc_encode.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(Params), C.c_void_p,
                                 C.c_uint64, u64p]
        L.orc_assemble.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                   u32p, u32p, u32p, u64p, C.c_void_p, C.c_uint64, u64p]
        L.orc_info.argtypes = [C.c_void_p, C.c_uint64, u64p, u32p, u32p, u32p, u32p]
        L.orc_decode.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64]
        L.orc_decode_levels.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, C.c_int,
                                        C.POINTER(C.c_int)]
        L.orc_seek.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint64, C.c_void_p]
        L.orc_closure.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint64, C.c_void_p,
                                  u32p]
        L.orc_block_facts.argtypes = [C.c_void_p, C.c_uint64, u32p, u32p, C.c_void_p]
        L.orc_block_tokens.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_void_p, u32p,
                                       u32p, u32p, u64p, u32p]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != OK:
        raise OracleError(rc, lib().orc_last_error().decode(errors="replace"))


def _buf(b):
    """(pointer, keepalive) for a bytes-like or numpy array."""
    a = np.frombuffer(b, dtype=np.uint8) if not isinstance(b, np.ndarray) else b
    return a.ctypes.data_as(C.c_void_p), a


def fnv1a64(b) -> int:
    p, keep = _buf(b)
    return int(lib().orc_fnv1a64(p, len(keep)))


def params(block_size=16384, interleave=32, min_match=20, hash_len=20, max_chain=32,
           max_level=0, flags=MODE_AUTO) -> Params:
    return Params(block_size, interleave, min_match, hash_len, max_chain, max_level, flags)


def normalize(counts) -> np.ndarray:
    c = np.ascontiguousarray(counts, dtype=np.uint64)
    assert c.size == 256
    f = np.zeros(256, dtype=np.uint16)
    _check(lib().orc_normalize(c.ctypes.data_as(C.POINTER(C.c_uint64)),
                               f.ctypes.data_as(C.POINTER(C.c_uint16))))
    return f


def rans_encode(sym, W: int, freq) -> bytes:
    s = np.ascontiguousarray(np.frombuffer(bytes(sym), dtype=np.uint8))
    f = np.ascontiguousarray(freq, dtype=np.uint16)
    cap = 4 * W + 2 * len(s) + 16
    out = np.zeros(cap, dtype=np.uint8)
    n = C.c_uint32(0)
    _check(lib().orc_rans_encode(s.ctypes.data_as(C.c_void_p), len(s), W,
                                 f.ctypes.data_as(C.POINTER(C.c_uint16)),
                                 out.ctypes.data_as(C.c_void_p), cap, C.byref(n)))
    return out[:n.value].tobytes()


def rans_decode(data: bytes, n: int, W: int, freq) -> bytes:
    d = np.frombuffer(bytes(data) if data else b"\0", dtype=np.uint8)
    f = np.ascontiguousarray(freq, dtype=np.uint16)
    out = np.zeros(max(n, 1), dtype=np.uint8)
    _check(lib().orc_rans_decode(d.ctypes.data_as(C.c_void_p), len(data), n, W,
                                 f.ctypes.data_as(C.POINTER(C.c_uint16)),
                                 out.ctypes.data_as(C.c_void_p)))
    return out[:n].tobytes()


def encode(x: bytes, **kw) -> bytes:
    p = params(**kw)
    src, keep = _buf(x)
    bound = C.c_uint64(0)
    _check(lib().orc_encode_bound(len(keep), C.byref(p), C.byref(bound)))
    out = np.empty(max(bound.value, 1), dtype=np.uint8)
    ln = C.c_uint64(0)
    rc = lib().orc_encode(src, len(keep), C.byref(p), out.ctypes.data_as(C.c_void_p),
                          out.size, C.byref(ln))
    if rc == E_NOSPACE:
        out = np.empty(ln.value, dtype=np.uint8)
        rc = lib().orc_encode(src, len(keep), C.byref(p), out.ctypes.data_as(C.c_void_p),
                              out.size, C.byref(ln))
    _check(rc)
    return out[:ln.value].tobytes()


def assemble(x: bytes, block_size: int, interleave: int, seq_count, L, M, O,
             flags: int = MODE_AUTO) -> bytes:
    src, keep = _buf(x)
    sc = np.ascontiguousarray(seq_count, dtype=np.uint32)
    La = np.ascontiguousarray(L, dtype=np.uint32)
    Ma = np.ascontiguousarray(M, dtype=np.uint32)
    Oa = np.ascontiguousarray(O, dtype=np.uint64)
    u32p, u64p = C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)
    ln = C.c_uint64(0)
    rc = lib().orc_assemble(src, len(keep), block_size, interleave, flags,
                            sc.ctypes.data_as(u32p), La.ctypes.data_as(u32p),
                            Ma.ctypes.data_as(u32p), Oa.ctypes.data_as(u64p), None, 0,
                            C.byref(ln))
    if rc != E_NOSPACE:
        _check(rc)
    out = np.empty(max(ln.value, 1), dtype=np.uint8)
    _check(lib().orc_assemble(src, len(keep), block_size, interleave, flags,
                              sc.ctypes.data_as(u32p), La.ctypes.data_as(u32p),
                              Ma.ctypes.data_as(u32p), Oa.ctypes.data_as(u64p),
                              out.ctypes.data_as(C.c_void_p), out.size, C.byref(ln)))
    return out[:ln.value].tobytes()


def info(a: bytes) -> dict:
    p, keep = _buf(a)
    n = C.c_uint64(0)
    B, nb, depth, W = C.c_uint32(0), C.c_uint32(0), C.c_uint32(0), C.c_uint32(0)
    _check(lib().orc_info(p, len(keep), C.byref(n), C.byref(B), C.byref(nb), C.byref(depth),
                          C.byref(W)))
    return dict(n_total=n.value, block_size=B.value, n_blocks=nb.value, depth=depth.value,
                interleave=W.value)


def decode(a: bytes) -> bytes:
    p, keep = _buf(a)
    n = info(a)["n_total"]
    out = np.empty(max(n, 1), dtype=np.uint8)
    _check(lib().orc_decode(p, len(keep), out.ctypes.data_as(C.c_void_p), n))
    return out[:n].tobytes()


def decode_levels(a: bytes, threads: int = 0):
    """Decode with each dependency level's blocks in parallel on `threads`
    host threads (0 = all).  Returns (bytes, threads used)."""
    p, keep = _buf(a)
    n = info(a)["n_total"]
    out = np.empty(max(n, 1), dtype=np.uint8)
    used = C.c_int(0)
    _check(lib().orc_decode_levels(p, len(keep), out.ctypes.data_as(C.c_void_p), n, int(threads),
                                   C.byref(used)))
    return out[:n].tobytes(), used.value


def decode_rc(a: bytes) -> int:
    """Return code of a full decode (for corruption tests); never raises."""
    p, keep = _buf(a)
    n = C.c_uint64(0)
    B, nb, depth, W = C.c_uint32(0), C.c_uint32(0), C.c_uint32(0), C.c_uint32(0)
    rc = lib().orc_info(p, len(keep), C.byref(n), C.byref(B), C.byref(nb), C.byref(depth),
                        C.byref(W))
    if rc:
        return rc
    if n.value > (1 << 31):
        return E_CORRUPT
    out = np.empty(max(n.value, 1), dtype=np.uint8)
    return lib().orc_decode(p, len(keep), out.ctypes.data_as(C.c_void_p), n.value)


def seek(a: bytes, lo: int, hi: int) -> bytes:
    p, keep = _buf(a)
    out = np.empty(max(hi - lo, 1), dtype=np.uint8)
    _check(lib().orc_seek(p, len(keep), lo, hi, out.ctypes.data_as(C.c_void_p)))
    return out[:hi - lo].tobytes()


def closure(a: bytes, lo: int, hi: int) -> np.ndarray:
    p, keep = _buf(a)
    nb = info(a)["n_blocks"]
    need = np.zeros(max(nb, 1), dtype=np.uint8)
    cnt = C.c_uint32(0)
    _check(lib().orc_closure(p, len(keep), lo, hi, need.ctypes.data_as(C.c_void_p),
                             C.byref(cnt)))
    return np.nonzero(need[:nb])[0].astype(np.uint32)


def block_facts(a: bytes):
    p, keep = _buf(a)
    nb = info(a)["n_blocks"]
    level = np.zeros(max(nb, 1), dtype=np.uint32)
    nseq = np.zeros(max(nb, 1), dtype=np.uint32)
    modes = np.zeros(max(3 * nb, 1), dtype=np.uint8)
    u32p = C.POINTER(C.c_uint32)
    _check(lib().orc_block_facts(p, len(keep), level.ctypes.data_as(u32p),
                                 nseq.ctypes.data_as(u32p), modes.ctypes.data_as(C.c_void_p)))
    return level[:nb], nseq[:nb], modes[:3 * nb].reshape(nb, 3)


def block_tokens(a: bytes, block: int):
    """(literals, L, M, O) of one block after the entropy layer."""
    p, keep = _buf(a)
    B = info(a)["block_size"]
    lit = np.zeros(B, dtype=np.uint8)
    Ls = np.zeros(B, dtype=np.uint32)
    Ms = np.zeros(B, dtype=np.uint32)
    Os = np.zeros(B, dtype=np.uint64)
    nl, ns = C.c_uint32(0), C.c_uint32(0)
    u32p, u64p = C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)
    _check(lib().orc_block_tokens(p, len(keep), block, lit.ctypes.data_as(C.c_void_p),
                                  C.byref(nl), Ls.ctypes.data_as(u32p), Ms.ctypes.data_as(u32p),
                                  Os.ctypes.data_as(u64p), C.byref(ns)))
    k = ns.value
    return lit[:nl.value].tobytes(), Ls[:k].copy(), Ms[:k].copy(), Os[:k].copy()
