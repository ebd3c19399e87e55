"""Python binding of libaceseek (argument marshalling only).

Every decode step runs in the library's HIP kernels; torch supplies device
memory and streams.  Entry points mirror include/aceseek.h.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libaceseek.so")

ARCH_PAD = 4096
OK, E_ARG, E_RANGE, E_CORRUPT, E_NOSPACE, E_HIP, E_TIMEOUT, E_NOMEM = 0, -1, -2, -3, -4, -5, -6, -7
# encoder flags beside the stream-mode policy (bits 0-1)
ENC_WIDE_OFFSETS, ENC_DEVICE_ENTROPY = 4, 8

EXPORTS = ["ace_last_error", "ace_encode_bound", "ace_encode_archive", "ace_archive_open",
           "ace_archive_close", "ace_archive_info", "ace_workspace_bytes", "ace_decode_all",
           "ace_seek", "ace_seek_batch", "ace_check", "ace_read_counters",
           "ace_batch_workspace_bytes", "ace_batch_create", "ace_batch_run", "ace_batch_destroy",
           "ace_batch_pin",
           "ace_set_timing", "ace_last_timings", "ace_plan_bytes", "ace_archive_attach_plan",
           "ace_set_block_trace", "ace_seek_static", "ace_last_host_times",
           "ace_workspace_bound", "ace_archive_open_ooc", "ace_seek_ooc_bytes", "ace_seek_ooc"]


class AceError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"aceseek error {code}: {msg}")
        self.code = code


class EncodeParams(C.Structure):
    _fields_ = [(n, C.c_uint32) for n in ("block_size", "interleave", "min_match", "hash_len",
                                          "max_chain", "max_level", "flags", "n_threads")]


class Range(C.Structure):
    _fields_ = [("lo", C.c_uint64), ("hi", C.c_uint64)]


class Tuning(C.Structure):
    _fields_ = [(n, C.c_uint32) for n in ("waves_per_block", "blocks_per_wg", "lut_variant",
                                          "grid_wgs", "mode")]


_lib = None


def library_path() -> str:
    return _LIB


def lib():
    """The loaded libaceseek; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise ImportError("libaceseek.so is not built (run __graft_entry__.build() or "
                              "python paper_2606_24531_amd/build.py)")
        L = C.CDLL(_LIB)
        vp, u64, u32 = C.c_void_p, C.c_uint64, C.c_uint32
        u64p, u32p = C.POINTER(C.c_uint64), C.POINTER(C.c_uint32)
        L.ace_last_error.restype = C.c_char_p
        L.ace_encode_bound.argtypes = [u64, C.POINTER(EncodeParams), u64p]
        L.ace_encode_archive.argtypes = [vp, u64, C.POINTER(EncodeParams), vp, u64, u64p]
        L.ace_archive_open.argtypes = [vp, u64, vp, C.POINTER(vp)]
        L.ace_archive_close.argtypes = [vp]
        L.ace_archive_close.restype = None
        L.ace_archive_info.argtypes = [vp, u64p, u32p, u32p, u32p]
        L.ace_workspace_bytes.argtypes = [vp, vp, u32, u64p]
        L.ace_workspace_bound.argtypes = [vp, u32, u64, u64p]
        L.ace_decode_all.argtypes = [vp, vp, u64, vp, u64, C.POINTER(Tuning), vp]
        L.ace_seek.argtypes = [vp, u64, u64, vp, vp, u64, C.POINTER(Tuning), vp]
        L.ace_seek_static.argtypes = [vp, u64, u64, vp, vp, C.POINTER(Tuning), vp]
        L.ace_seek_batch.argtypes = [vp, vp, u32, vp, vp, vp, u64, C.POINTER(Tuning), vp]
        L.ace_check.argtypes = [vp, vp]
        L.ace_read_counters.argtypes = [vp, vp, u64p]
        L.ace_batch_workspace_bytes.argtypes = [vp, u32, u64p]
        L.ace_batch_create.argtypes = [vp, u32, vp, u64, C.POINTER(Tuning), vp, C.POINTER(vp)]
        L.ace_batch_run.argtypes = [vp, vp, u32, vp, vp]
        L.ace_batch_pin.argtypes = [vp, u32]
        L.ace_batch_destroy.argtypes = [vp]
        L.ace_batch_destroy.restype = None
        L.ace_set_timing.argtypes = [C.c_int]
        L.ace_set_block_trace.argtypes = [vp, u64]
        L.ace_last_timings.argtypes = [C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.ace_last_host_times.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.ace_plan_bytes.argtypes = [vp, u64p]
        L.ace_archive_attach_plan.argtypes = [vp, vp, u64, vp]
        L.ace_archive_open_ooc.argtypes = [vp, u64, C.POINTER(vp)]
        L.ace_seek_ooc_bytes.argtypes = [vp, u64, u64, u64p]
        L.ace_seek_ooc.argtypes = [vp, u64, u64, vp, vp, u64, C.POINTER(Tuning), vp]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != OK:
        raise AceError(rc, lib().ace_last_error().decode(errors="replace"))


def _params(block_size=16384, interleave=32, min_match=20, hash_len=20, max_chain=32,
            max_level=0, flags=0, n_threads=0) -> EncodeParams:
    return EncodeParams(block_size, interleave, min_match, hash_len, max_chain, max_level,
                        flags, n_threads)


def encode_bound(n: int, **kw) -> int:
    p = _params(**kw)
    b = C.c_uint64(0)
    _check(lib().ace_encode_bound(n, C.byref(p), C.byref(b)))
    return b.value


def encode(x, **kw) -> bytes:
    """Host encoder of the library (multi-threaded parse); with
    flags | ENC_DEVICE_ENTROPY the rANS step runs on the current GPU (same
    archive bytes)."""
    p = _params(**kw)
    src = np.frombuffer(x, dtype=np.uint8) if not isinstance(x, np.ndarray) else x
    bound = encode_bound(len(src), **kw)
    out = np.empty(max(bound, 1), dtype=np.uint8)
    ln = C.c_uint64(0)
    rc = lib().ace_encode_archive(src.ctypes.data_as(C.c_void_p), len(src), C.byref(p),
                                  out.ctypes.data_as(C.c_void_p), out.size, C.byref(ln))
    if rc == E_NOSPACE:
        out = np.empty(ln.value, dtype=np.uint8)
        rc = lib().ace_encode_archive(src.ctypes.data_as(C.c_void_p), len(src), C.byref(p),
                                      out.ctypes.data_as(C.c_void_p), out.size, C.byref(ln))
    _check(rc)
    return out[:ln.value].tobytes()


def archive_facts(data) -> dict:
    """Sizes read from an archive's index: blocks, sequences, literal count,
    and the decoded token bytes (literals + 4-byte lengths + offsets)."""
    import struct
    b = bytes(data[:64]) if not isinstance(data, (bytes, bytearray)) else data
    nb = struct.unpack_from("<I", b, 24)[0]
    ow = b[15]
    arr = np.frombuffer(data, dtype=np.uint8)
    tbl = arr[64:64 + 32 * nb].view("<u4").reshape(nb, 8) if nb else np.zeros((0, 8), np.uint32)
    pay = tbl[:, 0].astype(np.uint64) | (tbl[:, 1].astype(np.uint64) << np.uint64(32))
    n_seq = tbl[:, 3].astype(np.int64)
    n_lit = np.array([int(np.frombuffer(arr[int(p) + 4:int(p) + 8].tobytes(), "<u4")[0])
                      for p in pay], dtype=np.int64) if nb else np.zeros(0, np.int64)
    return {"n_blocks": nb, "n_seq": int(n_seq.sum()), "n_lit": int(n_lit.sum()),
            "token_bytes": int(n_lit.sum() + (4 + ow) * n_seq.sum())}


def stream_table(data) -> dict:
    """Per-stream sizes summed over an archive's blocks (the paper's Table 2
    view): for LIT, LEN and OFF the decoded bytes, the stored bytes, the
    ratio raw/stored (< 1: the entropy coder inflated the stream) and the
    share of blocks that store the stream rANS-coded."""
    import struct
    arr = np.frombuffer(data, dtype=np.uint8)
    nb = struct.unpack_from("<I", bytes(arr[:64]), 24)[0]
    out = {}
    names = ("LIT", "LEN", "OFF")
    raw = np.zeros(3, np.int64)
    stored = np.zeros(3, np.int64)
    rans = np.zeros(3, np.int64)
    rans_raw = np.zeros(3, np.int64)
    rans_stored = np.zeros(3, np.int64)
    for b in range(nb):
        pay = int(arr[64 + 32 * b:64 + 32 * b + 8].view("<u8")[0])
        d = arr[pay:pay + 48].view("<u4").reshape(3, 4)
        for t in range(3):
            raw[t] += int(d[t, 1])
            stored[t] += int(d[t, 2])
            if int(d[t, 0] & 0xFF) == 1:
                rans[t] += 1
                rans_raw[t] += int(d[t, 1])
                rans_stored[t] += int(d[t, 2])
    for t, nm in enumerate(names):
        out[nm] = {"raw": int(raw[t]), "stored": int(stored[t]),
                   "ratio": round(float(raw[t]) / max(1, int(stored[t])), 4),
                   "rans_share": round(float(rans[t]) / max(1, nb), 4),
                   "rans_raw": int(rans_raw[t]), "rans_stored": int(rans_stored[t])}
    return out


def set_timing(on: bool):
    _check(lib().ace_set_timing(1 if on else 0))


def set_block_trace(trace=None):
    """Per-block clock trace of this thread's later decodes into `trace` (a
    device uint8/int64 tensor, 64 bytes per planned block); None turns it off."""
    if trace is None:
        _check(lib().ace_set_block_trace(None, 0))
    else:
        _check(lib().ace_set_block_trace(C.c_void_p(trace.data_ptr()),
                                         trace.numel() * trace.element_size()))


def last_timings():
    """(entropy ms, match ms) of the last timed decode on this thread."""
    a, b = C.c_float(0), C.c_float(0)
    _check(lib().ace_last_timings(C.byref(a), C.byref(b)))
    return a.value, b.value


def last_host_times():
    """(planning us, enqueue us) of the last timed decode on this thread."""
    a, b = C.c_double(0), C.c_double(0)
    _check(lib().ace_last_host_times(C.byref(a), C.byref(b)))
    return a.value, b.value


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Archive:
    """A compressed archive resident in HBM, with a reusable workspace."""

    def __init__(self, data, device="cuda", resident_plan=True):
        import torch
        self._torch = torch
        host = np.frombuffer(data, dtype=np.uint8) if not isinstance(data, np.ndarray) else data
        self.nbytes = int(host.size)
        self.device = torch.device(device)
        d = torch.zeros(self.nbytes + ARCH_PAD, dtype=torch.uint8, device=self.device)
        if self.nbytes:
            d[:self.nbytes].copy_(torch.from_numpy(np.array(host, dtype=np.uint8, copy=True)))
        self.d_arch = d
        h = C.c_void_p()
        _check(lib().ace_archive_open(host.ctypes.data_as(C.c_void_p), self.nbytes,
                                      C.c_void_p(d.data_ptr()), C.byref(h)))
        self._h = h
        n, B, nb, depth = C.c_uint64(0), C.c_uint32(0), C.c_uint32(0), C.c_uint32(0)
        _check(lib().ace_archive_info(h, C.byref(n), C.byref(B), C.byref(nb), C.byref(depth)))
        self.n_total, self.block_size, self.n_blocks, self.depth = n.value, B.value, nb.value, depth.value
        self.interleave = int(host[12]) | (int(host[13]) << 8) if self.nbytes >= 64 else 0
        self._ws = None
        # the whole-archive decode plan, resident next to the archive (else
        # it is copied from the host on every whole-archive decode)
        self.d_plan = None
        if resident_plan:
            pb = C.c_uint64(0)
            _check(lib().ace_plan_bytes(h, C.byref(pb)))
            self.d_plan = torch.empty(max(pb.value, 1), dtype=torch.uint8, device=self.device)
            _check(lib().ace_archive_attach_plan(h, C.c_void_p(self.d_plan.data_ptr()), pb.value,
                                                 _stream_ptr(torch.cuda.current_stream(self.device))))

    def close(self):
        if getattr(self, "_h", None):
            lib().ace_archive_close(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- workspace
    def workspace_bytes(self, ranges=None) -> int:
        b = C.c_uint64(0)
        if ranges is None:
            _check(lib().ace_workspace_bytes(self._h, None, 0, C.byref(b)))
        else:
            r = self._ranges(ranges)
            _check(lib().ace_workspace_bytes(self._h, r.ctypes.data_as(C.c_void_p), len(r) // 2,
                                             C.byref(b)))
        return b.value

    def workspace_bound(self, n_ranges: int, total_bytes: int) -> int:
        """Workspace bytes that suffice for any seek_batch of at most n_ranges
        ranges of at most total_bytes bytes in all."""
        b = C.c_uint64(0)
        _check(lib().ace_workspace_bound(self._h, int(n_ranges), int(total_bytes), C.byref(b)))
        return b.value

    def workspace(self, nbytes: int):
        """A zero-initialised device workspace of at least nbytes (reused)."""
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = self._torch.zeros(max(nbytes, 256), dtype=self._torch.uint8,
                                         device=self.device)
        return self._ws

    @staticmethod
    def _ranges(ranges):
        if isinstance(ranges, tuple) and len(ranges) == 2 and hasattr(ranges[0], "__len__"):
            lo, hi = ranges
            r = np.empty(2 * len(lo), dtype=np.uint64)
            r[0::2] = lo
            r[1::2] = hi
            return r
        r = np.asarray(ranges, dtype=np.uint64).reshape(-1)
        return np.ascontiguousarray(r)

    @staticmethod
    def _tuning(t):
        if t is None:
            return None
        if isinstance(t, Tuning):
            return C.byref(t)
        return C.byref(Tuning(**t))

    # -- decode
    def decode_all(self, out=None, ws=None, tuning=None, stream=None):
        torch = self._torch
        if out is None:
            out = torch.empty(self.n_total, dtype=torch.uint8, device=self.device)
        if ws is None:
            ws = self.workspace(self.workspace_bytes())
        _check(lib().ace_decode_all(self._h, C.c_void_p(out.data_ptr()), out.numel(),
                                    C.c_void_p(ws.data_ptr()), ws.numel(), self._tuning(tuning),
                                    _stream_ptr(stream)))
        return out

    def seek_device_bytes(self) -> int:
        """Workspace bytes with which ace_seek plans on the device (the
        archive's plan is attached by default)."""
        b = C.c_uint64(0)
        _check(lib().ace_batch_workspace_bytes(self._h, 1, C.byref(b)))
        return b.value

    def seek(self, lo: int, hi: int, out=None, ws=None, tuning=None, stream=None, plan: str = "auto"):
        """[lo, hi) as a device tensor.  plan: "host" walks the closure on the
        host (the workspace capacity passed is the host plan's need), "device"
        plans on the device (needs the resident plan), "auto" lets the
        library choose by the workspace's size."""
        torch = self._torch
        if out is None:
            out = torch.empty(max(hi - lo, 0), dtype=torch.uint8, device=self.device)
        host_need = self.workspace_bytes([lo, hi]) if hi > lo else 256
        if plan == "device":
            if self.d_plan is None:
                raise AceError(E_ARG, "device planning needs the resident plan")
            need = self.seek_device_bytes()
        else:
            need = host_need
        if ws is None:
            ws = self.workspace(need)
        cap = ws.numel()
        if plan == "host":
            cap = min(cap, host_need)
        elif plan == "device" and cap < need:
            raise AceError(E_NOSPACE, "device planning needs a %d-byte workspace" % need)
        _check(lib().ace_seek(self._h, lo, hi, C.c_void_p(out.data_ptr()),
                              C.c_void_p(ws.data_ptr()), cap, self._tuning(tuning),
                              _stream_ptr(stream)))
        return out

    def seek_static(self, lo: int, hi: int, out, status, tuning=None, stream=None):
        """ace_seek_static: the seek with the library's fixed device scratch as
        its workspace (allocates nothing); status (a device int32/uint8 tensor
        of at least 4 bytes) receives the device error word."""
        _check(lib().ace_seek_static(self._h, lo, hi, C.c_void_p(out.data_ptr()),
                                     C.c_void_p(status.data_ptr()), self._tuning(tuning),
                                     _stream_ptr(stream)))
        return out

    def seek_batch(self, ranges, out=None, out_offsets=None, ws=None, tuning=None, stream=None):
        """ranges: (lo array, hi array) or a flat [lo0, hi0, lo1, hi1, ...]."""
        torch = self._torch
        r = self._ranges(ranges)
        n = len(r) // 2
        lens = r[1::2].astype(np.int64) - r[0::2].astype(np.int64)
        if out_offsets is None:
            out_offsets = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.uint64)
        offs = np.ascontiguousarray(out_offsets, dtype=np.uint64)
        if out is None:
            total = int(lens.sum()) if n else 0
            out = torch.empty(max(total, 1), dtype=torch.uint8, device=self.device)
        if ws is None:
            ws = self.workspace(self.workspace_bytes(r))
        _check(lib().ace_seek_batch(self._h, r.ctypes.data_as(C.c_void_p), n,
                                    C.c_void_p(out.data_ptr()), offs.ctypes.data_as(C.c_void_p),
                                    C.c_void_p(ws.data_ptr()), ws.numel(), self._tuning(tuning),
                                    _stream_ptr(stream)))
        return out

    def batch(self, max_requests: int, tuning=None, stream=None):
        """A graph-replayed batched-seek context with its own workspace."""
        return Batch(self, max_requests, tuning, stream)

    def read_counters(self, ws=None, stream=None) -> dict:
        """Synchronises, returns and clears the workspace counters."""
        ws = self._ws if ws is None else ws
        v = C.c_uint64(0)
        _check(lib().ace_read_counters(C.c_void_p(ws.data_ptr()), _stream_ptr(stream),
                                       C.byref(v)))
        return {"ext_src_bytes": v.value}

    def check(self, ws=None, stream=None):
        """Synchronises and raises if the device flagged a corrupt stream."""
        ws = self._ws if ws is None else ws
        if ws is None:
            return
        _check(lib().ace_check(C.c_void_p(ws.data_ptr()), _stream_ptr(stream)))


class OutOfCoreArchive:
    """An archive kept in host memory (ace_archive_open_ooc): each seek
    copies only its dependency closure's payloads to the device."""

    def __init__(self, data, device="cuda"):
        import torch
        self._torch = torch
        host = np.frombuffer(data, dtype=np.uint8) if not isinstance(data, np.ndarray) else data
        self._host = np.ascontiguousarray(host)  # the library reads it on every seek
        self.nbytes = int(self._host.size)
        self.device = torch.device(device)
        h = C.c_void_p()
        _check(lib().ace_archive_open_ooc(self._host.ctypes.data_as(C.c_void_p), self.nbytes, C.byref(h)))
        self._h = h
        n, B, nb, depth = C.c_uint64(0), C.c_uint32(0), C.c_uint32(0), C.c_uint32(0)
        _check(lib().ace_archive_info(h, C.byref(n), C.byref(B), C.byref(nb), C.byref(depth)))
        self.n_total, self.block_size, self.n_blocks, self.depth = n.value, B.value, nb.value, depth.value
        self._ws = None

    def close(self):
        if getattr(self, "_h", None):
            lib().ace_archive_close(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, lo: int, hi: int) -> int:
        b = C.c_uint64(0)
        _check(lib().ace_seek_ooc_bytes(self._h, int(lo), int(hi), C.byref(b)))
        return b.value

    def seek(self, lo: int, hi: int, out=None, ws=None, tuning=None, stream=None):
        """[lo, hi) as a device tensor; returns when the seek has finished."""
        torch = self._torch
        if out is None:
            out = torch.empty(max(hi - lo, 0), dtype=torch.uint8, device=self.device)
        if ws is None:
            need = self.workspace_bytes(lo, hi)
            if self._ws is None or self._ws.numel() < need:
                self._ws = torch.zeros(max(need, 256), dtype=torch.uint8, device=self.device)
            ws = self._ws
        _check(lib().ace_seek_ooc(self._h, int(lo), int(hi), C.c_void_p(out.data_ptr()),
                                  C.c_void_p(ws.data_ptr()), ws.numel(), Archive._tuning(tuning),
                                  _stream_ptr(stream)))
        self._last_ws = ws
        return out

    def check(self, ws=None, stream=None):
        """Raises if the device flagged a corrupt stream in the last seek."""
        ws = getattr(self, "_last_ws", None) if ws is None else ws
        if ws is None:
            return
        _check(lib().ace_check(C.c_void_p(ws.data_ptr()), _stream_ptr(stream)))


class Batch:
    """Batched seek replayed as one captured HIP graph (see ace_batch_create)."""

    def __init__(self, arc: Archive, max_requests: int, tuning=None, stream=None):
        torch = arc._torch
        self.arc = arc
        self.cap = int(max_requests)
        # graph capture needs a stream of its own (not the legacy default stream)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=arc.device)
        b = C.c_uint64(0)
        _check(lib().ace_batch_workspace_bytes(arc._h, self.cap, C.byref(b)))
        self.ws = torch.zeros(b.value, dtype=torch.uint8, device=arc.device)
        h = C.c_void_p()
        _check(lib().ace_batch_create(arc._h, self.cap, C.c_void_p(self.ws.data_ptr()), b.value,
                                      arc._tuning(tuning), _stream_ptr(self.stream), C.byref(h)))
        self._h = h

    def run(self, ranges, out, out_offsets=None):
        r = Archive._ranges(ranges)
        n = len(r) // 2
        if out_offsets is None:
            lens = r[1::2].astype(np.int64) - r[0::2].astype(np.int64)
            out_offsets = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.uint64)
        offs = np.ascontiguousarray(out_offsets, dtype=np.uint64)
        torch = self.arc._torch
        cur = torch.cuda.current_stream(self.arc.device)
        self.stream.wait_stream(cur)  # `out` was made on the caller's stream
        _check(lib().ace_batch_run(self._h, r.ctypes.data_as(C.c_void_p), n,
                                   C.c_void_p(out.data_ptr()), offs.ctypes.data_as(C.c_void_p)))
        cur.wait_stream(self.stream)  # later work on the caller's stream sees the bytes
        return out

    def pin(self, levels: int):
        """Decodes dependency levels [0, levels) once and keeps them for every
        later run (see ace_batch_pin)."""
        torch = self.arc._torch
        self.stream.wait_stream(torch.cuda.current_stream(self.arc.device))
        _check(lib().ace_batch_pin(self._h, int(levels)))

    def check(self):
        _check(lib().ace_check(C.c_void_p(self.ws.data_ptr()), _stream_ptr(self.stream)))

    def close(self):
        if getattr(self, "_h", None):
            lib().ace_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
