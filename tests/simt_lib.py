"""Driver for the CPU build of libaceseek (tests/simt): the library's own
kernels and host code, executed lane by lane on the host, with numpy arrays
standing in for device memory.  Test infrastructure only."""
import ctypes as C
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "simt"))

ARCH_PAD = 4096
ACE_E_ARG = -1
_lib = None


class Tuning(C.Structure):
    _fields_ = [(n, C.c_uint32) for n in ("waves_per_block", "blocks_per_wg", "lut_variant",
                                          "grid_wgs", "mode")]


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("SIMT_LIB")
        if not path:
            import build as simt_build
            path = simt_build.build()
        L = C.CDLL(path)
        vp, u64, u32 = C.c_void_p, C.c_uint64, C.c_uint32
        u64p, u32p = C.POINTER(C.c_uint64), C.POINTER(C.c_uint32)
        L.ace_last_error.restype = C.c_char_p
        L.ace_archive_open.argtypes = [vp, u64, vp, C.POINTER(vp)]
        L.ace_archive_close.argtypes = [vp]
        L.ace_archive_close.restype = None
        L.ace_archive_info.argtypes = [vp, u64p, u32p, u32p, u32p]
        L.ace_workspace_bytes.argtypes = [vp, vp, u32, u64p]
        L.ace_decode_all.argtypes = [vp, vp, u64, vp, u64, C.POINTER(Tuning), vp]
        L.ace_seek.argtypes = [vp, u64, u64, vp, vp, u64, C.POINTER(Tuning), vp]
        L.ace_seek_batch.argtypes = [vp, vp, u32, vp, vp, vp, u64, C.POINTER(Tuning), vp]
        L.ace_check.argtypes = [vp, vp]
        L.ace_read_counters.argtypes = [vp, vp, u64p]
        L.ace_batch_workspace_bytes.argtypes = [vp, u32, u64p]
        L.ace_batch_create.argtypes = [vp, u32, vp, u64, C.POINTER(Tuning), vp, C.POINTER(vp)]
        L.ace_batch_run.argtypes = [vp, vp, u32, vp, vp]
        L.ace_batch_destroy.argtypes = [vp]
        L.ace_batch_destroy.restype = None
        L.ace_plan_bytes.argtypes = [vp, u64p]
        L.ace_archive_attach_plan.argtypes = [vp, vp, u64, vp]
        L.ace_archive_open_ooc.argtypes = [vp, u64, C.POINTER(vp)]
        L.ace_seek_ooc_bytes.argtypes = [vp, u64, u64, u64p]
        L.ace_seek_ooc.argtypes = [vp, u64, u64, vp, vp, u64, C.POINTER(Tuning), vp]
        L.simt_stream_create.restype = vp
        _lib = L
    return _lib


class AceError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("aceseek (cpu build) error %d: %s" % (code, msg))
        self.code = code


def _check(rc):
    if rc:
        raise AceError(rc, lib().ace_last_error().decode(errors="replace"))


def _p(a):
    return C.c_void_p(a.ctypes.data)


class Archive:
    """An archive opened by the CPU build: host arrays play device memory."""

    def __init__(self, data: bytes):
        self.host = np.frombuffer(data, dtype=np.uint8)
        self.dev = np.zeros(len(data) + ARCH_PAD, dtype=np.uint8)
        self.dev[:len(data)] = self.host
        h = C.c_void_p()
        _check(lib().ace_archive_open(_p(self.host), len(data), _p(self.dev), C.byref(h)))
        self._h = h
        n, B, nb, depth = C.c_uint64(0), C.c_uint32(0), C.c_uint32(0), C.c_uint32(0)
        _check(lib().ace_archive_info(h, C.byref(n), C.byref(B), C.byref(nb), C.byref(depth)))
        self.n_total, self.block_size, self.n_blocks, self.depth = n.value, B.value, nb.value, depth.value

    def close(self):
        if self._h:
            lib().ace_archive_close(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, ranges=None):
        b = C.c_uint64(0)
        if ranges is None:
            _check(lib().ace_workspace_bytes(self._h, None, 0, C.byref(b)))
        else:
            r = np.ascontiguousarray(np.asarray(ranges, dtype=np.uint64).reshape(-1))
            _check(lib().ace_workspace_bytes(self._h, _p(r), len(r) // 2, C.byref(b)))
        return np.zeros(max(b.value, 256), dtype=np.uint8)

    def decode_all(self, tuning=None):
        out = np.zeros(max(self.n_total, 1), dtype=np.uint8)
        ws = self.workspace()
        t = C.byref(Tuning(**tuning)) if tuning else None
        _check(lib().ace_decode_all(self._h, _p(out), self.n_total, _p(ws), ws.size, t, None))
        _check(lib().ace_check(_p(ws), None))
        return out[:self.n_total].tobytes()

    def seek_device(self, lo, hi, tuning=None):
        """ace_seek planned on the device: the plan attached, and a workspace
        of the size that selects device planning."""
        L = lib()
        if getattr(self, "_plan", None) is None:
            b = C.c_uint64(0)
            _check(L.ace_plan_bytes(self._h, C.byref(b)))
            self._plan = np.zeros(max(b.value, 1), dtype=np.uint8)
            _check(L.ace_archive_attach_plan(self._h, _p(self._plan), b.value, None))
        b = C.c_uint64(0)
        _check(L.ace_batch_workspace_bytes(self._h, 1, C.byref(b)))
        out = np.zeros(max(hi - lo, 1), dtype=np.uint8)
        ws = np.zeros(b.value, dtype=np.uint8)
        t = C.byref(Tuning(**tuning)) if tuning else None
        _check(L.ace_seek(self._h, lo, hi, _p(out), _p(ws), ws.size, t, None))
        _check(L.ace_check(_p(ws), None))
        return out[:hi - lo].tobytes()

    def seek(self, lo, hi, tuning=None):
        out = np.zeros(max(hi - lo, 1), dtype=np.uint8)
        ws = self.workspace([lo, hi])
        t = C.byref(Tuning(**tuning)) if tuning else None
        _check(lib().ace_seek(self._h, lo, hi, _p(out), _p(ws), ws.size, t, None))
        _check(lib().ace_check(_p(ws), None))
        return out[:hi - lo].tobytes()


class OocArchive:
    """An archive opened out of core by the CPU build: only what each seek
    needs is staged into its workspace."""

    def __init__(self, data: bytes):
        self.host = np.frombuffer(data, dtype=np.uint8).copy()
        h = C.c_void_p()
        _check(lib().ace_archive_open_ooc(_p(self.host), len(data), C.byref(h)))
        self._h = h

    def close(self):
        if self._h:
            lib().ace_archive_close(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, lo, hi):
        b = C.c_uint64(0)
        _check(lib().ace_seek_ooc_bytes(self._h, lo, hi, C.byref(b)))
        return b.value

    def seek(self, lo, hi, tuning=None):
        out = np.zeros(max(hi - lo, 1), dtype=np.uint8)
        ws = np.zeros(max(self.workspace_bytes(lo, hi), 256), dtype=np.uint8)
        t = C.byref(Tuning(**tuning)) if tuning else None
        _check(lib().ace_seek_ooc(self._h, lo, hi, _p(out), _p(ws), ws.size, t, None))
        _check(lib().ace_check(_p(ws), None))
        return out[:hi - lo].tobytes()


def seek_batch_graph(arc, lo, hi, tuning=None):
    """The requests [lo_i, hi_i) through a captured batch graph (ace_batch_*),
    replayed twice; returns each request's bytes from the second replay."""
    L = lib()
    n = len(lo)
    b = C.c_uint64(0)
    _check(L.ace_batch_workspace_bytes(arc._h, n, C.byref(b)))
    ws = np.zeros(b.value, dtype=np.uint8)
    h = C.c_void_p()
    t = C.byref(Tuning(**tuning)) if tuning else None
    _check(L.ace_batch_create(arc._h, n, _p(ws), ws.size, t, C.c_void_p(L.simt_stream_create()), C.byref(h)))
    r = np.empty(2 * n, dtype=np.uint64)
    r[0::2], r[1::2] = lo, hi
    ln = (np.asarray(hi, dtype=np.int64) - np.asarray(lo, dtype=np.int64))
    offs = np.concatenate([[0], np.cumsum(ln)[:-1]]).astype(np.uint64)
    out = np.zeros(max(int(ln.sum()), 1), dtype=np.uint8)
    for _ in range(2):
        out[:] = 0
        _check(L.ace_batch_run(h, _p(r), n, _p(out), _p(offs)))
    _check(L.ace_check(_p(ws), None))
    L.ace_batch_destroy(h)
    return [out[int(o):int(o) + int(l)].tobytes() for o, l in zip(offs, ln)]


def decode_all_ext(arc, tuning=None):
    """Whole-archive decode; returns (bytes, the workspace's count of match
    bytes read from earlier blocks)."""
    L = lib()
    out = np.zeros(max(arc.n_total, 1), dtype=np.uint8)
    ws = arc.workspace()
    t = C.byref(Tuning(**tuning)) if tuning else None
    _check(L.ace_decode_all(arc._h, _p(out), arc.n_total, _p(ws), ws.size, t, None))
    _check(L.ace_check(_p(ws), None))
    ext = C.c_uint64(0)
    _check(L.ace_read_counters(_p(ws), None, C.byref(ext)))
    return out[:arc.n_total].tobytes(), ext.value
