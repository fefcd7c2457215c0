"""ctypes binding of libdisthist (argument marshalling only).

Every computation runs in the library's HIP kernels. PyTorch is used only to
hold device buffers and to name streams. If the compiled library is missing
this module raises ImportError at import time: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

BOX_NONE, BOX_ORTHO, BOX_TRICLINIC = 0, 1, 2
FP32, FP64 = 0, 1
DH_OK, DH_EINVAL, DH_ENOMEM, DH_EDEVICE, DH_EBUDGET, DH_EUNSUPPORTED = 0, -1, -2, -3, -4, -5

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdisthist.so")

# Every symbol declared in include/disthist.h, with its ctypes signature.
_vp, _i32, _i64, _f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
SIGNATURES = {
    "dh_version": ([], ctypes.c_char_p),
    "dh_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "dh_check_args": ([_vp, _vp, _i32, _i32, _vp, _f64, _i32, _i32], ctypes.c_int),
    "dh_histo": ([_vp, _vp, _i32, _i32, _vp, _f64, _i32, _i32, _vp], ctypes.c_int),
    "dh_ctx_create": ([_i32, _i64, ctypes.POINTER(_vp)], ctypes.c_int),
    "dh_ctx_destroy": ([_vp], None),
    "dh_ctx_last_error": ([_vp], ctypes.c_char_p),
    "dh_histo_async": ([_vp, _vp, _vp, _vp, _i32, _i32, _vp, _f64, _i32, _i32, _vp, _vp],
                       ctypes.c_int),
    "dh_pair_t_async": ([_vp, _vp, _vp, _i64, _i32, _vp, _f64, _i32, _i32, _vp, _vp, _i64, _vp],
                        ctypes.c_int),
    "dh_histo_noalloc": ([_vp, _vp, _vp, _i32, _i32, _vp, _f64, _i32, _i32, _vp, _vp],
                         ctypes.c_int),
    "dh_batch_create": ([_vp, _vp, _i32, _i32, _i32, ctypes.POINTER(_vp)], ctypes.c_int),
    "dh_batch_launch": ([_vp, _vp], ctypes.c_int),
    "dh_batch_info": ([_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i32), ctypes.POINTER(_f64)],
                      ctypes.c_int),
    "dh_batch_destroy": ([_vp], None),
    "dh_server_create": ([_i32, _i64, _i32, _f64, ctypes.POINTER(_vp)], ctypes.c_int),
    "dh_server_submit": ([_vp, _vp, _vp, _i32, _i32, _vp, _f64, _i32, _i32, ctypes.POINTER(_i64)],
                         ctypes.c_int),
    "dh_server_status": ([_vp, _i64], ctypes.c_int),
    "dh_server_set_policy": ([_vp, _i32], ctypes.c_int),
    "dh_server_wait": ([_vp, _i64, _vp, _vp, _vp], ctypes.c_int),
    "dh_server_stats": ([_vp, _vp], ctypes.c_int),
    "dh_server_launch_stats": ([_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                                ctypes.POINTER(_i64)], ctypes.c_int),
    "dh_server_destroy": ([_vp], None),
    "dh_sched_select": ([_vp, _vp, _vp, _i32, _i64, _i32, _f64, _vp], ctypes.c_int32),
    "dh_cpu_histo": ([_vp, _vp, _i32, _i32, _vp, _f64, _i32, _i32, _i32, _vp, _vp], ctypes.c_int),
    "dh_traj_open": ([ctypes.c_char_p, ctypes.POINTER(_vp)], ctypes.c_int),
    "dh_traj_info": ([_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i32)],
                     ctypes.c_int),
    "dh_traj_close": ([_vp], None),
    "dh_traj_histo": ([_vp, _vp, _vp, _i32, _f64, _i32, _i32, _i64, _i64, _i64, ctypes.c_char_p,
                       _i64, ctypes.POINTER(_i64)], ctypes.c_int),
    "dh_traj_histo_hybrid": ([_vp, _vp, _vp, _i32, _f64, _i32, _i32, _i64, _i64, _i64,
                              ctypes.c_char_p, _i64, _i32, _i32, ctypes.POINTER(_i64),
                              ctypes.POINTER(_i64)], ctypes.c_int),
    "dh_ctx_set_tuning": ([_vp, _i32, ctypes.c_char_p], ctypes.c_int),
    "dh_ctx_set_config": ([_vp, _vp], ctypes.c_int),
    "dh_ctx_last_config": ([_vp, _vp], ctypes.c_int),
    "dh_ctx_set_launch_pairs": ([_vp, _i64], ctypes.c_int),
    "dh_ctx_profile": ([_vp, _i32], ctypes.c_int),
    "dh_ctx_profile_read": ([_vp, ctypes.POINTER(_f64), ctypes.POINTER(_i64)], ctypes.c_int),
    "dh_ctx_searched_pairs": ([_vp, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "dh_ctx_searched_images": ([_vp, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "dh_search_images": ([_vp, _vp, _vp, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
}


class FrameDesc(ctypes.Structure):
    """dh_frame_desc."""
    _fields_ = [("d_coords", _vp), ("offsets", _vp), ("n_species", _i32), ("box_type", _i32),
                ("box", _vp), ("r_max", _f64), ("n_bins", _i32), ("d_out", _vp),
                ("d_out_of_range", _vp)]


BATCH_GRAPH = 1
TUNE_OFF, TUNE_CACHED, TUNE_ON = 0, 1, 2
KNOB_NAMES = ("r", "copies", "tj", "noclamp", "occ_cap", "items_per_wg", "threads", "wide")
# accumulation modes reported by dh_ctx_last_config
MODE_LDS, MODE_SWEEP, MODE_GLOBAL = 0, 1, 2


def _load() -> ctypes.CDLL:
    # One HIP runtime per process: PyTorch ships its own libamdhip64.so.7 and
    # fails to initialise the GPU if another copy with that soname was loaded
    # first. Importing torch before the library makes the library bind to
    # torch's copy.
    try:
        import torch  # noqa: F401
    except ImportError:  # pragma: no cover - torch is optional for the C ABI
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"libdisthist.so not found at {LIB_PATH}; build it with "
            "`python -m paper_1808_01478_amd.build` (there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


LIB = _load()


class DisthistError(RuntimeError):
    def __init__(self, code: int, detail: str = ""):
        self.code = code
        msg = LIB.dh_strerror(code).decode()
        super().__init__(f"{msg} ({code})" + (f": {detail}" if detail else ""))


def _check(rc: int, ctx=None):
    if rc != DH_OK:
        detail = LIB.dh_ctx_last_error(ctx if ctx else None).decode()
        raise DisthistError(rc, detail)


def version() -> str:
    return LIB.dh_version().decode()


def n_hist(n_species: int) -> int:
    return n_species * (n_species + 1) // 2


def _np_ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _host_box(box) -> Optional[np.ndarray]:
    if box is None:
        return None
    return np.ascontiguousarray(np.asarray(box, np.float64).reshape(9))


def _offsets(offsets) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(offsets, np.int64))


def check_args(coords, offsets, box_type: int, box, r_max: float, n_bins: int,
               precision: int) -> int:
    """dh_check_args: host-only validation; returns the status code."""
    c = None if coords is None else np.ascontiguousarray(coords, np.float64)
    o = _offsets(offsets)
    b = _host_box(box)
    return int(LIB.dh_check_args(_np_ptr(c), _np_ptr(o), len(o) - 1, int(box_type), _np_ptr(b),
                                 float(r_max), int(n_bins), int(precision)))


def search_images(box):
    """dh_search_images: (lists int32 [8, 26], counts int32 [8], full_mask) of
    the image search for a triclinic cell (host only)."""
    b = _host_box(box)
    lists = np.zeros((8, 26), np.int32)
    counts = np.zeros(8, np.int32)
    full = ctypes.c_int32()
    _check(LIB.dh_search_images(_np_ptr(b), _np_ptr(lists), _np_ptr(counts), ctypes.byref(full)))
    return lists, counts, int(full.value)


def histo_noalloc(d_coords, offsets, box_type: int, box, r_max: float, n_bins: int,
                  precision: int, d_out, d_out_of_range=None, stream=None) -> None:
    """dh_histo_noalloc on torch device tensors (the current device): the
    allocation-free variant of Context.histo_async."""
    o = _offsets(offsets)
    b = _host_box(box)
    _check(LIB.dh_histo_noalloc(_stream_handle(stream), ctypes.c_void_p(d_coords.data_ptr()),
                                _np_ptr(o), len(o) - 1, int(box_type), _np_ptr(b),
                                float(r_max), int(n_bins), int(precision),
                                ctypes.c_void_p(d_out.data_ptr()),
                                None if d_out_of_range is None
                                else ctypes.c_void_p(d_out_of_range.data_ptr())))


def histo(coords, offsets, box_type: int, box, r_max: float, n_bins: int,
          precision: int = FP32) -> np.ndarray:
    """dh_histo: synchronous histogram of a host frame; returns uint64 [H, n_bins]."""
    c = np.ascontiguousarray(coords, np.float64)
    o = _offsets(offsets)
    b = _host_box(box)
    out = np.empty((n_hist(len(o) - 1), int(n_bins)), np.uint64)
    _check(LIB.dh_histo(_np_ptr(c), _np_ptr(o), len(o) - 1, int(box_type), _np_ptr(b),
                        float(r_max), int(n_bins), int(precision), _np_ptr(out)))
    return out


def cpu_histo(coords, offsets, box_type: int, box, r_max: float, n_bins: int,
              precision: int = FP32, n_threads: int = 0):
    """dh_cpu_histo: the tuned CPU kernel; returns (uint64 [H, n_bins],
    out-of-range uint64 [H])."""
    c = np.ascontiguousarray(coords, np.float64)
    o = _offsets(offsets)
    b = _host_box(box)
    k = len(o) - 1
    out = np.empty((n_hist(k), int(n_bins)), np.uint64)
    oor = np.empty(n_hist(k), np.uint64)
    _check(LIB.dh_cpu_histo(_np_ptr(c), _np_ptr(o), k, int(box_type), _np_ptr(b), float(r_max),
                            int(n_bins), int(precision), int(n_threads), _np_ptr(out),
                            _np_ptr(oor)))
    return out, oor


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Context:
    """A dh_ctx on one device (owns reusable device scratch). hbm_budget_bytes
    bounds the device memory of its scratch and live batches (0: no limit);
    a call that needs more raises DisthistError with code DH_EBUDGET."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = ctypes.c_void_p()
        _check(LIB.dh_ctx_create(int(device), int(hbm_budget_bytes), ctypes.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            LIB.dh_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):  # pragma: no cover - interpreter shutdown order
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def last_error(self) -> str:
        return LIB.dh_ctx_last_error(self.handle).decode()

    def histo_async(self, d_coords, offsets, box_type: int, box, r_max: float, n_bins: int,
                    precision: int, d_out, d_out_of_range=None, stream=None) -> None:
        """dh_histo_async on torch device tensors: d_coords float64 [N,3],
        d_out uint64/int64 [H, n_bins], d_out_of_range [H] or None."""
        o = _offsets(offsets)
        b = _host_box(box)
        _check(LIB.dh_histo_async(self.handle, _stream_handle(stream),
                                  ctypes.c_void_p(d_coords.data_ptr()), _np_ptr(o), len(o) - 1,
                                  int(box_type), _np_ptr(b), float(r_max), int(n_bins),
                                  int(precision), ctypes.c_void_p(d_out.data_ptr()),
                                  None if d_out_of_range is None
                                  else ctypes.c_void_p(d_out_of_range.data_ptr())),
               self.handle)

    def set_tuning(self, mode: int, cache_path: Optional[str] = None) -> None:
        """dh_ctx_set_tuning: TUNE_OFF, TUNE_CACHED or TUNE_ON, optional JSON cache."""
        _check(LIB.dh_ctx_set_tuning(self.handle, int(mode),
                                     None if cache_path is None else cache_path.encode()),
               self.handle)

    def set_config(self, knobs=None) -> None:
        """dh_ctx_set_config: force a launch shape (dict or 8 ints, KNOB_NAMES order) or None."""
        if knobs is None:
            _check(LIB.dh_ctx_set_config(self.handle, None), self.handle)
            return
        if isinstance(knobs, dict):
            knobs = [knobs[k] for k in KNOB_NAMES]
        arr = np.ascontiguousarray(np.asarray(knobs, np.int32))
        if arr.shape != (len(KNOB_NAMES),):
            raise ValueError(f"expected {len(KNOB_NAMES)} knobs {KNOB_NAMES}, got {arr.shape}")
        _check(LIB.dh_ctx_set_config(self.handle, _np_ptr(arr)), self.handle)

    def last_config(self) -> dict:
        """dh_ctx_last_config: the shape of the last single-frame launch."""
        out = np.zeros(13, np.int32)
        _check(LIB.dh_ctx_last_config(self.handle, _np_ptr(out)), self.handle)
        d = {k: int(v) for k, v in zip(KNOB_NAMES, out[:8])}
        d.update(grid=int(out[8]), lds_bytes=int(out[9]), sweeps=int(out[10]), items=int(out[11]),
                 mode=int(out[12]))
        return d

    def set_launch_pairs(self, max_pairs: int) -> None:
        """dh_ctx_set_launch_pairs: split histograms into launches of at most
        max_pairs pairs (0 = one launch per frame)."""
        _check(LIB.dh_ctx_set_launch_pairs(self.handle, int(max_pairs)), self.handle)

    def profile(self, enable: bool = True) -> None:
        """dh_ctx_profile: time the pair kernel of every launch with HIP events."""
        _check(LIB.dh_ctx_profile(self.handle, 1 if enable else 0), self.handle)

    def profile_read(self):
        """dh_ctx_profile_read: (summed pair-kernel ms, launches) since the last read."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(LIB.dh_ctx_profile_read(self.handle, ctypes.byref(ms), ctypes.byref(n)),
               self.handle)
        return float(ms.value), int(n.value)

    def searched_pairs(self) -> int:
        """dh_ctx_searched_pairs: pairs of the last single-frame call that went
        through the 27-image search (wait for its stream first)."""
        v = ctypes.c_uint64()
        _check(LIB.dh_ctx_searched_pairs(self.handle, ctypes.byref(v)), self.handle)
        return int(v.value)

    def searched_images(self) -> int:
        """dh_ctx_searched_images: images evaluated for the searched pairs of
        the last single-frame call (wait for its stream first)."""
        v = ctypes.c_uint64()
        _check(LIB.dh_ctx_searched_images(self.handle, ctypes.byref(v)), self.handle)
        return int(v.value)

    def pair_t_async(self, d_coords, box_type: int, box, r_max: float, n_bins: int,
                     precision: int, d_pi, d_pj, d_t, stream=None) -> None:
        """dh_pair_t_async on torch device tensors (int32 indices, float64 output)."""
        b = _host_box(box)
        _check(LIB.dh_pair_t_async(self.handle, _stream_handle(stream),
                                   ctypes.c_void_p(d_coords.data_ptr()), int(d_coords.shape[0]),
                                   int(box_type), _np_ptr(b), float(r_max), int(n_bins),
                                   int(precision), ctypes.c_void_p(d_pi.data_ptr()),
                                   ctypes.c_void_p(d_pj.data_ptr()), int(d_pi.numel()),
                                   ctypes.c_void_p(d_t.data_ptr())),
               self.handle)


class Batch:
    """dh_batch: many frames planned once and run as one graph of launches.

    ``frames`` is a sequence of dicts with keys d_coords (torch float64 [N,3]
    on the device), offsets, box_type, box, r_max, n_bins, d_out (torch
    int64/uint64 [H, n_bins]) and optionally d_out_of_range ([H]). The device
    tensors must stay alive and at the same address for the batch's life; each
    launch reads their current contents."""

    def __init__(self, ctx: Context, frames, precision: int, graph: bool = True):
        self.ctx = ctx
        self._keep = []
        descs = (FrameDesc * len(frames))()
        for k, f in enumerate(frames):
            o = _offsets(f["offsets"])
            b = _host_box(f.get("box"))
            self._keep += [o, b, f["d_coords"], f["d_out"], f.get("d_out_of_range")]
            descs[k].d_coords = f["d_coords"].data_ptr()
            descs[k].offsets = o.ctypes.data
            descs[k].n_species = len(o) - 1
            descs[k].box_type = int(f["box_type"])
            descs[k].box = None if b is None else b.ctypes.data
            descs[k].r_max = float(f["r_max"])
            descs[k].n_bins = int(f["n_bins"])
            descs[k].d_out = f["d_out"].data_ptr()
            oor = f.get("d_out_of_range")
            descs[k].d_out_of_range = None if oor is None else oor.data_ptr()
        h = ctypes.c_void_p()
        _check(LIB.dh_batch_create(ctx.handle, ctypes.cast(descs, _vp), len(frames),
                                   int(precision), BATCH_GRAPH if graph else 0,
                                   ctypes.byref(h)), ctx.handle)
        self.handle = h

    def launch(self, stream=None) -> None:
        _check(LIB.dh_batch_launch(self.handle, _stream_handle(stream)), self.ctx.handle)

    def info(self):
        n, l, p = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_double()
        _check(LIB.dh_batch_info(self.handle, ctypes.byref(n), ctypes.byref(l), ctypes.byref(p)))
        return {"items": int(n.value), "launches": int(l.value), "pairs": float(p.value)}

    def close(self):
        if getattr(self, "handle", None):
            LIB.dh_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


JOB_DONE, JOB_QUEUED, JOB_RUNNING = 0, 1, 2
SCHED_SHORTEST, SCHED_ARRIVAL = 0, 1


def sched_select(need_bytes, waited_s, free_bytes: int, free_slots: int,
                 head_wait_limit_s: float, work=None):
    """dh_sched_select: queue positions the server would start now."""
    need = np.ascontiguousarray(np.asarray(need_bytes, np.int64))
    wait = np.ascontiguousarray(np.asarray(waited_s, np.float64))
    wk = None if work is None else np.ascontiguousarray(np.asarray(work, np.float64))
    out = np.zeros(max(1, len(need)), np.int32)
    n = LIB.dh_sched_select(_np_ptr(need), _np_ptr(wait), _np_ptr(wk), len(need),
                            int(free_bytes), int(free_slots), float(head_wait_limit_s),
                            _np_ptr(out))
    return [int(v) for v in out[:n]]


class Server:
    """dh_server: continuous-batching request loop on one GPU."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 8 << 30, max_inflight: int = 4,
                 head_wait_limit_s: float = 1.0, policy: int = None):
        h = ctypes.c_void_p()
        _check(LIB.dh_server_create(int(device), int(hbm_budget_bytes), int(max_inflight),
                                    float(head_wait_limit_s), ctypes.byref(h)))
        self.handle = h
        self._shapes = {}
        if policy is not None:
            self.set_policy(policy)

    def set_policy(self, policy: int):
        """SCHED_SHORTEST (least work first, the default) or SCHED_ARRIVAL."""
        _check(LIB.dh_server_set_policy(self.handle, int(policy)))

    def submit(self, coords, offsets, box_type: int, box, r_max: float, n_bins: int,
               precision: int = FP32) -> int:
        c = np.ascontiguousarray(coords, np.float64)
        o = _offsets(offsets)
        b = _host_box(box)
        jid = ctypes.c_int64()
        _check(LIB.dh_server_submit(self.handle, _np_ptr(c), _np_ptr(o), len(o) - 1, int(box_type),
                                    _np_ptr(b), float(r_max), int(n_bins), int(precision),
                                    ctypes.byref(jid)))
        self._shapes[jid.value] = (n_hist(len(o) - 1), int(n_bins))
        return int(jid.value)

    def status(self, job_id: int) -> int:
        return int(LIB.dh_server_status(self.handle, int(job_id)))

    def wait(self, job_id: int):
        """(histograms uint64 [H, n_bins], out_of_range [H], (queued_s, run_s, latency_s))."""
        h, nb = self._shapes.pop(job_id)
        out = np.empty((h, nb), np.uint64)
        oor = np.empty(h, np.uint64)
        times = np.zeros(3, np.float64)
        _check(LIB.dh_server_wait(self.handle, int(job_id), _np_ptr(out), _np_ptr(oor),
                                  _np_ptr(times)))
        return out, oor, tuple(float(t) for t in times)

    def stats(self) -> dict:
        st = np.zeros(6, np.int64)
        _check(LIB.dh_server_stats(self.handle, _np_ptr(st)))
        out = dict(zip(("submitted", "completed", "failed", "max_running", "peak_bytes",
                        "budget_bytes"), (int(v) for v in st)))
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(LIB.dh_server_launch_stats(self.handle, ctypes.byref(a), ctypes.byref(b),
                                          ctypes.byref(c)))
        out.update(launches=int(a.value), shared_launches=int(b.value),
                   max_jobs_per_launch=int(c.value))
        return out

    def close(self):
        if getattr(self, "handle", None):
            LIB.dh_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


class Trajectory:
    """dh_traj: a trajectory file opened for the trajectory engine."""

    def __init__(self, path: str):
        h = ctypes.c_void_p()
        _check(LIB.dh_traj_open(os.fsencode(path), ctypes.byref(h)))
        self.handle = h
        self.path = path

    def info(self) -> dict:
        nf, n = ctypes.c_int64(), ctypes.c_int64()
        bt = ctypes.c_int32()
        _check(LIB.dh_traj_info(self.handle, ctypes.byref(nf), ctypes.byref(n), ctypes.byref(bt)))
        return {"n_frames": nf.value, "n_points": n.value, "box_type": bt.value}

    def histo(self, ctx: "Context", offsets, r_max: float, n_bins: int, precision: int,
              results_path: str, interval: int = 1, frame_begin: int = 0,
              frame_end: Optional[int] = None, max_intervals: int = 0) -> int:
        """dh_traj_histo: interval sums appended to results_path (which is also
        the checkpoint); returns the number of complete intervals recorded."""
        o = _offsets(offsets)
        if frame_end is None:
            frame_end = self.info()["n_frames"]
        done = ctypes.c_int64()
        _check(LIB.dh_traj_histo(ctx.handle, self.handle, _np_ptr(o), len(o) - 1, float(r_max),
                                 int(n_bins), int(precision), int(frame_begin), int(frame_end),
                                 int(interval), os.fsencode(results_path), int(max_intervals),
                                 ctypes.byref(done)), ctx.handle)
        return done.value

    def histo_hybrid(self, ctx: "Context", offsets, r_max: float, n_bins: int, precision: int,
                     results_path: str, cpu_threads: int, interval: int = 1,
                     frame_begin: int = 0, frame_end: Optional[int] = None,
                     max_intervals: int = 0, greedy: bool = False):
        """dh_traj_histo_hybrid: as histo, with a CPU worker of cpu_threads
        threads beside the GPU; returns (intervals recorded, frames the CPU
        computed)."""
        o = _offsets(offsets)
        if frame_end is None:
            frame_end = self.info()["n_frames"]
        done, cpu = ctypes.c_int64(), ctypes.c_int64()
        _check(LIB.dh_traj_histo_hybrid(ctx.handle, self.handle, _np_ptr(o), len(o) - 1,
                                        float(r_max), int(n_bins), int(precision),
                                        int(frame_begin), int(frame_end), int(interval),
                                        os.fsencode(results_path), int(max_intervals),
                                        int(cpu_threads), 1 if greedy else 0,
                                        ctypes.byref(done), ctypes.byref(cpu)), ctx.handle)
        return done.value, cpu.value

    def close(self) -> None:
        if self.handle:
            LIB.dh_traj_close(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def exported_symbols() -> Sequence[str]:
    return list(SIGNATURES)
