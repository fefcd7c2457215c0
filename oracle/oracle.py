"""TEST INFRASTRUCTURE ONLY: ctypes wrapper and build step for dh_oracle.c.

The oracle is a plain FP64 double loop (see the header of dh_oracle.c for the
definition and the passages of the paper it follows). ``build()`` compiles it
with gcc; ``histogram()`` runs it on numpy arrays.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import Optional

import numpy as np

BOX_NONE, BOX_ORTHO, BOX_TRICLINIC = 0, 1, 2
IMAGES_PAPER, IMAGES_27, IMAGES_125 = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dh_oracle.c")
# -ffp-contract=off: no fused multiply-add beyond the explicit fma() calls.
# -mfma lets the explicit fma() calls compile to the hardware instruction.
_CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-mfma",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra"]


def lib_path(mutant: int = 0) -> str:
    name = "libdh_oracle.so" if mutant == 0 else f"libdh_oracle_mutant{mutant}.so"
    return os.path.join(_HERE, name)


def build(mutant: int = 0, force: bool = True, out: Optional[str] = None) -> str:
    """Compile the oracle (or a planted-mistake variant) into a shared library."""
    path = out or lib_path(mutant)
    if not force and os.path.exists(path) and os.path.getmtime(path) >= os.path.getmtime(_SRC):
        return path
    tmp = path + f".tmp{os.getpid()}"
    cmd = ["gcc", *_CFLAGS, f"-DDHO_MUTANT={mutant}", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, path)
    return path


_LIBS = {}


def load(mutant: int = 0, path: Optional[str] = None) -> ctypes.CDLL:
    key = path or mutant
    if key in _LIBS:
        return _LIBS[key]
    p = path or lib_path(mutant)
    if not os.path.exists(p) or os.path.getmtime(p) < os.path.getmtime(_SRC):
        build(mutant, out=path)
    lib = ctypes.CDLL(p)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.dho_histogram.argtypes = [vp, vp, i32, i32, vp, f64, i32, i32, f64, vp, vp, vp, i32]
    lib.dho_histogram.restype = ctypes.c_int
    lib.dho_pair_t.argtypes = [vp, i64, i32, vp, f64, i32, i32, vp, vp, i64, vp]
    lib.dho_pair_t.restype = ctypes.c_int
    lib.dho_min_width.argtypes = [vp]
    lib.dho_min_width.restype = f64
    lib.dho_max_threads.restype = ctypes.c_int
    lib.dho_mutant.restype = ctypes.c_int
    _LIBS[key] = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclasses.dataclass
class OracleResult:
    hist: np.ndarray            # (H, n_bins) uint64
    out_of_range: np.ndarray    # (H,) uint64
    edges: Optional[np.ndarray]  # (H, n_bins) uint64; edge k at column k-1


def _prep(coords, offsets, box):
    c = np.ascontiguousarray(coords, dtype=np.float64)
    o = np.ascontiguousarray(offsets, dtype=np.int64)
    b = None if box is None else np.ascontiguousarray(np.asarray(box, np.float64).reshape(9))
    return c, o, b


def histogram(coords, offsets, box_type: int, box, r_max: float, n_bins: int,
              image_mode: int = IMAGES_PAPER, edge_window: float = 0.0,
              n_threads: int = 0, mutant: int = 0, lib: Optional[ctypes.CDLL] = None) -> OracleResult:
    """All species-pair histograms of one frame (FP64 definition)."""
    c, o, b = _prep(coords, offsets, box)
    k = len(o) - 1
    n_hist = k * (k + 1) // 2
    hist = np.zeros((n_hist, n_bins), np.uint64)
    oor = np.zeros(n_hist, np.uint64)
    edges = np.zeros((n_hist, n_bins), np.uint64) if edge_window > 0 else None
    lib = lib or load(mutant)
    rc = lib.dho_histogram(_ptr(c), _ptr(o), k, box_type, _ptr(b), float(r_max), int(n_bins),
                           int(image_mode), float(edge_window), _ptr(hist), _ptr(oor), _ptr(edges),
                           int(n_threads))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return OracleResult(hist, oor, edges)


def frame_histogram(frame, **kw) -> OracleResult:
    return histogram(frame.coords, frame.offsets, frame.box_type, frame.box, frame.r_max,
                     frame.n_bins, **kw)


def pair_t(coords, box_type: int, box, r_max: float, n_bins: int, pi, pj,
           image_mode: int = IMAGES_PAPER, mutant: int = 0) -> np.ndarray:
    """t = r * n_bins / r_max for explicit global index pairs."""
    c, _, b = _prep(coords, [0, len(coords)], box)
    pi = np.ascontiguousarray(pi, np.int64)
    pj = np.ascontiguousarray(pj, np.int64)
    out = np.empty(len(pi), np.float64)
    rc = load(mutant).dho_pair_t(_ptr(c), len(c), box_type, _ptr(b), float(r_max), int(n_bins),
                                 int(image_mode), _ptr(pi), _ptr(pj), len(pi), _ptr(out))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out


def min_width(box) -> float:
    b = np.ascontiguousarray(np.asarray(box, np.float64).reshape(9))
    return float(load().dho_min_width(_ptr(b)))


def max_threads() -> int:
    return int(load().dho_max_threads())


def edge_window(coords, box, r_max: float, ulps: int = 4) -> float:
    """Window for edge pairs of a binary32 computation: ulps * ulp32(S) with
    S = max(max |coordinate component|, max |box entry|, r_max) and
    ulp32(S) = 2**(floor(log2 S) - 23)."""
    s = float(np.max(np.abs(coords))) if len(coords) else 0.0
    if box is not None:
        s = max(s, float(np.max(np.abs(box))))
    s = max(s, float(r_max))
    e = math.frexp(s)[1] - 1          # floor(log2 s)
    return ulps * math.ldexp(1.0, e - 23)
