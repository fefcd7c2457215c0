"""Trajectory files and interval results of the trajectory engine
(dh_traj_open / dh_traj_histo); the layouts are described in
include/disthist.h. Plain numpy, no device work."""
from __future__ import annotations

import os
from typing import Iterable, Optional

import numpy as np

TRAJ_MAGIC = b"DHTRAJ01"
RES_MAGIC = b"DHRES001"
TRAJ_HEADER = 64
RES_HEADER = 128


def write_trajectory(path: str, frames: Iterable[np.ndarray], box_type: int,
                     boxes: Optional[Iterable[np.ndarray]] = None) -> int:
    """Writes frames (each [N][3] binary64, same N) with their boxes ([3][3]
    rows a, b, c; None for box_type 0). Returns the number of frames."""
    frames = list(frames)
    boxes = [None] * len(frames) if boxes is None else list(boxes)
    if len(boxes) != len(frames):
        raise ValueError("one box per frame")
    n = frames[0].shape[0] if frames else 0
    tmp = path + ".tmp"
    with open(tmp, "wb") as fh:
        hdr = bytearray(TRAJ_HEADER)
        hdr[0:8] = TRAJ_MAGIC
        hdr[8:16] = np.int64(len(frames)).tobytes()
        hdr[16:24] = np.int64(n).tobytes()
        hdr[24:28] = np.int32(box_type).tobytes()
        fh.write(bytes(hdr))
        for x, b in zip(frames, boxes):
            x = np.ascontiguousarray(x, np.float64)
            if x.shape != (n, 3):
                raise ValueError("every frame must be [N][3] with the same N")
            bb = np.zeros(9) if b is None else np.ascontiguousarray(b, np.float64).reshape(9)
            fh.write(bb.tobytes())
            fh.write(x.tobytes())
    os.replace(tmp, path)
    return len(frames)


def read_results(path: str, n_hist: int):
    """(header fields, hist uint64 [k][H][n_bins], out_of_range [k][H],
    frames per interval [k]) of a results file written by dh_traj_histo."""
    raw = open(path, "rb").read()
    if raw[:8] != RES_MAGIC:
        raise ValueError("not a results file")
    h = np.frombuffer(raw[8:RES_HEADER], np.uint8)
    fb, fe, iv = np.frombuffer(h[8:32].tobytes(), np.int64)
    n_species, n_bins, precision, box_type = np.frombuffer(h[32:48].tobytes(), np.int32)
    r_max = float(np.frombuffer(h[48:56].tobytes(), np.float64)[0])
    words = n_hist * int(n_bins) + n_hist + 1
    k = (len(raw) - RES_HEADER) // (8 * words)         # complete records only
    rec = np.frombuffer(raw[RES_HEADER:RES_HEADER + 8 * words * k], np.uint64).reshape(k, words)
    hist = rec[:, :n_hist * int(n_bins)].reshape(k, n_hist, int(n_bins))
    oor = rec[:, n_hist * int(n_bins):n_hist * int(n_bins) + n_hist]
    frames = rec[:, -1]
    info = dict(frame_begin=int(fb), frame_end=int(fe), interval=int(iv),
                n_species=int(n_species), n_bins=int(n_bins), precision=int(precision),
                box_type=int(box_type), r_max=r_max)
    return info, hist, oor, frames
