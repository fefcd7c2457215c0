"""Write the stored oracle results for the full-size workloads.

    python tests/golden/make_golden.py [triclinic1M] [image_search200k] [trajectory32]

Calls only the oracle (oracle/) on inputs from the seeded generators
(workloads/), and stores per workload:

  hist   (H, n_bins) uint64   binary64 histogram (Sec. 2.1 Eq. 4, Algorithm 1,
                              Sec. 2.3 Eq. 5 with the 27-image search where
                              2 r_max reaches the smallest cell width)
  oor    (H,) uint64          pairs at or beyond r_max
  edges  (H, n_bins) uint64   pairs within the binary32 window of edge k
                              (column k-1), the tolerance of a binary32 run
  window float64              that window (4 ulp32 of the largest magnitude)
  input_sha256                hash of the generated coordinates, offsets, box,
                              r_max and n_bins, so that a test can tell a
                              different input from a different result

Multi-frame workloads store the frames' arrays concatenated along the
histogram axis with per-frame histogram offsets (hist_offsets). Nothing here
comes from the GPU library.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle      # noqa: E402
import workloads   # noqa: E402


def input_hash(fr) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(fr.coords, np.float64).tobytes())
    h.update(np.ascontiguousarray(fr.offsets, np.int64).tobytes())
    if fr.box is not None:
        h.update(np.ascontiguousarray(fr.box, np.float64).tobytes())
    h.update(np.float64(fr.r_max).tobytes())
    h.update(np.int64(fr.n_bins).tobytes())
    h.update(np.int64(fr.box_type).tobytes())
    return h.hexdigest()


def frames_for(name: str):
    if name == "triclinic1M":
        return [workloads.triclinic()]
    if name == "image_search200k":
        return [workloads.image_search()]
    if name == "trajectory32":
        return [workloads.trajectory_frame(f) for f in range(32)]
    raise SystemExit(f"unknown workload {name}")


def make(name: str) -> str:
    frames = frames_for(name)
    hists, oors, edges, windows, hashes, hoff = [], [], [], [], [], [0]
    t0 = time.time()
    for fr in frames:
        w = oracle.edge_window(fr.coords, fr.box, fr.r_max)
        ref = oracle.frame_histogram(fr, edge_window=w)
        hists.append(ref.hist)
        oors.append(ref.out_of_range)
        edges.append(ref.edges)
        windows.append(w)
        hashes.append(input_hash(fr))
        hoff.append(hoff[-1] + fr.n_hist)
        print(f"{name}: {fr.name} N={fr.n} H={fr.n_hist} done at {time.time() - t0:.0f} s",
              flush=True)
    path = os.path.join(HERE, f"{name}.npz")
    np.savez_compressed(
        path,
        hist=np.concatenate(hists), oor=np.concatenate(oors), edges=np.concatenate(edges),
        window=np.asarray(windows, np.float64), input_sha256=np.asarray(hashes),
        hist_offsets=np.asarray(hoff, np.int64),
        command=np.asarray(f"python tests/golden/make_golden.py {name}"),
        threads=np.int64(oracle.max_threads()))
    return path


def load(name: str):
    """The stored arrays of one workload (dict of numpy arrays)."""
    with np.load(os.path.join(HERE, f"{name}.npz"), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


if __name__ == "__main__":
    names = sys.argv[1:] or ["trajectory32", "image_search200k", "triclinic1M"]
    for n in names:
        print(make(n), flush=True)
