"""Host threads: several threads, each with its own context and stream, and
several threads sharing the synchronous entry point's library-owned context,
all give the same counts as one thread alone (ctypes releases the GIL, so the
library calls really overlap)."""
import threading

import numpy as np
import pytest

import workloads
from cases import parity_cases
from gpu_util import run_gpu

pytestmark = pytest.mark.gpu

FRAMES = [f for f in parity_cases() if f.n_bins <= 2000][:8]


def test_contexts_per_thread():
    import torch
    import paper_1808_01478_amd as dh
    with dh.Context(0) as c:
        ref = [[run_gpu(c, f, p)[0] for p in (0, 1)] for f in FRAMES]
    errors, results = [], {}

    def worker(t):
        try:
            s = torch.cuda.Stream()
            with dh.Context(0) as c, torch.cuda.stream(s):
                for rep in range(3):
                    for k, f in enumerate(FRAMES):
                        p = (k + t + rep) % 2
                        results[t, rep, k, p] = run_gpu(c, f, p, stream=s)[0]
        except Exception as e:  # surfaced below
            errors.append(repr(e))
    th = [threading.Thread(target=worker, args=(t,)) for t in range(4)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    assert not errors, errors
    assert len(results) == 4 * 3 * len(FRAMES)
    for (t, rep, k, p), h in results.items():
        assert np.array_equal(h, ref[k][p]), f"thread {t} rep {rep} frame {k} prec {p}"


def test_sync_entry_point_from_threads():
    import paper_1808_01478_amd as dh
    f = FRAMES[2]
    ref = dh.histo(f.coords, f.offsets, f.box_type, f.box, f.r_max, f.n_bins, 1)
    out, errors = [], []

    def worker():
        try:
            for _ in range(5):
                out.append(dh.histo(f.coords, f.offsets, f.box_type, f.box, f.r_max, f.n_bins, 1))
        except Exception as e:
            errors.append(repr(e))
    th = [threading.Thread(target=worker) for _ in range(4)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    assert not errors, errors
    assert len(out) == 20 and all(np.array_equal(h, ref) for h in out)
