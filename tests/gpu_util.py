"""Helpers for GPU tests: run the library on torch device buffers and apply
the binary32 edge-pair bound."""
from __future__ import annotations

import numpy as np


def run_gpu(ctx, frame, precision, stream=None):
    """(hist uint64 [H, n_bins], out_of_range uint64 [H]) via dh_histo_async."""
    import torch
    dev = torch.device("cuda")
    x = torch.from_numpy(np.ascontiguousarray(frame.coords)).to(dev)
    h = frame.n_hist
    out = torch.full((h, frame.n_bins), -1, dtype=torch.int64, device=dev)
    oor = torch.full((h,), -1, dtype=torch.int64, device=dev)
    ctx.histo_async(x, frame.offsets, frame.box_type, frame.box, frame.r_max, frame.n_bins,
                    precision, out, oor, stream=stream)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64), oor.cpu().numpy().view(np.uint64)


def oor_bound_violations(oor32, oor64, edges):
    """Binary32 out-of-range counts against the binary64 ones: only pairs
    within the window of the last edge (t near n_bins) can move across it.
    The device keeps out-of-range counts as the pair count less every flushed
    in-range count, so comparing them with the sum of the bins would hold by
    construction; this compares them with the oracle's instead."""
    bad = []
    for h in range(len(oor64)):
        d = abs(int(oor32[h]) - int(oor64[h]))
        e = int(edges[h, -1])
        if d > e:
            bad.append(f"h{h}: out-of-range differs by {d} > E = {e}")
    return bad


def fp32_bound_violations(h32, h64, edges):
    """Per edge k the cumulative counts C(k) = sum_{b<k} H[b] of the binary32
    and binary64 histograms may differ by at most the number of pairs within
    the window of edge k (edges[:, k-1]); also L1 <= 2 * sum(edges).
    Returns a list of human-readable violations (empty when within bound)."""
    bad = []
    for h in range(h64.shape[0]):
        c32 = np.cumsum(h32[h].astype(np.int64))
        c64 = np.cumsum(h64[h].astype(np.int64))
        e = edges[h].astype(np.int64)
        d = np.abs(c32 - c64)
        over = np.nonzero(d > e)[0]
        if len(over):
            k = int(over[0])
            bad.append(f"h{h}: edge {k + 1}: |dC| = {d[k]} > E = {e[k]} ({len(over)} edges)")
        l1 = int(np.abs(h32[h].astype(np.int64) - h64[h].astype(np.int64)).sum())
        if l1 > 2 * int(e.sum()):
            bad.append(f"h{h}: L1 {l1} > 2*sum(E) = {2 * int(e.sum())}")
    return bad
