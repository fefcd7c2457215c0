"""Tune the launch shapes of named workloads on the current GPU and store
them in the JSON cache that bench.py and callers load with dh_ctx_set_tuning.

    python -m paper_1808_01478_amd.tune [--out PATH] [--workloads a,b,...]

Every shape gives identical counts; the cache only records which one was
fastest for each bucket (arch, precision, box kind, log2 bins, log2 N,
species).
"""
from __future__ import annotations

import argparse
import json
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(PKG, "tuning", "launch_shapes.json")


def main(argv=None) -> int:
    sys.path.insert(0, os.path.dirname(PKG))
    import torch
    import workloads
    import paper_1808_01478_amd as dh

    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--workloads",
                    default="ortho100k,tiny,triclinic1M,image_search,trajectory")
    args = ap.parse_args(argv)
    makers = {"ortho100k": workloads.ortho, "tiny": workloads.tiny,
              "triclinic1M": workloads.triclinic, "image_search": workloads.image_search}
    # tune into a fresh file so that every listed workload is measured again,
    # then merge its entries over the existing cache
    fresh = args.out + ".new"
    if os.path.exists(fresh):
        os.remove(fresh)
    ctx = dh.Context(0)
    ctx.set_tuning(dh.TUNE_ON, fresh)
    dev = torch.device("cuda")
    for name in args.workloads.split(","):
        if name == "trajectory":
            # binary32 buckets of the 512-frame trajectory (log2 N 14-18,
            # one to four species): the first frame of each bucket is tuned,
            # the others find its entry
            for fr in workloads.trajectory(512):
                x = torch.from_numpy(fr.coords).to(dev)
                out = torch.empty((fr.n_hist, fr.n_bins), dtype=torch.int64, device=dev)
                ctx.histo_async(x, fr.offsets, fr.box_type, fr.box, fr.r_max, fr.n_bins,
                                dh.FP32, out)
            torch.cuda.synchronize()
            print(f"trajectory precision={dh.FP32}: 512 frames", flush=True)
            continue
        fr = makers[name]()
        x = torch.from_numpy(fr.coords).to(dev)
        out = torch.empty((fr.n_hist, fr.n_bins), dtype=torch.int64, device=dev)
        for prec in (dh.FP32, dh.FP64):
            ctx.histo_async(x, fr.offsets, fr.box_type, fr.box, fr.r_max, fr.n_bins, prec, out)
            torch.cuda.synchronize()
            print(f"{name} precision={prec}: {ctx.last_config()}", flush=True)
    ctx.close()
    merge(args.out, fresh)
    os.remove(fresh)
    return 0


def merge(out: str, fresh: str) -> None:
    """Entries of `fresh` replace those of `out` with the same key; entries
    of an older cache format are dropped."""
    with open(fresh) as fh:
        new = json.load(fh)
    entries = {}
    if os.path.exists(out):
        with open(out) as fh:
            old = json.load(fh)
        if old.get("version") == new["version"]:
            entries.update(old["entries"])
    entries.update(new["entries"])
    with open(out + ".tmp", "w") as fh:
        fh.write(f'{{"version": {new["version"]}, "knobs": {json.dumps(new["knobs"])}, '
                 '"entries": {')
        fh.write(",".join(f'\n  "{k}": {json.dumps(v)}' for k, v in sorted(entries.items())))
        fh.write("\n}}\n")
    os.replace(out + ".tmp", out)


if __name__ == "__main__":
    sys.exit(main())
