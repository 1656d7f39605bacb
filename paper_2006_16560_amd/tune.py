"""Fills the package's autotuner cache (tuned.jsonl) for the benchmark
workloads: for each (workload, theta) it runs petar_autotune on that
workload's particles and radii, which times a full step for every candidate
leaf size, group size and number of targets per lane and appends the fastest
to the cache (keyed by floor(log2 N), theta and precision).

Run from the repository root on a GPU:
    python -m paper_2006_16560_amd.tune [--fresh]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# (workload, theta): the 1M cluster at the paper's opening angles and the
# 10M cluster at theta 0.5
JOBS = [("plummer1m_b100", 0.5), ("plummer1m_b100", 0.3), ("plummer1m_b100", 0.7),
        ("plummer10m_b10", 0.5)]


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--fresh", action="store_true", help="start from an empty cache")
    ap.add_argument("--cache", default=None, help="cache file (default: the package's)")
    args = ap.parse_args()

    import torch

    import paper_2006_16560_amd as pt
    import workloads

    cache = pt.TUNED_CACHE if args.cache is None else args.cache
    if args.fresh and os.path.exists(cache):
        os.remove(cache)
    dev = "cuda:0"
    made = {}
    for name, theta in JOBS:
        wl = workloads.WORKLOADS[name]
        if name not in made:
            made.clear()
            torch.cuda.empty_cache()
            c = workloads.make_cluster(wl.n, 0, imf=wl.imf, binary_fraction=wl.binary_fraction)
            made[name] = (torch.from_numpy(c.pos).to(dev), torch.from_numpy(c.mass).to(dev))
        pos, mass = made[name]
        ctx = pt.petar_create(0)
        try:
            pt.petar_set_params(ctx, precision=pt.PETAR_MIXED)
            ri, ro, rs = pt.petar_changeover_radii(ctx, mass, wl.r_in_ref, wl.r_out_ref,
                                                   wl.search_factor)
            t0 = time.time()
            best = pt.petar_autotune(ctx, pos, mass, theta, ri, ro, rs, cache_path=cache)
            print(json.dumps({"workload": name, "theta": theta, "tuned": best,
                              "seconds": round(time.time() - t0, 1)}), flush=True)
        finally:
            pt.petar_destroy(ctx)
    return 0


if __name__ == "__main__":
    sys.exit(main())
