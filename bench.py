#!/usr/bin/env python3
"""Benchmark of the long-range P3T tree force on one MI355X.

One step is the whole hot path on one batch of particles: changeover radii
(eq. rcut), tree build (root box, Morton keys, radix sort, octree,
multipoles), then the long-range force with neighbour lists (radii in tree
order, cell search radii, i-groups, fused walk + interactions, neighbour
CSR). Inputs are resident in HBM before the timed region.

The headline is N = 1M (Plummer, Kroupa IMF, 100% binaries) at theta 0.5
with the leaf size, group size and targets per lane that the autotuner
stored for (N, theta). The same JSON line carries, as extra keys, the other
measured workloads: the 1M cluster at theta 0.3 and 0.7, the batched step
of 128 clusters (hipGraph replay, eager, 128 sequential calls), the 10M
cluster (mixed against FP64 pair arithmetic, memory), and the second-stage
neighbour filter, clusters, SDAR groups and artificial particles.

Prints ONE JSON line on stdout. Everything else goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak
FLOPS_PER_INTERACTION = 23    # counting convention for the headline figure

# The paper's N1mkb model (Table inpar: 10^6 stars, all in binaries):
# r_out,ref = 0.199039e-2, r_out/r_in = 10, long step 1/2048.
N1MKB_R_OUT_REF = 1.99039e-3
N1MKB_DT = 1.0 / 2048.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


FORCE_SOURCES = ["paper_2006_16560_amd/csrc/force.hip", "paper_2006_16560_amd/csrc/walk.h",
                 "paper_2006_16560_amd/csrc/common.h"]


def force_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in FORCE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_value(workload: str, cfg: dict, key: str = "hbm_bytes_per_launch"):
    """A per-launch figure of the force kernel (HBM bytes, FP32 operations)
    from the committed counter summary, if it was taken on the current
    force-kernel sources and the same launch configuration (else None)."""
    import re
    path = os.path.join(ROOT, "profiles", "k_force_pmc_%s_ipl%d.md" % (workload, cfg["i_per_lane"]))
    if not os.path.exists(path):
        return None
    text = open(path).read()
    b = re.search(r"^%s: (\d+)" % key, text, re.M)
    h = re.search(r"^sources_sha256_16: ([0-9a-f]+)", text, re.M)
    shape = re.search(r"^launch: leaf (\d+) group (\d+) theta ([0-9.]+)", text, re.M)
    if not b or not h or h.group(1) != force_sources_hash():
        return None
    if not shape or (int(shape.group(1)), int(shape.group(2)), float(shape.group(3))) != \
            (cfg["leaf_size"], cfg["group_size"], cfg["theta"]):
        return None
    return int(b.group(1))


def rel_err(a, ref):
    return np.linalg.norm(a - ref, axis=0) / np.linalg.norm(ref, axis=0)


def pick_config(pt, ctx, n, theta, wl, args):
    """(leaf, group, targets per lane): the autotuner's stored choice for
    (N, theta) unless given on the command line."""
    cfg = pt.launch_config(ctx, n, theta, leaf_default=wl.leaf_size)
    over = {"leaf_size": args.leaf, "group_size": args.group, "i_per_lane": args.ipl}
    for k, v in over.items():
        if v is not None:
            cfg[k] = v
            cfg["source"] = "command line"
    cfg["theta"] = theta
    return cfg


class Step:
    """Radii, tree build and force (+ neighbour lists) of one workload, with
    every buffer allocated once."""

    def __init__(self, pt, ctx, wl, pos, mass, theta, cfg, nb_per_particle=64):
        import torch
        self.pt, self.ctx, self.wl = pt, ctx, wl
        self.pos, self.mass, self.theta, self.cfg = pos, mass, theta, cfg
        n = mass.shape[0]
        dev = pos.device
        self.r_in = torch.empty(n, dtype=torch.float64, device=dev)
        self.r_out = torch.empty_like(self.r_in)
        self.r_s = torch.empty_like(self.r_in)
        self.acc = torch.empty((3, n), dtype=torch.float64, device=dev)
        self.pot = torch.empty(n, dtype=torch.float64, device=dev)
        self.nb_cap = nb_per_particle * n
        self.nb_bufs = (torch.empty(n + 1, dtype=torch.int64, device=dev),
                        torch.empty(self.nb_cap, dtype=torch.int32, device=dev))

    def radii(self):
        wl = self.wl
        if wl.uniform_radii:
            self.r_in.fill_(wl.r_in_ref)
            self.r_out.fill_(wl.r_out_ref)
            self.r_s.fill_(wl.search_factor * wl.r_out_ref)
        else:
            self.pt.petar_changeover_radii(self.ctx, self.mass, wl.r_in_ref, wl.r_out_ref,
                                           wl.search_factor, out=(self.r_in, self.r_out, self.r_s))

    def __call__(self, graph=False):
        pt, cfg = self.pt, self.cfg
        self.radii()
        if not graph:
            pt.petar_tree_build(self.ctx, self.pos, self.mass, self.theta, cfg["leaf_size"])
            return pt.petar_force_long(self.ctx, cfg["group_size"], self.r_in, self.r_out,
                                       self.r_s, acc=self.acc, pot=self.pot,
                                       nb_capacity=self.nb_cap)
        # the whole step (tree build, force, neighbour lists) replayed as one
        # hipGraph
        return pt.petar_step_graph(self.ctx, self.pos, self.mass, self.theta, cfg["leaf_size"],
                                   cfg["group_size"], self.r_in, self.r_out, self.r_s, self.acc,
                                   self.pot, nb=self.nb_bufs)

    def timed(self, steps, warmup, graph=False, label=""):
        """Wall time per step over `steps` steps after `warmup` untimed ones;
        interactions and force-kernel time (HIP events) per step."""
        import torch
        pt, ctx = self.pt, self.ctx
        pt.petar_set_params(ctx, precision=pt.PETAR_MIXED, i_per_lane=self.cfg["i_per_lane"])
        for k in range(warmup):
            self(graph)
            log("%swarmup step %d done" % (label, k))
        torch.cuda.synchronize()
        inter, k_ms = [], []
        t0 = time.perf_counter()
        for _ in range(steps):
            self(graph)
            st = pt.petar_get_stats(ctx)
            inter.append(st["inter_pc"] + st["inter_far"] + st["inter_near"])
            k_ms.append(st["ms_force_kernel"])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        if graph:  # stage times are not visible inside a replay: one eager step
            self(False)
            k_ms = [pt.petar_get_stats(ctx)["ms_force_kernel"]]
        st = pt.petar_get_stats(ctx)
        ms_step = 1e3 * elapsed / steps
        out = {"ms_step": ms_step, "inter": float(np.mean(inter)),
               "kernel_ms": float(np.mean(k_ms)), "stats": st}
        log("%stimed %d steps: %.3f ms/step; force kernel %.3f ms; build %.3f ms; nb %.3f ms"
            % (label, steps, ms_step, out["kernel_ms"], st["ms_build"], st["ms_nb"]))
        return out

    def fp64_pass(self, reps=2):
        """The same force with FP64 pair arithmetic on the last tree: its
        kernel time and accelerations (left in self.acc)."""
        pt, ctx = self.pt, self.ctx
        pt.petar_set_params(ctx, precision=pt.PETAR_FP64, i_per_lane=self.cfg["i_per_lane"])
        ms = []
        for _ in range(reps):
            pt.petar_force_long(ctx, self.cfg["group_size"], self.r_in, self.r_out, self.r_s,
                                acc=self.acc, pot=self.pot)
            ms.append(pt.petar_get_stats(ctx)["ms_force_kernel"])
        pt.petar_set_params(ctx, precision=pt.PETAR_MIXED, i_per_lane=self.cfg["i_per_lane"])
        return ms[-1]


def oracle_sample(c, step, sample, threads):
    """FP64 direct sum of the changeover-weighted long-range force for the
    sampled targets (all sources) and its CPU time."""
    import oracle
    rin_h, rout_h = step.r_in.cpu().numpy(), step.r_out.cpu().numpy()
    t1 = time.perf_counter()
    a_ref, p_ref = oracle.force_long(c.pos, c.mass, rin_h, rout_h, idx=sample)
    return a_ref, p_ref, time.perf_counter() - t1


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plummer1m_b100")
    ap.add_argument("--theta", type=float, default=None)
    ap.add_argument("--leaf", type=int, default=None)
    ap.add_argument("--group", type=int, default=None)
    ap.add_argument("--ipl", type=int, default=None)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--graph", action="store_true",
                    help="replay the step as a hipGraph (the force kernel is then timed on one "
                         "eager step after the timed region)")
    ap.add_argument("--sample", type=int, default=4096, help="targets in the error / CPU sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg")
    ap.add_argument("--no-next-rows", dest="next_rows", action="store_false",
                    help="skip the second-stage filter, clusters, groups and artificial particles")
    ap.add_argument("--no-extras", dest="extras", action="store_false",
                    help="skip the theta scan, the batched and the 10M workloads")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (calibrates the "
                         "HBM byte counters of a profiler) and exit")
    ap.add_argument("--autotune", default=None, metavar="CACHE",
                    help="only run petar_autotune for every (workload, theta) of this benchmark "
                         "and petar_autotune_batch for the batched systems, adding what CACHE "
                         "lacks (the package reads paper_2006_16560_amd/tuned.jsonl), and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(one GPU's share of a sharded run is the single-GPU workload)", file=sys.stderr)
        return 2

    import torch
    import paper_2006_16560_amd as pt
    import workloads

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied %d bytes 5 times" % nbytes)
        return 0
    if args.autotune:
        return autotune(pt, workloads, args.autotune)
    if args.workload == "batched128":
        line = run_batched(pt, workloads, args, args.steps, args.warmup)
        print(json.dumps(line), flush=True)
        return 0 if (line["bitwise_batched_eq_sequential"] and line["bitwise_graph_eq_batched"]) \
            else 1
    wl = workloads.WORKLOADS[args.workload]
    theta = wl.theta if args.theta is None else args.theta
    n = wl.n

    t0 = time.time()
    c = workloads.make_cluster(n, args.seed, imf=wl.imf, binary_fraction=wl.binary_fraction)
    log("workload %s: N=%d generated in %.1fs" % (wl.name, n, time.time() - t0))

    dev = "cuda:0"
    pos = torch.from_numpy(c.pos).to(dev)
    mass = torch.from_numpy(c.mass).to(dev)
    ctx = pt.petar_create(0)
    cfg = pick_config(pt, ctx, n, theta, wl, args)
    log("launch configuration: %s" % json.dumps(cfg))
    step = Step(pt, ctx, wl, pos, mass, theta, cfg)
    res = step.timed(args.steps, args.warmup, graph=args.graph)
    st = res["stats"]
    ms_step, inter_step, kernel_ms = res["ms_step"], res["inter"], res["kernel_ms"]
    value = inter_step / (ms_step * 1e-3)
    achieved = inter_step * FLOPS_PER_INTERACTION / (kernel_ms * 1e-3) / 1e12
    log("interactions/step: pc %d far %d near %d" % (st["inter_pc"], st["inter_far"],
                                                    st["inter_near"]))

    # ---- accuracy on a seeded sample (outside the timed region)
    sample = workloads.sample_indices(n, args.sample, args.seed)
    acc_mixed = step.acc.cpu().numpy()[:, sample].copy()
    pot_mixed = step.pot.cpu().numpy()[sample].copy()
    fp64_ms = step.fp64_pass()
    torch.cuda.synchronize()
    acc64 = step.acc.cpu().numpy()[:, sample]
    log("fp64 force kernel %.3f ms (mixed %.3f ms)" % (fp64_ms, kernel_ms))
    e_arith = rel_err(acc_mixed, acc64)
    err = {"sample": int(sample.size),
           "p50_arith_vs_fp64gpu": float(np.median(e_arith)),
           "p99_arith_vs_fp64gpu": float(np.percentile(e_arith, 99))}

    cpu = None
    a_ref = None
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    if not args.no_cpu:
        a_ref, p_ref, dt = oracle_sample(c, step, sample, threads)
        pairs = float(sample.size) * (n - 1)
        cpu = {"value": pairs / dt, "unit": "interactions/s", "cores": threads, "kind": "oracle",
               "sample": "FP64 direct sum (changeover-weighted long-range force + potential) "
                         "for %d seeded targets x all %d sources, %.1f s" % (sample.size, n, dt),
               "extrapolated_full_direct_sum_s": float(n) * (n - 1) / (pairs / dt),
               "cpu_model": cpu_model()}
        e_tot = rel_err(acc_mixed, a_ref)
        e64 = rel_err(acc64, a_ref)
        err.update({"p50_vs_oracle": float(np.median(e_tot)),
                    "p99_vs_oracle": float(np.percentile(e_tot, 99)),
                    "p99_fp64gpu_vs_oracle": float(np.percentile(e64, 99)),
                    "p99_pot_vs_oracle": float(np.percentile(np.abs(pot_mixed / p_ref - 1), 99))})
        log("oracle sample: %.1f s on %d threads" % (dt, threads))

    fp32_ops = profiled_value(wl.name, cfg, "fp32_flops_per_launch")
    line = {
        "metric": "tree-force interactions/s and % FP32 peak at N=1M; p99 force rel. err vs FP64",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "n": n, "imf": "kroupa 0.08-150", "binary_fraction":
                   wl.binary_fraction, "theta": theta, "leaf_size": cfg["leaf_size"],
                   "group_size": cfg["group_size"], "i_per_lane": cfg["i_per_lane"],
                   "tuning": cfg["source"], "r_in_ref": wl.r_in_ref, "r_out_ref": wl.r_out_ref,
                   "search_factor": wl.search_factor, "precision": "mixed fp32 pair / fp64 tree",
                   "launch": "hipGraph replay" if args.graph else "eager",
                   "parallelism": "1 gpu"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": profiled_value(wl.name, cfg),
                     "counter_fp32_tflops": (fp32_ops / (kernel_ms * 1e-3) / 1e12
                                             if fp32_ops else None),
                     "kernel": "k_force<float, %d, false>" % cfg["i_per_lane"],
                     "kernel_ms": kernel_ms,
                     "flops_per_interaction": FLOPS_PER_INTERACTION,
                     "interactions_per_launch": inter_step},
        "cpu_baseline": cpu,
        "particles_per_s": n / (ms_step * 1e-3),
        "interactions": {"pc": st["inter_pc"], "far": st["inter_far"], "near": st["inter_near"]},
        "stages_ms": {"build": st["ms_build"], "force_total": st["ms_force"],
                      "force_kernel": kernel_ms, "neighbours": st["ms_nb"]},
        "neighbour_entries": st["nb_total"],
        "errors": err,
        "fp64_gpu": {"force_kernel_ms": fp64_ms, "mixed_speedup": fp64_ms / kernel_ms},
        "workspace_bytes": st["workspace_bytes"],
    }

    if args.extras and not args.graph and args.theta is None and args.workload == "plummer1m_b100":
        scan_steps = max(1, min(args.steps, 5))
        line["theta_scan"] = theta_scan(pt, ctx, wl, c, pos, mass, args, sample, a_ref,
                                        scan_steps)
    if args.next_rows:
        line["next_rows"] = bench_next_rows(pt, ctx, c, wl, theta, cfg, dev)
    pt.petar_destroy(ctx)
    del step
    torch.cuda.empty_cache()
    if args.extras and args.workload == "plummer1m_b100":
        line["batched128"] = run_batched(pt, workloads, args, max(1, min(args.steps, 5)), 1)
        torch.cuda.empty_cache()
        line["plummer10m_b10"] = run_10m(pt, workloads, args, threads)
    print(json.dumps(line), flush=True)
    return 0


# (workload, theta) pairs whose launch configuration the autotuner picks: the
# 1M cluster at the paper's opening angles and the 10M cluster at theta 0.5
TUNED_JOBS = [("plummer1m_b100", 0.5), ("plummer1m_b100", 0.3), ("plummer1m_b100", 0.7),
              ("plummer10m_b10", 0.5)]


def autotune(pt, workloads, cache) -> int:
    """petar_autotune on each job's particles and radii, and
    petar_autotune_batch on the batched systems: they time a full step for
    every candidate leaf size, group size and number of targets per lane and
    append the fastest to `cache` (keyed by floor(log2 N), floor(log2 n_sys),
    theta and precision). Jobs already in the cache are kept (a cache hit
    launches nothing): remove the file to tune afresh."""
    import torch
    dev = "cuda:0"
    made = {}
    for name, theta in TUNED_JOBS:
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
            log(json.dumps({"workload": name, "theta": theta, "tuned": best,
                            "seconds": round(time.time() - t0, 1)}))
        finally:
            pt.petar_destroy(ctx)
    made.clear()
    torch.cuda.empty_cache()
    ctx = pt.petar_create(0)
    try:
        pt.petar_set_params(ctx, precision=pt.PETAR_MIXED)
        offs, pos, mass, r_in, r_out, r_s = batched_inputs(pt, workloads, ctx, 0)
        t0 = time.time()
        best = pt.petar_autotune_batch(ctx, offs, pos, mass, BATCHED_THETA, r_in, r_out, r_s,
                                       cache_path=cache)
        log(json.dumps({"workload": "batched128", "theta": BATCHED_THETA, "tuned": best,
                        "seconds": round(time.time() - t0, 1)}))
    finally:
        pt.petar_destroy(ctx)
    return 0


def theta_scan(pt, ctx, wl, c, pos, mass, args, sample, a_ref, steps):
    """The 1M workload at the paper's other opening angles (Table inpar runs
    theta 0.3 and 0.5), each with its own tuned launch configuration."""
    out = {}
    for th in (0.3, 0.7):
        cfg = pick_config(pt, ctx, wl.n, th, wl, args)
        step = Step(pt, ctx, wl, pos, mass, th, cfg)
        res = step.timed(steps, 1, label="theta %g: " % th)
        st = res["stats"]
        acc_m = step.acc.cpu().numpy()[:, sample].copy()
        fp64_ms = step.fp64_pass(1)
        acc64 = step.acc.cpu().numpy()[:, sample]
        e = rel_err(acc_m, acc64)
        r = {"leaf_size": cfg["leaf_size"], "group_size": cfg["group_size"],
             "i_per_lane": cfg["i_per_lane"], "tuning": cfg["source"],
             "steps": steps, "ms_per_step": res["ms_step"],
             "interactions_per_s": res["inter"] / (res["ms_step"] * 1e-3),
             "particles_per_s": wl.n / (res["ms_step"] * 1e-3),
             "force_kernel_ms": res["kernel_ms"],
             "frac": res["inter"] * FLOPS_PER_INTERACTION / (res["kernel_ms"] * 1e-3) / 1e12
             / PEAK_FP32_TFLOPS,
             "interactions": {"pc": st["inter_pc"], "far": st["inter_far"],
                              "near": st["inter_near"]},
             "fp64_force_kernel_ms": fp64_ms,
             "p50_arith_vs_fp64gpu": float(np.median(e)),
             "p99_arith_vs_fp64gpu": float(np.percentile(e, 99))}
        if a_ref is not None:
            et = rel_err(acc_m, a_ref)
            r.update({"p50_vs_oracle": float(np.median(et)),
                      "p99_vs_oracle": float(np.percentile(et, 99)),
                      "p99_fp64gpu_vs_oracle": float(np.percentile(rel_err(acc64, a_ref), 99))})
        out["%g" % th] = r
        del step
    return out


def run_10m(pt, workloads, args, threads):
    """N = 10M (10% binaries), theta 0.5: the mixed step against the same
    walk with FP64 pair arithmetic, library workspace and device memory."""
    import torch
    wl = workloads.WORKLOADS["plummer10m_b10"]
    t0 = time.time()
    c = workloads.make_cluster(wl.n, args.seed, imf=wl.imf, binary_fraction=wl.binary_fraction)
    log("workload %s: N=%d generated in %.1fs" % (wl.name, wl.n, time.time() - t0))
    dev = "cuda:0"
    free0, total = torch.cuda.mem_get_info(0)
    pos = torch.from_numpy(c.pos).to(dev)
    mass = torch.from_numpy(c.mass).to(dev)
    ctx = pt.petar_create(0)
    try:
        cfg = pick_config(pt, ctx, wl.n, wl.theta, wl, args)
        step = Step(pt, ctx, wl, pos, mass, wl.theta, cfg, nb_per_particle=16)
        res = step.timed(3, 1, label="10M: ")
        free1, _ = torch.cuda.mem_get_info(0)
        st = res["stats"]
        sample = workloads.sample_indices(wl.n, args.sample, args.seed)
        acc_m = step.acc.cpu().numpy()[:, sample].copy()
        fp64_ms = step.fp64_pass()
        acc64 = step.acc.cpu().numpy()[:, sample]
        e = rel_err(acc_m, acc64)
        out = {"n": wl.n, "theta": wl.theta, "leaf_size": cfg["leaf_size"],
               "group_size": cfg["group_size"], "i_per_lane": cfg["i_per_lane"],
               "tuning": cfg["source"], "steps": 3, "ms_per_step": res["ms_step"],
               "interactions_per_s": res["inter"] / (res["ms_step"] * 1e-3),
               "particles_per_s": wl.n / (res["ms_step"] * 1e-3),
               "force_kernel_ms": res["kernel_ms"],
               "frac": res["inter"] * FLOPS_PER_INTERACTION / (res["kernel_ms"] * 1e-3) / 1e12
               / PEAK_FP32_TFLOPS,
               "interactions": {"pc": st["inter_pc"], "far": st["inter_far"],
                                "near": st["inter_near"]},
               "stages_ms": {"build": st["ms_build"], "force_total": st["ms_force"],
                             "neighbours": st["ms_nb"]},
               "fp64_gpu": {"force_kernel_ms": fp64_ms, "mixed_speedup": fp64_ms /
                            res["kernel_ms"]},
               "errors": {"sample": int(sample.size),
                          "p50_arith_vs_fp64gpu": float(np.median(e)),
                          "p99_arith_vs_fp64gpu": float(np.percentile(e, 99))},
               "memory": {"workspace_bytes": st["workspace_bytes"],
                          "io_bytes": int(sum(t.numel() * t.element_size() for t in
                                              (pos, mass, step.r_in, step.r_out, step.r_s,
                                               step.acc, step.pot, *step.nb_bufs))),
                          "device_bytes_used_by_step": int(free0 - free1),
                          "device_total_bytes": int(total)}}
        if not args.no_cpu:  # a small oracle sample: 256 targets x all 10M sources
            s = sample[:: max(1, sample.size // 256)][:256]
            a_ref, _, dt = oracle_sample(c, step, s, threads)
            k = np.searchsorted(sample, s)
            out["errors"].update({"oracle_sample": int(s.size),
                                  "p99_vs_oracle": float(np.percentile(rel_err(acc_m[:, k], a_ref),
                                                                       99)),
                                  "p99_fp64gpu_vs_oracle": float(np.percentile(
                                      rel_err(acc64[:, k], a_ref), 99)),
                                  "oracle_s": dt})
        log("10M: %s" % json.dumps(out))
        del step
        return out
    finally:
        pt.petar_destroy(ctx)
        torch.cuda.empty_cache()


def bench_next_rows(pt, ctx, c, wl, theta, cfg, dev, reps=5):
    """Second-stage neighbour filter (Kepler pericentre, c_v = 1.5) and
    clusters on the same particles with velocity-dependent search radii
    (eq. rnb, C_r = 3), for two sets of changeover radii: those of the
    benchmark workload (long step r_out,ref / (10 sigma_1D), eq. routdts)
    and the paper's own for a million stars in binaries (Table inpar, N1mkb).
    Then SDAR groups and artificial particles. Outside the timed region of
    the step; times are device-synchronised wall clock."""
    v2 = (c.vel ** 2).sum(axis=0)
    sigma = float(np.sqrt((c.mass * v2).sum() / (3.0 * c.mass.sum())))
    out = next_rows_for(pt, ctx, c, wl.r_out_ref, wl.r_out_ref / (10.0 * sigma), theta, cfg, dev,
                        reps, "workload radii")
    out["paper_n1mkb_radii"] = next_rows_for(pt, ctx, c, N1MKB_R_OUT_REF, N1MKB_DT, theta, cfg,
                                             dev, reps, "Table inpar N1mkb radii")
    out["groups_and_artificial"] = bench_artificial(pt, ctx, c, wl, theta, cfg, dev, reps)
    return out


def next_rows_for(pt, ctx, c, r_out_ref, dt, theta, cfg, dev, reps, label):
    import torch
    n = c.mass.size
    mass = torch.from_numpy(c.mass).to(dev)
    vel = torch.from_numpy(c.vel).to(dev)
    pos = torch.from_numpy(c.pos).to(dev)
    ri, ro, rnb = pt.petar_changeover_radii(ctx, mass, 0.1 * r_out_ref, r_out_ref, 1.2, vel=vel,
                                            cr_dt=3.0 * dt)
    pt.petar_set_params(ctx, precision=pt.PETAR_MIXED, i_per_lane=cfg["i_per_lane"])
    pt.petar_tree_build(ctx, pos, mass, theta, cfg["leaf_size"])
    _, _, (offs, idx) = pt.force_long_with_retry(ctx, cfg["group_size"], ri, ro, rnb, 64 * n)
    t_f, t_c = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f_off, f_idx = pt.petar_nb_filter(ctx, pos, vel, mass, rnb, 1.5, offs, idx)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        label_, cl, members = pt.petar_clusters(ctx, f_off, f_idx)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        t_f.append(t1 - t0)
        t_c.append(t2 - t1)
    sizes = torch.diff(cl).cpu().numpy()
    out = {"nb_filter_ms": 1e3 * float(np.median(t_f)), "clusters_ms": 1e3 * float(np.median(t_c)),
           "candidates": int(idx.numel()), "kept": int(f_idx.numel()),
           "n_clusters": int(sizes.size), "largest_cluster": int(sizes.max()),
           "particles_in_clusters_gt1": int(sizes[sizes > 1].sum()),
           "radii": "%s: r_out,ref = %.6g, r_in,ref = r_out,ref/10, eq. rnb with C_r = 3, "
                    "dt = %.4g" % (label, r_out_ref, dt)}
    log("next rows (%s): filter %.3f ms, clusters %.3f ms, %d -> %d pairs, %d clusters "
        "(largest %d)" % (label, out["nb_filter_ms"], out["clusters_ms"], out["candidates"],
                          out["kept"], out["n_clusters"], out["largest_cluster"]))
    return out


def bench_artificial(pt, ctx, c, wl, theta, cfg, dev, reps=5, order=3):
    """SDAR groups (eq. rbin) from the neighbour lists of the step's radii,
    the artificial set of the bound binaries (third-order tidal tensor and
    pseudoparticles), tree build and long-range force on that set, post-fit
    and kick: each stage's median device-synchronised wall time."""
    import torch
    n = wl.n
    leaf, group = cfg["leaf_size"], cfg["group_size"]
    pos = torch.from_numpy(c.pos).to(dev)
    vel = torch.from_numpy(c.vel).to(dev)
    mass = torch.from_numpy(c.mass).to(dev)
    ri, ro, rs = pt.petar_changeover_radii(ctx, mass, wl.r_in_ref, wl.r_out_ref, wl.search_factor)
    pt.petar_set_params(ctx, precision=pt.PETAR_MIXED, i_per_lane=cfg["i_per_lane"])
    pt.petar_tree_build(ctx, pos, mass, theta, leaf)
    _, _, (offs, idx) = pt.force_long_with_retry(ctx, group, ri, ro, rs, 64 * n)
    times = {k: [] for k in ("groups", "make", "set_build", "set_force", "fit", "kick")}

    def timed(key, fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        times[key].append(time.perf_counter() - t0)
        return r

    cfg_set = None
    for _ in range(reps):
        pt.petar_set_params(ctx, precision=pt.PETAR_MIXED, i_per_lane=cfg["i_per_lane"])
        label, go, members, pairs = timed(
            "groups", lambda: pt.petar_groups(ctx, pos, vel, mass, ri, theta, offs, idx))
        g = timed("make", lambda: pt.petar_artificial_make(ctx, pos, vel, mass, ri, ro, rs, pairs,
                                                           order, 1.0))
        if cfg_set is None:  # the set's own launch configuration (autotuner's cache)
            cfg_set = pt.launch_config(ctx, int(g["mass"].numel()), theta, leaf_default=leaf,
                                       group_default=group, ipl_default=cfg["i_per_lane"])
        pt.petar_set_params(ctx, precision=pt.PETAR_MIXED, i_per_lane=cfg_set["i_per_lane"])
        timed("set_build", lambda: pt.petar_tree_build(ctx, g["pos"], g["mass"], theta,
                                                       cfg_set["leaf_size"]))
        # pseudoparticles act as sources only: the force is wanted on the
        # singles, centres and measure points
        pt.petar_set_targets(ctx, g["target"])
        a_set, p_set = timed("set_force", lambda: pt.petar_force_long(
            ctx, cfg_set["group_size"], g["r_in"], g["r_out"], g["r_search"]))
        st = pt.petar_get_stats(ctx)
        ten, acc, pot = timed("fit", lambda: pt.petar_tidal_fit(ctx, g, pairs, a_set, p_set,
                                                                pos=pos))
        v = vel.clone()
        timed("kick", lambda: pt.petar_kick(ctx, v, acc, 0.5 * wl.r_out_ref))
    out = {k + "_ms": 1e3 * float(np.median(t)) for k, t in times.items()}
    out.update({"order": order, "n_groups": int(go.numel() - 1), "binaries": int(pairs.shape[1]),
                "set_particles": int(g["mass"].numel()),
                "set_targets": int(g["target"].sum().item()),
                "set_interactions": int(st["inter_pc"] + st["inter_far"] + st["inter_near"]),
                "set_force_kernel_ms": st["ms_force_kernel"],
                "set_launch": {"leaf_size": cfg_set["leaf_size"],
                               "group_size": cfg_set["group_size"],
                               "i_per_lane": cfg_set["i_per_lane"], "tuning": cfg_set["source"]}})
    log("groups/artificial: %s" % json.dumps(out))
    return out


BATCHED_THETA = 0.5


def batched_inputs(pt, workloads, ctx, seed):
    """The 128 systems of the batched workload on the device: offsets (list),
    positions, masses and each system's own changeover and search radii
    (eq. rcut with the system's <m> and r_out,ref ~ N^-1/3)."""
    import torch
    t0 = time.time()
    offs, pos_h, vel_h, mass_h, sizes = workloads.make_batched(seed)
    n = int(offs[-1])
    log("batched workload: %d systems, N=%d generated in %.1fs" % (sizes.size, n, time.time() - t0))
    dev = "cuda:0"
    pos = torch.from_numpy(pos_h).to(dev)
    mass = torch.from_numpy(mass_h).to(dev)
    r_in = torch.empty(n, dtype=torch.float64, device=dev)
    r_out, r_s = torch.empty_like(r_in), torch.empty_like(r_in)
    for k in range(sizes.size):
        a, b = int(offs[k]), int(offs[k + 1])
        ro = workloads.r_out_ref_for(int(sizes[k]))
        pt.petar_changeover_radii(ctx, mass[a:b], 0.1 * ro, ro, 1.2,
                                  out=(r_in[a:b], r_out[a:b], r_s[a:b]))
    return [int(v) for v in offs], pos, mass, r_in, r_out, r_s


def run_batched(pt, workloads, args, steps, warmup) -> dict:
    """128 independent clusters (N log-uniform in [1024, 131072], 20% binaries).

    Three ways to run the same step (tree build + long-range force +
    neighbour lists): the whole batched step replayed as one hipGraph, the
    batched step launched eagerly, and 128 sequential per-cluster calls. The
    batched outputs must equal the sequential ones bit for bit.
    """
    import torch

    theta = BATCHED_THETA if args.theta is None else args.theta
    ctx = pt.petar_create(0)
    ctx_g = pt.petar_create(0)
    try:
        pt.petar_set_params(ctx, precision=pt.PETAR_MIXED)
        offs_l, pos, mass, r_in, r_out, r_s = batched_inputs(pt, workloads, ctx, args.seed)
        n = offs_l[-1]
        n_sys = len(offs_l) - 1
        dev = pos.device
        cfg = pt.launch_config(ctx, n, theta, leaf_default=8, group_default=64, ipl_default=2,
                               n_sys=n_sys)
        over = {"leaf_size": args.leaf, "group_size": args.group, "i_per_lane": args.ipl}
        for k, v in over.items():
            if v is not None:
                cfg[k] = v
                cfg["source"] = "command line"
        leaf, group, ipl = cfg["leaf_size"], cfg["group_size"], cfg["i_per_lane"]
        for c in (ctx, ctx_g):
            pt.petar_set_params(c, precision=pt.PETAR_MIXED, i_per_lane=ipl)
        nb_cap = 64 * n
        acc_b = torch.empty((3, n), dtype=torch.float64, device=dev)
        pot_b = torch.empty(n, dtype=torch.float64, device=dev)
        acc_g, pot_g = torch.empty_like(acc_b), torch.empty_like(pot_b)
        acc_s, pot_s = torch.empty_like(acc_b), torch.empty_like(pot_b)
        nb_g = (torch.empty(n + 1, dtype=torch.int64, device=dev),
                torch.empty(nb_cap, dtype=torch.int32, device=dev))

        def graph():
            pt.petar_step_graph(ctx_g, pos, mass, theta, leaf, group, r_in, r_out, r_s, acc_g,
                                pot_g, sys_offsets=offs_l, nb=nb_g)

        def batched():
            pt.petar_batch_build(ctx, offs_l, pos, mass, theta, leaf)
            return pt.petar_force_long(ctx, group, r_in, r_out, r_s, acc=acc_b, pot=pot_b,
                                       nb_capacity=nb_cap)

        def sequential():
            tot = 0
            for k in range(n_sys):
                a, b = offs_l[k], offs_l[k + 1]
                pt.petar_batch_build(ctx, [0, b - a], pos[:, a:b].contiguous(), mass[a:b], theta,
                                     leaf)
                acc_k, pot_k, _ = pt.petar_force_long(ctx, group, r_in[a:b], r_out[a:b],
                                                      r_s[a:b], nb_capacity=64 * (b - a))
                acc_s[:, a:b] = acc_k
                pot_s[a:b] = pot_k
                st = pt.petar_get_stats(ctx)
                tot += st["inter_pc"] + st["inter_far"] + st["inter_near"]
            return tot

        def timed(fn, k):
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(k):
                fn()
            torch.cuda.synchronize()
            return 1e3 * (time.perf_counter() - t) / k

        for _ in range(warmup):
            graph()
            batched()
        ms_g = timed(graph, steps)
        ms_b = timed(batched, steps)
        st = pt.petar_get_stats(ctx)
        inter = st["inter_pc"] + st["inter_far"] + st["inter_near"]
        inter_seq = sequential()
        ms_s = timed(sequential, 1)
        same_b = bool(torch.equal(acc_b, acc_s) and torch.equal(pot_b, pot_s))
        same_g = bool(torch.equal(acc_g, acc_b) and torch.equal(pot_g, pot_b))
        log("batched: graph %.3f ms/step, eager %.3f ms/step, sequential %.3f ms/step; "
            "bitwise batched==sequential %s, graph==batched %s"
            % (ms_g, ms_b, ms_s, same_b, same_g))
        return {
            "metric": "tree-force interactions/s (batched clusters)",
            "value": inter / (ms_g * 1e-3), "unit": "interactions/s", "n_gpus": 1,
            "steps": steps, "warmup": warmup, "ms_per_step": ms_g,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "batched128", "n_systems": n_sys, "n": n,
                       "theta": theta, "leaf_size": leaf, "group_size": group,
                       "i_per_lane": ipl, "tuning": cfg["source"], "binary_fraction": 0.2,
                       "mode": "hipGraph replay of the batched step"},
            "batched_eager_ms_per_step": ms_b, "sequential_ms_per_step": ms_s,
            "speedup_vs_sequential": ms_s / ms_g,
            "bitwise_batched_eq_sequential": same_b, "bitwise_graph_eq_batched": same_g,
            "interactions": inter, "interactions_sequential": inter_seq,
            "stages_ms": {"build": st["ms_build"], "force_total": st["ms_force"],
                          "force_kernel": st["ms_force_kernel"], "neighbours": st["ms_nb"]},
        }
    finally:
        pt.petar_destroy(ctx)
        pt.petar_destroy(ctx_g)


if __name__ == "__main__":
    sys.exit(main())
