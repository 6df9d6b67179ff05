#!/usr/bin/env python3
"""Benchmark of the fused two-component MRT lattice step on one MI355X.

Workload: the 3-D co-flow device, D3Q19, 600 x 120 x 120 fluid nodes (square
channel with a one-node wall shell, box 600 x 122 x 122), coaxial 30 x 30
dispersed-phase inlet, corrected inlet and outlet, viscosity ratio 5,
G12 = 0.9.  One step is the whole hot path: forces, MRT collision, streaming,
alpha-corrected inlet and the mass-flow corrected outlet.

Prints one JSON line: MLUPS (fluid nodes x steps / s / 1e6) with the inputs
resident in HBM, the roofline of the dominant kernel (HBM bytes of the
algorithm: read and write every population once, 2 Q C b_f bytes per fluid
node) and the FP64 CPU oracle timed on the host cores on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (2-comp MRT) + %HBM peak; batched/surrogate vs plain at stated error"
# rocprofv3 summary of the node update on this workload (HBM bytes per launch
# from FETCH_SIZE and WRITE_SIZE, scaled by the calibration kernel)
PROFILE = os.path.join(ROOT, "profiles", "k_main_coflow3d_600x120x120_f32.md")
KERNEL_SOURCES = ["kernels.h", "lattice.h", "params.h", "launch.h", "launch_impl.h", "k3d.hip"]


def sources_sha():
    """Digest of the sources the node update is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2512_12934_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic():
    """HBM bytes per launch of the node update as profiled, or None when the
    profile is missing or was taken from other kernel sources."""
    import re
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    m = re.search(r"traffic_per_launch: fetch_bytes=(\d+) write_bytes=(\d+) sources_sha256=([0-9a-f]+)", text)
    if not m or m.group(3) != sources_sha():
        return None
    return int(m.group(1)) + int(m.group(2))
HBM_PEAK_GBS = 8000.0
GRAPH_STEPS = 16


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", choices=["f32", "f16"], default="f32")
    ap.add_argument("--length", type=int, default=600)
    ap.add_argument("--width", type=int, default=120)
    ap.add_argument("--inner", type=int, default=30)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate CPU time budget of the oracle baseline (0 disables it)")
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary FP16, 2-D and batched measurements")
    ap.add_argument("--batch-members", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=400)
    ap.add_argument("--batch-only", action="store_true",
                    help="only time the batched sweep (no one-by-one comparison): a short run for profilers")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (scale reference for HBM counters)")
    return ap.parse_args()


def batched(args, dev, t0, t1, compare=True):
    """The 256-instance T-junction sweep (W 32..128, FP16-offset storage):
    one batch (one launch per stage for all members, graph-replayed) against
    the same members stepped one context at a time (compare=False skips the
    one-at-a-time leg)."""
    import torch
    from paper_2512_12934_amd import cases
    from paper_2512_12934_amd.lbm import Batch, lib
    cs = cases.sweep(args.batch_members)
    fluid = sum(c.fluid_nodes for c in cs)
    tc = time.perf_counter()
    b = Batch(cs, storage="f16", device=dev)
    t_create = time.perf_counter() - tc
    b.set_graph_steps(GRAPH_STEPS)
    b.step(32)
    torch.cuda.synchronize()
    nb = args.batch_steps
    t0.record(b.stream)
    b.step(nb)
    t1.record(b.stream)
    torch.cuda.synchronize()
    mb = t0.elapsed_time(t1) / nb
    if not compare:
        del b
        torch.cuda.empty_cache()
        return {"members": len(cs), "fluid_nodes": fluid, "storage": "f16",
                "batched_ms_per_step": round(mb, 4), "batched_MLUPS": round(fluid / (mb / 1e3) / 1e6, 1),
                "create_s": round(t_create, 2)}
    # the same members, one context at a time (plain launches, as a caller
    # without the batch would run them)
    L = lib()
    ns = max(4, nb // 16)
    for m in b.members:
        m.set_graph_steps(0)
    t0.record(b.stream)
    for m in b.members:
        L.lbm_step(m._h, ns)
    t1.record(b.stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / ns
    del b
    torch.cuda.empty_cache()
    return {"members": len(cs), "fluid_nodes": fluid, "storage": "f16",
            "batched_ms_per_step": round(mb, 4), "batched_MLUPS": round(fluid / (mb / 1e3) / 1e6, 1),
            "one_by_one_ms_per_step": round(ms, 4), "one_by_one_MLUPS": round(fluid / (ms / 1e3) / 1e6, 1),
            "speedup": round(ms / mb, 2), "create_s": round(t_create, 2)}


def surrogate(dev, t0, t1, batch):
    """Ensemble inference (5 members, MLP 4 -> 128 -> 128 -> 2, layer 2 on BF16
    MFMA) over 4096 queries, timed live, beside the cost of the LBM run that
    a query replaces: one member's share of the batched sweep just timed, over
    a 320,000-step labelling run.  The weights are seeded random: inference
    cost does not depend on them.  The accuracy of a trained ensemble comes
    from the held-out study, not from this timing."""
    import torch
    from paper_2512_12934_amd.surrogate import Surrogate
    n, reps, label_steps = 4096, 50, 320000
    stream = torch.cuda.current_stream(dev)
    s = Surrogate(members=5, hidden=128, max_n=n, seed=7, device=dev, stream=stream)
    g = torch.Generator(device="cpu").manual_seed(11)
    X = torch.rand((n, 4), generator=g).to(dev)
    s.predict(X)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(reps):
        s.predict(X)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    s.close()
    q = ms / 1e3 / n
    out = {"members": 5, "queries": n, "predict_ms": round(ms, 4), "s_per_query": q}
    if batch:
        run_s = batch["batched_ms_per_step"] / 1e3 * label_steps / batch["members"]
        out.update({"lbm_run_s": round(run_s, 4), "lbm_run": f"{label_steps} steps of one sweep member, batched",
                    "cost_ratio": round(run_s / q, 1)})
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seconds):
    """The FP64 oracle (test infrastructure, never tuned) on the host cores:
    the co-flow device at 1/4 scale, about `seconds` of steps with every
    OpenMP thread the oracle runs with, then a quarter of that budget on one
    thread."""
    import oracle
    from paper_2512_12934_amd import cases
    q = cases.coflow3d_quarter()

    def rate(budget):
        o = oracle.Sim(q)
        o.step(1)
        t = time.perf_counter()
        o.step(2)
        per = (time.perf_counter() - t) / 2
        nsteps = max(2, int(budget / per))
        t = time.perf_counter()
        o.step(nsteps)
        dt = time.perf_counter() - t
        o.close()
        return q.fluid_nodes * nsteps / dt / 1e6, nsteps, dt

    threads = oracle.threads()
    v, nsteps, dt = rate(seconds)
    oracle.set_threads(1)
    v1, n1, dt1 = rate(seconds / 4)
    oracle.set_threads(threads)
    return {"value": round(v, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle, co-flow device at 1/4 scale (150x30x30 fluid, D3Q19), {nsteps} steps, "
                      f"{dt:.1f} s on {threads} OpenMP threads",
            "cpu_model": cpu_model(), "one_thread_MLUPS": round(v1, 3),
            "one_thread_sample": f"{n1} steps, {dt1:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this implementation runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU decomposition is a design, not an executable path.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            torch.mul(a, 2.0, out=b)      # one elementwise kernel: reads a, writes b
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": n * 4, "launches": 5}), flush=True)
        return

    from paper_2512_12934_amd import cases
    from paper_2512_12934_amd.lbm import LBM

    dev = torch.device("cuda:0")
    if args.batch_only:
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        print(json.dumps({"batched_sweep": batched(args, dev, t0, t1, compare=False)}), flush=True)
        return
    # the rates plain streaming kernels reach here: the practical ceiling
    # next to the published peak
    from paper_2512_12934_amd.lbm import stream_probe
    practical = stream_probe(device=dev)
    print(f"[bench] stream probe {practical} GB/s", file=sys.stderr, flush=True)
    case = cases.coflow3d(length=args.length, width=args.width, inner=args.inner)
    fluid = case.fluid_nodes
    print(f"[bench] building {case.name} box {case.n} fluid {fluid}", file=sys.stderr, flush=True)
    sim = LBM(case, storage=args.storage, device=dev, tile_config="auto")
    stream = sim.stream
    # set-up: capture and upload the step graphs of both A/B parities now, so
    # the timed region replays graphs and never captures one
    sim.set_graph_steps(GRAPH_STEPS)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    sim.step(args.steps)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    ms_step = ms / args.steps
    mlups = fluid * args.steps / (ms / 1e3) / 1e6
    print(f"[bench] {ms_step:.4f} ms/step, {mlups:.1f} MLUPS", file=sys.stderr, flush=True)

    # roofline of the fused node update, timed per launch with HIP events on
    # the context stream
    kms = sim.time_kernels(args.steps)
    bf = 4 if args.storage == "f32" else 2
    Q = 19
    b_alg = 2 * Q * 2 * bf            # bytes per fluid node per step: read and write every population once
    two_pass = kms[4] > 0
    # algorithmic bytes of one launch of the node update: every population of
    # every fluid node read and written once (a density pass, where there is
    # one, is overhead counted against the step, not against the kernel)
    achieved = fluid * b_alg / (kms[0] / 1e3) / 1e9
    step_gbs = fluid * b_alg / (ms_step / 1e3) / 1e9
    flux = sim.mass_flux()
    finite = bool(np.isfinite(flux["mass"]).all())
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": profiled_traffic() if args.storage == "f32" and args.length == 600 else None,
            "kernel": "k_main<3,%d>" % (0 if args.storage == "f32" else 1),
            "kernel_ms": round(kms[0], 5), "bytes_per_node": b_alg, "nodes_per_launch": fluid,
            "step_achieved": round(step_gbs, 1), "step_frac": round(step_gbs / HBM_PEAK_GBS, 4),
            "mode": "two-pass (k_psi + k_main)" if two_pass else "fused (k_main only)",
            "tile_config": sim.tile_config,
            "stream_probe_GBs": practical}
    del sim
    torch.cuda.empty_cache()

    extra = {}
    if not args.no_extra:
        # FP16-offset storage of the same workload, and the 2-D T-junction
        other = "f16" if args.storage == "f32" else "f32"
        s2 = LBM(case, storage=other, device=dev, tile_config="auto")
        s2.set_graph_steps(GRAPH_STEPS)
        s2.step(10)
        torch.cuda.synchronize()
        t0.record(s2.stream)
        s2.step(args.steps)
        t1.record(s2.stream)
        torch.cuda.synchronize()
        m2 = t0.elapsed_time(t1) / args.steps
        extra[f"{other}_storage"] = {"ms_per_step": round(m2, 4), "MLUPS": round(fluid / (m2 / 1e3) / 1e6, 1)}
        del s2
        tj = cases.tjunction()
        s3 = LBM(tj, storage="f32", device=dev, tile_config="auto")
        s3.set_graph_steps(GRAPH_STEPS)
        s3.step(50)
        torch.cuda.synchronize()
        n3 = 2000
        t0.record(s3.stream)
        s3.step(n3)
        t1.record(s3.stream)
        torch.cuda.synchronize()
        m3 = t0.elapsed_time(t1) / n3
        extra["tjunction_800x100_d2q9_f32"] = {"ms_per_step": round(m3, 4),
                                               "MLUPS": round(tj.fluid_nodes / (m3 / 1e3) / 1e6, 1)}
        del s3
        torch.cuda.empty_cache()
        extra["batched_sweep"] = batched(args, dev, t0, t1)
        extra["surrogate"] = surrogate(dev, t0, t1, extra["batched_sweep"])

    cpu = None
    if args.cpu_seconds > 0:
        cpu = cpu_baseline(args.cpu_seconds)

    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"co-flow device D3Q19 {args.length}x{args.width}x{args.width} fluid "
                               f"(box {case.n[0]}x{case.n[1]}x{case.n[2]}), inner inlet {args.inner}x{args.inner}, "
                               f"M=5, G12=0.9, corrected inlet/outlet",
                   "storage": args.storage, "fluid_nodes": fluid, "box_nodes": case.N},
        "hbm_frac_step": round(step_gbs / HBM_PEAK_GBS, 4),
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernel_ms": {"main": kms[0], "psi": kms[4], "faces": kms[1], "inlet_uc": kms[2], "outlet_fill": kms[3]},
        "finite": finite,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
