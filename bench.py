"""Benchmark: batched MOREA objective evaluation on one MI355X.

A step is one full evaluation (all three objectives, fold flags, severity and
sample counts) of the population of 512 dual-dynamic mesh candidates on the
128x128x96 synthetic abdominal phantom pair with a 10x10x8-point Kuhn mesh
(3,402 tets), 6 organs (one missing in the target), 200 guidance points in 5
sets.  Inputs are seeded and synthetic and already resident in HBM when the
timed region starts.

Prints one JSON line (see the design doc for every field).  --gpus above 1 is
refused: this build evaluates on one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SAMPLE_OPS = 60           # algorithmic VALU lane-ops per voxel sample (map, trilinear, h, sums)
SAMPLE_BYTES = 9          # algorithmic bytes per sample at FP32 storage (own voxel, footprint, band)
VALU_PEAK = 256 * 64 * 2.4e9   # lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz (packed FP32 disabled)
HBM_PEAK = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="CPU time budget of the oracle baseline sample (0 = skip)")
    ap.add_argument("--parity-samples", type=int, default=3)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this size first (counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; --gpus %d refused"
                          % args.gpus}), flush=True)
        sys.exit(2)
    import torch

    import paper_2303_04873_amd as morea
    import synth

    torch.cuda.set_device(0)
    t0 = time.time()
    p = synth.make_problem(args.config)
    pop_np = synth.make_population(p)
    pop = pop_np.shape[0]
    print(f"# inputs ready in {time.time() - t0:.1f}s: dims {p.dims}, {p.n_tets} tets, pop {pop}",
          file=sys.stderr, flush=True)
    prob = morea.Problem.from_synth(p, max_population=pop)
    pts = torch.from_numpy(pop_np).cuda()
    out = prob.outputs(pop)
    stream = torch.cuda.current_stream()

    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        prob.eval_full(pts, out=out)
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        ev[s][0].record(stream)
        prob.eval_full(pts, out=out)
        ev[s][1].record(stream)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    ms_per_step = (t_end - t_start) * 1e3 / args.steps
    launch_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))

    g = {k: v.cpu().numpy() for k, v in out.items()}
    samples = int(g["counts"].astype(np.int64).sum())
    evals_per_s = pop / (ms_per_step * 1e-3)
    samples_per_s = samples / (ms_per_step * 1e-3)

    # parity of this very output against the oracle on a few candidates
    parity = None
    cpu = None
    if args.parity_samples > 0 or args.cpu_seconds > 0:
        import oracle
        op = oracle.Problem.from_synth(p)
        if args.parity_samples > 0:
            idx = np.linspace(0, pop - 1, args.parity_samples).astype(int)
            o = op.evaluate(pop_np[idx])
            ok = (g["flags"][idx] == o["flags"]).all() and (g["counts"][idx] == o["counts"]).all()
            rel = np.abs(g["obj"][idx] - o["obj"]) / np.maximum(np.abs(o["obj"]), 1e-30)
            parity = {"candidates": idx.tolist(), "counts_flags_exact": bool(ok),
                      "max_rel_err": [float(x) for x in rel.max(axis=0)]}
        if args.cpu_seconds > 0:
            n_done, t_cpu, chunk = 0, 0.0, 8
            t1 = time.perf_counter()
            while t_cpu < args.cpu_seconds and n_done < pop:
                op.evaluate(pop_np[n_done:n_done + chunk])
                n_done += chunk
                t_cpu = time.perf_counter() - t1
            cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))
            cpu = {"value": n_done / t_cpu, "unit": "candidate evals/s", "cores": cores,
                   "kind": "oracle",
                   "sample": f"first {n_done} of {pop} candidates of the same population "
                             f"(FP64 C oracle, OpenMP), {t_cpu:.1f}s"}

    achieved_ops = samples * SAMPLE_OPS / (launch_ms * 1e-3)
    line = {
        "metric": "candidate objective evals/s + voxel samples/s vs plain GPU at <=1e-5 rel err",
        "value": evals_per_s,
        "unit": "candidate evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"config {args.config}: {p.dims[0]}x{p.dims[1]}x{p.dims[2]} FP32 "
                               f"phantom pair, {p.n_points}-point Kuhn mesh ({p.n_tets} tets), "
                               f"{sum(len(s) for s in p.sets_src)} guidance points, population "
                               f"{pop}, full evaluation",
                   "population": pop, "tets": p.n_tets, "voxels": int(np.prod(p.dims))},
        "samples_per_s": samples_per_s,
        "samples_per_step": samples,
        "roofline": {"bound": "alu", "achieved": achieved_ops / 1e12, "peak": VALU_PEAK / 1e12,
                     "unit": "T lane-ops/s", "frac": achieved_ops / VALU_PEAK, "traffic": None,
                     "kernel": "k_eval_full (event-timed launch incl. k_finalize)",
                     "launch_ms": launch_ms,
                     "hbm_algorithmic_frac": samples * SAMPLE_BYTES / (launch_ms * 1e-3) / HBM_PEAK},
        "parity": parity,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
