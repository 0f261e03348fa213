#!/usr/bin/env python
"""Batched workload: 64 independent water clusters of 8..128 molecules
(24..384 atoms each, ~13.7k atoms in all) built in one HIP-graph replay.

Prints one JSON line with K matrices/s and batches/s of the FP64 path and of
the distance-split mixed path (with its error against the FP64 path per
cluster), the algorithmic flops of one batch and the per-stage times of an
eager build.
Inputs are generated on the host (slow: about a minute) and copied to HBM
before timing.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--clusters", type=int, default=64)
    ap.add_argument("--mixed-split", type=float, default=5.0)
    args = ap.parse_args()
    import numpy as np
    import torch

    import synth
    import paper_2403_10343_amd as exx

    t0 = time.perf_counter()
    b = synth.cluster_batch(args.clusters)
    inp = synth.make_inputs(b)
    t_gen = time.perf_counter() - t0
    print(f"generated {b.n_atoms} atoms in {t_gen:.1f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    plan = exx.Plan.for_system(b)
    t_plan = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    C, V, D = (torch.from_numpy(a).to(dev) for a in (inp.C, inp.V, inp.D))
    K = torch.empty(plan.info["d_size"], dtype=torch.float64, device=dev)
    Ex = torch.empty(b.n_systems, dtype=torch.float64, device=dev)
    s = torch.cuda.Stream()
    names = exx._lib.STAGE_NAMES
    sizes = np.diff(b.sys_off)

    def run(prec):
        plan.set_profiling(True)
        plan.build_K(C, V, D, K, Ex, precision=prec, stream=s.cuda_stream)
        torch.cuda.synchronize()
        stage_ms, _ = plan.stage_times()
        plan.set_profiling(False)
        plan.graph_build(C, V, D, K, Ex, stream=s.cuda_stream, precision=prec)
        for _ in range(args.warmup):
            plan.graph_launch(stream=s.cuda_stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.graph_launch(stream=s.cuda_stream)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        alg, _ = plan.stage_flops(prec == exx.PREC_MIXED)
        return dt, {names[i]: float(stage_ms[i]) for i in range(len(names))}, alg

    plan.autotune(C, V, D, K, stream=s.cuda_stream)
    tuning = plan.tuning()
    dt64, st64, alg64 = run(exx.PREC_FP64)
    K64, E64 = K.clone(), Ex.clone()
    plan.set_mixed_split(args.mixed_split)
    dtm, stm, algm = run(exx.PREC_MIXED)
    dE = ((Ex - E64).abs().cpu().numpy() / sizes)
    dK = float((K - K64).abs().max().item())
    flops = plan.flops()
    within = dK <= 1e-5 and float(dE.max()) <= 1e-6
    use_mixed = within and dtm < dt64          # the faster path that meets the bar
    dt = dtm if use_mixed else dt64
    out = {
        "metric": "K matrices/s, batched clusters (one HIP-graph replay per batch; faster of the FP64 path and "
                  "the mixed FP32/FP64 path at |dE_x|<=1e-6 Ha/atom and max|dK|<=1e-5; both reported)",
        "value": b.n_systems / dt, "unit": "K matrices/s", "batches_per_s": 1.0 / dt,
        "ms_per_batch": 1e3 * dt, "steps": args.steps, "warmup": args.warmup,
        "dtype": "f32+f64" if use_mixed else "f64", "data": "synthetic",
        "config": {"workload": f"{b.n_systems} water clusters of 8..128 molecules",
                   "atoms": b.n_atoms, "basis_total": int(inp.layout.sys_nbas.sum()),
                   "path": "mixed" if use_mixed else "fp64", "mixed_split_A": args.mixed_split,
                   "sizes_molecules": [int(x) // 3 for x in sizes]},
        "algorithmic_gflop_per_batch": flops / 1e9,
        "tile_shapes": {k: {"chosen": v[0], "ms": v[1]} for k, v in tuning.items()},
        "fp64": {"K_per_s": b.n_systems / dt64, "ms_per_batch": 1e3 * dt64, "tflops": flops / dt64 / 1e12,
                 "frac_fp64_peak": flops / dt64 / 78.6e12, "eager_stage_ms": st64},
        "mixed": {"K_per_s": b.n_systems / dtm, "ms_per_batch": 1e3 * dtm, "tflops": flops / dtm / 1e12,
                  "fp32_flop_fraction": (algm[3] + algm[5]) / max(sum(algm), 1), "eager_stage_ms": stm,
                  "max_abs_dK_vs_fp64": dK, "max_dE_x_per_atom_vs_fp64": float(dE.max()),
                  "within_bar": within},
        "host_seconds": {"generate_inputs": t_gen, "plan": t_plan},
        "E_x_sum": float(E64.sum().item()),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
