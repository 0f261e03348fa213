#!/usr/bin/env python
"""Benchmark: RI-LVL exchange-matrix (K) builds per second on one MI355X.

A step is one complete build_K call (zero-fill, repack of C, E = M D, the V
stage, the T2 blocks, the final owner-computes contraction and the E_x
reduction) on the 768-atom open ice box (256 H2O, 6144 basis / 17920 aux
functions, r_cut 6 A) with C, V, D already resident in HBM.  Both paths are
timed: FP64, and the distance-split mixed path (pair terms at or beyond the
split in FP32 MFMA).  "value" is the rate of the faster path among those
whose K and E_x meet max|dK| <= 1e-5 and |dE_x|/atom <= 1e-6 against the FP64
path (the FP64 path itself always does); "config.path" names it.

Prints ONE JSON line (rank 0).  The "roofline" object describes the dominant
kernel, timed with HIP events recorded by the library on its launch stream
during the timed steps; "cpu_baseline" times the CPU oracle (block route) on a
bounded sample of rows of the same workload, scaled to builds/s, and the rows
it computes give the error of both GPU paths against the oracle.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "hbm": 8.0e12}
CSRC = os.path.join(ROOT, "paper_2403_10343_amd", "csrc")
# HBM bytes per dispatch, from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs of
# this script on the 768-atom box, scaled by what the counters read for kernels
# of known traffic in the same runs (k_repack reads C once: read x1.939; k_zero
# writes K once: write x1.000).  They describe the
# kernels built from the sources with this fingerprint only; for any other
# sources the roofline's traffic is reported as null.
MEASURED_TRAFFIC = {
    "sources": "280086a1867b8e10",
    "workload": "ice768",
    "bytes": {("fp64", "H"): 29.228e9 + 4.206e9, ("fp64", "T2"): 25.185e9 + 0.036e9,
              ("fp64", "final"): 10.246e9 + 4.282e9, ("fp64", "E"): 2.847e9 + 2.473e9,
              ("mixed", "H"): 12.329e9 + 3.757e9, ("mixed", "H32"): 25.900e9 + 4.117e9},
}
KERNEL_OF_STAGE = {"repack": "k_repack", "E": "k_rowD", "H": "k_H<U, double, 1>", "H32": "k_H<U, float, 1>",
                   "T2": "k_T2<NT, NS, double, COLS, WAVES, 1>", "T2_32": "k_T2<NT, NS, float, COLS, WAVES, 1>",
                   "final": "k_Y + k_symreduce", "energy": "k_energy_part + k_energy_sum"}


def sources_fingerprint():
    import hashlib
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]
WORKLOADS = {
    "ice768": (2, "ice_box_4x4x2_768_atoms_6144_basis_rcut6"),
    "water24": (1, "water_cluster_8_24_atoms_192_basis_rcut6"),
}


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:
        return os.cpu_count()


def cpu_baseline(inp, flops_per_build, repeats=3):
    """Time the oracle's block route (rows of K atom by atom, every step a BLAS
    product over structural blocks) on the rows of one interior water molecule:
    one warm-up, then the median of `repeats` runs on all BLAS threads, and one
    run on a single thread (one H atom's rows).  Rates are scaled to whole
    builds by the fraction of K's rows computed; GFLOP/s use the library's
    algorithmic flop count of a build times the same fraction.  Returns the
    record and the rows computed (for the error report)."""
    import numpy as np
    from oracle import exx_oracle as O
    blk = O.Blocks(inp)
    n = blk.n
    deg = np.array([len(x) for x in blk.nbrs])
    o_atoms = np.nonzero(inp.system.species[:blk.nat] == 0)[0]
    o = int(o_atoms[np.argmax(deg[o_atoms])])           # most-connected O: an interior molecule
    mol = [o, o + 1, o + 2]
    rows = np.concatenate([np.arange(blk.bo[a], blk.bo[a + 1]) for a in mol])
    O.k_atom_rows(inp, [o + 1], blk=blk)                # warm-up
    times = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        Krows = O.k_atom_rows(inp, mol, blk=blk)
        times.append(time.perf_counter() - t0)
    t_med = float(np.median(times))
    frac = len(rows) / n
    one = None
    try:
        from threadpoolctl import threadpool_limits
        h_rows = int(blk.nb[o + 1])
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            O.k_atom_rows(inp, [o + 1], blk=blk)
            t1 = time.perf_counter() - t0
        one = {"builds_per_s": (h_rows / n) / t1, "gflops": (h_rows / n) * flops_per_build / t1 / 1e9,
               "sample": f"the {h_rows} rows of one H atom, one run, {t1:.2f} s", "cores": 1}
    except Exception as e:   # threadpoolctl missing: report the multi-threaded rate only
        one = {"error": str(e)}
    rec = {"value": frac / t_med, "unit": "builds/s", "cores": int(_blas_threads()), "kind": "oracle",
           "route": "block route (oracle.k_atom_rows): the definition over structural blocks, atom by atom",
           "sample": f"the {len(rows)} rows of one interior water molecule ({len(rows)} of {n} rows of K), "
                     f"median of {repeats} runs after one warm-up: {t_med:.2f} s "
                     f"(runs {', '.join(f'{t:.2f}' for t in times)} s); builds/s = {len(rows)}/{n} / time",
           "gflops": frac * flops_per_build / t_med / 1e9,
           "gflop_note": "library algorithmic flop count of a build times the fraction of rows computed",
           "one_thread": one, "host": host_description()}
    return rec, rows, Krows


def host_description():
    """CPU model, logical CPUs and the BLAS library behind NumPy (for the baseline record)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = ""
    try:
        from threadpoolctl import threadpool_info
        blas = ", ".join(sorted({f"{t.get('internal_api')} {t.get('version')}" for t in threadpool_info()}))
    except Exception:
        pass
    return {"cpu": model, "logical_cpus": os.cpu_count(), "blas": blas}


def small_config_comparison(exx, torch, repeats=3):
    """The 24-atom cluster: full oracle builds (4-index route, which also gives
    E_x directly from (ij|kl); one warm-up, median of `repeats`) against the
    GPU FP64 build."""
    import numpy as np
    import synth
    from oracle import exx_oracle as O
    inp = synth.make_inputs(synth.config(1))
    O.k_4index(inp)
    ts = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        K4, _, e_direct = O.k_4index(inp)
        ts.append(time.perf_counter() - t0)
    t_cpu = float(np.median(ts))
    plan = exx.Plan.for_system(inp.system)
    dev = torch.device("cuda:0")
    C, V, D = (torch.from_numpy(a).to(dev) for a in (inp.C, inp.V, inp.D))
    K = torch.empty(plan.info["d_size"], dtype=torch.float64, device=dev)
    Ex = torch.empty(1, dtype=torch.float64, device=dev)
    plan.build_K(C, V, D, K, Ex)
    torch.cuda.synchronize()
    n = 20
    t0 = time.perf_counter()
    for _ in range(n):
        plan.build_K(C, V, D, K, Ex)
    torch.cuda.synchronize()
    t_gpu = (time.perf_counter() - t0) / n
    Kg = K.cpu().numpy().reshape(K4.shape)
    return {"workload": "water_cluster_8_24_atoms_192_basis", "oracle_4index_s": t_cpu,
            "oracle_4index_runs_s": ts, "oracle_cores": int(_blas_threads()),
            "gpu_fp64_ms": 1e3 * t_gpu, "max_rel_dK": float(np.abs(Kg - K4).max() / np.abs(K4).max()),
            "rel_dE_x_direct": float(abs(Ex.item() - e_direct) / abs(e_direct))}


def time_builds(plan, C, V, D, K, Ex, prec, steps, warmup, stream):
    """Mean wall time per build over `steps` timed builds and the mean
    per-stage HIP-event times (ms) recorded by the library during them."""
    import torch
    for _ in range(warmup):
        plan.build_K(C, V, D, K, Ex, precision=prec, stream=stream.cuda_stream)
    torch.cuda.synchronize()
    plan.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.build_K(C, V, D, K, Ex, precision=prec, stream=stream.cuda_stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stage_ms, nrec = plan.stage_times()
    plan.set_profiling(False)
    return (t1 - t0) / steps, stage_ms / max(nrec, 1)


def path_record(plan, dt, stage_ms, mixed, names, workload):
    """Per-stage rates and the roofline of the dominant stage of one path."""
    import numpy as np
    alg, issued = plan.stage_flops(mixed)
    dom = int(np.argmax(stage_ms))
    fp32_stage = names[dom].endswith("_32") or names[dom] == "H32"
    peak = PEAK["fp32"] if fp32_stage else PEAK["fp64"]
    achieved = alg[dom] / (stage_ms[dom] * 1e-3) if stage_ms[dom] > 0 else 0.0
    path = "mixed" if mixed else "fp64"
    measured = {}
    if MEASURED_TRAFFIC["workload"] == workload and sources_fingerprint() == MEASURED_TRAFFIC["sources"]:
        measured = {st: b for (pth, st), b in MEASURED_TRAFFIC["bytes"].items() if pth == path}
    traffic = measured.get(names[dom])
    per_stage = lambda f: {names[i]: f(i) for i in range(len(names))}
    return {
        "builds_per_s": 1.0 / dt, "ms_per_build": 1e3 * dt,
        "stage_ms": per_stage(lambda i: float(stage_ms[i])),
        "stage_tflops": per_stage(lambda i: alg[i] / (stage_ms[i] * 1e-3) / 1e12 if stage_ms[i] > 0 else 0.0),
        "stage_issued_mfma_frac": per_stage(
            lambda i: issued[i] / (stage_ms[i] * 1e-3) / (PEAK["fp32"] if names[i] in ("H32", "T2_32") else PEAK["fp64"])
            if stage_ms[i] > 0 else 0.0),
        "fp32_flop_fraction": (alg[3] + alg[5]) / max(sum(alg), 1),
        # HBM read + write bytes of a stage's kernels from the committed counter runs (same
        # sources and workload only) over the stage's time
        "stage_hbm_gb_per_s": {st: float(b / (stage_ms[names.index(st)] * 1e-3) / 1e9)
                               for st, b in measured.items() if st in names and stage_ms[names.index(st)] > 0},
        "roofline": {"bound": "mfma", "kernel": KERNEL_OF_STAGE[names[dom]], "stage": names[dom],
                     "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "traffic_unit": "bytes per launch (HBM read + write)"},
    }


def attainable_peaks(torch, n=8192, reps=5):
    """What the vendor libraries reach on this GPU, beside the published peaks: a dense
    n x n x n GEMM in binary64 and binary32 (torch.matmul, rocBLAS / hipBLASLt) and a
    device-to-device copy of 2 GiB (read + write bytes), median of reps after a warm-up,
    timed with HIP events."""
    dev = torch.device("cuda:0")
    out = {}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b) * 1e-3)
        return sorted(ts)[len(ts) // 2]

    for name, dt, peak in (("dgemm", torch.float64, 78.6), ("sgemm", torch.float32, 157.3)):
        x = torch.randn(n, n, dtype=dt, device=dev)
        y = torch.randn(n, n, dtype=dt, device=dev)
        t = timed(lambda: torch.matmul(x, y))
        out[name] = {"n": n, "tflops": 2.0 * n ** 3 / t / 1e12, "published_peak_tflops": peak,
                     "frac": 2.0 * n ** 3 / t / 1e12 / peak}
        del x, y
    src = torch.empty(1 << 28, dtype=torch.float64, device=dev)
    src.fill_(1.0)
    dst = torch.empty_like(src)
    t = timed(lambda: dst.copy_(src))
    out["copy"] = {"bytes": 2 * src.numel() * 8, "tb_per_s": 2 * src.numel() * 8 / t / 1e12,
                   "published_peak_tb_per_s": 8.0}
    return out


def progress(msg):
    """One line on stderr as each part of the run ends."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def periodic_record(exx, torch, steps, backward_steps=1):
    """The periodic 1024-water box (3072 atoms, 24576 basis, r_cut 8 A): FP64 and
    mixed K builds per second (the pattern-folded real-space X), stage times,
    the mixed error against the FP64 build, and forward (FP64 or mixed) plus FP64
    backward with forces."""
    import synth
    t0 = time.perf_counter()
    sysm = synth.config(5)
    inp = synth.make_inputs(sysm)
    t_in = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan = exx.Plan.for_system(sysm)
    t_plan = time.perf_counter() - t0
    progress(f"periodic box: inputs {t_in:.1f} s, plan {t_plan:.1f} s")
    dev = torch.device("cuda:0")
    C, V, D = (torch.from_numpy(a).to(dev) for a in (inp.C, inp.V, inp.D))
    del inp
    K = torch.empty_like(D)
    Ex = torch.empty(1, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    plan.autotune(C, V, D, K, stream=stream.cuda_stream)
    names = exx._lib.STAGE_NAMES
    rec = {"workload": "ice_box_periodic_8x4x4_3072_atoms_24576_basis_rcut8 (57.3 x 28.6 x 28.6 A cell)",
           "atoms": sysm.n_atoms, "pairs": int(plan.info["n_pairs"]), "input_generation_s": t_in,
           "plan_create_s": t_plan, "algorithmic_gflop_per_build": plan.flops() / 1e9,
           "workspace_gb": plan.info["workspace_bytes"] / 1e9}
    progress("periodic box: autotuned")
    dt, st = time_builds(plan, C, V, D, K, Ex, exx.PREC_FP64, steps, 1, stream)
    progress(f"periodic box: FP64 {1e3 * dt:.1f} ms per build")
    K64, E64 = K.clone(), float(Ex.item())
    rec["fp64"] = {"ms_per_build": 1e3 * dt, "builds_per_s": 1.0 / dt,
                   "tflops": plan.flops() / dt / 1e12, "frac_fp64_peak": plan.flops() / dt / PEAK["fp64"],
                   "stage_ms": {n_: float(x) for n_, x in zip(names, st)}}
    plan.set_mixed_split(5.0)
    dt, st = time_builds(plan, C, V, D, K, Ex, exx.PREC_MIXED, steps, 1, stream)
    rec["mixed"] = {"ms_per_build": 1e3 * dt, "builds_per_s": 1.0 / dt,
                    "stage_ms": {n_: float(x) for n_, x in zip(names, st)},
                    "max_abs_dK_vs_fp64": float((K - K64).abs().max().item()),
                    "dE_x_per_atom_vs_fp64": abs(float(Ex.item()) - E64) / sysm.n_atoms}
    rec["mixed"]["within_bar"] = rec["mixed"]["max_abs_dK_vs_fp64"] <= 1e-5 and rec["mixed"]["dE_x_per_atom_vs_fp64"] <= 1e-6
    progress(f"periodic box: mixed {1e3 * dt:.1f} ms per build")
    rec["E_x_per_atom"] = E64 / sysm.n_atoms
    if backward_steps > 0:
        dC, dV, dD = torch.empty_like(C), torch.empty_like(V), torch.empty_like(D)
        F = torch.empty(sysm.n_atoms * 3, dtype=torch.float64, device=dev)
        fb = {}
        for name, prec in (("fp64", exx.PREC_FP64), ("mixed", exx.PREC_MIXED)):
            plan.build_K(C, V, D, K, Ex, precision=prec)
            plan.exchange_backward(C, V, D, 1.0, dC=dC, dV=dV, dD=dD, forces=F, K=K, build_id=plan.build_id())
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(backward_steps):
                plan.build_K(C, V, D, K, Ex, precision=prec)
                reused = plan.exchange_backward(C, V, D, 1.0, dC=dC, dV=dV, dD=dD, forces=F, K=K,
                                                build_id=plan.build_id())
            torch.cuda.synchronize()
            tb = (time.perf_counter() - t0) / backward_steps
            progress(f"periodic box: {name} forward + backward {1e3 * tb:.1f} ms")
            fb[name] = {"workload": f"{name} forward E_x; FP64 backward: dE/dC, dE/dV, dE/dD, forces",
                        "forward_intermediates_reused": reused,
                        "ms_per_step": 1e3 * tb, "steps_per_s": 1.0 / tb,
                        "net_force_max": float(F.view(-1, 3).sum(0).abs().max().item()),
                        "euler_C": float((dC * C).sum().item() / (2 * E64)),
                        "euler_V": float((dV * V).sum().item() / E64)}
        rec["forward_backward"] = fb
        del dC, dV, dD, F
    del C, V, D, K, K64
    plan.close()
    torch.cuda.empty_cache()
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ice768", choices=sorted(WORKLOADS))
    ap.add_argument("--mixed-split", type=float, default=5.0,
                    help="pair distance (A) at and beyond which the mixed path runs pair terms in FP32")
    ap.add_argument("--no-mixed", action="store_true", help="time the FP64 path only")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tile shapes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--backward-steps", type=int, default=3,
                    help="also time forward + exchange_backward (dE/dC, dE/dV, dE/dD, forces); 0 = skip")
    ap.add_argument("--spin-steps", type=int, default=5,
                    help="also time the collinear-spin build (two density matrices, FP64); 0 = skip")
    ap.add_argument("--two-kernel-steps", type=int, default=5,
                    help="also time two Coulomb matrices in one call (FP64); 0 = skip")
    ap.add_argument("--screening-steps", type=int, default=3,
                    help="timed FP64 builds per screening threshold (0: no screening record)")
    ap.add_argument("--peaks", action="store_true",
                    help="print what the vendor GEMMs and a copy reach on this GPU, then exit")
    ap.add_argument("--periodic-only", action="store_true",
                    help="time only the periodic 3072-atom box (its record as the JSON line)")
    ap.add_argument("--periodic-steps", type=int, default=2,
                    help="also time the periodic 3072-atom box (FP64 and mixed builds); 0 = skip")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 1 GiB device copy (reference dispatch for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the exchange build runs on a single MI355X "
              "(sharding over several GPUs is not implemented). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2403_10343_amd as exx

    if args.periodic_only:
        print(json.dumps({"periodic": periodic_record(exx, torch, max(args.periodic_steps, 1),
                                                      min(args.backward_steps, 1))}), flush=True)
        return
    if args.peaks:
        print(json.dumps({"attainable_peaks": attainable_peaks(torch)}), flush=True)
        return
    cfg, wname = WORKLOADS[args.workload]
    sysm = synth.config(cfg)
    inp = synth.make_inputs(sysm)
    t_plan = time.perf_counter()
    plan = exx.Plan.for_system(sysm)
    t_plan = time.perf_counter() - t_plan
    dev = torch.device("cuda:0")
    C, V, D = (torch.from_numpy(a).to(dev) for a in (inp.C, inp.V, inp.D))
    K = torch.empty(plan.info["d_size"], dtype=torch.float64, device=dev)
    Ex = torch.empty(plan.n_systems, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    names = exx._lib.STAGE_NAMES

    progress(f"{wname}: plan and inputs ready")
    if not args.no_autotune:
        plan.autotune(C, V, D, K, stream=stream.cuda_stream)
        progress("autotuned")
    tuning = plan.tuning()
    dt64, st64 = time_builds(plan, C, V, D, K, Ex, exx.PREC_FP64, args.steps, args.warmup, stream)
    progress(f"FP64 {1e3 * dt64:.2f} ms per build")
    K64, E64 = K.clone(), float(Ex[0].item())
    rec64 = path_record(plan, dt64, st64, False, names, args.workload)
    recm = None
    if not args.no_mixed:
        plan.set_mixed_split(args.mixed_split)
        dtm, stm = time_builds(plan, C, V, D, K, Ex, exx.PREC_MIXED, args.steps, args.warmup, stream)
        recm = path_record(plan, dtm, stm, True, names, args.workload)
        progress(f"mixed {1e3 * dtm:.2f} ms per build")
        Em = float(Ex[0].item())
        recm["mixed_split_A"] = args.mixed_split
        recm["error_vs_fp64_gpu"] = {
            "max_abs_dK": float((K - K64).abs().max().item()),
            "dE_x_per_atom": abs(Em - E64) / sysm.n_atoms,
            "max_abs_K": float(K64.abs().max().item()),
        }
        err = recm["error_vs_fp64_gpu"]
        recm["within_bar"] = err["max_abs_dK"] <= 1e-5 and err["dE_x_per_atom"] <= 1e-6
        Km = K.clone()
    # the faster of the paths that meet the bar (FP64 always does)
    use_mixed = recm is not None and recm["within_bar"] and recm["ms_per_build"] < rec64["ms_per_build"]
    main_rec = recm if use_mixed else rec64
    total_flops = plan.flops()

    out = {
        "metric": "K-matrix builds/s (RI-LVL exchange; faster of the FP64 path and the mixed FP32/FP64 path "
                  "at |dE_x|<=1e-6 Ha/atom and max|dK|<=1e-5; both reported)",
        "value": main_rec["builds_per_s"],
        "unit": "builds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_rec["ms_per_build"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if use_mixed else "f64",
        "data": "synthetic",
        "config": {"workload": wname, "atoms": sysm.n_atoms,
                   "basis": int(inp.layout.sys_nbas[0]), "aux": int(sysm.naux().sum()),
                   "r_cut_A": sysm.r_cut, "path": "mixed" if use_mixed else "fp64",
                   "mixed_split_A": args.mixed_split if use_mixed else None},
        "roofline": main_rec["roofline"],
        "algorithmic_gflop_per_build": total_flops / 1e9,
        "tile_shapes": {k: {"chosen": v[0], "ms": v[1]} for k, v in tuning.items()},
        "fp64": rec64,
        "mixed": recm,
        "mixed_speedup_vs_fp64": (dt64 / recm["ms_per_build"] * 1e3) if recm else None,
        "E_x": E64,
        "E_x_per_atom": E64 / sysm.n_atoms,
        "plan_create_s": t_plan,
    }
    if args.backward_steps > 0:
        dC, dV, dD = torch.empty_like(C), torch.empty_like(V), torch.empty_like(D)
        F = torch.empty(sysm.n_atoms * 3, dtype=torch.float64, device=dev)
        fb = {}
        for name, prec in (("fp64", exx.PREC_FP64), ("mixed", exx.PREC_MIXED)):
            if prec == exx.PREC_MIXED and recm is None:
                continue
            plan.build_K(C, V, D, K, Ex, precision=prec)
            plan.exchange_backward(C, V, D, 1.0, dC=dC, dV=dV, dD=dD, forces=F, K=K, build_id=plan.build_id())
            torch.cuda.synchronize()
            tb0 = time.perf_counter()
            for _ in range(args.backward_steps):
                plan.build_K(C, V, D, K, Ex, precision=prec)
                reused = plan.exchange_backward(C, V, D, 1.0, dC=dC, dV=dV, dD=dD, forces=F, K=K,
                                                build_id=plan.build_id())
            torch.cuda.synchronize()
            tb = (time.perf_counter() - tb0) / args.backward_steps
            Ff = F.view(-1, 3)
            fb[name] = {
                "workload": wname + f" ({name} forward E_x; FP64 backward: dE/dC, dE/dV, dE/dD, forces)",
                "forward_intermediates_reused": reused,
                "ms_per_step": 1e3 * tb, "steps_per_s": 1.0 / tb,
                "net_force_max": float(Ff.sum(0).abs().max().item()),
                "euler_C": float((dC * C).sum().item() / (2 * E64)),
                "euler_V": float((dV * V).sum().item() / E64),
            }
        out["forward_backward"] = fb
    if args.spin_steps > 0:
        Ds = torch.from_numpy(synth.spin_densities(inp).reshape(-1)).to(dev)
        K2 = torch.empty(2 * plan.info["d_size"], dtype=torch.float64, device=dev)
        plan.build_K_spin(C, V, Ds, K2, Ex)
        torch.cuda.synchronize()
        plan.set_profiling(True)
        ts0 = time.perf_counter()
        for _ in range(args.spin_steps):
            plan.build_K_spin(C, V, Ds, K2, Ex)
        torch.cuda.synchronize()
        ts = (time.perf_counter() - ts0) / args.spin_steps
        sst, nrec = plan.stage_times()
        plan.set_profiling(False)
        out["spin"] = {
            "workload": wname + " (collinear spin: two density matrices D^0, D^1, FP64)",
            "ms_per_build": 1e3 * ts, "builds_per_s": 1.0 / ts,
            "vs_two_one_density_builds": 2 * dt64 / ts,
            "stage_ms": {n_: float(x) for n_, x in zip(names, sst / max(nrec, 1))},
            "E_x": float(Ex[0].item()),
        }
        if args.backward_steps > 0:
            dCs, dVs, dDs = torch.empty_like(C), torch.empty_like(V), torch.empty_like(Ds)
            Fs = torch.empty(3 * sysm.n_atoms, dtype=torch.float64, device=dev)
            plan.exchange_backward_spin(C, V, Ds, 1.0, dC=dCs, dV=dVs, dD=dDs, forces=Fs, K=K2)
            torch.cuda.synchronize()
            tsb0 = time.perf_counter()
            for _ in range(args.backward_steps):
                plan.build_K_spin(C, V, Ds, K2, Ex)
                reused = plan.exchange_backward_spin(C, V, Ds, 1.0, dC=dCs, dV=dVs, dD=dDs, forces=Fs, K=K2,
                                                     build_id=plan.build_id())
            torch.cuda.synchronize()
            tsb = (time.perf_counter() - tsb0) / args.backward_steps
            out["spin"]["forward_backward_ms"] = 1e3 * tsb
            out["spin"]["forward_intermediates_reused"] = reused
            out["spin"]["net_force_max"] = float(Fs.view(-1, 3).sum(0).abs().max().item())
    if args.two_kernel_steps > 0:
        V2 = torch.from_numpy(synth.short_range_V(inp)).to(dev)
        K2 = torch.empty(2 * plan.info["d_size"], dtype=torch.float64, device=dev)
        E2 = torch.empty(2 * plan.n_systems, dtype=torch.float64, device=dev)
        plan.build_K_two_kernels(C, V, V2, D, K2, E2)
        torch.cuda.synchronize()
        plan.set_profiling(True)
        tk0 = time.perf_counter()
        for _ in range(args.two_kernel_steps):
            plan.build_K_two_kernels(C, V, V2, D, K2, E2)
        torch.cuda.synchronize()
        tk = (time.perf_counter() - tk0) / args.two_kernel_steps
        kst, nrec = plan.stage_times()
        plan.set_profiling(False)
        out["two_kernels"] = {
            "workload": wname + " (two Coulomb matrices: V and a shorter-range V2, one D, FP64)",
            "ms_per_build": 1e3 * tk, "builds_per_s": 1.0 / tk,
            "vs_two_one_kernel_builds": 2 * dt64 / tk,
            "stage_ms": {n_: float(x) for n_, x in zip(names, kst / max(nrec, 1))},
            "E_x": [float(x) for x in E2.cpu().numpy()],
        }
    if args.screening_steps > 0:
        progress("screening")
        Kref = torch.empty_like(K)
        Eref = torch.empty_like(Ex)
        plan.build_K(C, V, D, Kref, Eref)
        runs = []
        for eps in (0.3, 1.0):
            plan.set_screening(eps)
            plan.build_K(C, V, D, K, Ex)
            torch.cuda.synchronize()
            tq0 = time.perf_counter()
            for _ in range(args.screening_steps):
                plan.build_K(C, V, D, K, Ex)
            torch.cuda.synchronize()
            tq = (time.perf_counter() - tq0) / args.screening_steps
            frac = float(plan.screened_pairs().float().mean().item())
            plan.set_screening(0.0)
            runs.append({"eps": eps, "pairs_screened": frac, "ms_per_build": 1e3 * tq,
                         "vs_unscreened": dt64 / tq,
                         "max_abs_dK": float((K - Kref).abs().max().item()),
                         "dE_x_per_atom": float(abs(Ex[0].item() - Eref[0].item()) / sysm.n_atoms)})
        out["screening"] = {
            "workload": wname + " (FP64 build_K with V blocks skipped below a maximum-norm estimate; lossy)",
            "runs": runs}
    if args.periodic_steps > 0:
        out["periodic"] = periodic_record(exx, torch, args.periodic_steps, min(args.backward_steps, 1))
    if args.calibrate_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = {"read": src.numel() * 8, "write": dst.numel() * 8}
    if not args.no_cpu_baseline:
        out["config1_oracle_vs_gpu"] = small_config_comparison(exx, torch)
        rec, rows, Krows = cpu_baseline(inp, total_flops)
        out["cpu_baseline"] = rec
        n = int(inp.layout.sys_nbas[0])
        ridx = torch.as_tensor(rows, device=dev)
        g64 = K64.view(n, n)[ridx].cpu().numpy()
        rep = {"rows": int(len(rows)), "fp64_max_abs_dK": float(np.abs(g64 - Krows).max()),
               "fp64_rel": float(np.abs(g64 - Krows).max() / np.abs(Krows).max())}
        if recm is not None:
            gm = Km.view(n, n)[ridx].cpu().numpy()
            rep["mixed_max_abs_dK"] = float(np.abs(gm - Krows).max())
        out["error_vs_oracle_sampled_rows"] = rep
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
