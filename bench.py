"""Throughput of the fused ERI + compression path on one MI355X.

A step computes every quartet of the workload once: contracted Cartesian ERIs
of all 256 classes (s-f on each centre) with the per-quartet n-bit compression
of eqs. 9-10 fused in (codes and scales written to HBM).  The metric is GERIS:
1e9 compressed ERIs per second.  Inputs (the plan's pair tables) are resident
in HBM before the timed region.

Default workload: all 256 classes, 65536 quartets per class, K uniform in
{1,2,3} per shell, centres uniform in a 10 Bohr cube, exponents log-uniform in
[0.1, 100], coefficients uniform in [0.1, 1]; FP64 recurrences, int16 codes.

Prints one JSON line (rank 0, N = 1).
"""
import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GERIS (1e9 ERIs/s) incl. int16 compression, FP64 vs FP32-mixed, + fwd+grad"
# MI355X vector peaks: FP64 78.6 TFLOP/s (published).  The published FP32 vector peak, 157.3 TFLOP/s,
# counts packed FP32 instructions, which this build does not emit; unpacked FP32 issues at the FP64
# rate, so FP32-mixed kernels are held to 78.6 as well.
PEAK_TFLOPS = {"fp64": 78.6, "mixed": 78.6, "rys": 78.6, "rys32": 78.6}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(qpc, classes, k_fixed=None):
    from paper_2303_13632_amd import workloads as W
    if k_fixed is None:
        parts = [W.class_case(cid, n_quartets=qpc) for cid in classes]
    else:
        # same generator and seeds, every shell with k_fixed primitives
        parts = [W.random_class_quartets(*W.class_of(cid), qpc, (W.SEED_BASE + 1) * 1000 + cid, k_fixed=k_fixed)
                 for cid in classes]
    return W.merge(parts)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(classes, seconds, per_class_out=""):
    """The oracle on a bounded sample of the same workload (n quartets of
    every class from the same seeded generator), class by class on the host's
    threads (at most 16), and a smaller sample of the same kind on one
    thread.  Per-class oracle rates go to per_class_out (JSON) when given.
    Returns a dict for the JSON line."""
    import oracle as O
    from paper_2303_13632_amd import workloads as W
    threads = min(16, os.cpu_count() or 1)

    def run(n, nthr, per=None):
        tot_t, tot_e, tot_q = 0.0, 0, 0
        for cid in classes:
            sh, q = W.class_case(cid, n_quartets=n)
            t0 = time.perf_counter()
            _, _, sizes = O.eri(sh, q, n_threads=nthr)
            dt = time.perf_counter() - t0
            tot_t += dt
            tot_e += int(sizes.sum())
            tot_q += len(q)
            if per is not None:
                per[cid] = int(sizes.sum()) / dt / 1e9
        return tot_t, tot_e, tot_q

    # quartets per class for about `seconds`: the cost per quartet from runs
    # with 1 and 8 quartets per class (their difference drops the fixed cost)
    t1, _, _ = run(1, threads)
    t8, _, _ = run(8, threads)
    per_q = max((t8 - t1) / 7.0, 1e-6)
    n = max(8, min(8192, int(seconds / per_q)))
    per = {}
    t, neri, nq = run(n, threads, per)
    n1 = max(1, n // (2 * threads))
    t1, neri1, _ = run(n1, 1)
    if per_class_out:
        with open(per_class_out, "w") as f:
            json.dump({"threads": threads, "quartets_per_class": n, "oracle_geris": per}, f, indent=1)
    rates = sorted(per.values())
    return {"value": neri / t / 1e9, "unit": "GERIS", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "one_core_value": neri1 / t1 / 1e9,
            "per_class_geris": {"min": rates[0], "median": rates[len(rates) // 2], "max": rates[-1]},
            "sample": "%d quartets of each of the %d classes, same generator as the workload (%d quartets, %d ERIs), "
                      "class by class, %.1f s, FP64 uncompressed, Rys quadrature, OpenMP over quartets; one "
                      "thread: %d quartets per class, %.1f s" % (n, len(classes), nq, neri, t, n1, t1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed", "rys", "rys32"])
    ap.add_argument("--bits", type=int, default=16)
    ap.add_argument("--packed", action="store_true",
                    help="codes as the packed 512-bit word stream written by the kernels (ERI_PLAN_PACKED)")
    ap.add_argument("--quartets-per-class", type=int, default=65536)
    ap.add_argument("--classes", default="all", help="'all' or comma-separated class ids")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="default launch variants (no autotuning)")
    ap.add_argument("--tune-cache", default="", help="JSON cache of the autotuner's choices")
    ap.add_argument("--secondary", default="mixed,int12,fp64_out,int8,int32,gradient,molecule,rys",
                    help="extra measurements in the same line: mixed (FP32-mixed path on the same workload), "
                         "int12 (12-bit codes packed into 512-bit words, pack kernel included), "
                         "fp64_out / int8 / int32 (same workload with FP64 output or 8-/32-bit codes), "
                         "gradient (fwd+grad on the 64-atom basis), molecule (every screened quartet of the "
                         "384-atom molecule-like basis in one graph launch), rys (the Rys-quadrature kernels, "
                         "FP64 and with FP32 stages, against the Obara-Saika ones on every class, K~U{1,2,3} "
                         "and K = 1); 'none' for the headline only")
    ap.add_argument("--per-class-out", default="", help="write per-class times/GERIS to this JSON file")
    ap.add_argument("--workload", default="classes", choices=["classes", "molecule", "gradient", "copy", "lattice"],
                    help="classes: 256 classes x quartets-per-class; molecule: every Schwarz-screened "
                         "unique quartet of the 384-atom molecule-like basis in one graph launch; "
                         "gradient: E = sum D D (ab|cd) and its gradient on the 64-atom basis")
    ap.add_argument("--molecule-scale", type=float, default=1.0, help="fraction of the molecule's atoms")
    ap.add_argument("--schwarz", type=float, default=1e-10)
    ap.add_argument("--fd-sample", type=int, default=0,
                    help="gradient workload: check this many coordinates and as many exponents by central "
                         "differences (h = 1e-4) of the GPU energy on the same quartet set")
    ap.add_argument("--ring-gb", type=float, default=48.0)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch  # noqa: F401
    from paper_2303_13632_amd import eri  # noqa: F401

    if args.workload == "molecule":
        print(json.dumps(bench_molecule(args)), flush=True)
        return
    if args.workload == "gradient":
        print(json.dumps(bench_gradient(args)), flush=True)
        return
    if args.workload == "copy":
        print(json.dumps(bench_copy(args)), flush=True)
        return
    if args.workload == "lattice":
        print(json.dumps(bench_lattice(args)), flush=True)
        return
    classes = list(range(256)) if args.classes == "all" else [int(c) for c in args.classes.split(",")]
    res = bench_classes(args, classes, args.precision, args.bits, args.steps, args.warmup, args.per_class_out)
    out = {
        "metric": METRIC, "value": res["geris"], "unit": "GERIS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64" if args.precision in ("mixed", "rys32") else "f64",
        "data": "synthetic",
        "config": res["config"],
        "whole_step_tflops": res["whole_step_tflops"],
        "tuned": res["tuned"], "tune_s": res["tune_s"],
        "roofline": res["roofline"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(res["active"], args.cpu_seconds,
                                           (args.per_class_out + ".oracle.json") if args.per_class_out else "")
    sec = [x for x in args.secondary.split(",") if x and x != "none"]
    if sec:
        out["secondary"] = {}
    if "mixed" in sec and args.precision == "fp64":
        m = bench_classes(args, classes, "mixed", args.bits, max(1, args.steps // 2), 1, "")
        out["secondary"]["fp32_mixed"] = {
            "value": m["geris"], "unit": "GERIS", "ms_per_step": m["ms_per_step"], "tuned": m["tuned"],
            "note": "same workload; FP32 VRR/HRR with FP64 Boys/prefactor/accumulation for the %d classes "
                    "whose FP32 error was measured within 1e-8 Ha, FP64 kernels for the other %d (FP32 "
                    "recurrences miss the 1e-7 Ha target there); roofline against the unpacked-FP32 = FP64 "
                    "rate of 78.6 TFLOP/s" % (m["n_fp32"], 256 - m["n_fp32"]),
            "n_fp32_classes": m["n_fp32"],
            "roofline_class": m["roofline"]["class"], "roofline_frac": m["roofline"]["frac"]}
    if "int12" in sec:
        out["secondary"]["int12_packed"] = bench_packed(args, classes, 12)
    for name, bits in (("fp64_out", 0), ("int8", 8), ("int32", 32)):
        if name in sec and args.precision == "fp64":
            m = bench_classes(args, classes, "fp64", bits, max(1, args.steps // 2), 1, "")
            out["secondary"][name] = {
                "value": m["geris"], "unit": "GERIS", "ms_per_step": m["ms_per_step"], "tuned": m["tuned"],
                "bits": bits, "note": "same workload, " + m["config"]["workload"].split("; ")[-1],
                "roofline_class": m["roofline"]["class"], "roofline_frac": m["roofline"]["frac"]}
    if "gradient" in sec:
        g = bench_gradient(args, steps=1, warmup=1)
        out["secondary"]["fwd_grad"] = {k: g[k] for k in ("value", "unit", "ms_per_step", "forward_ms", "adjoint_ms",
                                                          "forward_geris", "adjoint_geris")}
        out["secondary"]["fwd_grad"]["workload"] = g["config"]["workload"]
        out["secondary"]["fwd_grad"]["n_eri"] = g["config"]["n_eri"]
    if "molecule" in sec:
        import copy
        margs = copy.copy(args)
        margs.steps, margs.warmup = 1, 1
        mol = bench_molecule(margs)
        out["secondary"]["molecule"] = {k: mol[k] for k in ("value", "unit", "ms_per_step", "dtype")}
        out["secondary"]["molecule"].update({k: mol["config"][k] for k in ("workload", "n_quartets", "n_eri")})
        for k in ("tune_s", "plan_s", "whole_step_tflops"):
            if k in mol:
                out["secondary"]["molecule"][k] = mol[k]
    if "rys" in sec and args.precision == "fp64":
        out["secondary"]["rys"] = bench_rys(args, res)
    print(json.dumps(out), flush=True)


def bench_rys(args, os_workload=None):
    """The Rys-quadrature kernels (one lane per quartet for L_tot <= 4, one
    workgroup per quartet above; FP64, and with the paper's FP32 stages)
    against the Obara-Saika/HGP kernels on the same quartets of every class,
    all tuned, int16 codes: GERIS of each and the per-class time ratios, on
    the workload (K~U{1,2,3}; the Obara-Saika figures are the headline run's
    when given) and with one primitive per shell (K = 1, where the paper
    expects Rys to need fewer operations for high angular momenta)."""
    from paper_2303_13632_amd import workloads as W
    classes = list(range(256))
    steps = max(1, args.steps // 2)

    def ratios(r, o):
        ratio = {c: r["per_class_ms"][c] / o["per_class_ms"][c] for c in r["per_class_ms"]}
        vals = sorted(ratio.values())
        by_l = {}
        for c, v in ratio.items():
            by_l.setdefault(sum(W.class_of(c)), []).append(v)
        return {"min": vals[0], "median": vals[len(vals) // 2], "max": vals[-1],
                "best_class": "[%d%d|%d%d]" % W.class_of(min(ratio, key=ratio.get)),
                "median_by_L_tot": {str(k): round(float(np.median(v)), 3) for k, v in sorted(by_l.items())}}
    out = {}
    for key, kf in (("workload", None), ("k1", 1)):
        o = os_workload if (kf is None and os_workload is not None) else \
            bench_classes(args, classes, "fp64", args.bits, steps, 1, "", k_fixed=kf)
        r = bench_classes(args, classes, "rys", args.bits, steps, 1, "", k_fixed=kf)
        r32 = bench_classes(args, classes, "rys32", args.bits, steps, 1, "", k_fixed=kf)
        out[key] = {"value": r["geris"], "unit": "GERIS", "fp32_stages_value": r32["geris"], "os_value": o["geris"],
                    "n_classes": len(classes), "ms_per_step": r["ms_per_step"],
                    "fp32_stages_ms_per_step": r32["ms_per_step"], "os_ms_per_step": o["ms_per_step"],
                    "time_ratio_rys_over_os": ratios(r, o), "time_ratio_rys_fp32_stages_over_os": ratios(r32, o),
                    "roofline_class": r["roofline"]["class"], "roofline_kernel": r["roofline"]["kernel"],
                    "roofline_frac": r["roofline"]["frac"], "whole_step_tflops": r["whole_step_tflops"],
                    "config": r["config"]["workload"]}
    res = dict(out["workload"])
    res["k1"] = out["k1"]
    res["note"] = ("every class, %d quartets each; value = Rys in FP64, fp32_stages_value = Rys with FP32 "
                   "recurrences, transfers and node sums (FP64 rule, prefactor, contraction); the Rys FLOP count "
                   "(node/weight series, 2D recurrences and transfers per node and axis, three products per ERI "
                   "and node) is its own" % args.quartets_per_class)
    return res


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE passes summarised in profiles/<kernel>_traffic.md, or None
    when there is no summary or it was taken with another build of the
    library (the kernel may have changed since)."""
    import hashlib
    from paper_2303_13632_amd import eri
    path = os.path.join(ROOT, "profiles", "%s_traffic.md" % kernel)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    with open(eri.LIB_PATH, "rb") as f:
        sha = hashlib.sha1(f.read()).hexdigest()
    if fields.get("liberi_hip.so sha1") != sha:
        return None
    return float(fields["fetch bytes per launch"]) + float(fields["write bytes per launch"])


def bench_packed(args, classes, bits):
    """The 256-class workload with n-bit codes written by the ERI kernels as the
    packed stream of 512-bit words (ERI_PLAN_PACKED: each quartet's codes
    staged in LDS and packed in the same kernel), timed like the headline;
    then eq. 11 on the host: a bounded prefix of the stream (whole quartets)
    copied to host memory and decompressed by eri_unpack_host on every host
    thread."""
    import torch
    from paper_2303_13632_amd import eri
    shells, quartets = build_workload(args.quartets_per_class, classes)
    plan = eri.Plan(shells, quartets, precision="fp64", bits=bits, device=0, packed=True)
    del shells, quartets
    if not args.no_tune:
        plan.tune(sample_quartets=args.quartets_per_class, trials=2, cache=args.tune_cache or None)
    _, words, scales = plan.alloc(eri=False, codes=True)
    stream = torch.cuda.current_stream()
    plan.compute(None, words, scales, stream=stream)
    torch.cuda.synchronize()
    steps = max(1, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.compute(None, words, scales, stream=stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    res = {"value": plan.n_eri / (ms / 1e3) / 1e9, "unit": "GERIS", "bits": bits, "ms_per_step": ms,
           "packed_bytes": int(plan.class_word_off[256]) * 64, "int16_container_bytes": int(plan.n_eri) * 2,
           "note": "same workload; the ERI kernels write the packed stream themselves (floor(512/n) codes per "
                   "512-bit word, every quartet word-aligned), no container array and no second pass"}
    # host decompression of a prefix of whole quartets (about 2 GB of words)
    off = []
    for c in range(256):
        n = int(plan.class_quartets[c])
        if n:
            m = int((plan.class_eri_off[c + 1] - plan.class_eri_off[c]) // n)
            off.append(plan.class_eri_off[c] + m * np.arange(n))
    off = np.concatenate(off + [np.array([plan.n_eri], dtype=np.int64)])
    woff = eri.packed_word_offsets(bits, off)
    nq = int(np.searchsorted(woff, (2 << 30) // 64, side="right")) - 1
    nw = int(woff[nq])
    host_words = words[: 8 * nw].cpu().numpy()
    host_scales = scales[:nq].cpu().numpy()
    threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    _, vals = eri.unpack_host(bits, host_words, off[: nq + 1], woff[: nq + 1], scales=host_scales, codes=False,
                              values=True, n_threads=threads)
    th = time.perf_counter() - t0
    res["host_decompress"] = {"value": float(off[nq]) / th / 1e9, "unit": "GERIS", "threads": threads,
                              "sample": "first %d quartets (%d ERIs, %.2f GB of packed words) to FP64" %
                                        (nq, int(off[nq]), nw * 64 / 1e9)}
    del vals, host_words, words, scales
    plan.close()
    torch.cuda.empty_cache()
    res["decompression_error"] = packed_error_sample(classes, (bits, 16), 256)
    return res


def packed_error_sample(classes, bits_list, nq):
    """Largest decompression error of the packed stream on nq quartets per
    class (same generator): plans writing the FP64 values and the packed
    stream together, the stream decoded on the host (eq. 11) and compared
    with the values, per width; also the largest error in units of half a
    quantisation step (at most 1 by eq. 10)."""
    import torch
    from paper_2303_13632_amd import eri
    shells, quartets = build_workload(nq, classes)
    out = {"sample": "%d quartets of each class, FP64 values and the packed stream of the same plan" % nq}
    for b in bits_list:
        plan = eri.Plan(shells, quartets, precision="fp64", bits=b, device=0, packed=True)
        e, words, scales = plan.alloc(eri=True, codes=True)
        plan.compute(e, words, scales)
        torch.cuda.synchronize()
        off = []
        for c in range(256):
            n = int(plan.class_quartets[c])
            if n:
                m = int((plan.class_eri_off[c + 1] - plan.class_eri_off[c]) // n)
                off.append(plan.class_eri_off[c] + m * np.arange(n))
        off = np.concatenate(off + [np.array([plan.n_eri], dtype=np.int64)])
        woff = eri.packed_word_offsets(b, off)
        sc = scales.cpu().numpy()[: plan.n_quartets]
        _, v = eri.unpack_host(b, words[: 8 * int(woff[-1])].cpu().numpy(), off, woff, scales=sc, codes=False,
                               values=True)
        x = e.cpu().numpy()[: plan.n_eri]
        err = np.abs(v - x)
        step = np.repeat(sc, np.diff(off))
        m = step >= np.finfo(np.float64).tiny * 1024   # normal scales (subnormal ones carry no bound)
        out["bits%d" % b] = {"max_abs_Ha": float(err.max()),
                             "max_over_half_step": float((2.0 * err[m] / step[m]).max()) if m.any() else 0.0,
                             "non_finite": int((~np.isfinite(v)).sum() + (~np.isfinite(x)).sum())}
        del e, words, scales
        plan.close()
        torch.cuda.empty_cache()
    return out


def bench_classes(args, classes, precision, bits, steps, warmup, per_class_out, k_fixed=None):
    """The 256-class workload: all classes once per step (HIP events around
    every class launch on the launch stream)."""
    import torch
    from paper_2303_13632_amd import eri
    from paper_2303_13632_amd import workloads as W
    t0 = time.time()
    shells, quartets = build_workload(args.quartets_per_class, classes, k_fixed)
    log("workload: %d quartets, %d shells (%.1fs)" % (len(quartets), len(shells["L"]), time.time() - t0))
    t0 = time.time()
    packed = bool(getattr(args, "packed", False)) and bits > 0
    plan = eri.Plan(shells, quartets, precision=precision, bits=bits, device=0, packed=packed)
    del shells, quartets
    log("plan %s: %d ERIs, %d primitive quartets, %.1f GB on device (%.1fs)"
        % (precision, plan.n_eri, plan.n_prim_quartets, plan.device_bytes / 1e9, time.time() - t0))
    tune_s = 0.0
    if not args.no_tune:
        t0 = time.time()
        plan.tune(sample_quartets=args.quartets_per_class, trials=2, cache=args.tune_cache or None)
        tune_s = time.time() - t0
        log("tuned in %.1fs: %d classes off the default variant" % (tune_s, int((plan.class_variant > 0).sum())))
    # bits = 0: FP64 values are the output (no compression)
    values, codes, scales = plan.alloc(eri=bits == 0, codes=bits > 0)
    stream = torch.cuda.current_stream()
    active = [c for c in classes if plan.class_quartets[c] > 0]

    def step(events=None):
        for i, c in enumerate(active):
            if events is not None:
                events[i][0].record(stream)
            plan.compute_class(c, values, codes, scales, stream=stream)
            if events is not None:
                events[i][1].record(stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in active]
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(ev[k])
        log("step %d done" % k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / steps
    per_class_ms = np.array([[ev[k][i][0].elapsed_time(ev[k][i][1]) for i in range(len(active))]
                             for k in range(steps)]).mean(axis=0)
    geris = plan.n_eri / (ms_step / 1e3) / 1e9
    # roofline of the dominant kernel (the class with the largest time per step)
    dom = int(np.argmax(per_class_ms))
    c_dom = active[dom]
    t_dom = per_class_ms[dom] / 1e3
    achieved = plan.class_flops[c_dom] / t_dom / 1e12
    peak = PEAK_TFLOPS[precision]
    roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": measured_traffic(plan.kernel_name(c_dom)), "traffic_unit": "HBM bytes per launch",
            "kernel": plan.kernel_name(c_dom),
            "class": "[%d%d|%d%d]" % W.class_of(c_dom), "avg_ms": per_class_ms[dom],
            "algorithmic_flops_per_launch": plan.class_flops[c_dom]}
    total_flops = float(sum(plan.class_flops[c] for c in active))
    if per_class_out:
        rows = []
        for i, c in enumerate(active):
            n_eri_c = int(plan.class_eri_off[c + 1] - plan.class_eri_off[c])
            rows.append({"class": c, "L": W.class_of(c), "ms": per_class_ms[i], "n_eri": n_eri_c,
                         "geris": n_eri_c / (per_class_ms[i] / 1e3) / 1e9,
                         "tflops": plan.class_flops[c] / (per_class_ms[i] / 1e3) / 1e12,
                         "kernel": plan.kernel_name(c), "variant": int(plan.class_variant[c]),
                         "block": int(plan.class_block[c])})
        with open(per_class_out, "w") as f:
            json.dump(rows, f, indent=1)
    config = {"workload": "%d classes x %d quartets, %s, centres U[0,10)^3 Bohr, exponents "
                          "log-U[0.1,100], coefs U[0.1,1]; %s recurrences, %s"
                          % (len(active), args.quartets_per_class,
                             "K~U{1,2,3}" if k_fixed is None else "K=%d" % k_fixed, precision,
                             ("int%d per-quartet compression" % bits + (", codes packed in 512-bit words" if packed else ""))
                             if bits else "FP64 output, no compression"),
              "n_eri": int(plan.n_eri), "n_quartets": int(plan.n_quartets),
              "n_prim_quartets": int(plan.n_prim_quartets), "precision": precision, "bits": bits}
    res = {"geris": geris, "ms_per_step": ms_step, "config": config, "roofline": roof,
           "per_class_ms": {c: float(per_class_ms[i]) for i, c in enumerate(active)},
           "n_fp32": int(plan.class_fp32[active].sum()),
           "whole_step_tflops": total_flops / (ms_step / 1e3) / 1e12, "active": active,
           "tuned": not args.no_tune, "tune_s": tune_s}
    del codes, scales
    plan.close()
    torch.cuda.empty_cache()
    return res


# the paper's measured FPGA throughput for these classes on this lattice (Table V: one Stratix 10,
# 16-bit; [ss|ss] and [ff|ds]: two FPGAs, Sec. IV-D), for context
PAPER_FPGA_GERIS = {"[fd|ps]": 3.33, "[ps|fd]": 1.05, "[ff|dp]": 10.03, "[dp|ff]": 6.65, "[fd|fd]": 11.17,
                    "[df|fd]": 10.93, "[ss|ss]": 0.08, "[ff|ds]": 15.3}
PAPER_CLASSES = {"[fd|ps]": (3, 2, 1, 0), "[ps|fd]": (1, 0, 3, 2), "[ff|dp]": (3, 3, 2, 1), "[dp|ff]": (2, 1, 3, 3),
                 "[fd|fd]": (3, 2, 3, 2), "[df|fd]": (2, 3, 3, 2), "[ss|ss]": (0, 0, 0, 0), "[ff|ds]": (3, 3, 2, 0),
                 "[ff|ff]": (3, 3, 3, 3)}


def bench_lattice(args):
    """The paper's own benchmark system (Sec. IV-A): 32 sites on a 4x4x2
    lattice at 1 Angstrom, primitive s, p, d, f shells with exponent 1.5 on
    every site, no screening.  Per class, every unique site quartet
    (i >= j, k >= l, ij >= kl; 139656 quartets); all 256 classes per step,
    with int`bits` codes.  Reports GERIS overall and for the classes the
    paper tabulates, and the largest quantisation error of the decompressed
    codes per class (against the GPU FP64 values)."""
    import torch
    from paper_2303_13632_amd import eri, workloads as W
    sh = W.paper_lattice()
    nsite = len(sh["L"]) // 4
    pairs = [(i, j) for i in range(nsite) for j in range(i + 1)]
    site_q = np.array([(p[0], p[1], q[0], q[1]) for a, p in enumerate(pairs) for q in pairs[:a + 1]], dtype=np.int32)
    quartets = []
    for cid in range(256):
        la, lb, lc, ld = (cid >> 6) & 3, (cid >> 4) & 3, (cid >> 2) & 3, cid & 3
        quartets.append(site_q * 4 + np.array([la, lb, lc, ld], dtype=np.int32))
    quartets = np.concatenate(quartets)
    t0 = time.time()
    plan = eri.Plan(sh, quartets, precision=args.precision, bits=args.bits)
    log("lattice plan: %d quartets, %d ERIs (%.1fs)" % (plan.n_quartets, plan.n_eri, time.time() - t0))
    if not args.no_tune:
        plan.tune(sample_quartets=65536, trials=2)
    _, codes, scales = plan.alloc(eri=False, codes=True)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(256)]
    for _ in range(max(1, args.warmup)):
        plan.compute(None, codes, scales, stream=stream)
    torch.cuda.synchronize()
    per = np.zeros(256)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for c in range(256):
            ev[c][0].record(stream)
            plan.compute_class(c, None, codes, scales, stream=stream)
            ev[c][1].record(stream)
        torch.cuda.synchronize()
        per += np.array([ev[c][0].elapsed_time(ev[c][1]) for c in range(256)])
    wall = (time.perf_counter() - t0) / args.steps
    per /= args.steps
    n_eri_c = np.diff(plan.class_eri_off)
    n_quartets_all, n_eri_all = int(plan.n_quartets), int(plan.n_eri)
    del codes, scales
    plan.close()
    torch.cuda.empty_cache()
    # quantisation error of the tabulated classes: FP64 values and codes of
    # one class at a time, decompressed and compared
    maxerr = {}
    for name, Lq in PAPER_CLASSES.items():
        sub = eri.Plan(sh, site_q * 4 + np.array(Lq, dtype=np.int32), precision=args.precision, bits=args.bits)
        v, cq, sc = sub.alloc(eri=True, codes=True)
        sub.compute(v, cq, sc)
        m = int(sub.n_eri // sub.n_quartets)
        eps = torch.repeat_interleave(sc[: sub.n_quartets], m)
        maxerr[name] = float((v[: sub.n_eri] - cq[: sub.n_eri].to(torch.float64) * eps).abs().max().item())
        del v, cq, sc, eps
        sub.close()
        torch.cuda.empty_cache()
    out = {"workload": "paper benchmark lattice: 32 sites 4x4x2 at 1 Angstrom, primitive s,p,d,f (alpha 1.5), "
                       "139656 unique site quartets per class, all 256 classes, int%d codes, %s" % (args.bits, args.precision),
           "value": float(n_eri_all / wall / 1e9), "unit": "GERIS", "ms_per_step": wall * 1e3,
           "n_eri": n_eri_all, "n_quartets": n_quartets_all,
           "paper_classes": {name: {"geris": float(n_eri_c[c] / (per[c] / 1e3) / 1e9), "ms": float(per[c]),
                                    "max_abs_quantisation_error": maxerr[name],
                                    "paper_fpga_geris": PAPER_FPGA_GERIS.get(name)}
                             for name, Lq in PAPER_CLASSES.items()
                             for c in [(Lq[0] << 6) | (Lq[1] << 4) | (Lq[2] << 2) | Lq[3]]},
           "best_class_geris": float(np.max(n_eri_c / (per / 1e3) / 1e9))}
    return out


def bench_copy(args):
    """A plain 1 GiB device-to-device copy, the reference for scaling the
    FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    n = 1 << 27
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(max(1, args.steps)):
        y.copy_(x)
    torch.cuda.synchronize()
    return {"workload": "copy", "bytes_read_per_launch": 8 * n, "bytes_written_per_launch": 8 * n,
            "launches": max(1, args.steps)}


def bench_molecule(args):
    """Every unique quartet of the molecule-like basis with Q_ab Q_cd >= tau,
    computed with int16 compression in one hipGraph launch per step."""
    import torch
    from paper_2303_13632_amd import eri, workloads as W
    n_heavy = max(1, int(round(128 * args.molecule_scale)))
    n_h = max(1, int(round(256 * args.molecule_scale)))
    sh = W.molecule_basis(n_heavy=n_heavy, n_h=n_h)
    t0 = time.time()
    plan = eri.Plan(sh, None, precision=args.precision, bits=args.bits, schwarz=args.schwarz,
                    ring_bytes=int(args.ring_gb * 1e9))
    plan_s = time.time() - t0
    log("plan: %d atoms, %d shells, %d screened quartets, %d ERIs, %d primitive quartets (%.1fs)"
        % (n_heavy + n_h, len(sh["L"]), plan.n_quartets, plan.n_eri, plan.n_prim_quartets, time.time() - t0))
    tune_s = 0.0
    if not args.no_tune:
        t0 = time.time()
        plan.tune(sample_quartets=65536, trials=2, cache=args.tune_cache or None)
        tune_s = time.time() - t0
        log("tuned in %.1fs: %d classes off the default variant" % (tune_s, int((plan.class_variant > 0).sum())))
    _, codes, scales = plan.alloc(eri=False, codes=True)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        plan.compute(None, codes, scales, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    for k in range(args.steps):
        plan.compute(None, codes, scales, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / args.steps
    geris = plan.n_eri / (ms_step / 1e3) / 1e9
    flops = float(plan.class_flops.sum())
    out = {
        "metric": METRIC, "value": geris, "unit": "GERIS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "wall_ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if args.precision in ("mixed", "rys32") else "f64", "data": "synthetic",
        "config": {"workload": "molecule-like basis: %d heavy (s,s,s,p,p,d; K 1-6; exps log-U[0.1,5000]) + %d H "
                               "(s,s,p) atoms on a jittered 3.5 Bohr lattice; all unique quartets with "
                               "Q_ab Q_cd >= %g in one graph launch; int%d codes, %.0f GB output ring"
                               % (n_heavy, n_h, args.schwarz, args.bits, args.ring_gb),
                   "n_shells": int(len(sh["L"])), "n_quartets": int(plan.n_quartets),
                   "n_eri": int(plan.n_eri), "n_prim_quartets": int(plan.n_prim_quartets)},
        "whole_step_tflops": flops / (ms_step / 1e3) / 1e12, "tuned": not args.no_tune, "tune_s": tune_s,
        "plan_s": plan_s,
    }
    return out


def bench_gradient(args, steps=None, warmup=None):
    """Forward + adjoint on the 64-atom basis (22 heavy + 42 H on a 4x4x4
    lattice, s-d shells): every unique Schwarz-screened quartet computed with
    int16 codes (one graph launch), then E = sum D D (ab|cd) with the
    gradient for all centres and exponents (eri_backward, density form)."""
    import torch
    from paper_2303_13632_amd import eri, workloads as W
    sh = W.gradient_basis()
    t0 = time.time()
    plan = eri.Plan(sh, None, precision="fp64", bits=args.bits, schwarz=args.schwarz)
    D = torch.tensor(W.random_density(plan.nbf), device="cuda")
    log("plan: %d shells, %d basis functions, %d screened quartets, %d ERIs (%.1fs)"
        % (len(sh["L"]), plan.nbf, plan.n_quartets, plan.n_eri, time.time() - t0))
    _, codes, scales = plan.alloc(eri=False, codes=True)
    gc = torch.zeros((len(sh["L"]), 3), dtype=torch.float64, device="cuda")
    ge = torch.zeros(plan.n_prims, dtype=torch.float64, device="cuda")
    en = torch.zeros(1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        plan.compute(None, codes, scales, stream=stream)
        if ev:
            ev[1].record(stream)
        gc.zero_()
        ge.zero_()
        en.zero_()
        if ev:
            ev[2].record(stream)
        plan.backward(density=D, grad_centers=gc, grad_exps=ge, energy=en, stream=stream)
        if ev:
            ev[3].record(stream)

    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    t0 = time.time()
    for _ in range(max(1, warmup)):
        step()
    torch.cuda.synchronize()
    log("warmup (incl. derived tables) %.1fs" % (time.time() - t0))
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        step(evs[k])
        log("step %d done" % k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    bwd = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))
    ms_step = wall * 1e3 / steps
    out = {
        "metric": METRIC, "value": plan.n_eri / (ms_step / 1e3) / 1e9, "unit": "GERIS", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "adjoint: 64-atom basis (22 heavy s,s,s,p,p,d K 1-6 + 42 H s,s,p; 4x4x4 jittered "
                               "3.5 Bohr lattice), all unique quartets with Q_ab Q_cd >= %g; forward with int%d "
                               "codes, then E = sum D D (ab|cd), D symmetric N(0, 0.1), and dE/d(centres, "
                               "exponents)" % (args.schwarz, args.bits),
                   "n_shells": int(len(sh["L"])), "n_quartets": int(plan.n_quartets), "n_eri": int(plan.n_eri)},
        "forward_ms": fwd, "adjoint_ms": bwd,
        "forward_geris": plan.n_eri / (fwd / 1e3) / 1e9, "adjoint_geris": plan.n_eri / (bwd / 1e3) / 1e9,
        "energy": float(en.item()), "grad_centres_norm": float(gc.norm().item()),
        "grad_exps_norm": float(ge.norm().item()),
    }
    if args.fd_sample > 0:
        out["fd_check"] = fd_check(plan, D, gc.cpu().numpy(), ge.cpu().numpy(), args)
    return out


def fd_check(plan, D, gc, ge, args, h=1e-4):
    """Central differences of the GPU energy E = sum D D (ab|cd) for a seeded
    sample of coordinates and exponents, on the plan's own quartet set (the
    geometry is changed in place with eri_plan_set_geometry, so the screened
    set stays fixed) with the energy summed in a fixed order (energy-only
    eri_backward).  Errors relative to max(|g_FD|, 1e-8 max|g|); the plain
    difference at h and a Richardson extrapolation from h and 2h."""
    rng = np.random.default_rng(20230323 + 5)
    gmax = max(np.abs(gc).max(), np.abs(ge).max())
    xyz0 = np.array(plan.shells["xyz"], dtype=np.float64).reshape(-1)
    exps0 = np.array(plan.shells["exps"], dtype=np.float64)

    def energy(key, idx, d):
        x, e = xyz0.copy(), exps0.copy()
        (x if key == "xyz" else e)[idx] += d
        plan.set_geometry(xyz=x, exps=e)
        _, _, en = plan.backward(density=D, energy_only=True)
        return float(en.item())

    def central(key, idx, step):
        return (energy(key, idx, step) - energy(key, idx, -step)) / (2 * step)

    rows = []
    for key, n_all, g in (("xyz", len(xyz0), gc.reshape(-1)), ("exps", len(exps0), ge)):
        for idx in rng.choice(n_all, size=min(args.fd_sample, n_all), replace=False):
            fd = central(key, idx, h)
            rich = (4 * fd - central(key, idx, 2 * h)) / 3
            floor = 1e-8 * gmax
            rows.append({"param": key, "index": int(idx), "analytic": float(g[idx]), "fd": fd, "fd_richardson": rich,
                         "rel": abs(fd - g[idx]) / max(abs(fd), floor),
                         "rel_richardson": abs(rich - g[idx]) / max(abs(rich), floor)})
        log("fd %s done" % key)
    plan.set_geometry(xyz=xyz0, exps=exps0)
    return {"h": h, "n": len(rows), "max_rel": max(r["rel"] for r in rows),
            "max_rel_richardson": max(r["rel_richardson"] for r in rows),
            "n_rel_above_1e-6": int(sum(r["rel"] > 1e-6 for r in rows)),
            "max_abs_over_gmax": max(abs(r["fd"] - r["analytic"]) for r in rows) / gmax,
            "max_abs_over_gmax_richardson": max(abs(r["fd_richardson"] - r["analytic"]) for r in rows) / gmax,
            "n_rel_richardson_above_1e-6": int(sum(r["rel_richardson"] > 1e-6 for r in rows)),
            "worst": max(rows, key=lambda r: r["rel"]),
            "worst_richardson": max(rows, key=lambda r: r["rel_richardson"]), "gmax": float(gmax)}


if __name__ == "__main__":
    main()
