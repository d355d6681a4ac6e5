"""Benchmark: whole asymmetric-plmDCA pass on one MI355X.

One step = reweighting (0.8 identity) + the all-sites batched L-BFGS fit to
||grad g_r^reg||_2 <= 1e-6 (every per-site objective+gradient evaluation on the
GPU) + Ising-gauge/FN/APC scoring, on a seeded synthetic planted-Potts
alignment of N = 500 columns and B = 50000 rows (q = 21), resident in HBM.
`--workload ragged16` runs the ragged batch instead: 16 alignments with N in
[60, 300] and B in [2000, 30000], fitted together by plm_fit_batch.
`--method symmetric` fits the symmetric pseudolikelihood instead (one
minimisation over all parameters, plm_fit_symmetric) on the same alignment.
`--init mf` starts the fit from the mean-field estimate (plm_mf_init, inside
the timed step) instead of the origin.

metric: objective+gradient updates per second, one update being one
(site r, sequence b, column i, state s) term of the energy sums -- B*N*q per
site evaluation, B*N^2*q per evaluation of every site; converged sites are
not counted.  Also reported: time to fit, the same fit on the plain
single-site GPU path (one site per launch, eager, host sync every iteration;
sampled and extrapolated), per-kernel roofline of the dominant kernel, and the
FP64 CPU oracle on a bounded sample of the same evaluations.

The evaluation schedule (path, forward tile) is the autotuner's choice for
the workload, timed on the device before the warm-up (--path to force one).
A fit on the int8 fixed-point path (6) ends with the library's refinement fit
on path 5 (inside the timed step; its evaluations are counted and reported).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload W] [--path auto|0..6]
                       [--method asymmetric|symmetric] [--init zero|mf]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

Q = 21
# one FP32 add per lane per clock: 256 CUs x 64 lanes x 2.4 GHz
ALU_ADD_PEAK = 256 * 64 * 2.4e9
# dense BF16 matrix-core peak of the MI355X
MFMA_BF16_PEAK = 2.5e15
# dense int8 matrix-core peak (ops/s)
MFMA_I8_PEAK = 5.0e15
PATH_NAMES = {0: "gather_fp32", 1: "mfma_bf16x2", 2: "gather_mfma_fp32", 3: "mfma_fp32",
              4: "gather_mfma_f16x2", 5: "gather_mfma_i8x3", 6: "mfma_i8x3"}
# 16-bit pieces of the non-one-hot operand, per path: (forward, backward); 0 = LDS gather/scatter
PATH_PIECES = {0: (0, 0), 1: (2, 2), 2: (0, 3), 3: (3, 3), 4: (0, 2), 5: (0, 3), 6: (3, 3)}
# the int8 matrix-core kernels (path, direction)
INT8_KERNELS = {(5, "backward"), (6, "backward"), (6, "forward")}


def measured_traffic(kernel: str, workload: str):
    """Per-launch HBM bytes from the committed PMC summary, if it was taken on
    the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            d = json.load(fh)
    except Exception:
        return None
    from paper_1401_4832_amd.profiling import source_hash
    if d.get("source_hash") != source_hash(kernel):
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(s, w_np, beff, budget_s=12.0):
    """The FP64 oracle (as it stands) on a bounded sample of the same site
    evaluations: rounds of one site per host thread, at the origin, until
    about budget_s seconds of CPU work have run."""
    import numpy as np

    import oracle
    threads = oracle._threads()
    hr = np.zeros((threads, Q))
    Jr = np.zeros((threads, s.N, Q, Q))
    done = 0
    t = time.perf_counter()
    while True:
        sites = (np.arange(threads, dtype=np.int32) + done) % s.N
        oracle.objgrad_slices(s.msa, w_np, beff, hr, Jr, sites, nthreads=threads)
        done += threads
        dt = time.perf_counter() - t
        if dt >= budget_s:
            break
    units = done * s.B * s.N * Q
    return {"value": units / dt, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} site objective+gradient evaluations ({threads} threads, one site per "
                      f"thread per round) of the N={s.N}, B={s.B} alignment at h=J=0, FP64, {dt:.1f} s"}


def load_sets(name: str):
    import synth
    if name == "ragged16":
        return synth.ragged_set(16)
    return [synth.workload(name)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="potts_n500_b50000")
    ap.add_argument("--path", default="auto", help="auto (autotuner) or an evaluation path 0..6")
    ap.add_argument("--tile-seqs", type=int, default=0)
    ap.add_argument("--method", default="asymmetric", choices=("asymmetric", "symmetric"))
    ap.add_argument("--init", default="zero", choices=("zero", "mf"))
    ap.add_argument("--pseudocount", type=float, default=0.5)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--plain-sites", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (for HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the per-site "
              "problems would shard by site across GPUs; only the one-GPU path is implemented).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1401_4832_amd as plm

    dev = torch.device("cuda:0")
    sets = load_sets(args.workload)
    ragged = len(sets) > 1
    symmetric = args.method == "symmetric"
    mf_start = args.init == "mf"
    if mf_start and ragged:
        print("--init mf takes a single alignment", file=sys.stderr)
        sys.exit(2)
    if symmetric and ragged:
        print("--method symmetric takes a single alignment", file=sys.stderr)
        sys.exit(2)
    print(f"[bench] workload {args.workload}: " + ", ".join(f"N={s.N} B={s.B}" for s in sets),
          file=sys.stderr, flush=True)
    msas = [torch.from_numpy(s.msa).to(dev) for s in sets]
    torch.cuda.synchronize()
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def weights():
        return [plm.reweight(m, theta=0.8) for m in msas]

    # the schedule: the autotuner's choice for this workload (outside the timed region)
    tuned = None
    if args.path == "auto":
        items = [(m, w, beff) for m, (_, w, beff) in zip(msas, weights())]
        t = time.perf_counter()
        # the symmetric fit's tolerance is on the norm over all parameters: the
        # tuner weighs the fixed-point rounding against it over that many entries
        tuned = plm.autotune.choose(items, plm.FitOptions(tol=args.tol), Q, symmetric=symmetric)
        print(f"[bench] schedule path={tuned['path']} tile_seqs={tuned['tile_seqs']} "
              f"({time.perf_counter() - t:.1f} s to choose)", file=sys.stderr, flush=True)
        path, tile = int(tuned["path"]), int(tuned["tile_seqs"])
    else:
        path, tile = int(args.path), args.tile_seqs
    opts = plm.FitOptions(tol=args.tol, path=path, tile_seqs=tile, timing=True)

    mf_ms = []

    def start_point(w, beff):
        if not mf_start:
            return None, None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h0, J0 = plm.mf_init(msas[0], w, beff, pseudocount=args.pseudocount, q=Q)
        torch.cuda.synchronize()
        mf_ms.append((time.perf_counter() - t0) * 1e3)
        return h0, J0

    def step():
        ws = weights()
        if ragged:
            res = plm.fit_batch([(m, w, beff) for m, (_, w, beff) in zip(msas, ws)], opts)
        elif symmetric:
            _, w, beff = ws[0]
            h0, J0 = start_point(w, beff)
            res = [plm.fit_symmetric(msas[0], w, beff, opts, h0=h0, J0=J0)]
        else:
            _, w, beff = ws[0]
            h0, J0 = start_point(w, beff)
            res = [plm.fit(msas[0], w, beff, opts, h0=h0, J0=J0)]
        cfn = [plm.score(r.J)[1] for r in res]
        torch.cuda.synchronize()
        return ws, res, cfn

    for k in range(args.warmup):
        t = time.perf_counter()
        step()
        print(f"[bench] warmup {k} {time.perf_counter() - t:.2f} s", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    tot_time = 0.0
    tot_units = 0
    kt = dict(forward_ms=0.0, quant_ms=0.0, backward_ms=0.0, lbfgs_ms=0.0, iterations=0, site_evals=0,
              refine_forward_ms=0.0, refine_backward_ms=0.0, refine_lbfgs_ms=0.0, refine_iterations=0,
              refine_site_evals=0)
    last = None
    for k in range(args.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        last = step()
        dt = time.perf_counter() - t
        tm = plm.last_fit_timing(dev)
        for key in kt:
            kt[key] += tm[key]
        ws, res, _ = last
        # one symmetric evaluation covers every site of the alignment
        per_eval = (lambda s: s.B * s.N * s.N * Q) if symmetric else (lambda s: s.B * s.N * Q)
        units = sum(sum(st["evaluations"] for st in r.stats) * per_eval(s) for r, s in zip(res, sets))
        tot_time += dt
        tot_units += units
        print(f"[bench] step {k} {dt:.2f} s, site evals {tm['site_evals']}, "
              f"fwd {tm['forward_ms']:.0f} ms (quant {tm['quant_ms']:.0f}) bwd {tm['backward_ms']:.0f} ms lbfgs {tm['lbfgs_ms']:.0f} ms",
              file=sys.stderr, flush=True)
    ws, res, cfn = last
    statuses = {}
    for r in res:
        for st in r.stats:
            statuses[st["status"]] = statuses.get(st["status"], 0) + 1
    gmax = max(st["gnorm"] for r in res for st in r.stats)
    mu = 2 * min(0.01, 0.01 if symmetric else 0.005)

    # dominant kernel: the one with the largest share of device time, in the main
    # fit (the refinement fit, a few evaluations on another path, is left out)
    shares = {"backward": kt["backward_ms"] - kt["refine_backward_ms"],
              "forward": kt["forward_ms"] - kt["refine_forward_ms"],
              "lbfgs": kt["lbfgs_ms"] - kt["refine_lbfgs_ms"]}
    dom = max(shares, key=shares.get)
    main_evals = kt["site_evals"] - kt["refine_site_evals"]
    units_all = tot_units * (main_evals / kt["site_evals"] if kt["site_evals"] else 1.0)
    main_launches = kt["iterations"] - kt["refine_iterations"]
    roofline = None
    if dom in ("backward", "forward"):
        np_dom = PATH_PIECES[path][0 if dom == "forward" else 1]
        # the forward's time includes the coupling quantisation of path 6 (kernels of their own)
        t_kern = shares[dom] - (kt["quant_ms"] if dom == "forward" else 0.0)
        t_dom = t_kern * 1e-3
        if np_dom:
            # dense matrix-core flops of the one-hot product: q MACs per unit and piece
            flops = units_all * 2 * Q * np_dom
            # path 4's gradient is the grouped three-site kernel, path 5's its int8 form
            kname = {4: "backward_g3", 5: "backward_i8", 6: "backward_i8"}.get(path, "backward_mfma") \
                if dom == "backward" else ("forward_i8" if path == 6 else "forward_mfma")
            # BF16 and FP16 dense matrix-core peaks are the same on this chip; int8 runs at twice the rate
            peak = MFMA_I8_PEAK if (path, dom) in INT8_KERNELS else MFMA_BF16_PEAK
            roofline = {"bound": "mfma", "achieved": flops / t_dom / 1e12, "peak": peak / 1e12,
                        "unit": "TOP/s" if peak == MFMA_I8_PEAK else "TFLOP/s", "frac": flops / t_dom / peak,
                        "flops_per_unit": 2 * Q * np_dom}
        else:
            kname = dom
            adds = units_all  # one FP32 add per update in the gather or the scatter
            roofline = {"bound": "alu", "achieved": adds / t_dom / 1e12, "peak": ALU_ADD_PEAK / 1e12,
                        "unit": "TFLOP/s", "frac": adds / t_dom / ALU_ADD_PEAK, "flops_per_unit": 1}
        # (bytes were counted on one all-sites evaluation of the asymmetric fit; a fit's
        # launch covers only its active sites, so they are scaled by the units per launch)
        traffic_all = None if symmetric or ragged else measured_traffic(kname, args.workload)
        traffic = None
        if traffic_all is not None:
            s0 = sets[0]
            traffic = traffic_all * (units_all / max(1, main_launches)) / (s0.B * s0.N * s0.N * Q)
        roofline.update({"traffic": traffic, "traffic_all_sites_launch": traffic_all, "kernel": kname,
                         "launches": main_launches, "avg_launch_ms": t_kern / max(1, main_launches)})

    plain = None
    if not args.no_plain and not ragged and not symmetric and not mf_start:
        _, w, beff = ws[0]
        po = plm.FitOptions(tol=args.tol, path=path, tile_seqs=tile, single_site=True, site_limit=args.plain_sites)
        torch.cuda.synchronize()
        t = time.perf_counter()
        plm.fit(msas[0], w, beff, po)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - t
        est = dtp / args.plain_sites * sets[0].N
        plain = {"sites_sampled": args.plain_sites, "seconds_sampled": dtp,
                 "time_to_fit_s_extrapolated": est,
                 "speedup_batched_vs_plain": est / (tot_time / args.steps)}

    cpu = None
    if not args.no_cpu:
        k = max(range(len(sets)), key=lambda j: sets[j].B * sets[j].N ** 2)
        _, w, beff = ws[k]
        cpu = cpu_baseline(sets[k], w.cpu().numpy(), float(beff.item()))

    ms_per_step = tot_time / args.steps * 1e3
    if ragged:
        cfg = {"workload": args.workload, "alignments": len(sets), "N": [s.N for s in sets],
               "B": [s.B for s in sets]}
    else:
        cfg = {"workload": args.workload, "N": sets[0].N, "B": sets[0].B}
    cfg.update({"q": Q, "theta": 0.8, "lambda_h": 0.01, "lambda_J": 0.01, "tol": args.tol,
                "path": PATH_NAMES[path], "tile_seqs": tile, "schedule": "autotuned" if tuned else "fixed",
                "method": args.method, "init": args.init,
                "refine": (PATH_NAMES[4] if symmetric else PATH_NAMES[5])
                if (path == 6 or (symmetric and path == 5)) else None})
    if mf_start:
        cfg["pseudocount"] = args.pseudocount
    line = {
        "metric": "plm objective+gradient updates/s (B*N^2*q, active sites) and time-to-fit at <=1e-4 vs plain",
        "value": tot_units / tot_time,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {1: "bf16x2 operands, f32 accumulate", 4: "f32 forward, f16x2 gradient operands (22-bit), "
                  "FP64 reductions, FP32 L-BFGS history",
                  5: "f32 forward, int8x3 fixed-point gradient (2^-23), exact int32 accumulation, "
                  "FP64 reductions, FP32 L-BFGS history",
                  6: "int8x3 fixed-point energies (2^-22 max|J_r|) and gradient (2^-23), exact int32 "
                  "accumulation, FP32 softmax, FP64 reductions, FP32 L-BFGS history"}.get(
                      path, "f32 (FP64 reductions, FP32 L-BFGS history)")
        + ({PATH_NAMES[5]: "; refined to the tolerance on f32 energies with the int8x3 gradient",
            PATH_NAMES[4]: "; refined to the tolerance on f32 energies with the f16x2 gradient"}
           .get(cfg["refine"], "")),
        "data": "synthetic planted-Potts alignment (seeded Gibbs sampling)",
        "config": cfg,
        "time_to_fit_s": ms_per_step / 1e3,
        "fit": {"site_evals": kt["site_evals"], "iterations": kt["iterations"], "status": statuses,
                "max_gnorm": gmax, "coupling_error_bound_l2": gmax / mu},
        "kernel_ms": {k: kt[k] for k in ("forward_ms", "quant_ms", "backward_ms", "lbfgs_ms")},
        "refinement": {k: kt["refine_" + k] for k in ("site_evals", "iterations", "forward_ms", "backward_ms",
                                                       "lbfgs_ms")},
        "mf_init_ms": (sum(mf_ms[-args.steps:]) / args.steps) if mf_start else None,
        "roofline": roofline,
        "plain_single_site": plain,
        "cpu_baseline": cpu,
    }
    if tuned:
        line["tuning"] = {"candidates": tuned.get("candidates", [])}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
