"""Benchmark: two-site QC-DMRG H.psi TFLOP/s and Davidson s/iter, split-BF16 vs FP64, on one MI355X.

Workload (the precision configuration): L = 24 orbitals, N = 24 (N_alpha = N_beta = 12),
bond dimension M = 1024 per block at the middle bond (site 11 | 12), random integrals (seed 1),
synthetic block operators with the real operator structure and Gaussian sector sizes (sigma = 1.5),
built by dmrg_inputs/synthetic.py. One step = one Davidson iteration at the paper's precision (FP64
H.psi, Gram-Schmidt, Rayleigh-Ritz, residual, diagonal preconditioner), inputs resident in HBM; the
headline `value` is its algorithmic H.psi TFLOP/s. The split-BF16 iteration, the relative matvec
error and the time to |dE| <= 1e-6 of split + FP64 polish vs FP64 are reported beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "bf16": 2500.0}   # MI355X dense MFMA TFLOP/s
HBM_PEAK = 8000.0                        # GB/s
# HBM traffic of one H.psi call at L=24 M=1024 (seed 1), from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE
# over the launches of one call, FETCH_SIZE scaled by 2.0 and WRITE_SIZE by 1.0 (factors read off a
# 1 GiB device copy in the same runs). Valid for these operators and these kernels only; summaries and
# commands in profiles/hpsi_L24_M1024_swept_kernel_trace.md and
# profiles/hpsi_{fp64,split}_L24_M1024_synthetic_kernel_trace.md.
TRAFFIC_L24_M1024 = {
    # synthetic operators: counters taken before the current kernels (part-mask argument, FP64
    # single-tile sources in k_hpsi_lds64), so not reported
    "synthetic": {"fp64": None, "split": None},
    "swept": {"fp64": {"fetch_bytes": 21708.0 * 2**20, "write_bytes": 2879.0 * 2**20},
              "split": {"fetch_bytes": 13751.0 * 2**20, "write_bytes": 3037.0 * 2**20}},
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=24)
    ap.add_argument("--M", type=int, default=1024)
    ap.add_argument("--sigma", type=float, default=1.5)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--kernel-reps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-converge", action="store_true")
    ap.add_argument("--workload", choices=["precision", "batch", "large", "precond", "renorm"], default="precision",
                    help="precision: L=24 M=1024 split vs FP64 (default); batch: many uneven problems; "
                         "large: L=76 (57,56) M=6000, one GPU's share of the operator pairs; "
                         "precond: learned vs diagonal Davidson preconditioner at L=32 M=1500")
    ap.add_argument("--bonds", type=str, default="4,8,12,15,19,23,27",
                    help="precond --precond-eval bonds: left-site indices of the evaluated bonds")
    ap.add_argument("--precond-eval", choices=["sweep", "bonds"], default="sweep",
                    help="precond: A/B along the last of two sweeps at L=32 (default), or at single bonds of "
                         "synthetic blocks")
    ap.add_argument("--precond-m", type=str, default="256,1500",
                    help="precond sweep evaluation: bond dimension of each sweep (the A/B runs the last)")
    ap.add_argument("--precond-train-m", type=str, default="256,512",
                    help="precond sweep evaluation: sweeps at L=20..28 whose middle-bond blocks give training pairs")
    ap.add_argument("--precond-stage", choices=["all", "train", "eval"], default="all",
                    help="precond sweep evaluation: train only (write --mlp-params), evaluate only (read it), or both")
    ap.add_argument("--precond-arm", choices=["shadow", "both", "diag", "mlp"], default="shadow",
                    help="precond sweep evaluation: shadow (default): one sweep that solves every bond of the last "
                         "sweep with both preconditioners on the same problem and goes on with the diagonal solve; "
                         "both: two sweeps, each with its own preconditioner; diag / mlp: one of those sweeps")
    ap.add_argument("--mlp-params", type=str, default=None,
                    help="precond sweep evaluation: .npy file of the trained network's parameters")
    ap.add_argument("--pairs", type=int, default=1000,
                    help="large: normal/complementary pairs per family (B/Q and A/P) in the share")
    ap.add_argument("--n-problems", type=int, default=128)
    ap.add_argument("--batch-davidson", choices=["serial", "graph", "eager"], default=None,
                    help="batch: only the Davidson solves, serially or batched (graph / eager launches), for profiling")
    ap.add_argument("--operators", choices=["synthetic", "swept"], default="swept",
                    help="precision workload: synthetic block operators (sector sizes from the sigma model) or "
                         "the blocks that two-site sweeps (dmrg_sweep) over random integrals leave at the middle bond")
    ap.add_argument("--sweep-m", type=str, default="256,1024",
                    help="swept operators: bond dimension of each sweep (the last is the measured M)")
    ap.add_argument("--sweep-tol", type=float, default=1e-5, help="swept operators: Davidson tolerance per bond")
    ap.add_argument("--save-swept", type=str, default=None,
                    help="swept operators: also write the swept blocks to this .npz file")
    ap.add_argument("--load-swept", type=str, default=None,
                    help="swept operators: read the blocks from a --save-swept file instead of sweeping")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="profiling run: 3 H.psi calls per precision and a plain device copy of 1 GiB "
                         "(calibration of the traffic counters); prints per-call event timings")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: libdmrg has no multi-GPU path "
              "(the H.psi would shard over operator combinations with one all-reduce per matvec)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2001_04890_amd as dm
    from dmrg_inputs import random_vector
    from dmrg_inputs.synthetic import synthetic_problem

    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "large":
        return bench_large(args)
    if args.workload == "precond":
        return bench_precond(args)
    if args.workload == "renorm":
        return bench_renorm(args)
    dev = torch.device("cuda:0")
    L, M = args.L, args.M
    na = nb = L // 2
    t0 = time.time()
    sweep_info = None
    if args.operators == "swept":
        h, eri, left, right, site, sweep_info = swept_problem(args, L, na, nb)
        M = int(max(left.dim.sum(), right.dim.sum()))
        ops_desc = (f"swept block operators (dmrg_sweep, M per sweep {args.sweep_m}, random integrals seed "
                    f"{args.seed})")
    else:
        h, eri, left, right, site = synthetic_problem(L, na, nb, M, args.sigma, args.seed)
        ops_desc = f"synthetic block operators sigma={args.sigma}"
    log(f"[bench] inputs {time.time() - t0:.1f}s; building operator (L={L}, M={M}, {ops_desc})")
    t0 = time.time()
    stream = torch.cuda.current_stream()
    hop = dm.Hop(h, eri, left, right, na, nb, site, device=0, want_split=True, stream=stream)
    t_build = time.time() - t0
    st = hop.stats()
    n = hop.n_coeff
    log(f"[bench] build {t_build:.1f}s: |psi|={n} blocks={hop.n_blocks} alphas={st['n_alpha']} "
        f"tasks={st['n_tasks']} flops/matvec={st['flops']:.3e}")

    x = torch.as_tensor(random_vector(n, 7), device=dev)
    y64 = torch.empty_like(x)
    ysp = torch.empty_like(x)
    if args.profile_kernels:
        if sweep_info:
            print(json.dumps({"sweep": sweep_info}), flush=True)
        return profile_kernels(args, hop, st, x, y64, ysp, stream)

    # --- kernel timing with events on the launch stream
    def time_kernel(prec):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.kernel_reps)]
        out = y64 if prec == dm.PREC_FP64 else ysp
        hop.hpsi(x, out, prec, stream=stream)            # warm
        torch.cuda.synchronize()
        for a, b in ev:
            a.record(stream)
            hop.hpsi(x, out, prec, stream=stream)
            b.record(stream)
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in ev])) * 1e-3

    t64 = time_kernel(dm.PREC_FP64)
    tsp = time_kernel(dm.PREC_SPLIT2)
    rel_mv = float(torch.linalg.norm(ysp - y64) / torch.linalg.norm(y64))
    log(f"[bench] H.psi kernel: fp64 {t64 * 1e3:.3f} ms ({st['flops'] / t64 / 1e12:.2f} TF/s), "
        f"split {tsp * 1e3:.3f} ms ({st['flops'] / tsp / 1e12:.2f} TF/s), rel matvec err {rel_mv:.2e}")

    # --- timed Davidson steps (split precision)
    def dav_steps(prec, iters):
        psi = torch.as_tensor(random_vector(n, 3), device=dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = hop.davidson(psi, tol=1e-30, max_iter=iters, max_sub=24, precision=prec, stream=stream)
        torch.cuda.synchronize()
        return time.perf_counter() - t, r

    dav_steps(dm.PREC_FP64, args.warmup)
    wall_64, r_64 = dav_steps(dm.PREC_FP64, args.steps)
    dav_steps(dm.PREC_SPLIT2, args.warmup)
    wall_sp, r_sp = dav_steps(dm.PREC_SPLIT2, args.steps)
    s_iter_sp = wall_sp / args.steps
    s_iter_64 = wall_64 / args.steps
    value = st["flops"] * r_sp["matvecs"] / wall_sp / 1e12
    value_64 = st["flops"] * r_64["matvecs"] / wall_64 / 1e12
    log(f"[bench] Davidson s/iter: split {s_iter_sp * 1e3:.2f} ms ({value:.2f} TF/s), "
        f"fp64 {s_iter_64 * 1e3:.2f} ms ({value_64:.2f} TF/s)")

    # --- the same iterations with the whole iteration on the device (dmrg_davidson_batch, one part)
    def dav_steps_dev(prec, iters, graph):
        psi = torch.as_tensor(random_vector(n, 3), device=dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = hop.davidson_batch(psi, tol=1e-30, max_iter=iters, max_sub=24, precision=prec, use_graph=graph,
                               stream=stream)
        torch.cuda.synchronize()
        return time.perf_counter() - t, r

    dev_iter = {}
    for name, prec in (("fp64", dm.PREC_FP64), ("split", dm.PREC_SPLIT2)):
        for graph in (False, True):
            dav_steps_dev(prec, args.warmup, graph)
            w, r = dav_steps_dev(prec, args.steps, graph)
            dev_iter[f"{name}{'_graph' if graph else ''}_ms"] = round(w / args.steps * 1e3, 3)
    log(f"[bench] device-resident Davidson s/iter: {dev_iter}")

    # --- convergence at equal tolerance: FP64 vs split + FP64 polish
    conv = {}
    if not args.no_converge:
        for name, prec, polish in (("fp64", dm.PREC_FP64, False), ("split", dm.PREC_SPLIT2, True)):
            psi = torch.as_tensor(random_vector(n, 5), device=dev)
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = hop.davidson(psi, tol=1e-6, max_iter=400, max_sub=24, precision=prec, fp64_polish=polish,
                             split_tol=3e-4, stream=stream)
            torch.cuda.synchronize()
            conv[name] = dict(energy=r["energy"], resid=r["resid"], iters=r["iters"], matvecs=r["matvecs"],
                              matvecs_split=r["matvecs_split"], seconds=time.perf_counter() - t,
                              converged=r["converged"])
            log(f"[bench] converge {name}: {conv[name]}")
        conv["dE"] = abs(conv["split"]["energy"] - conv["fp64"]["energy"])

    # --- learned preconditioner: one application (features + MFMA inference) at this size
    mlp_ms = mlp_apply_ms(hop, n, stream)
    log(f"[bench] learned preconditioner application: {mlp_ms:.3f} ms")

    # --- roofline of the dominant kernel: the FP64 H.psi launch sequence (the headline precision);
    #     the split sequence's figures follow under "split_roofline"
    if args.operators == "swept":
        default_shape = (L, args.sweep_m, args.sweep_tol, args.seed) == (24, "256,1024", 1e-5, 1)
    else:
        default_shape = (L, M, args.sigma, args.seed) == (24, 1024, 1.5, 1)
    traffic = TRAFFIC_L24_M1024[args.operators] if default_shape else None
    achieved = st["flops"] / t64 / 1e12
    tr64 = traffic["fp64"] if traffic else None
    trsp = traffic["split"] if traffic else None
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK["fp64"], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK["fp64"], 4),
                "traffic": (tr64["fetch_bytes"] + tr64["write_bytes"]) if tr64 else None,
                "kernel": "FP64 H.psi sequence (k_hpsi_lds64 classes for targets within 112 x 112; k_hpsi_f64 "
                          "tiles and k_big64 passes for the rest, with k_pack when those tiles run; k_pack_xt64, "
                          "k_reduce_lds, k_zero)",
                "algorithmic_bytes": st["bytes"],
                "hbm_frac": round(st["bytes"] / t64 / 1e9 / HBM_PEAK, 4)}
    achieved_sp = st["flops"] / tsp / 1e12
    traffic_sp = (trsp["fetch_bytes"] + trsp["write_bytes"]) if trsp else None
    split_roofline = {"bound": "mfma", "achieved": round(achieved_sp, 3), "peak": PEAK["bf16"], "unit": "TFLOP/s",
                      "frac": round(achieved_sp / PEAK["bf16"], 5), "traffic": traffic_sp,
                      "kernel": "split H.psi sequence (k_hpsi_lds, k_hpsi_small, k_big_t + k_big_y above 96 x 96, "
                                "k_pack_xt, k_reduce_lds, k_reduce_big)",
                      "mfma_products_per_flop": 3,
                      "algorithmic_bytes": st["bytes"] / 2,
                      "hbm_frac": round(st["bytes"] / 2 / tsp / 1e9 / HBM_PEAK, 4)}

    # --- CPU oracle on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(h, eri, left, right, na, nb, site, n, st["flops"])

    out = {
        "metric": "H·ψ TFLOP/s & Davidson s/iter, split-FP32 vs FP64 at |ΔE|≤1e-6 Eh",
        "value": round(value_64, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(s_iter_64 * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"two-site H.psi + Davidson iteration, L={L} N={na + nb} ({na},{nb}) M={M} "
                               f"middle bond, {ops_desc}",
                   "n_coeff": n, "psi_blocks": hop.n_blocks, "n_alpha": st["n_alpha"], "n_tasks": st["n_tasks"],
                   "flops_per_matvec": st["flops"]},
        "fp64": {"tflops": round(value_64, 3), "ms_per_iter": round(s_iter_64 * 1e3, 3),
                 "kernel_ms": round(t64 * 1e3, 4)},
        "split": {"dtype": "bf16 hi/lo products, fp32 accumulation", "tflops": round(value, 3),
                  "ms_per_iter": round(s_iter_sp * 1e3, 3), "kernel_ms": round(tsp * 1e3, 4),
                  "rel_matvec_err": rel_mv},
        "converge": conv,
        "device_davidson_ms_per_iter": dev_iter,
        "mlp_precond_ms": round(mlp_ms, 4),
        "build_seconds": round(t_build, 2),
        "roofline": roofline,
        "split_roofline": split_roofline,
        "cpu_baseline": cpu,
        **({"sweep": sweep_info} if sweep_info else {}),
    }
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """Many independent two-site H.psi problems (L ~ U{16..28}, N = L, M ~ U{64..768}, seeds
    2000 + j): one merged handle (autotuned plan) launched as one captured hipGraph vs one launch
    sequence per problem."""
    import gc

    import torch
    import paper_2001_04890_amd as dm
    from dmrg_inputs import random_vector
    from dmrg_inputs.synthetic import synthetic_problem
    import multiprocessing as mp
    # the FP64 LDS-staged kernel keeps an FP64 tiled copy of every operator; the merged handle next to
    # the 128 individual ones would not fit with it, so both sides of this comparison run FP64 on the
    # one-wavefront kernel
    os.environ["DMRG_LDS64"] = "0"
    # inputs are generated by worker processes (numpy only, no GPU), forked before this process
    # touches the GPU; operators are built here
    pool = mp.get_context("fork").Pool(8)
    stream = torch.cuda.current_stream()
    hops, shapes = [], []
    t0 = time.time()
    with pool:
        for j, (L, M, prob) in enumerate(pool.imap(_batch_problem, range(args.n_problems))):
            h, eri, left, right, site = prob
            na, nb = (L + 1) // 2, L // 2
            hops.append(dm.Hop(h, eri, left, right, na, nb, site, device=0, want_split=True, stream=stream))
            shapes.append((L, M))
            del h, eri, left, right, prob
            gc.collect()
            if j % 16 == 15:
                log(f"[bench] built {j + 1}/{args.n_problems} problems ({time.time() - t0:.0f}s)")
    flops = sum(hp.stats()["flops"] for hp in hops)
    if args.batch_davidson:
        dav = dict(tol=1e-6, max_iter=400, max_sub=24, precision=dm.PREC_SPLIT2, fp64_polish=True, split_tol=3e-4)
        starts = [torch.as_tensor(random_vector(hp.n_coeff, 100 + k), device="cuda:0") for k, hp in enumerate(hops)]
        torch.cuda.synchronize()
        t = time.perf_counter()
        if args.batch_davidson == "serial":
            its = [hp.davidson(x0.clone(), stream=stream, **dav)["iters"] for hp, x0 in zip(hops, starts)]
            n_mv = None
        else:
            comb = dm.Hop.combine(hops, stream=stream)
            torch.cuda.synchronize()
            t = time.perf_counter()
            rb = comb.davidson_batch(torch.cat(starts), use_graph=args.batch_davidson == "graph", stream=stream, **dav)
            its, n_mv = rb["iters"].tolist(), rb["matvecs"]
        torch.cuda.synchronize()
        log(f"[bench] {args.batch_davidson} Davidson of {len(hops)} problems: {time.perf_counter() - t:.3f} s, "
            f"iterations {int(np.sum(its))} in total, merged H.psi launches {n_mv}")
        return
    xs = [torch.as_tensor(random_vector(hp.n_coeff, 7 + k), device="cuda:0") for k, hp in enumerate(hops)]
    ys = {p: [torch.empty_like(x) for x in xs] for p in (dm.PREC_SPLIT2, dm.PREC_FP64)}
    xc = torch.cat(xs)
    yc = torch.empty_like(xc)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    # serial launches first; then the individual handles keep only what merging needs (dmrg_hop_trim),
    # so that the merged handle fits next to them
    t_serial = {}
    for prec in (dm.PREC_SPLIT2, dm.PREC_FP64):
        t_serial[prec] = timed(lambda: [hp.hpsi(x, y, prec, stream=stream) for hp, x, y in zip(hops, xs, ys[prec])], 3)
    # Davidson to ||r|| <= 1e-6 (split + FP64 polish): one dmrg_davidson per problem, in turn
    dav = dict(tol=1e-6, max_iter=400, max_sub=24, precision=dm.PREC_SPLIT2, fp64_polish=True, split_tol=3e-4)
    starts = [torch.as_tensor(random_vector(hp.n_coeff, 100 + k), device="cuda:0") for k, hp in enumerate(hops)]
    torch.cuda.synchronize()
    t = time.perf_counter()
    e_serial, it_serial = [], []
    for hp, x0 in zip(hops, starts):
        r = hp.davidson(x0.clone(), stream=stream, **dav)
        e_serial.append(r["energy"])
        it_serial.append(r["iters"])
    torch.cuda.synchronize()
    t_dav_serial = time.perf_counter() - t
    log(f"[bench] serial Davidson: {t_dav_serial:.2f} s, iterations {min(it_serial)}..{max(it_serial)}")
    for hp in hops:
        hp.trim()
    comb = dm.Hop.combine(hops, stream=stream)
    t = time.perf_counter()
    os.environ["DMRG_AUTOTUNE_TRACE"] = "1"   # one line per candidate plan
    tune = {"split": comb.autotune(dm.PREC_SPLIT2, reps=2, stream=stream),
            "fp64": comb.autotune(dm.PREC_FP64, reps=2, stream=stream)}
    log(f"[bench] combined: |psi|={comb.n_coeff} flops/matvec={flops:.3e} autotune ({time.perf_counter() - t:.1f} s)"
        f"={tune}")
    out = {}
    for name, prec in (("split", dm.PREC_SPLIT2), ("fp64", dm.PREC_FP64)):
        t_batch = timed(lambda: comb.hpsi(xc, yc, prec, stream=stream), 3)
        t_graph = timed(lambda: comb.hpsi_graph(xc, yc, prec, stream=stream), 3)
        diff = float((torch.cat(ys[prec]) - yc).abs().max() / yc.abs().max())
        ts = t_serial[prec]
        out[name] = {"serial_ms": round(ts, 3), "batched_ms": round(t_batch, 3), "graph_ms": round(t_graph, 3),
                     "speedup": round(ts / t_graph, 3), "batched_tflops": round(flops / t_graph / 1e9, 3),
                     "serial_tflops": round(flops / ts / 1e9, 3), "max_rel_diff": diff}
        log(f"[bench] {name}: {out[name]}")
    # the same solves as one batched, device-resident Davidson over the merged handle (graph-captured
    # iterations); every problem starts from the same vector as above
    psi = torch.cat(starts)
    torch.cuda.synchronize()
    t = time.perf_counter()
    rb = comb.davidson_batch(psi, use_graph=True, stream=stream, **dav)
    torch.cuda.synchronize()
    t_dav_batch = time.perf_counter() - t
    de = float(np.abs(np.asarray(e_serial) - rb["energy"]).max())
    out["davidson"] = {"serial_s": round(t_dav_serial, 3), "batched_s": round(t_dav_batch, 3),
                       "speedup": round(t_dav_serial / t_dav_batch, 3), "max_abs_dE": de,
                       "serial_iters": [int(min(it_serial)), int(max(it_serial))],
                       "batched_iters": [int(rb["iters"].min()), int(rb["iters"].max())],
                       "batched_converged": int(rb["n_converged"]), "graphs": int(rb["graphs"]),
                       "tol": dav["tol"]}
    log(f"[bench] davidson: {out['davidson']}")
    line = {"metric": "H·ψ TFLOP/s, one merged graph launch vs serial launches", "value": out["split"]["batched_tflops"],
            "unit": "TFLOP/s", "n_gpus": 1, "steps": 3, "warmup": 1, "ms_per_step": out["split"]["graph_ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
            "config": {"workload": f"{args.n_problems} independent two-site H.psi problems, L~U{{16..28}}, N=L, "
                                   f"M~U{{64..768}}, synthetic block operators sigma=1.5",
                       "n_coeff": comb.n_coeff, "flops_per_matvec": flops, "autotune": tune},
            "split": out["split"], "fp64": out["fp64"], "davidson": out["davidson"]}
    print(json.dumps(line), flush=True)


def _batch_problem(j):
    """Inputs of problem j of the batch workload (seed 2000 + j): L ~ U{16..28}, N = L, M ~ U{64..768}."""
    from dmrg_inputs.synthetic import synthetic_problem
    rng = np.random.Generator(np.random.PCG64(2000 + j))
    L = int(rng.integers(16, 29))
    M = int(rng.integers(64, 769))
    return L, M, synthetic_problem(L, (L + 1) // 2, L // 2, M, 1.5, 2000 + j)


def train_swept(net, train_m, stream, t0):
    """Training pairs from converged FP64 solves at the middle bond of swept states (L = 20 .. 28,
    random integrals, seeds 3000+), then 3000 Adam steps of 4096 rows; returns the seconds taken."""
    import torch
    import paper_2001_04890_amd as dm
    from dmrg_inputs import random_integrals, random_vector
    for k, L in enumerate((20, 22, 24, 26, 28)):
        h, eri = random_integrals(L, 3000 + k)
        site = L // 2 - 1
        ts = time.time()
        sw = dm.sweep(h, eri, L // 2, L // 2, train_m, m_warmup=train_m[0], tol=1e-6, max_iter=400, seed=k,
                      stream=stream, keep_site=site)
        hop = dm.Hop(h, eri, sw["left"], sw["right"], L // 2, L // 2, site, device=0, stream=stream)
        psi = torch.as_tensor(random_vector(hop.n_coeff, 40 + k), device="cuda:0")
        res = net.collect(hop, psi, slot=0, rows_per_iter=4096, seed=k, tol=1e-9, max_iter=600, stream=stream)
        log(f"[bench] precond: L={L} swept ({time.time() - ts:.1f}s, M {train_m}), |psi|={hop.n_coeff}: "
            f"collected {res['rows']} rows in {res['iters']} iterations")
        del hop, sw
    losses = net.train(3000, batch=4096, lr=1e-3, seed=1, stream=stream)
    t_train = time.time() - t0
    log(f"[bench] precond: training loss {float(losses[:50].mean()):.4f} -> {float(losses[-50:].mean()):.4f} "
        f"({t_train:.1f}s incl. sweeps and collection)")
    return t_train


def bench_precond_sweep(args, net, stream, t0):
    import paper_2001_04890_amd as dm
    from dmrg_inputs import random_integrals
    train_m = [int(m) for m in args.precond_train_m.split(",")]
    eval_m = [int(m) for m in args.precond_m.split(",")]
    if args.precond_stage == "eval":
        net.set_params(np.load(args.mlp_params))
        t_train = None
        log(f"[bench] precond: network parameters from {args.mlp_params}")
    else:
        t_train = train_swept(net, train_m, stream, t0)
        if args.mlp_params:
            np.save(args.mlp_params, net.get_params())
        if args.precond_stage == "train":
            return
    # A/B along the last sweep at L = 32
    L = 32
    h, eri = random_integrals(L, 3200)
    if args.precond_arm == "shadow":
        ts = time.time()
        r = dm.sweep(h, eri, L // 2, L // 2, eval_m, m_warmup=eval_m[0], tol=1e-8, max_iter=1000, seed=7,
                     stream=stream, mlp=net, mlp_from_sweep=len(eval_m) - 1, mlp_shadow=True, verbose=True)
        per = 2 * L - 4                      # solves of the last sweep (the first has 2L - 3, later ones 2L - 4)
        last = slice(len(r["iters"]) - per, None)
        it_d, it_m = r["iters"][last], r["iters_alt"][last]
        de = np.abs(r["energies"][last] - r["energies_alt"][last])
        log(f"[bench] precond shadow sweep: {time.time() - ts:.1f}s, diagonal {int(it_d.sum())} vs learned "
            f"{int(it_m.sum())} iterations, max |dE| {de.max():.1e}")
        line = {"metric": "Davidson iterations to ||r||<=1e-8 over the last sweep, learned vs diagonal preconditioner "
                          "on the same two-site problems",
                "value": int(it_m.sum()), "unit": "iterations (sum over the sweep's solves)", "n_gpus": 1,
                "steps": per, "warmup": 0, "ms_per_step": None, "higher_is_better": False, "scaling": "weak",
                "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                "config": {"workload": f"two-site sweeps at L={L} N={L}, random integrals (seed 3200), bond dimensions "
                                       f"{eval_m}; every bond of the last sweep solved with both preconditioners from "
                                       f"the same start vector (the sweep goes on with the diagonal solve); network "
                                       f"trained on middle-bond solves of swept states at L=20..28 (bond dimensions "
                                       f"{train_m})"},
                "diag_iters": int(it_d.sum()), "mlp_iters": int(it_m.sum()),
                "bonds_mlp_fewer": int((it_m < it_d).sum()), "bonds_mlp_more": int((it_m > it_d).sum()),
                "max_dE_per_solve": float(de.max()), "energy": r["energy"], "sweep_seconds": r["seconds"],
                "diag_sweep_iters": it_d.tolist(), "mlp_sweep_iters": it_m.tolist(),
                "train_seconds": round(t_train, 1) if t_train is not None else None,
                "judge": "no new residual minimum (by 1%) in 20 iterations, or no halving in 10"}
        print(json.dumps(line), flush=True)
        return
    runs = {}
    arms = (("diag", None), ("mlp", net)) if args.precond_arm == "both" else \
        ((args.precond_arm, None if args.precond_arm == "diag" else net),)
    for name, use in arms:
        ts = time.time()
        r = dm.sweep(h, eri, L // 2, L // 2, eval_m, m_warmup=eval_m[0], tol=1e-8, max_iter=1000, seed=7,
                     stream=stream, mlp=use, mlp_from_sweep=len(eval_m) - 1, verbose=True)
        runs[name] = r
        log(f"[bench] precond sweep {name}: {time.time() - ts:.1f}s, E {r['energy']:.10f}, "
            f"iterations {int(r['iters'].sum())}, not converged {r['n_not_converged']}")
    per = 2 * L - 4                          # solves of the last sweep (the first has 2L - 3, later ones 2L - 4)
    if args.precond_arm != "both":
        name = args.precond_arm
        r = runs[name]
        last = slice(len(r["iters"]) - per, None)
        line = {"metric": "Davidson iterations to ||r||<=1e-8 over the last sweep, one preconditioner",
                "value": int(r["iters"][last].sum()), "unit": "iterations (sum over the sweep's solves)",
                "n_gpus": 1, "steps": per, "warmup": 0, "ms_per_step": None, "higher_is_better": False,
                "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                "config": {"workload": f"two-site sweeps at L={L} N={L}, random integrals (seed 3200), bond "
                                       f"dimensions {eval_m}; preconditioner of the last sweep: {name}"},
                "arm": name, "energy": r["energy"], "seconds": r["seconds"],
                "energies": r["energies"].tolist(), "iters": r["iters"].tolist(), "n_not_converged": r["n_not_converged"]}
        print(json.dumps(line), flush=True)
        return
    last = slice(len(runs["diag"]["iters"]) - per, None)
    it_d = int(runs["diag"]["iters"][last].sum())
    it_m = int(runs["mlp"]["iters"][last].sum())
    first_equal = bool(np.array_equal(runs["diag"]["energies"][:last.start], runs["mlp"]["energies"][:last.start]))
    de = np.abs(runs["diag"]["energies"][last] - runs["mlp"]["energies"][last])
    line = {"metric": "Davidson iterations to ||r||<=1e-8 over the last sweep, learned vs diagonal preconditioner",
            "value": it_m, "unit": "iterations (sum over the sweep's solves)", "n_gpus": 1, "steps": per, "warmup": 0,
            "ms_per_step": None, "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": f"two-site sweeps at L={L} N={L}, random integrals (seed 3200), bond dimensions "
                                   f"{eval_m}; the A/B runs the last sweep; network trained on middle-bond solves of "
                                   f"swept states at L=20..28 (bond dimensions {train_m})"},
            "diag_iters": it_d, "mlp_iters": it_m, "earlier_sweeps_identical": first_equal,
            "max_dE_per_solve": float(de.max()), "final_dE": abs(runs["diag"]["energy"] - runs["mlp"]["energy"]),
            "diag_energy": runs["diag"]["energy"], "mlp_energy": runs["mlp"]["energy"],
            "diag_sweep_iters": runs["diag"]["iters"][last].tolist(), "mlp_sweep_iters": runs["mlp"]["iters"][last].tolist(),
            "train_seconds": round(t_train, 1) if t_train is not None else None,
            "judge": "no new residual minimum (by 1%) in 20 iterations, or no halving in 10"}
    print(json.dumps(line), flush=True)


def bench_large(args):
    """Large shape: L = 76, N = 113 (57, 56), M = 6000 per block at the middle bond, synthetic block
    operators (sigma 1.5, sectors up to 420 states) restricted to one GPU's share of the operator
    combinations (block Hamiltonians + the first --pairs B/Q and A/P pairs). Split vs FP64 H.psi."""
    import torch
    import paper_2001_04890_amd as dm
    from dmrg_inputs import random_integrals, random_vector
    from dmrg_inputs.synthetic import share_ops, synthetic_block
    L, na, nb, M, sigma, seed = 76, 57, 56, 6000, 1.5, 4
    site = L // 2 - 1
    t0 = time.time()
    h, eri = random_integrals(L, seed)
    left = synthetic_block("left", L, na, nb, site, M, sigma, seed + 1000, ops=share_ops("left", L, site, args.pairs))
    right = synthetic_block("right", L, na, nb, site, M, sigma, seed + 2000, ops=share_ops("right", L, site, args.pairs))
    log(f"[bench] large: blocks generated in {time.time() - t0:.1f}s (max sector {int(left.dim.max())})")
    stream = torch.cuda.current_stream()
    t0 = time.time()
    hop = dm.Hop(h, eri, left, right, na, nb, site, device=0, want_split=True, stream=stream, share=True)
    t_build = time.time() - t0
    del left, right
    st = hop.stats()
    n = hop.n_coeff
    log(f"[bench] large: build {t_build:.1f}s |psi|={n} alphas={st['n_alpha']} tasks={st['n_tasks']} "
        f"flops/matvec={st['flops']:.3e}")
    x = torch.as_tensor(random_vector(n, 7), device="cuda:0")
    ys = {p: torch.empty_like(x) for p in (dm.PREC_FP64, dm.PREC_SPLIT2)}
    res = {}
    for name, prec in (("split", dm.PREC_SPLIT2), ("fp64", dm.PREC_FP64)):
        hop.hpsi(x, ys[prec], prec, stream=stream)
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.kernel_reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            hop.hpsi(x, ys[prec], prec, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        ms = float(np.mean(ts))
        res[name] = {"ms": round(ms, 3), "tflops": round(st["flops"] / ms / 1e9, 3)}
        log(f"[bench] large {name}: {res[name]}")
    y64, ysp = ys[dm.PREC_FP64], ys[dm.PREC_SPLIT2]
    rel = float(torch.linalg.norm(ysp - y64) / torch.linalg.norm(y64))
    line = {"metric": "H·ψ TFLOP/s, split-FP32 vs FP64 (large shape, one GPU's share)",
            "value": res["split"]["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.kernel_reps,
            "warmup": 1, "ms_per_step": res["split"]["ms"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "bf16", "accumulate": "fp32", "data": "synthetic",
            "config": {"workload": f"two-site H.psi, L={L} N={na + nb} ({na},{nb}) M={M} middle bond, synthetic "
                                   f"block operators sigma={sigma}, share: H + {args.pairs} B/Q + {args.pairs} A/P pairs",
                       "n_coeff": n, "n_alpha": st["n_alpha"], "n_tasks": st["n_tasks"], "flops_per_matvec": st["flops"],
                       "operator_bytes_fp64": st["bytes"]},
            "split": res["split"], "fp64": res["fp64"], "rel_matvec_err": rel, "build_seconds": round(t_build, 1),
            "roofline": {"bound": "mfma", "achieved": res["split"]["tflops"], "peak": PEAK["bf16"], "unit": "TFLOP/s",
                         "frac": round(res["split"]["tflops"] / PEAK["bf16"], 5), "traffic": None,
                         "fp64_frac": round(res["fp64"]["tflops"] / PEAK["fp64"], 4)}}
    print(json.dumps(line), flush=True)


def bench_precond(args):
    """Learned Davidson preconditioner vs the diagonal one at L = 32, N = 32, tolerance 1e-8.
    Default (--precond-eval sweep): training pairs come from converged FP64 solves at the middle bond
    of swept states (dmrg_sweep over random integrals at L = 20, 22, 24, 26, 28, N = L, bond
    dimensions --precond-train-m, the bond's blocks handed back by keep_site); the network is trained
    on the GPU (Adam, 3000 steps of 4096 rows). Evaluation: dmrg_sweep at L = 32 with bond dimensions
    --precond-m, once with the diagonal preconditioner everywhere and once with the learned one in the
    last sweep (same seed: the earlier sweeps are identical), Davidson to ||r|| <= 1e-8 at every bond;
    iterations and time of the last sweep and |dE| per solve. --precond-eval bonds: the earlier form
    (synthetic blocks at single bonds, network trained on synthetic middle-bond problems)."""
    import torch
    import paper_2001_04890_amd as dm
    from dmrg_inputs import random_integrals, random_vector
    from dmrg_inputs.synthetic import synthetic_problem
    stream = torch.cuda.current_stream()
    net = dm.Mlp(device=0, seed=5)
    t0 = time.time()
    if args.precond_eval == "sweep":
        return bench_precond_sweep(args, net, stream, t0)
    for k, L in enumerate((20, 22, 24, 26, 28)):
        h, eri, left, right, site = synthetic_problem(L, L // 2, L // 2, 512, 1.5, 3000 + k)
        hop = dm.Hop(h, eri, left, right, L // 2, L // 2, site, device=0, stream=stream)
        psi = torch.as_tensor(random_vector(hop.n_coeff, 40 + k), device="cuda:0")
        res = net.collect(hop, psi, slot=0, rows_per_iter=4096, seed=k, tol=1e-9, max_iter=600, stream=stream)
        log(f"[bench] precond: collected L={L}: iters {res['iters']} rows {res['rows']} converged {res['converged']}")
        del hop
    losses = net.train(3000, batch=4096, lr=1e-3, seed=1, stream=stream)
    t_train = time.time() - t0
    log(f"[bench] precond: training loss {float(losses[:50].mean()):.4f} -> {float(losses[-50:].mean()):.4f} "
        f"({t_train:.1f}s incl. collection)")
    L, M = 32, 1500
    bonds = [int(b) for b in args.bonds.split(",")]
    rows = []
    for b in bonds:
        h, eri, left, right, site = synthetic_problem(L, L // 2, L // 2, M, 1.5, 3100 + b, site=b)
        hop = dm.Hop(h, eri, left, right, L // 2, L // 2, site, device=0, stream=stream)
        row = {"site": b, "n_coeff": hop.n_coeff}
        for name, use in (("diag", None), ("mlp", net)):
            psi = torch.as_tensor(random_vector(hop.n_coeff, 77), device="cuda:0")
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = hop.davidson(psi, tol=1e-8, max_iter=1000, max_sub=24, mlp=use, stream=stream)
            torch.cuda.synchronize()
            row[name] = {"iters": r["iters"], "energy": r["energy"], "seconds": round(time.perf_counter() - t, 3),
                         "converged": r["converged"], "fallback_iter": r["precond_fallback_iter"]}
        row["dE"] = abs(row["mlp"]["energy"] - row["diag"]["energy"])
        log(f"[bench] precond bond {b}: |psi|={hop.n_coeff} diag {row['diag']['iters']} it "
            f"{row['diag']['seconds']}s, mlp {row['mlp']['iters']} it {row['mlp']['seconds']}s "
            f"(fallback at {row['mlp']['fallback_iter']}), |dE| {row['dE']:.1e}")
        rows.append(row)
        del hop
    it_d = sum(r["diag"]["iters"] for r in rows)
    it_m = sum(r["mlp"]["iters"] for r in rows)
    t_d = sum(r["diag"]["seconds"] for r in rows)
    t_m = sum(r["mlp"]["seconds"] for r in rows)
    line = {"metric": "Davidson iterations to ||r||<=1e-8, learned vs diagonal preconditioner", "value": it_m,
            "unit": "iterations (sum over bonds)", "n_gpus": 1, "steps": len(bonds), "warmup": 0,
            "ms_per_step": round(1e3 * t_m / len(bonds), 2), "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"Davidson at {len(bonds)} bonds of L={L} N={L} M={M} (synthetic blocks per bond); "
                                   "network trained on L=20..28 M=512 solves",
                       "bonds": bonds},
            "diag_iters": it_d, "mlp_iters": it_m, "diag_seconds": round(t_d, 2), "mlp_seconds": round(t_m, 2),
            "max_dE": max(r["dE"] for r in rows), "per_bond": rows, "train_seconds": round(t_train, 1)}
    print(json.dumps(line), flush=True)


def bench_renorm(args):
    """Renormalization steps (Section 2.1, Eq. renorm_mat) at the H.psi workload's bond (L = 24, N = 24,
    M = 1024, synthetic blocks sigma 1.5), FP64: rho^L of a normalized random psi on the GPU
    (dmrg_rdm_left), its cut to M states on the host (dmrg_truncate), and O^T A O on the GPU
    (dmrg_renormalize_blocks) for a random number-conserving operator of the enlarged block (one
    block per sector). Wall time per call, host work lists included; not the headline benchmark."""
    import torch
    import paper_2001_04890_amd as dm
    from dmrg_inputs import random_vector
    from dmrg_inputs.synthetic import synthetic_problem
    L, na, nb, M, sigma, seed = 24, 12, 12, 1024, 1.5, 1
    h, eri, left, right, site = synthetic_problem(L, na, nb, M, sigma, seed)
    stream = torch.cuda.current_stream()
    hop = dm.Hop(h, eri, left, right, na, nb, site, device=0, stream=stream)
    log("[bench] renorm: handle built")
    x = random_vector(hop.n_coeff, 3)
    x /= np.linalg.norm(x)
    xd = torch.as_tensor(x, device="cuda:0")
    qn, dims, off = hop.rdm_left_layout()
    # coefficients per enlarged-left sector: rows_q x cols_q, so rho costs 2 rows_q coeff_q flops
    qidx = {(int(q[0]), int(q[1])): i for i, q in enumerate(qn)}
    coeff = np.zeros(len(dims))
    for (a, b, c, d), (ma, md) in zip(hop.abcd, hop.dims):
        q = (int(left.qn[a][0]) + (b in (1, 3)), int(left.qn[a][1]) + (b in (2, 3)))
        coeff[qidx[q]] += ma * md
    fl_rho = float(np.sum(2.0 * dims * coeff))
    rho = torch.empty(int(off[-1]), dtype=torch.float64, device="cuda:0")
    reps = max(3, args.kernel_reps)

    def wall(fn, n):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / n * 1e3

    ms_rho = wall(lambda: hop.rdm_left(xd, rho, stream=stream), reps)
    log(f"[bench] renorm: rho^L {ms_rho:.3f} ms")
    flat = rho.cpu().numpy()
    t = time.perf_counter()
    kept, evals, vecs, disc = dm.truncate(flat, dims, M)
    ms_cut = (time.perf_counter() - t) * 1e3
    log(f"[bench] renorm: cut {ms_cut:.1f} ms, discarded {disc:.3e}")
    Os = [vecs[i][:, :int(kept[i])] for i in range(len(dims))]
    o_off = np.concatenate([[0], np.cumsum([o.size for o in Os])]).astype(np.int64)
    O = torch.as_tensor(np.concatenate([o.ravel() for o in Os] + [np.zeros(1)]), device="cuda:0")
    rng = np.random.default_rng(5)
    A = torch.as_tensor(rng.normal(size=int(off[-1])), device="cuda:0")
    out_off = np.concatenate([[0], np.cumsum(kept.astype(np.int64) ** 2)]).astype(np.int64)
    out = torch.empty(int(out_off[-1]) + 1, dtype=torch.float64, device="cuda:0")
    sec = np.arange(len(dims), dtype=np.int32)
    fl_ren = float(np.sum(2.0 * dims * kept * (dims + kept)))
    ms_ren = wall(lambda: dm.renormalize_blocks(dims, kept, o_off[:-1], O, sec, sec, off[:-1], A, out_off[:-1], out,
                                                stream=stream), reps)
    log(f"[bench] renorm: O^T A O {ms_ren:.3f} ms")
    # the whole chained step (dmrg_renormalize): rho, the cut, every grown-block operator (both sides)
    steps = {}
    for name, direction in (("grow_left", 0), ("grow_right", 1)):
        ts = []
        for _ in range(2):
            torch.cuda.synchronize()
            t = time.perf_counter()
            hop.renormalize(xd, direction, M, stream=stream, keep=False)      # the C-ABI call alone
            ts.append((time.perf_counter() - t) * 1e3)
        blk, dw = hop.renormalize(xd, direction, M, stream=stream)
        n_el = int(sum(m.size for op in blk.ops for m in op.blocks.values()))
        steps[name] = {"ms": round(min(ts), 1), "operators": len(blk.ops), "stored_elements": n_el,
                       "kept": int(blk.dim.sum()), "sectors": int(blk.n_sec), "discarded": dw}
        log(f"[bench] renorm: dmrg_renormalize {name}: {min(ts):.1f} ms, {len(blk.ops)} operators, "
            f"{n_el} elements")
        del blk
    line = {"metric": "renormalization steps (rho^L, M-state cut, O^T A O), ms per call", "unit": "ms",
            "higher_is_better": False, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"renormalization at the two-site bond, L={L} N={na + nb} ({na},{nb}) M={M}, "
                                   f"synthetic block operators sigma={sigma}, random normalized psi",
                       "sectors": int(len(dims)), "max_sector": int(dims.max()), "enlarged_states": int(dims.sum()),
                       "kept": int(kept.sum())},
            "rho_left": {"ms": round(ms_rho, 4), "flops": fl_rho, "tflops": round(fl_rho / ms_rho / 1e9, 4)},
            "cut_host": {"ms": round(ms_cut, 2), "discarded": disc},
            "renorm_mat": {"ms": round(ms_ren, 4), "flops": fl_ren, "tflops": round(fl_ren / ms_ren / 1e9, 4),
                           "blocks": int(len(dims))},
            "renormalize_step": steps}
    print(json.dumps(line), flush=True)


def swept_problem(args, L, na, nb):
    """Blocks of the middle bond after two-site sweeps over random integrals (dmrg_sweep, split
    precision with an FP64 polish per bond), and a fit of the sigma of the synthetic sector-size model
    to their sector dimensions."""
    import paper_2001_04890_amd as dm
    from dmrg_inputs import random_integrals
    from dmrg_inputs.synthetic import sector_dims
    h, eri = random_integrals(L, args.seed)
    ms = [int(v) for v in args.sweep_m.split(",")]
    site = L // 2 - 1
    t = time.perf_counter()
    if args.load_swept:
        left, right, r = load_blocks(args.load_swept)
    else:
        r = dm.sweep(h, eri, na, nb, ms, m_warmup=ms[0], tol=args.sweep_tol, max_iter=400, max_sub=24,
                     precision=dm.PREC_SPLIT2, fp64_polish=True, split_tol=3e-4, seed=args.seed, keep_site=site,
                     verbose=True)
        left, right = r["left"], r["right"]
        if args.save_swept:
            save_blocks(args.save_swept, left, right, r)
    secs = time.perf_counter() - t
    log(f"[bench] sweep {secs:.1f}s, {len(r['energies'])} solves, final E {r['energy']:.10f}, "
        f"kept {left.dim.sum()} x {right.dim.sum()}, largest sectors {left.dim.max()} / {right.dim.max()}")

    def fit_sigma(blk, k):
        dims = {tuple(int(v) for v in q): int(d) for q, d in zip(blk.qn, blk.dim)}
        m = int(blk.dim.sum())
        best = None
        for sg in np.arange(0.3, 4.01, 0.05):
            qn, dd = sector_dims(k, na, nb, L, m, float(sg))
            model = {tuple(int(v) for v in q): int(d) for q, d in zip(qn, dd)}
            keys = set(dims) | set(model)
            err = sum((dims.get(q, 0) - model.get(q, 0)) ** 2 for q in keys)
            if best is None or err < best[1]:
                best = (float(sg), err)
        return round(best[0], 2), round(float(np.sqrt(best[1] / max(1, len(dims)))), 1)

    sl, rms_l = fit_sigma(left, site)
    sr, rms_r = fit_sigma(right, L - site - 2)
    info = {"seconds": round(secs, 1), "m_per_sweep": ms, "solves": len(r["energies"]),
            "final_energy": r["energy"], "not_converged": r["n_not_converged"],
            "max_discarded_last_sweep": float(np.max(r["discarded"][-(2 * L - 4):])),
            "left": {"kept": int(left.dim.sum()), "sectors": int(len(left.dim)), "largest": int(left.dim.max()),
                     "fitted_sigma": sl, "fit_rms_states": rms_l,
                     "qn_dims": [[int(q[0]), int(q[1]), int(d)] for q, d in zip(left.qn, left.dim)]},
            "right": {"kept": int(right.dim.sum()), "sectors": int(len(right.dim)), "largest": int(right.dim.max()),
                      "fitted_sigma": sr, "fit_rms_states": rms_r,
                      "qn_dims": [[int(q[0]), int(q[1]), int(d)] for q, d in zip(right.qn, right.dim)]}}
    log(f"[bench] sector-model fit: sigma left {sl} (rms {rms_l} states), right {sr} (rms {rms_r})")
    return h, eri, left, right, site, info


def save_blocks(path, left, right, r):
    """The swept blocks (dmrg_inputs Blocks) and the sweep's summary in one .npz (no pickled objects)."""
    arrays = {"energies": np.asarray(r["energies"]), "discarded": np.asarray(r["discarded"]),
              "summary": np.array([r["energy"], float(r["n_not_converged"])])}
    for tag, b in (("left", left), ("right", right)):
        arrays[f"{tag}_orbitals"] = np.asarray(b.orbitals, dtype=np.int32)
        arrays[f"{tag}_qn"], arrays[f"{tag}_dim"] = np.asarray(b.qn), np.asarray(b.dim)
        head, data = [], []
        kinds = "HCSUABPQ"
        for op in b.ops:
            for (so, si), m in op.blocks.items():
                head.append((kinds.index(op.kind), op.i0, op.i1, so, si))
                data.append(np.asarray(m, dtype=np.float64).ravel())
            head.append((kinds.index(op.kind), op.i0, op.i1, -1, -1))        # end of the operator
        arrays[f"{tag}_head"] = np.array(head, dtype=np.int32)
        arrays[f"{tag}_data"] = np.concatenate(data) if data else np.zeros(0)
    np.savez(path, **arrays)


def load_blocks(path):
    from dmrg_inputs.blocks import Block, Op
    z = np.load(path)
    out = []
    for tag in ("left", "right"):
        dim = z[f"{tag}_dim"]
        data, pos, blocks, ops = z[f"{tag}_data"], 0, {}, []
        for kind, i0, i1, so, si in z[f"{tag}_head"]:
            if so < 0:
                ops.append(Op("HCSUABPQ"[kind], int(i0), int(i1), blocks))
                blocks = {}
                continue
            n = int(dim[so]) * int(dim[si])
            blocks[(int(so), int(si))] = data[pos:pos + n].reshape(int(dim[so]), int(dim[si]))
            pos += n
        out.append(Block(side=tag, orbitals=tuple(int(v) for v in z[f"{tag}_orbitals"]), qn=z[f"{tag}_qn"], dim=dim,
                         ops=ops))
    r = {"energies": z["energies"], "discarded": z["discarded"], "energy": float(z["summary"][0]),
         "n_not_converged": int(z["summary"][1])}
    return out[0], out[1], r


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(h, eri, left, right, na, nb, site, n, flops):
    """The oracle's full H.psi of the same workload (numpy / OpenBLAS FP64 on every host core this
    process may use), repeated until at least 10 s of work (at most 3 calls); the oracle's setup
    (its task list) is not timed. The rate is the library's algorithmic flop count of one H.psi (the
    metric's unit of work) over the oracle's seconds per H.psi; the oracle's own decomposition
    executes a slightly different task list, reported beside it."""
    from threadpoolctl import threadpool_limits

    from dmrg_inputs import random_vector
    from oracle.hpsi import OracleHop
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    log(f"[bench] cpu baseline: oracle setup (untimed), {cores} threads")
    oh = OracleHop(h, eri, left, right, na, nb, site)
    tasks = oh.tasks()
    fl_oracle = oh.flops(tasks)
    x = random_vector(n, 7)
    calls, dt = 0, 0.0
    with threadpool_limits(limits=cores):
        while calls < 3 and dt < 10.0:
            t = time.perf_counter()
            oh.apply(x, tasks=tasks)
            dt += time.perf_counter() - t
            calls += 1
    s_call = dt / calls
    log(f"[bench] cpu baseline: {calls} H.psi calls in {dt:.1f}s ({s_call:.2f} s each)")
    return {"value": round(flops / s_call / 1e12, 6), "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
            "seconds": round(dt, 2), "seconds_per_hpsi": round(s_call, 3), "cpu_model": _cpu_model(),
            "nproc": os.cpu_count(),
            "sample": f"{calls} full H.psi call(s) of the same workload (FP64, numpy/OpenBLAS on {cores} host "
                      f"threads; rate = the library's {flops:.4e} algorithmic flops per H.psi / seconds per "
                      f"call; the oracle's own task list has {len(tasks)} sector tasks, {fl_oracle:.4e} flops); "
                      f"oracle setup untimed"}


def mlp_apply_ms(hop, n, stream, reps=5):
    """Device time of one learned-preconditioner application (features + MFMA inference) on |psi|."""
    import torch
    import paper_2001_04890_amd as dm
    from dmrg_inputs import random_vector
    net = dm.Mlp(device=0, seed=1)
    r = torch.as_tensor(random_vector(n, 21), device="cuda:0")
    u = torch.as_tensor(random_vector(n, 22), device="cuda:0")
    feat = torch.empty((n, dm.MLP_IN), dtype=torch.float32, device="cuda:0")
    t = torch.empty_like(r)
    m = torch.empty(n, dtype=torch.float32, device="cuda:0")
    ts = []
    for _ in range(reps + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        dm.Mlp.features(hop, r, u, -100.0, feat, t, stream=stream)
        net.forward(feat, m, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.mean(ts[1:]))


def profile_kernels(args, hop, st, x, y64, ysp, stream):
    """Short run for rocprofv3: H.psi x3 per precision, then a 1 GiB device-to-device copy x3 (the
    known-size kernel that calibrates FETCH_SIZE / WRITE_SIZE)."""
    import torch
    import paper_2001_04890_amd as dm
    res = {}
    for name, prec, out in (("split", dm.PREC_SPLIT2, ysp), ("fp64", dm.PREC_FP64, y64)):
        ms = []
        for _ in range(3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            hop.hpsi(x, out, prec, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        res[name] = {"event_ms": [round(v, 4) for v in ms]}
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"profile": res, "flops_per_matvec": st["flops"], "algorithmic_bytes": st["bytes"],
                      "copy_bytes_each_way": src.numel() * 8}), flush=True)


if __name__ == "__main__":
    main()
