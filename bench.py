#!/usr/bin/env python
"""Benchmark of the ESMP2-TOP(1) hot path on one MI355X.

Workload: n_occ=16, n_vir=160, n_aux=480, seed 2 (synthetic ESMF-shaped
inputs, resident in HBM before the timed region).

A step is one pass of the whole hot path: rotation to the TOP basis,
right-hand side + S-triple energy, FP64 Jacobi-preconditioned CG to
||b+Ax||_W/||b||_W <= 1e-8 and E2, with the Krylov solve in the
pinned-semicanonical basis (the library's fastest FP64 solve; E2 is the same
in every basis).  ms_per_step is that step's time-to-E2.  The same steps are
also timed with the solve in the TOP basis and with the mixed-precision solves
(FP32 inner CG inside FP64 refinement, and the same around the operator with
BF16 Sylvester operands; same FP64 stopping test), each with its E2 difference.

value = H0-sigma GFLOP/s of the paper's operator (the TOP-basis sigma, all
its kernels, FP64): algorithmic sigma flops / sigma time, timed with HIP events
on the library's stream.  The roofline object covers its dominant kernel (the
virtual-pair Sylvester kernel on the FP64 matrix cores), timed with HIP events
around each of its launches in sigma applications of their own.  cpu_baseline times the CPU oracle's sigma on the same
workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 matrix peak
PEAK_FP32_TFLOPS = 157.3     # MI355X dense FP32 matrix peak
PEAK_BF16_TFLOPS = 2500.0    # MI355X dense BF16 matrix peak
PEAK_HBM_GBS = 8000.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 32-state batched workload")
    ap.add_argument("--counter-run", type=int, default=0, metavar="N",
                    help="for hardware-counter passes: a 256 MiB device copy (the calibration "
                         "kernel of known size), then N FP64 and N FP32 sigma applications in the TOP "
                         "basis and N FP64 in the pinned-semicanonical basis; no timing")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "sharding of the path is described in DESIGN.md but not implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_2003_12923_amd as P
    from paper_2003_12923_amd import costs

    if args.counter_run:
        counter_run(args)
        return

    prob = synth.config_problem(args.workload)
    no, nv = prob.n_occ, prob.n_vir
    vv_flops, oo_flops = costs.sigma_flops(no, nv)
    sig_flops = vv_flops + oo_flops
    torch.cuda.set_device(0)
    h = P.Handle(0).load(prob)
    torch.cuda.synchronize()

    def step(precision=P.ESMP2_FP64, basis=P.ESMP2_BASIS_TOP):
        h.rotate_top(lam_out=False)
        h.build_rhs(e2_s=False)
        return h.solve(tol=args.tol, max_iter=300, precision=precision, basis=basis)

    def timed(precision, basis):
        for _ in range(args.warmup):
            step(precision, basis)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r = step(precision, basis)
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / args.steps, r

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    n_sigma = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
        n_sigma += res["iterations"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    ms_per_step = 1e3 * wall / args.steps
    value = n_sigma * sig_flops / wall / 1e9

    # the same steps with the mixed-precision solve
    for _ in range(args.warmup):
        step(P.ESMP2_FP32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res_m = step(P.ESMP2_FP32)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mixed_ms = 1e3 * (t1 - t0) / args.steps

    # the same steps refined around the BF16 operator (TOP basis: BF16 operands
    # in the Sylvester products, FP32 elsewhere, FP64 refinement)
    for _ in range(args.warmup):
        step(P.ESMP2_BF16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res_b = step(P.ESMP2_BF16)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    bf16_ms = 1e3 * (t1 - t0) / args.steps

    # the same solves in the pinned-semicanonical basis
    sc_ms, res_sc = timed(P.ESMP2_FP64, P.ESMP2_BASIS_SEMICANONICAL)
    scm_ms, res_scm = timed(P.ESMP2_FP32, P.ESMP2_BASIS_SEMICANONICAL)

    # sigma alone (all its kernels), FP64 and FP32; events on the library's stream
    n_amp, _ = h.space()
    x = torch.from_numpy(synth.random_amplitudes(n_amp, 5)).cuda()

    def time_sigma(xv, precision, reps=20):
        y = torch.empty_like(xv)
        for _ in range(3):
            h.sigma(xv, y, precision)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            h.sigma(xv, y, precision)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    sigma_ms = time_sigma(x, P.ESMP2_FP64)
    sigma32_ms = time_sigma(x.float(), P.ESMP2_FP32)
    sigmab_ms = time_sigma(x.float(), P.ESMP2_BF16)

    # the Sylvester kernel alone: HIP events on the library's stream around each
    # of its launches in 20 more sigma applications per precision (nothing runs
    # beside them; inside a solve the S-triple sum may share the GPU)
    def profile_vv(xv, precision, reps=20):
        y = torch.empty_like(xv)
        h.profile(True)
        for _ in range(reps):
            h.sigma(xv, y, precision)
        torch.cuda.synchronize()
        return h.profile(False)[precision]

    vv_ms, vv_n = profile_vv(x, P.ESMP2_FP64)
    vv32_ms, vv32_n = profile_vv(x.float(), P.ESMP2_FP32)
    vvb_ms, vvb_n = profile_vv(x.float(), P.ESMP2_BF16)

    # the batched workload: 32 independent states of uneven size, one handle and one
    # stream each, set up concurrently and solved together (pinned-semicanonical
    # basis, FP64: every CG step one launch over all states, stops decided on the device)
    batch = None
    if not args.no_batch:
        hs = [P.Handle(0, stream="new").load(synth.make_problem(*sz)) for sz in synth.batched_sizes()]
        torch.cuda.synchronize()
        P.solve_batch(hs, tol=args.tol, basis=P.ESMP2_BASIS_SEMICANONICAL)          # warm-up
        t0 = time.perf_counter()
        rb = P.solve_batch(hs, tol=args.tol, basis=P.ESMP2_BASIS_SEMICANONICAL)
        batch_ms = 1e3 * (time.perf_counter() - t0)
        t0 = time.perf_counter()
        for hh in hs:
            hh.rotate_top(lam_out=False)
            hh.build_rhs(e2_s=False)
            hh.solve(tol=args.tol, max_iter=300, basis=P.ESMP2_BASIS_SEMICANONICAL)
        torch.cuda.synchronize()
        seq_ms = 1e3 * (time.perf_counter() - t0)
        gb = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_values.json"))).get("c4")
        err = None if gb is None else max(abs(r["e2"] - g["e2"]) for r, g in zip(rb, gb["states"]))
        batch = {"states": len(hs), "ms": round(batch_ms, 3), "states_per_s": round(len(hs) / batch_ms * 1e3, 2),
                 "one_by_one_ms": round(seq_ms, 3), "speedup_vs_one_by_one": round(seq_ms / batch_ms, 3),
                 "max_abs_e2_minus_oracle": err, "basis": "pinned semicanonical", "dtype": "f64"}
        # the same states in the TOP basis, Sylvester tile variant chosen per
        # (n_occ, n_vir) class by the autotuner (FP64)
        t0 = time.perf_counter()
        choice = {}
        for hh, sz in zip(hs, synth.batched_sizes()):
            key = (sz[0], sz[1])
            if key not in choice:
                choice[key] = hh.autotune(P.ESMP2_FP64, reps=3)[0]
        tune_ms = 1e3 * (time.perf_counter() - t0)
        P.solve_batch(hs, tol=args.tol, basis=P.ESMP2_BASIS_TOP)           # warm-up
        t0 = time.perf_counter()
        rt = P.solve_batch(hs, tol=args.tol, basis=P.ESMP2_BASIS_TOP)
        top_ms = 1e3 * (time.perf_counter() - t0)
        errt = None if gb is None else max(abs(r["e2"] - g["e2"]) for r, g in zip(rt, gb["states"]))
        hist = {}
        for v in choice.values():
            hist[str(v)] = hist.get(str(v), 0) + 1
        batch["top_basis_autotuned"] = {"ms": round(top_ms, 3), "states_per_s": round(len(hs) / top_ms * 1e3, 2),
                                        "max_abs_e2_minus_oracle": errt, "classes": len(choice),
                                        "variant_histogram": hist, "autotune_ms": round(tune_ms, 3)}
        for hh in hs:
            hh.close()
        del hs

    # the adjoint: dE2/dF~ and dE2/dB~ after the FP64 solve, on the differentiation
    # workload (n_occ=8, n_vir=80, n_aux=240, seed 4) and on this workload
    grad = {}
    gall = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_values.json")))
    for wl in ("c5", args.workload):
        pg = synth.config_problem(wl)
        hg = P.Handle(0).load(pg)
        ng = pg.n_occ + pg.n_vir
        hg.rotate_top(lam_out=False)
        hg.build_rhs()
        namp_g, _ = hg.space()
        xg = torch.empty(namp_g, dtype=torch.float64, device="cuda")
        dFg = torch.empty((ng, ng), dtype=torch.float64, device="cuda")
        dBg = torch.empty((pg.n_aux, ng, ng), dtype=torch.float64, device="cuda")
        rg = hg.solve(tol=1e-10, max_iter=500, basis=P.ESMP2_BASIS_SEMICANONICAL, x_out=xg)
        hg.gradient(xg, dFg, dBg)                       # first call allocates the workspace
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 3
        ev0.record()
        for _ in range(reps):
            hg.gradient(xg, dFg, dBg)
        ev1.record()
        torch.cuda.synchronize()
        g_ms = ev0.elapsed_time(ev1) / reps
        t0 = time.perf_counter()
        hg.rotate_top(lam_out=False)
        hg.build_rhs()
        hg.solve(tol=1e-10, max_iter=500, basis=P.ESMP2_BASIS_SEMICANONICAL, x_out=xg)
        hg.gradient(xg, dFg, dBg)
        torch.cuda.synchronize()
        fb_ms = 1e3 * (time.perf_counter() - t0)
        entry = {"n_occ": pg.n_occ, "n_vir": pg.n_vir, "n_aux": pg.n_aux, "gradient_ms": round(g_ms, 3),
                 "e2_and_gradient_ms": round(fb_ms, 3), "e2": rg["e2"], "solve_tol": 1e-10}
        gg = gall.get(wl + "_grad")
        if gg is not None:
            dFh, dBh = dFg.cpu().numpy(), dBg.cpu().numpy()
            sc = max(abs(dFh).max(), abs(dBh).max())
            err = max(max(abs(dFh[a, b] - v) for (a, b), v in zip(gg["f_entries"], gg["f_grad"])),
                      max(abs(dBh[Q, a, b] - v) for (Q, a, b), v in zip(gg["b_entries"], gg["b_grad"])))
            entry["max_err_vs_oracle_samples_rel"] = err / sc
        grad[wl] = entry
        hg.close()
        del xg, dFg, dBg

    vv_avg_ms = vv_ms / max(vv_n, 1)
    achieved = vv_flops / (vv_avg_ms * 1e-3) / 1e12
    # HBM bytes per launch from the committed counter passes, valid while the
    # kernel source is the one they were taken on
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "k_vv3_c3_traffic.json")
    if os.path.exists(tfile):
        import hashlib
        t = json.load(open(tfile))
        srcs = [os.path.join(ROOT, "paper_2003_12923_amd", "csrc", f) for f in ("vv3.hip", "vv3.h")]
        digest = hashlib.sha256(b"".join(open(f, "rb").read() for f in srcs)).hexdigest()
        if t.get("workload") == args.workload and t.get("source_sha256") == digest:
            traffic = round(t["fetch_bytes"] + t["write_bytes"])

    gold = None
    gfile = os.path.join(ROOT, "tests", "golden", "oracle_values.json")
    if os.path.exists(gfile):
        gold = json.load(open(gfile)).get(args.workload)

    sigma_gflops = sig_flops / sigma_ms / 1e6
    out = {
        "metric": "H0 sigma GFLOP/s + time-to-E2 (1e-8 resid), FP64 vs mixed at 1e-6 Eh, N_o=16",
        "value": round(sigma_gflops, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sc_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"ESMP2-TOP(1) singlet, n_occ={no}, n_vir={nv}, n_aux={prob.n_aux}, "
                               f"seed {prob.seed}, PCG to 1e-8",
                   "n_amplitudes": n_amp, "sigma_alg_flops": sig_flops},
        "time_to_e2_ms": round(sc_ms, 4),
        "sigma_fp64": {"ms": round(sigma_ms, 4), "gflops": round(sigma_gflops, 2),
                       "frac_fp64_peak": round(sigma_gflops / 1e3 / PEAK_FP64_TFLOPS, 4),
                       "alg_flops": sig_flops, "basis": "TOP (the paper's operator)"},
        "fp64_top_basis": {"time_to_e2_ms": round(ms_per_step, 4), "e2": res["e2"],
                           "iterations": res["iterations"], "rel_resid": res["rel_resid"],
                           "e2_minus_oracle": None if gold is None else res["e2"] - gold["e2"],
                           "effective_sigma_gflops": round(value, 2)},
        "mixed_top_basis": {"time_to_e2_ms": round(mixed_ms, 4), "speedup_vs_fp64": round(ms_per_step / mixed_ms, 3),
                  "e2": res_m["e2"], "e2_minus_fp64": res_m["e2"] - res["e2"],
                  "e2_minus_oracle": None if gold is None else res_m["e2"] - gold["e2"],
                  "inner_fp32_iterations": res_m["iterations"], "outer_fp64_steps": res_m["outer"],
                  "rel_resid": res_m["rel_resid"], "sigma_fp32_ms": round(sigma32_ms, 4),
                  "sigma_fp32_gflops": round(sig_flops / sigma32_ms / 1e6, 2),
                  "sylvester_fp32": {"avg_launch_ms": round(vv32_ms / max(vv32_n, 1), 4), "launches": vv32_n,
                                     "achieved_tflops": round(vv_flops / (vv32_ms / max(vv32_n, 1) * 1e-3) / 1e12, 3),
                                     "peak_tflops": PEAK_FP32_TFLOPS}},
        "mixed_bf16_top_basis": {"time_to_e2_ms": round(bf16_ms, 4), "speedup_vs_fp64": round(ms_per_step / bf16_ms, 3),
                  "e2": res_b["e2"], "e2_minus_fp64": res_b["e2"] - res["e2"],
                  "e2_minus_oracle": None if gold is None else res_b["e2"] - gold["e2"],
                  "inner_iterations": res_b["iterations"], "outer_fp64_steps": res_b["outer"],
                  "rel_resid": res_b["rel_resid"], "sigma_bf16_ms": round(sigmab_ms, 4),
                  "sigma_bf16_gflops": round(sig_flops / sigmab_ms / 1e6, 2),
                  "sylvester_bf16": {"avg_launch_ms": round(vvb_ms / max(vvb_n, 1), 4), "launches": vvb_n,
                                     "achieved_tflops": round(vv_flops / (vvb_ms / max(vvb_n, 1) * 1e-3) / 1e12, 3),
                                     "peak_tflops": PEAK_BF16_TFLOPS}},
        "semicanonical": {
            "fp64": {"time_to_e2_ms": round(sc_ms, 4), "speedup_vs_top_fp64": round(ms_per_step / sc_ms, 3),
                     "e2": res_sc["e2"], "iterations": res_sc["iterations"],
                     "rel_resid": res_sc["rel_resid"], "e2_minus_top_fp64": res_sc["e2"] - res["e2"],
                     "e2_minus_oracle": None if gold is None else res_sc["e2"] - gold["e2"]},
            "mixed": {"time_to_e2_ms": round(scm_ms, 4), "speedup_vs_semican_fp64": round(sc_ms / scm_ms, 3),
                      "inner_fp32_iterations": res_scm["iterations"],
                      "outer_fp64_steps": res_scm["outer"], "rel_resid": res_scm["rel_resid"],
                      "e2_minus_top_fp64": res_scm["e2"] - res["e2"]}},
        "batched_32_states": batch,
        "gradient_fp64": grad,
        "roofline": {"bound": "mfma", "kernel": "k_vv3 (virtual-pair Sylvester, FP64 MFMA)",
                     "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": traffic,
                     "alg_flops_per_launch": vv_flops, "avg_launch_ms": round(vv_avg_ms, 4),
                     "alg_bytes_per_launch": 16 * n_amp,
                     "launches": vv_n},
    }
    h.close()

    if not args.no_cpu_baseline:
        # the GPU's time-to-E2 on the same smaller workload (FP64, pinned-semicanonical solve)
        p2 = synth.config_problem("c2")
        h2 = P.Handle(0).load(p2)
        c2_ms = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h2.rotate_top(lam_out=False)
            h2.build_rhs(e2_s=False)
            h2.solve(tol=args.tol, max_iter=300, basis=P.ESMP2_BASIS_SEMICANONICAL)
            torch.cuda.synchronize()
            c2_ms.append(1e3 * (time.perf_counter() - t0))
        h2.close()
        out["cpu_baseline"] = cpu_baseline(prob, sig_flops, min(c2_ms[1:]))
    print(json.dumps(out), flush=True)


def counter_run(args):
    """Kernels for the hardware-counter passes: one copy of 2^25 doubles (256 MiB
    read + 256 MiB written), then sigma applications of the workload: N FP64 and
    N FP32 in the TOP basis, N FP64 in the pinned-semicanonical basis."""
    import torch
    import synth
    import paper_2003_12923_amd as P
    src = torch.ones(1 << 25, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print("copy done", flush=True)
    prob = synth.config_problem(args.workload)
    h = P.Handle(0).load(prob)
    h.rotate_top(lam_out=False)
    n_amp, _ = h.space()
    x = torch.from_numpy(synth.random_amplitudes(n_amp, 5)).cuda()
    y = torch.empty_like(x)
    for _ in range(args.counter_run):
        h.sigma(x, y)
    x32, y32 = x.float(), torch.empty(n_amp, dtype=torch.float32, device="cuda")
    for _ in range(args.counter_run):
        h.sigma(x32, y32, P.ESMP2_FP32)
    # the operator of the pinned-semicanonical basis (the timed solve's), FP64
    h.build_rhs(e2_s=False)
    for _ in range(args.counter_run):
        h.sigma_basis(x, y, P.ESMP2_FP64, P.ESMP2_BASIS_SEMICANONICAL)
    torch.cuda.synchronize()
    h.close()
    print("sigma done", flush=True)


def blas_threads():
    """Threads of the BLAS pool NumPy's contractions run on (threadpoolctl), else
    the OpenMP setting."""
    try:
        import threadpoolctl
        n = [p["num_threads"] for p in threadpoolctl.threadpool_info() if p.get("user_api") == "blas"]
        if n:
            return max(n)
    except Exception:
        pass
    return int(os.environ.get("OMP_NUM_THREADS", "1"))


def cpu_baseline(prob, sig_flops, gpu_c2_ms, reps=3):
    """The CPU oracle (numpy FP64, as it stands): `reps` applications of its
    TOP-basis sigma on the timed workload (the same operator and flop count as
    `value`), and its whole time-to-E2 (rotation, right-hand side, S-triple
    energy, Jacobi PCG to the same tolerance) on the n_occ=10, n_vir=100
    workload beside the GPU's."""
    import numpy as np
    import synth
    from oracle import structured, topbasis
    lam, R = topbasis.top_rotation(prob.F, prob.C, prob.n_occ)
    Ft, Bt = topbasis.rotate(prob.F, prob.B, R)
    op = structured.Structured(Ft, lam, prob.n_occ)
    x = synth.random_amplitudes(op.dim, 5)
    t = time.perf_counter()
    for _ in range(reps):
        op.sigma(x)
    dt = (time.perf_counter() - t) / reps
    p2 = synth.config_problem("c2")
    t = time.perf_counter()
    r2 = structured.solve_problem(p2, tol=1e-8, max_iter=300)
    t2 = time.perf_counter() - t
    return {"value": round(sig_flops / dt / 1e9, 4), "unit": "GFLOP/s", "cores": blas_threads(), "kind": "oracle",
            "sample": f"{reps} sigma applications at the timed workload, {dt:.2f} s each (numpy FP64); "
                      f"time-to-E2 at n_occ=10, n_vir=100, n_aux=300 (seed 1, PCG to 1e-8)",
            "time_to_e2_c2": {"cpu_s": round(t2, 3), "iterations": r2["iters"], "e2": r2["e2"],
                              "gpu_ms": round(gpu_c2_ms, 3), "gpu_speedup": round(t2 * 1e3 / gpu_c2_ms, 1)}}


if __name__ == "__main__":
    main()
