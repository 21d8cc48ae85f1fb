"""Benchmark of the MI355X IRN-PICCS hot path.

One step = one full IRN-PICCS reconstruction (weights, augmented LSQR with the
projector pair, stencils, device-side recurrences) of the 256^3 / 90-view /
512x512-detector workload: 5 reweightings x 10 LSQR iterations, float32, warm-
started from the prior.  Inputs are seeded synthetic phantoms resident in HBM
before the timed region.

Printed: ONE JSON line.  ``value`` is the whole-job voxel-projection rate of
the reconstruction: (A and A^T applications in a step) x nx*ny*nz*n_views /
step time.  Extra fields report the isolated A and A^T rates, the roofline of
the dominant projector kernel (timed with HIP events on the stream it runs
on) and the FP64 CPU oracle timed on this host on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--workload c2]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2"])
    ap.add_argument("--prior", default="720", choices=["720", "truth"],
                    help="prior image: 720-view plain-LSQR reconstruction, or the true base object")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--fp32-only", action="store_true", help="skip the mixed-precision forms")
    ap.add_argument("--op-reps", type=int, default=10)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (profiler calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU view sharding is a design note only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2509_08574_amd import cbct, synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    wl = args.workload
    gd = synth.geometry(wl)
    sp = synth.SOLVE_PARAMS[wl]
    g = cbct.Geometry.from_dict(gd)
    M, N = g.sizes()
    V = gd["n_views"]

    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---------------- inputs (not timed)
    t0 = time.time()
    if wl == "c2":
        base, cur = synth.c2_case(sp["seed"])
    else:
        base, cur = synth.c1_case(sp["seed"])
    log(f"[bench] phantom {gd['nx']}x{gd['ny']}x{gd['nz']} in {time.time() - t0:.1f}s")
    cur_d = torch.from_numpy(cur.astype(np.float32)).to(dev)
    base_d = torch.from_numpy(base.astype(np.float32)).to(dev)
    if wl == "c2" and args.prior == "720":
        # prior: plain LSQR (alpha = lambda = 0), 30 iterations, noise-free 720-view scan
        gp = cbct.Geometry.from_dict(synth.geometry("c2_prior"))
        bp = cbct.forward(gp, base_d)
        xprior = torch.zeros_like(base_d)
        t0 = time.time()
        cbct.solve(gp, bp, xprior, xprior, cbct.SolveParams(0.0, 0.0, sp["tau"], 1, 30),
                   report=False)
        torch.cuda.synchronize()
        log(f"[bench] 720-view prior reconstruction in {time.time() - t0:.1f}s")
        del bp
        gp.close()
    else:
        xprior = base_d.clone()
    y = cbct.forward(g, cur_d)
    b = synth.noisy_line_integrals(y.cpu().numpy(), sp["I0"], seed=sp["seed"] + 100)
    b_d = torch.from_numpy(b.astype(np.float32)).to(dev)
    p = cbct.SolveParams(sp["alpha"], sp["lam"], sp["tau"], sp["n_outer"], sp["n_inner"])
    ws = cbct.alloc_workspace(g, p, device=dev)
    x = torch.empty_like(xprior)
    products = p.n_outer * (p.n_inner + 1)
    vox_proj_step = 2.0 * products * M * V

    # ---------------- timed steps
    for _ in range(args.warmup):
        x.copy_(xprior)
        cbct.solve(g, b_d, xprior, x, p, workspace=ws, report=False)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} done")
    step_ms = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        x.copy_(xprior)
        cbct.solve(g, b_d, xprior, x, p, workspace=ws, report=False)
        torch.cuda.synchronize()
        step_ms.append(1e3 * (time.perf_counter() - ts))
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    ms_per_step = 1e3 * total / args.steps
    value = vox_proj_step * args.steps / total / 1e9
    err_truth = float(torch.linalg.norm(x - cur_d) / torch.linalg.norm(cur_d))
    err_prior = float(torch.linalg.norm(xprior - cur_d) / torch.linalg.norm(cur_d))
    log(f"[bench] {args.steps} steps: {ms_per_step:.1f} ms/recon; rel err vs truth "
        f"{err_truth:.4f} (prior {err_prior:.4f})")

    # ---------------- precision forms: s/recon at this workload
    forms = {}
    if not args.fp32_only:
        for name, pr in (("mixed_bf16", cbct.PREC_MIXED_BF16), ("mixed_f16", cbct.PREC_MIXED_F16)):
            pm = cbct.SolveParams(sp["alpha"], sp["lam"], sp["tau"], sp["n_outer"],
                                  sp["n_inner"], precision=pr)
            wsm = cbct.alloc_workspace(g, pm, device=dev)
            xm = torch.empty_like(xprior)
            xm.copy_(xprior)
            cbct.solve(g, b_d, xprior, xm, pm, workspace=wsm, report=False)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(args.steps):
                xm.copy_(xprior)
                cbct.solve(g, b_d, xprior, xm, pm, workspace=wsm, report=False)
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t) / args.steps
            forms[name] = {"s_per_recon": round(sec, 4),
                           "speedup_vs_fp32": round(ms_per_step / 1e3 / sec, 3),
                           "rel_l2_vs_fp32_gpu": float(torch.linalg.norm(xm - x)
                                                       / torch.linalg.norm(x))}
            del wsm
            log(f"[bench] {name}: {sec * 1e3:.1f} ms/recon")
    forms["fp32"] = {"s_per_recon": round(ms_per_step / 1e3, 4), "speedup_vs_fp32": 1.0}

    # ---------------- isolated projector kernels (HIP events on this stream)
    vf, voff, pf = cbct.col_sizes(g)
    xc = cbct.vol_to_cols(g, cur_d)
    yc = torch.empty(pf, dtype=torch.float32, device=dev)
    ywc = cbct.proj_to_cols(g, b_d, weighted=True)
    xo = torch.empty(vf, dtype=torch.float32, device=dev)

    def time_op(fn, reps):
        fn()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(reps):
            fn()
        ev1.record(stream)
        ev1.synchronize()
        return ev0.elapsed_time(ev1) / reps

    t_fwd = time_op(lambda: cbct.forward_cols(g, xc, yc), args.op_reps)
    t_back = time_op(lambda: cbct.back_cols(g, ywc, xo), args.op_reps)
    nnz = g.nnz()
    bytes_fwd = 4.0 * nnz + 4.0 * N
    bytes_back = 4.0 * nnz + 4.0 * M
    gvp_fwd = M * V / (t_fwd * 1e-3) / 1e9
    gvp_back = M * V / (t_back * 1e-3) / 1e9
    dom = ("k_back", t_back, bytes_back) if t_back >= t_fwd else ("k_fwd", t_fwd, bytes_fwd)
    achieved = dom[2] / (dom[1] * 1e-3) / 1e9
    log(f"[bench] A {t_fwd:.3f} ms ({gvp_fwd:.1f} Gvp/s), A^T {t_back:.3f} ms "
        f"({gvp_back:.1f} Gvp/s), nnz {nnz}")
    roofline = {"bound": "hbm", "kernel": dom[0], "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None, "avg_launch_ms": round(dom[1], 4),
                "algorithmic_bytes_per_launch": dom[2], "units_per_launch": nnz,
                "unit_bytes": "4 B per chord + 4 B per output element"}

    # ---------------- CPU oracle baseline (bounded sample)
    cpu = None
    if not args.no_cpu:
        from oracle import oracle as orc
        nthreads = orc.num_threads()
        # the oracle's own full A and A^T on the first `nvs` views of the same scan
        nvs = max(1, min(V, 12 if wl == "c2" else V))
        ang = 2.0 * np.pi * np.arange(V) / V
        og = orc.Geometry.from_dict(dict(gd, n_views=nvs, angles=ang[:nvs]))
        xr = cur.astype(np.float64)
        yr = b.astype(np.float64).reshape(V, gd["nv"], gd["nu"])[:nvs]
        t = time.perf_counter()
        orc.forward(og, xr)
        t_A = (time.perf_counter() - t) * V / nvs
        t = time.perf_counter()
        orc.back(og, yr)
        t_AT = (time.perf_counter() - t) * V / nvs
        cpu_rate = 2.0 * M * V / (t_A + t_AT) / 1e9
        cpu = {"value": round(cpu_rate, 4), "unit": "Gvoxel-proj/s", "cores": nthreads,
               "kind": "oracle",
               "sample": f"full FP64 A and A^T of {nvs} of the {V} views of {wl}, "
                         f"{nthreads} host threads, scaled to all views",
               "A_s": round(t_A, 2), "AT_s": round(t_AT, 2),
               "s_per_recon_extrapolated": round(products * (t_A + t_AT), 1)}
        log(f"[bench] oracle: A {t_A:.1f}s, A^T {t_AT:.1f}s per full application")

        # every precision form against the FP64 oracle on the full 64^3 / 48-view
        # solve (3 x 5 iterations), which the oracle finishes in seconds
        gd1 = synth.geometry("c1")
        sp1 = synth.SOLVE_PARAMS["c1"]
        og1 = orc.Geometry.from_dict(gd1)
        prior1, cur1 = synth.c1_case()
        b1 = synth.noisy_line_integrals(orc.forward(og1, cur1), sp1["I0"], seed=101)
        b1 = b1.astype(np.float32).astype(np.float64)
        prior1 = prior1.astype(np.float32).astype(np.float64)
        t = time.perf_counter()
        ref1 = orc.irn_piccs(og1, b1, prior1, prior1, sp1["alpha"], sp1["lam"], sp1["tau"],
                             sp1["n_outer"], sp1["n_inner"])
        t_or1 = time.perf_counter() - t
        g1 = cbct.Geometry.from_dict(gd1)
        for name, pr in (("fp32", cbct.PREC_FP32), ("mixed_bf16", cbct.PREC_MIXED_BF16),
                         ("mixed_f16", cbct.PREC_MIXED_F16)):
            if name not in forms:
                continue
            x1 = torch.from_numpy(prior1.astype(np.float32)).to(dev)
            cbct.solve(g1, torch.from_numpy(b1.astype(np.float32)).to(dev), x1.clone(), x1,
                       cbct.SolveParams(sp1["alpha"], sp1["lam"], sp1["tau"], sp1["n_outer"],
                                        sp1["n_inner"], precision=pr), report=False)
            xg1 = x1.cpu().numpy().astype(np.float64)
            forms[name]["rel_l2_vs_fp64_oracle_c1"] = float(
                np.linalg.norm(xg1 - ref1.x) / np.linalg.norm(ref1.x))
        cpu["oracle_c1_solve_s"] = round(t_or1, 2)

    out = {
        "metric": "Gvoxel-proj/s for A and A^T; s/recon + p99 latency, FP32 vs mixed",
        "value": round(value, 3),
        "unit": "Gvoxel-proj/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{wl}: {gd['nx']}x{gd['ny']}x{gd['nz']} volume, {V} views, "
                        f"{gd['nu']}x{gd['nv']} detector, IRN-PICCS {p.n_outer}x{p.n_inner} "
                        f"LSQR, fp32 storage, fp64 scalars",
            "voxel_proj_per_step": vox_proj_step,
            "products_per_step": products,
            "s_per_recon": round(ms_per_step / 1e3, 4),
            "step_ms_p50": round(float(np.percentile(step_ms, 50)), 3),
            "step_ms_max": round(float(max(step_ms)), 3),
            "A_ms": round(t_fwd, 4), "AT_ms": round(t_back, 4),
            "A_gvoxel_proj_s": round(gvp_fwd, 2), "AT_gvoxel_proj_s": round(gvp_back, 2),
            "nnz": nnz,
            "rel_err_vs_truth": round(err_truth, 5),
            "rel_err_prior_vs_truth": round(err_prior, 5),
            "prior": args.prior,
        },
        "precision_forms": forms,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
