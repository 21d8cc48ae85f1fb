"""Benchmark of the MI355X IRN-PICCS hot path.

One step = one full IRN-PICCS reconstruction (weights, augmented LSQR with the
projector pair, stencils, device-side FP64 recurrences) of one scan of the
repeated-scan sequence: a 512 x 512 x 400 volume at 0.4 mm, 180 views on a
1024 x 1024 detector at 0.3 mm, 4 reweightings x 10 LSQR iterations.  Ten
successive scans carry a needle advancing 3 mm per scan; each scan starts from
the previous reconstruction, which stays on the device (scans cycle 1..10).
Float32 storage and projector arithmetic, float64 Krylov scalars.  The same
sequence is then run in the mixed BF16 form.  Inputs are seeded synthetic
phantoms and noisy projections resident in HBM before the timed region.

Printed: ONE JSON line.  ``value`` is the whole-job voxel-projection rate of
the reconstruction: (A and A^T applications in a step) x nx*ny*nz*n_views /
step time.  Extra fields: the 256^3 / 90-view case in all three precision
forms, each form's error against the FP64 oracle (on reduced problems the
oracle finishes in seconds, labelled as such), the isolated A and A^T rates,
the roofline of the dominant projector kernel (timed with HIP events on the
stream it runs on), the serving stream, and the FP64 CPU oracle timed on this
host on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps 3] [--warmup 1]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue capacity: 256 CUs x 4 SIMDs, one issue cycle each per clock at 2.4 GHz.
# A wave64 instruction occupies its SIMD for 2 cycles (full-rate float32 add / mul
# / fma, 32-bit integer add, bitwise ops), 4 cycles (min / max / med3, conversions,
# 24-bit multiplies, VOP3 selects and shifts) or 8 cycles (reciprocal), as the
# issue-rate probe measures on the device.
SIMD_ISSUE_PEAK_CYCLES_S = 256 * 4 * 2.4e9
# Vector-memory data path: one texture-data (TD) unit per CU, busy at most every
# cycle; a probe of plain loads from L2 keeps it busy about all of the time.
TD_PEAK_BUSY_CYCLES_S = 256 * 2.4e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


PROFILES = os.path.join(ROOT, "profiles")
# sources that define the projector kernels: a recorded figure is only used
# while these are byte-identical to what was profiled
KERNEL_SOURCES = ("paper_2509_08574_amd/csrc/proj.hip", "paper_2509_08574_amd/csrc/chord.h",
                  "paper_2509_08574_amd/csrc/internal.h")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_profile(kernel, workload, key):
    """A per-launch figure from the committed rocprofv3 summary of `kernel` on
    `workload` (profiles/<kernel>_<workload>.md, section "Recorded for
    bench.py"), or None if there is none or the kernel sources changed since it
    was taken."""
    path = os.path.join(PROFILES, f"{kernel}_{workload}.md")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.startswith("- `"):
                k, v = line[3:].split("`", 1)[0], line.split(":", 1)[1].strip().strip("`")
                rec[k] = v
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(rec[key])
    except (KeyError, ValueError):
        return None


def time_op(torch, stream, fn, reps):
    """Average duration (ms) of fn() over `reps` back-to-back launches, HIP
    events recorded on `stream` (the stream fn launches its kernel on)."""
    fn()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        fn()
    ev1.record(stream)
    ev1.synchronize()
    return ev0.elapsed_time(ev1) / reps


def projector_pair(args, cbct, torch, g, xc, ywc, stream, workload):
    """Event-timed isolated A and A^T (column layout, on `stream`), and the
    roofline object of the slower one (the dominant kernel of a solve)."""
    M, N = g.sizes()
    V = g.proj_shape[0]
    yc = torch.empty_like(ywc)
    xo = torch.empty_like(xc)
    t_fwd = time_op(torch, stream, lambda: cbct.forward_cols(g, xc, yc, stream=stream),
                    args.op_reps)
    t_back = time_op(torch, stream, lambda: cbct.back_cols(g, ywc, xo, stream=stream),
                     args.op_reps)
    nnz = g.nnz()
    gvp_fwd = M * V / (t_fwd * 1e-3) / 1e9
    gvp_back = M * V / (t_back * 1e-3) / 1e9
    log(f"[bench] {workload}: A {t_fwd:.3f} ms ({gvp_fwd:.1f} Gvp/s), A^T {t_back:.3f} ms "
        f"({gvp_back:.1f} Gvp/s), nnz {nnz}")
    out = {"A_ms": round(t_fwd, 4), "AT_ms": round(t_back, 4),
           "A_gvoxel_proj_s": round(gvp_fwd, 2), "AT_gvoxel_proj_s": round(gvp_back, 2),
           "nnz": nnz}
    dom = ("k_back", t_back, 4.0 * nnz + 4.0 * M) if t_back >= t_fwd else \
          ("k_fwd", t_fwd, 4.0 * nnz + 4.0 * N)
    return out, roofline(dom, nnz, workload)


def roofline(dom, nnz, workload):
    """Roofline of the dominant projector kernel.

    Both projectors are gathers whose operands come mostly from L2 and L1: their
    HBM traffic stays well below the HBM peak, and the operand-bytes rate (4 B
    per chord, `effective_GBps`) exceeds it.  Two on-chip resources bound them:
    VALU issue (`alu`: the issue cycles the kernel's instructions occupy on the
    main VALU pipe, over 1024 SIMDs x 2.4 GHz) and the vector-memory data path
    (`vmem`: busy cycles of the 256 texture-data units, over 256 x 2.4 GHz).
    Both per-launch figures come from the committed profile of the same
    sources and are divided by this run's event-timed launch; the one closer to
    its peak is reported as the bound."""
    kernel, t_ms, opbytes = dom
    t = t_ms * 1e-3
    cyc = recorded_profile(kernel, workload, "valu_issue_cycles_per_launch")
    td = recorded_profile(kernel, workload, "td_busy_cycles_per_launch")
    traffic = recorded_profile(kernel, workload, "traffic_bytes_per_launch")
    parts = {}
    if cyc:
        parts["alu"] = {"achieved": round(cyc / t / 1e9, 1),
                        "peak": round(SIMD_ISSUE_PEAK_CYCLES_S / 1e9, 1),
                        "unit": "G VALU issue cycles/s (main pipe, SIMD-cycles)",
                        "frac": round(cyc / t / SIMD_ISSUE_PEAK_CYCLES_S, 4)}
    if td:
        parts["vmem"] = {"achieved": round(td / t / 1e9, 1),
                         "peak": round(TD_PEAK_BUSY_CYCLES_S / 1e9, 1),
                         "unit": "G texture-data busy cycles/s (256 units)",
                         "frac": round(td / t / TD_PEAK_BUSY_CYCLES_S, 4)}
    if traffic:
        parts["hbm"] = {"achieved": round(traffic / t / 1e9, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s (measured FETCH_SIZE + WRITE_SIZE)",
                        "frac": round(traffic / t / 1e9 / HBM_PEAK_GBS, 4)}
    bound = max(("alu", "vmem"), key=lambda k: parts[k]["frac"] if k in parts else -1.0)
    main = parts.get(bound, {})
    r = {"bound": bound if main else None, "kernel": kernel, "achieved": main.get("achieved"),
         "peak": main.get("peak"), "unit": main.get("unit"), "frac": main.get("frac"),
         "traffic": traffic, "avg_launch_ms": round(t_ms, 4), "units_per_launch": nnz,
         "unit_name": "chord", "effective_GBps": round(opbytes / t / 1e9, 1),
         "profile": f"profiles/{kernel}_{workload}.md"}
    r.update(parts)
    l2 = recorded_profile(kernel, workload, "l2_hit_rate")
    if l2 is not None:
        r["l2_hit_rate"] = l2
    # A^T runs as one kernel dispatch per chunk of views: a "launch" here is one
    # application, the dispatches one call issues back to back on its stream
    nd = recorded_profile(kernel, workload, "dispatches_per_launch")
    if nd is not None:
        r["dispatches_per_launch"] = int(nd)
    return r


def stream_copy_gbps(torch, dev):
    """A plain device copy of 1 GiB (torch's copy kernel), timed with HIP events:
    the HBM rate a streaming kernel reaches in practice, beside the 8 TB/s of the
    data sheet."""
    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    return 2.0 * 4.0 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9


def noisy_b(torch, synth, y, I0, seed, dev):
    """Poisson counts at I0 exp(-mu p), clamped >= 1, back to line integrals
    (seeded, on the device)."""
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    lam = I0 * torch.exp(-synth.MU_WATER_PER_MM * y.double())
    counts = torch.clamp(torch.poisson(lam, generator=gen), min=1.0)
    return (-torch.log(counts / I0) / synth.MU_WATER_PER_MM).float()


def repeated_scans(args, cbct, synth, np, torch, dev, stream):
    """The headline workload: the ten-scan 512 x 512 x 400 sequence, FP32 then
    mixed BF16, each started from x_p at scan 1 and warm-started from the
    previous reconstruction at every later step."""
    gd = synth.geometry("c5")
    sp = synth.SOLVE_PARAMS["c5"]
    t = time.time()
    base, centre, axis = synth.c5_case(sp["seed"])
    log(f"[bench] phantom 512x512x400 in {time.time() - t:.1f}s")
    g = cbct.Geometry.from_dict(gd)
    M, N = g.sizes()
    V = gd["n_views"]
    xp = torch.from_numpy(base.astype(np.float32)).to(dev)
    needles, bs = [], []
    for s_ in range(1, 11):
        idx = torch.from_numpy(synth.c5_scan(base, centre, axis, s_)).to(dev)
        cur = xp.clone()
        cur.view(-1)[idx] = 2.0
        bs.append(noisy_b(torch, synth, cbct.forward(g, cur), sp["I0"], 500 + s_, dev))
        needles.append(idx)
        del cur
    torch.cuda.synchronize()
    log(f"[bench] 10 scans ready ({time.time() - t:.1f}s)")

    def truth(scan):
        cur = xp.clone()
        cur.view(-1)[needles[scan]] = 2.0
        return cur

    products = sp["n_outer"] * (sp["n_inner"] + 1)
    vox_proj_step = 2.0 * products * M * V
    forms, xs = {}, {}
    for name, pr in (("fp32", cbct.PREC_FP32), ("mixed_bf16", cbct.PREC_MIXED_BF16)):
        if name != "fp32" and args.fp32_only:
            continue
        p = cbct.SolveParams(sp["alpha"], sp["lam"], sp["tau"], sp["n_outer"], sp["n_inner"],
                             precision=pr)
        ws = cbct.alloc_workspace(g, p, device=dev)
        x = xp.clone()

        def step(i):
            cbct.solve(g, bs[i % 10], xp, x, p, workspace=ws, report=False)

        for i in range(args.warmup):
            step(i)
        torch.cuda.synchronize()
        step_ms = []
        t0 = time.perf_counter()
        for i in range(args.warmup, args.warmup + args.steps):
            ts = time.perf_counter()
            step(i)
            torch.cuda.synchronize()
            step_ms.append(1e3 * (time.perf_counter() - ts))
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        last = (args.warmup + args.steps - 1) % 10
        tr = truth(last)
        err = float(torch.linalg.norm(x - tr) / torch.linalg.norm(tr))
        err_prior = float(torch.linalg.norm(xp - tr) / torch.linalg.norm(tr))
        # the change against the prior is the needle: its recovery (1 = none of it,
        # 0 = exact) over the needle's voxels
        nd = needles[last]
        chg = float(torch.linalg.norm(x.view(-1)[nd] - tr.view(-1)[nd])
                    / torch.linalg.norm(tr.view(-1)[nd] - xp.view(-1)[nd]))
        forms[name] = {"s_per_recon": round(total / args.steps, 4),
                       "step_ms_p50": round(float(np.percentile(step_ms, 50)), 2),
                       "step_ms_max": round(float(max(step_ms)), 2),
                       "value_gvoxel_proj_s": round(vox_proj_step * args.steps / total / 1e9, 3),
                       "last_scan": last + 1, "rel_err_vs_truth": round(err, 5),
                       "rel_err_prior_vs_truth": round(err_prior, 5),
                       "improves_on_prior": err < err_prior,
                       "needle_change_err": round(chg, 4)}
        # later scans of the same chain with b arriving in page-locked host memory
        # and x returned there: H2D of b, the solve, D2H of x; median of three
        b_host = torch.empty(bs[0].shape, dtype=torch.float32, pin_memory=True)
        x_host = torch.empty(x.shape, dtype=torch.float32, pin_memory=True)
        b_dev = torch.empty_like(bs[0])
        with_copies = []
        for r in range(3):
            b_host.copy_(bs[(args.warmup + args.steps + r) % 10])
            torch.cuda.synchronize()
            ts = time.perf_counter()
            b_dev.copy_(b_host, non_blocking=True)
            cbct.solve(g, b_dev, xp, x, p, workspace=ws, report=False)
            x_host.copy_(x, non_blocking=True)
            torch.cuda.synchronize()
            with_copies.append(time.perf_counter() - ts)
        forms[name]["s_per_recon_with_copies"] = round(float(np.median(with_copies)), 4)
        del b_host, x_host, b_dev
        xs[name] = x
        log(f"[bench] 512x512x400 {name}: {args.steps} steps, {1e3 * total / args.steps:.1f} "
            f"ms/recon; scan {last + 1}: rel err vs truth {err:.4f} (prior {err_prior:.4f}), "
            f"needle change error {chg:.3f}")
        del ws, tr
    if "mixed_bf16" in forms:
        f32, bf = forms["fp32"], forms["mixed_bf16"]
        bf["speedup_vs_fp32"] = round(f32["s_per_recon"] / bf["s_per_recon"], 3)
        bf["rel_l2_vs_fp32_gpu"] = float(torch.linalg.norm(xs["mixed_bf16"] - xs["fp32"])
                                         / torch.linalg.norm(xs["fp32"]))
    forms["fp32"]["speedup_vs_fp32"] = 1.0
    del xs
    # isolated projectors on this workload (column layout, HIP events on this stream)
    xc = cbct.vol_to_cols(g, truth(0))
    ywc = cbct.proj_to_cols(g, bs[0], weighted=True)
    ops, roof = projector_pair(args, cbct, torch, g, xc, ywc, stream, "c5")
    del xc, ywc, bs
    g.close()
    return dict(gd=gd, sp=sp, M=M, V=V, products=products, vox_proj_step=vox_proj_step,
                forms=forms, ops=ops, roofline=roof, base=base, centre=centre, axis=axis)


def c2_case_forms(args, cbct, synth, np, torch, dev, stream):
    """The 256^3 / 90-view / 512^2 workload (5 x 10, prior from a 720-view plain
    LSQR reconstruction): FP32 and both mixed forms, FDK, isolated projectors."""
    gd = synth.geometry("c2")
    sp = synth.SOLVE_PARAMS["c2"]
    g = cbct.Geometry.from_dict(gd)
    M, N = g.sizes()
    V = gd["n_views"]
    base, cur = synth.c2_case(sp["seed"])
    cur_d = torch.from_numpy(cur.astype(np.float32)).to(dev)
    base_d = torch.from_numpy(base.astype(np.float32)).to(dev)
    gp = cbct.Geometry.from_dict(synth.geometry("c2_prior"))
    bp = cbct.forward(gp, base_d)
    xprior = torch.zeros_like(base_d)
    cbct.solve(gp, bp, xprior, xprior, cbct.SolveParams(0.0, 0.0, sp["tau"], 1, 30), report=False)
    del bp
    gp.close()
    y = cbct.forward(g, cur_d)
    b = synth.noisy_line_integrals(y.cpu().numpy(), sp["I0"], seed=sp["seed"] + 100)
    b_d = torch.from_numpy(b.astype(np.float32)).to(dev)
    products = sp["n_outer"] * (sp["n_inner"] + 1)
    err_prior = float(torch.linalg.norm(xprior - cur_d) / torch.linalg.norm(cur_d))
    # the change against the object the prior was made from: the grown lesion
    changed = cur_d != base_d
    d_changed = (cur_d - xprior)[changed]
    out, ref = {}, None
    for name, pr in (("fp32", cbct.PREC_FP32), ("mixed_bf16", cbct.PREC_MIXED_BF16),
                     ("mixed_f16", cbct.PREC_MIXED_F16)):
        p = cbct.SolveParams(sp["alpha"], sp["lam"], sp["tau"], sp["n_outer"], sp["n_inner"],
                             precision=pr)
        ws = cbct.alloc_workspace(g, p, device=dev)
        x = xprior.clone()
        cbct.solve(g, b_d, xprior, x, p, workspace=ws, report=False)
        torch.cuda.synchronize()
        reps = max(1, args.c2_steps)
        t = time.perf_counter()
        for _ in range(reps):
            x.copy_(xprior)
            cbct.solve(g, b_d, xprior, x, p, workspace=ws, report=False)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t) / reps
        if ref is None:
            ref = x.clone()
        err = float(torch.linalg.norm(x - cur_d) / torch.linalg.norm(cur_d))
        out[name] = {"s_per_recon": round(sec, 4),
                     "gvoxel_proj_s": round(2.0 * products * M * V / sec / 1e9, 2),
                     "rel_err_vs_truth": round(err, 5),
                     "improves_on_prior": err < err_prior,
                     "lesion_change_err": round(float(torch.linalg.norm((x - cur_d)[changed])
                                                      / torch.linalg.norm(d_changed)), 4),
                     "rel_l2_vs_fp32_gpu": float(torch.linalg.norm(x - ref)
                                                 / torch.linalg.norm(ref))}
        del ws
        log(f"[bench] 256^3 {name}: {sec * 1e3:.1f} ms/recon")
    for k in out:
        out[k]["speedup_vs_fp32"] = round(out["fp32"]["s_per_recon"] / out[k]["s_per_recon"], 3)
    out["rel_err_prior_vs_truth"] = round(err_prior, 5)
    # FDK of the same scan (direct method, no prior)
    xf = cbct.fdk(g, b_d, stream=stream)
    out["fdk_ms"] = round(time_op(torch, stream, lambda: cbct.fdk(g, b_d, xf, stream=stream),
                                  args.op_reps), 3)
    out["rel_err_fdk_vs_truth"] = round(float(torch.linalg.norm(xf - cur_d)
                                              / torch.linalg.norm(cur_d)), 5)
    del xf
    xc = cbct.vol_to_cols(g, cur_d)
    ywc = cbct.proj_to_cols(g, b_d, weighted=True)
    ops, roof = projector_pair(args, cbct, torch, g, xc, ywc, stream, "c2")
    out.update(ops)
    out["roofline"] = roof
    out["workload"] = ("256x256x256 volume at 1 mm, 90 views, 512x512 detector at 0.8 mm, "
                       "IRN-PICCS 5x10, prior from a 720-view plain LSQR reconstruction")
    g.close()
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline_and_oracle_errors(args, cbct, synth, np, torch, dev, c5):
    """The FP64 oracle on this host: (1) its A and A^T on a bounded sample of the
    headline workload (4 of the 180 views, all host threads) and on one view of
    the 256^3 workload with one thread (per-core rate); (2) every precision form
    against the oracle's IRN-PICCS on reduced problems it finishes in seconds to
    a minute: the full 64^3 / 48-view solve (3 x 5), and the headline volume and
    detector with 4 of its 180 views (1 x 2)."""
    from oracle import oracle as orc
    nthreads = orc.num_threads()
    gd, sp = c5["gd"], c5["sp"]
    V = gd["n_views"]
    nvs = 4
    ang = 2.0 * np.pi * np.arange(V) / V
    sub = dict(gd, n_views=nvs, angles=list(ang[::V // nvs][:nvs]))
    og = orc.Geometry.from_dict(sub)
    cur = c5["base"].copy()
    cur.reshape(-1)[synth.c5_scan(c5["base"], c5["centre"], c5["axis"], 1)] = 2.0
    t = time.perf_counter()
    y_or = orc.forward(og, cur)
    t_A = (time.perf_counter() - t) * V / nvs
    t = time.perf_counter()
    orc.back(og, y_or)
    t_AT = (time.perf_counter() - t) * V / nvs
    M = c5["M"]
    rate = 2.0 * M * V / (t_A + t_AT) / 1e9
    log(f"[bench] oracle, {nthreads} threads: A {t_A:.1f}s, A^T {t_AT:.1f}s per full "
        f"512x512x400 / 180-view application (from {nvs} views)")
    errs = {}
    # (a) the full 64^3 / 48-view solve
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
    t_or1 = round(time.perf_counter() - t, 2)
    # (b) the headline volume and detector, 4 views, 1 x 2
    b5 = synth.noisy_line_integrals(y_or, sp["I0"], seed=sp["seed"] + 300)
    b5 = b5.astype(np.float32).astype(np.float64)
    prior5 = c5["base"].astype(np.float32).astype(np.float64)
    t = time.perf_counter()
    n_ops = [0]

    def progress(fn):
        def op(v):
            n_ops[0] += 1
            log(f"[bench] oracle 512x512x400 / 4 views: product {n_ops[0]} "
                f"({time.perf_counter() - t:.0f}s)")
            return fn(og, v)
        return op
    ref5 = orc.irn_piccs(og, b5, prior5, prior5, sp["alpha"], sp["lam"], sp["tau"], 1, 2,
                         A=progress(orc.forward), AT=progress(orc.back))
    t_or5 = round(time.perf_counter() - t, 2)
    log(f"[bench] oracle IRN-PICCS: 64^3 3x5 in {t_or1}s, 512x512x400 4 views 1x2 in {t_or5}s")
    cases = (("c1_64cubed_48views_3x5", gd1, b1, prior1, sp1, sp1["n_outer"], sp1["n_inner"],
              ref1),
             ("c5_geometry_4views_1x2", sub, b5, prior5, sp, 1, 2, ref5))
    for label, gdx, bx, px, spx, no, ni, ref in cases:
        gx = cbct.Geometry.from_dict(gdx)
        bd = torch.from_numpy(bx.astype(np.float32)).to(dev)
        pd = torch.from_numpy(px.astype(np.float32)).to(dev)
        for name, pr in (("fp32", cbct.PREC_FP32), ("mixed_bf16", cbct.PREC_MIXED_BF16),
                         ("mixed_f16", cbct.PREC_MIXED_F16)):
            x = pd.clone()
            cbct.solve(gx, bd, pd, x, cbct.SolveParams(spx["alpha"], spx["lam"], spx["tau"], no,
                                                     ni, precision=pr), report=False)
            xg = x.cpu().numpy().astype(np.float64)
            errs.setdefault(name, {})[label] = float(np.linalg.norm(xg - ref.x)
                                                     / np.linalg.norm(ref.x))
        gx.close()
        del bd, pd
    cpu_extra = {"oracle_c1_solve_s": t_or1, "oracle_c5_4views_1x2_solve_s": t_or5}
    # one thread, one view of the 256^3 workload
    g2 = synth.geometry("c2")
    og1 = orc.Geometry.from_dict(dict(g2, n_views=1, angles=[0.0]))
    x2 = np.random.default_rng(9).uniform(size=og1.vol_shape)
    t = time.perf_counter()
    y1 = orc.forward(og1, x2, nthreads=1)
    t1_A = time.perf_counter() - t
    t = time.perf_counter()
    orc.back(og1, y1, nthreads=1)
    t1_AT = time.perf_counter() - t
    # the oracle keeps the thread count it was last given: restore all threads
    orc.back(orc.Geometry.from_dict(dict(g2, nx=4, ny=4, nz=4, n_views=1, angles=[0.0])),
             np.zeros((1, g2["nv"], g2["nu"])), nthreads=nthreads)
    m2 = g2["nx"] * g2["ny"] * g2["nz"]
    per_core = 2.0 * m2 / (t1_A + t1_AT) / 1e9
    log(f"[bench] oracle, 1 thread, one 256^3 view: A {t1_A:.2f}s, A^T {t1_AT:.2f}s")
    cpu = {"value": round(rate, 4), "unit": "Gvoxel-proj/s", "cores": nthreads, "kind": "oracle",
           "sample": f"FP64 A and A^T of {nvs} of the 180 views of the 512x512x400 / 1024^2 "
                     f"workload, {nthreads} host threads, scaled to all views",
           "A_s": round(t_A, 2), "AT_s": round(t_AT, 2),
           "s_per_recon_extrapolated": round(c5["products"] * (t_A + t_AT), 1),
           "per_core": {"value": round(per_core, 5), "unit": "Gvoxel-proj/s",
                        "sample": "FP64 A and A^T of one view of the 256^3 / 512^2 workload, "
                                  "one thread", "A_s": round(t1_A, 3), "AT_s": round(t1_AT, 3)},
           "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}

    cpu.update(cpu_extra)
    return cpu, errs


def cpu_baseline_c2_solve(args, cbct, synth, np, torch, dev):
    """The cpu_baseline leg at full size (--oracle-c2-solve): the 256^3 / 90-view /
    512^2 workload solved on both sides, the FP64 oracle's IRN-PICCS
    (args.oracle_c2_outer outer steps of 10 LSQR iterations, all host threads)
    timed on this host, and each GPU precision form's final x and phi-bar
    history compared with the oracle's.  Both sides get the same
    inputs, made by the oracle and the seeded generator only: b is the oracle's
    projection of the current object with Poisson noise, and the prior is the
    object without the change.  Four outer steps (44 products) fit one 20-minute
    session on 16 host threads; the time per product gives the 5 x 10 figure."""
    from oracle import oracle as orc
    gd = synth.geometry("c2")
    sp = synth.SOLVE_PARAMS["c2"]
    n_outer, n_inner = args.oracle_c2_outer, sp["n_inner"]
    base, cur = synth.c2_case(sp["seed"])
    og = orc.Geometry.from_dict(gd)
    nthreads = orc.num_threads()
    t = time.perf_counter()
    y = orc.forward(og, cur)
    log(f"[oracle-c2] oracle projection of the current object: {time.perf_counter() - t:.0f}s")
    b = synth.noisy_line_integrals(y, sp["I0"], seed=sp["seed"] + 100)
    b = b.astype(np.float32).astype(np.float64)
    prior = base.astype(np.float32).astype(np.float64)
    del y
    products = n_outer * (n_inner + 1)
    out = {"workload": f"256x256x256 volume at 1 mm, 90 views, 512x512 detector at 0.8 mm, "
                       f"IRN-PICCS {n_outer}x{n_inner} ({products} products), prior = the "
                       f"object without the change"}
    g = cbct.Geometry.from_dict(gd)
    b_d = torch.from_numpy(b.astype(np.float32)).to(dev)
    p_d = torch.from_numpy(prior.astype(np.float32)).to(dev)
    xs = {}
    for name, pr in (("fp32", cbct.PREC_FP32), ("mixed_bf16", cbct.PREC_MIXED_BF16),
                     ("mixed_f16", cbct.PREC_MIXED_F16)):
        x = p_d.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, rep = cbct.solve(g, b_d, p_d, x, cbct.SolveParams(
            sp["alpha"], sp["lam"], sp["tau"], n_outer, n_inner, precision=pr))
        xs[name] = (x.cpu().numpy().astype(np.float64), rep["phibar"],
                    time.perf_counter() - t)
        log(f"[oracle-c2] GPU {name}: {xs[name][2]:.3f}s")
    g.close()
    del b_d, p_d
    n_ops = [0]
    t0 = time.perf_counter()

    def progress(fn, what):
        def op(v):
            n_ops[0] += 1
            log(f"[oracle-c2] {what} {n_ops[0]} of {2 * products} "
                f"({time.perf_counter() - t0:.0f}s)")
            return fn(og, v)
        return op
    ref = orc.irn_piccs(og, b, prior, prior, sp["alpha"], sp["lam"], sp["tau"], n_outer,
                        n_inner, A=progress(orc.forward, "A"), AT=progress(orc.back, "A^T"))
    t_or = time.perf_counter() - t0
    log(f"[oracle-c2] FP64 IRN-PICCS {n_outer}x{n_inner} at 256^3: {t_or:.0f}s on "
        f"{nthreads} threads")
    out["oracle"] = {"s_per_recon": round(t_or, 1), "threads": nthreads,
                     "cpu_model": cpu_model(), "products": n_ops[0] // 2,
                     "s_per_product": round(t_or / max(1, n_ops[0] // 2), 2)}
    for name, (xg, ph, sec) in xs.items():
        err = float(np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x))
        ph_err = float(np.max(np.abs(np.asarray(ph) - np.asarray(ref.phibar))
                              / np.abs(np.asarray(ref.phibar))))
        out[name] = {"rel_l2_vs_fp64_oracle": err, "phibar_max_rel_err": ph_err,
                     "gpu_s_with_report": round(sec, 4),
                     "oracle_over_gpu": round(t_or / sec, 1)}
        log(f"[oracle-c2] {name}: rel L2 vs FP64 oracle {err:.3e}, phi-bar {ph_err:.3e}")
    out["moved_from_prior"] = float(np.linalg.norm(ref.x - prior) / np.linalg.norm(ref.x))
    return out


def serving_bench(args, cbct, synth, np, torch, dev):
    """Serving stream: 8 patients with resident priors (volumes 128/256/384^3,
    detector 2n x 2n, 30..120 views per request, needle moved 2..5 voxels),
    IRN-PICCS 3x10 in mixed BF16.  Returns a dict for the JSON line.

    Requests come from a seeded pool of distinct scans (projections made on the
    device before timing).  Three passes: each pool request alone (service
    time), the whole pool submitted at once (closed-loop capacity), then a
    Poisson stream at rate rho x capacity.  Latency runs from the scheduled
    arrival to the moment the result is ready to poll.
    """
    sp = synth.SERVING_PARAMS
    params = cbct.SolveParams(sp["alpha"], sp["lam"], sp["tau"], sp["n_outer"], sp["n_inner"],
                              precision=cbct.PREC_MIXED_BF16)
    t_setup = time.time()
    n_pat = 8
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(8) as ex:
        pats = list(ex.map(synth.serving_patient, range(n_pat)))
    log(f"[serve] {n_pat} patients, sizes {[n for n, _, _ in pats]} "
        f"({time.time() - t_setup:.1f}s)")
    srv = cbct.Server(hbm_budget_bytes=args.serve_budget_gib << 30, max_slots=args.serve_slots)
    base_d = {}
    for i, (n, prior, state) in enumerate(pats):
        srv.add_prior(i, synth.serving_geometry(n, 30), prior.astype(np.float32))
        base_d[i] = torch.from_numpy(state[0].astype(np.float32)).to(dev)

    # request pool: (patient, geometry, b)
    gen = torch.Generator(device=dev)
    pool = []
    for i in range(args.serve_pool):
        pid, nv, shift = synth.serving_request_draw(i, n_pat)
        n, _, state = pats[pid]
        gdict = synth.serving_geometry(n, nv)
        gq = cbct.Geometry.from_dict(gdict)
        cur = base_d[pid].clone()
        cur.view(-1)[torch.from_numpy(synth.serving_needle(state, shift)).to(dev)] = 2.0
        y = cbct.forward(gq, cur)
        gen.manual_seed(4000 + i)
        lam = sp["I0"] * torch.exp(-synth.MU_WATER_PER_MM * y.double())
        counts = torch.clamp(torch.poisson(lam, generator=gen), min=1.0)
        b = (-torch.log(counts / sp["I0"]) / synth.MU_WATER_PER_MM).float().cpu().numpy()
        pool.append((pid, gdict, b))
        gq.close()
        del cur, y, lam, counts
    torch.cuda.synchronize()
    del base_d
    log(f"[serve] pool of {len(pool)} requests ready ({time.time() - t_setup:.1f}s)")
    outs = {i: np.empty((n, n, n), np.float32) for i, (n, _, _) in enumerate(pats)}

    def run_one(k):
        pid, gdict, b = pool[k]
        t = srv.submit(pid, gdict, b, params)
        rc, _, info = srv.wait(t, outs[pid], timeout=600)
        assert rc == 0, info["error"]
        return info

    # pass 1: alone (also warms geometry tables and pinned buffers)
    alone = [run_one(k) for k in range(len(pool))]
    service = [a["t_done"] - a["t_submit"] for a in alone]
    by_size = {}
    for (pid, _, _), s_ in zip(pool, service):
        by_size.setdefault(pats[pid][0], []).append(s_)
    log(f"[serve] alone: mean service {np.mean(service) * 1e3:.1f} ms; "
        + ", ".join(f"{n}^3 {np.mean(v) * 1e3:.0f} ms" for n, v in sorted(by_size.items())))

    # pass 2: closed loop, the whole pool at once
    t = time.perf_counter()
    tickets = [srv.submit(pid, g_, b, params) for pid, g_, b in pool]
    for tk, (pid, _, _) in zip(tickets, pool):
        rc, _, info = srv.wait(tk, outs[pid], timeout=600)
        assert rc == 0, info["error"]
    t_closed = time.perf_counter() - t
    capacity = len(pool) / t_closed
    log(f"[serve] closed loop: {capacity:.2f} recon/s "
        f"(serial {len(pool) / sum(service):.2f} recon/s)")

    # pass 3: Poisson arrivals at rho x capacity
    results = {}
    for rho in args.serve_rho:
        rate = rho * capacity
        rng = np.random.default_rng(499)
        n_req = args.serve_requests + args.serve_warmup
        gaps = rng.exponential(1.0 / rate, size=n_req)
        picks = rng.integers(len(pool), size=n_req)
        arrivals = np.cumsum(gaps)
        lat, pending = [], {}
        st0 = srv.stats()
        t0 = time.perf_counter()
        nxt = 0
        while nxt < n_req or pending:
            now = time.perf_counter() - t0
            if nxt < n_req and now >= arrivals[nxt]:
                pid, g_, b = pool[picks[nxt]]
                t_sub = time.perf_counter() - t0
                tk = srv.submit(pid, g_, b, params)
                pending[tk] = (nxt, pid, arrivals[nxt], t_sub)
                nxt += 1
                continue
            for tk in list(pending):
                k, pid, arr, t_sub = pending[tk]
                r = srv.poll(tk, outs[pid])
                if r is None:
                    continue
                rc, _, info = r
                assert rc == 0, info["error"]
                del pending[tk]
                if k >= args.serve_warmup:
                    # late submission adds to the latency
                    lat.append(info["t_done"] - info["t_submit"] + (t_sub - arr))
                    if len(lat) % 100 == 0:
                        log(f"[serve] rho {rho}: {len(lat)} of {args.serve_requests} requests "
                            f"done ({time.perf_counter() - t0:.0f}s)")
            time.sleep(2e-4)
        wall = time.perf_counter() - t0
        st = srv.stats()
        lat = np.array(lat)
        results[f"rho_{rho}"] = {
            "offered_recon_per_s": round(rate, 3),
            "achieved_recon_per_s": round(n_req / wall, 3),
            "requests_measured": int(lat.size),
            "latency_p50_s": round(float(np.percentile(lat, 50)), 4),
            "latency_p99_s": round(float(np.percentile(lat, 99)), 4),
            "latency_mean_s": round(float(lat.mean()), 4),
            "peak_in_flight": st["peak_in_flight"],
            "failed": st["failed"] - st0["failed"],
        }
        log(f"[serve] rho {rho}: p50 {results[f'rho_{rho}']['latency_p50_s'] * 1e3:.0f} ms, "
            f"p99 {results[f'rho_{rho}']['latency_p99_s'] * 1e3:.0f} ms, "
            f"{n_req / wall:.2f} recon/s over {wall:.1f}s")
    st = srv.stats()
    srv.close()
    return {
        "workload": "8 patients (128/256/384^3, detector 2n x 2n), 30..120 views, "
                    "IRN-PICCS 3x10 mixed bf16, Poisson arrivals",
        "slots": args.serve_slots,
        "hbm_budget_gib": args.serve_budget_gib,
        "pool_requests": len(pool),
        "service_alone_mean_s": round(float(np.mean(service)), 4),
        "service_alone_by_size_s": {str(n): round(float(np.mean(v)), 4)
                                    for n, v in sorted(by_size.items())},
        "serial_recon_per_s": round(len(pool) / sum(service), 3),
        "closed_loop_recon_per_s": round(capacity, 3),
        "streams": results,
        "peak_used_gib": round(st["peak_used"] / 2 ** 30, 2),
        "geom_placements": st["geom_placements"],
        "geom_evictions": st["geom_evictions"],
    }


def quality_bench(args, cbct, synth, np, torch, dev):
    """Stand-ins for the paper's two experiments (Sec. 3): head with a cubic
    tumour (20 views, noise-free projections) and thorax with a needle (180 / 50 /
    20 views, Poisson noise at I0 = 5e4).  FDK, plain least squares (LSQR, 20
    iterations), IRN-TV, IRN-PIPLE and IRN-PICCS (alpha = lambda = 1, tau = 0.1;
    25 inner iterations per outer step, errors after 1..4 outer steps).  PSNR,
    SSIM and relative L2 error against the ground truth over the whole volume."""
    from paper_2509_08574_amd import metrics
    cases = [("head", synth.head_case, synth.head_geometry, [20], None)]
    if not args.quality_head_only:
        cases.append(("thorax", synth.thorax_case, synth.thorax_geometry, [180, 50, 20], 5e4))
    out = {}
    gen = torch.Generator(device=dev)
    for name, make, geom, views, I0 in cases:
        prior, truth = make()
        xp_d = torch.from_numpy(prior.astype(np.float32)).to(dev)
        tr_d = torch.from_numpy(truth.astype(np.float32)).to(dev)
        for V in views:
            gd = geom(V)
            g = cbct.Geometry.from_dict(gd)
            y = cbct.forward(g, tr_d)
            if I0:
                gen.manual_seed(1000 + V)
                lam = I0 * torch.exp(-synth.MU_WATER_PER_MM * y.double())
                counts = torch.clamp(torch.poisson(lam, generator=gen), min=1.0)
                y = (-torch.log(counts / I0) / synth.MU_WATER_PER_MM).float()
            rows = []

            def record(label, iters, x, sec):
                xh = x.detach().cpu().numpy().astype(np.float64)
                rows.append({"method": label, "iterations": iters, "time_s": round(sec, 4),
                             "psnr": round(metrics.psnr(xh, truth), 3),
                             "ssim": round(metrics.ssim(xh, truth), 4),
                             "rel_l2": round(metrics.rel_l2(xh, truth), 5),
                             "change_err": round(metrics.change_recovery(xh, truth, prior), 4)})
                log(f"[quality] {name} {V} views {label:10s} {iters:>14s}: PSNR "
                    f"{rows[-1]['psnr']:.2f} SSIM {rows[-1]['ssim']:.4f} "
                    f"rel {rows[-1]['rel_l2']:.4f} change {rows[-1]['change_err']:.3f} "
                    f"({sec * 1e3:.0f} ms)")

            def timed(fn):
                torch.cuda.synchronize()
                t = time.perf_counter()
                r = fn()
                torch.cuda.synchronize()
                return r, time.perf_counter() - t

            xf, sec = timed(lambda: cbct.fdk(g, y))
            record("FDK", "-", xf, sec)
            zero = torch.zeros_like(xp_d)

            def solve(x0, p):
                x = x0.clone()
                cbct.solve(g, y, xp_d, x, p, report=False)
                return x
            xl, sec = timed(lambda: solve(zero, cbct.SolveParams(0.0, 0.0, 0.1, 1, 20)))
            record("LSQR", "20", xl, sec)
            for label, lam_, meth, x0 in (("IRN-TV", 0.0, cbct.METHOD_PICCS, zero),
                                         ("IRN-PIPLE", 1.0, cbct.METHOD_PIPLE, xp_d),
                                         ("IRN-PICCS", 1.0, cbct.METHOD_PICCS, xp_d)):
                for k in (1, 2, 3, 4):
                    p = cbct.SolveParams(1.0, lam_, 0.1, k, 25, method=meth)
                    xk, sec = timed(lambda: solve(x0, p))
                    record(label, f"{25 * k} ({k} outer)", xk, sec)
            record("prior x_p", "-", xp_d, 0.0)
            out[f"{name}_{V}views"] = rows
            g.close()
    return out


def c3_precision_bench(args, cbct, synth, np, torch, dev):
    """512^3 / 120 views / 1024 x 768: FP32 vs mixed BF16 vs mixed FP16 solves
    (5 x 10), prior = the object without the change, I0 = 5e4."""
    gd = synth.geometry("c3_512")
    sp = synth.SOLVE_PARAMS["c2"]
    t = time.time()
    prior, cur = synth.c3_case()
    log(f"[c3] phantom 512^3 in {time.time() - t:.1f}s")
    g = cbct.Geometry.from_dict(gd)
    xp = torch.from_numpy(prior.astype(np.float32)).to(dev)
    tr = torch.from_numpy(cur.astype(np.float32)).to(dev)
    del prior, cur
    y = cbct.forward(g, tr)
    gen = torch.Generator(device=dev)
    gen.manual_seed(3)
    lam = sp["I0"] * torch.exp(-synth.MU_WATER_PER_MM * y.double())
    b = (-torch.log(torch.clamp(torch.poisson(lam, generator=gen), min=1.0) / sp["I0"])
         / synth.MU_WATER_PER_MM).float()
    del lam, y
    out, ref = {}, None
    for name, pr in (("fp32", cbct.PREC_FP32), ("mixed_bf16", cbct.PREC_MIXED_BF16),
                     ("mixed_f16", cbct.PREC_MIXED_F16)):
        p = cbct.SolveParams(sp["alpha"], sp["lam"], sp["tau"], sp["n_outer"], sp["n_inner"],
                             precision=pr)
        ws = cbct.alloc_workspace(g, p, device=dev)
        x = xp.clone()
        cbct.solve(g, b, xp, x, p, workspace=ws, report=False)   # warm-up
        torch.cuda.synchronize()
        reps = args.c3_reps
        t = time.perf_counter()
        for _ in range(reps):
            x.copy_(xp)
            cbct.solve(g, b, xp, x, p, workspace=ws, report=False)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t) / reps
        if ref is None:
            ref = x.clone()
        out[name] = {"s_per_recon": round(sec, 3),
                     "rel_err_vs_truth": round(float(torch.linalg.norm(x - tr)
                                                     / torch.linalg.norm(tr)), 5),
                     "rel_l2_vs_fp32": float(torch.linalg.norm(x - ref) / torch.linalg.norm(ref))}
        del ws
        log(f"[c3] {name}: {sec:.3f} s/recon, err vs truth {out[name]['rel_err_vs_truth']}")
    for k in out:
        out[k]["speedup_vs_fp32"] = round(out["fp32"]["s_per_recon"] / out[k]["s_per_recon"], 3)
    out["prior_rel_err_vs_truth"] = round(float(torch.linalg.norm(xp - tr)
                                                / torch.linalg.norm(tr)), 5)
    return out


def c5_repeated_bench(args, cbct, synth, np, torch, dev):
    """Ten 180-view scans of 512 x 512 x 400 with a needle advancing 3 mm per
    scan, served for one patient: x_p = anatomy without the needle resident on
    the device, each scan warm-started from the previous reconstruction
    (device-resident), 4 x 10 iterations.  FP32, then mixed BF16."""
    gd = synth.geometry("c5")
    sp = synth.SOLVE_PARAMS["c5"]
    t = time.time()
    base, centre, axis = synth.c5_case()
    log(f"[c5] phantom 512x512x400 in {time.time() - t:.1f}s")
    g = cbct.Geometry.from_dict(gd)
    base_d = torch.from_numpy(base.astype(np.float32)).to(dev)
    gen = torch.Generator(device=dev)
    scans = []
    for s_ in range(1, 11):
        cur = base_d.clone()
        cur.view(-1)[torch.from_numpy(synth.c5_scan(base, centre, axis, s_)).to(dev)] = 2.0
        y = cbct.forward(g, cur)
        gen.manual_seed(500 + s_)
        lam = sp["I0"] * torch.exp(-synth.MU_WATER_PER_MM * y.double())
        b = (-torch.log(torch.clamp(torch.poisson(lam, generator=gen), min=1.0) / sp["I0"])
             / synth.MU_WATER_PER_MM).float().cpu().numpy()
        scans.append((b, cur.cpu().numpy()))
        del y, lam, cur
    g.close()
    log(f"[c5] 10 scans ready ({time.time() - t:.1f}s)")
    out = {}
    for name, pr in (("fp32", cbct.PREC_FP32), ("mixed_bf16", cbct.PREC_MIXED_BF16)):
        p = cbct.SolveParams(sp["alpha"], sp["lam"], sp["tau"], sp["n_outer"], sp["n_inner"],
                             precision=pr)
        rows = []
        with cbct.Server(hbm_budget_bytes=32 << 30, max_slots=1) as srv:
            srv.add_prior(0, gd, base.astype(np.float32))
            xo = np.empty(base.shape, np.float32)
            for s_, (b, truth) in enumerate(scans, 1):
                tk = srv.submit(0, gd, b, p, cbct.X0_PREVIOUS)
                rc, _, info = srv.wait(tk, xo, timeout=600)
                assert rc == 0, info["error"]
                err = float(np.linalg.norm(xo - truth) / np.linalg.norm(truth))
                rows.append({"scan": s_, "latency_s": round(info["t_done"] - info["t_submit"], 3),
                             "gpu_s": round(info["t_done"] - info["t_admit"], 3),
                             "rel_err_vs_truth": round(err, 5)})
                log(f"[c5] {name} scan {s_}: {rows[-1]['latency_s']:.2f} s, err {err:.4f}")
        out[name] = rows
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--c2-steps", type=int, default=3,
                    help="timed solves per precision form of the 256^3 case")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-c2", action="store_true", help="skip the 256^3 case")
    ap.add_argument("--no-c3", action="store_true", help="skip the 512^3 precision comparison")
    ap.add_argument("--c3-reps", type=int, default=1,
                    help="timed solves per precision form of the 512^3 case")
    ap.add_argument("--fp32-only", action="store_true", help="skip the mixed-precision forms")
    ap.add_argument("--op-reps", type=int, default=10)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (profiler calibration)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving stream")
    ap.add_argument("--oracle-c2-solve", action="store_true",
                    help="a full-size 256^3 IRN-PICCS solve on the FP64 oracle (about 17 min "
                         "on 16 host threads at 4 outer steps) against every GPU precision form")
    ap.add_argument("--oracle-c2-outer", type=int, default=4)
    ap.add_argument("--quality", action="store_true",
                    help="only the head / thorax stand-in quality table (PSNR, SSIM)")
    ap.add_argument("--quality-head-only", action="store_true")
    ap.add_argument("--c3-precision", action="store_true",
                    help="only the 512^3 / 120-view FP32 vs mixed comparison")
    ap.add_argument("--c5-repeated", action="store_true",
                    help="only the ten-scan 512x512x400 repeated sequence through the server")
    ap.add_argument("--ops-only", action="store_true",
                    help="time only the projector pair on random data (profiler passes)")
    ap.add_argument("--workload", default="c5", choices=["c1", "c2", "c5"],
                    help="geometry of --ops-only")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving stream and print its JSON")
    ap.add_argument("--serve-requests", type=int, default=80,
                    help="measured requests per arrival rate")
    ap.add_argument("--serve-warmup", type=int, default=10)
    ap.add_argument("--serve-rho", type=lambda s: [float(v) for v in s.split(",")],
                    default=[0.5, 0.9],
                    help="arrival rates as fractions of capacity, e.g. 0.5,0.7,0.9")
    ap.add_argument("--serve-pool", type=int, default=24)
    ap.add_argument("--serve-slots", type=int, default=2)
    ap.add_argument("--serve-budget-gib", type=int, default=64)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the projectors and solver run on one GPU; --gpus {args.gpus} is not "
              "supported (view sharding over several GPUs is described, not built)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2509_08574_amd import cbct, synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.ops_only:
        # the projector pair alone on random data of the workload's shape
        # (their cost does not depend on the values); for profiler passes
        gq = cbct.Geometry.from_dict(synth.geometry(args.workload))
        vf, voff, pf = cbct.col_sizes(gq)
        gen = torch.Generator(device=dev)
        gen.manual_seed(7)
        xc = torch.rand(vf, generator=gen, device=dev)
        ywc = torch.rand(pf, generator=gen, device=dev)
        xc = cbct.vol_to_cols(gq, cbct.cols_to_vol(gq, xc))     # zero pads and guards
        ops, roof = projector_pair(args, cbct, torch, gq, xc, ywc, stream, args.workload)
        del xc, ywc
        # then one short FP32 solve (1 x 4), so that profiler passes also see the
        # stencils, vector updates and reductions at this size
        b = torch.rand(gq.proj_shape, generator=gen, device=dev) * 5.0
        xp = torch.rand(gq.vol_shape, generator=gen, device=dev)
        cbct.solve(gq, b, xp, xp.clone(), cbct.SolveParams(1.0, 1.0, 0.1, 1, 4), report=False)
        torch.cuda.synchronize()
        print(json.dumps(dict(ops, roofline=roof)), flush=True)
        return
    if args.serve_only:
        print(json.dumps({"serving": serving_bench(args, cbct, synth, np, torch, dev)}),
              flush=True)
        return
    if args.c3_precision:
        print(json.dumps({"c3_precision": c3_precision_bench(args, cbct, synth, np, torch, dev)}),
              flush=True)
        return
    if args.c5_repeated:
        print(json.dumps({"c5_repeated": c5_repeated_bench(args, cbct, synth, np, torch, dev)}),
              flush=True)
        return
    if args.quality:
        print(json.dumps({"quality": quality_bench(args, cbct, synth, np, torch, dev)}),
              flush=True)
        return
    if args.oracle_c2_solve:
        print(json.dumps({"oracle_c2_solve": cpu_baseline_c2_solve(args, cbct, synth, np,
                                                                   torch, dev)}), flush=True)
        return

    copy_gbps = stream_copy_gbps(torch, dev)
    log(f"[bench] device copy of 1 GiB: {copy_gbps:.0f} GB/s")
    c5 = repeated_scans(args, cbct, synth, np, torch, dev, stream)
    for part in (c5["roofline"].get("hbm"),):
        if part:
            part["stream_copy_GBps"] = round(copy_gbps, 1)
            part["frac_of_stream_copy"] = round(part["achieved"] / copy_gbps, 4)
    f32 = c5["forms"]["fp32"]
    c2 = None if args.no_c2 else c2_case_forms(args, cbct, synth, np, torch, dev, stream)
    c3 = None if args.no_c3 else c3_precision_bench(args, cbct, synth, np, torch, dev)
    cpu, errs = (None, {}) if args.no_cpu else cpu_baseline_and_oracle_errors(
        args, cbct, synth, np, torch, dev, c5)
    forms = c5["forms"]
    for name, e in errs.items():
        if name in forms:
            forms[name]["rel_l2_vs_fp64_oracle"] = e
    serving = None if args.no_serve else serving_bench(args, cbct, synth, np, torch, dev)

    gd, sp = c5["gd"], c5["sp"]
    out = {
        "metric": "Gvoxel-proj/s for A and A^T; s/recon + p99 latency, FP32 vs mixed",
        "value": f32["value_gvoxel_proj_s"],
        "unit": "Gvoxel-proj/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * f32["s_per_recon"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"c5: ten-scan repeated sequence, {gd['nx']}x{gd['ny']}x{gd['nz']} volume "
                        f"at {gd['vx']} mm, {gd['n_views']} views, {gd['nu']}x{gd['nv']} detector "
                        f"at {gd['du']} mm, needle +3 mm per scan, IRN-PICCS "
                        f"{sp['n_outer']}x{sp['n_inner']} LSQR per scan warm-started from the "
                        f"previous reconstruction, fp32 storage, fp64 Krylov scalars",
            "voxel_proj_per_step": c5["vox_proj_step"],
            "products_per_step": c5["products"],
            "s_per_recon": f32["s_per_recon"],
            "step_ms_p50": f32["step_ms_p50"],
            "step_ms_max": f32["step_ms_max"],
            "rel_err_vs_truth": f32["rel_err_vs_truth"],
            "rel_err_prior_vs_truth": f32["rel_err_prior_vs_truth"],
            **c5["ops"],
        },
        "precision_forms": forms,
        # every form against the FP64 oracle on reduced problems (labelled by case)
        "precision_vs_fp64_oracle": errs,
        "c2": c2,
        # 512^3 at 0.5 mm, 1024 x 768 at 0.4 mm, 120 views, 5 x 10: the three forms
        "c3_512": c3,
        "serving": serving,
        "roofline": c5["roofline"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
