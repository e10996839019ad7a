"""Benchmark: batched 12-RHS solves of the Wilson-clover operator with the
two-level DD-alpha-AMG solver on one MI355X.

Workload (default): 32^3x64 lattice, links exp(i*0.2*H) reunitarised, c_sw = 1,
m0 from the tuned-mass table, 4^4 aggregates/SAP domains, n = 20 test vectors,
4 adaptive setup iterations, the 12 spin-colour point sources at the origin
solved together to a true relative residual of 1e-10 with the FP64 operator.
Links, clover, clover inverse and test vectors are stored in BF16 for the FP32
inner solver (--store f32 / f16 for the other forms); the outer solver, the
Gram-Schmidt and the coarse-operator build run in FP64.
Inputs are synthetic and seeded (there is no gauge-field dataset here).

A step is one batched solve of the 12 right-hand sides with the setup resident
on the device; `value` is right-hand sides solved per second over the timed
steps.  The line also carries the roofline of the dominant kernel (timed with
HIP events on its launch stream over the timed steps) and the oracle's CPU
throughput on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config C3] [--store bf16|f16|f32[,...]]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz = 78.6 TFLOP/s for
# non-packed instructions; the published 157.3 TFLOP/s counts packed FP32 (2 per lane), which
# this library does not emit.  Kernels whose arithmetic intensity at the workload's batch is above
# the FP32 ridge (157.3 / 8 = 19.7 flop/byte) are rated against the FP32 peak ("alu").
FP32_PEAK_TFLOPS = 157.3
FP32_NONPACKED_TFLOPS = 78.6
ALU_BOUND = {"k_sap_colour", "k_sap_dom", "k_sap_dom_persist"}
TOL = 1e-10

# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs of this workload
# (scaled by the copy-kernel calibration: FETCH_SIZE x2.000, WRITE_SIZE x1.000; see
# profiles/k_sap_dom_c3_pmc.md), per smoother layout.  Reported only while the
# kernel's sources are unchanged since the measurement.
_SAP_DOM_SOURCES = ["paper_1811_00355_amd/csrc/sap_dom.hip", "paper_1811_00355_amd/csrc/dslash.h",
                    "paper_1811_00355_amd/csrc/dd_internal.h"]
MEASURED_TRAFFIC = {
    ("k_sap_dom", "C3", "bf16", "dom2"): dict(bytes=9.7722e9 + 1.2079e9, sha="4e22c633ba1d7a63", sources=_SAP_DOM_SOURCES),
    ("k_sap_dom", "C3", "bf16", "dom4"): dict(bytes=8.0589e9 + 1.2079e9, sha="4e22c633ba1d7a63", sources=_SAP_DOM_SOURCES),
}


def sap_layout(t):
    """Name of the smoother layout a tuning selects: domD (domain-resident, D RHS per workgroup) or wpeW."""
    return f"dom{t['sap_dom_rhs']}" if t.get("sap_dom_rhs") else f"wpe{t['sap_wpe']}"


def measured_traffic(kernel, config, store, layout):
    import hashlib
    m = MEASURED_TRAFFIC.get((kernel, config, store, layout))
    if m is None:
        return None
    h = hashlib.sha256()
    for f in m["sources"]:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return m["bytes"] if h.hexdigest()[:16] == m["sha"] else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _oracle_sample(cfg, n_vec, coarse_iters, coarse_restart, budget_s):
    """One worker of the CPU baseline: time outer FGMRES iterations (FP64
    operator apply + V-cycle with SAP and the coarse even-odd GMRES) of the
    oracle, as it is, on an 8^3x16 sub-volume with the workload's parameters,
    on one core.  Returns seconds per iteration and the repetitions."""
    from threadpoolctl import threadpool_limits
    from oracle.lattice import Lattice
    from oracle.dirac import WilsonClover
    from oracle import amg
    from workloads import su3_field, gauss_vectors, gauss_spinor
    L_s = (8, 8, 8, 16)
    with threadpool_limits(limits=1):
        lat = Lattice(L_s, cfg["block"])
        U = su3_field(L_s, cfg["eps"], cfg["gauge_seed"])
        W = WilsonClover(U, lat, cfg["m0"], cfg["c_sw"])
        tv = gauss_vectors(n_vec, lat.V, cfg["tv_seed"]).reshape(n_vec, lat.V, 4, 3)
        p = amg.MGParams(n_vec=n_vec, coarse_fixed_iters=coarse_iters, coarse_restart=min(coarse_restart, coarse_iters))
        mg = amg.TwoLevel(W, tv, p)
        v = gauss_spinor(L_s, 1, 5)[0]
        t0 = time.perf_counter()
        reps = 0
        while True:
            z = mg.vcycle(v)
            W.apply(z)
            reps += 1
            if time.perf_counter() - t0 > budget_s or reps >= 10:
                break
        return (time.perf_counter() - t0) / reps, reps, lat.V


def cpu_baseline(cfg, lat_shape, n_vec, gpu_outer_iters, gpu_coarse_iters_per_vcycle, coarse_restart):
    """The oracle on the host's cores: one worker process per core (at most the
    16 cores a one-GPU share has), each timing the bounded sample of
    _oracle_sample; independent solves run side by side, so the host's rate is
    workers / (time per solve), with time per solve = time per outer iteration
    x the volume ratio to the full lattice x the GPU's outer iteration count
    (an extrapolation, labelled as such)."""
    import multiprocessing as mp
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    coarse_iters = max(1, int(round(gpu_coarse_iters_per_vcycle)))
    ctx = mp.get_context("spawn")      # fresh interpreters: nothing of this process's GPU state
    with ctx.Pool(cores) as pool:
        res = pool.starmap(_oracle_sample, [(cfg, n_vec, coarse_iters, coarse_restart, 12.0)] * cores)
    t_iter = float(np.mean([r[0] for r in res]))
    reps = int(sum(r[1] for r in res))
    V_s = res[0][2]
    V_full = int(np.prod(lat_shape))
    t_solve = t_iter * (V_full / V_s) * gpu_outer_iters
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), model)
    except OSError:
        pass
    return dict(value=cores / t_solve, unit="solves/s", cores=cores, cpu_model=model, kind="oracle",
                sample=(f"{cores} worker processes, one per core, each timing outer FGMRES iterations (FP64 D + "
                        f"V-cycle: SAP 4x4, coarse GMRES {coarse_iters} its, restart {min(coarse_restart, coarse_iters)}) "
                        f"of the numpy oracle on an 8^3x16 sub-volume ({reps} iterations in all, "
                        f"{t_iter:.2f} s each); extrapolated by volume x{V_full // V_s} and {gpu_outer_iters:.1f} "
                        f"outer iterations per solve"))


def dapply_table(B, g, reps=20):
    """D apply throughput on this lattice for the storage forms of the operator:
    algorithmic bytes (spinors in and out per RHS, links and clover once) over
    the mean launch time from the library's kernel timer."""
    import torch
    rows = {}
    for name, dt, nrhs in (("f64_1rhs", B.DD_F64, 1), ("f32_1rhs", B.DD_F32, 1), ("f16ops_1rhs", B.DD_F16, 1),
                           ("bf16ops_1rhs", B.DD_BF16, 1), ("f64_12rhs", B.DD_F64, 12), ("f32_12rhs", B.DD_F32, 12),
                           ("f16ops_12rhs", B.DD_F16, 12), ("bf16ops_12rhs", B.DD_BF16, 12)):
        src, dst = g.new_packed(dt, nrhs), g.new_packed(dt, nrhs)
        g.dd_dirac_apply(dt, nrhs, src, dst)
        torch.cuda.synchronize()
        B.kernel_timer_enable("k_dirac")
        for _ in range(reps):
            g.dd_dirac_apply(dt, nrhs, src, dst)
        torch.cuda.synchronize()
        k = B.kernel_timer_read("k_dirac")
        B.kernel_timer_enable(None)
        gbs = k["bytes"] / (k["ms"] * 1e-3) / 1e9
        rows[name] = dict(ms=round(k["ms"] / k["launches"], 4), GBs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4))
        del src, dst
    return rows


def sap_table(B, g, cfg, store_name, reps=5, mr=4, layouts=("wpe2", "wpe3", "dom4")):
    """SAP smoother alone on this lattice (12 RHS, N_SAP = 1 sweep per call, mr
    MR steps per domain solve) in the given layouts: mean launch time and the
    roofline figures from the kernel timer."""
    import torch
    dt = B.DTYPES[store_name]
    nrhs = 12
    p = B.default_params(block=cfg["block"], sap_sweeps=1, sap_mr_iters=mr)
    b, x = g.new_packed(dt, nrhs), g.new_packed(dt, nrhs)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(77)
    bf = b.view(torch.float32)            # packed FP32 vectors (the buffer is raw bytes)
    bf.copy_(torch.randn(bf.shape, generator=gen, device="cuda", dtype=torch.float32))
    rows = {}
    t0 = g.dd_gauge_get_tuning()
    all_layouts = {"wpe2": dict(sap_wpe=2, sap_dom_rhs=0), "wpe3": dict(sap_wpe=3, sap_dom_rhs=0),
                   "dom4": dict(sap_dom_rhs=4), "dom2": dict(sap_dom_rhs=2)}
    for name, lay in ((n, all_layouts[n]) for n in layouts):
        g.dd_gauge_set_tuning(**dict(t0, **lay))
        x.zero_()
        g.dd_sap_smooth(p, dt, nrhs, b, x)
        torch.cuda.synchronize()
        B.kernel_timer_enable("*")
        for _ in range(reps):
            g.dd_sap_smooth(p, dt, nrhs, b, x)
        torch.cuda.synchronize()
        k = {n: B.kernel_timer_read(n) for n in B.kernel_timer_names()}
        B.kernel_timer_enable(None)
        (kn, ks), = k.items()
        ms = ks["ms"] / ks["launches"]
        rows[name] = dict(kernel=kn, ms=round(ms, 4), TFLOPs=round(ks["flops"] / (ks["ms"] * 1e-3) / 1e12, 2),
                          frac=round(ks["flops"] / (ks["ms"] * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4))
        log(f"[bench] SAP {store_name} k={mr} {name}: {rows[name]}")
    g.dd_gauge_set_tuning(**t0)
    return rows


def baseline_dd(B, g, b, args, store_name):
    """The paper's comparison solver on the same 12 sources: FP64 defect
    correction around an FP32 BiCGstab right-preconditioned by SAP with
    N_SAP = 5.  Run one defect-correction step per call (each continuing from
    the previous iterate) so that every step reports its progress; the timed
    figure is the sum of the calls."""
    import torch
    p = B.bicgstab_params(store_dtype=B.DTYPES[store_name], max_outer_iters=1, use_x0=1)
    x = torch.zeros_like(b)
    total, inner, outer = 0.0, 0, 0
    info = None
    prev = float("inf")
    for step in range(20):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info, st = g.dd_solve_bicgstab(p, b.shape[0], b, x, TOL, raise_on_noconv=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        total += dt
        inner += info[0]["inner_iters"]
        outer += info[0]["outer_iters"]
        worst = max(i["true_relres"] for i in info)
        log(f"[bench] baseline step {step}: {dt:.2f} s, inner steps {info[0]['inner_iters']}, "
            f"max true relres {worst:.2e}")
        if st == 0 or worst >= prev or total > 120.0:    # converged, diverging, or out of time
            break
        prev = worst
    ok = all(i["converged"] and i["true_relres"] <= TOL for i in info)
    return dict(solves_per_s=round(b.shape[0] / total, 4), seconds=round(total, 3), converged=ok,
                outer_iters=outer, inner_iters=inner, max_true_relres=max(i["true_relres"] for i in info),
                sap_sweeps=p.sap_sweeps, inner_tol=p.inner_tol, store_dtype=store_name)


def fp64_single_rhs(B, g, cfg, b, args):
    """The comparison form: an all-FP64 setup, then the 12 sources solved one at
    a time (single-RHS FP64 solves, one after another)."""
    import torch
    blk, n_vec = cfg["block"], cfg["n_vec"]
    p = B.default_params(block=blk, n_vec=n_vec, setup_iters=cfg["setup_iters"], inner_dtype=B.DD_F64,
                         store_dtype=B.DD_F64, seed=cfg["tv_seed"], coarse_restart=args.coarse_restart,
                         coarse_max_iters=args.coarse_max_iters, coarse_cgs_passes=args.coarse_cgs_passes,
                         outer_cgs_passes=args.outer_cgs_passes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mg = B.MG(g, p)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    mg.dd_mg_set_graphs(args.graphs)
    x = torch.zeros_like(b[:1])
    mg.dd_solve(1, b[:1].contiguous(), x, TOL)        # workspace allocation and graph capture, untimed
    torch.cuda.synchronize()
    iters = []
    t0 = time.perf_counter()
    for k in range(b.shape[0]):
        x = torch.zeros_like(b[k:k + 1])
        info, st = mg.dd_solve(1, b[k:k + 1].contiguous(), x, TOL, raise_on_noconv=False)
        if st or not info[0]["converged"]:
            raise RuntimeError(f"FP64 single-RHS solve {k} did not converge: {info}")
        iters.append(info[0]["outer_iters"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    mg.destroy()
    return dict(solves_per_s=round(b.shape[0] / elapsed, 3), setup_s=round(t_setup, 3),
                outer_iters_mean=round(float(np.mean(iters)), 2), seconds=round(elapsed, 3))


def _mixed_mg(B, g, cfg, args, store_name):
    p = B.default_params(block=cfg["block"], n_vec=cfg["n_vec"], setup_iters=cfg["setup_iters"],
                         inner_dtype=B.DD_F32, store_dtype=B.DTYPES[store_name], seed=cfg["tv_seed"],
                         coarse_restart=args.coarse_restart, coarse_max_iters=args.coarse_max_iters,
                         coarse_cgs_passes=args.coarse_cgs_passes, outer_cgs_passes=args.outer_cgs_passes)
    mg = B.MG(g, p)
    mg.dd_mg_set_graphs(args.graphs)
    return mg


def sigma_leg(B, g, cfg, args, store_name, b, light):
    """sigma_min(D) at the benchmark's mass by block inverse iteration through
    the solver (an upper bound that tightens with the iterations), and, where
    the mass search recorded one, the 12-RHS solve rate at the mass of the
    smallest sigma_min found on this field."""
    import torch
    from paper_1811_00355_amd.spectrum import sigma_min
    t0 = time.perf_counter()
    mg = _mixed_mg(B, g, cfg, args, store_name)
    sig, hist, its = sigma_min(mg, g.V, nvec=4, iters=args.sigma_iters, tol=1e-8, rtol=0.01,
                               log=lambda m: log("[bench] " + m))
    mg.destroy()
    out = dict(value=round(sig, 5), history=[round(h, 5) for h in hist], m0=cfg["m0"], nvec=4, solve_tol=1e-8,
               bound="upper (Rayleigh-Ritz on (D^dag D)^-1)", seconds=round(time.perf_counter() - t0, 1),
               free_field_floor=round(math.sin(math.pi / cfg["L"][3]), 5))
    if light:
        out["search"] = {k: light[k] for k in ("target", "reached", "m0", "sigma_min")}
        out["search"]["trials"] = len(light["trials"])
        g.dd_gauge_set_mass(light["m0"])
        mg = _mixed_mg(B, g, cfg, args, store_name)
        t = g.dd_gauge_get_tuning()
        t.update(coarse_half=0, coarse_basis_half=0, coarse_mfma_half=0)
        g.dd_gauge_set_tuning(**t)
        x = torch.zeros_like(b)
        mg.dd_solve(b.shape[0], b, x, TOL)               # workspace and graphs, untimed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 2
        for _ in range(reps):
            x = torch.zeros_like(b)
            info, _ = mg.dd_solve(b.shape[0], b, x, TOL)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        mg.destroy()
        g.dd_gauge_set_mass(cfg["m0"])
        out["at_search_mass"] = dict(m0=light["m0"], solves_per_s=round(b.shape[0] / dt, 3),
                                     outer_iters=max(i["outer_iters"] for i in info),
                                     max_true_relres=max(i["true_relres"] for i in info))
    return out


def _roofline(kernel, ks, elapsed_ms_per_launch_set, args, store_name, layout):
    """Roofline entry of one kernel from its kernel-timer record (algorithmic
    bytes and flops per launch over the mean event-timed launch duration)."""
    avg_ms = ks["ms"] / max(ks["launches"], 1)
    gbs = ks["bytes"] / (ks["ms"] * 1e-3) / 1e9
    tfs = ks["flops"] / (ks["ms"] * 1e-3) / 1e12
    ai = ks["flops"] / max(ks["bytes"], 1.0)
    if kernel in ALU_BOUND and ai > FP32_PEAK_TFLOPS * 1e3 / HBM_PEAK_GBS:
        r = dict(bound="alu", achieved=round(tfs, 2), peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                 frac=round(tfs / FP32_PEAK_TFLOPS, 4), frac_of_nonpacked_peak=round(tfs / FP32_NONPACKED_TFLOPS, 4),
                 algorithmic_flops_per_launch=round(ks["flops"] / max(ks["launches"], 1)))
    else:
        r = dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(gbs / HBM_PEAK_GBS, 4))
    r.update(traffic=measured_traffic(kernel, args.config, store_name, layout), kernel=kernel,
             algorithmic_bytes_per_launch=round(ks["bytes"] / max(ks["launches"], 1)),
             hbm_GBs_algorithmic=round(gbs, 1), arithmetic_intensity=round(ai, 2),
             avg_launch_ms=round(avg_ms, 4), launches=ks["launches"])
    return r


def _level3_params(B, args):
    return B.level3_params(n_vec2=args.l3_nvec2, setup_iters=args.l3_setup_iters, mr_steps=args.l3_mr,
                           kcycle_max_iters=args.l3_kmax, l3_tol=args.l3_tol)


def level3_leg(B, mg, args, step, value2, half_store):
    """The same solves with the third level added to the same setup (the coarse
    correction then a level-2 FGMRES cycle preconditioned by the level-3 solve
    and MR smoothing): its setup time, one untimed step with every kernel
    timed, then args.steps timed steps; the level is removed afterwards."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mg.add_level(_level3_params(B, args))
    torch.cuda.synchronize()
    t_l3 = time.perf_counter() - t0
    vc3, nc3 = mg.level3_shape()
    step()
    mg.dd_mg_set_graphs(0)
    B.kernel_timer_enable("*")
    binfo = step()
    torch.cuda.synchronize()
    kf = {k: B.kernel_timer_read(k) for k in B.kernel_timer_names()}
    B.kernel_timer_enable(None)
    mg.dd_mg_set_graphs(args.graphs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    half = None
    if half_store and not args.no_half_coarse:
        # the same with half-precision coarse blocks (D_c and D3) on half matrix cores, FP16 bases
        t = mg.g.dd_gauge_get_tuning()
        mg.g.dd_gauge_set_tuning(**dict(t, coarse_half=1, coarse_basis_half=1, coarse_mfma_half=1))
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infh = [step() for _ in range(args.steps)]
        torch.cuda.synchronize()
        elh = time.perf_counter() - t0
        mg.g.dd_gauge_set_tuning(**t)
        half = dict(value=round(len(infh[0]) * args.steps / elh, 3), ms_per_step=round(1e3 * elh / args.steps, 2),
                    outer_iters_mean=round(float(np.mean([i["outer_iters"] for inf in infh for i in inf])), 2),
                    max_true_relres=float(max(i["true_relres"] for inf in infh for i in inf)))
    mg.remove_level()
    nrhs = len(infos[0])
    value = nrhs * args.steps / el
    outer = [i["outer_iters"] for inf in infos for i in inf]
    tot = sum(v["ms"] for v in kf.values())
    out = dict(value=round(value, 3), ms_per_step=round(1e3 * el / args.steps, 2),
               speedup_vs_two_levels=round(value / value2, 3), setup_s=round(t_l3, 3),
               level3_sites=vc3, level3_components=nc3, n_vec2=args.l3_nvec2, setup_iters=args.l3_setup_iters,
               mr_steps=args.l3_mr, kcycle_max_iters=args.l3_kmax, l3_tol=args.l3_tol,
               outer_iters_mean=round(float(np.mean(outer)), 2),
               level2_steps_total=[i["coarse_iters_total"] for i in binfo[::max(1, min(args.rhs_batch, nrhs))]],
               max_true_relres=float(max(i["true_relres"] for inf in infos for i in inf)),
               half_coarse_arithmetic=half,
               kernels={k: dict(ms_per_step=round(v["ms"], 3), share=round(v["ms"] / max(tot, 1e-9), 3),
                                launches_per_step=v["launches"])
                        for k, v in sorted(kf.items(), key=lambda kv: -kv[1]["ms"])[:14]})
    log(f"[bench] three levels: {out}")
    return out


def measure(B, g, cfg, args, store_name, b):
    """Setup with operands stored as `store_name`, autotune, warm up, one
    untimed step with every kernel timed (the breakdown, which names the
    dominant kernel), then args.steps timed solves of the 12 sources (in calls
    of args.rhs_batch) with only the dominant kernel bracketed by events."""
    import torch
    blk, n_vec = cfg["block"], cfg["n_vec"]
    nrhs = b.shape[0]
    store = B.DTYPES[store_name]
    p = B.default_params(block=blk, n_vec=n_vec, setup_iters=cfg["setup_iters"], inner_dtype=B.DD_F32,
                         store_dtype=store, seed=cfg["tv_seed"], coarse_restart=args.coarse_restart,
                         coarse_max_iters=args.coarse_max_iters, coarse_cgs_passes=args.coarse_cgs_passes,
                         outer_cgs_passes=args.outer_cgs_passes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mg = B.MG(g, p)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    log(f"[bench] store {store_name}: setup {t_setup:.2f} s")
    mg.dd_mg_set_graphs(args.graphs)
    half_store = store_name in ("f16", "bf16")
    t = g.dd_gauge_get_tuning()
    t.update(coarse_half=args.coarse_half if half_store else 0, coarse_basis_half=args.coarse_basis_half,
             coarse_mfma_half=args.coarse_mfma_half if half_store else 0)
    g.dd_gauge_set_tuning(**t)
    kb = min(args.rhs_batch, nrhs)
    tuning = None
    if args.autotune:
        t0 = time.perf_counter()
        rep = mg.dd_autotune(kb, args.tune_cache)
        tuning = dict(chosen=g.dd_gauge_get_tuning(), seconds=round(time.perf_counter() - t0, 2),
                      candidates=[l for l in rep.splitlines() if " ms" in l])
        log(f"[bench] autotune ({tuning['seconds']} s): " + "; ".join(rep.splitlines()[1:]))
    level3 = None
    if args.levels == 3:
        # third level after the tuning (the autotuner refuses a setup with one); its setup time counts
        p3 = _level3_params(B, args)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mg.add_level(p3)
        torch.cuda.synchronize()
        t_l3 = time.perf_counter() - t0
        t_setup += t_l3
        vc3, nc3 = mg.level3_shape()
        level3 = dict(setup_s=round(t_l3, 3), sites=vc3, components=nc3, n_vec2=args.l3_nvec2,
                      setup_iters=args.l3_setup_iters, mr_steps=args.l3_mr, kcycle_max_iters=args.l3_kmax)
        log(f"[bench] third level: {level3}")

    def step():
        info = []
        for k0 in range(0, nrhs, kb):
            bk = b[k0:k0 + kb]
            xk = torch.zeros_like(bk)
            ik, st = mg.dd_solve(bk.shape[0], bk, xk, TOL, raise_on_noconv=False)
            bad = [k0 + r for r, i in enumerate(ik) if not (i["converged"] and i["true_relres"] <= TOL)]
            if st or bad:
                raise RuntimeError(f"solve did not converge (status {st}, rhs {bad}): {ik}")
            info += ik
            if level3 is not None:
                k2, k3 = mg.level3_last()
                level3_steps.append((k2, k3))
        return info

    level3_steps = []

    for w in range(args.warmup):
        info = step()
        log(f"[bench] warmup {w}: outer iterations {[i['outer_iters'] for i in info]}")

    # breakdown: one untimed step, graphs off so that every launch is seen, every kernel timed
    mg.dd_mg_set_graphs(0)
    B.kernel_timer_enable("*")
    binfo = step()
    torch.cuda.synchronize()
    kfull = {k: B.kernel_timer_read(k) for k in B.kernel_timer_names()}
    B.kernel_timer_enable(None)
    mg.dd_mg_set_graphs(args.graphs)
    dom = max(kfull, key=lambda k: kfull[k]["ms"])
    model_bytes = sum(v["bytes"] for v in kfull.values())
    model_flops = sum(v["flops"] for v in kfull.values())
    kernels = {k: dict(ms_per_step=round(v["ms"], 3), launches_per_step=v["launches"],
                       GBs=round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1))
               for k, v in sorted(kfull.items(), key=lambda kv: -kv[1]["ms"])}

    # timed steps: only the dominant kernel carries events
    B.kernel_timer_enable(dom)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for s_ in range(args.steps):
        ts = time.perf_counter()
        infos.append(step())
        log(f"[bench] step {s_}: {time.perf_counter() - ts:.3f} s, max relres "
            f"{max(i['true_relres'] for i in infos[-1]):.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kd = B.kernel_timer_read(dom)
    B.kernel_timer_enable(None)
    layout = sap_layout(g.dd_gauge_get_tuning())
    seen = kd["launches"] == kfull[dom]["launches"] * args.steps
    roofline = _roofline(dom, kd if seen else kfull[dom], None, args, store_name, layout)
    roofline.update(share_of_step=round((kd["ms"] if seen else kfull[dom]["ms"] * args.steps) / (1e3 * elapsed), 3),
                    timed_in="timed steps" if seen else "the breakdown step (launches inside graphs)")
    outer = float(np.mean([i["outer_iters"] for inf in infos for i in inf]))
    coarse_per_vcycle = float(np.mean([sum(i["coarse_iters_total"] for i in inf[::kb]) /
                                       max(sum(max(i["outer_iters"] for i in inf[k0:k0 + kb])
                                               for k0 in range(0, nrhs, kb)), 1) for inf in infos]))
    value = nrhs * args.steps / elapsed
    V = int(np.prod(cfg["L"]))
    # whole-step model (the breakdown step's launches): algorithmic bytes and flops of every kernel
    step_model = dict(GB=round(model_bytes / 1e9, 2), GFLOP=round(model_flops / 1e9, 1),
                      mflop_per_site_per_solve=round(model_flops / (V * nrhs) / 1e6, 2),
                      hbm_frac_of_step=round(model_bytes / (elapsed / args.steps) / (HBM_PEAK_GBS * 1e9), 4),
                      info_flops_model=int(binfo[0]["flops_model"]), info_bytes_model=int(binfo[0]["bytes_model"]))
    log(f"[bench] store {store_name}: {value:.2f} solves/s; dominant kernel {dom}: {roofline}; kernels {kernels}")
    log(f"[bench] step model {step_model}")
    if level3 is not None:
        level3["last_cycle_steps"] = level3_steps[-1] if level3_steps else None
    whole_m = None
    if args.graphs != 2 and not args.no_whole_m_graph and level3 is None:
        # the same solves with all of M replayed from one graph per call (graph mode 2: no host
        # synchronisation inside M, the coarse GMRES stopped on the device): bits and iterations equal
        mg.dd_mg_set_graphs(2)
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infw = [step() for _ in range(args.steps)]
        torch.cuda.synchronize()
        elw = time.perf_counter() - t0
        mg.dd_mg_set_graphs(args.graphs)
        whole_m = dict(value=round(nrhs * args.steps / elw, 3), ms_per_step=round(1e3 * elw / args.steps, 2),
                       outer_iters_mean=round(float(np.mean([i["outer_iters"] for inf in infw for i in inf])), 2),
                       coarse_max_iters=args.coarse_max_iters)
        log(f"[bench] store {store_name}, all of M from one graph: {whole_m}")
    half_coarse = None
    if half_store and not args.no_half_coarse and not (args.coarse_half and args.coarse_mfma_half and args.coarse_basis_half):
        # the same setup with half-precision coarse blocks on half matrix cores and an FP16 coarse basis
        t = g.dd_gauge_get_tuning()
        g.dd_gauge_set_tuning(**dict(t, coarse_half=1, coarse_basis_half=1, coarse_mfma_half=1))
        if args.autotune and level3 is None:
            mg.dd_autotune(kb, args.tune_cache)
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infh = [step() for _ in range(args.steps)]
        torch.cuda.synchronize()
        elh = time.perf_counter() - t0
        g.dd_gauge_set_tuning(**t)
        half_coarse = dict(value=round(nrhs * args.steps / elh, 3), ms_per_step=round(1e3 * elh / args.steps, 2),
                           coarse=f"{store_name} blocks on {store_name} matrix cores, f16 basis",
                           outer_iters_mean=round(float(np.mean([i["outer_iters"] for inf in infh for i in inf])), 2),
                           max_true_relres=float(max(i["true_relres"] for inf in infh for i in inf)))
        log(f"[bench] store {store_name}, half-precision coarse arithmetic: {half_coarse}")
    three = None
    if level3 is None and not args.no_level3_leg:
        three = level3_leg(B, mg, args, step, value, half_store)
    mg.destroy()
    return dict(value=round(value, 3), ms_per_step=round(1e3 * elapsed / args.steps, 2), elapsed=elapsed,
                setup_s=round(t_setup, 3), outer=round(outer, 2), coarse_per_vcycle=coarse_per_vcycle,
                tuning=tuning, roofline=roofline, kernels=kernels, half_coarse=half_coarse, step_model=step_model,
                whole_m=whole_m, level3=level3, three_level=three)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="C3")
    ap.add_argument("--store", default="bf16",
                    help="operand storage f32|f16|bf16; a comma list measures each in turn (the first is `value`)")
    ap.add_argument("--rhs-batch", type=int, default=12,
                    help="right-hand sides per solve call (the 12 sources go in sub-batches of this size)")
    ap.add_argument("--coarse-restart", type=int, default=60)
    ap.add_argument("--coarse-max-iters", type=int, default=300)
    ap.add_argument("--coarse-cgs-passes", type=int, default=1)
    ap.add_argument("--outer-cgs-passes", type=int, default=1, choices=[1, 2],
                    help="classical Gram-Schmidt passes of the FP64 outer FGMRES")
    ap.add_argument("--graphs", type=int, default=1, choices=[0, 1, 2],
                    help="0: launches; 1: coarse GMRES chunks replayed from HIP graphs; 2: all of M from one graph")
    ap.add_argument("--autotune", type=int, default=1, choices=[0, 1],
                    help="time the launch-shape candidates before the timed steps")
    ap.add_argument("--tune-cache", default=None, help="JSON cache of autotuner choices")
    ap.add_argument("--coarse-half", type=int, default=0, choices=[0, 1],
                    help="half-precision storage: keep the coarse blocks in that type (0: FP32 blocks)")
    ap.add_argument("--coarse-basis-half", type=int, default=0, choices=[0, 1],
                    help="store the FP32 coarse GMRES basis in FP16")
    ap.add_argument("--coarse-mfma-half", type=int, default=0, choices=[0, 1],
                    help="half-precision coarse blocks on FP16/BF16 matrix cores (x rounded to that type)")
    ap.add_argument("--no-whole-m-graph", action="store_true",
                    help="skip the timing with all of M replayed from one graph (graph mode 2)")
    ap.add_argument("--no-half-coarse", action="store_true",
                    help="skip the second timing with half-precision coarse blocks, products and basis")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-single", action="store_true",
                    help="skip the 12 sequential FP64 single-RHS solves")
    ap.add_argument("--no-dapply", action="store_true", help="skip the D-apply bandwidth table")
    ap.add_argument("--dapply-only", action="store_true",
                    help="only prepare the gauge field and print the D-apply bandwidth table (for counter runs)")
    ap.add_argument("--sap-only", action="store_true",
                    help="only prepare the gauge field and time the SAP smoother in every layout (for counter runs)")
    ap.add_argument("--sap-mr", default="4", help="--sap-only: comma list of MR step counts")
    ap.add_argument("--baseline-dd", action="store_true",
                    help="also time the paper's comparison solver (SAP-preconditioned BiCGstab) on the same sources")
    ap.add_argument("--sigma-iters", type=int, default=8,
                    help="inverse-iteration steps of the sigma_min leg (0: skip it)")
    ap.add_argument("--levels", type=int, default=2, choices=[2, 3],
                    help="3: add the third multigrid level (level-2 FGMRES cycle as the coarse solve)")
    ap.add_argument("--l3-nvec2", type=int, default=24, help="third level: level-2 test vectors")
    ap.add_argument("--l3-setup-iters", type=int, default=6, help="third level: inverse iterations of its vectors")
    ap.add_argument("--l3-mr", type=int, default=6, help="third level: MR smoothing steps on D_c")
    ap.add_argument("--l3-kmax", type=int, default=40, help="third level: level-2 FGMRES steps at most")
    ap.add_argument("--l3-tol", type=float, default=0.2, help="third level: level-3 GMRES relative residual")
    ap.add_argument("--no-level3-leg", action="store_true",
                    help="skip the side run with the third level added to the same setup")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU (asked for {args.gpus}); "
              "the multi-GPU domain decomposition is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1811_00355_amd import binding as B
    from workloads import get_config, su3_field

    cfg = get_config(args.config)
    L, blk, n_vec = cfg["L"], cfg["block"], cfg["n_vec"]
    V = int(np.prod(L))
    nrhs = 12
    log(f"[bench] workload {args.config}: L={L} block={blk} n={n_vec} m0={cfg['m0']:.5f} store={args.store}")
    t0 = time.perf_counter()
    U = su3_field(L, cfg["eps"], cfg["gauge_seed"])
    log(f"[bench] gauge field generated on the host in {time.perf_counter() - t0:.1f} s")

    ctx = B.Context(0, hbm_budget_bytes=270 << 30)
    g = B.Gauge(ctx, L, blk, U, cfg["m0"], cfg["c_sw"])
    del U
    if args.sap_only:
        rows = {}
        for st_ in args.store.split(","):
            for mr in (int(v) for v in args.sap_mr.split(",")):
                lay = ("wpe2", "wpe3", "dom4", "dom2") if mr == 4 else ("dom4", "dom2")
                rows[f"{st_}_k{mr}"] = sap_table(B, g, cfg, st_, mr=mr, layouts=lay)
        print(json.dumps({"workload": args.config, "sap": rows}))
        g.destroy()
        ctx.close()
        return
    if args.dapply_only:
        print(json.dumps({"workload": args.config, "dapply": dapply_table(B, g)}))
        g.destroy()
        ctx.close()
        return
    # the 12 spin-colour point sources at the origin, canonical complex128 on the device
    b = torch.zeros((nrhs, V * 12), dtype=torch.complex128, device="cuda")
    for k in range(nrhs):
        b[k, k] = 1.0
    stores = [s_.strip() for s_ in args.store.split(",")]
    runs = [measure(B, g, cfg, args, st_, b) for st_ in stores]
    r0 = runs[0]
    value, ms_per_step, elapsed = r0["value"], r0["ms_per_step"], r0["elapsed"]
    outer, coarse_per_vcycle = r0["outer"], r0["coarse_per_vcycle"]

    out = {
        "metric": "solves/s @ true rel.res 1e-10 (32^3x64, 12 RHS)",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 outer / f32 inner" + (f" ({stores[0]} coarse products, f32 accumulation)"
                                            if args.coarse_mfma_half and args.coarse_half and stores[0] in ("f16", "bf16")
                                            else " (f32 coarse blocks and products on matrix cores)"),
        "data": "synthetic (seeded SU(3) links, point sources)",
        "config": {"workload": f"{args.config}: {L[0]}^3x{L[3]} Wilson-clover, 12 point-source RHS "
                               f"(solve calls of {args.rhs_batch}), {args.levels}-level DD-alpha-AMG n={n_vec}, 4^4 blocks",
                   "lattice": list(L), "rhs": nrhs, "rhs_batch": args.rhs_batch, "m0": cfg["m0"],
                   "c_sw": cfg["c_sw"], "eps": cfg["eps"], "store_dtype": stores[0], "graphs": args.graphs,
                   "coarse_restart": args.coarse_restart, "coarse_cgs_passes": args.coarse_cgs_passes,
                   "outer_cgs_passes": args.outer_cgs_passes,
                   "coarse_blocks": stores[0] if args.coarse_half and stores[0] in ("f16", "bf16") else "f32",
                   "coarse_basis": "f16" if args.coarse_basis_half else "f32",
                   "coarse_mfma_half": bool(args.coarse_mfma_half and args.coarse_half),
                   "outer_iters_mean": round(float(outer), 2),
                   "coarse_iters_per_vcycle": round(float(coarse_per_vcycle), 1),
                   "setup_s": r0["setup_s"],
                   "solves_per_s_incl_setup": round(nrhs / (r0["setup_s"] + elapsed / args.steps), 3),
                   "tuning": r0["tuning"],
                   "half_coarse_arithmetic": r0["half_coarse"],
                   "whole_m_graph": r0["whole_m"],
                   "level3": r0["level3"],
                   "three_level": r0["three_level"],
                   "step_model": r0["step_model"],
                   "other_stores": {st_: {k: r[k] for k in ("value", "ms_per_step", "setup_s", "outer")}
                                    for st_, r in zip(stores[1:], runs[1:])},
                   "parallelism": "1 GPU"},
        "roofline": r0["roofline"],
        "kernels": r0["kernels"],
    }
    if args.sigma_iters:
        log("[bench] sigma_min of the benchmark's operator")
        light = None
        lpath = os.path.join(os.path.dirname(os.path.abspath(__file__)), "workloads", "m0_light.json")
        if os.path.exists(lpath):
            with open(lpath) as f:
                light = json.load(f).get(args.config)
        sg = sigma_leg(B, g, cfg, args, stores[0], b, light)
        out["sigma_min_measured"] = sg["value"]
        out["config"]["sigma_min"] = sg
        log(f"[bench] sigma_min: {sg}")
    if not args.no_dapply:
        log("[bench] D-apply bandwidth table")
        out["dapply"] = dapply_table(B, g)
        log(f"[bench] D apply: {out['dapply']}")
    if args.baseline_dd:
        log("[bench] the paper's comparison solver (SAP-preconditioned BiCGstab)")
        dd = baseline_dd(B, g, b, args, stores[0])
        dd["amg_speedup"] = round(value / dd["solves_per_s"], 2)
        out["config"]["baseline_dd_bicgstab"] = dd
        log(f"[bench] baseline: {dd}")
    if not args.no_fp64_single:
        log("[bench] 12 sequential FP64 single-RHS solves")
        out["config"]["fp64_single_rhs"] = fp64_single_rhs(B, g, cfg, b, args)
        log(f"[bench] FP64 single-RHS: {out['config']['fp64_single_rhs']}")
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(cfg, L, n_vec, float(outer), float(coarse_per_vcycle),
                                           args.coarse_restart)
    print(json.dumps(out), flush=True)
    g.destroy()
    ctx.close()


if __name__ == "__main__":
    main()
