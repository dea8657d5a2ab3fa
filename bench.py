"""Benchmark of the distillation low-mode-averaging hot path on one MI355X.

Workload (the headline configuration): 24^3 x 48 lattice, synthetic SU(3) links
U = exp(i 0.25 H) (seed 6), Wilson-clover kappa = 0.121, c_sw = 1.2, source
timeslice t' = 0; 128 distillation right-hand sides (N = 32 Laplacian modes x 4
spins) and 64 noise right-hand sides (8 Z2 wall sources x 4 spins x {eta,
(1 - box) eta}); every right-hand side solved to a true FP64 relative residual
of 1e-10.

One step = gauge load and clover construction, the Laplacian modes on t', the
sources and the (1 - box) projection of the noise, and the batched solve of all
192 right-hand sides (mixed precision: FP16-stored links/spinors, FP32 inner CG,
FP64 defect correction).  The metric is right-hand sides solved per second.
Sources and fields are resident in GPU memory before the timed region.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RHS solved/s to 1e-10 at 24^3x48 + Dslash HBM GB/s vs peak; mixed vs FP64"
HBM_PEAK_GBS = 8000.0
NXCD = 8  # accelerator complex dies of an MI355X
DIMS = (48, 24, 24, 24)
EPS, SEED, KAPPA, CSW = 0.25, 6, 0.121, 1.2
T0, NEV, NNOISE, TOL = 0, 32, 8, 1e-10
# stencil kernel classes timed by the library (include/dlma.h, dlma_profile_read) and the
# template parameters (kind, flags) of the hop_kernel instantiation each one is
KCLASS = {0: "hop_k1 (odd sites: y = A_oo^-1 D_oe x)",
          1: "hop_k1_dag (odd sites: y = A_oo^-1 D_oe g5 x)",
          2: "hop_k2_dag (even sites: w = A_ee x - g5 D_eo y, with |w|^2)",
          3: "hop_k2_cg (even sites: q = A_ee w - D_eo y fused with r -= alpha q, x += alpha w, |r|^2)",
          4: "hop_k2 (even sites: z = A_ee x - D_eo y)",
          8: "hop_k2_dotr (even sites: v = A_ee p - D_eo y with (rh, v))",
          9: "hop_k2_dotx (even sites: t = A_ee s - D_eo y with (t, s) and |t|^2)"}
KTEMPLATE = {0: (0, 0), 1: (0, 1), 2: (1, 6), 3: (1, 8), 4: (1, 0), 8: (1, 512), 9: (1, 256)}


def ktemplate(kc, prec):
    """(kind, flags) of a class's hop_kernel: FP16 BiCGStab's K2 for t also forms (rh, t) (flag 1024)."""
    if kc == 9 and prec == "mix_fp16":
        return (1, 256 | 1024)
    return KTEMPLATE[kc]
PREC_ID = {"fp64": 0, "mix_fp32": 1, "mix_fp16": 2, "mix_bf16": 3}
HOP_SOURCES = ["paper_2201_09729_amd/csrc/hop.h", "paper_2201_09729_amd/csrc/hop16.h", "paper_2201_09729_amd/csrc/common.h",
               "paper_2201_09729_amd/csrc/hop_inst.h"]


def pair_bytes(prec):
    return {"fp64": 16, "mix_fp32": 8, "mix_fp16": 4, "mix_bf16": 4}[prec]


def spinor_bytes(prec):
    """bytes of one half-lattice spinor per site: 12 complex pairs (+ the FP16 site scale)"""
    return 12 * pair_bytes(prec) + (4 if prec == "mix_fp16" else 0)


def hop_bytes_split(prec, kind, flags, dims):
    """Algorithmic HBM bytes of one stencil launch: (per launch, per active right-hand side).
    Links (all 8 per output site) and the clover block of the output parity are read once;
    each right-hand side streams its spinor passes once (inputs, outputs, fused vectors).
    BiCGStab's shadow residual, read by K2 with (rh, v), is one field shared by all of them."""
    vh = dims[0] * dims[1] * dims[2] * dims[3] // 2
    pb = pair_bytes(prec)
    fixed = vh * (72 * pb + (0 if (kind == 1 and flags & 32) else 36 * pb))
    if kind == 1 and flags & (512 | 1024):  # the shared shadow residual
        fixed += vh * spinor_bytes(prec)
    if kind == 0:
        passes = 2 + (1 if flags & 64 else 0) + (1 if flags & 128 else 0)
    else:
        passes = 6 if flags & 8 else 3 + (1 if flags & 16 else 0)
    return fixed, vh * passes * spinor_bytes(prec)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sources_sha():
    h = hashlib.sha256()
    for f in HOP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="mix_fp16")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-variants", action="store_true", help="skip the FP64 / BF16 / single-RHS comparisons")
    ap.add_argument("--copy-probe", action="store_true", help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--prof-steps", type=int, default=1,
                    help="extra steps run with per-launch HIP events for the kernel-class times")
    ap.add_argument("--inner-solver", type=int, default=1, choices=(0, 1),
                    help="Krylov method of the inner solves: 1 = BiCGStab on Dhat, 0 = CG on Dhat Dhat^dag")
    ap.add_argument("--rhs-block", type=int, default=None,
                    help="right-hand sides per thread in the stencil kernels (0 = autotune; default 2, 1 for fp64)")
    ap.add_argument("--summarize", nargs="+", metavar="DIR",
                    help="write profiles/ summaries from rocprofv3 output directories and exit: TRACE_DIR "
                         "FETCH_DIR WRITE_DIR [COUNTER_DIR] (COUNTER_DIR: the run with SQ_INSTS_VALU, "
                         "SQ_ACTIVE_INST_VALU, SQ_BUSY_CYCLES, SQ_WAVES, SQ_INSTS_VMEM, GRBM_GUI_ACTIVE, "
                         "TA_TA_BUSY_sum, TD_TD_BUSY_sum, TCC_HIT_sum, TCC_MISS_sum)")
    ap.add_argument("--profile-cmd", default="", help="command line recorded in the summaries")
    ap.add_argument("--lap-scaling", action="store_true",
                    help="Laplacian eigensolver cost vs number of modes on a 64x32^3 lattice (matvec / "
                         "orthogonalisation / Ritz split), instead of the headline benchmark")
    ap.add_argument("--lap-nev", default="20,40,80,160,320", help="modes per timeslice for --lap-scaling")
    ap.add_argument("--lap-nt", type=int, default=16, help="timeslices per eigensolver call for --lap-scaling")
    ap.add_argument("--lap-variants", default="chebyshev,thick_restart,block",
                    help="eigensolver variants for --lap-scaling (chebyshev, thick_restart, block)")
    ap.add_argument("--dist-noise", type=int, default=64, help="Z2 noise vectors of C for --dist-scan")
    ap.add_argument("--dist-scan", action="store_true",
                    help="C_dist / C against the number of Laplacian modes N on 16^3x32 with the cost-model "
                         "relation of the paper evaluated on measured GPU times, instead of the headline benchmark")
    args = ap.parse_args()
    if args.rhs_block is None:
        args.rhs_block = 1 if args.prec == "fp64" else 2
    if args.summarize:
        summarize(args)
        return
    if args.lap_scaling:
        lap_scaling(args)
        return
    if args.dist_scan:
        dist_scan(args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs the whole hot path on a single MI355X "
              "and has no multi-GPU sharding.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2201_09729_amd import dlma, synth

    dlma.load_library()
    dev = "cuda"
    T = DIMS[0]
    t_setup = time.time()
    U = torch.from_numpy(synth.gauge_field(DIMS, EPS, SEED)).to(dev)
    v0 = torch.from_numpy(synth.gaussian_start(DIMS, T, 600 + SEED)).to(dev)
    xi = torch.from_numpy(synth.z2_noise(DIMS, T0, NNOISE, 1000 + SEED)).to(dev)
    nd, nn = 4 * NEV, 4 * NNOISE
    nrhs = nd + 2 * nn
    b = torch.zeros((nrhs,) + DIMS + (4, 3), dtype=torch.complex128, device=dev)
    x = torch.zeros_like(b)
    log("setup: fields on the GPU in %.1f s" % (time.time() - t_setup))
    if not args.no_variants:  # measured copy peak, before the solves fill the library's memory pool
        copy_torch = copy_peak(torch, dev)
        copy_gbs = dlma.dlma_bench_copy(1 << 31, 10)
        log("measured 2 GiB stream copy: %.0f GB/s (library kernel), %.0f GB/s (torch copy_)" % (copy_gbs, copy_torch))

    def step(prec, timed_stats=None):
        g = dlma.dlma_load_gauge(U, KAPPA, CSW)                       # gauge ingest, clover, A_oo^-1
        V, ev = dlma.dlma_lap_eigs(g, NEV, T0, 1, v0[T0:T0 + 1],      # Laplacian modes on t' (block variant:
                                   block_size=min(64, NEV + 24))       # one timeslice leaves Lanczos latency-bound)
        b[:, T0].zero_()                                              # b is zero off t' (allocated so)
        for s in range(4):                                            # spin-diluted sources
            b[s:nd:4, T0, ..., s, :] = V[0]
            b[nd + s:nd + nn:4, T0, ..., s, :] = xi
        dlma.dlma_project(g, T0, V[0], b[nd:nd + nn], 1, out=b[nd + nn:])  # (1 - box(t')) eta
        opts = dlma.default_opts(tol=TOL, prec=prec, rhs_block=args.rhs_block, inner_solver=args.inner_solver)
        xs, st = dlma.dlma_solve([g], [b], xs=[x], opts=opts)
        if timed_stats is not None:
            timed_stats.append(st)
        return g, V, st

    # ------------------------------------------------------------ timed region
    for w in range(args.warmup):
        t = time.time()
        step(args.prec)
        torch.cuda.synchronize()
        log("warmup %d: %.3f s" % (w, time.time() - t))
    # the timed steps run the product path as a caller gets it: per-launch timing off,
    # so the inner iterations are replayed from hipGraphs
    stats = []
    torch.cuda.synchronize()
    t_start = time.time()
    for k in range(args.steps):
        step(args.prec, stats)
        log("step %d done at %.3f s" % (k, time.time() - t_start))
    torch.cuda.synchronize()
    elapsed = time.time() - t_start
    ms_per_step = 1e3 * elapsed / args.steps
    value = nrhs * args.steps / elapsed
    for st in stats:
        assert all(s["converged"] and s["relres"] <= TOL for s in st), "not every right-hand side converged"
    st = stats[-1]
    iters = [s["inner_iters"] for s in st]
    outer = [s["outer"] for s in st]
    log("headline: %.2f RHS/s, %.1f ms/step, inner iterations %d..%d, outer passes %d..%d"
        % (value, ms_per_step, min(iters), max(iters), min(outer), max(outer)))
    # kernel timing: the same step again with every stencil launch bracketed by HIP events
    # on its stream (direct launches: events around single kernels need them)
    dlma.dlma_profile_reset()
    dlma.dlma_profile_enable(True)
    pstats = []
    torch.cuda.synchronize()
    t = time.time()
    for k in range(args.prof_steps):
        step(args.prec, pstats)
    torch.cuda.synchronize()
    prof_ms_per_step = 1e3 * (time.time() - t) / args.prof_steps
    dlma.dlma_profile_enable(False)
    prof = {kc: dlma.dlma_profile_read(kc) for kc in KCLASS}
    log("profiled steps (direct launches, per-launch events): %.1f ms/step" % prof_ms_per_step)

    # dominant stencil kernel of the timed region (HIP events around each launch).  Its
    # algorithmic bytes count only right-hand sides still iterating: a launch reads
    # every link and clover entry once, plus the spinor passes of each active
    # right-hand side; a right-hand side is active in inner_iters launches of each
    # class per inner iteration: one per class, except BiCGStab's K1, which runs for
    # v = Dhat p and for t = Dhat s.
    kc = max(prof, key=lambda k: prof[k][1])
    n_l, ms_tot, by_all = prof[kc]
    fixed, per_rhs = hop_bytes_split(args.prec, *ktemplate(kc, args.prec), DIMS)
    per_iter = 2 if (args.inner_solver == 1 and kc == 0) else 1  # BiCGStab applies K1 twice per iteration
    rhs_launches = per_iter * sum(s["inner_iters"] for stp in pstats for s in stp)
    by_tot = n_l * fixed + rhs_launches * per_rhs
    achieved = by_tot / (ms_tot * 1e-3) / 1e9
    roofline = {"kernel": KCLASS[kc], "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "launches": n_l, "avg_launch_ms": round(ms_tot / max(n_l, 1), 4),
                "alg_bytes_per_launch": round(by_tot / max(n_l, 1)),
                "active_rhs_per_launch": round(rhs_launches / max(n_l, 1), 1),
                "bytes_model": "Vh*(72 b_pair links + 36 b_pair clover) per launch [+ Vh*(12 b_pair [+4]) for the "
                               "shared BiCGStab shadow residual read by K2 with (rh, v)] + Vh*passes*(12 b_pair "
                               "[+4 FP16 scale]) per active RHS; passes = %d" % round(
                                   per_rhs / (DIMS[0] * DIMS[1] * DIMS[2] * DIMS[3] // 2) / spinor_bytes(args.prec)),
                "timing": "HIP events around every launch of this class on its stream, in %d extra step(s) of the "
                          "same workload run with direct launches (%.1f ms/step); the timed steps replay hipGraphs "
                          "and carry no per-launch events" % (args.prof_steps, prof_ms_per_step)}
    tfile = os.path.join(ROOT, "profiles", "traffic_%s.json" % KCLASS[kc].split()[0])
    if os.path.exists(tfile):
        with open(tfile) as fh:
            tr = json.load(fh)
        if (tr.get("source_sha") == sources_sha() and tr.get("precision") == args.prec
                and tr.get("rhs_block") == args.rhs_block):
            roofline["traffic"] = tr.get("traffic_bytes_per_launch")
            roofline["traffic_note"] = tr.get("note")
            if tr.get("valu_busy_frac") is not None:
                # vector-ALU issue: SQ_INSTS_VALU wave instructions x 4 cycles over the SIMD cycles
                # of the dispatch (1024 SIMDs x GRBM_GUI_ACTIVE), from the committed counter runs
                roofline["issue"] = {"valu_busy_frac": tr["valu_busy_frac"], "derivation": tr.get("valu_note")}

    out = {"metric": METRIC, "value": round(value, 3), "unit": "RHS/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 2), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32" if args.prec != "fp64" else "f64", "data": "synthetic",
           "config": {"workload": "24^3x48 Wilson-clover solves, 128 distillation + 64 Z2-noise RHS to rel. residual 1e-10",
                      "lattice": "24^3x48", "eps": EPS, "seed": SEED, "kappa": KAPPA, "csw": CSW, "t_src": T0,
                      "nev": NEV, "nnoise": NNOISE, "nrhs": nrhs,
                      "precision": {"mix_fp16": "FP16 storage (FP32 scale per site), FP32 arithmetic, FP64 defect correction",
                                    "mix_bf16": "BF16 storage, FP32 arithmetic, FP64 defect correction",
                                    "mix_fp32": "FP32 storage and arithmetic, FP64 defect correction",
                                    "fp64": "FP64 everywhere"}[args.prec],
                      "inner_solver": "BiCGStab on the even-odd operator" if args.inner_solver == 1
                      else "CG on the even-odd normal equations",
                      "step": "gauge load + clover + Laplacian modes on t' + sources + projection + batched solve"},
           "roofline": roofline,
           "iterations": {"inner_min": min(iters), "inner_max": max(iters), "outer_max": max(outer)},
           "profiled_ms_per_step": round(prof_ms_per_step, 2),
           "kernel_classes": {KCLASS[k].split()[0]: {"launches": prof[k][0], "total_ms": round(prof[k][1], 3),
                                                     "GBps": round(prof[k][2] / max(prof[k][1], 1e-9) / 1e6, 1)}
                              for k in prof if prof[k][0] > 0}}

    # ------------------------------------------------------------ comparisons (outside the timed region)
    if not args.no_variants:
        var = {}
        g, V, _ = step(args.prec)
        for prec in ("fp64", "mix_fp16", "mix_bf16", "mix_fp32"):
            # one short capped solve first, so the RHS-block autotuner's search is not timed
            dlma.dlma_solve([g], [b], xs=[x], opts=dlma.default_opts(tol=TOL, prec=prec, maxiter=8, max_outer=1,
                                                                     inner_solver=args.inner_solver),
                            allow_notconv=True)
            torch.cuda.synchronize()
            t = time.time()
            (xx,), st2 = dlma.dlma_solve([g], [b], xs=[x], opts=dlma.default_opts(tol=TOL, prec=prec,
                                                                                  inner_solver=args.inner_solver))
            torch.cuda.synchronize()
            dt = time.time() - t
            var[prec] = {"rhs_per_s": round(nrhs / dt, 3), "solve_s": round(dt, 3),
                         "inner_iters_max": max(s["inner_iters"] for s in st2),
                         "max_relres": max(s["relres"] for s in st2)}
            log("variant %s: %.2f RHS/s (batched solve only)" % (prec, nrhs / dt))
        # plain single-RHS FP64 even-odd CG (CG on the normal equations), one right-hand
        # side at a time (sample of 4)
        sample = [0, 1, nd, nd + nn]
        single = dict(tol=TOL, prec="fp64", rhs_block=1, inner_solver=0)
        # autotuning for one right-hand side, outside the timing
        dlma.dlma_solve([g], [b[:1]], xs=[x[:1]], opts=dlma.default_opts(maxiter=8, max_outer=1, **single),
                        allow_notconv=True)
        torch.cuda.synchronize()
        t = time.time()
        for i in sample:
            dlma.dlma_solve([g], [b[i:i + 1]], xs=[x[i:i + 1]], opts=dlma.default_opts(**single))
        torch.cuda.synchronize()
        dt = (time.time() - t) / len(sample)
        var["fp64_single_rhs"] = {"rhs_per_s": round(1.0 / dt, 3), "sample": "4 right-hand sides solved one at a time"}
        out["variants"] = var
        out["speedup_vs_fp64_single_rhs"] = round(value * dt, 2)
        log("fp64 single-RHS baseline: %.2f RHS/s; headline speedup %.1fx" % (1.0 / dt, value * dt))
        # Dslash (Schur operator) bandwidth per precision and right-hand sides
        dsl = {"copy_peak_GBps": round(copy_gbs, 1), "torch_copy_GBps": round(copy_torch, 1),
               "note": "frac_hbm against 8 TB/s, frac_copy against the measured 2 GiB stream copy (dlma_bench_copy)"}
        for prec in ("fp64", "mix_fp32", "mix_fp16", "mix_bf16"):
            for n in (1, 8, 16, 32, 64, 128):
                ms, by = dlma.dlma_bench_schur(g, prec, n, 0, 10)
                dsl["%s_n%d" % (prec, n)] = {"ms_per_apply": round(ms, 4), "GBps": round(by / ms / 1e6, 1),
                                             "frac_hbm": round(by / ms / 1e6 / HBM_PEAK_GBS, 4),
                                             "frac_copy": round(by / ms / 1e6 / copy_gbs, 4)}
            log("Schur operator %s: %s" % (prec, ", ".join("n=%d %.2f" % (n, dsl["%s_n%d" % (prec, n)]["frac_hbm"])
                                                          for n in (1, 8, 16, 32, 64, 128))))
        out["dslash"] = dsl
        # off the timed metric: Laplacian modes on every timeslice and the correlators
        torch.cuda.synchronize()
        t = time.time()
        Vall, _ = dlma.dlma_lap_eigs(g, NEV, 0, T, v0)
        torch.cuda.synchronize()
        t_lap = time.time() - t
        t = time.time()
        C = dlma.dlma_correlators(g, T0, Vall, x[:nd], x[nd:nd + nn], x[nd + nn:])
        t_cor = time.time() - t
        out["off_metric"] = {"lap_eigs_all_timeslices_s": round(t_lap, 3), "correlators_s": round(t_cor, 3),
                             "C_dist_over_C_PS_delta1": float((C["PS"]["PP_exact"][1] / C["PS"]["11_est"][1]).real)}
        log("Laplacian modes on all %d timeslices: %.2f s; correlators %.2f s" % (T, t_lap, t_cor))
        del Vall

    if not args.no_variants:
        del b, x
        dlma.dlma_release_cache()
        torch.cuda.empty_cache()
        out["uneven_batch"] = uneven_batch(torch, dlma, synth)
        dlma.dlma_release_cache()
        torch.cuda.empty_cache()
        out["correlator_error"] = correlator_error(torch, dlma, synth)
        dlma.dlma_release_cache()
        torch.cuda.empty_cache()

    if args.copy_probe:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        c = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        c.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 2 * a.numel() * 8

    # ------------------------------------------------------------ CPU oracle baseline (after all GPU timing)
    if not args.no_cpu:
        import oracle
        Uh = U.cpu().numpy()
        t = time.time()
        A = oracle.clover(Uh, KAPPA, CSW)
        t_cl = time.time() - t
        src = oracle.noise_sources(xi.cpu().numpy()[:1], T, T0)[:1]
        # bounded sample: one noise right-hand side solved to the headline's tolerance (about
        # 15-30 s of CGLS on the host cores; the oracle checks its true residual itself)
        t = time.time()
        _, its, res, conv = oracle.solve(Uh, A, src, tol=TOL)
        tk = time.time() - t
        assert conv[0] and res[0] <= TOL, (res, its)
        rate = 1.0 / tk
        out["cpu_baseline"] = {"value": round(rate, 6), "unit": "RHS/s", "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": "one spin-diluted Z2 noise right-hand side of the same 24^3x48 workload solved "
                                         "by the oracle's FP64 CGLS (unpreconditioned, C with OpenMP) to true relative "
                                         "residual %.1e in %.1f s (%d iterations, residual %.2e)" % (TOL, tk, its[0], res[0]),
                               "clover_build_s": round(t_cl, 2)}
        log("cpu baseline: %.4g RHS/s (%d threads)" % (rate, oracle.num_threads()))
    print(json.dumps(out), flush=True)


def copy_peak(torch, dev, nbytes=1 << 31, reps=10):
    """Measured stream bandwidth: a 2 GiB device-to-device copy, read + write bytes per second."""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    c = torch.empty_like(a)
    c.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        c.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, c
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def uneven_batch(torch, dlma, synth):
    """The uneven batch in one solve: 3 x 12^3x24 (seeds 1-3), 2 x 16^3x32 (seeds 4, 5) and
    1 x 24^3x48 (seed 6), eps 0.25, kappa cycling 0.119, 0.120, 0.121, c_sw 1.2; per
    configuration 4N distillation sources plus as many Z2 noise sources (N_r x 4 spins x
    {eta, (1 - box) eta}): 256, 128 and 64 right-hand sides for the three volumes.  BF16
    storage, FP32 inner BiCGStab, FP64 defect correction to 1e-10; every launch covers every
    configuration.  The autotuner runs in an untimed capped solve first."""
    shapes = [(24, 12, 12, 12)] * 3 + [(32, 16, 16, 16)] * 2 + [(48, 24, 24, 24)]
    kappas = [0.119, 0.120, 0.121, 0.119, 0.120, 0.121]
    nevs = {24: 32, 32: 16, 48: 8}
    gs, bs = [], []
    for i, dims in enumerate(shapes):
        seed = i + 1
        T = dims[0]
        nev = nevs[T]
        nn = nev // 2  # noise vectors: 4 spins x {eta, (1 - box) eta} each, as many RHS as the distillation ones
        U = torch.from_numpy(synth.gauge_field(dims, EPS, seed)).to("cuda")
        g = dlma.dlma_load_gauge(U, kappas[i], CSW)
        V, _ = dlma.dlma_lap_eigs(g, nev, T0, 1, torch.from_numpy(synth.gaussian_start(dims, 1, 600 + seed)).to("cuda"),
                                  block_size=min(64, nev + max(8, nev // 2)))
        eta = dlma.noise_sources(torch.from_numpy(synth.z2_noise(dims, T0, nn, 1000 + seed)).to("cuda"), T, T0)
        bs.append(torch.cat([dlma.dist_sources(V[0], T, T0), eta, dlma.dlma_project(g, T0, V[0], eta, 1)]))
        gs.append(g)
        del U, V, eta
    xs = [torch.zeros_like(b) for b in bs]
    nrhs = sum(b.shape[0] for b in bs)
    dlma.dlma_solve(gs, bs, xs=xs, opts=dlma.default_opts(tol=TOL, prec="mix_bf16", maxiter=8, max_outer=1),
                    allow_notconv=True)
    torch.cuda.synchronize()
    t = time.time()
    xs, st = dlma.dlma_solve(gs, bs, xs=xs, opts=dlma.default_opts(tol=TOL, prec="mix_bf16"))
    torch.cuda.synchronize()
    dt = time.time() - t
    assert all(s["converged"] and s["relres"] <= TOL for s in st)
    res = {"configs": "3 x 12^3x24 (256 RHS each), 2 x 16^3x32 (128 each), 1 x 24^3x48 (64)",
           "nrhs": nrhs, "precision": "BF16 storage, FP32 arithmetic, FP64 defect correction",
           "solve_s": round(dt, 3), "rhs_per_s": round(nrhs / dt, 2),
           "site_rhs_per_s": round(sum(b.shape[0] * int(np.prod(b.shape[1:5])) for b in bs) / dt, 1),
           "inner_iters_max": max(s["inner_iters"] for s in st), "outer_max": max(s["outer"] for s in st),
           "max_relres": max(s["relres"] for s in st)}
    log("uneven batch: %d RHS over 6 configurations in %.2f s (%.1f RHS/s)" % (nrhs, dt, nrhs / dt))
    del gs, bs, xs
    return res


def tslice_norms(torch, f):
    """[n][T] 2-norms of each field per timeslice."""
    return torch.sqrt((f.abs() ** 2).sum(dim=(2, 3, 4, 5, 6)))


def correlator_error(torch, dlma, synth, dims=(32, 16, 16, 16), seed=3, nev=32, nnoise=8):
    """Correlator error of the mixed-precision solves against FP64 solves, per timeslice (paper
    eqs. (2)-(4): every piece dlma_correlators returns), on 16^3 x 32 (eps 0.25, kappa 0.121,
    c_sw 1.2, seed 3): N = 32 modes on every timeslice, 128 distillation right-hand sides and
    8 Z2 noise vectors (32 eta + 32 (1 - box) eta), solved in FP64 (to 1e-12), MIX_FP16 and
    MIX_BF16 (to 1e-10).  For each piece, Gamma and precision: the largest relative error
    |dC(t)| / |C(t)| over t, and the largest ratio of |dC(t)| to its bound
      (1/N_r) sum_r [|dY_r|_t |phi_r|_t + |Y_r|_t |dphi_r|_t + |dY_r|_t |dphi_r|_t]
    (Cauchy-Schwarz with |X_t| <= 1 and unit-modulus Gamma g5 entries; Y the source-side
    solution of the piece, d the difference of the mixed solution from the FP64 one, norms
    over timeslice t and the four spins of a group)."""
    T = dims[0]
    U = torch.from_numpy(synth.gauge_field(dims, EPS, seed)).to("cuda")
    g = dlma.dlma_load_gauge(U, KAPPA, CSW)
    Vall, _ = dlma.dlma_lap_eigs(g, nev, 0, T, torch.from_numpy(synth.gaussian_start(dims, T, 600 + seed)).to("cuda"))
    eta = dlma.noise_sources(torch.from_numpy(synth.z2_noise(dims, T0, nnoise, 1000 + seed)).to("cuda"), T, T0)
    b = torch.cat([dlma.dist_sources(Vall[T0], T, T0), eta, dlma.dlma_project(g, T0, Vall[T0], eta, 1)])
    nd, nn = 4 * nev, 4 * nnoise
    sol, C = {}, {}
    for prec, tol in (("fp64", 1e-12), ("mix_fp16", TOL), ("mix_bf16", TOL)):
        (x,), st = dlma.dlma_solve([g], [b], opts=dlma.default_opts(tol=tol, prec=prec))
        assert all(s_["converged"] for s_ in st)
        sol[prec] = x
        C[prec] = dlma.dlma_correlators(g, T0, Vall, x[:nd], x[nd:nd + nn], x[nd + nn:])
    ref = sol["fp64"]
    # (sink solution, source-side solution, number of averaged groups) of every piece
    parts = {"QQ_est": ("phi", "phibar", nnoise), "PQ_est": ("phi", "phibar", nnoise),
             "QP_est": ("phi", "phiP", nnoise), "PP_est": ("phi", "phiP", nnoise), "11_est": ("phi", "phi", nnoise),
             "PP_exact": ("dist", "dist", 1), "QP_exact": ("dist", "dist", 1)}

    def fields(x):
        return {"dist": x[:nd], "phi": x[nd:nd + nn], "phibar": x[nd + nn:], "phiP": x[nd:nd + nn] - x[nd + nn:]}

    def group_norms(f):  # [groups][T]: norm over the four spins of each group, per timeslice
        n = tslice_norms(torch, f)
        return torch.sqrt((n.reshape(-1, 4, T) ** 2).sum(dim=1))

    fr = fields(ref)
    nref = {k: group_norms(v) for k, v in fr.items()}
    out = {}
    for prec in ("mix_fp16", "mix_bf16"):
        fm = fields(sol[prec])
        nd_ = {k: group_norms(fm[k] - fr[k]) for k in fr}
        eps_x = float((torch.linalg.vector_norm((sol[prec] - ref).reshape(ref.shape[0], -1), dim=1)
                       / torch.linalg.vector_norm(ref.reshape(ref.shape[0], -1), dim=1)).max())
        rp = {"solution_rel_err_max": eps_x}
        for gname in ("PS", "V"):
            for part, (xs_, ys_, ngrp) in parts.items():
                c0 = np.asarray(C["fp64"][gname][part])
                dc = np.abs(np.asarray(C[prec][gname][part]) - c0)
                bound = ((nd_[ys_] * nref[xs_] + nref[ys_] * nd_[xs_] + nd_[ys_] * nd_[xs_]).sum(dim=0)
                         / ngrp).cpu().numpy()
                rel = dc / np.maximum(np.abs(c0), 1e-300)
                rp["%s_%s" % (gname, part)] = {"max_rel": float(rel.max()),  # time index is Delta = t - t'
                                               "rel_at_delta_0_1_8_16": [float(rel[d]) for d in (0, 1, 8, 16)],
                                               "max_err_over_bound": float((dc / np.maximum(bound, 1e-300)).max())}
        out[prec] = rp
        worst = max(v["max_rel"] for k, v in rp.items() if isinstance(v, dict))
        wb = max(v["max_err_over_bound"] for k, v in rp.items() if isinstance(v, dict))
        log("correlator error %s vs fp64 (16^3x32): max relative %.2e, max error/bound %.2e, solution error %.2e"
            % (prec, worst, wb, eps_x))
    del sol, b, Vall
    return {"lattice": "16^3x32", "eps": EPS, "seed": seed, "kappa": KAPPA, "csw": CSW, "nev": nev,
            "noise_vectors": nnoise, "nrhs": nd + 2 * nn, "reference": "FP64 solves to 1e-12", **out}


def lap_scaling(args):
    """Cost of the Laplacian modes of every timeslice against the number of modes N,
    split into applications of the operator, orthogonalisation and Ritz extraction
    (the quantities of the paper's Table 2, on a synthetic field of the paper's
    lattice size 64 x 32^3).  One JSON line per N on stdout."""
    import torch
    from paper_2201_09729_amd import dlma, synth
    dims = (64, 32, 32, 32)
    T = dims[0]
    dlma.load_library()
    t = time.time()
    U = torch.from_numpy(synth.gauge_field(dims, 0.2, 5)).to("cuda")
    g = dlma.dlma_load_gauge(U, 0.1215, 1.3)
    v0 = torch.from_numpy(synth.gaussian_start(dims, T, 605)).to("cuda")
    log("setup %.1f s" % (time.time() - t))
    paper = {20: (46.3, 3.5, 31.1), 40: (104.0, 10.8, 68.7), 80: (243.0, 41.8, 152.0), 160: (777.0, 251.0, 346.0),
             320: (2140.0, 1140.0, 740.0)}
    nevs = [int(x) for x in args.lap_nev.split(",")]
    variants = [v for v in args.lap_variants.split(",") if v]
    for variant in variants:
        for nev in nevs:
            nt = max(1, min(args.lap_nt, T))
            # chebyshev: Chebyshev-filtered Lanczos, basis growing to convergence;
            # thick_restart: the same filter with the basis capped at 2N + 32 vectors
            # (restarts keep N + half the rest as Ritz vectors)
            # block: Chebyshev-filtered subspace iteration on N + max(8, N/2) vectors (at most 64)
            cheb = 0
            maxb = 3 * nev + 300 if variant == "chebyshev" else 0
            rb = 2 * nev + 32 if variant == "thick_restart" else 0
            bs = min(64, nev + max(8, nev // 2)) if variant == "block" else 0
            if variant == "block" and bs <= nev:
                log("block nev %d: skipped (the block kernels hold at most 64 vectors)" % nev)
                continue
            dlma.dlma_profile_reset()
            dlma.dlma_profile_enable(True)
            torch.cuda.synchronize()
            t = time.time()
            for t0 in range(0, T, nt):
                V, ev = dlma.dlma_lap_eigs(g, nev, t0, min(nt, T - t0), v0[t0:t0 + nt], tol=1e-10,
                                           max_basis=maxb, cheb_degree=cheb, restart_basis=rb, block_size=bs)
                del V
            torch.cuda.synchronize()
            wall = time.time() - t
            dlma.dlma_profile_enable(False)
            ph = {name: dlma.dlma_profile_read(kc) for name, kc in (("matvec", 5), ("ortho", 6), ("ritz", 7))}
            row = {"lattice": "64x32^3", "timeslices": T, "nev": nev, "variant": variant, "basis_cap": rb or maxb or bs,
                   "wall_s": round(wall, 3),
                   "matvec_s": round(ph["matvec"][1] / 1e3, 3), "ortho_s": round(ph["ortho"][1] / 1e3, 3),
                   "ritz_s": round(ph["ritz"][1] / 1e3, 3), "lanczos_steps_per_call": ph["ortho"][0] // max(1, -(-T // nt)),
                   "matvec_GBps": round(ph["matvec"][2] / max(ph["matvec"][1], 1e-9) / 1e6, 1),
                   "ortho_GBps": round(ph["ortho"][2] / max(ph["ortho"][1], 1e-9) / 1e6, 1)}
            if nev in paper and variant == "chebyshev":
                row["paper_table2_s"] = {"total": paper[nev][0], "ortho": paper[nev][1], "matvec": paper[nev][2],
                                         "note": "E5 configuration, PRIMME on the authors' (unstated) cluster; context only"}
            print(json.dumps(row), flush=True)
            log("%s nev %d: %.2f s (matvec %.2f, ortho %.2f, ritz %.2f)" % (variant, nev, wall, row["matvec_s"],
                                                                             row["ortho_s"], row["ritz_s"]))


def dist_scan(args):
    """How much of the correlator the distillation part carries, against N, and what
    the stochastic part would have to cost for the method to pay off (paper Sec. 3,
    Figs. 3-5 and the cost relations of eqs. 6-9), on the synthetic 16^3 x 32 field
    (eps 0.25, seed 3, kappa 0.121, c_sw 1.2), source timeslice 0.

    C is the one-end estimate of the full correlator from --dist-noise Z2 noise vectors
    (spin-diluted: 4 solves each; 64 by default, so that its own noise stays below the
    ratios at the larger distances); C_dist(N) is exact from the perambulator of the
    first N modes.  The cost relation takes R_1 = 32 stochastic solves (8 vectors x 4
    spins, as in the headline workload).  Times are
    measured on the GPU: t_lap(N) (modes of every timeslice), the per-right-hand-side
    time of the batched mixed-precision solve, from which t_{N,D} = 4N * t_rhs and
    t_{R,D} = R * t_rhs.  Equal cost, eq. (6): R_0 = (t_lap + t_{N,D}) / t_rhs + 2 R_1
    stochastic solves; the method pays off only if 1 - C_dist/C <= R_1 / R_0 (eq. 9)."""
    import torch
    from paper_2201_09729_amd import dlma, synth
    dims = (32, 16, 16, 16)
    T = dims[0]
    t0, nnoise = 0, args.dist_noise
    nlist = [8, 16, 32, 64, 128]
    nmax = max(nlist)
    dlma.load_library()
    U = torch.from_numpy(synth.gauge_field(dims, 0.25, 3)).to("cuda")
    g = dlma.dlma_load_gauge(U, 0.121, 1.2)
    v0 = torch.from_numpy(synth.gaussian_start(dims, T, 603)).to("cuda")
    t_lap = {}
    Vall = None
    for nev in nlist:
        torch.cuda.synchronize()
        t = time.time()
        V, _ = dlma.dlma_lap_eigs(g, nev, 0, T, v0)
        torch.cuda.synchronize()
        t_lap[nev] = time.time() - t
        if nev == nmax:
            Vall = V
        else:
            del V
        log("modes N = %d on all %d timeslices: %.2f s" % (nev, T, t_lap[nev]))
    xi = torch.from_numpy(synth.z2_noise(dims, t0, nnoise, 1003)).to("cuda")
    eta = dlma.noise_sources(xi, T, t0)
    b = torch.cat([dlma.dist_sources(Vall[t0], T, t0), eta])
    opts = dlma.default_opts(tol=TOL, prec="mix_fp16")
    # autotuning (keyed on the right-hand-side count) and warm-up outside the timing
    dlma.dlma_solve([g], [b], opts=dlma.default_opts(tol=TOL, prec="mix_fp16", max_outer=1), allow_notconv=True)
    torch.cuda.synchronize()
    t = time.time()
    (x,), st = dlma.dlma_solve([g], [b], opts=opts)
    torch.cuda.synchronize()
    t_rhs = (time.time() - t) / b.shape[0]
    assert all(s_["converged"] for s_ in st)
    log("batched solve of %d right-hand sides: %.3f ms per right-hand side" % (b.shape[0], 1e3 * t_rhs))
    nd = 4 * nmax
    R1 = 32  # stochastic solves (spin-diluted) of one estimate in the cost relation
    rows = []
    for nev in nlist:
        C = dlma.dlma_correlators(g, t0, Vall[:, :nev].contiguous(), x[:4 * nev], x[nd:], x[nd:])
        tND = 4 * nev * t_rhs
        R0 = (t_lap[nev] + tND) / t_rhs + 2 * R1
        row = {"lattice": "16^3x32", "N_modes": nev, "N_solves": 4 * nev, "R1_solves": R1,
               "t_lap_s": round(t_lap[nev], 3), "t_ND_s": round(tND, 3), "t_rhs_ms": round(1e3 * t_rhs, 3),
               "R0_equal_cost": round(R0, 1), "payoff_bound_R1_over_R0": round(R1 / R0, 4)}
        for name in ("PS", "V"):
            full = C[name]["11_est"].real
            dist = C[name]["PP_exact"].real
            row["%s_Cdist_over_C" % name] = [round(float(dist[d] / full[d]), 4) for d in range(1, T // 2 + 1)]
            row["%s_one_minus_ratio_le_bound" % name] = [bool(1 - dist[d] / full[d] <= R1 / R0) for d in range(1, T // 2 + 1)]
        rows.append(row)
        print(json.dumps(row), flush=True)
        log("N = %d: C_dist/C (PS) at Delta = 1, 4, 8, 16: %s; R_0 = %.0f" % (
            nev, [row["PS_Cdist_over_C"][d - 1] for d in (1, 4, 8, 16)], R0))


def summarize(args):
    """rocprofv3 CSVs -> profiles/: per-kernel time summary and HBM traffic of the
    stencil kernels, with FETCH_SIZE / WRITE_SIZE scaled by what the counters read for
    the 1 GiB device copy of --copy-probe (kernel __amd_rocclr_copyBuffer).  The
    per-class averages and counters cover the timed step only: the dispatches after
    its gauge load (the last k_pack_links), so that the autotuner's and the warm-up's
    launches of the same kernels do not enter them."""
    import csv
    import collections
    trace, fetch, write = args.summarize[:3]
    cdir = args.summarize[3] if len(args.summarize) > 3 else None
    prec = args.prec

    def find(d, suffix):
        for f in sorted(os.listdir(d)):
            if f.endswith(suffix):
                return os.path.join(d, f)
        raise FileNotFoundError(suffix)

    stats = list(csv.DictReader(open(find(trace, "kernel_stats.csv"))))

    def timed_step(rows):
        rows = sorted(rows, key=lambda r: int(r["Start_Timestamp"]))
        starts = [i for i, r in enumerate(rows) if "k_pack_links" in r["Kernel_Name"]]
        return rows[starts[-1]:] if starts else rows

    step_ms = collections.defaultdict(list)
    for r in timed_step(list(csv.DictReader(open(find(trace, "kernel_trace.csv"))))):
        step_ms[r["Kernel_Name"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6)
    counters = {}
    copy_ref = {}
    for name, d in (("FETCH_SIZE", fetch), ("WRITE_SIZE", write)):
        agg = collections.defaultdict(list)
        for row in timed_step(list(csv.DictReader(open(find(d, "counter_collection.csv"))))):
            agg[row["Kernel_Name"]].append(float(row["Counter_Value"]))
        counters[name] = agg
        # the calibration copy is the last device copy of the run (bench.py --copy-probe)
        cp = [r for r in csv.DictReader(open(find(d, "counter_collection.csv"))) if "copyBuffer" in r["Kernel_Name"]]
        cp.sort(key=lambda r: int(r["Dispatch_Id"]))
        copy_ref[name] = float(cp[-1]["Counter_Value"]) if cp else None
    copy_kib = (1 << 30) / 1024.0  # the probe reads and writes 1 GiB
    scale = {k: (copy_kib / v if v else None) for k, v in copy_ref.items()}
    pid = PREC_ID[prec]

    def hop_name(kc, nb):
        """The full kernel name of the class as rocprofv3 prints it (matched on the
        template arguments, whatever the parameter list)."""
        kind, fl = ktemplate(kc, prec)
        head = "void dlma::hop_kernel<%d, %d, %d, %d, 128>(" % (pid, nb, kind, fl)
        for nm in step_ms:
            if nm.startswith(head):
                return nm
        return head

    by_name = {r["Name"]: r for r in stats}
    nb = args.rhs_block
    lines = ["# Stencil kernels, 24^3x48 headline step (%s, %d right-hand sides per thread)" % (prec, nb), "",
             "Command: `%s`" % args.profile_cmd, "",
             "## rocprofv3 --kernel-trace --stats (top kernels)", "",
             "| kernel | calls | total ms | avg ms |", "|---|---|---|---|"]
    for r in stats[:14]:
        lines.append("| `%s` | %s | %.2f | %.4f |" % (r["Name"][:110], r["Calls"], float(r["TotalDurationNs"]) / 1e6,
                                                  float(r["AverageNs"]) / 1e6))
    lines += ["", "## HBM traffic per dispatch (rocprofv3 --pmc, one counter per run)", "",
              "Copy calibration (1 GiB device copy): FETCH_SIZE reads %.0f KiB (scale %.4f), WRITE_SIZE %.0f KiB (scale %.4f)."
              % (copy_ref["FETCH_SIZE"] or 0, scale["FETCH_SIZE"] or 0, copy_ref["WRITE_SIZE"] or 0, scale["WRITE_SIZE"] or 0), "",
              "Classes below: dispatches of the timed step only (after its gauge load).", "",
              "| class | kernel | dispatches | FETCH KiB | WRITE KiB | scaled traffic GB | avg ms |", "|---|---|---|---|---|---|---|"]
    out = {}
    for kc in KCLASS:
        nm = hop_name(kc, nb)
        f = counters["FETCH_SIZE"].get(nm)
        w = counters["WRITE_SIZE"].get(nm)
        if not f or not w or not step_ms.get(nm):
            continue
        fk, wk = sum(f) / len(f), sum(w) / len(w)
        tb = (fk * scale["FETCH_SIZE"] + wk * scale["WRITE_SIZE"]) * 1024.0
        avg_ms = sum(step_ms[nm]) / len(step_ms[nm])
        lines.append("| %s | `hop_kernel<%d,%d,%d,%d>` | %d | %.0f | %.0f | %.3f | %.4f |"
                     % (KCLASS[kc].split()[0], pid, nb, ktemplate(kc, prec)[0], ktemplate(kc, prec)[1], len(f), fk, wk,
                        tb / 1e9, avg_ms))
        out[kc] = {"kernel": nm, "precision": prec, "rhs_block": nb, "source_sha": sources_sha(),
                   "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk, "copy_scale": scale,
                   "traffic_bytes_per_launch": tb, "avg_ms_rocprof": avg_ms,
                   "note": "FETCH_SIZE and WRITE_SIZE per dispatch scaled by the 1 GiB copy calibration",
                   "command": args.profile_cmd}
    if cdir:
        crows = timed_step(list(csv.DictReader(open(find(cdir, "counter_collection.csv")))))
        cnt = collections.defaultdict(lambda: collections.defaultdict(list))
        for r in crows:
            cnt[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
        # the kernels of the timed step by their total time there
        top = sorted(step_ms, key=lambda k: -sum(step_ms[k]))[:10]
        nsimd, ncu = 1024, 256
        lines += ["", "## Issue and cache counters per dispatch (rocprofv3 --pmc, one run)", "",
                  "Per kernel: averages over its dispatches in the timed step.  VALU issue = SQ_INSTS_VALU x 4 cycles "
                  "(a wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles) / (%d SIMDs x GRBM_GUI_ACTIVE); "
                  "VALU busy = SQ_ACTIVE_INST_VALU / (%d CUs x GRBM_GUI_ACTIVE) (rocprofv3's VALUBusy); TA, TD busy = "
                  "TA_TA_BUSY_sum, TD_TD_BUSY_sum / (%d x GRBM_GUI_ACTIVE); L2 hit = TCC_HIT / (TCC_HIT + TCC_MISS); "
                  "GRBM_GUI_ACTIVE is divided by the %d XCDs it is summed over; clock = those cycles / the "
                  "kernel-trace duration." % (nsimd, ncu, ncu, NXCD), "",
                  "| kernel | ms | clock GHz | VALU issue | VALU busy | TA busy | TD busy | L2 hit | VALU inst/wave | VMEM inst/wave |",
                  "|---|---|---|---|---|---|---|---|---|---|"]
        issue = {}
        for k in top:
            c = {n: sum(v) / len(v) for n, v in cnt.get(k, {}).items()}
            if "GRBM_GUI_ACTIVE" not in c or c["GRBM_GUI_ACTIVE"] <= 0:
                continue
            gui = c["GRBM_GUI_ACTIVE"] / NXCD  # rocprofv3 sums the counter over the XCDs
            ms = sum(step_ms[k]) / len(step_ms[k])
            vi = 4.0 * c.get("SQ_INSTS_VALU", 0) / (nsimd * gui)
            vb = c.get("SQ_ACTIVE_INST_VALU", 0) / (ncu * gui)
            ta = c.get("TA_TA_BUSY_sum", 0) / (ncu * gui)
            td = c.get("TD_TD_BUSY_sum", 0) / (ncu * gui)
            hit = c.get("TCC_HIT_sum", 0)
            miss = c.get("TCC_MISS_sum", 0)
            l2 = hit / (hit + miss) if hit + miss > 0 else float("nan")
            issue[k] = vi
            nw = c.get("SQ_WAVES", None)
            lines.append("| `%s` | %.4f | %.2f | %.3f | %.3f | %.3f | %.3f | %.3f | %s | %s |" % (
                k[:90], ms, gui / (ms * 1e6), vi, vb, ta, td, l2,
                "%.0f" % (c["SQ_INSTS_VALU"] / nw) if nw else "-", "%.0f" % (c["SQ_INSTS_VMEM"] / nw) if nw else "-"))
        for kc, d in out.items():
            if d["kernel"] in issue:
                d["valu_busy_frac"] = round(issue[d["kernel"]], 4)
                d["valu_note"] = ("SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x GRBM_GUI_ACTIVE / 8 XCDs), per dispatch of the timed "
                                  "step (rocprofv3 --pmc; profiles/hop_kernels_24x48_%s.md)" % prec)
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    tag = "24x48_%s" % prec
    with open(os.path.join(ROOT, "profiles", "hop_kernels_%s.md" % tag), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    for kc, d in out.items():
        with open(os.path.join(ROOT, "profiles", "traffic_%s.json" % KCLASS[kc].split()[0]), "w") as fh:
            json.dump(d, fh, indent=1)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
