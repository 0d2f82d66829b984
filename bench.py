#!/usr/bin/env python3
"""Time-to-tr(A^-1) benchmark of the MI355X multilevel Monte-Carlo trace estimator.

Workloads (--workload):
  poisson1024 (default): 2D Poisson 5-point operator on a 1024 x 1024 Dirichlet
    grid (n = 1,048,576), 6-level 2x2 aggregation hierarchy (coarsest 32^2
    inverted densely), 128 Rademacher right-hand sides per launch, FP32 Krylov +
    V-cycle inside FP64 refinement to a 1e-10 relative residual, MLMC to
    relative error 1e-3 with the optimal (Giles) allocation.  One step = one
    complete mlmc_trace call (pilot, all level differences, coarsest term) with
    a fresh seed; all data is generated on the device.
  wilson256: the Wilson-like 2-spin operator on a 256^2 periodic lattice
    (U(1) phases ~ N(0, 0.5^2), mass at |lambda_min| ~ 1e-2), 3 levels of 4x4
    aggregates with 8 test vectors, Z4 probes, complex64 FGMRES inside complex128
    refinement, MLMC to 1e-3.
  wilson512: the same operator on 512^2 with 4 solver levels (3 MLMC levels);
    the learned smoother (trained first, on the method's own plain solves)
    replaces two of the four finest-level sweeps.  value = learned + FP32 time
    per trace; the plain FP32 and plain FP64 MLMC times are in `compare`.
  varcoef_batch: 32 uneven 3D diffusion problems (log-normal faces, sides
    32..128) sampled concurrently; one step = 64 level-1 samples of every
    problem (128 solves each); value = aggregate solves/s.
  graph1m: a general sparse operator (the csr kind): the shifted Laplacian
    L + 0.01 I of a random geometric graph with 2^20 vertices and mean degree
    about 8, 4-level greedy aggregation hierarchy built by the library,
    multicolour Gauss-Seidel V-cycle inside FP32 CG with FP64 refinement, MLMC
    to relative error 1e-3.
  laplace_bilinear: Example 4.1's own hierarchy at N = 1023 (bilinear
    interpolation, R = P^T, Galerkin 9-point coarse operators) through the csr
    kind with the general decomposition (finest-level probes), 7 MLMC levels
    (coarsest 15^2) and 8 solver levels (coarsest 7^2).
  gauge256: the gauge Laplacian of Example 4.2 on a 256^2 periodic lattice
    (U(1) phases N(0, 0.3^2)), 4 levels of 4x4 test-vector aggregation, Z4
    probes, complex64 FGMRES inside complex128 refinement, MLMC to 1e-3.

Printed JSON line: the contract fields plus `roofline` (the dominant kernel,
timed with HIP events carried in its own dispatches during the timed steps),
`cpu_baseline` (the FP64 CPU oracle on a bounded sample, extrapolated with the
GPU run's sample counts; the oracle also supplies the exact trace of the
Poisson workload for the accuracy report), and comparisons measured outside the
timed region.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
METRIC = "time-to-tr(A^-1) at rel err 1e-3 (learned+FP32 vs plain FP64 MLMC); HBM GB/s"
# the sweep kernels and the V-cycle / Krylov code that sets their launch mix
GS_SOURCES = [os.path.join(ROOT, "paper_2108_11281_amd", "csrc", f)
              for f in ("kernels_poisson.hip", "context.cpp")]
GS_TRAFFIC = os.path.join(ROOT, "profiles", "rbgs_sweep_poisson1024_traffic.md")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# CPU oracle leg (the only part of this script that uses oracle/)
# ---------------------------------------------------------------------------
def cpu_baseline(n_samples, N, L, budget_s=12.0):
    """FP64 CPU oracle time per trace: per-sample time of each level difference
    on a bounded sample, scaled by the GPU run's per-level sample counts."""
    from oracle import mlmc
    orc = mlmc.PoissonDSTSampler(N, L)
    per_level = []
    spent = 0.0
    for l in range(1, L):
        k, t = 0, 0.0
        while k < 8 and (k < 1 or spent + t < budget_s):
            t0 = time.perf_counter()
            orc.sample(l, 99, k, 1)
            t += time.perf_counter() - t0
            k += 1
        spent += t
        per_level.append((k, t / k))
    t0 = time.perf_counter()
    orc.hutchinson(99, 0, 1, stream=1)
    t_h = time.perf_counter() - t0
    coarse_t0 = time.perf_counter()
    orc.coarse()
    t_c = time.perf_counter() - coarse_t0
    total = sum(n * per_level[l][1] for l, n in enumerate(n_samples)) + 5 * t_h + t_c
    sample = ", ".join("l%d: %d samples" % (l + 1, per_level[l][0]) for l in range(L - 1))
    return dict(value=round(total, 2), unit="s", cores=1, kind="oracle",
                sample="2D Poisson %d^2, %d levels, exact sine-transform solves (scipy.fft, "
                       "1 worker); per-sample time measured on %s, scaled by the mean N_l %s "
                       "of the GPU run's timed steps, plus 5 pilot solves; extrapolated time "
                       "per trace"
                       % (N, L, sample, list(n_samples)))


def cpu_exact_poisson_trace(N):
    from oracle import operators
    return operators.poisson2d_trace_inverse(N)


def cpu_baseline_varcoef(sides, seeds, nsamples, budget_s=20.0):
    """Oracle time per level-1 sample (sparse LU of both levels, factorisation
    included once) on the smallest and the largest problem that fit the budget,
    scaled to solves/s."""
    from oracle import hierarchy, mlmc
    from workloads import varcoef_faces, varcoef_levels
    out = []
    for N in sorted(set([min(sides)])):
        p = sides.index(N)
        t0 = time.perf_counter()
        L = varcoef_levels(N)
        A, P = hierarchy.varcoef_hierarchy(N, varcoef_faces(N, seed=1000 + p), 1e-3, L)
        smp = mlmc.LevelSampler(A, P, complex_probe=False)
        k = 0
        while k < nsamples and time.perf_counter() - t0 < budget_s:
            smp.sample(1, seeds[p], k, 1)
            k += 1
        dt = time.perf_counter() - t0
        out.append(dict(N=N, samples=k, seconds=round(dt, 2), solves_per_s=round(2 * k / dt, 2)))
    return dict(value=out[0]["solves_per_s"], unit="solves/s", cores=1, kind="oracle",
                sample="3D diffusion %d^3 (smallest batch problem): %d level-1 samples "
                       "(2 sparse-LU solves each, hierarchy and factorisations included) in "
                       "%.1f s; the larger problems do not fit a bounded CPU sample"
                       % (out[0]["N"], out[0]["samples"], out[0]["seconds"]))


# ---------------------------------------------------------------------------
def source_digest(paths):
    import hashlib
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic():
    """HBM bytes per launch of the sweep kernel from the committed FETCH_SIZE /
    WRITE_SIZE counter summary, or None when the kernel source has changed
    since the counters were taken (the summary records the source digest)."""
    try:
        with open(GS_TRAFFIC) as f:
            text = f.read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if line.startswith("traffic_bytes_per_launch:") or line.startswith("source_digest:"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_digest") != source_digest(GS_SOURCES):
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def kernel_table(est):
    """Launches, time and achieved rate of every timed kernel; the FP64 refinement
    kernels (residual, fold) are read from their FP64 instantiation."""
    out = {}
    for k in est.KERNELS:
        if k.startswith("unused"):
            continue
        launches, ms, amount = est.kernel_stats(k, fp64=k.startswith("ir_"))
        rate = amount / (ms * 1e-3) if ms > 0 else 0.0
        if k == "nn_apply":
            out[k] = dict(launches=launches, ms=round(ms, 2), tflops=round(rate / 1e12, 2))
        else:
            out[k] = dict(launches=launches, ms=round(ms, 2), gbs=round(rate / 1e9, 1))
    return out


CSR_SWEEP_LABEL = ("multicolour Gauss-Seidel sweep: k_csr_gs + k_csr_gs_tail<float> "
                   "(all colour classes)")


def hbm_roofline(name, stats, stride, traffic=None):
    launches, ms, nbytes = stats
    achieved = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    return dict(bound="hbm", kernel=name, achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                launches_timed=launches, timing_stride=stride,
                avg_launch_us=round(1000.0 * ms / max(launches, 1), 2),
                algorithmic_bytes_per_launch=round(nbytes / max(launches, 1)))


def per_level_fractions(est, kernel, levels, fp64=False):
    """Achieved HBM fraction of one kernel family on each level (event-timed launches
    of the timed steps)."""
    out = []
    for l in range(1, levels + 1):
        launches, ms, nbytes = est.kernel_stats(kernel, fp64=fp64, level=l)
        if launches == 0:
            continue
        gbs = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        out.append(dict(level=l, n=est.level_size(l), launches_timed=launches,
                        avg_launch_us=round(1000.0 * ms / launches, 2),
                        gbs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4),
                        time_share=None, _ms=ms))
    tot = sum(d["_ms"] for d in out) or 1.0
    for d in out:
        d["time_share"] = round(d.pop("_ms") / tot, 4)
    return out


def copy_bandwidth(torch, mib=1024, reps=20, library=False):
    """Measured device-to-device copy rate (read + write bytes per second) on
    this GPU, beside the 8 TB/s vendor peak: torch's copy kernel, or (library)
    the library's streaming copy of 16-byte loads and stores."""
    import paper_2108_11281_amd as m
    n = mib * (1 << 20) // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)

    def once():
        if library:
            m.stream_copy(a, b)
        else:
            b.copy_(a)
    for _ in range(3):
        once()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        once()
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) * 1e-3 / reps
    if library:
        assert bool(torch.equal(a, b))
    del a, b
    return round(2.0 * n * 4 / s / 1e9, 1)


def timed_traces(est, args, torch, method="trace"):
    """Seconds per trace of `est` over the timed steps' own seeds (1..steps),
    after one warm-up trace; returns (mean seconds, per-seed sample counts)."""
    run = getattr(est, method)
    run(args.eps, 1000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ns = [run(args.eps, i + 1)["n_samples"] for i in range(args.steps)]
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / args.steps, ns


def contract(args, value, unit, hib, ms_per_step, dtype, data, config, roofline, cpu, **extra):
    out = {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 2), "higher_is_better": hib,
           "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": data,
           "config": config, "roofline": roofline, "cpu_baseline": cpu}
    out.update(extra)
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------
def run_poisson(args, m, torch):
    N, L = args.N, args.levels
    log("setup poisson2d N=%d L=%d nb=%d" % (N, L, args.nb))
    t0 = time.perf_counter()
    vc = dict(nu_pre=args.nu, nu_post=args.nu)
    est = m.TraceEstimator("poisson2d", N, L, L, precision="fp32_ir64", nb=args.nb,
                           solve_tol=1e-10, alloc=args.alloc, narrow_fp64=args.narrow_fp64, **vc)
    setup_s = time.perf_counter() - t0
    log("setup %.2fs" % setup_s)
    for i in range(args.warmup):
        r = est.trace(args.eps, 1000 + i)
        log("warmup %d: %.3fs N_l=%s" % (i, r["seconds"], r["n_samples"]))
    # only the dominant kernel (the fused smoother sweep) is timed inside the
    # timed region; the per-kernel table comes from one extra step afterwards
    est.set_timing(["rbgs_sweep"], stride=args.timing_stride)
    est.reset_kernel_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for i in range(args.steps):
        r = est.trace(args.eps, i + 1)
        runs.append(r)
        log("step %d: %.3fs N_l=%s trace=%.6f rmsd=%.3f level_s=%s"
            % (i, r["seconds"], r["n_samples"], r["trace"].real, r["rmsd"],
               [round(v, 3) for v in r["level_seconds"]]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gs = est.kernel_stats("rbgs_sweep")
    per_level = per_level_fractions(est, "rbgs_sweep", L)
    est.set_timing(True)
    est.reset_kernel_stats()
    est.trace(args.eps, 777)
    kernels = kernel_table(est)
    est.set_timing(False)
    ms_per_step = 1000.0 * elapsed / args.steps
    roofline = hbm_roofline("rbgs_sweep<float>", gs, args.timing_stride, stored_traffic())
    roofline["per_level"] = per_level
    # sustained HBM rate of a plain copy (1 GiB each way): the library's
    # streaming kernel and torch's copy, beside the vendor peak
    copy_gbs = copy_bandwidth(torch, library=True)
    roofline["copy_kernel_gbs"] = copy_gbs
    roofline["copy_torch_gbs"] = copy_bandwidth(torch)
    roofline["frac_of_copy"] = round(roofline["achieved"] / copy_gbs, 4)
    for d in per_level:
        d["frac_of_copy"] = round(d["gbs"] / copy_gbs, 4)
    log("per-level sweep fractions %s; copy kernel %.1f GB/s (torch copy %.1f)" % (
        [(d["level"], d["frac"]) for d in per_level], copy_gbs, roofline["copy_torch_gbs"]))

    compare = {}
    if not args.no_compare:
        est.close()
        log("plain FP64 MLMC, same workload")
        log("FP32 + refinement with HIP-graph replay of the CG iterations (no kernel timing)")
        eg = m.TraceEstimator("poisson2d", N, L, L, precision="fp32_ir64", nb=args.nb,
                              solve_tol=1e-10, alloc=args.alloc, graphs=1,
                              narrow_fp64=args.narrow_fp64, **vc)
        eg.trace(args.eps, 1000)
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for i in range(args.steps):
            eg.trace(args.eps, i + 1)
        torch.cuda.synchronize()
        compare["graphs_s_per_trace"] = round((time.perf_counter() - tg) / args.steps, 4)
        eg.set_timing(False)
        eg.close()
        log("graphs: %.3fs per trace" % compare["graphs_s_per_trace"])
        e64 = m.TraceEstimator("poisson2d", N, L, L, precision="fp64", nb=args.nb,
                               solve_tol=1e-10, alloc=args.alloc, **vc)
        t64, n64 = timed_traces(e64, args, torch)
        compare["fp64_mlmc_s"] = round(t64, 3)
        compare["fp64_mlmc_n_samples"] = n64
        log("plain FP64 MLMC %.3fs per trace, N_l=%s" % (t64, n64))
        log("plain FP64 Hutchinson, same accuracy")
        th, nh = timed_traces(e64, args, torch, "hutchinson")
        compare["fp64_hutchinson_s"] = round(th, 3)
        compare["fp64_hutchinson_n_samples"] = [n[0] for n in nh]
        log("plain FP64 Hutchinson %.3fs per trace, N=%s" % (th, [n[0] for n in nh]))
        e64.close()
        compare["speedup_vs_fp64_mlmc"] = round(t64 / (ms_per_step / 1000.0), 2)
        compare["speedup_vs_fp64_hutchinson"] = round(th / (ms_per_step / 1000.0), 2)
        if args.defl_scan:
            log("deflated Hutchinson, same workload")
            dh = deflated_compare(args, m, torch, lambda: m.TraceEstimator(
                "poisson2d", N, L, L, precision="fp32_ir64", nb=args.nb, solve_tol=1e-10,
                alloc=args.alloc, **vc))
            dh["speedup_mlmc_vs_deflated"] = round(dh["s_per_trace"] / (ms_per_step / 1000.0), 2)
            dh["speedup_mlmc_vs_deflated_with_setup"] = round(
                (dh["s_per_trace"] + dh["setup_s"]) / (ms_per_step / 1000.0), 2)
            compare["deflated_hutchinson"] = dh
        if not args.no_c4:
            compare["c4_learned"] = c4_compare(args, m, torch)

    cpu, accuracy = None, {"n_samples": [r["n_samples"] for r in runs],
                           "rmsd_rel": [round(r["rmsd"] / abs(r["trace"].real), 7) for r in runs]}
    if not args.no_cpu:
        log("CPU oracle baseline")
        # the oracle's time for the mean sample counts of the timed steps
        mean_n = [int(round(sum(r["n_samples"][j] for r in runs) / len(runs)))
                  for j in range(len(runs[0]["n_samples"]))]
        cpu = cpu_baseline(mean_n, N, L)
        exact = cpu_exact_poisson_trace(N)
        accuracy.update(exact_trace=exact,
                        rel_err=[round(abs(r["trace"].real - exact) / exact, 7) for r in runs],
                        z=[round((r["trace"].real - exact) / r["rmsd"], 2) for r in runs])

    config = {"workload": "poisson2d_%dx%d_L%d_agg2x2_nb%d_fp32ir64_eps%g"
                          % (N, N, L, args.nb, args.eps),
              "variant": "FP32 inner Krylov + V-cycle, FP64 reliable-update refinement "
                         "(no learned smoother on this operator)",
              "n": N * N, "levels": L, "nb": args.nb, "eps": args.eps, "alloc": args.alloc,
              "solve_tol": 1e-10, "nu_pre": args.nu, "nu_post": args.nu, "omega": 1.8,
              "narrow_fp64": args.narrow_fp64}
    contract(args, round(ms_per_step / 1000.0, 4), "s", False, ms_per_step, "f32+f64ir",
             "synthetic (Rademacher probes from Philox4x64-10 on the device)", config,
             roofline, cpu, accuracy=accuracy, setup_s=round(setup_s, 3), kernels=kernels,
             compare=compare)


def _wilson_est(m, N, Ls, L, precision, learned, nb, alloc, n_vec=8, spin_split=False,
                top_cycles=0, graphs=0):
    from workloads import gauge_field, wilson_mass
    return m.TraceEstimator("wilson2d", N, Ls, L, mass=wilson_mass(N),
                            field=gauge_field(N, sigma=0.5, seed=1), block=4, n_vec=n_vec,
                            spin_split=spin_split, setup_sweeps=20, setup_seed=1,
                            precision=precision, nb=nb, nu_pre=2, nu_post=2, solve_tol=1e-10,
                            alloc=alloc, learned=1 if learned else 0, top_cycles=top_cycles,
                            graphs=graphs)


def deflated_compare(args, m, torch, make):
    """Deflated Hutchinson (Sec. 4.2 eq. defl; the comparison method of Sec. 5) on
    the same operator and seeds: a rough scan of n_defl on the first seed (as the
    paper does to find a near time-optimal value), then the timed traces with the
    best one.  The eigenpair setup (subspace iteration on the library's own
    solves) is reported separately, as the paper excludes it from its cost."""
    est = make()
    scan = []
    best = None
    for k in args.defl_scan:
        rep = est.deflation_setup(k, eig_tol=1e-3, max_iter=100, solve_tol=1e-6, seed=1)
        est.deflated_hutchinson(args.eps, 1000)      # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = est.deflated_hutchinson(args.eps, 1)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        row = dict(n_defl=k, setup_s=round(rep["seconds"], 3), setup_iterations=rep["iterations"],
                   setup_solves=rep["solves"], trace_s=round(t, 4), n_samples=r["n_samples"][0])
        scan.append(row)
        log("deflated Hutchinson n_defl=%d: setup %.2fs (%d iterations), %.3fs per trace, N=%d"
            % (k, rep["seconds"], rep["iterations"], t, r["n_samples"][0]))
        if best is None or t + rep["seconds"] < best[0]:
            best = (t + rep["seconds"], k)
    k = best[1]
    rep = est.deflation_setup(k, eig_tol=1e-3, max_iter=100, solve_tol=1e-6, seed=1)
    td, nd = timed_traces(est, args, torch, "deflated_hutchinson")
    est.close()
    return dict(n_defl=k, scan=scan, setup_s=round(rep["seconds"], 3), s_per_trace=round(td, 4),
                n_samples=[n[0] for n in nd],
                note="FP32 + FP64-refinement solves as in MLMC; setup (eigenpairs + direct "
                     "term) not included in s_per_trace")


def c4_compare(args, m, torch):
    """The learned-smoother configuration (Wilson 512^2, 4 solver / 3 MLMC levels):
    time per trace with the trained network + FP32, plain FP32 and plain FP64 MLMC
    on the same seeds, training (pair generation from the method's own plain solves
    and Adam) timed separately, and the number of traces after which training
    pays for itself against plain FP32."""
    from workloads import nn_init_weights
    N, Ls, L = 512, 4, 3
    steps = max(1, min(args.steps, args.c4_steps))
    sub = argparse.Namespace(**vars(args))
    sub.steps = steps
    out = {"workload": "wilson2d_512x512_Ls4_L3_agg4x4x8_nb%d_c64ir128_eps%g_learned"
                       % (args.nb, args.eps), "traces_timed": steps}
    log("C4: learned smoother on Wilson 512^2 (training on %d plain solves)"
        % (args.train_batches * args.nb))
    est = _wilson_est(m, N, Ls, L, "fp32_ir64", True, args.nb, args.alloc)
    t0 = time.perf_counter()
    train = est.learned_train(nn_init_weights(1), n_batches=args.train_batches,
                              crops_per_column=4, steps=args.train_steps, batch=256, lr=2e-3,
                              seed=5)
    train["wall_s"] = round(time.perf_counter() - t0, 3)
    out["training"] = train
    tl, nl = timed_traces(est, sub, torch)
    out["learned_fp32_s"] = round(tl, 4)
    out["learned_n_samples"] = nl
    out["learned_stats"] = list(est.learned_stats())
    est.close()
    ep = _wilson_est(m, N, Ls, L, "fp32_ir64", False, args.nb, args.alloc)
    tp, npl = timed_traces(ep, sub, torch)
    ep.close()
    e64 = _wilson_est(m, N, Ls, L, "fp64", False, args.nb, args.alloc)
    t64, n64 = timed_traces(e64, sub, torch)
    e64.close()
    out.update(plain_fp32_s=round(tp, 4), plain_fp32_n_samples=npl, fp64_mlmc_s=round(t64, 4),
               fp64_n_samples=n64, speedup_learned_vs_fp64=round(t64 / tl, 3),
               speedup_learned_vs_plain_fp32=round(tp / tl, 3))
    gain = tp - tl
    out["training_break_even_traces"] = (round(train["wall_s"] / gain, 1) if gain > 0
                                         else None)
    log("C4: learned %.4fs, plain FP32 %.4fs, plain FP64 %.4fs per trace; training %.1fs"
        % (tl, tp, t64, train["wall_s"]))
    return out


def run_wilson(args, m, torch, N, learned):
    from workloads import nn_init_weights
    Ls, L = (4, 3) if N >= 512 else (3, 3)
    log("setup wilson2d N=%d Ls=%d L=%d nb=%d learned=%s" % (N, Ls, L, args.nb, learned))
    t0 = time.perf_counter()
    nv = args.n_vec if args.n_vec > 0 else (4 if args.spin_split else 8)
    est = _wilson_est(m, N, Ls, L, "fp32_ir64", learned, args.nb, args.alloc, nv, args.spin_split,
                      args.top_cycles)
    setup_s = time.perf_counter() - t0
    log("setup %.2fs" % setup_s)
    train = None
    if learned:
        t0 = time.perf_counter()
        train = est.learned_train(nn_init_weights(1), n_batches=args.train_batches,
                                  crops_per_column=4, steps=args.train_steps, batch=256,
                                  lr=2e-3, seed=5)
        train["wall_s"] = round(time.perf_counter() - t0, 3)
        log("training %s" % json.dumps(train))
    for i in range(args.warmup):
        r = est.trace(args.eps, 1000 + i)
        log("warmup %d: %.3fs N_l=%s" % (i, r["seconds"], r["n_samples"]))
    timed_kernel = "nn_apply" if learned else "rbgs_sweep"
    est.set_timing([timed_kernel], stride=args.timing_stride)
    est.reset_kernel_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for i in range(args.steps):
        r = est.trace(args.eps, i + 1)
        runs.append(r)
        log("step %d: %.3fs N_l=%s trace=%s rmsd=%.4g iters=%d"
            % (i, r["seconds"], r["n_samples"], r["trace"], r["rmsd"], r["iterations"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ks = est.kernel_stats(timed_kernel)
    est.set_timing(False)
    ms_per_step = 1000.0 * elapsed / args.steps
    if learned:
        launches, ms, flops = ks
        ach = flops / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        roofline = dict(bound="mfma", kernel="k_nn_apply (bf16 16x16x32)", achieved=round(ach, 2),
                        peak=BF16_PEAK_TFLOPS, unit="TFLOP/s",
                        frac=round(ach / BF16_PEAK_TFLOPS, 4), traffic=None,
                        launches_timed=launches, timing_stride=args.timing_stride,
                        avg_launch_us=round(1000.0 * ms / max(launches, 1), 2),
                        algorithmic_flops_per_launch=round(flops / max(launches, 1)))
    else:
        roofline = hbm_roofline("smoother sweeps: k_wilson_gs2<c32> (finest, both colours "
                                "per pass) and k_bsr_gs / k_bsr_gs_rows<8, c32> (coarse block "
                                "stencils)", ks,
                                args.timing_stride)
    compare = {"learned_stats": list(est.learned_stats())} if learned else {}
    weights = est.get_nn_weights() if learned else None
    est.close()
    if not args.no_compare:
        # the same configuration with every FGMRES iteration replayed from a HIP
        # graph (no kernel timing), the trained weights set
        eg = _wilson_est(m, N, Ls, L, "fp32_ir64", learned, args.nb, args.alloc, nv,
                         args.spin_split, args.top_cycles, graphs=1)
        if learned:
            eg.set_nn_weights(weights)
        tg, _ = timed_traces(eg, args, torch)
        eg.close()
        compare["graphs_s_per_trace"] = round(tg, 4)
        log("graphs: %.3fs per trace" % tg)
        if learned:
            log("plain FP32 MLMC (no network), same workload")
            ep = _wilson_est(m, N, Ls, L, "fp32_ir64", False, args.nb, args.alloc, nv,
                             args.spin_split, args.top_cycles)
            tp, npl = timed_traces(ep, args, torch)
            ep.close()
            compare["plain_fp32_mlmc_s"] = round(tp, 3)
            compare["plain_fp32_mlmc_n_samples"] = npl
            log("plain FP32 MLMC %.3fs per trace, N_l=%s" % (tp, npl))
        log("plain FP64 MLMC, same workload")
        e64 = _wilson_est(m, N, Ls, L, "fp64", False, args.nb, args.alloc, nv, args.spin_split,
                          args.top_cycles)
        t64, n64 = timed_traces(e64, args, torch)
        e64.close()
        compare["fp64_mlmc_s"] = round(t64, 3)
        compare["fp64_mlmc_n_samples"] = n64
        compare["speedup_vs_fp64_mlmc"] = round(t64 / (ms_per_step / 1000.0), 2)
        if learned:
            compare["speedup_vs_plain_fp32_mlmc"] = round(
                compare["plain_fp32_mlmc_s"] / (ms_per_step / 1000.0), 2)
        log("plain FP64 MLMC %.3fs per trace, N_l=%s" % (t64, n64))
    dof = 2 * nv if args.spin_split else nv
    config = {"workload": "wilson2d_%dx%d_Ls%d_L%d_agg4x4x%d%s_nb%d_c64ir128_eps%g%s"
                          % (N, N, Ls, L, dof, "spin" if args.spin_split else "", args.nb,
                             args.eps, "_learned" if learned else ""),
              "n_vec": nv, "spin_split": bool(args.spin_split),
              "variant": ("learned smoother (2 of 4 finest sweeps) + complex64 FGMRES in "
                          "complex128 refinement" if learned else
                          "complex64 FGMRES + V-cycle in complex128 refinement"),
              "n": 2 * N * N, "levels_solver": Ls, "levels_mlmc": L, "nb": args.nb,
              "eps": args.eps, "alloc": args.alloc, "solve_tol": 1e-10}
    contract(args, round(ms_per_step / 1000.0, 4), "s", False, ms_per_step,
             "c64+c128ir" + ("+bf16net" if learned else ""),
             "synthetic (U(1) phases N(0,0.5^2), Z4 probes from Philox4x64-10)", config,
             roofline, None,
             accuracy={"n_samples": [r["n_samples"] for r in runs],
                       "rmsd_rel": [round(r["rmsd"] / abs(r["trace"].real), 7) for r in runs],
                       "trace": [[r["trace"].real, r["trace"].imag] for r in runs]},
             setup_s=round(setup_s, 3), training=train, compare=compare)


def run_batch(args, m, torch):
    from workloads import batch_problem_sizes, varcoef_faces, varcoef_levels
    sides = batch_problem_sizes(32)
    seeds = [1000 + p for p in range(len(sides))]
    log("setup %d varcoef3d problems, sides %s" % (len(sides), sides))
    t0 = time.perf_counter()
    ests = []
    for p, N in enumerate(sides):
        L = varcoef_levels(N)
        ests.append(m.TraceEstimator("varcoef3d", N, L, L, shift=1e-3,
                                     field=varcoef_faces(N, seed=1000 + p), nb=64,
                                     precision="fp32_ir64", solve_tol=1e-10,
                                     top_cycles=args.top_cycles,
                                     stream=torch.cuda.Stream()))
    setup_s = time.perf_counter() - t0
    log("setup %.2fs" % setup_s)
    ns = 64
    grouped = args.workers <= 0

    def step(first, workers):
        # workers 0: every problem in lockstep on one stream, each V-cycle one
        # launch per stage position; -1: the same with each V-cycle one
        # persistent launch (a workgroup per problem and column pair); else host
        # worker threads, one HIP stream per problem
        if workers <= 0:
            s, _ = m.batch_sample_grouped(ests, 1, seeds, first, ns, persistent=workers < 0)
            return s, None
        return m.batch_sample(ests, 1, seeds, first, ns, workers=workers)

    for i in range(args.warmup):
        step(10 ** 6 + i * ns, args.workers)
    for e in ests:
        e.set_timing(["rbgs_sweep"], stride=args.timing_stride)
        e.reset_kernel_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per = []
    for i in range(args.steps):
        t1 = time.perf_counter()
        _, sec = step(i * ns, args.workers)
        per.append(sec)
        log("step %d: %.3fs" % (i, time.perf_counter() - t1))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tot = [0, 0.0, 0.0]
    for e in ests:
        st = e.kernel_stats("rbgs_sweep")
        tot = [tot[0] + st[0], tot[1] + st[1], tot[2] + st[2]]
        e.set_timing(False)
    solves = 2 * ns * len(ests) * args.steps
    value = solves / elapsed
    ms_per_step = 1000.0 * elapsed / args.steps
    import numpy as np
    per_problem = None
    if not grouped:
        per_problem = [dict(N=N, solves_per_s=round(2 * ns / float(np.mean([s[p] for s in per])),
                                                    1)) for p, N in enumerate(sides)]
    compare = {}
    if not args.no_compare:
        # the other schedules on the same samples: host workers on four streams,
        # and one worker
        for label, workers in (("grouped_positions", 0), ("grouped_persistent", -1),
                               ("four_workers", 4), ("one_worker", 1)):
            if workers == args.workers:
                continue
            step(0, workers)  # warm-up of this schedule
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            step(0, workers)
            torch.cuda.synchronize()
            compare[label + "_solves_per_s"] = round(2 * ns * len(ests) /
                                                     (time.perf_counter() - t1), 1)
        if grouped:
            s_g, _ = step(0, args.workers)
            s_w, _ = step(0, 4)
            compare["grouped_equals_workers_bitwise"] = bool(np.array_equal(s_g, s_w))
    for e in ests:
        e.close()
    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline (smallest problem)")
        cpu = cpu_baseline_varcoef(sides, seeds, ns)
    config = {"workload": "varcoef3d_batch32_N32-128_agg2x2x2_nb64_fp32ir64",
              "problems": len(sides), "sides": sides, "probes_per_problem": ns,
              "schedule": ({0: "grouped lockstep, one launch per V-cycle position",
                            -1: "grouped lockstep, one persistent launch per V-cycle"}
                           .get(args.workers, "%d host workers, one stream per problem"
                                % args.workers)),
              "solve_tol": 1e-10}
    kname = {0: "V-cycle stage kernels kg_stage (3D sweeps, residual restriction, coarsest "
                "solve of all problems)",
             -1: "persistent V-cycle kernel kg_vcycle_units (every stage of all problems)"}.get(
        args.workers, "3D red-black sweep: k_vc_march<float> (both colours, one pass)")
    contract(args, round(value, 1), "solves/s", True, ms_per_step, "f32+f64ir",
             "synthetic (log-normal face coefficients sigma=1, Rademacher probes)", config,
             hbm_roofline(kname, tot, args.timing_stride), cpu, per_problem=per_problem,
             setup_s=round(setup_s, 2), compare=compare)


def run_graph(args, m, torch):
    from workloads import graph_laplacian, workload
    w = workload("graph1m_fp32ir")
    n, Ls, L = w["n"], w["levels_solver"], w["levels_mlmc"]
    log("generate graph n=%d degree=%g shift=%g" % (n, w["degree"], w["shift"]))
    A = graph_laplacian(n, degree=w["degree"], shift=w["shift"], seed=w["graph_seed"])
    vc = dict(nu_pre=args.nu, nu_post=args.nu)
    if args.omega > 0:
        vc["omega"] = args.omega

    def make(precision, graphs=0):
        return m.TraceEstimator("csr", 0, Ls, L, matrix=A, precision=precision, nb=args.nb,
                                solve_tol=w["solve_tol"], alloc=args.alloc,
                                narrow_fp64=args.narrow_fp64 if precision != "fp64" else 0,
                                top_cycles=args.top_cycles, graphs=graphs, **vc)
    t0 = time.perf_counter()
    est = make("fp32_ir64")
    setup_s = time.perf_counter() - t0
    sizes = [est.level_size(l) for l in range(1, Ls + 1)]
    log("setup %.2fs, level sizes %s" % (setup_s, sizes))
    for i in range(args.warmup):
        r = est.trace(args.eps, 1000 + i)
        log("warmup %d: %.3fs N_l=%s iters=%d" % (i, r["seconds"], r["n_samples"],
                                                  r["iterations"]))
    est.set_timing(["rbgs_sweep"], stride=args.timing_stride)
    est.reset_kernel_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for i in range(args.steps):
        r = est.trace(args.eps, i + 1)
        runs.append(r)
        log("step %d: %.3fs N_l=%s trace=%.6f rmsd=%.3f iters=%d level_s=%s"
            % (i, r["seconds"], r["n_samples"], r["trace"].real, r["rmsd"], r["iterations"],
               [round(v, 3) for v in r["level_seconds"]]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gs = est.kernel_stats("rbgs_sweep")
    est.set_timing(True)
    est.reset_kernel_stats()
    est.trace(args.eps, 777)
    kernels = kernel_table(est)
    est.set_timing(False)
    est.close()
    ms_per_step = 1000.0 * elapsed / args.steps
    compare = {}
    if not args.no_compare:
        eg = make("fp32_ir64", graphs=1)  # CG iteration pairs replayed from HIP graphs
        tg, _ = timed_traces(eg, args, torch)
        eg.close()
        compare["graphs_s_per_trace"] = round(tg, 4)
        log("graphs: %.3fs per trace" % tg)
        log("plain FP64 MLMC, same workload")
        e64 = make("fp64")
        t64, n64 = timed_traces(e64, args, torch)
        compare.update(fp64_mlmc_s=round(t64, 3), fp64_mlmc_n_samples=n64,
                       speedup_vs_fp64_mlmc=round(t64 / (ms_per_step / 1000.0), 2))
        log("plain FP64 MLMC %.3fs per trace, N_l=%s" % (t64, n64))
        th, nh = timed_traces(e64, args, torch, "hutchinson")
        compare.update(fp64_hutchinson_s=round(th, 3),
                       fp64_hutchinson_n_samples=[v[0] for v in nh],
                       speedup_vs_fp64_hutchinson=round(th / (ms_per_step / 1000.0), 2))
        log("plain FP64 Hutchinson %.3fs per trace, N=%s" % (th, [v[0] for v in nh]))
        e64.close()
    config = {"workload": "graph_laplacian_rgg_n%d_deg%g_shift%g_L%d_greedyagg_nb%d_fp32ir64_eps%g"
                          % (n, w["degree"], w["shift"], L, args.nb, args.eps),
              "variant": "general CSR operator: FP32 CG + multicolour Gauss-Seidel V-cycle, "
                         "FP64 reliable-update refinement",
              "n": n, "nnz": int(A.nnz), "level_sizes": sizes, "levels": L, "nb": args.nb,
              "eps": args.eps, "alloc": args.alloc, "solve_tol": w["solve_tol"],
              "nu_pre": args.nu, "nu_post": args.nu, "narrow_fp64": args.narrow_fp64,
              "omega": args.omega if args.omega > 0 else 1.0}
    contract(args, round(ms_per_step / 1000.0, 4), "s", False, ms_per_step, "f32+f64ir",
             "synthetic (random geometric graph Laplacian + shift, Rademacher probes)", config,
             hbm_roofline(CSR_SWEEP_LABEL, gs, args.timing_stride),
             None, accuracy={"n_samples": [r["n_samples"] for r in runs],
                             "rmsd_rel": [round(r["rmsd"] / abs(r["trace"].real), 7)
                                          for r in runs]},
             setup_s=round(setup_s, 3), kernels=kernels, compare=compare)


def run_laplace_bilinear(args, m, torch):
    """Example 4.1's setup at N = 1023: the 5-point Laplacian, bilinear
    interpolation, Galerkin coarse operators, the general decomposition with
    finest-level probes, MLMC levels down to 15^2, solver levels down to 7^2."""
    from workloads import bilinear_prolongations, laplace_matrix, workload
    w = workload("laplace1023_bilinear_fp32ir")
    N, Ls, L = w["N"], w["levels_solver"], w["levels_mlmc"]
    A = laplace_matrix(N)
    P = bilinear_prolongations(N, Ls)
    vc = dict(nu_pre=args.nu, nu_post=args.nu)
    if args.omega > 0:
        vc["omega"] = args.omega

    def make(precision, graphs=0):
        return m.TraceEstimator("csr", 0, Ls, L, matrix=A, prolongations=P, precision=precision,
                                nb=args.nb, solve_tol=w["solve_tol"], alloc=args.alloc,
                                narrow_fp64=args.narrow_fp64 if precision != "fp64" else 0,
                                top_cycles=args.top_cycles, graphs=graphs, **vc)
    t0 = time.perf_counter()
    est = make("fp32_ir64")
    setup_s = time.perf_counter() - t0
    sizes = [est.level_size(l) for l in range(1, Ls + 1)]
    log("setup %.2fs, level sizes %s" % (setup_s, sizes))
    for i in range(args.warmup):
        r = est.trace(args.eps, 1000 + i)
        log("warmup %d: %.3fs N_l=%s iters=%d" % (i, r["seconds"], r["n_samples"],
                                                  r["iterations"]))
    est.set_timing(["rbgs_sweep"], stride=args.timing_stride)
    est.reset_kernel_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for i in range(args.steps):
        r = est.trace(args.eps, i + 1)
        runs.append(r)
        log("step %d: %.3fs N_l=%s trace=%.6f rmsd=%.3f iters=%d level_s=%s"
            % (i, r["seconds"], r["n_samples"], r["trace"].real, r["rmsd"], r["iterations"],
               [round(v, 3) for v in r["level_seconds"]]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gs = est.kernel_stats("rbgs_sweep")
    est.set_timing(True)
    est.reset_kernel_stats()
    est.trace(args.eps, 777)
    kernels = kernel_table(est)
    est.set_timing(False)
    est.close()
    ms_per_step = 1000.0 * elapsed / args.steps
    compare = {}
    if not args.no_compare:
        eg = make("fp32_ir64", graphs=1)  # CG iteration pairs replayed from HIP graphs
        tg, _ = timed_traces(eg, args, torch)
        eg.close()
        compare["graphs_s_per_trace"] = round(tg, 4)
        log("graphs: %.3fs per trace" % tg)
        log("plain FP64 MLMC, same workload")
        e64 = make("fp64")
        t64, n64 = timed_traces(e64, args, torch)
        compare.update(fp64_mlmc_s=round(t64, 3), fp64_mlmc_n_samples=n64,
                       speedup_vs_fp64_mlmc=round(t64 / (ms_per_step / 1000.0), 2))
        log("plain FP64 MLMC %.3fs per trace, N_l=%s" % (t64, n64))
        # (plain Hutchinson at this accuracy needs thousands of finest-level
        # solves per trace; the aggregation workload reports that comparison)
        e64.close()
    accuracy = {"n_samples": [r["n_samples"] for r in runs],
                "rmsd_rel": [round(r["rmsd"] / abs(r["trace"].real), 7) for r in runs]}
    if not args.no_cpu:
        exact = cpu_exact_poisson_trace(N)
        accuracy.update(exact_trace=exact,
                        rel_err=[round(abs(r["trace"].real - exact) / exact, 7) for r in runs],
                        z=[round((r["trace"].real - exact) / r["rmsd"], 2) for r in runs])
    config = {"workload": "laplace2d_%dx%d_bilinear_Ls%d_L%d_general_nb%d_fp32ir64_eps%g"
                          % (N, N, Ls, L, args.nb, args.eps),
              "variant": "Example 4.1 hierarchy (bilinear interpolation, R = P^T, Galerkin), "
                         "general decomposition with finest-level probes; FP32 CG + "
                         "multicolour Gauss-Seidel V-cycle, FP64 reliable-update refinement",
              "n": N * N, "level_sizes": sizes, "levels_mlmc": L, "levels_solver": Ls,
              "nb": args.nb, "eps": args.eps, "alloc": args.alloc, "solve_tol": w["solve_tol"],
              "nu_pre": args.nu, "nu_post": args.nu, "narrow_fp64": args.narrow_fp64,
              "omega": args.omega if args.omega > 0 else 1.0}
    contract(args, round(ms_per_step / 1000.0, 4), "s", False, ms_per_step, "f32+f64ir",
             "synthetic (Example 4.1 Laplacian, Rademacher probes)", config,
             hbm_roofline(CSR_SWEEP_LABEL, gs, args.timing_stride),
             None, accuracy=accuracy, setup_s=round(setup_s, 3), kernels=kernels,
             compare=compare)


def run_gauge(args, m, torch):
    """Gauge Laplacian of Example 4.2 at 256^2 (U(1) phases N(0, 0.3^2), m = 0),
    test-vector aggregation (4 x 4 aggregates, n_vec test vectors), 4 levels."""
    from workloads import gauge_field, workload
    w = workload("gauge256_c64ir")
    N, Ls, L = w["N"], w["levels_solver"], w["levels_mlmc"]
    nv = args.n_vec if args.n_vec > 0 else w["n_vec"]
    th = gauge_field(N, sigma=w["theta_sigma"], seed=w["gauge_seed"])

    def make(precision, graphs=0):
        return m.TraceEstimator("gauge2d", N, Ls, L, mass=w["mass"], field=th, block=4,
                                n_vec=nv, setup_sweeps=w["setup_sweeps"], setup_seed=1,
                                precision=precision, nb=args.nb, nu_pre=args.nu,
                                nu_post=args.nu, solve_tol=w["solve_tol"], alloc=args.alloc,
                                graphs=graphs)
    t0 = time.perf_counter()
    est = make("fp32_ir64")
    setup_s = time.perf_counter() - t0
    sizes = [est.level_size(l) for l in range(1, Ls + 1)]
    log("setup %.2fs, level sizes %s" % (setup_s, sizes))
    for i in range(args.warmup):
        r = est.trace(args.eps, 1000 + i)
        log("warmup %d: %.3fs N_l=%s" % (i, r["seconds"], r["n_samples"]))
    est.set_timing(["rbgs_sweep"], stride=args.timing_stride)
    est.reset_kernel_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for i in range(args.steps):
        r = est.trace(args.eps, i + 1)
        runs.append(r)
        log("step %d: %.3fs N_l=%s trace=%s rmsd=%.4g iters=%d"
            % (i, r["seconds"], r["n_samples"], r["trace"], r["rmsd"], r["iterations"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ks = est.kernel_stats("rbgs_sweep")
    est.set_timing(False)
    est.close()
    ms_per_step = 1000.0 * elapsed / args.steps
    compare = {}
    if not args.no_compare:
        eg = make("fp32_ir64", graphs=1)  # FGMRES iterations replayed from HIP graphs
        tg, _ = timed_traces(eg, args, torch)
        eg.close()
        compare["graphs_s_per_trace"] = round(tg, 4)
        log("graphs: %.3fs per trace" % tg)
        log("plain FP64 MLMC, same workload")
        e64 = make("fp64")
        t64, n64 = timed_traces(e64, args, torch)
        e64.close()
        compare.update(fp64_mlmc_s=round(t64, 3), fp64_mlmc_n_samples=n64,
                       speedup_vs_fp64_mlmc=round(t64 / (ms_per_step / 1000.0), 2))
        log("plain FP64 MLMC %.3fs per trace, N_l=%s" % (t64, n64))
    config = {"workload": "gauge_laplacian2d_%dx%d_Ls%d_L%d_agg4x4x%d_nb%d_c64ir128_eps%g"
                          % (N, N, Ls, L, nv, args.nb, args.eps),
              "variant": "complex64 FGMRES + block Gauss-Seidel V-cycle in complex128 "
                         "refinement; test-vector aggregation",
              "n": N * N, "level_sizes": sizes, "levels_solver": Ls, "levels_mlmc": L,
              "n_vec": nv, "nb": args.nb, "eps": args.eps, "alloc": args.alloc,
              "solve_tol": w["solve_tol"], "nu_pre": args.nu, "nu_post": args.nu}
    contract(args, round(ms_per_step / 1000.0, 4), "s", False, ms_per_step, "c64+c128ir",
             "synthetic (U(1) phases N(0,0.3^2), Z4 probes from Philox4x64-10)", config,
             hbm_roofline("smoother sweeps: k_bsr_gs / k_bsr_gs_rows<1, c32> (finest, 1 x 1 "
                          "blocks) and <n_vec, c32> (coarse block stencils)", ks,
                          args.timing_stride),
             None, accuracy={"n_samples": [r["n_samples"] for r in runs],
                             "rmsd_rel": [round(r["rmsd"] / abs(r["trace"].real), 7)
                                          for r in runs],
                             "trace": [[r["trace"].real, r["trace"].imag] for r in runs]},
             setup_s=round(setup_s, 3), compare=compare)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="poisson1024",
                    choices=["poisson1024", "wilson256", "wilson512", "varcoef_batch",
                             "graph1m", "laplace_bilinear", "gauge256"])
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--N", type=int, default=1024)
    ap.add_argument("--levels", type=int, default=6)
    ap.add_argument("--nb", type=int, default=128)
    ap.add_argument("--alloc", default="giles")
    ap.add_argument("--nu", type=int, default=2, help="poisson1024: sweeps before and after")
    ap.add_argument("--workers", type=int, default=4,
                    help="varcoef_batch: host workers (0: all problems grouped in lockstep "
                         "on one stream, one launch per V-cycle position; -1: the same with "
                         "one persistent launch per V-cycle)")
    ap.add_argument("--spin-split", action="store_true",
                    help="wilson*: spin-structure-preserving aggregation (Example 4.3)")
    ap.add_argument("--n-vec", type=int, default=0,
                    help="wilson*: test vectors per aggregate (0: 8, or 4 with --spin-split)")
    ap.add_argument("--narrow-fp64", type=int, default=0,
                    help="real operators: batches of at most this many columns solved in "
                         "plain FP64 inside the FP32 + refinement run")
    ap.add_argument("--top-cycles", type=int, default=0,
                    help="all but poisson1024: coarse-grid cycles below each solve's top "
                         "level (0: the library default)")
    ap.add_argument("--omega", type=float, default=0.0,
                    help="graph1m: coarse-correction scaling (0 = the library default)")
    ap.add_argument("--train-batches", type=int, default=80,
                    help="wilson512: plain solves used for training = this x nb")
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the comparison runs after the timed region")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-c4", action="store_true",
                    help="poisson1024: skip the learned-smoother (Wilson 512^2) comparison")
    ap.add_argument("--defl-scan", type=lambda s: [int(v) for v in s.split(",") if v],
                    default=[32, 64, 128],
                    help="poisson1024: n_defl values scanned for deflated Hutchinson "
                         "(empty: skip the comparison)")
    ap.add_argument("--c4-steps", type=int, default=5,
                    help="poisson1024: traces per variant in the learned-smoother comparison")
    ap.add_argument("--timing-stride", type=int, default=32,
                    help="bracket about one launch in k of the timed kernel with HIP events "
                         "(on the Poisson workload 1 in 8 took 1.5%% more time per trace "
                         "than 1 in 32)")
    ap.add_argument("--copy-check", action="store_true",
                    help="run one 256 MiB device copy first (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(MLMC samples shard across GPUs by sample index; not built here)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2108_11281_amd as m

    torch.cuda.set_device(0)
    if args.copy_check:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "poisson1024":
        run_poisson(args, m, torch)
    elif args.workload == "wilson256":
        run_wilson(args, m, torch, 256, learned=False)
    elif args.workload == "wilson512":
        run_wilson(args, m, torch, 512, learned=True)
    elif args.workload == "graph1m":
        run_graph(args, m, torch)
    elif args.workload == "laplace_bilinear":
        run_laplace_bilinear(args, m, torch)
    elif args.workload == "gauge256":
        run_gauge(args, m, torch)
    else:
        run_batch(args, m, torch)


if __name__ == "__main__":
    main()
