"""Benchmark of the EPWI SERTA hot path on one MI355X.

One step = one eph_scattering_rates call (grid tables, states, Re transform,
fused rate kernel) + one eph_conductivity call, on the Al-like 100^3 k x
100^3 q workload with the 100/300/500 K batch (synthetic inputs, seeded).

The three forms (FP64, FP32, BF16x3 transforms) are each timed for a few
steps; the headline is the fastest form whose sigma is within 1e-3 relative
of the FP64 sigma of the same run, timed for --steps after --warmup.

Prints ONE JSON line:
  value       (k,q) pairs with >= 1 kept term, per second of step time
  ms_per_step step time = the sigma wall time (rates + conductivity)
  roofline    the fused rate kernel of the headline form against its vector
              peak (FP64 78.6, FP32 157.3 TFLOP/s), with the flops of the
              algorithm it runs (from the call's own counts) over its
              HIP-event-timed duration; roofline_fp64 the same for FP64
  forms       every form's step time, speedup over FP64 and sigma error
  cpu_baseline the FP64 C oracle on a seeded sample of k points (all q),
              on all host threads and on one
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "(k,q) el-ph pair evals/s + σ wall time at ≤1e-3 rel σ error vs FP64"
# FP64 / FP32 vector peaks of MI355X; the rate kernel of the BF16x3 form runs in FP32
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 157.3}


# sources that define the rate-kernel instances (template, dispatch, instances)
KERNEL_SOURCES = ("rates_wave.h", "k_rates_wave.hip", "k_rates_wave_d3.hip", "k_rates_wave_s3.hip",
                  "k_rates_wave_d6.hip", "k_rates_wave_s6.hip", "dev_util.h", "internal.h")


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2306_16493_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload, precision):
    """HBM bytes per rate-kernel launch from the committed counter summary
    (profiles/rates_wave_traffic.json: FETCH_SIZE and WRITE_SIZE per dispatch,
    scaled by a copy kernel of known size), or None when no entry was taken
    on this workload and form with the present kernel sources."""
    path = os.path.join(ROOT, "profiles", "rates_wave_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        entries = json.load(f).get("entries", [])
    sha = kernel_source_sha()
    for t in entries:
        if t.get("source_sha256") == sha and t.get("workload") == workload and t.get("precision") == precision:
            return (t["fetch_kib_per_launch"] * 1024 * t["fetch_scale"] +
                    t["write_kib_per_launch"] * 1024 * t["write_scale"])
    return None


def rate_kernel_flops(counts, ns, N, box, C, nm, nw):
    """FP64 flops the fused rate kernel executes (8 per complex MAC):
    Y stage 8*ns*N*nbox*C, Z stage 8*ns*N^2*n1*n2*C, and per vertex
    contraction 8*(n1*nm*nw + n1*nm + nm*nm).  Transcendentals (delta,
    occupations) are not counted."""
    n1, n2, n3 = box
    y = 8.0 * ns * N * n1 * n2 * n3 * C
    z = 8.0 * ns * N * N * n1 * n2 * C
    v = 8.0 * counts["n_vertex"] * (n1 * nm * nw + n1 * nm + nm * nm)
    return y + z + v


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(system, w, mu, lo, hi, state_k, n_pick, n_pick_single=2):
    """The FP64 oracle's rate loop on a seeded sample of k points (all q),
    on all the threads its OpenMP runtime uses and on one thread."""
    import ctypes
    import numpy as np
    import oracle
    from oracle import Oracle
    o = Oracle(system)
    N = w.grid
    t0 = time.perf_counter()
    eps, evec, vel = o.electrons(N)
    om, u, _ = o.phonons(N)
    t_tables = time.perf_counter() - t0
    rng = np.random.default_rng(20240601)
    kall = np.unique(state_k)
    kpick = np.sort(rng.choice(kall, size=min(n_pick, kall.size), replace=False))
    sk, sn = o.select_states(eps, w.band_lo, w.band_hi, lo, hi, k_subset=kpick)
    threads = int(oracle.lib().orc_num_threads())
    t0 = time.perf_counter()
    r = o.rates(N, eps, evec, om, u, sk, sn, mu, w.temps, w.eta)
    t = time.perf_counter() - t0
    out = {"value": r["n_kq"] / t, "unit": "(k,q) pairs/s", "cores": threads, "kind": "oracle",
           "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
           "sample": f"{kpick.size} seeded k points ({sk.size} states, {r['n_kq']} (k,q) pairs, all {N}^3 q) of "
                     f"{w.name}; rate loop {t:.2f} s on {threads} threads; full-grid oracle tables "
                     f"{t_tables:.2f} s not counted"}
    # one thread, on the first k points of the same sample
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(1)
        k1 = kpick[:n_pick_single]
        sk1, sn1 = o.select_states(eps, w.band_lo, w.band_hi, lo, hi, k_subset=k1)
        t0 = time.perf_counter()
        r1 = o.rates(N, eps, evec, om, u, sk1, sn1, mu, w.temps, w.eta)
        t1 = time.perf_counter() - t0
        gomp.omp_set_num_threads(threads)
        out["single_thread"] = {"value": r1["n_kq"] / t1, "unit": "(k,q) pairs/s", "cores": 1,
                                "sample": f"{k1.size} of the same k points ({sk1.size} states, {r1['n_kq']} "
                                          f"(k,q) pairs); rate loop {t1:.2f} s"}
    except OSError:
        out["single_thread"] = None
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=None,
                    help="default al_fcc_100 (bench line), si_fcc_150 (--report precision), al_fcc_200 (--report "
                         "surrogate)")
    ap.add_argument("--grid", type=int, default=None)
    ap.add_argument("--precision", default="auto",
                    help="form of the headline: auto (the fastest within 1e-3 relative sigma error of the FP64 "
                         "run), fp64, fp32 or bf16x3")
    ap.add_argument("--cpu-sample", type=int, default=40, help="k points of the oracle sample (0 = skip)")
    ap.add_argument("--report", choices=["precision", "surrogate", "surrogate-sweep", "ablation", "full"], default=None,
                    help="instead of the bench line, measure the FP32/BF16x3 forms or the surrogate on "
                         "their own workloads (one JSON line)")
    ap.add_argument("--subset-frac", type=float, default=0.01, help="k-point fraction of --report precision")
    ap.add_argument("--train-fracs", default="0.01,0.02,0.05", help="training fractions of --report surrogate-sweep")
    ap.add_argument("--thresholds", default="0.01,0.02,0.05", help="spread thresholds of --report surrogate-sweep")
    ap.add_argument("--reference", default=None,
                    help="JSON with the sigma and time of the full plain run (--report surrogate-sweep; measured "
                         "when absent)")
    ap.add_argument("--only", choices=["fp64", "fp32", "bf16x3"], default=None,
                    help="time only this form for --steps after --warmup (no other forms, no oracle baseline) and "
                         "print its kernel times; for profiler runs")
    ap.add_argument("--source-sha", action="store_true", help="print the hash of the rate-kernel sources")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy 5 times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the rate path runs on one GPU; --gpus must be 1"}), flush=True)
        sys.exit(2)

    if args.source_sha:
        print(kernel_source_sha())
        return
    import numpy as np
    import torch
    if args.copy_calibration:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": 2 * x.numel() * 4, "launches": 5}), flush=True)
        return
    if args.report == "precision":
        from paper_2306_16493_amd import reports
        wl = args.workload or "si_fcc_150"
        print(json.dumps(reports.precision(wl, args.subset_frac, grid=args.grid)), flush=True)
        return
    if args.report == "surrogate-sweep":
        from paper_2306_16493_amd import reports
        ref = None
        if args.reference:
            with open(args.reference) as f:
                ref = json.load(f)
        fr = [float(x) for x in args.train_fracs.split(",") if x]
        th = [float(x) for x in args.thresholds.split(",") if x]
        prec = args.precision if args.precision != "auto" else "fp32"
        print(json.dumps(reports.surrogate_sweep(args.workload or "al_fcc_200", fr, th, grid=args.grid,
                                                 precision=prec, ref=ref)), flush=True)
        return
    if args.report == "full":
        from paper_2306_16493_amd import reports
        forms = ("fp32", "fp64") if args.precision == "auto" else (args.precision,)
        print(json.dumps(reports.full_run(args.workload or "si_fcc_150", forms, grid=args.grid)), flush=True)
        return
    if args.report == "ablation":
        from paper_2306_16493_amd import reports
        print(json.dumps(reports.ablation(args.workload or "al_fcc_100", grid=args.grid or 40)), flush=True)
        return
    if args.report == "surrogate":
        from paper_2306_16493_amd import reports
        wl = args.workload or "al_fcc_200"
        prec = args.precision if args.precision != "auto" else "fp32"
        print(json.dumps(reports.surrogate(wl, grid=args.grid, precision=prec)), flush=True)
        return
    from synth import make_system, workload
    from paper_2306_16493_amd import Context

    w = workload(args.workload or "al_fcc_100", args.grid)
    s = make_system(w.system)
    mu = s.mu_centroid
    lo, hi = mu + w.window[0], mu + w.window[1]
    ctx = Context(s, device=0)
    P = lambda prec: ctx.params(w.grid, mu, w.temps, w.eta, lo, hi, w.band_lo, w.band_hi, precision=prec)
    ns = ctx.count_states(P("fp64"))
    ctx.set_profiling(True)
    say = lambda m: print(m, file=sys.stderr, flush=True)
    say(f"[bench] {w.name} N={w.grid} states={ns}")
    bufs = {}

    def timed(prec, warmup, steps):
        """warmup + steps of one form (rates call + conductivity); per-step
        wall times, the last call's result and sigma, mean kernel times."""
        p = P(prec)
        res = sig = None
        for i in range(warmup):
            res, bufs[prec] = ctx.scattering_rates(p, capacity=ns, buffers=bufs.get(prec))
            ctx.conductivity(res.energy, res.vel, res.inv_tau.reshape(-1), mu, w.temps, w.grid ** 3)
            say(f"[bench] {prec} warmup {i} done")
        torch.cuda.synchronize()
        rates_ms, xform_ms, launches, step_s = [], [], 0, []
        t0 = time.perf_counter()
        for i in range(steps):
            ts = time.perf_counter()
            res, bufs[prec] = ctx.scattering_rates(p, capacity=ns, buffers=bufs.get(prec))
            sig = ctx.conductivity(res.energy, res.vel, res.inv_tau.reshape(-1), mu, w.temps, w.grid ** 3)
            torch.cuda.synchronize()
            step_s.append(time.perf_counter() - ts)
            st = ctx.stage_times()
            rates_ms.append(st["rates_ms"])
            xform_ms.append(st["xform_ms"])
            launches += st["rates_launches"]
            say(f"[bench] {prec} step {i}: call {st['call_ms']:.1f} ms (tables {st['tables_ms']:.1f}, prep "
                f"{st['prep_ms']:.1f}, xform {st['xform_ms']:.1f}, rates {st['rates_ms']:.1f})")
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        return dict(t=t, step_s=step_s, res=res, sig=sig, rates_ms=float(np.mean(rates_ms)),
                    xform_ms=float(np.mean(xform_ms)), launches=launches / steps, st=st)

    if args.only:
        one = timed(args.only, args.warmup, args.steps)
        print(json.dumps({"only": args.only, "workload": w.name, "grid": w.grid, "steps": args.steps,
                          "ms_per_step": one["t"] * 1e3, "rates_ms": one["rates_ms"], "xform_ms": one["xform_ms"],
                          "rate_launches_per_step": one["launches"],
                          "avg_rate_launch_ms": one["rates_ms"] / one["launches"],
                          "n_kq": one["res"].counts["n_kq"]}), flush=True)
        ctx.close()
        return
    # the FP64 path (the reference of the sigma error), then the reduced
    # forms; the headline is the fastest form within 1e-3 relative sigma
    # error of the FP64 run, timed for the requested steps
    side = max(1, min(args.steps, 3))
    forms = {"fp64": timed("fp64", 1, side)}
    sig64 = forms["fp64"]["sig"]
    for prec in ("fp32", "bf16x3"):
        forms[prec] = timed(prec, 1, side)
        forms[prec]["sigma_err"] = float(np.max(np.abs(forms[prec]["sig"] - sig64)) / np.max(np.abs(sig64)))
    forms["fp64"]["sigma_err"] = 0.0
    ok = [f for f in forms if forms[f]["sigma_err"] <= 1e-3]
    head = args.precision if args.precision != "auto" else min(ok, key=lambda f: forms[f]["t"])
    say(f"[bench] headline form {head}: " + ", ".join(f"{f} {forms[f]['t']:.3f} s (sigma err "
                                                      f"{forms[f]['sigma_err']:.1e})" for f in forms))
    hd = timed(head, args.warmup, args.steps)
    sig = hd["sig"]
    hd["sigma_err"] = float(np.max(np.abs(sig - sig64)) / np.max(np.abs(sig64)))
    res = hd["res"]
    t = hd["t"]
    counts = res.counts
    nm, nw = 3 * s.na, s.nw
    box = [len(np.unique(s.rp[:, a])) for a in range(3)]
    flops = rate_kernel_flops(counts, ns, w.grid, box, nm * nw, nm, nw)
    achieved = flops / (hd["rates_ms"] / 1e3) / 1e12
    peak = PEAK_TFLOPS[head]
    n_launch = hd["launches"]
    st = hd["st"]
    out = {
        "metric": METRIC,
        "value": counts["n_kq"] / t,
        "unit": "(k,q) pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t * 1e3,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3+f32"}[head],
        "data": "synthetic",
        "config": {"workload": w.name, "grid": w.grid, "temps_K": list(w.temps), "eta_eV": w.eta,
                   "window_eV": [lo, hi], "precision": head, "n_states": ns,
                   "n_kq": counts["n_kq"], "n_nkq": counts["n_nkq"], "n_terms": counts["n_terms"],
                   "n_vertex": counts["n_vertex"]},
        "sigma_wall_s": t,
        "sigma_rel_err_vs_fp64": hd["sigma_err"],
        "ms_per_step_median": float(np.median(hd["step_s"])) * 1e3,
        "sigma_S_per_m_xx": [float(sig[i, 0, 0]) for i in range(sig.shape[0])],
        "stages_ms": {"tables": st["tables_ms"], "prep": st["prep_ms"], "xform": hd["xform_ms"],
                      "rates": hd["rates_ms"], "call": st["call_ms"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": measured_traffic(w.name, head),
                     "kernel": "rates_wave_kernel", "flops_per_step": flops, "launches_per_step": n_launch,
                     "avg_launch_ms": hd["rates_ms"] / n_launch, "flops_per_launch": flops / n_launch},
        "forms": {f: {"ms_per_step": forms[f]["t"] * 1e3, "value": forms[f]["res"].counts["n_kq"] / forms[f]["t"],
                      "speedup_vs_fp64": forms["fp64"]["t"] / forms[f]["t"],
                      "sigma_rel_err_vs_fp64": forms[f]["sigma_err"], "rates_ms": forms[f]["rates_ms"],
                      "xform_ms": forms[f]["xform_ms"], "steps": side} for f in forms},
    }
    out["roofline_fp64"] = {"achieved": flops / (forms["fp64"]["rates_ms"] / 1e3) / 1e12, "peak": PEAK_TFLOPS["fp64"],
                            "frac": flops / (forms["fp64"]["rates_ms"] / 1e3) / 1e12 / PEAK_TFLOPS["fp64"],
                            "unit": "TFLOP/s"}
    if args.cpu_sample > 0:
        say("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(s, w, mu, lo, hi, res.state_k.cpu().numpy(), args.cpu_sample)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
