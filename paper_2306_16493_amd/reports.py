"""Measurements beside the bench line (host-side orchestration only; every
number comes from the HIP path through the C ABI).

precision():       the FP32 and split-BF16x3 forms against the FP64 GPU path
                   (which the parity tests tie to the FP64 oracle) on a
                   seeded subset of the k points that carry states: per-state
                   1/tau and sigma errors, and each form's speedup.
surrogate():       the MLP-ensemble surrogate with plain fallback against the
                   full plain run on the same grid: sigma error and
                   end-to-end speedup.
surrogate_sweep(): the same over training fractions and spread thresholds,
                   against one full plain run.
full_run():        one or two forms over every window state of a workload.
ablation():        the k-batch order of the vertex and the state-batch size
                   of the q-batch kernel (Sec. III.D, Sec. IV.C).

Each prints progress lines and returns one dict (bench.py prints it as
JSON).
"""
from __future__ import annotations

import time

import numpy as np


def _log(msg):
    print(msg, flush=True)


def window(ctx, system, w, N):
    """(mu, win_lo, win_hi) of a workload: relative to mu (metals, mu = band
    centroid) or to the conduction-band minimum found on the grid (the
    semiconductor, mu = CBM - 0.25 eV)."""
    if w.window_relative_to == "mu":
        mu = system.mu_centroid
        return mu, mu + w.window[0], mu + w.window[1]
    # lowest energy of band band_lo over the grid, from the library's own state list
    p = ctx.params(N, 0.0, [300.0], w.eta, -1e6, 1e6, band_lo=w.band_lo, band_hi=w.band_lo)
    _, _, e, _ = ctx.select_states(p)
    cbm = float(e.min().item())
    mu = cbm - 0.25 if w.mu_rule == "cbm-0.25" else system.mu_centroid
    # 1e-7 eV below the CBM, so that the CBM state itself is inside the window
    return mu, cbm + w.window[0] - 1e-7, cbm + w.window[1]


def _timed_rates(ctx, params):
    import torch
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, _ = ctx.scattering_rates(params)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = ctx.stage_times()
    return res, wall, st


def precision(workload_name="si_fcc_150", subset_frac=0.01, seed=1649307, grid=None):
    from synth import make_system, workload
    from .eph import Context
    w = workload(workload_name, grid)
    s = make_system(w.system)
    ctx = Context(s, device=0)
    N = w.grid
    mu, lo, hi = window(ctx, s, w, N)
    p_all = ctx.params(N, mu, w.temps, w.eta, lo, hi, w.band_lo, w.band_hi)
    sk, _, _, _ = ctx.select_states(p_all)
    kall = np.unique(sk.cpu().numpy())
    rng = np.random.default_rng(seed)
    nk = max(1, int(round(subset_frac * kall.size)))
    ksub = np.sort(rng.choice(kall, size=nk, replace=False))
    _log(f"[precision] {w.name} N={N}: {sk.shape[0]} states at {kall.size} k points; subset {nk} k points")
    out = {"report": "precision", "workload": w.name, "grid": N, "n_states_total": int(sk.shape[0]),
           "subset_k_points": int(nk), "subset_seed": seed, "forms": {}}
    ref = None
    for prec in ("fp64", "fp32", "bf16x3"):
        p = ctx.params(N, mu, w.temps, w.eta, lo, hi, w.band_lo, w.band_hi, precision=prec, k_subset=ksub)
        _timed_rates(ctx, p)  # warm-up (tables, lazy FP32/BF16 copies)
        res, wall, st = _timed_rates(ctx, p)
        sig = ctx.conductivity(res.energy, res.vel, res.inv_tau.reshape(-1), mu, w.temps, N ** 3)
        it = res.inv_tau.cpu().numpy()
        entry = {"call_s": wall, "rates_ms": st["rates_ms"], "xform_ms": st["xform_ms"],
                 "n_states": int(res.counts["n_states"]), "n_kq": int(res.counts["n_kq"]),
                 "n_vertex": int(res.counts["n_vertex"]), "pairs_per_s": res.counts["n_kq"] / wall,
                 "sigma_xx": [float(sig[t, 0, 0]) for t in range(sig.shape[0])]}
        if prec == "fp64":
            ref = (it, sig, wall, res.counts)
        else:
            it0, sig0, wall0, c0 = ref
            pos = it0 > 0
            rel = np.abs(it[pos] - it0[pos]) / it0[pos]
            entry.update({"inv_tau_max_rel_err": float(rel.max()) if rel.size else 0.0,
                          "inv_tau_median_rel_err": float(np.median(rel)) if rel.size else 0.0,
                          "sigma_rel_err": float(np.max(np.abs(sig - sig0)) / np.max(np.abs(sig0))),
                          "counts_equal": bool(res.counts["n_kq"] == c0["n_kq"]
                                               and res.counts["n_terms"] == c0["n_terms"]),
                          "speedup_vs_fp64": wall0 / wall})
        out["forms"][prec] = entry
        _log(f"[precision] {prec}: {wall:.2f} s, rates {st['rates_ms']:.0f} ms"
             + (f", 1/tau max rel err {entry['inv_tau_max_rel_err']:.2e}, sigma rel err "
                f"{entry['sigma_rel_err']:.2e}, speedup {entry['speedup_vs_fp64']:.2f}x" if prec != "fp64" else ""))
    ctx.close()
    return out


def surrogate(workload_name="al_fcc_200", train_frac=0.02, chunks=8, threshold=0.01, members=5,
              steps=30000, batch=512, decay=True, seed=1649307, grid=None, precision="fp64"):
    """The surrogate run, then the plain kernel on every k point the
    surrogate did not already compute with it (the full plain run is the
    union of these disjoint k-subset runs: its 1/tau is the reference and its
    time is the sum of their times)."""
    import torch
    from synth import make_system, workload
    from .eph import Context, merge_rates
    from . import surrogate as sg
    w = workload(workload_name, grid)
    s = make_system(w.system)
    ctx = Context(s, device=0)
    N = w.grid
    mu, lo, hi = window(ctx, s, w, N)
    temps = list(w.temps)
    P = lambda ks: ctx.params(N, mu, temps, w.eta, lo, hi, w.band_lo, w.band_hi, precision=precision, k_subset=ks)
    # ---- surrogate with fallback ----
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r = sg.run(ctx, N, mu, temps, w.eta, lo, hi, w.band_lo, w.band_hi, train_frac=train_frac, members=members,
               steps=steps, batch=batch, threshold=threshold, seed=seed, precision=precision, log=_log, decay=decay)
    torch.cuda.synchronize()
    t_sur = time.perf_counter() - t1
    _log(f"[surrogate] surrogate run {t_sur:.1f} s: {r.times}")
    sk, sn, se, sv = r.states
    # ---- plain kernel on the remaining k points, in chunks ----
    kall = np.unique(sk.cpu().numpy())
    done = np.union1d(r.train_k, r.fallback_k)
    rest = np.setdiff1d(kall, done)
    ref = r.inv_tau.clone()  # plain values at the training and fallback k points
    t_rest = 0.0
    parts = [x for x in np.array_split(rest, chunks) if x.size]
    for i, ks in enumerate(parts):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, _ = ctx.scattering_rates(P(ks))
        torch.cuda.synchronize()
        t_rest += time.perf_counter() - t0
        merge_rates(ctx, sk, sn, ref, res.state_k, res.state_n, res.inv_tau)
        _log(f"[surrogate] plain chunk {i + 1}/{len(parts)}: {res.counts['n_states']} states, {t_rest:.1f} s")
    sig_ref = ctx.conductivity(se, sv, ref.reshape(-1), mu, temps, N ** 3)
    t_plain = t_rest + r.times["train_rates_s"] + r.times["fallback_s"] + r.times["select_s"]
    err = float(np.max(np.abs(r.sigma - sig_ref)) / np.max(np.abs(sig_ref)))
    sig_net = ctx.conductivity(se, sv, r.raw_inv_tau.reshape(-1), mu, temps, N ** 3)
    err_net = float(np.max(np.abs(sig_net - sig_ref)) / np.max(np.abs(sig_ref)))
    out = {"report": "surrogate", "workload": w.name, "grid": N, "precision": precision,
           "n_states": int(r.n_states), "k_points": int(kall.size), "train_k_points": int(r.n_train_k),
           "train_states": int(r.n_train_states), "flagged_states": int(r.n_flagged),
           "fallback_k_points": int(r.n_fallback_k), "threshold": threshold, "members": members,
           "train_steps": steps, "member_loss": [float(x) for x in r.loss], "plain_s": t_plain,
           "surrogate_s": t_sur, "speedup": t_plain / t_sur, "sigma_rel_err": err,
           "sigma_rel_err_network_only": err_net, "stage_s": r.times,
           "plain_time_note": "sum of the plain-kernel runs over disjoint k subsets covering every k point"}
    _log(f"[surrogate] plain {t_plain:.1f} s, surrogate {t_sur:.1f} s (speedup {t_plain / t_sur:.2f}x), flagged "
         f"{r.n_flagged}/{r.n_states}, sigma rel err {err:.2e} (network only {err_net:.2e})")
    ctx.close()
    return out


def surrogate_sweep(workload_name="al_fcc_200", train_fracs=(0.01, 0.02, 0.05), thresholds=(0.01, 0.02, 0.05),
                    members=5, steps=30000, batch=512, decay=True, seed=1649307, grid=None, precision="fp32",
                    ref=None, chunks=8):
    """The surrogate over training fractions and spread thresholds against
    one full plain run.  The plain run (unless `ref` gives its sigma and
    time) is timed over disjoint k-point chunks; the table time every chunk
    call repeats is taken off all but one.  Per training fraction the
    ensemble is fitted once; per threshold the blend, the plain fallback and
    sigma are timed on their own, so each setting's time is selection +
    training rates + fit + prediction + blend + fallback."""
    import torch
    from synth import make_system, workload
    from .eph import Context, merge_rates
    from . import surrogate as sg
    w = workload(workload_name, grid)
    s = make_system(w.system)
    ctx = Context(s, device=0)
    N = w.grid
    mu, lo, hi = window(ctx, s, w, N)
    temps = list(w.temps)
    P = lambda ks: ctx.params(N, mu, temps, w.eta, lo, hi, w.band_lo, w.band_hi, precision=precision, k_subset=ks)
    out = {"report": "surrogate_sweep", "workload": w.name, "grid": N, "precision": precision, "members": members,
           "train_steps": steps, "batch": batch, "lr_decay": list(sg.DECAY) if decay else None, "settings": []}
    if ref is None:
        ctx.set_profiling(True)
        sk, sn, se, sv = ctx.select_states(P(None))
        kall = np.unique(sk.cpu().numpy())
        inv = torch.zeros((len(temps), sk.shape[0]), dtype=torch.float64, device=sk.device)
        t_sum, t_tab = 0.0, []
        parts = [x for x in np.array_split(kall, chunks) if x.size]
        for i, ks in enumerate(parts):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res, _ = ctx.scattering_rates(P(ks))
            torch.cuda.synchronize()
            t_sum += time.perf_counter() - t0
            t_tab.append(ctx.stage_times()["tables_ms"] / 1e3)
            merge_rates(ctx, sk, sn, inv, res.state_k, res.state_n, res.inv_tau)
            _log(f"[sweep] plain chunk {i + 1}/{len(parts)}: {res.counts['n_states']} states, {t_sum:.1f} s")
        sig_ref = ctx.conductivity(se, sv, inv.reshape(-1), mu, temps, N ** 3)
        ref = {"sigma": sig_ref.tolist(), "plain_s": t_sum - sum(t_tab[1:]), "plain_chunks_s": t_sum,
               "tables_s_per_call": float(np.mean(t_tab)), "n_states": int(sk.shape[0]), "k_points": int(kall.size)}
        del inv
        _log(f"[sweep] plain run {ref['plain_s']:.1f} s ({t_sum:.1f} s over {len(parts)} chunk calls)")
    out["reference"] = ref
    sig_ref = np.asarray(ref["sigma"])
    scale = np.max(np.abs(sig_ref))
    for tf in train_fracs:
        f = sg.fit(ctx, N, mu, temps, w.eta, lo, hi, w.band_lo, w.band_hi, train_frac=tf, members=members,
                   steps=steps, batch=batch, seed=seed, precision=precision, log=_log, decay=decay)
        for th in thresholds:
            r = sg.finish(f, th, log=_log)
            sk, sn, se, sv = r.states
            err = float(np.max(np.abs(r.sigma - sig_ref)) / scale)
            sig_net = ctx.conductivity(se, sv, r.raw_inv_tau.reshape(-1), mu, temps, N ** 3)
            err_net = float(np.max(np.abs(sig_net - sig_ref)) / scale)
            t = r.times["total_s"]
            row = {"train_frac": tf, "threshold": th, "n_states": int(r.n_states), "train_k_points": int(r.n_train_k),
                   "flagged_states": int(r.n_flagged), "flagged_frac": r.n_flagged / r.n_states,
                   "fallback_k_points": int(r.n_fallback_k), "sigma_rel_err": err,
                   "sigma_rel_err_network_only": err_net, "surrogate_s": t, "speedup": ref["plain_s"] / t,
                   "member_loss": [float(x) for x in r.loss], "stage_s": r.times}
            out["settings"].append(row)
            _log(f"[sweep] train {tf:.0%} threshold {th:.0%}: flagged {row['flagged_frac']:.1%}, sigma err {err:.2e} "
                 f"(network only {err_net:.2e}), {t:.1f} s, speedup {row['speedup']:.2f}x")
        f.mlp.close()
    ctx.close()
    return out


def full_run(workload_name="si_fcc_150", precisions=("fp32", "fp64"), chunks=10, grid=None):
    """One form over every window state of a workload: the plain rates call
    over disjoint k-point chunks (so that each call ends within a minute or
    so and reports), then sigma from all of them.  Per form: the sum of the
    chunk calls less the grid-table time that every chunk after the first
    repeats, pairs per second, sigma, and sigma's error against the first
    form."""
    import torch
    from synth import make_system, workload
    from .eph import Context, merge_rates
    w = workload(workload_name, grid)
    s = make_system(w.system)
    ctx = Context(s, device=0)
    N = w.grid
    mu, lo, hi = window(ctx, s, w, N)
    temps = list(w.temps)
    out = {"report": "full", "workload": w.name, "grid": N, "forms": {}}
    ctx.set_profiling(True)
    P = lambda prec, ks: ctx.params(N, mu, temps, w.eta, lo, hi, w.band_lo, w.band_hi, precision=prec, k_subset=ks)
    sk, sn, se, sv = ctx.select_states(P("fp64", None))
    kall = np.unique(sk.cpu().numpy())
    out["n_states"] = int(sk.shape[0])
    out["k_points"] = int(kall.size)
    parts = [x for x in np.array_split(kall, chunks) if x.size]
    sig0 = None
    for prec in precisions:
        inv = torch.zeros((len(temps), sk.shape[0]), dtype=torch.float64, device=sk.device)
        t_sum, t_tab, n_kq, rates_ms = 0.0, [], 0, 0.0
        for i, ks in enumerate(parts):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res, _ = ctx.scattering_rates(P(prec, ks))
            torch.cuda.synchronize()
            t_sum += time.perf_counter() - t0
            st = ctx.stage_times()
            t_tab.append(st["tables_ms"] / 1e3)
            rates_ms += st["rates_ms"]
            n_kq += int(res.counts["n_kq"])
            merge_rates(ctx, sk, sn, inv, res.state_k, res.state_n, res.inv_tau)
            _log(f"[full] {w.name} {prec} chunk {i + 1}/{len(parts)}: {res.counts['n_states']} states, {t_sum:.1f} s")
        sig = ctx.conductivity(se, sv, inv.reshape(-1), mu, temps, N ** 3)
        t = t_sum - sum(t_tab[1:])
        row = {"call_s": t, "chunk_calls_s": t_sum, "rates_s": rates_ms / 1e3, "tables_s_per_call": float(np.mean(t_tab)),
               "n_kq": n_kq, "pairs_per_s": n_kq / t, "sigma": sig.tolist()}
        if sig0 is None:
            sig0 = sig
        else:
            row["sigma_rel_err_vs_first"] = float(np.max(np.abs(sig - sig0)) / np.max(np.abs(sig0)))
        out["forms"][prec] = row
        _log(f"[full] {w.name} {prec}: {t:.1f} s, {n_kq / t:.3e} (k,q) pairs/s")
        del inv
    ctx.close()
    return out


def _budget_parts(ctx, N, mu, w, lo, hi):
    """(fixed bytes, bytes per state of a batch, states per group) of a rates
    call, from the minimum that too small a mem_budget_bytes reports."""
    import re
    from .eph import EphError
    msg = ""
    for b in (1, None):
        try:
            bb = b if b is not None else int(re.search(r"\((\d+) bytes\)", msg).group(1)) + 1
            ctx.count_states(ctx.params(N, mu, w.temps, w.eta, lo, hi, w.band_lo, w.band_hi))
            ctx.scattering_rates(ctx.params(N, mu, w.temps, w.eta, lo, hi, w.band_lo, w.band_hi,
                                            mem_budget_bytes=bb))
        except EphError as e:
            msg = str(e)
    m = re.search(r"\((\d+) bytes of tables and lists plus (\d+) bytes per state of a batch, (\d+) states", msg)
    return int(m.group(1)), int(m.group(2)), int(m.group(3))


def ablation(workload_name="al_fcc_100", grid=40, q_batches=(16, 64, 256, 1024, 4096),
             state_batches=(64, 256, 1024, 4096, 16384, None)):
    """The comparison of Sec. III.D and the batch-size study of Sec. IV.C on
    this GPU: the q-batch rate kernel against the k-batch order of the same
    sum (eph_rates_kbatch) for several q-batch sizes, and the q-batch kernel
    for several numbers of states per batch (mem_budget_bytes).  Per run:
    time of the rates call and of its kernels, launches, (k,q) pairs per
    second; the k-batch rates are checked against the q-batch ones."""
    import torch
    from synth import make_system, workload
    from .eph import Context
    w = workload(workload_name, grid)
    s = make_system(w.system)
    ctx = Context(s, device=0)
    N = w.grid
    mu, lo, hi = window(ctx, s, w, N)
    out = {"report": "ablation", "workload": w.name, "grid": N, "q_batch": {}, "state_batch": {}}
    p = ctx.params(N, mu, w.temps, w.eta, lo, hi, w.band_lo, w.band_hi)
    _timed_rates(ctx, p)
    ref, wall, st = _timed_rates(ctx, p)
    n_kq = int(ref.counts["n_kq"])
    it_ref = ref.inv_tau.cpu().numpy()
    nw, nm = s.nw, 3 * s.na
    nbox = s.rp.shape[0]
    nre = s.re.shape[0]
    out["n_states"] = int(ref.counts["n_states"])
    out["n_kq"] = n_kq
    out["n_nkq"] = int(ref.counts["n_nkq"])
    # inner-product volume of the third step (complex MACs), Sec. III.D
    out["volume_q_batch_cmac"] = float(ref.counts["n_nkq"]) * nw * nm * nbox
    out["volume_k_batch_cmac"] = float(n_kq) * nw * nw * nre * nm
    out["q_batch_order"] = {"call_s": wall, "rates_ms": st["rates_ms"], "xform_ms": st["xform_ms"],
                            "launches": st["rates_launches"] + st["xform_launches"], "pairs_per_s": n_kq / wall}
    _log(f"[ablation] {w.name} N={N}: {out['n_states']} states, {n_kq} (k,q) pairs; q-batch order {wall:.3f} s")
    for qb in q_batches:
        pk = ctx.params(N, mu, w.temps, w.eta, lo, hi, w.band_lo, w.band_hi)
        ctx.set_profiling(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kb, _ = ctx.rates_kbatch(pk, q_batch=qb)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        stk = ctx.stage_times()
        err = float(np.max(np.abs(kb.inv_tau.cpu().numpy() - it_ref)) / np.max(np.abs(it_ref)))
        out["q_batch"][str(qb)] = {"call_s": t, "step1_ms": stk["xform_ms"], "step2_ms": stk["rates_ms"],
                                   "launches": 2 * stk["rates_launches"], "pairs_per_s": n_kq / t,
                                   "slowdown_vs_q_batch_order": t / wall, "inv_tau_rel_diff": err}
        _log(f"[ablation] k-batch order, {qb} q per batch: {t:.3f} s ({t / wall:.1f}x), 1/tau diff {err:.1e}")
    fixed, per_state, gmax = _budget_parts(ctx, N, mu, w, lo, hi)
    for sb in state_batches:
        budget = 0 if sb is None else fixed + per_state * max(sb, gmax)
        pb = ctx.params(N, mu, w.temps, w.eta, lo, hi, w.band_lo, w.band_hi, mem_budget_bytes=budget)
        _timed_rates(ctx, pb)
        r2, t2, st2 = _timed_rates(ctx, pb)
        same = bool(np.array_equal(r2.inv_tau.cpu().numpy(), it_ref))
        key = "all" if sb is None else str(sb)
        out["state_batch"][key] = {"call_s": t2, "rates_ms": st2["rates_ms"], "batches": st2["xform_launches"],
                                   "launches": st2["rates_launches"] + st2["xform_launches"],
                                   "pairs_per_s": n_kq / t2, "relative_time": t2 / wall, "bitwise_equal": same}
        _log(f"[ablation] q-batch order, states per batch {key}: {t2:.3f} s in {st2['xform_launches']} batches")
    ctx.close()
    return out
