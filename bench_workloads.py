"""The non-default measurement configurations of ``bench.py``.

  direct    Plummer sphere N = 4096 (eps = 0.01): direct summation in FP64 and
            with FP32 pair terms; time, pairs/s, error against the oracle.
  adaptive  64 Plummer clumps, N = 2^22 (eps = 1e-3, theta = 0.7 with the
            offset-aware opening test, eta = 0.01):
            the integrator of ``driver.py`` for q_f in {0, 1/8, 1/4, 1/2, 1}
            (q_f = 0 is the every-step scheme); force evaluations, gravity
            and total GPU time, and the error of the force actually used
            (fresh or predicted) against the oracle at sampled steps.
  batched   256 Plummer systems of 1k-64k particles with 1-100% active
            (eps = 0.01, theta = 0.5): one batched build and one persistent
            walk recorded in a HIP graph and replayed; walk options from the
            autotuner; error on 64 sampled targets per system.
  adjoint   uniform sphere N = 2^18 (eps = 1e-3, theta = 0.6), Gaussian w:
            forward and adjoint walks, errors against the oracle gradient.
  periodic  periodic cube with one collapsing plane-wave mode (the pancake
            geometry of the paper's cosmological test), 64^3 and 128^3
            particles, every pair at its nearest image; build + walk time,
            evaluations/s and errors against the oracle on sampled targets.
  softening N = 2^20 turbulent sphere with a softening length per particle
            (the distance to the 32nd neighbour) against the same step with
            one length: time, interactions and error against the oracle.
  build     the tree build alone on the 2^22 clumps and the 2^20 turbulent
            sphere (n_leaf = 16): time per build and its algorithmic bytes.
  copy      a plain device copy of 1 GiB, the calibration of the HBM byte
            counters (FETCH_SIZE, WRITE_SIZE) used for the walk's traffic.
Inputs are seeded synthetic particle sets standing in for the paper's
hydro test problems.
"""
from __future__ import annotations

import statistics
import sys
import time

import numpy as np
import torch

import workloads
import paper_2010_13792_amd as ag
from paper_2010_13792_amd import autotune
from paper_2010_13792_amd.driver import AdaptiveIntegrator

DEV = torch.device("cuda:0")
DIRECT_PP_FLOPS = 60                 # pair_interact as written
PP_FLOPS, PN_FLOPS = 57, 179         # the walk's pair and node interactions as written
PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12   # FP64 vector and unpacked FP32 FMA issue rate


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _t(a, dtype=None):
    return torch.tensor(a, device=DEV) if dtype is None else torch.tensor(a, dtype=dtype, device=DEV)


def _events():
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _rel(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


# ---------------------------------------------------------------------------
def run_direct(args):
    import oracle
    n, eps = 4096, 0.01
    x, v, m = workloads.plummer(n, seed=1)
    tx, tv, tm = _t(x), _t(v), _t(m)
    acc = torch.zeros((n, 3), dtype=torch.float64, device=DEV)
    jerk, tid = torch.zeros_like(acc), torch.zeros((n, 6), dtype=torch.float64, device=DEV)
    ar, jr, tr = oracle.direct(x, v, m, eps, 1.0)
    out = {"workload": "direct Plummer N=4096 eps=0.01", "pairs": n * (n - 1)}
    with ag.Context(0) as c:
        for name, prec in (("fp64", ag.AG_FP64), ("fp32_pairs", ag.AG_FP32_PAIRS)):
            for _ in range(3):
                c.grav_direct(tx, tv, tm, None, eps, 1.0, acc, jerk, tid, precision=prec)
            torch.cuda.synchronize()
            e0, e1 = _events()
            reps = 20
            e0.record()
            for _ in range(reps):
                c.grav_direct(tx, tv, tm, None, eps, 1.0, acc, jerk, tid, precision=prec)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            err = _rel(acc.cpu().numpy(), ar)
            out[name] = {"ms": ms, "pairs_per_s": n * (n - 1) / (ms * 1e-3), "evals_per_s": n / (ms * 1e-3),
                         "tflops": n * (n - 1) * DIRECT_PP_FLOPS / (ms * 1e-3) / 1e12,
                         "frac_of_peak": n * (n - 1) * DIRECT_PP_FLOPS / (ms * 1e-3) / 1e12 / PEAK_TFLOPS,
                         "median_rel_err": float(np.median(err)), "max_rel_err": float(err.max())}
    t_a = time.perf_counter()
    oracle.direct(x, v, m, eps, 1.0)
    t_o = time.perf_counter() - t_a
    out["cpu_baseline"] = {"value": n / t_o, "unit": "force evals/s", "cores": oracle.num_threads(),
                           "kind": "oracle", "sample": f"all {n} targets"}
    return out


# ---------------------------------------------------------------------------
def adaptive_comparison(n=1 << 22, steps=200, qs=(0.0, 0.125, 0.25, 0.5, 1.0), step_shift=0,
                        predictors=("jerk",), rebuild_every=1, mac_offset=1, n_rows=4096, checkpoints=None,
                        graph=False, group_span=None):
    """The C3 comparison: the integrator of ``driver.py`` on 64 Plummer clumps
    for every q_f of ``qs`` (0 = every step), eager steps with per-phase GPU
    timing; the median error of the force in use against the oracle on
    ``n_rows`` sampled particles at ``checkpoints``.  With ``graph`` each run
    is repeated with one captured step replayed for every step (its total
    time only; a graph carries no phase timing)."""
    import oracle
    log(f"adaptive: generating {n} particles in 64 clumps")
    x, v, m, _ = workloads.clumps(n, seed=3)
    tx, tv, tm = _t(x), _t(v), _t(m)
    rng = np.random.default_rng(33)
    rows = rng.choice(n, n_rows, replace=False)
    if checkpoints is None:
        checkpoints = sorted({0, steps // 4, steps // 2, 3 * steps // 4, steps})
    # targets per walk group: autotuned on the initial particle set, all active
    with ag.Context(0) as c:
        c.set_option(ag.AG_OPT_MAC_OFFSET, mac_offset)
        c.tree_build(tx, tv, tm, 16)
        acc = torch.zeros((n, 3), dtype=torch.float64, device=DEV)
        jerk, tid = torch.zeros_like(acc), torch.zeros((n, 6), dtype=torch.float64, device=DEV)

        def trial(p):
            c.set_option(ag.AG_OPT_GROUP_TARGETS, p["group_targets"])
            c.timing_enable(True)
            c.timing_read(reset=True)
            c.grav_eval(None, 0.7, 1e-3, 1.0, acc, jerk, tid)
            ph = c.timing_read(reset=True)
            c.timing_enable(False)
            return ph["groups"]["ms"] + ph["walk"]["ms"]

        tuned, tune_table = autotune.tune(trial, autotune.grid(group_targets=[64, 32]), f"clumps|n={n}",
                                          reps=2, use_cache=False)
        del acc, jerk, tid
    log(f"adaptive: autotuner picked {tuned}")
    preds = list(predictors)
    plan = [(preds[0], q) for q in qs] + [(p, q) for p in preds[1:] for q in qs if q > 0]
    runs = {}
    for pred, q in plan:
        kw = dict(q_f=q, theta=0.7, eps=1e-3, eta=0.01, rebuild_every=rebuild_every, step_shift=step_shift,
                  predictor=pred)
        with ag.Context(0) as c:
            c.set_option(ag.AG_OPT_MAC_OFFSET, mac_offset)
            c.set_option(ag.AG_OPT_GROUP_TARGETS, tuned["group_targets"])
            if group_span is not None:
                c.set_option(ag.AG_OPT_GROUP_SPAN, group_span)
            integ = AdaptiveIntegrator(c, tx, tv, tm, **kw)
            c.sync()
            errs = {}
            pooled = []

            def check(step):
                xs = integ.x.cpu().numpy()
                vs = integ.vpred.cpu().numpy() if step > 0 else integ.v.cpu().numpy()
                ar, _, _ = oracle.direct(xs, vs, m, 1e-3, 1.0, rows)
                e = _rel(integ.acc.cpu().numpy()[rows], ar)
                errs[step] = float(np.median(e))
                pooled.append(e)
                log(f"adaptive {pred} q_f={q} step {step}: median error of the force in use {errs[step]:.2e}")

            if 0 in checkpoints:
                check(0)
            c.timing_enable(True)
            c.timing_read(reset=True)
            ev0, ev1 = _events()
            total_ms = 0.0
            active_hist = []
            for s in range(1, steps + 1):
                ev0.record()
                integ.step()
                ev1.record()
                torch.cuda.synchronize()
                total_ms += ev0.elapsed_time(ev1)
                active_hist.append(integ.active_count())
                if s in checkpoints:
                    check(s)
            ph = c.timing_read(reset=True)
            c.timing_enable(False)
            grav_ms = ph["build"]["ms"] + ph["groups"]["ms"] + ph["walk"]["ms"]
            runs[(pred, q)] = {"evaluations": int(integ.evaluations - n), "gravity_ms": grav_ms,
                               "walk_ms": ph["walk"]["ms"], "build_ms": ph["build"]["ms"],
                               "total_ms": total_ms, "median_rel_err_used_force": errs,
                               "worst_step_median_rel_err": max(errs.values()) if errs else None,
                               "pooled_median_rel_err": float(np.median(np.concatenate(pooled))) if pooled else None,
                               "dt_step": integ.dt,
                               "tick_bin": integ.tick_bin, "mean_active_fraction": float(np.mean(active_hist)) / n}
            final = {k: integ.state()[k] for k in ("x", "acc")}
        if graph and (pred == "jerk" or pred == "none") and rebuild_every == 1:
            # the same run with one captured step replayed (no host work per step)
            s_ = torch.cuda.Stream()
            with ag.Context(0, s_) as c:
                c.set_option(ag.AG_OPT_MAC_OFFSET, mac_offset)
                c.set_option(ag.AG_OPT_GROUP_TARGETS, tuned["group_targets"])
                g = AdaptiveIntegrator(c, tx, tv, tm, **kw)
                g.capture()                  # runs step 1 eagerly
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                c.sync()
                e0.record(s_)
                for _ in range(steps - 1):
                    g.step()
                e1.record(s_)
                s_.synchronize()
                same = all(torch.equal(g.state()[k], final[k]) for k in final)
                runs[(pred, q)].update(graph_ms_per_step=e0.elapsed_time(e1) / (steps - 1),
                                       graph_matches_eager=bool(same))
                log(f"adaptive {pred} q_f={q}: graph replay {e0.elapsed_time(e1) / (steps - 1):.3f} ms/step, "
                    f"final state equal to the eager run: {same}")
        log(f"adaptive {pred} q_f={q}: {runs[(pred, q)]}")
    base = runs.get((preds[0], 0.0))
    res = {}
    for (pred, q), r in runs.items():
        key = str(q) if pred == preds[0] else f"{pred}:{q}"
        res[key] = dict(r, predictor=pred, q_f=q)
        if base is not None:
            res[key].update(eval_ratio=base["evaluations"] / max(1, r["evaluations"]),
                            gravity_speedup=base["gravity_ms"] / r["gravity_ms"],
                            walk_speedup=base["walk_ms"] / r["walk_ms"],
                            total_speedup=base["total_ms"] / r["total_ms"])
            if "graph_ms_per_step" in r and "graph_ms_per_step" in base:
                res[key]["graph_total_speedup"] = base["graph_ms_per_step"] / r["graph_ms_per_step"]
    # the metric's bound must hold at every checked step: the error of the
    # force in use rises and falls with the phase of the bins' update cycles
    ok = {}
    for (pred, q), r in runs.items():
        if max(r["median_rel_err_used_force"].values()) <= 1e-3:
            ok[pred] = max(ok.get(pred, 0.0), q)
    return {"workload": f"64 Plummer clumps N={n}, {steps} steps, theta=0.7 eps=1e-3 eta=0.01",
            "metric": "adaptive vs every-step speedup", "rebuild_every": rebuild_every,
            "mac_offset": mac_offset, "autotune": {"best": tuned, "walk_ms": tune_table},
            "step_shift": step_shift, "predictors": preds, "sampled_rows": n_rows, "checkpoints": checkpoints,
            "runs": res, "largest_q_f_within_1e-3": ok.get(preds[0]),
            "largest_q_f_within_1e-3_by_predictor": ok}


def run_adaptive(args):
    n = 1 << 22 if args.n == (1 << 20) else args.n
    qs = [float(q) for q in args.q_list.split(",")]
    preds = [p.strip() for p in args.predictors.split(",") if p.strip()]
    every = args.checkpoint_every
    cps = sorted(set(range(0, args.adaptive_steps + 1, every)) | {args.adaptive_steps}) if every > 0 else None
    return adaptive_comparison(n=n, steps=args.adaptive_steps, qs=qs, step_shift=args.step_shift,
                               predictors=preds, rebuild_every=args.rebuild_every, mac_offset=args.mac_offset,
                               graph=args.graph, group_span=args.group_span, n_rows=args.adaptive_rows,
                               checkpoints=cps)


# ---------------------------------------------------------------------------
def run_batched(args):
    import oracle
    d = workloads.batched_plummer(256, seed=4)
    x, v, m = d["x"], d["v"], d["m"]
    n = len(m)
    act = d["active"]
    tx, tv, tm = _t(x), _t(v), _t(m)
    toff = _t(d["offsets"], torch.int64)
    tact = _t(act, torch.int32)
    acc = torch.zeros((n, 3), dtype=torch.float64, device=DEV)
    jerk, tid = torch.zeros_like(acc), torch.zeros((n, 6), dtype=torch.float64, device=DEV)
    theta, eps = 0.5, 0.01
    stream = torch.cuda.Stream()
    out = {"workload": f"256 Plummer systems, N={n}, active={len(act)}, theta=0.5 eps=0.01"}
    with torch.cuda.stream(stream), ag.Context(0, stream) as c:
        def once(p):
            c.set_option(ag.AG_OPT_WALK_WAVES_PER_CU, p["waves_per_cu"])
            c.set_option(ag.AG_OPT_GROUP_TARGETS, p["group_targets"])
            c.tree_build_batched(tx, tv, tm, toff, p["n_leaf"])
            c.grav_eval_batched(tact, theta, eps, 1.0, acc, jerk, tid)

        def run(p):
            once(p)
            e0, e1 = _events()
            e0.record(stream)
            for _ in range(3):
                once(p)
            e1.record(stream)
            stream.synchronize()
            return e0.elapsed_time(e1) / 3

        cands = autotune.grid(n_leaf=[8, 16, 32], waves_per_cu=[8, 12, 16], group_targets=[64, 32])
        best, table = autotune.tune(run, cands, f"batched256|n={n}|act={len(act)}", use_cache=False)
        log(f"batched: autotuner picked {best}")
        once(best)
        c.sync()
        c.graph_begin()
        c.tree_build_batched(tx, tv, tm, toff, best["n_leaf"])
        c.grav_eval_batched(tact, theta, eps, 1.0, acc, jerk, tid)
        c.graph_end()
        for _ in range(3):
            c.graph_replay()
        stream.synchronize()
        c.stats_reset()
        reps = 20
        e0, e1 = _events()
        e0.record(stream)
        for _ in range(reps):
            c.graph_replay()
        e1.record(stream)
        stream.synchronize()
        ms = e0.elapsed_time(e1) / reps
        st = c.stats_read()
        c.sync()
    a = acc.cpu().numpy()
    errs = []
    rng = np.random.default_rng(44)
    off, aoff = d["offsets"], d["act_offsets"]
    for s in range(256):
        sa = act[aoff[s]:aoff[s + 1]]
        pick = rng.choice(sa, min(64, len(sa)), replace=False)
        ar, _, _ = oracle.direct(x[off[s]:off[s + 1]], v[off[s]:off[s + 1]], m[off[s]:off[s + 1]], eps, 1.0,
                                 pick - off[s])
        errs.append(_rel(a[pick], ar))
    e = np.concatenate(errs)
    pp, pn = st["n_pp"] / reps, st["n_pn"] / reps
    out.update({"value": len(act) / (ms * 1e-3), "unit": "force evals/s", "graph_replay_ms": ms,
                "interactions_per_s": (pp + pn) / (ms * 1e-3),
                "flops_per_replay": pp * PP_FLOPS + pn * PN_FLOPS,
                "autotune": {"best": best, "table_ms": table},
                "median_rel_force_err": float(np.median(e)), "p99_rel_force_err": float(np.percentile(e, 99))})
    return out


# ---------------------------------------------------------------------------
def _adjoint_fd_check(oracle, x, m, w, eps, gx, gm, ks, h=1e-6):
    """Central differences (FP64, step h) of L = sum_i w_i . a_i in one
    coordinate of each of the particles ks, and in their masses, against the
    oracle's gradient gx, gm.  Only the terms of L that involve particle k
    change: w_k . a_k (k as a target) and sum_i w_i . a_(i <- k) (k as a
    source), each O(N) through the oracle's probe-point field."""
    zero = np.zeros((1, 3))

    def L_k(k, xk, mk):
        others = np.delete(np.arange(len(m)), k)
        a_k, _, _ = oracle.field(x[others], np.zeros((len(others), 3)), m[others], eps, 1.0, xk[None])
        a_from, _, _ = oracle.field(xk[None], zero, np.array([mk]), eps, 1.0, x[others])
        return float(np.dot(w[k], a_k[0]) + np.sum(w[others] * a_from))

    ex, em = [], []
    for t, k in enumerate(ks):
        c = t % 3
        xp, xm = x[k].copy(), x[k].copy()
        xp[c] += h
        xm[c] -= h
        fd = (L_k(k, xp, m[k]) - L_k(k, xm, m[k])) / (2 * h)
        ex.append(abs(fd - gx[t, c]) / max(abs(gx[t, c]), 1e-30))
        fdm = (L_k(k, x[k], m[k] + h) - L_k(k, x[k], m[k] - h)) / (2 * h)
        em.append(abs(fdm - gm[t]) / max(abs(gm[t]), 1e-30))
    return {"coordinates": len(ks), "masses": len(ks), "h": h,
            "max_rel_diff_dLdx": float(max(ex)), "max_rel_diff_dLdm": float(max(em))}


def run_adjoint(args):
    import oracle
    n = 1 << 18
    x, m, _ = workloads.uniform_sphere(n, seed=5)
    v = np.zeros_like(x)
    w = workloads.adjoint_weights(n, seed=5)
    theta, eps = 0.6, 1e-3
    tx, tv, tm, tw = _t(x), _t(v), _t(m), _t(w)
    acc = torch.zeros((n, 3), dtype=torch.float64, device=DEV)
    jerk, tid = torch.zeros_like(acc), torch.zeros((n, 6), dtype=torch.float64, device=DEV)
    dx = torch.zeros_like(acc)
    dm = torch.zeros(n, dtype=torch.float64, device=DEV)
    out = {"workload": f"uniform sphere N=2^18 theta=0.6 eps=1e-3, L = sum w.a"}
    with ag.Context(0) as c:
        def fwd():
            c.tree_build(tx, tv, tm, 16)
            c.grav_eval(None, theta, eps, 1.0, acc, jerk, tid)

        def bwd():
            c.tree_build(tx, tv, tm, 16)
            c.grav_backward(None, tw, theta, eps, 1.0, dx, dm)

        def trial(p):
            c.set_option(ag.AG_OPT_GROUP_TARGETS, p["group_targets"])
            e0, e1 = _events()
            e0.record()
            fwd()
            bwd()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1)

        tuned, _ = autotune.tune(trial, autotune.grid(group_targets=[64, 32]), "adjoint", reps=2, use_cache=False)
        c.set_option(ag.AG_OPT_GROUP_TARGETS, tuned["group_targets"])
        out["autotune"] = tuned
        for name, fn in (("forward", fwd), ("backward", bwd)):
            for _ in range(2):
                fn()
            torch.cuda.synchronize()
            c.stats_reset()
            e0, e1 = _events()
            reps = 10
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            st = c.stats_read()
            out[name] = {"ms": ms, "interactions_per_s": (st["n_pp"] + st["n_pn"]) / reps / (ms * 1e-3)}
    rows = np.random.default_rng(6).choice(n, 16384, replace=False)
    rx, rm = oracle.adjoint(x, m, w, eps, 1.0, rows)
    out["oracle_fd_check"] = _adjoint_fd_check(oracle, x, m, w, eps, rx[:64], rm[:64], rows[:64])
    ex = _rel(dx.cpu().numpy()[rows], rx)
    out["dLdx_rel_err"] = {"median": float(np.median(ex)), "p99": float(np.percentile(ex, 99))}
    em = np.abs(dm.cpu().numpy()[rows] - rm) / np.abs(rm)
    out["dLdm_rel_err_plain"] = {"median": float(np.median(em)), "p99": float(np.percentile(em, 99))}
    return out


# ---------------------------------------------------------------------------
def run_periodic(args):
    import oracle
    out = {"workload": "periodic pancake box (one plane-wave mode at growth 0.9), eps = 1/8 lattice spacing; "
                       "nearest images, and Ewald sums for g and T (j nearest-image)", "runs": {}}
    for n_side in (64, 128):
        x, v, m = workloads.zeldovich_box(n_side, seed=6, box=1.0, growth=0.9)
        n = len(m)
        eps = 1.0 / n_side / 8
        tx, tv, tm = _t(x), _t(v), _t(m)
        acc = torch.zeros((n, 3), dtype=torch.float64, device=DEV)
        jerk, tid = torch.zeros_like(acc), torch.zeros((n, 6), dtype=torch.float64, device=DEV)
        rows = np.random.default_rng(7).choice(n, 2048, replace=False)
        log(f"periodic: nearest-image oracle on {rows.size} targets of {n}")
        ref = {"nearest": (rows, *oracle.direct(x, v, m, eps, 1.0, rows, box=1.0))}
        if n_side == 64:
            er = rows[:32]
            log(f"periodic: Ewald oracle on {er.size} targets of {n}")
            t_a = time.perf_counter()
            ref["ewald"] = (er, *oracle.direct(x, v, m, eps, 1.0, er, box=1.0, ewald=True))
            t_ew = time.perf_counter() - t_a
        tuned_sets = {}
        for mode in ("nearest", "ewald"):
            for theta in (0.5, 0.7):
                with ag.Context(0) as c:
                    c.set_periodic(1.0, ewald=(mode == "ewald"))

                    def step():
                        c.tree_build(tx, tv, tm, 16)
                        c.grav_eval(None, theta, eps, 1.0, acc, jerk, tid)

                    # group size and split depend on the box size (64^3 runs
                    # faster with 32-target groups, 128^3 with 64)
                    def trial(p):
                        c.set_option(ag.AG_OPT_GROUP_TARGETS, p["group_targets"])
                        c.set_option(ag.AG_OPT_GROUP_SPLIT, p["group_split"])
                        e0, e1 = _events()
                        e0.record()
                        step()
                        e1.record()
                        torch.cuda.synchronize()
                        return e0.elapsed_time(e1)

                    tuned, _ = autotune.tune(trial, autotune.grid(group_targets=[64, 32], group_split=[0, 42]),
                                             f"periodic|{mode}|{n_side}|{theta}", reps=2, use_cache=False)
                    trial(tuned)
                    tuned_sets[(mode, theta)] = tuned
                    for _ in range(2):
                        step()
                    torch.cuda.synchronize()
                    c.stats_reset()
                    e0, e1 = _events()
                    reps = 10
                    e0.record()
                    for _ in range(reps):
                        step()
                    e1.record()
                    torch.cuda.synchronize()
                    ms = e0.elapsed_time(e1) / reps
                    st = c.stats_read()
                    # phase split from a second, separately timed pass
                    c.timing_enable(True)
                    c.timing_read(reset=True)
                    for _ in range(reps):
                        step()
                    ph = c.timing_read(reset=True)
                    c.timing_enable(False)
                walk_ms = ph["walk"]["ms"] / reps
                flops = (st["n_pp"] * PP_FLOPS + st["n_pn"] * PN_FLOPS) / reps
                r = {"n": n, "theta": theta, "eps": eps, "autotune": tuned, "ms_per_step": ms,
                     "evals_per_s": n / (ms * 1e-3),
                     "build_ms": ph["build"]["ms"] / reps, "walk_ms": walk_ms, "ewald_ms": ph["ewald"]["ms"] / reps,
                     "walk_tflops": flops / (walk_ms * 1e-3) / 1e12,
                     "walk_frac_of_peak": flops / (walk_ms * 1e-3) / 1e12 / PEAK_TFLOPS,
                     "per_target": {"pp": st["n_pp"] / reps / n, "pn": st["n_pn"] / reps / n}}
                if mode in ref:
                    rr, ar, jr, tr = ref[mode]
                    a = acc.cpu().numpy()[rr]
                    sa = oracle.abs_scale(x, m, eps, 1.0, rr, box=1.0)
                    ea = _rel(a, ar)
                    eas = np.linalg.norm(a - ar, axis=1) / sa
                    r["error_targets"] = int(rr.size)
                    r["acc_rel_err"] = {"median": float(np.median(ea)), "p99": float(np.percentile(ea, 99))}
                    r["acc_err_vs_abs_scale"] = {"median": float(np.median(eas)), "p99": float(np.percentile(eas, 99))}
                log(f"periodic {mode} n={n} theta={theta}: {r}")
                out["runs"][f"{mode} {n_side}^3 theta={theta}"] = r
        # Ewald with fully adaptive softening: every step builds with the
        # lengths found on the previous step's tree (32nd neighbour at its
        # nearest image), then finds the new ones on the device
        hl = workloads.neighbour_lengths(x, 32, box=1.0)
        hdev = _t(hl)
        with ag.Context(0) as c:
            c.set_periodic(1.0, ewald=True)
            c.set_option(ag.AG_OPT_GROUP_TARGETS, tuned_sets[("ewald", 0.5)]["group_targets"])
            c.set_option(ag.AG_OPT_GROUP_SPLIT, tuned_sets[("ewald", 0.5)]["group_split"])

            def step():
                c.set_softening(hdev)
                c.tree_build(tx, tv, tm, 16)
                c.neighbour_lengths(32, hdev)
                c.grav_eval(None, 0.5, eps, 1.0, acc, jerk, tid)

            for _ in range(2):
                step()
            torch.cuda.synchronize()
            e0, e1 = _events()
            reps = 10
            e0.record()
            for _ in range(reps):
                step()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            c.timing_enable(True)
            c.timing_read(reset=True)
            for _ in range(reps):
                step()
            ph = c.timing_read(reset=True)
            c.timing_enable(False)
        r = {"n": n, "theta": 0.5, "lengths": "32nd-neighbour distance at the nearest image",
             "options": tuned_sets[("ewald", 0.5)],
             "ms_per_step": ms, "evals_per_s": n / (ms * 1e-3), "build_ms": ph["build"]["ms"] / reps,
             "neighbour_ms": ph["neighbour"]["ms"] / reps, "walk_ms": ph["walk"]["ms"] / reps,
             "ewald_ms": ph["ewald"]["ms"] / reps,
             "lengths_equal_host": bool(np.array_equal(hdev.cpu().numpy(), hl))}
        if n_side == 64:
            # the oracle: the mean-kernel sum at the nearest images plus the
            # images' Ewald correction (the softening acts within half a box)
            er, ae, _, _ = ref["ewald"]
            an, _, _ = oracle.direct(x, v, m, 1e-9, 1.0, er, box=1.0)
            ae0, _, _ = oracle.direct(x, v, m, 1e-9, 1.0, er, box=1.0, ewald=True)
            a_soft = np.empty((er.size, 3))
            for t, i in enumerate(er):
                dd = x - x[i]
                dd -= np.round(dd)
                a_soft[t] = oracle.direct_soft(x[i] + dd, np.zeros_like(x), m, hl, 1.0, [i])[0][0]
            ref_s = a_soft + (ae0 - an)
            e = _rel(acc.cpu().numpy()[er], ref_s)
            r["error_targets"] = int(er.size)
            r["acc_rel_err"] = {"median": float(np.median(e)), "p99": float(np.percentile(e, 99))}
        log(f"periodic ewald adaptive softening n={n}: {r}")
        out["runs"][f"ewald {n_side}^3 theta=0.5 adaptive softening"] = r
        t_a = time.perf_counter()
        oracle.direct(x, v, m, eps, 1.0, rows[:256], box=1.0)
        t_o = time.perf_counter() - t_a
        out["runs"][f"nearest {n_side}^3 theta=0.5"]["cpu_baseline"] = {
            "value": 256 / t_o, "unit": "force evals/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"256 targets of the {n} particles, nearest-image direct sum"}
        if n_side == 64:
            out["runs"][f"ewald {n_side}^3 theta=0.5"]["cpu_baseline"] = {
                "value": 32 / t_ew, "unit": "force evals/s", "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"32 targets of the {n} particles, Ewald direct sum"}
    return out


# ---------------------------------------------------------------------------
def run_softening(args):
    import oracle
    n = args.n
    x, v, m = workloads.turbulent_sphere(n, seed=2, grid=128)
    log("softening: neighbour lengths (k = 32)")
    h = workloads.neighbour_lengths(x, 32)
    tx, tv, tm, th = _t(x), _t(v), _t(m), _t(h)
    acc = torch.zeros((n, 3), dtype=torch.float64, device=DEV)
    jerk, tid = torch.zeros_like(acc), torch.zeros((n, 6), dtype=torch.float64, device=DEV)
    rows = np.random.default_rng(8).choice(n, 4096, replace=False)
    out = {"workload": f"turbulent sphere N={n}, theta={args.theta}, lengths = 32nd-neighbour distance "
                       f"(median {np.median(h):.2e}, 1-99% {np.percentile(h, 1):.2e}-{np.percentile(h, 99):.2e}) "
                       f"vs one length eps={args.eps}", "runs": {}}
    # "adaptive": every step builds with the lengths found on the previous
    # step's tree, then finds the new ones on the device (the particles do
    # not move here, so from the second step on they are the host's lengths)
    hdev = torch.zeros(n, dtype=torch.float64, device=DEV)
    for mode in ("per-particle", "adaptive", "uniform"):
        with ag.Context(0) as c:
            c.set_option(ag.AG_OPT_MAC_OFFSET, args.mac_offset)
            if mode == "per-particle":
                c.set_softening(th)
            if mode == "adaptive":
                c.tree_build(tx, tv, tm, args.n_leaf)
                c.neighbour_lengths(32, hdev)

            def step():
                if mode == "adaptive":
                    c.set_softening(hdev)
                c.tree_build(tx, tv, tm, args.n_leaf)
                if mode == "adaptive":
                    c.neighbour_lengths(32, hdev)
                c.grav_eval(None, args.theta, args.eps, 1.0, acc, jerk, tid)

            for _ in range(2):
                step()
            torch.cuda.synchronize()
            c.stats_reset()
            e0, e1 = _events()
            reps = 10
            e0.record()
            for _ in range(reps):
                step()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            st = c.stats_read()
            c.timing_enable(True)
            c.timing_read(reset=True)
            for _ in range(reps):
                step()
            ph = c.timing_read(reset=True)
            c.timing_enable(False)
        walk_ms = ph["walk"]["ms"] / reps
        flops = (st["n_pp"] * PP_FLOPS + st["n_pn"] * PN_FLOPS) / reps
        a = acc.cpu().numpy()[rows]
        extra = {}
        if mode == "adaptive":
            hd = hdev.cpu().numpy()
            extra = {"neighbour_ms": ph["neighbour"]["ms"] / reps,
                     "lengths_equal_host": bool(np.array_equal(hd, h)),
                     "lengths_max_rel_diff": float(np.max(np.abs(hd - h) / h))}
        if mode != "uniform":
            ar, _, _ = oracle.direct_soft(x, v, m, h, 1.0, rows)
        else:
            ar, _, _ = oracle.direct(x, v, m, args.eps, 1.0, rows)
        e = _rel(a, ar)
        out["runs"][mode] = {"ms_per_step": ms, "evals_per_s": n / (ms * 1e-3), "build_ms": ph["build"]["ms"] / reps,
                             "walk_ms": walk_ms, "walk_tflops": flops / (walk_ms * 1e-3) / 1e12,
                             "per_target": {"pp": st["n_pp"] / reps / n, "pn": st["n_pn"] / reps / n},
                             "median_rel_force_err": float(np.median(e)), "p99_rel_force_err": float(np.percentile(e, 99)),
                             **extra}
        log(f"softening {mode}: {out['runs'][mode]}")
    return out


# ---------------------------------------------------------------------------
def run_pm(args):
    """Fully adaptive softening with the Price & Monaghan terms: each step
    solves the lengths and Omega on the previous tree, rebuilds with those
    lengths, evaluates the softened tree force, then the factors Z and the
    correction.  Checked on sampled rows against the density condition and
    Omega's definition (the lengths' definition over every particle)."""
    import oracle
    n, n_ngb = args.n, 32.0
    x, v, m = workloads.turbulent_sphere(n, seed=2, grid=128)
    tx, tv, tm = _t(x), _t(v), _t(m)
    acc = torch.zeros((n, 3), dtype=torch.float64, device=DEV)
    jerk, tid = torch.zeros_like(acc), torch.zeros((n, 6), dtype=torch.float64, device=DEV)
    h = torch.empty(n, dtype=torch.float64, device=DEV)
    om, z = torch.empty_like(h), torch.empty_like(h)
    corr = torch.empty_like(acc)
    names = ("lengths", "build", "gravity", "factors", "correction")
    with ag.Context(0) as c:
        c.set_option(ag.AG_OPT_MAC_OFFSET, args.mac_offset)
        c.tree_build(tx, tv, tm, args.n_leaf)
        c.pm_lengths(n_ngb, h, om)

        def step(ev=None):
            mark = (lambda i: ev[i].record()) if ev else (lambda i: None)
            mark(0)
            c.pm_lengths(n_ngb, h, om)
            mark(1)
            c.set_softening(h)
            c.tree_build(tx, tv, tm, args.n_leaf)
            mark(2)
            c.grav_eval(None, args.theta, args.eps, 1.0, acc, jerk, tid)
            mark(3)
            c.pm_factors(n_ngb, 1.0, om, z)
            mark(4)
            c.pm_correct(z, corr)
            mark(5)

        for _ in range(2):
            step()
        torch.cuda.synchronize()
        reps = 5
        e0, e1 = _events()
        e0.record()
        for _ in range(reps):
            step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        phase = dict.fromkeys(names, 0.0)
        for _ in range(reps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
            step(ev)
            torch.cuda.synchronize()
            for i, k in enumerate(names):
                phase[k] += ev[i].elapsed_time(ev[i + 1]) / reps
    hh, oo = h.cpu().numpy(), om.cpu().numpy()
    rows = np.random.default_rng(9).choice(n, 64, replace=False)
    dens, omer = [], []
    for i in rows:
        u = np.sqrt(np.sum((x - x[i])**2, axis=1)) / hh[i]
        w, wp = oracle.m4_shape(u)
        dens.append(abs(w.sum() / (3.0 * n_ngb / 32.0) - 1.0))
        omer.append(abs(oo[i] + 32.0 / (9.0 * n_ngb) * np.sum(u * wp)))
    cn = np.linalg.norm(corr.cpu().numpy(), axis=1) / np.linalg.norm(acc.cpu().numpy(), axis=1)
    out = {"workload": f"turbulent sphere N={n}, n_ngb={n_ngb:g}, theta={args.theta}",
           "ms_per_step": ms, "phase_ms": phase,
           "h_median": float(np.median(hh)), "h_1_99": [float(np.percentile(hh, 1)), float(np.percentile(hh, 99))],
           "density_max_rel_err": float(max(dens)), "omega_max_abs_err": float(max(omer)),
           "omega_median": float(np.median(oo)),
           "correction_over_gravity_median": float(np.median(cn))}
    log(f"pm: {out}")
    return out


# ---------------------------------------------------------------------------
def run_relative(args):
    """Geometric opening test alone at several theta against the combined
    geometric + relative test at several alpha (|a_old| from the previous
    evaluation, theta = 0.7): time per tree build + evaluation, interactions
    per target and the force error against the oracle on sampled rows."""
    import oracle
    n = args.n
    x, v, m = workloads.turbulent_sphere(n, seed=2, grid=128)
    tx, tv, tm = _t(x), _t(v), _t(m)
    acc = torch.zeros((n, 3), dtype=torch.float64, device=DEV)
    jerk, tid = torch.zeros_like(acc), torch.zeros((n, 6), dtype=torch.float64, device=DEV)
    rows = np.random.default_rng(8).choice(n, 4096, replace=False)
    log("relative: oracle direct sum on 4096 sampled rows")
    ar, _, _ = oracle.direct(x, v, m, args.eps, 1.0, rows)
    # |a_old|: the previous evaluation (geometric test, theta = 0.7)
    with ag.Context(0) as c:
        c.tree_build(tx, tv, tm, args.n_leaf)
        c.grav_eval(None, 0.7, args.eps, 1.0, acc, jerk, tid)
        c.sync()
    a_old = acc.clone()
    out = {"workload": f"turbulent sphere N={n}, eps={args.eps}; |a_old| from a theta=0.7 evaluation", "runs": {}}
    cases = [("geometric", th, 0.0) for th in (0.7, 0.5, 0.35)] + [("combined", 0.7, al)
                                                                    for al in (0.01, 0.0025, 0.0005)]
    for kind, th, al in cases:
        with ag.Context(0) as c:
            c.set_option(ag.AG_OPT_MAC_OFFSET, args.mac_offset)
            if al > 0:
                c.set_relative_opening(al, a_old)
            # targets per walk group by the autotuner (untimed): the relative
            # test opens more near groups of small |a_old|, where smaller
            # groups share the work over more waves
            c.tree_build(tx, tv, tm, args.n_leaf)

            def trial(p):
                c.set_option(ag.AG_OPT_GROUP_TARGETS, p["group_targets"])
                c.timing_enable(True)
                c.timing_read(reset=True)
                c.grav_eval(None, th, args.eps, 1.0, acc, jerk, tid)
                ph = c.timing_read(reset=True)
                c.timing_enable(False)
                return ph["groups"]["ms"] + ph["walk"]["ms"]

            tuned, _ = autotune.tune(trial, autotune.grid(group_targets=[64, 32, 16]), "relative", use_cache=False)
            c.set_option(ag.AG_OPT_GROUP_TARGETS, tuned["group_targets"])

            def step():
                c.tree_build(tx, tv, tm, args.n_leaf)
                c.grav_eval(None, th, args.eps, 1.0, acc, jerk, tid)

            for _ in range(2):
                step()
            torch.cuda.synchronize()
            c.stats_reset()
            e0, e1 = _events()
            reps = 10
            e0.record()
            for _ in range(reps):
                step()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            st = c.stats_read()
            c.timing_enable(True)
            c.timing_read(reset=True)
            for _ in range(reps):
                step()
            ph = c.timing_read(reset=True)
            c.timing_enable(False)
        walk_ms = ph["walk"]["ms"] / reps
        flops = (st["n_pp"] * PP_FLOPS + st["n_pn"] * PN_FLOPS) / reps
        e = _rel(acc.cpu().numpy()[rows], ar)
        key = f"{kind} theta={th}" + (f" alpha={al}" if al > 0 else "")
        out["runs"][key] = {"ms_per_step": ms, "evals_per_s": n / (ms * 1e-3), "walk_ms": walk_ms,
                            "group_targets": tuned["group_targets"],
                            "walk_tflops": flops / (walk_ms * 1e-3) / 1e12,
                            "per_target": {"pp": st["n_pp"] / reps / n, "pn": st["n_pn"] / reps / n},
                            "median_rel_force_err": float(np.median(e)),
                            "p99_rel_force_err": float(np.percentile(e, 99))}
        log(f"relative {key}: {out['runs'][key]}")
    return out


# ---------------------------------------------------------------------------
# algorithmic bytes of one build: per particle, read x, v, m (56), write them
# in key order (positions and masses as double4, FP32 velocities and masses:
# 48), Morton keys
# and row indices (8 + 4, written and read once: 24); per node, link 16,
# centre 32, box 32, FP32 moments 64 and FP64 moments 200 (344)
BUILD_BYTES_PER_PARTICLE = 56 + 48 + 24
BUILD_BYTES_PER_NODE = 344


def run_build(args):
    out = {"workload": "tree build (n_leaf 16)", "peak_hbm_gbs": 8000.0,
           "bytes_per_particle": BUILD_BYTES_PER_PARTICLE, "bytes_per_node": BUILD_BYTES_PER_NODE, "sets": {}}
    sets = {"clumps_2p22": lambda: workloads.clumps(1 << 22, seed=3)[:3],
            "turbulent_sphere_2p20": lambda: workloads.turbulent_sphere(1 << 20, seed=2, grid=128)}
    for name, make in sets.items():
        x, v, m = make()
        n = len(m)
        tx, tv, tm = _t(x), _t(v), _t(m)
        with ag.Context(0) as c:
            for _ in range(3):
                c.tree_build(tx, tv, tm, 16)
            c.sync()
            c.timing_enable(True)
            c.timing_read(reset=True)
            reps = 20
            for _ in range(reps):
                c.tree_build(tx, tv, tm, 16)
            ph = c.timing_read(reset=True)
            c.timing_enable(False)
            nn, levels = c.tree_info()
        ms = ph["build"]["ms"] / reps
        nbytes = n * BUILD_BYTES_PER_PARTICLE + nn * BUILD_BYTES_PER_NODE
        gbs = nbytes / (ms * 1e-3) / 1e9
        out["sets"][name] = {"n": n, "nodes": nn, "levels": levels, "ms_per_build": ms,
                             "algorithmic_bytes": nbytes, "gbs": gbs, "frac_hbm": gbs / 8000.0}
        log(f"build {name}: {ms:.3f} ms, {nn} nodes, {gbs:.0f} GB/s")
    return out


def run_copy(args):
    n = 1 << 27                      # 2^27 doubles = 1 GiB
    a = torch.ones(n, dtype=torch.float64, device=DEV)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    for _ in range(3):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 3
    return {"workload": "device copy of 1 GiB (counter calibration)", "bytes_read": n * 8,
            "bytes_written": n * 8, "ms": ms, "gbs": 2 * n * 8 / (ms * 1e-3) / 1e9}
