"""Benchmark of the fast Monte Carlo hot path on one MI355X.

One step = one pass of the whole method (setup, LHS design, basis, KLE path
contraction, integration of every sample, statistics) on the 10-machine
workload: classical swing model on a seeded 39-bus-shaped synthetic network,
3 OU disturbances, K = 100 per process (M = 300), N = 1e4 samples,
T = 20 s, dt = 5 ms (4000 RK4 steps).  Inputs are synthetic and seeded.

Prints one JSON line.  value = N * S / (seconds per step) trajectory-steps/s of
the plain FP64 form; the FP32 and BF16x3 forms of the same workload are
reported under "forms" with their error against the FP64 oracle.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_FP64_VECTOR = 78.6e12
PEAK_FP32_VECTOR = 157.3e12
PEAK_HBM = 8.0e12
PEAK_FP32_MATRIX = 157.3e12


def say(msg: str):
    """Progress line on stderr (the JSON result line goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def integrator_flops_per_traj_step(n: int, P: int) -> float:
    """Algorithmic flops of one RK4 step of one trajectory (classical model).

    Per stage: complex matvec Y dE (n^2 complex MACs = 8 n^2 flops); per machine
    25 flops (rotation 11, power deviation 9, accelerating power 3, derivatives
    2) plus one sin/cos pair counted as 20 flops; per process 4 flops.  Per
    step: 4 stages and 13 flops per state variable for the RK4 combination.
    """
    stage = 8 * n * n + (25 + 20) * n + 4 * P
    return 4 * stage + 13 * (2 * n + P)


def integrator_flops_survey(n: int) -> float:
    """The integrator's flops per trajectory-step as the scope table counts
    them: 32 n^2 for the complex network product of four RK4 stages plus about
    60 per machine, with the 4 n sin/cos pairs counted separately (n = 10:
    3800 flops + 40 sin/cos pairs).  The headline roofline fraction uses this
    count with the sin/cos pairs at zero cost."""
    return 32.0 * n * n + 60.0 * n


SINCOS_FLOPS = 20.0  # one sin/cos pair as a flop count (two short polynomials)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def per_output(gpu_mean, gpu_var, gpu_traj, o_mean, o_var, o_traj):
    """Per output variable: trajectory error relative to max |oracle| of the
    variable (or to its excursion where it starts far from zero), mean error
    relative to max(|mean|, std), variance error relative to max |var|."""
    import numpy as np
    out = {}
    if gpu_traj is not None:
        V = o_traj.shape[-1]
        num = np.abs(gpu_traj - o_traj).reshape(-1, V).max(axis=0)
        den = np.abs(o_traj).reshape(-1, V).max(axis=0)
        out["traj_rel_per_output"] = (num / np.where(den == 0, 1, den)).tolist()
        exc = np.abs(o_traj - o_traj[:, :1, :]).reshape(-1, V).max(axis=0)
        out["traj_rel_to_excursion_per_output"] = (num / np.maximum(exc, 1e-12)).tolist()
    if gpu_mean is not None:
        sm = np.maximum(np.abs(o_mean).max(axis=0), np.sqrt(o_var).max(axis=0))
        out["mean_rel_per_output"] = (np.abs(gpu_mean - o_mean).max(axis=0)
                                      / np.where(sm == 0, 1, sm)).tolist()
        sv = np.abs(o_var).max(axis=0)
        out["var_rel_per_output"] = (np.abs(gpu_var - o_var).max(axis=0)
                                     / np.where(sv == 0, 1, sv)).tolist()
    for k in list(out):
        out[k.replace("_per_output", "_max")] = float(max(out[k]))
    return out


def config1_leg(ctx, fmc, workloads, oracle_mod, steps: int):
    """The single machine against an infinite bus (H = 3.5 s, D = 2, Pm = 0.8,
    E = 1.1, X = 0.5; one OU disturbance, theta = 0.5, sigma = 0.05; T = 10 s,
    dt = 0.01 s, K = 40, N = 1000) in FP64: trajectory-steps/s over whole runs
    and the error of every output against the FP64 oracle."""
    import numpy as np
    import torch
    sc = workloads.config1()
    N, S = sc["N"], fmc.steps(sc)
    ctx.run(sc, precision="f64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = ctx.run(sc, precision="f64")
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    res = {"workload": "SMIB, N=1000, K=40, T=10 s, dt=0.01 s (1000 RK4 steps), FP64",
           "ms_per_pass": t * 1e3, "trajectory_steps_per_s": N * S / t}
    if oracle_mod is not None:
        o = oracle_mod.run(sc)
        res["error_vs_oracle"] = per_output(r["mean"].cpu().numpy(), r["var"].cpu().numpy(),
                                            None, o["mean"], o["var"], None)
    say(f"config1 f64: {t * 1e3:.2f} ms per pass, {N * S / t:.3e} traj-steps/s")
    return res


def general_leg(ctx, fmc, workloads, oracle_mod, steps: int):
    """General Ito disturbances on the 10-machine workload (N = 1e4, K = 100,
    4000 steps): Table I's Beta and Gamma rows and the wind model of eq. 11 in
    place of the OU processes, FP64 and FP32 on the variant tuned for the
    shape, with the error of sampled trajectories against the FP64 oracle."""
    import numpy as np
    import torch
    sc = workloads.config2_general()
    N, S = sc["N"], fmc.steps(sc)
    sel = np.array([0, 1, N // 2, N - 1])
    ot = oracle_mod.run(sc, sel=sel, want_traj=True)["traj"] if oracle_mod is not None else None
    out = {"workload": "10-machine system, N=1e4, K=100, T=20 s, dt=5 ms; Beta (a=6, b=9), Gamma "
                       "(a=4, b=20) and eq. 11 wind processes (Ito reading)",
           "trajectory_steps": N * S}
    for form in ("f64", "f32"):
        r = ctx.run(sc, precision=form)
        outs = dict(mean=r["mean"], var=r["var"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = ctx.run(sc, precision=form, outputs=outs)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        res = {"ms_per_pass": t * 1e3, "trajectory_steps_per_s": N * S / t,
               "variant": r["report"]["variant_id"],
               "lanes_per_traj": r["report"]["lanes_per_traj"]}
        if ot is not None:
            rt = ctx.run(sc, precision=form, traj_idx=sel)["traj"].cpu().numpy()
            res["error_vs_oracle"] = per_output(None, None, rt, None, None, ot)
        out[form] = res
        say(f"general processes {form}: {t * 1e3:.2f} ms per pass, {N * S / t:.3e} traj-steps/s")
    return out


def config3_leg(ctx, fmc, workloads, oracle_mod, steps: int):
    """The mixed-precision workload (the 10-machine system with N = 1e5, LHS
    seed 3): every form timed over whole passes; error against the FP64 oracle
    on the subset n = 0, 100, ..., 99900 of the same design (per sample, and the
    subset's mean and variance from the GPU's trajectories), per output."""
    import numpy as np
    import torch
    sc = workloads.config3()
    n, P, N = sc["n_gen"], len(sc["dist"]["gen"]), sc["N"]
    S = fmc.steps(sc)
    sub = np.arange(0, N, 100)
    out = {"workload": "10-machine classical swing model, seeded 39-bus synthetic network, "
                       "3 OU disturbances, K=100 (300 x 1e5 LHS design, seed 3), N=1e5, "
                       "T=20 s, dt=5 ms (4000 RK4 steps)",
           "trajectory_steps": N * S, "error_subset": "n = 0, 100, ..., 99900 (1000 samples)"}
    ref = None
    if oracle_mod is not None:
        t0 = time.perf_counter()
        ref = oracle_mod.run(sc, sel=sub, want_traj=True)
        t_cpu = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": len(sub) * S / t_cpu, "unit": "trajectory-steps/s",
            "cores": oracle_mod.num_threads(), "kind": "oracle",
            "sample": f"the 1000-sample subset ({S} steps each) in {t_cpu:.1f} s; "
                      f"full N=1e5 extrapolated linearly: {t_cpu * N / len(sub):.0f} s"}
        say(f"config3: oracle subset {t_cpu:.1f} s")
    for form in ("bf16x3", "f32", "f64"):
        vid = ctx.autotune(sc, precision=form)
        r = ctx.run(sc, precision=form, variant=vid)
        outs = dict(mean=r["mean"], var=r["var"])
        torch.cuda.synchronize()
        t_int = 0.0
        t0 = time.perf_counter()
        for _ in range(steps):
            r = ctx.run(sc, precision=form, variant=vid, outputs=outs)
            t_int += r["report"]["t_integrate_s"]
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        t_int /= steps
        rep = r["report"]
        fs = integrator_flops_survey(n)
        peak = PEAK_FP64_VECTOR if form == "f64" else PEAK_FP32_VECTOR
        ent = {"value": N * S / sec, "unit": "trajectory-steps/s", "ms_per_pass": sec * 1e3,
               "integrator_ms": t_int * 1e3, "gemm_ms": rep["t_gemm_s"] * 1e3,
               "variant": rep["variant_id"], "time_chunk": rep["time_chunk"],
               "integrator_tflops": fs * N * S / t_int / 1e12,
               "integrator_frac": fs * N * S / t_int / peak,
               "peak_tflops": peak / 1e12}
        if ref is not None:
            rt = ctx.run(sc, precision=form, variant=vid, traj_idx=sub)["traj"].cpu().numpy()
            m = rt.mean(axis=0)
            v = ((rt - m) ** 2).sum(axis=0) / (len(sub) - 1)
            ent["error_vs_oracle_subset"] = per_output(m, v, rt, ref["mean"], ref["var"],
                                                       ref["traj"])
            del rt
        out[form] = ent
        say(f"config3 {form}: {sec * 1e3:.1f} ms per pass, integrator {t_int * 1e3:.1f} ms, "
            f"{N * S / sec:.3e} traj-steps/s")
    if "f64" in out:
        for form in ("bf16x3", "f32"):
            out[form]["speedup_vs_f64"] = out[form]["value"] / out["f64"]["value"]
    return out


def fd_flops_per_traj_step(n: int, P: int) -> float:
    """Algorithmic flops of one RK4 step of one flux-decay trajectory: per
    stage the complex network product (8 n^2), about 90 flops per machine
    (EMF rotation with one sin/cos pair counted as 20, electrical power, d-axis
    current, terminal voltage, six derivatives) and 4 per process; 13 per state
    variable for the RK4 combination."""
    return 4.0 * (8.0 * n * n + 90.0 * n + 4.0 * P) + 13.0 * (6 * n + P)


def oracle_mod():
    import oracle
    return oracle


def measured_traffic(variant: int, precision: str):
    """HBM bytes per integrator launch from the committed counter summary, or
    None when that summary is for another variant or the kernel source has
    changed since the counters were taken."""
    import glob
    import hashlib
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_traffic.json")):
        try:
            info = json.load(open(path))
            src = open(os.path.join(ROOT, info["source"]), "rb").read()
        except (OSError, ValueError, KeyError):
            continue
        if (info.get("variant") == variant and info.get("precision") == precision
                and hashlib.sha256(src).hexdigest() == info.get("source_sha256")):
            return info["hbm_bytes_per_launch"], info.get("steps_per_launch")
    return None, None


def batched_leg(ctx, fmc, workloads, oracle_mod, steps: int, with_fp64: bool):
    """The 64-scenario uneven set (n 3-50, P 1-6, T 5-30 s, K 40-150, N 500-2e4):
    batched forms (one graph replay = one pass over all scenarios) and, as the
    plain reference, FP64 fmc_run of every scenario in turn."""
    import numpy as np
    import torch
    scs = workloads.uneven_batch()
    ts = sum(sc["N"] * fmc.steps(sc) for sc in scs)
    out = {"workload": "64 uneven scenarios: seeded synthetic networks, n 3-50 machines, "
                       "P 1-6 OU processes, T 5-30 s, dt 5 ms, K 40-150, N 500-2e4 "
                       "(log-uniform), LHS seeds 4000-4063",
           "trajectory_steps": ts}
    pick = [0, 17, 40]
    sels = [np.array([1, sc["N"] // 2]) if i in pick else None for i, sc in enumerate(scs)]
    small = int(np.argmin([sc["N"] * fmc.steps(sc) * sc["n_gen"] ** 2 for sc in scs]))
    ref_small = ref_traj = None
    if oracle_mod is not None:
        ref_small = oracle_mod.run(scs[small])
        ref_traj = {i: oracle_mod.run(scs[i], sel=sels[i], want_traj=True)["traj"] for i in pick}
    say("batched: oracle references done" if oracle_mod is not None else "batched: start")
    for form in ("bf16x3", "f32"):
        res = ctx.run_batch(scs, precision=form, traj_idx=sels)  # tunes, captures the graph
        say(f"batched {form}: tuned and captured")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res = ctx.run_batch(scs, precision=form, traj_idx=sels)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        say(f"batched {form}: {sec * 1e3:.1f} ms per pass")
        # roofline of the summed integrator work (the scope table's count per
        # trajectory-step, 32 n^2 + 60 n, summed over the scenarios) against
        # the FP32 vector peak, and against the 78.6 TFLOP/s this build can
        # reach without packed FP32
        flops = sum(sc["N"] * fmc.steps(sc) * integrator_flops_survey(sc["n_gen"]) for sc in scs)
        entry = {"value": ts / sec, "unit": "trajectory-steps/s", "ms_per_pass": sec * 1e3,
                 "variants": sorted({r["report"]["variant_id"] for r in res}),
                 "roofline": {"bound": "alu", "flops_per_pass": flops,
                              "achieved_tflops": flops / sec / 1e12,
                              "peak_tflops": PEAK_FP32_VECTOR / 1e12,
                              "frac": flops / sec / PEAK_FP32_VECTOR,
                              "frac_of_unpacked_fp32": flops / sec / (PEAK_FP32_VECTOR / 2)}}
        if oracle_mod is not None:
            r = res[small]
            m, v = r["mean"].cpu().numpy(), r["var"].cpu().numpy()
            om, ov = ref_small["mean"], ref_small["var"]
            sm = np.maximum(np.abs(om).max(axis=0), np.sqrt(ov).max(axis=0))
            et = 0.0
            for i in pick:
                a = res[i]["traj"].cpu().numpy()
                b = ref_traj[i]
                num = np.abs(a - b).reshape(-1, a.shape[-1]).max(axis=0)
                den = np.abs(b).reshape(-1, a.shape[-1]).max(axis=0)
                et = max(et, float((num / np.where(den == 0, 1, den)).max()))
            entry["error_vs_oracle"] = {
                "scenario": small,
                "mean_rel": float((np.abs(m - om).max(axis=0) / sm).max()),
                "var_rel": float((np.abs(v - ov).max(axis=0) / np.abs(ov).max(axis=0)).max()),
                "traj_rel_sampled": et}
        out[form] = entry
    if with_fp64:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for sc in scs:
            ctx.run(sc, precision="f64")
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        say(f"plain f64 sequential: {sec * 1e3:.1f} ms")
        out["plain_f64_sequential"] = {"value": ts / sec, "unit": "trajectory-steps/s",
                                       "ms_per_pass": sec * 1e3}
    return out


def _latency_summary(lat, is_large, span, ts, n_req, refused, rate):
    import numpy as np
    ent = {"rate_req_per_s": rate, "requests": n_req, "large_requests": int(is_large.sum()),
           "p50_latency_s": float(np.median(lat)), "p99_latency_s": float(np.quantile(lat, 0.99)),
           "max_latency_s": float(lat.max()), "makespan_s": span,
           "completed_req_per_s": n_req / span, "trajectory_steps_per_s": ts / span,
           "ebusy_retries": refused}
    if (~is_large).any():
        ent["small_p50_latency_s"] = float(np.median(lat[~is_large]))
        ent["small_p99_latency_s"] = float(np.quantile(lat[~is_large], 0.99))
    if is_large.any():
        ent["large_p50_latency_s"] = float(np.median(lat[is_large]))
        ent["large_p99_latency_s"] = float(np.quantile(lat[is_large], 0.99))
    return ent


def _poisson_stream(ctx, fmc, reqs, arrive, precision="bf16x3"):
    """Open-loop client: submit each request at its arrival time (retrying
    every millisecond while the server answers EBUSY), poll for completion.
    Returns completion times relative to the start and the EBUSY count."""
    import numpy as np
    import torch
    n_req = len(reqs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pending = {}
    done_at = np.zeros(n_req)
    wait_q = list(range(n_req))
    refused = 0
    refused_req = set()
    last_note = 0.0
    while wait_q or pending:
        now = time.perf_counter() - t0
        if now - last_note >= 30.0:  # a progress line while a long stream drains
            last_note = now
            say(f"stream: {now:.0f} s, {n_req - len(wait_q) - len(pending)} of {n_req} done, "
                f"{len(pending)} in flight")
        while wait_q and arrive[wait_q[0]] <= now:
            i = wait_q[0]
            try:
                pending[i] = ctx.submit(reqs[i], precision=precision)
                wait_q.pop(0)
            except fmc.FmcError as e:
                if e.code != fmc.EBUSY:
                    raise
                refused += 1
                refused_req.add(i)
                break
        for i in list(pending):
            if pending[i].poll() is not None:
                done_at[i] = time.perf_counter() - t0
                del pending[i]
        time.sleep(0.001)
    _poisson_stream.refused_requests = len(refused_req)
    return done_at, refused


def serve_sweep(fmc, workloads, oracle_mod, rates, n_max: int, seconds: float, seed: int = 11):
    """The served form over Poisson rates: per rate min(n_max, seconds * rate)
    requests (nine in ten drawn from the 64 uneven classical scenarios, every
    tenth a large flux-decay request of 200 machines, T = 30 s, N = 5e4), in a
    context of its own; p50/p99 latency of small and large requests apart,
    completed requests and trajectory-steps per second.  Then one stream at
    the highest rate of the call, without the large requests, through a small
    serving arena (FMC_SERVE_ARENA_BYTES: 1.2 times the largest small request's
    footprint, so that two large ones never fit together), in which admission
    by footprint refuses requests (EBUSY) and the client retries; and one
    request of the large shape on a short horizon (N = 40) against the
    oracle."""
    import numpy as np
    scs = workloads.uneven_batch()
    large = workloads.fluxdecay()
    out = {"workload": "Poisson requests: 90% drawn uniformly from the 64 uneven classical "
                       "scenarios, 10% large flux-decay + IEEE type-1 requests (n=200, P=10, "
                       "T=30 s, N=5e4, K=100)",
           "precision": "bf16x3", "requests_per_rate": f"min({n_max}, {seconds:g} s x rate)",
           "rates": []}
    rng = np.random.default_rng(seed)

    def stream(rate):
        n_req = int(max(10, min(n_max, round(seconds * rate))))
        gaps = rng.exponential(1.0 / rate, size=n_req)
        arrive = np.cumsum(gaps) - gaps[0]
        pick = rng.integers(0, len(scs), size=n_req)
        is_large = np.array([i % 10 == 5 for i in range(n_req)])
        return [large if is_large[i] else scs[pick[i]] for i in range(n_req)], arrive, is_large

    def warm(ctx):
        for i in (0, 17, 40):
            ctx.submit(scs[i], precision="bf16x3").wait(timeout=300)
        ctx.submit(workloads.fluxdecay(T=0.25), precision="bf16x3").wait(timeout=300)

    ctx = fmc.Context(0)
    warm(ctx)
    say("serve sweep: warm")
    for rate in rates:
        reqs, arrive, is_large = stream(rate)
        done_at, refused = _poisson_stream(ctx, fmc, reqs, arrive)
        lat = done_at - arrive
        ts = float(sum(r["N"] * fmc.steps(r) for r in reqs))
        ent = _latency_summary(lat, is_large, float(done_at.max()), ts, len(reqs), refused, rate)
        out["rates"].append(ent)
        say(f"serve sweep rate {rate}/s: {len(reqs)} requests, p50 {ent['p50_latency_s']:.3f} s, "
            f"p99 {ent['p99_latency_s']:.3f} s, {ent['completed_req_per_s']:.2f} req/s done")
    ctx.close()
    # knee: the highest rate whose completed rate keeps up with the offered rate
    keep = [e for e in out["rates"] if e["completed_req_per_s"] >= 0.9 * e["rate_req_per_s"]]
    out["knee_req_per_s"] = max((e["rate_req_per_s"] for e in keep), default=None)
    out["saturation_req_per_s"] = max(e["completed_req_per_s"] for e in out["rates"])
    out["saturation_trajectory_steps_per_s"] = max(e["trajectory_steps_per_s"] for e in out["rates"])
    # a small arena: admission by footprint must refuse and the client retry
    arena = int(1.2 * max(fmc.footprint(sc, precision="bf16x3") for sc in scs))
    os.environ["FMC_SERVE_ARENA_BYTES"] = str(arena)
    ctx = fmc.Context(0)
    try:
        rate = max(rates)
        reqs, arrive, is_large = stream(rate)
        keep_small = ~is_large  # the large request needs more than the small arena
        reqs = [r for r, k in zip(reqs, keep_small) if k]
        arrive = arrive[keep_small]
        done_at, refused = _poisson_stream(ctx, fmc, reqs, arrive)
        lat = done_at - arrive
        ts = float(sum(r["N"] * fmc.steps(r) for r in reqs))
        ent = _latency_summary(lat, np.zeros(len(reqs), dtype=bool), float(done_at.max()), ts,
                               len(reqs), refused, rate)
        ent["arena_bytes"] = arena
        ent["requests_refused_at_least_once"] = _poisson_stream.refused_requests
        out["small_arena"] = ent
        say(f"small arena ({arena >> 20} MB) at {rate}/s: {refused} EBUSY retries, "
            f"p99 {ent['p99_latency_s']:.3f} s")
    finally:
        del os.environ["FMC_SERVE_ARENA_BYTES"]
        ctx.close()
    if oracle_mod is not None:
        ctx = fmc.Context(0)
        sc = workloads.fluxdecay(N=40, K=20, T=0.25)
        r = ctx.submit(sc, precision="bf16x3").wait(timeout=300)
        o = oracle_mod.run(sc)
        m, v = r["mean"].cpu().numpy(), r["var"].cpu().numpy()
        sm = np.maximum(np.abs(o["mean"]).max(axis=0), np.sqrt(o["var"]).max(axis=0))
        out["large_shape_vs_oracle"] = {
            "workload": "200 flux-decay machines, P=10, K=20, N=40, T=0.25 s (served)",
            "mean_rel": float((np.abs(m - o["mean"]).max(axis=0) / np.where(sm == 0, 1, sm)).max()),
            "var_rel": float((np.abs(v - o["var"]).max(axis=0)
                              / np.where(np.abs(o["var"]).max(axis=0) == 0, 1,
                                         np.abs(o["var"]).max(axis=0))).max())}
        ctx.close()
    return out


def served_leg(ctx, fmc, workloads, oracle_mod, rates, n_max: int, seed: int = 11):
    """Served form: a seeded Poisson request stream per rate.  Nine requests in
    ten are drawn from the 64-scenario uneven set (classical machines); every
    tenth (index 5, 15, ...) is a large flux-decay request (200 machines with
    IEEE type-1 exciters, 10 OU processes, T = 30 s, N = 5e4, K = 100).  A
    request refused for lack of HBM or slots (EBUSY) is retried by the client
    every millisecond; its latency runs from its scheduled arrival to the
    moment the client sees it complete."""
    import numpy as np
    import torch
    scs = workloads.uneven_batch()
    large = workloads.fluxdecay()
    rng = np.random.default_rng(seed)
    out = {"workload": "Poisson requests: 90% drawn uniformly from the 64 uneven classical "
                       "scenarios, 10% large flux-decay + IEEE type-1 requests (n=200, P=10, "
                       "T=30 s, N=5e4, K=100)",
           "precision": "bf16x3", "time_chunk": {"classical": 200, "flux_decay": 12},
           "rates": []}
    # warm-up: one request of every size class and one short flux-decay request
    for i in (0, 17, 40):
        ctx.submit(scs[i], precision="bf16x3").wait(timeout=300)
    ctx.submit(workloads.fluxdecay(T=0.25), precision="bf16x3").wait(timeout=300)
    say("served: warm")
    if oracle_mod is not None:
        small = int(np.argmin([sc["N"] * fmc.steps(sc) * sc["n_gen"] ** 2 for sc in scs]))
        r = ctx.submit(scs[small], precision="bf16x3").wait(timeout=300)
        o = oracle_mod.run(scs[small])
        m, v = r["mean"].cpu().numpy(), r["var"].cpu().numpy()
        sm = np.maximum(np.abs(o["mean"]).max(axis=0), np.sqrt(o["var"]).max(axis=0))
        out["error_vs_oracle"] = {
            "scenario": small,
            "mean_rel": float((np.abs(m - o["mean"]).max(axis=0) / sm).max()),
            "var_rel": float((np.abs(v - o["var"]).max(axis=0)
                              / np.abs(o["var"]).max(axis=0)).max())}
    for rate in rates:
        n_req = int(max(8, min(n_max, 8 * rate)))
        gaps = rng.exponential(1.0 / rate, size=n_req)
        arrive = np.cumsum(gaps) - gaps[0]
        pick = rng.integers(0, len(scs), size=n_req)
        is_large = np.array([i % 10 == 5 for i in range(n_req)])
        req = [large if is_large[i] else scs[pick[i]] for i in range(n_req)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pending = {}   # index -> ticket
        done_at = np.zeros(n_req)
        wait_q = list(range(n_req))
        refused = 0
        while wait_q or pending:
            now = time.perf_counter() - t0
            while wait_q and arrive[wait_q[0]] <= now:
                i = wait_q[0]
                try:
                    pending[i] = ctx.submit(req[i], precision="bf16x3")
                    wait_q.pop(0)
                except fmc.FmcError as e:
                    if e.code != fmc.EBUSY:
                        raise
                    refused += 1
                    break
            for i in list(pending):
                if pending[i].poll() is not None:
                    done_at[i] = time.perf_counter() - t0
                    del pending[i]
            time.sleep(0.001)
        lat = done_at - arrive
        span = float(done_at.max())
        ts = float(sum(r["N"] * fmc.steps(r) for r in req))
        ent = {"rate_req_per_s": rate, "requests": n_req, "large_requests": int(is_large.sum()),
               "p50_latency_s": float(np.median(lat)), "p99_latency_s": float(np.quantile(lat, 0.99)),
               "max_latency_s": float(lat.max()), "makespan_s": span,
               "completed_req_per_s": n_req / span, "trajectory_steps_per_s": ts / span,
               "ebusy_retries": refused}
        if (~is_large).any():
            ent["small_p50_latency_s"] = float(np.median(lat[~is_large]))
            ent["small_p99_latency_s"] = float(np.quantile(lat[~is_large], 0.99))
        if is_large.any():
            ent["large_p50_latency_s"] = float(np.median(lat[is_large]))
        out["rates"].append(ent)
        say(f"served rate {rate}/s: {n_req} requests ({int(is_large.sum())} large), p50 "
            f"{np.median(lat):.3f} s, p99 {np.quantile(lat, 0.99):.3f} s, {ts / span:.3e} traj-steps/s")
    return out


def convergence_leg(ctx, fmc, workloads, n_max: int, out_path: str = ""):
    """Sample-count convergence of the two estimators (the paper's comparison,
    Sec. V-B, on synthetic systems): for N = 2..n_max, each N with a design of
    its own (seed 1000 + N), the mean and variance of a response from (a) KLE
    (paper basis, K = 40 / 100 / 6) with LHS and (b) traditional Monte Carlo,
    eq. 5 increments with simple random sampling.  Responses: the SMIB rotor
    angle and a 10-machine frequency deviation at the final time, and the
    case-study RRF (the RMS centre-of-inertia frequency deviation over 60 s
    under the wind model of eq. 11 with a generator trip at t = 1 s).
    D(N) = max - min of the estimate over N-4..N; an estimator has converged
    at tolerance tol at the first N from which D stays below tol.  Tolerances
    are fractions of the response's standard deviation (mean) and variance
    (variance), both from the largest-N KLE+LHS estimate.  out_path, if given,
    receives the estimates (numpy .npz)."""
    import numpy as np
    fr_m, fr_v = (0.02, 0.05, 0.1), (0.05, 0.1, 0.2)
    out = {"definition": "D(N) = max-min of the estimate over N-4..N; N_conv(tol) = first N "
                         "after which D stays below tol; tol as fractions of the reference "
                         "std (mean) and variance (variance)",
           "n_max": n_max, "tol_mean_frac_of_std": list(fr_m), "tol_var_frac_of_var": list(fr_v)}
    # responses: the SMIB rotor angle (an infinite bus holds the angle
    # reference) and, for the 10-machine system, whose common rotor angle is a
    # neutral mode that drifts freely, the frequency deviation of machine 1
    # and the case-study shape of Sec. V-B: the wind model of eq. 11, a
    # generator trip at t = 1 s, the RMS centre-of-inertia frequency deviation
    # over 60 s as the response (the RRF accumulated in the integrator), KLE
    # order 6 as in the paper
    # (20 ms steps, and N up to 400 only: every N is a run of its own, and a
    # 60 s run of a thousand samples takes about a tenth of a second)
    wt = workloads.wind_trip(dt=0.02)
    systems = {"smib": (workloads.config1(), 0, "rotor angle of the machine at t = T (rad)", n_max),
               "10gen": (workloads.config2(), 10, "frequency deviation of machine 1 at t = T (pu)",
                         n_max),
               "wind_trip_rrf": (wt, None, "RMS centre-of-inertia frequency deviation over "
                                           "[0, 60 s] (pu), wind model of eq. 11 on one machine, "
                                           "generator trip at t = 1 s, dt = 20 ms",
                                 min(n_max, 400))}
    dump = {}
    for name, (base, col, what, n_max) in systems.items():
        S = fmc.steps(base)
        ests = {}
        M = base["K"] * len(base["dist"]["gen"])
        rrf_w = workloads.coi_frequency_weights(base) if col is None else None
        for meth, over, n_min in (("kle_lhs", dict(basis="paper", sampler="lhs"), 2),
                                  ("em_srs", dict(basis="em", sampler="srs", K=S), 2),
                                  ("kle_lhs_decor", dict(basis="paper", sampler="lhs_decor"),
                                   M + 1)):
            m = np.full(n_max + 1, np.nan); v = np.full(n_max + 1, np.nan)
            t_note = time.perf_counter()
            for N in range(n_min, n_max + 1):
                if time.perf_counter() - t_note > 30.0:
                    t_note = time.perf_counter()
                    say(f"convergence {name} {meth}: N = {N}")
                sc = dict(base, N=N, seed=1000 + N, **over)
                if col is None:
                    r = ctx.run(sc, precision="f64", rrf_weights=rrf_w)
                    y = r["rrf"].cpu().numpy()
                    m[N] = float(y.mean())
                    v[N] = float(y.var(ddof=1))
                else:
                    r = ctx.run(sc, precision="f64")
                    m[N] = float(r["mean"][S, col])
                    v[N] = float(r["var"][S, col])
            ests[meth] = (m, v)
            dump[f"{name}_{meth}_mean"] = m
            dump[f"{name}_{meth}_var"] = v
            say(f"convergence {name} {meth}: done")
        m_ref, v_ref = ests["kle_lhs"][0][n_max], ests["kle_lhs"][1][n_max]
        entry = {"response": what, "T_s": base["T"], "K_kle": base["K"], "n_max": n_max,
                 "ref_mean": m_ref, "ref_var": v_ref}
        if col is None:
            # sample paths of the disturbance (the paper's Fig. 5): five KLE
            # paths (K = 6) and three of the traditional scheme, in the .npz;
            # their roughness, the mean |increment| per sqrt(dt), in the JSON
            xc = 2 * base["n_gen"]
            for meth, over, k in (("kle_lhs", dict(basis="paper", sampler="lhs"), 5),
                                  ("em_srs", dict(basis="em", sampler="srs", K=S), 3)):
                sc = dict(base, N=8, seed=7, **over)
                rp = ctx.run(sc, precision="f64", traj_idx=np.arange(k))
                paths = rp["traj"].cpu().numpy()[:, :, xc]
                dump[f"{name}_{meth}_paths"] = paths
                entry[f"{meth}_paths"] = {
                    "n": k, "min": float(paths.min()), "max": float(paths.max()),
                    "mean_abs_increment_per_sqrt_dt":
                        float(np.mean(np.abs(np.diff(paths, axis=1))) / np.sqrt(base["dt"]))}

        def fin(x):
            return float(x) if np.isfinite(x) else None

        def dcurve(e):
            d = np.full(n_max + 1, np.inf)
            for N in range(6, n_max + 1):
                w = e[N - 4:N + 1]
                d[N] = w.max() - w.min()
            return d

        def n_conv(d, tol):
            ok = d <= tol
            for N in range(6, n_max + 1):
                if ok[N:].all():
                    return N
            return None
        # RMS error of the estimates against the reference over ranges of N
        # (relative to the std for the mean, to the variance for the
        # variance); with errors ~ 1/sqrt(N) the squared ratio of the two
        # methods' errors is their ratio of samples for equal accuracy
        ranges = ((10, 50), (100, 200), (max(200, n_max // 2), n_max))
        rms = {}
        for meth, (m, v) in ests.items():
            # NaN where a method has no estimate (the reduced design needs N > M)
            rms[meth] = [(float(np.sqrt(np.nanmean((m[a:b] - m_ref) ** 2)) / np.sqrt(v_ref))
                          if np.isfinite(m[a:b]).any() else None,
                          float(np.sqrt(np.nanmean((v[a:b] - v_ref) ** 2)) / v_ref)
                          if np.isfinite(v[a:b]).any() else None) for a, b in ranges]
        entry["rms_error_ranges"] = [f"{a}-{b - 1}" for a, b in ranges]
        def sq_ratio(a, b):
            return (a / b) ** 2 if a is not None and b else None
        entry["sample_ratio_em_over_kle"] = {
            "mean": [sq_ratio(e[0], k[0]) for e, k in zip(rms["em_srs"], rms["kle_lhs"])],
            "var": [sq_ratio(e[1], k[1]) for e, k in zip(rms["em_srs"], rms["kle_lhs"])]}
        # the reduced design exists for N > M only: both over the same N
        md, vd = ests["kle_lhs_decor"]
        ml, vl = ests["kle_lhs"]
        ratio = {"mean": [], "var": []}
        for a, b in ranges:
            ok = np.isfinite(md[a:b])
            for q, el, ed, ref in (("mean", ml, md, m_ref), ("var", vl, vd, v_ref)):
                if not ok.any():
                    ratio[q].append(None)
                    continue
                rl = np.mean((el[a:b][ok] - ref) ** 2)
                rd = np.mean((ed[a:b][ok] - ref) ** 2)
                ratio[q].append(float(rl / rd) if rd > 0 else None)
        entry["sample_ratio_lhs_over_lhs_decor"] = ratio
        entry["lhs_decor_first_N"] = int(M + 1)
        for meth, (m, v) in ests.items():
            dm, dv = dcurve(m), dcurve(v)
            entry[meth] = {
                "N_conv_mean": [n_conv(dm, f * np.sqrt(v_ref)) for f in fr_m],
                "N_conv_var": [n_conv(dv, f * v_ref) for f in fr_v],
                "D_mean_over_std_at": {str(N): fin(dm[N] / np.sqrt(v_ref))
                                       for N in (10, 50, 100, 500, n_max) if N <= n_max},
                "D_var_over_var_at": {str(N): fin(dv[N] / v_ref)
                                      for N in (10, 50, 100, 500, n_max) if N <= n_max},
                "rms_mean_over_std": [x[0] for x in rms[meth]],
                "rms_var_over_var": [x[1] for x in rms[meth]]}
        out[name] = entry
        say(f"convergence {name}: " + json.dumps({k: {q: entry[k][q] for q in ("N_conv_mean", "N_conv_var")}
                                                  for k in ("kle_lhs", "em_srs")})
            + " sample ratio " + json.dumps(entry["sample_ratio_em_over_kle"]))
    if out_path:
        np.savez(out_path, **dump)
    return out


def decor_leg(ctx, fmc, workloads, reps: int = 3):
    """Correlation-reducing LHS permutation (Sec. IV-B, LHS Step 2) on the
    10-machine workload's design (M = P*K = 300 rows, N = 1e4): the design
    alone with and without the reduction (host clock around the synchronous
    call), the off-diagonal correlation of the rows before and after, and a
    whole FP64 pass of the method with each design."""
    import numpy as np
    import torch
    sc = workloads.config2()
    M, N = len(sc["dist"]["gen"]) * sc["K"], sc["N"]
    out = {"M": M, "N": N}
    for name in ("lhs", "lhs_decor"):
        best = float("inf")
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, z = ctx.lhs(seed=sc["seed"], M=M, N=N, sampler=name)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        zz = z.cpu().numpy()
        c = np.corrcoef(zz)
        off = c[~np.eye(M, dtype=bool)]
        out[name] = {"design_ms": best * 1e3, "rms_offdiag_corr": float(np.sqrt(np.mean(off ** 2))),
                     "max_abs_offdiag_corr": float(np.abs(off).max())}
        sc2 = dict(sc, sampler=name)
        vid = ctx.autotune(sc, precision="f64")
        ctx.run(sc2, precision="f64", variant=vid)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.run(sc2, precision="f64", variant=vid)
        torch.cuda.synchronize()
        out[name]["run_ms"] = (time.perf_counter() - t0) / reps * 1e3
        say(f"design {name}: {best * 1e3:.2f} ms, whole FP64 pass {out[name]['run_ms']:.2f} ms, "
            f"rms off-diagonal correlation {out[name]['rms_offdiag_corr']:.2e}")
    return out


def corr_leg(ctx, fmc, workloads, reps: int = 3):
    """Correlated disturbances (a 3 x 3 diffusion matrix, eq. 4 with a full
    sigma) on the 10-machine workload: a whole FP64 pass with and without the
    matrix (the design is mixed once before the path contraction), and the
    correlation the matrix puts between the disturbances at t = T."""
    import numpy as np
    import torch
    sc = workloads.config2()
    smat = np.array([[0.09, 0.0, 0.03], [0.05, 0.07, 0.0], [-0.02, 0.04, 0.06]])
    mixed = dict(sc, dist=dict(sc["dist"], sigma_mat=smat))
    vid = ctx.autotune(sc, precision="f64")
    out = {"sigma_mat": smat.tolist()}
    for name, s in (("vector_sigma", sc), ("sigma_mat", mixed)):
        ctx.run(s, precision="f64", variant=vid)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = ctx.run(s, precision="f64", variant=vid)
        torch.cuda.synchronize()
        out[name + "_run_ms"] = (time.perf_counter() - t0) / reps * 1e3
    say(f"diffusion matrix: whole FP64 pass {out['sigma_mat_run_ms']:.2f} ms "
        f"(vector sigma {out['vector_sigma_run_ms']:.2f} ms)")
    return out


def rrf_leg(ctx, fmc, workloads, reps: int = 3):
    """Scalar RRF (eq. 3; Sec. V-B): every trajectory of the 10-machine
    workload stored by one FP64 pass (N x (S+1) x V doubles), then the RMS of
    the centre-of-inertia frequency deviation over the horizon for each, timed
    on the host clock around the synchronous fmc_rrf_rms call."""
    import numpy as np
    import torch
    sc = workloads.config2()
    n, N = sc["n_gen"], sc["N"]
    V = 2 * n + len(sc["dist"]["gen"])
    H = np.asarray(sc["H"], dtype=np.float64)
    w = np.zeros(V)
    w[n:2 * n] = H / H.sum()
    r = ctx.run(sc, precision="f64", traj_idx=np.arange(N))
    traj = r["traj"]
    rrf = ctx.rrf_rms(traj, w, sc["dt"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        rrf = ctx.rrf_rms(traj, w, sc["dt"])
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    nbytes = traj.numel() * 8
    out = {"n_traj": N, "traj_bytes": nbytes, "ms": sec * 1e3, "GB_per_s": nbytes / sec / 1e9,
           "rrf_mean": float(rrf.mean()), "rrf_var": float(rrf.var(unbiased=True))}
    say(f"RRF (RMS of the centre-of-inertia frequency deviation) over {N} stored trajectories "
        f"({nbytes / 1e9:.2f} GB): {sec * 1e3:.2f} ms, {nbytes / sec / 1e9:.0f} GB/s")
    del traj, r
    torch.cuda.empty_cache()
    return out


PEAK_MFMA_FP64 = 78.6e12
PEAK_MFMA_BF16 = 2.5e15
PEAK_HBM = 8.0e12


def kle_leg(ctx, fmc, reps: int, copy_check: bool = False):
    """The KLE path contraction (eqs. 8-9) alone, on the chunk shapes fmc_run
    uses: the 10-machine workload (N = 1e4, chunks of 209 steps: 419 stage
    columns) and the N = 1e5 workload (chunks of 41 steps: 83 columns), P = 3
    processes, K = 100.  Each form is one fmc_kle_paths call per repetition,
    timed with events on the context's stream; the BF16 x3 call includes the
    hi/lo split of both operands (two short launches before the contraction,
    which fmc_run makes once per run for the design).  Algorithmic work: 2 K
    flops per output element; bytes: the design read once (8 B per element in
    FP64, 4 B as BF16 hi/lo) and the paths written once."""
    import torch
    out = {}
    for name, (P, K, N, C) in {"N1e4_chunk209": (3, 100, 10000, 419),
                               "N1e5_chunk41": (3, 100, 100000, 83)}.items():
        _, z = ctx.lhs(seed=2, M=P * K, N=N)
        S = (C - 1) // 2
        phi = ctx.basis(0, K, S, 0.005 * S)
        for prec in ("f64", "f32", "bf16x3"):
            w = ctx.kle_paths(z, phi, P, K, C, precision=prec)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                w = ctx.kle_paths(z, phi, P, K, C, precision=prec)
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) * 1e-3 / reps
            flops = 2.0 * K * P * N * C
            zb = (8 if prec != "bf16x3" else 4) * P * K * N
            wb = w.numel() * w.element_size()
            r = {"shape": {"P": P, "K": K, "N": N, "C": C}, "call_ms": t * 1e3,
                 "tflops": flops / t / 1e12, "hbm_gbps": (zb + wb) / t / 1e9,
                 "hbm_frac": (zb + wb) / t / PEAK_HBM}
            if prec == "bf16x3":
                r["mfma_frac"] = 3 * flops / t / PEAK_MFMA_BF16
                # fmc_run splits the design once per run and only the basis
                # per chunk; this call splits both (the kernel trace under
                # profiles/ separates the split from the contraction)
                r["includes_design_split"] = True
            else:
                r["mfma_frac"] = flops / t / PEAK_MFMA_FP64
            out[f"{name}_{prec}"] = r
            note = " (with the hi/lo split of the design)" if prec == "bf16x3" else ""
            say(f"kle {name} {prec}{note}: {t * 1e6:.1f} us, {flops / t / 1e12:.1f} TFLOP/s")
        del z, phi, w
    if copy_check:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    return out


def fd_leg(ctx, fmc, workloads, oracle_mod, steps: int, reps: int = 2):
    """Large-request shape of the flux-decay model (200 machines with IEEE
    type-1 exciters, 10 OU processes, N = 5e4, K = 100) on a horizon of
    `steps` steps: throughput and the network product's rate against the FP32
    matrix-core peak; sampled trajectories against the oracle."""
    import numpy as np
    import torch
    sc = workloads.fluxdecay(T=steps * 0.005)
    n, P, N = sc["n_gen"], len(sc["dist"]["gen"]), sc["N"]
    S = fmc.steps(sc)
    out = {"workload": "flux-decay + IEEE type-1, n=200, P=10, K=100, N=5e4, dt=5 ms, "
                       f"{S} steps (the large served request's shape on a short horizon)",
           "flops_per_traj_step": fd_flops_per_traj_step(n, P)}
    sel = np.array([7, N // 2, N - 1])
    ref = None
    if oracle_mod is not None:
        ref = oracle_mod.run(sc, sel=sel, want_traj=True)["traj"]
    # bf16x3: BF16 x3 KLE paths, FP32 integration; bf16x3_net: the network
    # product in BF16 x3 split products as well (variant 1, opt-in)
    for form, prec, var in (("f32", "f32", -1), ("bf16x3", "bf16x3", -1),
                            ("bf16x3_net", "bf16x3", 1)):
        ctx.run(sc, precision=prec, variant=var)  # warm
        torch.cuda.synchronize()
        t_int = 0.0
        t0 = time.perf_counter()
        for _ in range(reps):
            r = ctx.run(sc, precision=prec, variant=var)
            t_int += r["report"]["t_integrate_s"]
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / reps
        t_int /= reps
        ent = {"trajectory_steps_per_s": N * S / sec, "ms_per_run": sec * 1e3,
               "integrator_ms": t_int * 1e3,
               "integrator_traj_steps_per_s": N * S / t_int,
               "network_product_tflops": 8.0 * n * n * 4 * N * S / t_int / 1e12,
               "frac_of_fp32_matrix_peak": 8.0 * n * n * 4 * N * S / t_int / PEAK_FP32_MATRIX}
        if ref is not None:
            rt = ctx.run(sc, precision=prec, traj_idx=sel, variant=var)["traj"].cpu().numpy()
            d = ref - ref[:, :1, :]
            num = np.abs(rt - ref).reshape(-1, rt.shape[-1]).max(axis=0)
            den = np.maximum(np.abs(d).reshape(-1, rt.shape[-1]).max(axis=0), 1e-6)
            ent["traj_rel_sampled"] = float((num / den).max())
        out[form] = ent
        say(f"flux-decay {form}: {sec * 1e3:.1f} ms per run, integrator {t_int * 1e3:.1f} ms, "
            f"{ent['network_product_tflops']:.1f} TFLOP/s network product")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--forms", default="f64,f32,bf16x3")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--variant", type=int, default=-1,
                    help="integrator variant; -1 lets the autotuner choose (untimed)")
    ap.add_argument("--batch-steps", type=int, default=2,
                    help="timed passes over the 64-scenario batched workload (0: skip)")
    ap.add_argument("--serve-rates", default="1,10,50,200",
                    help="Poisson request rates of the served leg (empty: skip)")
    ap.add_argument("--serve-max", type=int, default=20,
                    help="requests per rate of the served leg (at most)")
    ap.add_argument("--fd-steps", type=int, default=100,
                    help="horizon of the flux-decay leg in steps (0: skip)")
    ap.add_argument("--decor-reps", type=int, default=3,
                    help="passes of the reduced-design, diffusion-matrix and RRF legs (0: skip)")
    ap.add_argument("--convergence", type=int, default=300,
                    help="run the sample-count convergence comparison up to this N (0: skip; "
                         "1000 as in the paper takes about three minutes)")
    ap.add_argument("--convergence-out", default="",
                    help="write the convergence estimates to this .npz file")
    ap.add_argument("--serve-sweep", default="",
                    help="served form only: comma-separated Poisson rates, each run in its own "
                         "context (see serve_sweep); prints the sweep as one JSON line")
    ap.add_argument("--sweep-max", type=int, default=100,
                    help="requests per rate of the serve sweep (at most)")
    ap.add_argument("--sweep-seconds", type=float, default=60.0,
                    help="arrival window per rate of the serve sweep")
    ap.add_argument("--time-chunk", type=int, default=0,
                    help="time chunk of the forms' runs in steps (0: the library's choice; the "
                         "whole horizon leaves one statistics merge over all rows, after the "
                         "integrator)")
    ap.add_argument("--plain-f64", action="store_true",
                    help="batched leg: also run every scenario in turn through fmc_run in FP64 "
                         "(the plain reference; about 90 s)")
    ap.add_argument("--c1", type=int, default=1,
                    help="run the single-machine FP64 leg (1) or not (0)")
    ap.add_argument("--gen-steps", type=int, default=2,
                    help="timed passes of the general-Ito-process workload (0: skip)")
    ap.add_argument("--c3-steps", type=int, default=2,
                    help="timed passes of the N=1e5 mixed-precision workload (0: skip)")
    ap.add_argument("--kle-reps", type=int, default=20,
                    help="repetitions of the standalone KLE contraction leg (0: skip)")
    ap.add_argument("--kle-only", action="store_true",
                    help="run the standalone KLE contraction leg only and print it as one "
                         "JSON line (for kernel profiles)")
    ap.add_argument("--copy-check", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; every box has one GPU, "
                                   "run with --gpus 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2007_03847_amd as fmc
    import workloads

    if args.serve_sweep:
        rates = [float(x) for x in args.serve_sweep.split(",") if x.strip()]
        res = serve_sweep(fmc, workloads, None if args.no_cpu else oracle_mod(), rates,
                          args.sweep_max, args.sweep_seconds)
        print(json.dumps({"metric": "served p50/p99 latency and throughput", "serve_sweep": res}))
        return

    dev = torch.device("cuda", 0)
    ctx = fmc.Context(0)
    if args.kle_only:
        res = kle_leg(ctx, fmc, max(1, args.kle_reps), args.copy_check)
        print(json.dumps({"metric": "KLE path contraction alone", "kle_contraction": res}))
        ctx.close()
        return
    sc = workloads.config2()
    n, P, N, K = sc["n_gen"], len(sc["dist"]["gen"]), sc["N"], sc["K"]
    S = fmc.steps(sc)
    sel = np.array([0, 1, 2345, 5000, 7777, N - 1])
    forms = [f for f in args.forms.split(",") if f]

    results = {}
    tuned = {}
    for form in forms:
        # untimed: the autotuner picks the integrator variant for this workload
        vid = args.variant if args.variant >= 0 else ctx.autotune(sc, precision=form)
        tuned[form] = vid
        say(f"{form}: variant {vid}")
        outs = None
        for _ in range(args.warmup):
            r = ctx.run(sc, precision=form, variant=vid, time_chunk=args.time_chunk)
            outs = dict(mean=r["mean"], var=r["var"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_int = 0.0
        n_launch = 0
        reps = []
        for _ in range(args.steps):
            r = ctx.run(sc, precision=form, outputs=outs, variant=vid, time_chunk=args.time_chunk)
            outs = dict(mean=r["mean"], var=r["var"])
            reps.append(r["report"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms = (t1 - t0) * 1e3 / args.steps
        rep = reps[-1]
        t_int = sum(x["t_integrate_s"] for x in reps) / args.steps
        chunks = int(np.ceil(S / rep["time_chunk"]))
        # sampled trajectories for the error report
        rt = ctx.run(sc, precision=form, traj_idx=sel, variant=vid)
        say(f"{form}: {ms:.2f} ms per step, integrator {t_int * 1e3:.2f} ms")
        results[form] = dict(ms=ms, rep=rep, t_int=t_int, chunks=chunks,
                             mean=rt["mean"].cpu().numpy(), var=rt["var"].cpu().numpy(),
                             traj=rt["traj"].cpu().numpy())

    if args.copy_check:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters scale
        # the integrator's to bytes
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    # ---- CPU oracle: baseline timing and error reference
    cpu = None
    errs = {}
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        probe = oracle.run(sc, sel=np.arange(64))
        t_probe = time.perf_counter() - t0
        n_cpu = int(min(N, max(64, 64 * args.cpu_seconds / max(t_probe, 1e-3))))
        if n_cpu >= N:
            t0 = time.perf_counter()
            o = oracle.run(sc)
            t_cpu = time.perf_counter() - t0
            n_cpu = N
        else:
            cpu_sel = np.linspace(0, N - 1, n_cpu).round().astype(np.int64)
            t0 = time.perf_counter()
            o = oracle.run(sc, sel=cpu_sel)
            t_cpu = time.perf_counter() - t0
        say(f"cpu oracle: {n_cpu} samples in {t_cpu:.1f} s")
        threads = oracle.num_threads()
        # the same oracle on one thread, over a bounded sample
        oracle.set_num_threads(1)
        one_sel = np.linspace(0, N - 1, 32).round().astype(np.int64)
        t0 = time.perf_counter()
        oracle.run(sc, sel=one_sel)
        t_one = time.perf_counter() - t0
        oracle.set_num_threads(threads)
        cpu = {"value": n_cpu * S / t_cpu, "unit": "trajectory-steps/s",
               "cores": threads, "kind": "oracle",
               "sample": f"{n_cpu} of {N} samples of the same workload ({S} steps each), "
                         f"FP64 C oracle with OpenMP over samples, {t_cpu:.1f} s",
               "single_thread_value": len(one_sel) * S / t_one,
               "single_thread_sample": f"{len(one_sel)} samples on 1 thread, {t_one:.2f} s",
               "cpu_model": cpu_model(), "nproc": os.cpu_count()}
        ot = oracle.run(sc, sel=sel, want_traj=True)["traj"]
        for form, res in results.items():
            full = n_cpu == N
            errs[form] = per_output(res["mean"] if full else None, res["var"] if full else None,
                                    res["traj"], o["mean"] if full else None,
                                    o["var"] if full else None, ot)

    c1 = config1_leg(ctx, fmc, workloads, None if args.no_cpu else oracle_mod(), 10) \
        if args.c1 else None

    gen = general_leg(ctx, fmc, workloads, None if args.no_cpu else oracle_mod(), args.gen_steps) \
        if args.gen_steps > 0 else None

    c3 = None
    if args.c3_steps > 0:
        c3 = config3_leg(ctx, fmc, workloads, None if args.no_cpu else oracle_mod(), args.c3_steps)

    batched = None
    if args.batch_steps > 0:
        batched = batched_leg(ctx, fmc, workloads, None if args.no_cpu else oracle_mod(),
                              args.batch_steps, args.plain_f64)

    decor = corr = rrf = None
    if args.decor_reps > 0:
        decor = decor_leg(ctx, fmc, workloads, args.decor_reps)
        corr = corr_leg(ctx, fmc, workloads, args.decor_reps)
        rrf = rrf_leg(ctx, fmc, workloads, args.decor_reps)

    conv = None
    if args.convergence > 0:
        conv = convergence_leg(ctx, fmc, workloads, args.convergence, args.convergence_out)

    fdl = None
    if args.fd_steps > 0:
        fdl = fd_leg(ctx, fmc, workloads, None if args.no_cpu else oracle_mod(), args.fd_steps)

    kle = kle_leg(ctx, fmc, args.kle_reps) if args.kle_reps > 0 else None

    served = None
    rates = [float(x) for x in args.serve_rates.split(",") if x.strip()]
    if rates:
        served = served_leg(ctx, fmc, workloads, None if args.no_cpu else oracle_mod(), rates,
                            args.serve_max)

    head = "f64" if "f64" in results else forms[0]
    res = results[head]
    value = N * S / (res["ms"] * 1e-3)
    flops_step = integrator_flops_per_traj_step(n, P)
    fs = integrator_flops_survey(n)
    # dominant kernel: the integrator.  achieved = algorithmic flops per launch
    # (all launches of a pass, averaged) / mean launch time, both from the same
    # pass totals, so that flops_per_launch / mean_launch_ms == achieved
    chunks = res["chunks"]
    flops_launch = fs * N * S / chunks
    mean_launch_s = res["t_int"] / chunks
    achieved = flops_launch / mean_launch_s if mean_launch_s > 0 else 0.0
    peak = PEAK_FP64_VECTOR if head == "f64" else PEAK_FP32_VECTOR
    traffic, traffic_steps = measured_traffic(res["rep"]["variant_id"], head)
    if traffic is not None and traffic_steps != res["rep"]["time_chunk"]:
        traffic = None
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": traffic,
            "kernel": "k_rk4_group" if res["rep"]["lanes_per_traj"] > 1 else "k_rk4_lane",
            "flops_per_traj_step": fs, "flops_per_launch": flops_launch,
            "mean_launch_ms": mean_launch_s * 1e3, "launches_per_pass": chunks,
            "frac_sincos_as_20_flops": (fs + 4 * n * SINCOS_FLOPS) * N * S / res["t_int"] / peak,
            "frac_itemised_count": flops_step * N * S / res["t_int"] / peak,
            "itemised_flops_per_traj_step": flops_step}
    forms_out = {}
    for form, r in results.items():
        forms_out[form] = {"value": N * S / (r["ms"] * 1e-3), "ms_per_step": r["ms"],
                           "integrator_ms": r["t_int"] * 1e3,
                           "integrator_tflops": fs * N * S / r["t_int"] / 1e12,
                           "gemm_ms": r["rep"]["t_gemm_s"] * 1e3,
                           "lhs_ms": r["rep"]["t_lhs_s"] * 1e3,
                           "stats_ms": r["rep"]["t_stats_s"] * 1e3,
                           "variant": r["rep"]["variant_id"],
                           "lanes_per_traj": r["rep"]["lanes_per_traj"],
                           "group_size": r["rep"]["tile"],
                           "time_chunk": r["rep"]["time_chunk"],
                           "error_vs_oracle": errs.get(form)}
    line = {
        "metric": "trajectory-steps/s", "value": value, "unit": "trajectory-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "bf16x3": "bf16x3+f32"}[head],
        "data": "synthetic",
        "config": {"workload": "10-machine classical swing model, seeded 39-bus synthetic "
                               "network, 3 OU disturbances, K=100, N=1e4, T=20 s, dt=5 ms "
                               "(4000 RK4 steps), LHS seed 2",
                   "n_gen": n, "n_proc": P, "K": K, "N": N, "steps": S, "precision": head},
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": forms_out,
        "smib_N1e3": c1,
        "mixed_precision_N1e5": c3,
        "general_processes": gen,
        "kle_contraction": kle,
        "batched": batched,
        "served": served,
        "flux_decay": fdl,
        "convergence": conv,
        "lhs_decor": decor,
        "correlated_disturbances": corr,
        "rrf": rrf,
    }
    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()
