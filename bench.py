#!/usr/bin/env python3
"""Benchmark: sequence evaluations per second including the gradient, 2 qubits, FP64.

One step = one evaluation of the whole path on the two-qubit GST list: outcome
probabilities of every sequence, the negative log-likelihood of the counts and
its gradient with respect to every entry of rho, the effects and the gates
(resident request: the sequence list and counts stay on the device, the gate
set is new every step, as in the iterations of a fit).  Inputs are resident in
HBM before the timed region starts.

Prints one JSON line: metric, value, unit, timing, the workload, the roofline
of the dominant kernel family (algorithmic work per launch over its average
launch time, against the FP64 vector peak, with the HBM bytes per launch from
the committed counter file while the device sources are unchanged) and the
oracle's throughput on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sequence evals/s incl. gradient (2q, FP64); p50/p99 latency of served fits"
# MI355X published FP64 vector peak: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
PEAK_FP64 = 78.6
# predictions: the oracle runs the same workload (r = 0..1000, ~2 s a pass)
F3_CPU_RMAX = 1000


_DESC = {
    "c1": "c1: one-qubit GST list, 6 prep x 6 meas fiducials x 4 germs, powers 1..64, gates {Gi,Gx,Gy} "
          "with 1e-3 depolarizing + N(0,0.01) over-rotations, counts ~ Multinomial(1000)",
    "c2": "c2: two-qubit GST list, 11 prep x 11 meas fiducials x 12 germs, powers 1..256, "
          "gates {Gii,Gxi,Gix,Gyi,Giy,Gcz} with 1e-3 depolarizing + N(0,0.01) over-rotations, "
          "counts ~ Multinomial(1000)",
    "c4": "c4: three-qubit GST list, 16 prep x 16 meas fiducials x 98 germs, powers 1..128, gates "
          "{Gi,Gx,Gy,CZ01,CZ12} with 1e-3 depolarizing + N(0,0.01) over-rotations, counts ~ Multinomial(1000)",
}


def workload_desc(w):
    L = w.seqs.lengths()
    return {
        "workload": _DESC[w.name],
        "sequences": int(w.seqs.S),
        "sum_len": int(L.sum()),
        "max_len": int(L.max()),
        "n_qubits": int(w.model.n_qubits),
        "params": int(w.model.n_params()),
    }


# ---------------------------------------------------------------------------
# CPU baseline: the oracle, unchanged, on the machine's host cores
# ---------------------------------------------------------------------------
def _cpu_sample(name):
    """Oracle inputs for the CPU baseline: a list of (gate set, sequences, counts)."""
    from paper_2008_13490_amd import workloads as W
    if name == "c3":
        # the first 8 gate sets of the uneven batch, first 256 sequences of each
        out = []
        for kind, S, seed in W.c3_plan()[:8]:
            w = W.uneven_request(kind, S, seed)
            sub = w.seqs.subset(np.arange(256))
            out.append((w.model, sub, w.counts[:256]))
        return out, "first 8 gate sets of the uneven batch (6 one-qubit, 2 two-qubit by the seeded mix), " \
                    "256 sequences of each"
    if name == "c5":
        out = []
        for _, kind, S, seed in W.serving_trace(100.0, 8):
            d = W.serving_request(kind, S, seed, 1)
            out.append((d.iterates[0], d.seqs.subset(np.arange(256)), d.counts[:256]))
        return out, "first 8 requests of the serving trace, 256 sequences of each, first iterate"
    w = W.structured_workload(name)
    if name == "c4":
        # the full three-qubit list takes minutes per evaluation on one core
        idx = np.arange(0, w.seqs.S, 97)
        return [(w.model, w.seqs.subset(idx), w.counts[idx])], \
            f"c4 every 97th sequence ({len(idx)} of {w.seqs.S})"
    return [(w.model, w.seqs, w.counts)], f"{name} full list ({w.seqs.S} sequences)"


def _cpu_worker(args):
    name, seconds, param = args
    sys.path.insert(0, ROOT)
    import oracle
    n = 0
    seqs = 0
    t0 = time.perf_counter()
    if name == "f3":
        from paper_2008_13490_amd import workloads as W
        pw = W.prediction_workload(F3_CPU_RMAX)
        g, gi = pw.estimate, pw.ideal
        p_ideal = oracle.predict(gi.rho, gi.effects, gi.gates, pw.preps, pw.gates, pw.r_max)
        t0 = time.perf_counter()
        while True:
            oracle.tv_distance(oracle.predict(g.rho, g.effects, g.gates, pw.preps, pw.gates, pw.r_max), p_ideal)
            seqs += len(pw.preps) * len(pw.gates) * (pw.r_max + 1)
            n += 1
            if time.perf_counter() - t0 >= seconds:
                break
        return n, time.perf_counter() - t0, seqs
    sample, _ = _cpu_sample(name)
    if param != "full":
        from oracle import params as PR
        from paper_2008_13490_amd import workloads as W
        m, sl, cnt = sample[0]
        kind = {1: "1q", 2: "2q"}[m.n_qubits]
        G0 = W.ideal_targets(kind)
        th = W.param_point(param, m, 7)
        while True:
            rho, E, G = PR.forward(param, th, m.n_qubits, m.M, m.K, G0)
            _, _, g, _, _ = oracle.loglik(rho, E, G, sl.offsets, sl.gates, cnt)
            PR.backward(param, th, m.n_qubits, m.M, m.K, g, G0)
            seqs += sl.S
            n += 1
            if time.perf_counter() - t0 >= seconds:
                break
        return n, time.perf_counter() - t0, seqs
    while True:
        for m, sl, cnt in sample:
            oracle.loglik(m.rho, m.effects, m.gates, sl.offsets, sl.gates, cnt)
            seqs += sl.S
        n += 1
        if time.perf_counter() - t0 >= seconds:
            break
    return n, time.perf_counter() - t0, seqs


def cpu_baseline(name: str, seconds: float, workers: int, param: str = "full"):
    import multiprocessing as mp
    import oracle
    oracle.build(force=not os.path.exists(oracle.library_path()))
    if name == "f3":
        what = (f"the full workload: four initial states x 6 gates x r = 0..{F3_CPU_RMAX} as plain words, "
                f"with the distance to the ideal predictions")
    else:
        _, what = _cpu_sample(name)
    ctx = mp.get_context("spawn")
    # one thread per worker process: the parameterization oracle uses numpy /
    # scipy, whose BLAS would otherwise start a thread pool in every worker
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    print(f"[bench] cpu baseline: {workers} oracle processes for ~{seconds:.0f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    try:
        with ctx.Pool(workers) as pool:
            res = pool.map(_cpu_worker, [(name, seconds, param)] * workers)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    wall = time.perf_counter() - t0
    print(f"[bench] cpu baseline done in {wall:.1f} s", file=sys.stderr, flush=True)
    passes = sum(r[0] for r in res)
    seqs = sum(r[2] for r in res)
    busy = max(r[1] for r in res)
    return {
        "value": seqs / busy,
        "unit": "predicted distributions/s" if name == "f3" else "sequence evals/s",
        "cores": workers,
        "kind": "oracle",
        "sample": f"{what} evaluated {passes} times{'' if name == 'f3' else ' with gradient'}"
                  f"{'' if param == 'full' else f' in the {param.upper()} parameterization'}, "
                  f"{workers} single-threaded processes for ~{seconds:.0f} s each (wall {wall:.1f} s)",
    }


# ---------------------------------------------------------------------------
# the source file of each kernel family (the counters of a family stay valid
# while this file and the headers it includes are unchanged)
FAMILY_SOURCE = {
    "leaf": ["gst_plan_kernels.hip"], "trunk_fwd": ["gst_plan_kernels.hip"], "trunk_bwd": ["gst_plan_kernels.hip"],
    "inject": ["gst_plan_kernels.hip"], "fill": ["gst_plan_kernels.hip"], "grad_gemm": ["gst_plan_kernels.hip"],
    "reduce": ["gst_plan_kernels.hip"], "tiles_3q_fwd": ["gst_kernels64.hip"], "tiles_3q_bwd": ["gst_kernels64.hip"],
    "readout_3q": ["gst_kernels64.hip"], "gemm_3q": ["gst_kernels64.hip"],
    "reduce_3q": ["gst_kernels64.hip", "gst_kernels.hip"], "chain_3q": ["gst_kernels64.hip"],
    "tiles_2q": ["gst_batch.hip"], "tiles_1q": ["gst_lane1q.hip"], "tiles_reduce": ["gst_batch.hip"],
}


def kernel_source_hash(sources=None):
    """Hash of device code: the given .hip sources (default: all of them) and
    the headers they include (transitively); the counters recorded in
    profiles/ are used only while it is unchanged.  Host-only sources do not
    enter it."""
    import re
    csrc = os.path.join(ROOT, "paper_2008_13490_amd", "csrc")
    files = set(sources) if sources else {f for f in os.listdir(csrc) if f.endswith(".hip")}
    todo = sorted(files)
    while todo:
        f = todo.pop()
        for inc in re.findall(r'#include\s+"([^"]+)"', open(os.path.join(csrc, f)).read()):
            name = os.path.basename(inc)
            if name not in files and os.path.exists(os.path.join(csrc, name)):
                files.add(name)
                todo.append(name)
    h = hashlib.sha256()
    for f in sorted(files):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def read_counters(workload: str, family: str):
    """Counted FP64 flops and HBM bytes per launch of a kernel family from the
    committed counter summary (profiles/counters_<workload>.txt), if it was
    taken on the current kernel sources; else None.  FP64 flops are
    64 (ADD + MUL + TRANS + 2 FMA) per VALU instruction count plus 512 per
    MFMA_MOPS unit (the SQ_INSTS_VALU_*_F64 counters)."""
    path = os.path.join(ROOT, "profiles", f"counters_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("#") or "=" not in line:
            continue
        k, v = line.split("=", 1)
        vals[k.strip()] = v.strip()
    src = FAMILY_SOURCE.get(family)
    if not src or vals.get(f"{family}_source_hash") != kernel_source_hash(src):
        return None
    out = {}
    for q in ("fp64_flop", "fetch_bytes", "write_bytes"):
        key = f"{family}_{q}_per_launch"
        if key in vals:
            out[q] = float(vals[key])
    return out or None


def with_counters(roof, counters):
    """Adds the counter-measured figures to a roofline entry: FP64 FLOP/s and its
    fraction of peak, the ratio of counted to algorithmic flops, HBM traffic."""
    if not counters:
        roof["counter_flop_per_launch"] = None
        return roof
    avg_s = roof["avg_launch_us"] * 1e-6
    if "fp64_flop" in counters:
        cf = counters["fp64_flop"]
        roof["counter_flop_per_launch"] = cf
        roof["counter_tflops"] = cf / avg_s / 1e12
        roof["counter_frac"] = roof["counter_tflops"] / roof["peak"]
        roof["counter_to_algorithmic"] = cf / roof["algorithmic_flop_per_launch"] \
            if roof["algorithmic_flop_per_launch"] else None
    if "fetch_bytes" in counters and "write_bytes" in counters:
        tb = counters["fetch_bytes"] + counters["write_bytes"]
        roof["traffic"] = tb
        roof["hbm_gbs"] = tb / avg_s / 1e9
    return roof


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c2x64", "c3", "c4", "c4x8", "c5", "f2", "f3"])
    ap.add_argument("--fit-iters", type=int, default=100, help="f2: L-BFGS iterations per MLGST stage")
    ap.add_argument("--rate", type=float, default=100.0, help="c5 / serving: arrivals per second")
    ap.add_argument("--serving-rates", default="", help="c5: comma-separated arrival rates to sweep")
    ap.add_argument("--slots", type=int, default=8, help="serving: requests admitted at once")
    ap.add_argument("--requests", type=int, default=100, help="c5 / serving: requests in the trace")
    ap.add_argument("--iters", type=int, default=20, help="c5 / serving: iterations per request")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving measurement of the default run")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched measurement (c2x64 with c2, c4x8 with c4)")
    ap.add_argument("--no-autotune", action="store_true", help="c3: keep the default tile policy")
    ap.add_argument("--round-work", type=float, default=8e6,
                    help="serving: bound on the work of one round, in two-qubit sequence steps")
    ap.add_argument("--path", choices=["resident", "plain"], default="resident")
    ap.add_argument("--param", choices=["full", "tp", "cptp"], default="full",
                    help="c1/c2: estimation mode; the step maps theta to the gate set and the gradient back")
    ap.add_argument("--sets", type=int, default=0, help="c3: use only the first N gate sets")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--cpu-workers", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB mebibytes device to device a few times (reference kernel for the "
                         "HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the path would shard by sequence and all-reduce the "
                                   "gradient, but it has no multi-GPU run", "n_gpus": args.gpus}))
        sys.exit(2)

    if args.workload == "f2":
        out = run_fit_bench(args)
        print(json.dumps(out))
        return
    # CPU baseline first, before anything touches the GPU.
    cpu = None
    if not args.no_cpu:
        workers = args.cpu_workers or max(1, min(16, os.cpu_count() or 1))
        cpu = cpu_baseline(base_workload(args.workload), args.cpu_seconds, workers, args.param)
    if args.workload == "c3":
        out = run_uneven(args)
    elif args.workload == "c5":
        out = run_serving(args)
    elif args.workload == "f3":
        out = run_predict(args)
    else:
        out = run_structured(args)
        batched = {"c2": "c2x64", "c4": "c4x8"}.get(args.workload)
        if batched and args.path == "resident" and args.param == "full" and not args.no_batched:
            # the same list for many gate sets in one batch: the steady state of many
            # evaluations (one launch per kernel and level for all of them)
            import copy
            b_args = copy.copy(args)
            b_args.workload, b_args.steps, b_args.warmup = batched, (20 if batched == "c2x64" else 10), 3
            b = run_structured(b_args)
            key = "batched_" + batched
            out[key] = {k: b[k] for k in ("value", "unit", "ms_per_step", "steps", "roofline", "graph_replay",
                                          "one_by_one")}
            out[key]["workload"] = b["config"]["workload"]
        if args.workload == "c2" and not args.no_serving:
            out["serving"] = serving_summary(args)
    out["cpu_baseline"] = cpu
    print(json.dumps(out))


def base_workload(name: str) -> str:
    """c2x64 is the c2 list evaluated for 64 gate sets at once, c4x8 the c4
    list for 8."""
    return {"c2x64": "c2", "c4x8": "c4"}.get(name, name)


_SERVING_DATA = {}


def serving_summary(args, rate=None):
    """Served fits (continuous batching) and the plain per-request path on the
    same Poisson trace of mixed one/two/three-qubit fit requests."""
    import torch
    from paper_2008_13490_amd import api
    from paper_2008_13490_amd import serving as SV
    from paper_2008_13490_amd import workloads as W

    rate = args.rate if rate is None else rate
    t0 = time.perf_counter()
    trace = W.serving_trace(rate, args.requests)

    def data_fn(kind, S, seed):   # the same requests at every rate: generated once
        key = (kind, S, seed, args.iters)
        if key not in _SERVING_DATA:
            _SERVING_DATA[key] = W.serving_request(kind, S, seed, args.iters)
        return _SERVING_DATA[key]

    jobs = SV.make_jobs(trace, n_iter=args.iters, data_fn=data_fn)
    t_gen = time.perf_counter() - t0
    print(f"[bench] serving trace: {len(jobs)} requests at {rate} /s, generated in {t_gen:.1f} s",
          file=sys.stderr, flush=True)
    # the library on its own stream: requests loaded on the host thread upload
    # through the default stream without waiting for the rounds in flight
    ctx = api.Context(0, stream=torch.cuda.Stream())
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    # (no graph capture here: uploads through the default stream on the loading
    # thread would invalidate a capture taken meanwhile)
    served = SV.Scheduler(SV.GPUEngine(ctx, capture_graph=False), budget, max_active=args.slots,
                          round_work=args.round_work, depth=2, prefetch=True).run(jobs)
    ctx.sync()
    print(f"[bench] served: {served}", file=sys.stderr, flush=True)
    SV.reset(jobs)
    plain = SV.Scheduler(SV.PlainEngine(ctx), budget, max_active=1).run(jobs)
    ctx.sync()
    print(f"[bench] plain: {plain}", file=sys.stderr, flush=True)
    ctx.close()
    kinds = [k for _, k, _, _ in trace]
    return {
        "workload": f"c5: Poisson arrivals at {rate:g} requests/s, {len(jobs)} fit requests "
                    f"({kinds.count('1q')} one-qubit, {kinds.count('2q')} two-qubit, {kinds.count('3q')} "
                    f"three-qubit), S log-uniform in [1000, 100000], random words (L <= 256, three qubits "
                    f"L <= 128), {args.iters} closed-loop iterations each with gradient, HBM budget "
                    f"{budget / 2**30:.0f} GiB, {args.slots} slots, rounds of <= {args.round_work:.0e} two-qubit steps, "
                    f"two rounds in flight, requests loaded on a host thread",
        "rate": rate,
        "served": served,
        "plain_per_request": plain,
    }


def run_serving(args):
    rates = [float(x) for x in args.serving_rates.split(",")] if args.serving_rates else [args.rate]
    sweep = [serving_summary(args, r) for r in rates]
    s = sweep[0] if len(sweep) == 1 else max(sweep, key=lambda x: x["rate"] == args.rate)
    sv = s["served"]
    out = {
        "metric": "p50/p99 latency of served fits; sequence evals/s (FP64, with gradient)",
        "value": sv["seq_evals_per_s"],
        "unit": "sequence evals/s",
        "n_gpus": 1,
        "steps": sv["iterations"],
        "warmup": 0,
        "ms_per_step": sv["wall_s"] * 1e3 / max(sv["rounds"], 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": s["workload"]},
        "serving": s,
    }
    if len(sweep) > 1:
        out["sweep"] = [{"rate": x["rate"],
                         "served": {k: x["served"][k] for k in ("seq_evals_per_s", "request_latency_ms",
                                                                 "iteration_latency_ms", "rounds", "mean_round_size",
                                                                 "host_s")},
                         "plain": {k: x["plain_per_request"][k] for k in ("seq_evals_per_s", "request_latency_ms",
                                                                           "iteration_latency_ms")}}
                        for x in sweep]
    return out


def copy_calibration(mib: int):
    """A plain device-to-device copy of a known size: its FETCH_SIZE and
    WRITE_SIZE counters per dispatch, against mib MiB each, give the factor
    that turns the counters into HBM bytes."""
    import torch
    n = mib * (1 << 20) // 8
    x = torch.arange(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_mib": mib, "dispatches": 3, "equal": bool(torch.equal(x, y))}))


def _profile(api, ctx, families):
    fams = {}
    for fam in families:
        ms, n = api.profile_read(ctx, fam)
        if n:
            fams[fam] = (ms, n)
    return fams


def _roofline(dom, fams, flops, traffic):
    ms_tot, n_launch = fams[dom]
    avg_s = ms_tot / n_launch * 1e-3
    achieved = flops / avg_s / 1e12
    return {
        "bound": "alu",
        "kernel": dom,
        "achieved": achieved,
        "peak": PEAK_FP64,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP64,
        "traffic": traffic,
        "avg_launch_us": avg_s * 1e6,
        "algorithmic_flop_per_launch": flops,
    }


def run_structured(args):
    import torch
    from paper_2008_13490_amd import api
    from paper_2008_13490_amd import workloads as W

    w = W.structured_workload(base_workload(args.workload))
    desc = workload_desc(w)
    m = w.model
    ctx = api.Context(0)
    gs = api.DeviceGateSet.from_numpy(m.n_qubits, m.rho, m.effects, m.gates)
    dev = torch.device("cuda", 0)
    obj = torch.empty(1, dtype=torch.float64, device=dev)
    grad = torch.empty(m.n_params(), dtype=torch.float64, device=dev)
    n_sets = 1
    batch_extra = None
    if args.workload in ("c2x64", "c4x8"):
        # many gate sets (the model and seeded neighbours) over the one list:
        # resident requests whose plans run as one launch per kernel and level;
        # one step evaluates all of them
        if args.path != "resident" or args.param != "full":
            raise SystemExit(f"{args.workload}: resident path, full parameterization")
        n_sets = 64 if args.workload == "c2x64" else 8
        rng = np.random.default_rng(n_sets)
        kind = {2: "2q", 3: "3q"}[m.n_qubits]
        sets = [m] + [W.noisy_gateset(kind, W.LAMBDA, W.SIGMA, rng) for _ in range(n_sets - 1)]
        reqs = [api.Request(ctx, m.n_qubits, m.K, m.M, w.seqs.offsets, w.seqs.gates, w.counts)
                for _ in range(n_sets)]
        thetas = [api.DeviceGateSet.from_numpy(g.n_qubits, g.rho, g.effects, g.gates) for g in sets]
        req = reqs[0]
        batch = api.Batch(ctx, reqs, thetas, want_probs=False, want_grad=True, capture_graph=True)
        base = base_workload(args.workload)
        desc = dict(desc, workload=f"{args.workload}: the {base} list for {n_sets} gate sets (the model and "
                                   f"{n_sets - 1} seeded neighbours, same noise model) as {n_sets} resident requests "
                                   f"in one batch; " + desc["workload"])

        def step():
            batch.run()

        def alone():
            for r, t in zip(reqs, thetas):
                r.eval(t, want_probs=False, want_grad=True)

        batch_extra = (batch, alone)
    elif args.param != "full":
        if args.path != "resident" or m.n_qubits > 2:
            raise SystemExit("--param tp/cptp: resident path, one or two qubits")
        kind = {1: "1q", 2: "2q"}[m.n_qubits]
        par = api.Parameterization(ctx, args.param, m.n_qubits, m.M, m.K,
                                   torch.as_tensor(W.ideal_targets(kind), device=dev))
        theta = torch.as_tensor(W.param_point(args.param, m, 7), device=dev)
        gtheta = torch.empty(par.count, dtype=torch.float64, device=dev)
        req = api.Request(ctx, m.n_qubits, m.K, m.M, w.seqs.offsets, w.seqs.gates, w.counts)

        def step():
            par.forward(theta, out=gs)
            req.eval(gs, want_probs=False, want_grad=True, out=(obj, None, grad))
            par.backward(theta, grad, out=gtheta)
    elif args.path == "resident":
        req = api.Request(ctx, m.n_qubits, m.K, m.M, w.seqs.offsets, w.seqs.gates, w.counts)

        def step():
            req.eval(gs, want_probs=False, want_grad=True, out=(obj, None, grad))
    else:
        seqs = api.DeviceSeqs.from_numpy(w.seqs.offsets, w.seqs.gates)
        counts = torch.as_tensor(w.counts, device=dev)
        import ctypes

        def step():
            api._lib.check(ctx.lib.gst_loglik(ctx.handle, ctypes.byref(gs.as_struct()),
                                              ctypes.byref(seqs.as_struct()), api._ptr(counts), None,
                                              api._ptr(obj), api._ptr(grad)))

    families = ("leaf", "reduce", "trunk_fwd", "trunk_bwd", "inject", "grad_gemm", "fill", "tiles_2q", "tiles_1q",
                "tiles_reduce", "chain_3q", "gemm_3q", "reduce_3q", "tiles_3q_fwd", "tiles_3q_bwd", "readout_3q",
                "param_fwd", "param_bwd")
    for _ in range(args.warmup):
        step()
    ctx.sync()
    # breakdown pass: events around every kernel, to find the dominant family
    n_break = max(1, min(args.steps, 20))
    api.profile_enable(ctx, True)
    for _ in range(n_break):
        step()
    ctx.sync()
    brk = _profile(api, ctx, families)
    # the roofline is priced on the FP64 work of the longest family that has
    # arithmetic (the ordered sums and the injection gather carry none)
    D, M, S = m.D, m.M, w.seqs.S
    L = w.seqs.lengths()
    info = req_plan_info(req) if args.path == "resident" else None

    def fam_flops(f):
        return (param_flops(f, D, m.K) if f.startswith("param_")
                else algorithmic_flops(f, D, M, S, int(L.sum()), info))

    work = [f for f in brk if fam_flops(f) > 0] or list(brk)
    dom = max(work, key=lambda f: brk[f][0])
    # timed region: no events (a launch with timing events costs host and
    # queue time between the kernels: about 5 us per c2 evaluation)
    api.profile_enable(ctx, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # kernel pass: the same steps again, events around the dominant family
    # only (kernel-stamped, so the kernel's own duration is what they time)
    api.profile_enable(ctx, True)
    api.profile_only(ctx, dom)
    for _ in range(args.steps):
        step()
    ctx.sync()
    tot = _profile(api, ctx, (dom,))
    api.profile_only(ctx, None)
    api.profile_enable(ctx, False)
    fams = {dom: (tot[dom][0] - brk[dom][0], tot[dom][1] - brk[dom][1])}
    elapsed = t1 - t0
    value = n_sets * S * args.steps / elapsed
    extra = {}
    if batch_extra is None and args.path == "resident" and args.param == "full":
        # the same evaluation through the torch.autograd.Function wrapper:
        # forward (objective; the library computes the gradient in the same
        # launch sequence) and backward (hands the gradient to the leaves)
        from paper_2008_13490_amd import autograd as AG
        leaves = [torch.as_tensor(x, device=dev).clone().requires_grad_(True) for x in (m.rho, m.effects, m.gates)]

        def ag_step():
            for t in leaves:
                t.grad = None
            AG.gst_nll(leaves[0], leaves[1], leaves[2], req).backward()

        for _ in range(3):
            ag_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ag_step()
        torch.cuda.synchronize()
        ag_s = (time.perf_counter() - t0) / args.steps
        extra["autograd"] = {"ms_per_step": ag_s * 1e3, "value": S / ag_s,
                             "what": "forward + backward through torch.autograd.Function (gst_nll)"}
    if batch_extra is not None:
        # the same steps replayed from the captured graph (no per-kernel
        # events), and the 64 requests evaluated one after another
        batch, alone = batch_extra
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            batch.run()
        torch.cuda.synchronize()
        g_s = (time.perf_counter() - t0) / args.steps
        for _ in range(2):
            alone()
        ctx.sync()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            alone()
        ctx.sync()
        a_s = (time.perf_counter() - t0) / args.steps
        extra = {"graph_replay": {"ms_per_step": g_s * 1e3, "value": n_sets * S / g_s},
                 "one_by_one": {"ms_per_step": a_s * 1e3, "value": n_sets * S / a_s,
                                "what": f"the same {n_sets} requests evaluated one after another (own launch sequences)"}}
    flops = n_sets * fam_flops(dom)  # algorithmic FP64 work per launch of the dominant family
    if info and info.get("grouped"):
        steps_eval = info["trie_nodes"] - 1
    else:
        steps_eval = (info["trunk_steps"] + info["item_steps"]) if info else int(L.sum())
    return {
        "metric": METRIC,
        "value": value,
        "unit": "sequence evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": dict(desc, path=args.path, param=args.param),
        "roofline": with_counters(_roofline(dom, fams, flops, None),
                                  read_counters(args.workload, dom) if args.path == "resident" and args.param == "full"
                                  else None),
        "index_stream": index_stream(w, info, elapsed / args.steps / n_sets),
        "kernels_ms_per_step": {f: brk[f][0] / n_break for f in brk},
        "plan": info,
        "useful_tflops": n_sets * 6.0 * D * D * steps_eval / (elapsed / args.steps) / 1e12,
        **extra,
    }


def run_uneven(args):
    """The uneven batch: 512 gate sets (70% one-qubit, 30% two-qubit), each
    with 500..20000 random words of length 1..1024, evaluated with gradient
    in one graph-captured persistent launch per step."""
    import torch
    from paper_2008_13490_amd import api
    from paper_2008_13490_amd import workloads as W

    plan = W.c3_plan()
    if args.sets:
        plan = plan[:args.sets]
    ctx = api.Context(0)
    tuned = None
    if not args.no_autotune:
        from paper_2008_13490_amd import autotune
        t0 = time.perf_counter()
        tuned = autotune.tune(ctx, {1: (32, 16384, 1, 1024), 2: (16, 4096, 1, 1024)})
        print(f"[bench] autotune ({time.perf_counter() - t0:.1f} s): {tuned}", file=sys.stderr, flush=True)
    reqs, thetas = [], []
    S_tot = sum_len = 0
    flops = {16: 0.0, 4: 0.0}
    t0 = time.perf_counter()
    for kind, S, seed in plan:
        w = W.uneven_request(kind, S, seed)
        m = w.model
        reqs.append(api.Request(ctx, m.n_qubits, m.K, m.M, w.seqs.offsets, w.seqs.gates, w.counts))
        thetas.append(api.DeviceGateSet.from_numpy(m.n_qubits, m.rho, m.effects, m.gates))
        n = int(w.seqs.offsets[-1])
        S_tot += S
        sum_len += n
        flops[m.D] += 6.0 * m.D * m.D * n + 6.0 * m.D * m.M * S
        del w
        if len(reqs) % 64 == 0:
            print(f"[bench] {len(reqs)} requests resident", file=sys.stderr, flush=True)
    t_setup = time.perf_counter() - t0
    print(f"[bench] uneven batch: {len(plan)} gate sets, {S_tot} sequences, {sum_len} steps, "
          f"set-up {t_setup:.1f} s", file=sys.stderr, flush=True)
    batch = api.Batch(ctx, reqs, thetas, want_probs=False, want_grad=True, capture_graph=True)
    for _ in range(args.warmup):
        batch.run()
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.sync()
    elapsed = t1 - t0
    print(f"[bench] graph replays: {elapsed / args.steps * 1e3:.2f} ms per step", file=sys.stderr, flush=True)
    # the same launch sequence eagerly, each kernel bracketed by events
    n_prof = max(1, min(args.steps, 5))
    api.profile_enable(ctx, True)
    for _ in range(n_prof):
        batch.run()
    ctx.sync()
    fams = _profile(api, ctx, ("tiles_2q", "tiles_1q", "tiles_reduce", "batch"))
    api.profile_enable(ctx, False)
    # the plain per-request path: each request on its own, one after another
    t2 = time.perf_counter()
    outs = [r.eval(t, want_probs=False, want_grad=True) for r, t in zip(reqs, thetas)]
    torch.cuda.synchronize()
    ctx.sync()
    plain_s = time.perf_counter() - t2
    ok = all(torch.equal(o[0], batch.obj[x]) and torch.equal(o[2], batch.grad[x]) for x, o in enumerate(outs))
    dom = max((f for f in fams if f != "batch"), key=lambda f: fams[f][0])
    dom_flops = flops[16] if dom == "tiles_2q" else flops[4] if dom == "tiles_1q" else 0.0
    n1 = sum(1 for k, _, _ in plan if k == "1q")
    return {
        "metric": "sequence evals/s incl. gradient (uneven batch of 1q/2q gate sets, FP64)",
        "value": S_tot * args.steps / elapsed,
        "unit": "sequence evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"c3: uneven batch of {len(plan)} gate sets ({n1} one-qubit, {len(plan) - n1} "
                               "two-qubit), S ~ U{500..20000}, random words of length U{1..1024}, one "
                               "graph-captured persistent launch per step; counts ~ Multinomial(1000, uniform)",
                   "sequences": S_tot, "sum_len": sum_len, "gate_sets": len(plan)},
        "roofline": with_counters(_roofline(dom, fams, dom_flops, None), read_counters("c3", dom)),
        "index_stream": {"what": "gate indices, offsets, order", "bytes_per_eval": sum_len + 16 * S_tot,
                         "gbs": (sum_len + 16 * S_tot) / (elapsed / args.steps) / 1e9},
        "kernels_ms_per_step": {f: fams[f][0] / n_prof for f in fams},
        "useful_tflops": (flops[16] + flops[4]) / (elapsed / args.steps) / 1e12,
        "plain_per_request": {"ms_per_step": plain_s * 1e3, "value": S_tot / plain_s,
                              "same_bits_as_batch": bool(ok)},
        "setup_s": t_setup,
        "autotune": {str(n): {"best": f"{v['best'][0]} seqs/tile x {v['best'][1] or 'max'} blocks/CU",
                              "ms": v["ms"]} for n, v in tuned.items()} if tuned else None,
    }


def run_predict(args):
    """Predictions of repeated gate applications (thesis Sec. 6.3, Eq.
    GSTPrediction) and their statistical distance to the ideal predictions
    (Eq. statisticaldistance).  One step = one gst_predict of the estimate for
    the four initial states x 6 gates x r = 0..1000 plus the distance to the
    ideal gate set's predictions (resident)."""
    import torch
    from paper_2008_13490_amd import api
    from paper_2008_13490_amd import workloads as W

    pw = W.prediction_workload(1000)
    ctx = api.Context(0)
    est, ide = (api.DeviceGateSet.from_numpy(g.n_qubits, g.rho, g.effects, g.gates) for g in (pw.estimate, pw.ideal))
    pred = api.Predictor(ctx, pw.preps, pw.gates, pw.r_max)
    p_ideal = pred(ide)
    p = torch.empty_like(p_ideal)
    d = torch.empty(p.shape[:-1], dtype=torch.float64, device=p.device)

    def step():
        pred(est, out=p)
        api.tv_distance(ctx, p, p_ideal, out=d)

    families = ("predict_chain", "predict_fill", "tv_distance")
    for _ in range(args.warmup):
        step()
    ctx.sync()
    n_break = max(1, min(args.steps, 20))
    api.profile_enable(ctx, True)
    for _ in range(n_break):
        step()
    ctx.sync()
    brk = _profile(api, ctx, families)
    dom = max(brk, key=lambda f: brk[f][0])
    # timed region without events, then the kernel pass with events on the
    # dominant family (as in the evaluation benchmark)
    api.profile_enable(ctx, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    api.profile_enable(ctx, True)
    api.profile_only(ctx, dom)
    for _ in range(args.steps):
        step()
    ctx.sync()
    tot = _profile(api, ctx, (dom,))
    api.profile_only(ctx, None)
    api.profile_enable(ctx, False)
    fams = {dom: (tot[dom][0] - brk[dom][0], tot[dom][1] - brk[dom][1])}
    elapsed = t1 - t0
    n_pairs = len(pw.preps) * len(pw.gates)
    per_step = n_pairs * (pw.r_max + 1)
    D, M = pw.estimate.D, pw.estimate.M
    flops = predict_flops(dom, D, M, [len(w) for w in pw.preps], len(pw.gates), pw.r_max)
    return {
        "metric": "predicted outcome distributions/s with statistical distance (2q, FP64)",
        "value": per_step * args.steps / elapsed,
        "unit": "predicted distributions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"f3: two-qubit predictions <<E|(G_s)^r G_prep|rho>> for the 4 initial states "
                               f"x 6 gates x r = 0..{pw.r_max} of the C2 evaluation point, statistical distance "
                               f"to the ideal gate set's predictions",
                   "distributions_per_step": per_step},
        "roofline": _roofline(dom, fams, flops, None),
        "kernels_ms_per_step": {f: brk[f][0] / n_break for f in brk},
    }


def run_fit_bench(args):
    """The two-qubit GST fit (thesis Sec. 6.3.1-6.3.2) in the CPTP mode: LGST,
    gauge optimization, iterative MLGST over the six stages (maximum lengths
    1..32, at most --fit-iters L-BFGS iterations each) with the evaluations on
    the GPU, final gauge optimization.  One step = one whole fit; the stage
    requests (lists, counts and plans in HBM) are created before the timed
    region."""
    import torch
    from paper_2008_13490_amd import api
    from paper_2008_13490_amd import fit as FIT
    from paper_2008_13490_amd import workloads as W

    mode = "cptp" if args.param == "full" else args.param
    fw = W.fit_workload()
    ends = FIT.stage_ends(fw.stage_end)
    ctx = api.Context(0)
    reqs = []
    for e in ends:
        sub = fw.seqs.subset(np.arange(e))
        reqs.append(api.Request(ctx, 2, 6, 4, sub.offsets, sub.gates, fw.counts[:e]))

    def one_fit():
        return FIT.run_fit(ctx, fw.seqs, fw.counts, fw.stage_end, fw.prep_fids, fw.meas_fids, fw.target, mode=mode,
                           max_iter=args.fit_iters, gtol=1e-8, requests=reqs)

    # a step is a whole fit: the defaults of the evaluation benches (200 / 20) become 2 / 1
    steps = 2 if args.steps == 200 else args.steps
    warm = 1 if args.warmup == 20 else args.warmup
    for _ in range(warm):
        one_fit()
    families = ("leaf", "reduce", "trunk_fwd", "trunk_bwd", "inject", "grad_gemm", "fill", "tiles_2q", "param_fwd",
                "param_bwd")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [one_fit() for _ in range(steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # kernel breakdown from one more fit with per-launch events (not timed above)
    api.profile_enable(ctx, True)
    one_fit()
    ctx.sync()
    fams = _profile(api, ctx, families)
    api.profile_enable(ctx, False)
    res = results[-1]
    evals = [r["evaluations"] for r in res.reports]
    n_eval = sum(evals)
    dom = max(fams, key=lambda f: fams[f][0])
    # algorithmic flops per launch of the dominant family, weighted by the
    # evaluations of each stage
    infos = [req_plan_info(r) for r in reqs]
    tot = 0.0
    for e_s, info, end in zip(evals, infos, ends):
        L = np.diff(fw.seqs.offsets[:end + 1])
        fl = param_flops(dom, 16, 6) if dom.startswith("param_") else algorithmic_flops(dom, 16, 4, end, int(L.sum()),
                                                                                         info)
        tot += e_s * fl
    flops = tot / max(1, n_eval)
    out = {
        "metric": "seconds per two-qubit GST fit (LGST, gauge optimization, 6-stage CPTP MLGST, FP64)",
        "value": elapsed / steps,
        "unit": "s/fit",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"f2: two-qubit fit list ({fw.seqs.S} sequences, 16 prep x 11 meas product "
                               f"fiducials, 12 germs, maximum lengths 1..32, at most 38 gates), counts ~ "
                               f"Multinomial(1000) from the C2 truth; {mode.upper()} mode, <= {args.fit_iters} "
                               f"L-BFGS iterations per stage", "stages": ends,
                   "evaluations_per_fit": n_eval, "iterations": [r["iterations"] for r in res.reports],
                   "objectives": [r["objective"] for r in res.reports]},
        "roofline": _roofline(dom, {dom: fams[dom]}, flops, None),
        "kernels_ms_per_fit": {f: fams[f][0] for f in fams},
        "host_seconds": res.seconds,
        "gpu_evaluations_per_s": n_eval / (res.seconds["mlgst"]),
    }
    out["estimate_metrics"] = fit_metrics(api, fw, res)
    if not args.no_cpu:
        out["cpu_baseline"] = fit_cpu_baseline(fw, ends, evals, mode, args.cpu_seconds)
    return out


def fit_metrics(api, fw, res):
    """Post-fit metrics of the gauge-optimized estimate (thesis Sec. 6.3.3, App. J):
    per gate the average gate fidelity against the ideal gate, the Hamiltonian
    decomposition (rotation angle, decomposition error: the projection of the real
    principal logarithm where it exists, else the error minimized from the target's
    Hamiltonian), and the diamond distance between the ideal unitary and the
    decomposition's exp(-iH)."""
    import scipy.linalg as sla   # builds exp(-iH) of the reported h for the distance only
    from paper_2008_13490_amd import _lib
    t0 = time.perf_counter()
    f = api.avg_gate_fidelity(2, res.gates, fw.target.gates)
    P = [np.kron(a, b) for a in _PAULI1 for b in _PAULI1]
    per = {}
    for k, name in enumerate(fw.target.names):
        row = {"avg_gate_fidelity": float(f[k])}
        try:
            h, ang, gam = api.hamiltonian_decomposition(2, res.gates[k])
            row["decomposition"] = "projection of the real principal logarithm"
        except _lib.GSTError:
            # no real principal logarithm (CZ): h minimizing the decomposition
            # error from the target's Hamiltonian
            h, ang, gam = api.hamiltonian_decomposition_target(2, res.gates[k], fw.target.unitaries[k])
            row["decomposition"] = "minimized decomposition error from the target's Hamiltonian"
        U_eff = sla.expm(-1j * sum(h[i] * P[i] for i in range(16)) / 2)
        row.update(angle=ang, angle_over_pi=ang / np.pi, decomposition_error=gam,
                   diamond_to_ideal=api.diamond_unitary(fw.target.unitaries[k], U_eff))
        per[name] = row
    return {"gates": per, "seconds": time.perf_counter() - t0}



def fit_cpu_baseline(fw, ends, evals, mode, seconds):
    """The oracle on a bounded sample of the fit: its evaluation (parameter map,
    likelihood with gradient, chain rule) timed on each stage's list, times the
    evaluations the GPU fit made in that stage, plus its own LGST and gauge
    optimization; single-threaded."""
    import oracle
    from oracle import fit as FT
    from paper_2008_13490_amd import fit as FIT
    oracle.build(force=not os.path.exists(oracle.library_path()))
    print(f"[bench] cpu baseline of the fit (~{seconds:.0f} s)", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    e0 = fw.stage_end[0]
    r, E, G = FT.lgst(fw.seqs.offsets[:e0 + 1], fw.seqs.gates[:fw.seqs.offsets[e0]], fw.counts[:e0], fw.prep_fids,
                      fw.meas_fids, 2, 6)
    FT.gauge_opt(r, E, G, fw.target.rho, fw.target.effects, fw.target.gates)
    t_lin = time.perf_counter() - t0
    th = FIT.cptp_start(fw.target.effects, 6, 16) if mode == "cptp" else FT.contract_tp(r, E, G)
    per_stage = []
    budget = seconds / len(ends)
    for e in ends:
        sub = fw.seqs.subset(np.arange(e))
        n, t1 = 0, time.perf_counter()
        while True:
            FT.nll_in_mode(th, mode, 2, 4, 6, fw.target.gates, sub.offsets, sub.gates, fw.counts[:e])
            n += 1
            if time.perf_counter() - t1 >= budget:
                break
        per_stage.append((time.perf_counter() - t1) / n)
    est = t_lin + sum(t * k for t, k in zip(per_stage, evals))
    return {
        "value": est,
        "unit": "s/fit",
        "cores": 1,
        "kind": "oracle",
        "sample": f"oracle LGST + gauge optimization run once ({t_lin:.2f} s); one {mode.upper()} evaluation "
                  f"timed on each stage's list ({', '.join(f'{t:.3f}' for t in per_stage)} s) and multiplied by "
                  f"the GPU fit's evaluations per stage ({evals}); one thread",
    }


_PAULI1 = (np.eye(2, dtype=complex), np.array([[0, 1], [1, 0]], dtype=complex),
           np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]], dtype=complex))


def predict_flops(family, D, M, prep_lens, n_gates, r_max, B=32):
    """FP64 flops one launch of a prediction kernel does: the chain applies each
    preparation word and (Q - 1) block jumps per pair and builds (G_s)^B with
    log2(B) squarings (2D^3 each); the fill steps through every block with
    single mat-vecs (2D^2) and reads out every state (2DM)."""
    Q = (r_max + 1 + B - 1) // B
    pairs = len(prep_lens) * n_gates
    if family == "predict_chain":
        return 2.0 * D * D * (n_gates * sum(prep_lens) + pairs * (Q - 1)) + \
            pairs * 5 * 2.0 * D ** 3
    if family == "predict_fill":
        return pairs * (2.0 * D * D * (r_max + 1 - Q) + 2.0 * D * M * (r_max + 1))
    if family == "tv_distance":
        return pairs * (r_max + 1) * 3.0 * M
    return 0.0


def param_flops(family, D, K, taylor=16):
    """FP64 flops of one launch of a CPTP parameterization kernel (without the
    squarings, whose number depends on the generator's norm): per gate the
    generator from the structure tables (2 (D-1) complex terms per entry), the
    Taylor polynomial by Horner (one D x D product per degree) and the product
    with the target; backward: the block polynomial (three products per degree)
    and the contractions back to the parameters."""
    mm = 2.0 * D ** 3
    gen = 8.0 * D * D * (D - 1)
    if family == "param_fwd":
        return K * (gen + (taylor + 1) * mm)
    if family == "param_bwd":
        return K * (2 * gen + 3 * taylor * mm + mm)
    return 0.0


def index_stream(w, info, eval_s):
    """Bytes of sequence-list data one evaluation reads and their rate.  The
    per-sequence kernels stream the gate indices (1 B a step) with the offsets
    and the length order (8 B a sequence each); the sharing plans read compact
    plan tables instead: for the grouped three-qubit plan one gate index per
    tile step, for the trie plan one op word per trunk op plus its item table."""
    L = w.seqs.lengths()
    S = int(w.seqs.S)
    if info and info.get("grouped"):
        kind, nbytes = "grouped-plan words", int(info["rows"]) // 16
    elif info:
        kind, nbytes = "trie-plan ops and items", int(info["chain_steps"]) * 8 + S * 32 + int(info["item_steps"])
    else:
        kind, nbytes = "gate indices, offsets, order", int(L.sum()) + 16 * S
    return {"what": kind, "bytes_per_eval": nbytes, "gbs": nbytes / eval_s / 1e9}


def req_plan_info(req):
    info = req.plan_info()
    return info if info["plan_used"] else None


def algorithmic_flops(family, D, M, S, sum_len, info):
    """FP64 flops the method must do in one launch of `family`.

    Per step of a chain: forward mat-vec 2D^2, adjoint mat-vec 2D^2, gradient
    outer product 2D^2; per sequence: readout, seed and effect gradient 2DM
    each.  Without the sharing plan every sequence is its own chain; with it,
    the chains are the trunk chains (a germ-power jump is one mat-vec), the
    states and adjoints filled in inside the jumps, and the remaining item
    steps (launch counts: one per trunk level)."""
    if info is None:
        if family in ("leaf", "tiles_2q", "tiles_1q"):
            return 6.0 * D * D * sum_len + 6.0 * D * M * S
        if family == "chain_3q":   # forward and adjoint products, readout, seed, dE
            return 4.0 * D * D * sum_len + 6.0 * D * M * S
        if family == "gemm_3q":    # dG_k = sum b f^T
            return 2.0 * D * D * sum_len
        return 0.0
    if info.get("grouped"):
        # three qubits, grouped chains: every trie node is one step of its
        # chain (padding columns of a tile are not counted); launches per
        # evaluation: one per level in each direction
        nodes, lv = info["trie_nodes"] - 1, max(1, info["levels"])
        if family in ("tiles_3q_fwd", "tiles_3q_bwd"):
            return 2.0 * D * D * nodes / lv
        if family == "readout_3q":   # readout, seed and effect gradient of every sequence
            return 6.0 * D * M * S
        if family == "gemm_3q":
            return 2.0 * D * D * nodes
        return 0.0
    ts, its, lv = info["trunk_steps"], info["item_steps"], max(1, info["levels"])
    filled = ts - info.get("chain_steps", ts)   # trunk states / adjoints inside germ-power jumps
    if family == "leaf":   # items: forward + adjoint mat-vecs, readout, seed, dE; the forward fill tasks
        return 4.0 * D * D * its + 6.0 * D * M * S + 2.0 * D * D * filled
    if family == "fill":   # reverse fill tasks
        return 2.0 * D * D * filled
    if family in ("trunk_fwd", "trunk_bwd"):   # the chain's mat-vecs (a germ-power jump counts once)
        return 2.0 * D * D * info.get("chain_steps", ts) / lv
    if family == "grad_gemm":
        return 2.0 * D * D * (ts + its)
    return 0.0


if __name__ == "__main__":
    main()
