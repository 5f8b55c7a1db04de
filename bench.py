#!/usr/bin/env python3
"""Benchmark of the refinement loop on one MI355X.

A step is one complete refinement (every round of the hot path) of the
workload, with the input CDT already resident in HBM when timing starts.
Prints one JSON line:

  value        Steiner points inserted per second (whole call, wall clock)
  tets_per_s   output tetrahedra per second
  roofline     the dominant kernel family's algorithmic bytes / its event-timed
               device time against the 8 TB/s HBM peak
  cpu_baseline the oracle timed on a bounded sample of the same workload

Default workload: the 1M-point PLC (cube corners + 900 000 points from 8
isotropic Gaussians + 100 000 uniform points, three nested sphere surfaces
r = 0.15 / 0.30 / 0.45, B = 1.4).  --workload cfg2 runs the 50K-point one
(one sphere surface, B = 1.5), cfg1 the 1K-point cube (B = 2.0).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


KERNEL_SOURCES = ("qm_geom.h", "qm_kernels.h", "qm_grow.h", "qm_round.h", "qm_insert.h", "qm_setup.h", "qm_lib.hip")


def kernel_source_sha256():
    """Digest of the sources of the single-instance kernels and their
    launches (the batched and served forms' host code excluded): measured
    traffic is only valid for the kernels it was measured on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1903_03406_amd", "csrc")
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


def measured_traffic(workload, family, launches):
    """HBM bytes per launch of the kernel of `family` from a committed counter
    summary (profiles/*_traffic.md: FETCH_SIZE and WRITE_SIZE, each scaled by
    the copy-kernel calibration), or None when no summary is for these kernel
    sources, this workload and this kernel."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md"))):
        kv = {}
        for line in open(path):
            if "=" in line and line.strip().startswith("qm."):
                k, v = line.strip().split("=", 1)
                kv[k.strip()] = v.strip()
        if (kv.get("qm.source_sha256") == kernel_source_sha256() and kv.get("qm.workload") == workload
                and kv.get("qm.family") == family and int(kv.get("qm.launches", -1)) == launches):
            fetch = float(kv["qm.fetch_kib_total"]) * float(kv["qm.fetch_scale"])
            write = float(kv["qm.write_kib_total"]) * float(kv["qm.write_scale"])
            return (fetch + write) * 1024.0 / launches
    return None


TIER_OF = {"grow_validate": 0, "grow_hybrid": 1}
KERNEL_OF = {"grow_validate": "k_grow_lds (small LDS tiles, 64 lanes)",
             "grow_hybrid": "k_grow_hybrid (LDS hash tables, lists in HBM, 256 lanes)"}


def tier_bytes(t):
    """Algorithmic bytes of one grow tier's evaluations (its counters from
    QM_PROFILE): each tested tet costs its vertex ids (16 B) and one new
    vertex (32 B: it is reached across a face whose three vertices are
    already loaded); each region tet also its neighbour, facet and
    subsegment words (56 B) and its region entry (8 B); each boundary face
    of an accepted candidate its record (52 B); each extra claim 8 B."""
    return (48 * t["tested"] + 64 * t["region"] + 52 * t["acc_bfaces"]
            + 8 * max(t["acc_claims"] - t["acc_region"], 0))


def insertion_model_bytes(r, prof):
    """The whole refinement's algorithmic bytes by the per-insertion model:
    a kept point moves 36(k+s) + 24u + 36f + 4s + 24 + 16(k+s)P bytes, every
    other candidate 36(k+s) + 16(k+s) + 44, with k region tets, f new tets
    (boundary faces), s shell tets (claims beyond the region), u cavity
    vertices (f/2 + 2 for a ball) and P selection passes per round, all
    means over the accepted candidates of the run."""
    tiers = prof["tiers"]
    acc = sum(t["accepted"] for t in tiers)
    if acc == 0:
        return 0.0, {}
    k = sum(t["acc_region"] for t in tiers) / acc
    f = sum(t["acc_bfaces"] for t in tiers) / acc
    sh = sum(t["acc_claims"] - t["acc_region"] for t in tiers) / acc
    u = f / 2 + 2
    rounds_sel = max(int((r.rstats[:, 2] > 0).sum()), 1)
    P = r.mis_passes / rounds_sel
    kept = sum(r.inserted)
    other = r.candidates - kept
    per_kept = 36 * (k + sh) + 24 * u + 36 * f + 4 * sh + 24 + 16 * (k + sh) * P
    per_other = 36 * (k + sh) + 16 * (k + sh) + 44
    return kept * per_kept + other * per_other, {"k": k, "f": f, "s": sh, "u": u, "P": P,
                                                 "bytes_per_kept": per_kept, "bytes_per_other": per_other}


def make_workload(name):
    import qm_inputs as qi
    if name == "cfg3":
        return qi.config(3)
    if name == "cfg2":
        return qi.config(2)
    if name == "cfg1":
        return qi.config(1)
    if name.split(":")[0] == "rect":
        # rect[:n[:gamma[:dist[:B]]]]: a rectangle PLC like the paper's experiments
        # (Table 1: n points, gamma * n rectangles), each rectangle split in advance
        f = name.split(":")[1:]
        n = int(f[0]) if f else 200000
        gamma = float(f[1]) if len(f) > 1 else 0.1
        dist = f[2] if len(f) > 2 else "uniform"
        B = float(f[3]) if len(f) > 3 else 1.4
        return qi.rectangles_plc(n, gamma, seed=12, dist=dist, B=B)
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(w, target_s):
    """Oracle (as it stands) on the first R rounds of the workload, R doubled
    until the oracle's own round loop runs for at least target_s seconds."""
    import oracle
    r, res = 1, None
    while True:
        res = oracle.refine(w, max_rounds=r)
        print(f"[bench] cpu baseline: {res.rounds} rounds in {res.seconds:.1f}s", file=sys.stderr, flush=True)
        if res.seconds >= target_s or res.status == 0 or r >= 4096:
            break
        r *= 2
    steiner = len(res.xyz) - len(w.xyz)
    return {"value": steiner / res.seconds if res.seconds > 0 else 0.0, "unit": "Steiner pts/s",
            "cores": 1, "kind": "oracle",
            "sample": f"first {res.rounds} rounds of the same workload ({steiner} Steiner points, "
                      f"{res.seconds:.1f} s of oracle round loop, setup excluded)"}


def bench_batch(args, qm):
    """Batched workload (config 4 instances 0..N-1, uniform points + a rotated
    ellipsoid surface, B = 2.0): the whole set refined in lockstep by
    qm_refine_lockstep (one launch per phase per round over all instances of
    a group) with knobs qm_lockstep_autotune chose on a probe of the set
    (tuning not timed), against the same set on --streams concurrent
    streams (qm_refine_batch) and one instance at a time.  Host arrays in, host results out in every
    form; the three must give the same rounds and vertex counts."""
    import numpy as np
    import qm_inputs as qi
    t0 = time.time()
    ws = []
    for i in range(args.batch):
        ws.append(qi.config(4, i))
        if (i + 1) % 16 == 0:
            print(f"[bench] {i + 1} instances built", file=sys.stderr, flush=True)
    npts = [len(w.xyz) - 8 for w in ws]
    print(f"[bench] {len(ws)} instances, {sum(npts)} points (min {min(npts)}, max {max(npts)}), "
          f"built in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    qm.refine_batch(ws[:min(4, len(ws))], nstreams=args.streams)          # warm-up
    qm.refine_lockstep(ws[:min(4, len(ws))])
    a = time.perf_counter()
    tune, probe_s = qm.lockstep_autotune(ws, probe=args.tune_probe)
    tune_s = time.perf_counter() - a
    print(f"[bench] autotuned on {args.tune_probe} instances in {tune_s:.1f}s: {tune}", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    res_l = qm.refine_lockstep(ws, tune=tune)
    t2 = time.perf_counter()
    print(f"[bench] lockstep (tuned): {t2 - t1:.2f}s", file=sys.stderr, flush=True)
    res_b = qm.refine_batch(ws, nstreams=args.streams)
    t3 = time.perf_counter()
    print(f"[bench] {args.streams} streams: {t3 - t2:.2f}s", file=sys.stderr, flush=True)
    lat, res_1 = [], []
    for w in ws:
        a = time.perf_counter()
        res_1.append(qm.refine_workload(w))
        lat.append(time.perf_counter() - a)
    t4 = time.perf_counter()
    print(f"[bench] one at a time: {t4 - t3:.2f}s", file=sys.stderr, flush=True)
    for a, b, c in zip(res_l, res_b, res_1):
        assert a.rounds == b.rounds == c.rounds and len(a.xyz) == len(b.xyz) == len(c.xyz), "forms disagree"
    steiner = sum(r.steiner for r in res_l)
    ls, st, seq = t2 - t1, t3 - t2, t4 - t3
    out = {
        "metric": "batched jobs/sec (config 4 instances)", "value": len(ws) / ls, "unit": "jobs/s",
        "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"cfg4_instances_0_{len(ws) - 1}", "instances": len(ws), "points": int(sum(npts)),
                   "form": "lockstep"},
        "tune": tune, "tuning": {"probe_instances": args.tune_probe, "seconds": tune_s,
                                 "probe_seconds_best": probe_s},
        "streams_jobs_per_s": len(ws) / st, "streams": args.streams,
        "one_at_a_time_jobs_per_s": len(ws) / seq,
        "speedup_vs_one_at_a_time": seq / ls, "speedup_vs_streams": st / ls,
        "steiner_per_s_lockstep": steiner / ls, "max_rounds": max(r.rounds for r in res_l),
        "latency_one_at_a_time_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
    }
    print(json.dumps(out), flush=True)


def bench_serve(args, qm):
    """Served workload: Poisson arrivals of jobs from the served generator
    (clustered or ellipsoid instances, log-uniform sizes, B in {1.4, 2.0}),
    admitted by qm_server_* against a device-memory budget.  The job inputs
    are generated before the timed region and reused round-robin; each rate
    runs --serve-jobs arrivals.  Latency of a job: arrival to completion
    (time waiting for admission included)."""
    import numpy as np
    import qm_inputs as qi
    t0 = time.time()
    pool = [qi.serve_job(i, max_points=args.serve_max_points) for i in range(args.serve_pool)]
    npts = [len(w.xyz) - 8 for w in pool]
    print(f"[bench] serve pool: {len(pool)} jobs, {min(npts)}..{max(npts)} points, "
          f"built in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    budget = int(args.serve_budget_gib * (1 << 30))
    rates = [float(r) for r in args.serve_rates.split(",")]
    rng = np.random.Generator(np.random.PCG64(55))
    per_rate = []
    with qm.Server(budget, nworkers=args.streams) as srv:
        for t in [srv.submit(w) for w in pool[:min(4, len(pool))]]:      # warm-up
            srv.result(t)
        for rate in rates:
            arrive = np.cumsum(rng.exponential(1.0 / rate, size=args.serve_jobs))
            jobs = [pool[k % len(pool)] for k in range(args.serve_jobs)]
            lat, fails, steiner = [], 0, 0
            pending = {}                       # ticket -> (job index, submit delay)
            nxt = 0
            start = time.perf_counter()
            while nxt < len(jobs) or pending:
                now = time.perf_counter() - start
                while nxt < len(jobs) and arrive[nxt] <= now:
                    tk = srv.submit(jobs[nxt])
                    if tk is None:             # no room: retry after completions
                        break
                    pending[tk] = (nxt, time.perf_counter() - start - arrive[nxt])
                    nxt += 1
                for tk in list(pending):
                    got = srv.poll(tk, wait_ms=0)
                    if got is None:
                        continue
                    res, code, _, _, total = got
                    k, delay = pending.pop(tk)
                    lat.append(delay + total)
                    if res is None or code not in (0, -4):
                        fails += 1
                    else:
                        steiner += res.steiner
                time.sleep(0.0005)
            span = time.perf_counter() - start
            per_rate.append({"rate_jobs_per_s": rate, "jobs": len(jobs), "failed": fails,
                             "jobs_per_s": len(jobs) / span, "steiner_per_s": steiner / span,
                             "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99))})
            print(f"[bench] rate {rate:g}/s: {per_rate[-1]}", file=sys.stderr, flush=True)
        info = srv.info()
    best = max(per_rate, key=lambda r: r["jobs_per_s"])
    out = {
        "metric": "served jobs/sec (Poisson arrivals)", "value": best["jobs_per_s"], "unit": "jobs/s",
        "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"served_pool{len(pool)}_max{args.serve_max_points}", "workers": args.streams,
                   "budget_gib": args.serve_budget_gib, "points": [int(min(npts)), int(max(npts))]},
        "rates": per_rate, "server": info,
    }
    print(json.dumps(out), flush=True)


def bench_serve_stepped(args, qm):
    """Served workload on the stepped server (continuous batching): the
    resident jobs are one lockstep batch; the loop submits the jobs that have
    arrived, runs one step (one round of every resident job, each phase one
    launch over all of them) and collects finished jobs.  Inputs prepared
    before timing, as in --serve.  Latency: arrival to completion."""
    import numpy as np
    import qm_inputs as qi
    t0 = time.time()
    pool = [qi.serve_job(i, max_points=args.serve_max_points) for i in range(args.serve_pool)]
    npts = [len(w.xyz) - 8 for w in pool]
    print(f"[bench] serve pool: {len(pool)} jobs, {min(npts)}..{max(npts)} points, "
          f"built in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    budget = int(args.serve_budget_gib * (1 << 30))
    rates = [float(r) for r in args.serve_rates.split(",")]
    rng = np.random.Generator(np.random.PCG64(55))
    per_rate = []
    with qm.Server(budget, nworkers=0) as srv:
        t = srv.submit(pool[0])                          # warm-up
        while srv.step():
            pass
        srv.result(t)
        for rate in rates:
            arrive = np.cumsum(rng.exponential(1.0 / rate, size=args.serve_jobs))
            jobs = [pool[k % len(pool)] for k in range(args.serve_jobs)]
            lat, fails, steiner, steps, resident_sum = [], 0, 0, 0, 0
            pending = {}
            nxt = 0
            start = time.perf_counter()
            while nxt < len(jobs) or pending:
                now = time.perf_counter() - start
                while nxt < len(jobs) and arrive[nxt] <= now:
                    tk = srv.submit(jobs[nxt])
                    if tk is None:                     # no room: completions first
                        break
                    pending[tk] = arrive[nxt]
                    nxt += 1
                if not pending:
                    time.sleep(0.0005)
                    continue
                resident_sum += srv.step()
                steps += 1
                for tk in list(pending):
                    got = srv.poll(tk, wait_ms=0)
                    if got is None:
                        continue
                    res, code = got[0], got[1]
                    lat.append(time.perf_counter() - start - pending.pop(tk))
                    if res is None or code not in (0, -4):
                        fails += 1
                    else:
                        steiner += res.steiner
            span = time.perf_counter() - start
            per_rate.append({"rate_jobs_per_s": rate, "jobs": len(jobs), "failed": fails,
                             "jobs_per_s": len(jobs) / span, "steiner_per_s": steiner / span,
                             "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                             "steps": steps, "mean_resident": resident_sum / max(steps, 1)})
            print(f"[bench] stepped, rate {rate:g}/s: {per_rate[-1]}", file=sys.stderr, flush=True)
    best = max(per_rate, key=lambda r: r["jobs_per_s"])
    out = {
        "metric": "served jobs/sec, stepped server (continuous batching, Poisson arrivals)",
        "value": best["jobs_per_s"], "unit": "jobs/s", "n_gpus": 1, "higher_is_better": True,
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"served_pool{len(pool)}_max{args.serve_max_points}", "form": "stepped",
                   "budget_gib": args.serve_budget_gib, "points": [int(min(npts)), int(max(npts))]},
        "rates": per_rate,
    }
    print(json.dumps(out), flush=True)


def bench_serve_pipelined(args, qm):
    """Served workload with each job's input preparation in the latency: a
    job arrives as a generator index; its CDT is built on the host, then it
    is refined.  Serial: the arrival loop builds each job before submitting
    it.  Pipelined (the paper's gQM3D+ split): PipelinedServer builds jobs on
    --prep-threads host threads while the device refines others.  Latency of
    a job: arrival to completion."""
    import numpy as np
    import qm_inputs as qi
    budget = int(args.serve_budget_gib * (1 << 30))
    rates = [float(r) for r in args.serve_rates.split(",")]
    prep = lambda i: qi.serve_job(i, max_points=args.serve_max_points)
    t0 = time.perf_counter()
    for i in range(8):
        prep(i)
    print(f"[bench] preparation of 8 jobs: {time.perf_counter() - t0:.2f}s", file=sys.stderr, flush=True)
    out_rates = []
    for mode in ("serial", "pipelined"):
        rng = np.random.Generator(np.random.PCG64(55))
        for rate in rates:
            arrive = np.cumsum(rng.exponential(1.0 / rate, size=args.serve_jobs))
            lat, prep_s, fails = [], [], 0
            if mode == "serial":
                srv = qm.Server(budget, nworkers=args.streams)
            else:
                srv = qm.PipelinedServer(budget, nworkers=args.streams, prep_threads=args.prep_threads)
            pending = {}
            nxt = 0
            start = time.perf_counter()
            while nxt < len(arrive) or pending:
                now = time.perf_counter() - start
                while nxt < len(arrive) and arrive[nxt] <= now:
                    if mode == "serial":
                        a = time.perf_counter()
                        w = prep(nxt % args.serve_pool)
                        p_s = time.perf_counter() - a
                        tk = srv.submit(w)
                        while tk is None:             # no room: wait for completions, then retry
                            time.sleep(0.001)
                            tk = srv.submit(w)
                        pending[tk] = (arrive[nxt], p_s)
                    else:
                        pending[srv.submit(prep, nxt % args.serve_pool)] = (arrive[nxt], None)
                    nxt += 1
                for tk in list(pending):
                    got = srv.poll(tk, wait_ms=0)
                    if got is None:
                        continue
                    t_arr, p_s = pending.pop(tk)
                    res, code = got[0], got[1]
                    lat.append(time.perf_counter() - start - t_arr)
                    prep_s.append(p_s if p_s is not None else got[3])
                    fails += res is None or code not in (0, -4)
                time.sleep(0.0005)
            span = time.perf_counter() - start
            srv.close()
            r = {"mode": mode, "rate_jobs_per_s": rate, "jobs": len(arrive), "failed": int(fails),
                 "jobs_per_s": len(arrive) / span, "p50_s": float(np.percentile(lat, 50)),
                 "p99_s": float(np.percentile(lat, 99)), "prep_mean_s": float(np.mean(prep_s))}
            out_rates.append(r)
            print(f"[bench] {r}", file=sys.stderr, flush=True)
    best = max((r for r in out_rates if r["mode"] == "pipelined"), key=lambda r: r["jobs_per_s"])
    out = {
        "metric": "served jobs/sec, input preparation included (Poisson arrivals)", "value": best["jobs_per_s"],
        "unit": "jobs/s", "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"served_pool{args.serve_pool}_max{args.serve_max_points}_with_preparation",
                   "workers": args.streams, "prep_threads": args.prep_threads, "budget_gib": args.serve_budget_gib},
        "rates": out_rates,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg3",
                    help="cfg1, cfg2, cfg3, or rect[:n[:gamma[:uniform|gauss[:B]]]] (rectangle PLC)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-quality", action="store_true", help="skip the output quality report")
    ap.add_argument("--early-stop", action="store_true",
                    help="the early-stop blasting mode (not a parity mode: timing decides which points win)")
    ap.add_argument("--no-fast-modes", action="store_true",
                    help="skip the comparison run of the three-sub-phase mode in the single-instance line")
    ap.add_argument("--subphases", action="store_true",
                    help="three-sub-phase rounds (the other reading of the class order: each round runs SS, SF and TET in turn; bit-exact to the oracle's sub-phase reading, not to the paper-order refinement)")
    ap.add_argument("--batch", type=int, default=0,
                    help="instead of the single-instance line: the first N instances of the batched "
                         "workload (config 4), batched jobs/s against one-at-a-time jobs/s")
    ap.add_argument("--streams", type=int, default=8, help="streams (workers) of the batched or served run")
    ap.add_argument("--tune-probe", type=int, default=16,
                    help="instances of the probe batch on which --batch autotunes the lockstep knobs")
    ap.add_argument("--serve", action="store_true",
                    help="instead of the single-instance line: the served workload at --serve-rates")
    ap.add_argument("--serve-rates", default="5,20,80", help="Poisson arrival rates (jobs/s)")
    ap.add_argument("--serve-jobs", type=int, default=48, help="arrivals per rate")
    ap.add_argument("--serve-pool", type=int, default=24, help="distinct pre-generated jobs")
    ap.add_argument("--serve-max-points", type=int, default=50000,
                    help="largest job (the served workload's full range ends at 500000)")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0, help="device-memory budget of the server")
    ap.add_argument("--pipelined", action="store_true",
                    help="with --serve: jobs arrive unprepared; serial against pipelined input preparation")
    ap.add_argument("--prep-threads", type=int, default=8, help="host threads preparing jobs (--pipelined)")
    ap.add_argument("--stepped", action="store_true",
                    help="with --serve: the stepped server (continuous batching in one lockstep batch)")
    ap.add_argument("--dump-rounds", default=None,
                    help="write the last step's per-round records and per-round kernel-family ms (JSON)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the refinement of one instance runs on a single "
              "MI355X (the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1903_03406_amd as qm

    if args.serve:
        if args.pipelined:
            bench_serve_pipelined(args, qm)
        elif args.stepped:
            bench_serve_stepped(args, qm)
        else:
            bench_serve(args, qm)
        return
    if args.batch > 0:
        return bench_batch(args, qm)
    t0 = time.time()
    w = make_workload(args.workload)
    print(f"[bench] workload {w.name}: {len(w.xyz)} vertices, {len(w.tets)} tets, "
          f"{len(w.ftri)} PLC triangles, input built in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    names = ("xyz", "tets", "sf", "sf_facet", "ss", "ss_seg", "ftri", "ftri_facet")
    d = {k: torch.from_numpy(np.ascontiguousarray(getattr(w, k))).to(dev) for k in names}
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    def step(profile=False):
        return qm.refine(d["xyz"], d["tets"], d["sf"], d["sf_facet"], d["ss"], d["ss_seg"], d["ftri"],
                         d["ftri_facet"], w.B, stream=stream, profile=profile, verbose=True,
                         early_stop=args.early_stop, subphases=args.subphases)

    # The first untimed step runs with every kernel family timed and the
    # region counters on (the algorithmic bytes and the phase split come from
    # it); the timed steps time only the grow kernel, with HIP events around
    # its launches on the refinement's stream, and run the kernels unprofiled.
    detail = None
    for i in range(max(args.warmup, 1)):
        r = step(profile=detail is None)
        detail = detail or r
        print(f"[bench] {'warmup' if i < args.warmup else 'detail'} {i}: {r.rounds} rounds, {r.steiner} Steiner, "
              f"{len(r.tets)} tets, {r.seconds_total:.2f}s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    results = []
    for i in range(args.steps):
        results.append(step(profile="grow"))
        print(f"[bench] step {i}: {results[-1].seconds_total:.2f}s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    r = results[-1]
    sec = (t2 - t1) / args.steps
    steiner = r.steiner
    prof = detail.profile
    # dominant grow kernel by the timed steps' own events; its bytes from the
    # detail step's counters of the same tier
    live = {f: sum(x.profile["ms"][f] for x in results) / len(results) for f in TIER_OF}
    fam = max(live, key=live.get)
    kms = live[fam]
    # per launch: the detail step's bytes over its launches, the timed steps'
    # event time over theirs (the same launches, except in the early-stop
    # mode, where timing decides the rounds)
    launches = max(prof["launches"][fam], 1)
    t_launches = max(sum(x.profile["launches"][fam] for x in results) / len(results), 1)
    nbytes = tier_bytes(prof["tiers"][TIER_OF[fam]])
    mean_us = kms * 1e3 / t_launches
    achieved = (nbytes / launches) / (mean_us * 1e-6) / 1e9 if kms > 0 else 0.0
    dominant = max(prof["ms"], key=lambda k: prof["ms"][k])
    sbytes, smodel = insertion_model_bytes(r, prof)
    npts = len(w.xyz) - 8
    size = f"{npts // 1000000}M" if npts >= 1000000 else f"{npts // 1000}K"
    out = {
        "metric": f"Steiner pts/sec ({size}-pt PLC refinement)",
        "value": steiner / sec,
        "unit": "Steiner pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name + ("_early_stop" if args.early_stop else "")
                   + ("_subphases" if args.subphases else ""),
                   "mode": ", ".join(m for m, on in (("early-stop blasting (not a parity mode)", args.early_stop),
                                                     ("three-sub-phase rounds (the other class-order reading)", args.subphases))
                                     if on) or "parity",
                   "input_vertices": int(len(w.xyz)), "input_tets": int(len(w.tets)),
                   "plc_triangles": int(len(w.ftri)), "segments": int(len(w.seg)), "B": w.B,
                   "parallelism": "single instance, one GPU"},
        "tets_per_s": len(r.tets) / sec,
        "output": {"vertices": int(len(r.xyz)), "tets": int(len(r.tets)), "steiner": steiner,
                   "deferred": r.deferred,
                   "rounds": r.rounds, "device_refine_s": r.seconds_refine, "device_setup_s": r.seconds_setup},
        "profile_ms": {k: round(v, 3) for k, v in prof["ms"].items()},   # the untimed detail step
        "overflow_candidates": prof.get("overflow", 0), "poolfull_candidates": prof.get("poolfull", 0),
        "grow_tiers": prof.get("tiers"),
        "grow_phase_frac": (lambda c: {n: round(x / max(sum(c), 1), 4) for n, x in zip(
            ("setup_seeds", "facet_region", "tet_region", "encroach", "radius_rftets", "bfaces",
             "edges_closure", "claims_results"), c)})(prof.get("grow_cycles", [0] * 8)),
        "roofline": {"kernel": KERNEL_OF[fam],
                     "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(w.name, fam, prof["launches"][fam]),
                     "unit_of_bytes": "per launch (traffic and algorithmic_bytes alike)",
                     "launches": prof["launches"][fam], "kernel_ms_per_step": kms,
                     "mean_launch_us": mean_us,
                     "algorithmic_bytes": nbytes / launches, "dominant_family": dominant},
        "whole_step_model": {"bytes": sbytes, "frac_of_hbm_over_step": sbytes / sec / (HBM_PEAK_GBS * 1e9),
                             **{k: round(v, 2) for k, v in smodel.items()}},
    }
    if not (args.no_fast_modes or args.early_stop or args.subphases):
        # the non-parity three-sub-phase mode on the same resident inputs, for
        # comparison (one refinement, host clock; not `value`)
        torch.cuda.synchronize()
        a = time.perf_counter()
        f = qm.refine(d["xyz"], d["tets"], d["sf"], d["sf_facet"], d["ss"], d["ss_seg"], d["ftri"], d["ftri_facet"],
                      w.B, stream=stream, subphases=True)
        torch.cuda.synchronize()
        fs = time.perf_counter() - a
        print(f"[bench] three-sub-phase rounds: {f.rounds} rounds, {f.steiner} Steiner, {fs:.2f}s",
              file=sys.stderr, flush=True)
        out["fast_modes"] = {"three_sub_phase_rounds": {
            "note": "the other reading of the class order: equal to the oracle's sub-phase reading, not to the paper-order refinement (the insertion order differs); a CDT of the same kind",
            "seconds": fs, "steiner_per_s": f.steiner / fs, "tets_per_s": len(f.tets) / fs, "rounds": f.rounds,
            "steiner": f.steiner, "tets": int(len(f.tets))}}
    if not args.no_quality:
        from paper_1903_03406_amd import quality
        print("[bench] quality report ...", file=sys.stderr, flush=True)
        qin, qout = quality.report(w.xyz, w.tets, w.B), quality.report(r.xyz, r.tets, w.B)
        out["quality"] = {"input": {k: v for k, v in qin.items() if k != "dihedral_hist"}, "output": qout}
    if args.dump_rounds:
        with open(args.dump_rounds, "w") as f:
            json.dump({"fields": list(qm.ROUND_NAMES), "rounds": r.rstats.tolist(),
                       "families": list(qm.PROF_FAMILIES), "round_ms": prof["round_ms"].tolist()}, f)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
