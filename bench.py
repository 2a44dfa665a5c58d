#!/usr/bin/env python3
"""Benchmark: boxes/s and solves/s of the interval branch-and-bound search on one
MI355X, with the roofline fraction of the search kernel and the CPU oracle timed
beside it.

One step = one complete solve (every tree level, output sort) of the dense
planted system: n = 6 equations in 6 variables, 20 monomials of total degree
1..3 per equation plus a constant term, coefficients U[-1,1], a planted root
r ~ U[-1,1]^6, initial box [-2,2]^6, width tolerance 1e-8, FP64 intervals with
an FP32 preconditioner (seed 0).  Inputs are resident in device memory before
the timed region except the few-KB system description, which each solve
compiles and copies in.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "boxes/sec and solves/sec (p50/p99 latency), batched vs plain, bit-exact boxes"
WORKLOADS = {
    "dense6": "dense planted polynomial system, n=6, 20 monomials of degree 1..3 + constant per equation, "
              "box [-2,2]^6, tol 1e-8, one solve per step",
    "banded12": "banded system, n=12, f_i = a_i x_i + b_i x_i^3 + 1 - sum_{1<=|j-i|<=2} c_ij (x_j + x_j^2), "
                "box [-1,1]^12, tol 1e-10, one solve per step",
}
FP64_PEAK = 78.6e12  # MI355X FP64 vector, FLOP/s
# solves the schedule autotuner times (two per schedule) before it settles
TUNE_SOLVES = 4
HBM_PEAK = 8.0e12    # bytes/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def flop_model(s):
    """Algorithmic work per tree node (1 flop = one directed-rounded FP64 op;
    an interval op counts one flop per bound).  Returns (exclusion-only box,
    contracted box FP64, contracted box FP32)."""
    import numpy as np
    n = s.n
    deg = s.expo.sum(axis=1).astype(np.int64)
    f_eval = int(np.sum(2 * deg + 2))
    f_jac = 0
    nnz = 0
    for i in range(n):
        a, b = int(s.term_off[i]), int(s.term_off[i + 1])
        for k in range(n):
            dk = [int(deg[t]) for t in range(a, b) if s.expo[t, k] > 0]
            f_jac += sum(2 * d for d in dk)
            nnz += 1 if dk else 0
    f_hs = 2 * f_eval + f_jac + 2 * n * n + 4 * n * nnz + 8 * n * n + 4 * n
    f32 = (8 * n ** 3) // 3
    return f_eval, f_hs, f32


def host_cpu():
    """CPU model and the cores this process may use on the host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, cores


def oracle_pool(jobs, cores):
    """Runs oracle solves (callables) on a thread pool over `cores` host cores
    (the oracle's C calls release the interpreter lock); returns (results,
    wall seconds)."""
    from concurrent.futures import ThreadPoolExecutor
    t = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        res = list(ex.map(lambda f: f(), jobs))
    return res, time.perf_counter() - t


def same_members_leg(ctx, P, sample, sparams, res):
    """The first members solved two ways: the plain solver one system per call,
    and one batch of just these members (same budget)."""
    import numpy as np
    t = time.perf_counter()
    plain = [P.ibb_solve(ctx, s, p) for s, p in zip(sample, sparams)]
    pdt = time.perf_counter() - t
    pn = sum(r.stats["processed"] for r in plain)
    P.ibb_solve_batch(ctx, sample, sparams)
    t = time.perf_counter()
    sb = P.ibb_solve_batch(ctx, sample, sparams)
    sdt = time.perf_counter() - t
    sn = sum(r.stats["processed"] for r in sb)
    pdone = sum(1 for r in plain if r.status == P.OK)
    # finished members agree bit for bit; a budget error stops the two
    # schedules at different points, so only the status is compared there
    agree = all((a.status == P.OK) == (b.status == P.OK) for a, b in zip(plain, sb))
    agree = agree and all(a.stats == b.stats and np.array_equal(a.lo, b.lo) and np.array_equal(a.hi, b.hi)
                          and np.array_equal(a.tag, b.tag) for a, b in zip(plain, sb) if a.status == P.OK)
    agree = agree and all(a.status == b.status and a.stats == b.stats and np.array_equal(a.lo, b.lo)
                          for a, b in zip(sb, res[:len(sample)]))
    return {"systems": len(sample), "completed": pdone, "tree_nodes": pn,
            "plain_seconds": pdt, "plain_boxes_per_s": pn / pdt, "plain_solves_per_s": pdone / pdt,
            "batch_seconds": sdt, "batch_boxes_per_s": sn / sdt, "batch_solves_per_s": pdone / sdt,
            "batched_vs_plain_solves_per_s": pdt / sdt, "identical": bool(agree)}


def batched_leg(ctx, P, W, count, budget, plain_sample, cpu_members, log):
    """4096 planted systems (n 2..12, degree 2..4) in one batched pass; the
    plain per-system solver and the batch on the same sample of members; the
    oracle on all host cores on a smaller sample."""
    import numpy as np
    t = time.perf_counter()
    systems = W.batch_planted(0, count=count)
    log(f"[bench] batch: generated {count} systems in {time.perf_counter() - t:.1f} s")
    params = [P.make_params(s.tol, max_boxes=budget) for s in systems]
    P.ibb_solve_batch(ctx, systems[:64], params[:64])  # warm-up
    # launch configuration per lane-count class, timed on a sample of each class
    t = time.perf_counter()
    tuned = P.ibb_batch_tune(ctx, systems, params, sample=128)
    tune_s = time.perf_counter() - t
    log(f"[bench] batch: autotuned in {tune_s:.1f} s: {tuned}")
    # the first call at this size also allocates the context's batch workspace;
    # the second is the steady-state eager call
    t = time.perf_counter()
    P.ibb_solve_batch(ctx, systems, params)
    first_dt = time.perf_counter() - t
    t = time.perf_counter()
    res = P.ibb_solve_batch(ctx, systems, params)
    dt = time.perf_counter() - t
    kms = P.ibb_last_kernel_ms(ctx)
    nodes = sum(r.stats["processed"] for r in res)
    done = sum(1 for r in res if r.status == P.OK)
    over = sum(1 for r in res if r.status == P.ERR_BUDGET)
    by_n = {}
    for s, r in zip(systems, res):
        c = by_n.setdefault(s.n, [0, 0])
        c[0] += 1
        c[1] += r.status == P.OK
    # the same members two ways: the plain solver one system per call, and
    # one batch of just these members (same budget)
    same_members = None
    sample, sparams = systems[:plain_sample], params[:plain_sample]
    if plain_sample > 0:
        same_members = same_members_leg(ctx, P, sample, sparams, res)
    log(f"[bench] batch: {done} of {count} completed, {nodes} tree nodes in {dt:.3f} s "
        f"(first call {first_dt:.3f} s)")
    # the same batch recorded once and replayed from its graph (a plan is one
    # batch: one whose frontier exceeds the device memory is reported, not split)
    try:
        plan = P.BatchPlan(ctx, systems, params)
        plan.run()  # first replay
        t = time.perf_counter()
        rres = plan.run()
        rdt = time.perf_counter() - t
        rkms = P.ibb_last_kernel_ms(ctx)
        plan.close()
        same = all(a.status == b.status and a.stats == b.stats and np.array_equal(a.lo, b.lo)
                   and np.array_equal(a.hi, b.hi) and np.array_equal(a.tag, b.tag) for a, b in zip(rres, res))
        replay = {"seconds": rdt, "device_ms": rkms, "boxes_per_s": nodes / rdt, "solves_per_s": done / rdt,
                  "identical_to_batch": bool(same)}
    except RuntimeError as e:
        replay = {"error": str(e)}
    out = {"systems": count, "budget_nodes_per_system": budget, "completed": done, "over_budget": over,
           "completed_by_n": {str(k): {"members": v[0], "completed": v[1]} for k, v in sorted(by_n.items())},
           "autotune": {"seconds": tune_s, "sample_per_class": 128,
                        "classes": [{k: c[k] for k in ("lanes", "tiles_per_claim", "blocks_per_cu", "ms",
                                                       "front_per_member")}
                                    for c in tuned]},
           "tree_nodes": nodes, "seconds": dt, "first_call_seconds": first_dt, "kernel_ms": kms,
           "boxes_per_s": nodes / dt, "solves_per_s": done / dt, "members_per_s": count / dt,
           "same_members": same_members,
           "graph_replay": replay}
    if cpu_members > 0:
        import oracle
        model, cores = host_cpu()
        jobs = [(lambda s=s: oracle.solve(s, max_boxes=budget)) for s in systems[:cpu_members]]
        ores, odt = oracle_pool(jobs, cores)
        on = sum(r.stats["processed"] or budget for r in ores)
        odone = sum(1 for r in ores if r.status == 0)
        same_st = all((a.status == 0) == (b.status == P.OK) for a, b in zip(ores, res))
        out["cpu_baseline"] = {"value": on / odt, "unit": "boxes/s", "solves_per_s": odone / odt,
                               "cores": cores, "cpu": model, "kind": "oracle",
                               "sample": f"the first {cpu_members} members, same budget, one system per task "
                                         f"on {cores} threads, {odt:.1f} s",
                               "statuses_equal_device": bool(same_st)}
    return out


def served_leg(ctx, P, W, rate, duration, drain, log, gold=None):
    """Poisson arrivals (banded n=12 and products of quadratics, tol 1e-8)
    through the continuous-batching server; latency = arrival to result.
    Arrivals stop after `duration` s; requests still queued `drain` s later
    are cancelled (they count as not served)."""
    import numpy as np
    stream = W.served_stream(0, rate=rate, duration=duration)
    log(f"[bench] served: {len(stream)} requests over {duration} s at {rate}/s")
    srv = P.Server(ctx, max_slots=1024, frontier_cap=1 << 21, reserve_per_solve=1 << 11, levels_per_quantum=8,
                   pool_bytes=64 << 30)
    t0 = time.perf_counter()
    i = 0
    live = {}  # request id -> (arrival time, stream index)
    lat, ok, failed, nodes, cancelled = [], 0, {}, 0, 0
    exact = {"compared": 0, "equal": 0}
    cut = False
    while i < len(stream) or live:
        now = time.perf_counter() - t0
        while i < len(stream) and stream[i][0] <= now:
            live[srv.submit(stream[i][1])] = (stream[i][0], i)
            i += 1
        if not cut and now > duration + drain:
            # stop: cancel what has not been admitted yet
            cut = True
            for rid in list(live):
                if srv.cancel(rid):
                    del live[rid]
                    cancelled += 1
        if not live:
            if i < len(stream):
                time.sleep(max(0.0, stream[i][0] - now))
            continue
        srv.step()
        now = time.perf_counter() - t0
        for rid in srv.finished():
            arrival, k = live.pop(rid)
            r = srv.poll(rid)
            lat.append(now - arrival)
            nodes += r.stats["processed"]
            if r.status == P.OK:
                ok += 1
            else:
                failed[str(r.status)] = failed.get(str(r.status), 0) + 1
            if gold is not None and k in gold:
                g = gold[k]
                exact["compared"] += 1
                exact["equal"] += int(r.status == g["status"] and r.stats == g["stats"]
                                      and r.lo.tolist() == g["lo"] and r.hi.tolist() == g["hi"]
                                      and r.tag.tolist() == g["tag"])
    total = time.perf_counter() - t0
    srv.close()
    lat = np.array(lat) if lat else np.zeros(1)
    return {"requests": len(stream), "offered_rate_per_s": rate, "arrival_seconds": duration,
            "seconds": total, "completed": ok, "failed": failed, "cancelled_unserved": cancelled,
            "solves_per_s": ok / total, "boxes_per_s": nodes / total,
            "latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
            "latency_ms_p99": float(np.percentile(lat, 99) * 1e3),
            "bit_exact_vs_oracle": exact}


def served_gold():
    """Stored oracle results of served-stream requests (stream index -> result)."""
    path = os.path.join(ROOT, "tests", "golden", "expected_served_s0.json")
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    out = {}
    for r in g["requests"]:
        out[r["index"]] = {"status": r["status"], "stats": r["stats"], "tag": r["tag"],
                           "lo": [[float.fromhex(v) for v in row] for row in r["lo"]],
                           "hi": [[float.fromhex(v) for v in row] for row in r["hi"]]}
    return out


def served_cpu_baseline(W, rate, duration, requests, nodes_each, mean_nodes, log):
    """The oracle on all host cores over a bounded replay of the request
    stream: the first `nodes_each` tree nodes of each of the first `requests`
    requests, one request per task."""
    import oracle
    model, cores = host_cpu()
    stream = W.served_stream(0, rate=rate, duration=duration, max_requests=requests)
    jobs = [(lambda s=s: oracle.solve(s, max_boxes=nodes_each)) for _, s in stream]
    res, dt = oracle_pool(jobs, cores)
    nodes = sum(r.stats["processed"] or nodes_each for r in res)
    v = nodes / dt
    log(f"[bench] served oracle replay: {nodes} nodes in {dt:.1f} s on {cores} threads")
    return {"value": v, "unit": "boxes/s", "solves_per_s_estimate": v / mean_nodes if mean_nodes else None,
            "cores": cores, "cpu": model, "kind": "oracle",
            "sample": f"first {nodes_each} tree nodes of each of the first {requests} requests, one request "
                      f"per task on {cores} threads, {dt:.1f} s; solves/s = boxes/s / the served requests' mean "
                      f"tree size ({mean_nodes:.0f} nodes)"}


def variants_leg(ctx, P, W, batch_members, log):
    """The Krawczyk contractor and the mean-value exclusion test beside the
    default (Hansen-Sengupta, natural extension): tree nodes, kernel time and
    boxes/s of the dense n=6 (seed 0, tol 1e-8) and banded n=12 (seed 0, tol
    1e-10) solves, and of the first members of the 4096-system batch."""
    variants = {"hansen_sengupta": {}, "krawczyk": {"contractor": 1}, "mean_value": {"inclusion": 1},
                "krawczyk_mean_value": {"contractor": 1, "inclusion": 1}}
    out = {}
    for name, s in (("dense_n6_s0", W.dense_planted(0)), ("banded_n12_s0", W.banded(0))):
        out[name] = {}
        for v, kw in variants.items():
            for _ in range(TUNE_SOLVES):  # each variant's schedule is tuned on its first solves
                P.solve(ctx, s, **kw)
            r = P.solve(ctx, s, **kw)
            ms = P.ibb_last_kernel_ms(ctx)
            out[name][v] = {"status": r.status, "tree_nodes": r.stats.get("processed"),
                            "output_boxes": len(r.tag), "unique": int(r.tag.sum()) if len(r.tag) else 0,
                            "kernel_ms": ms, "boxes_per_s": r.stats.get("processed", 0) / (ms / 1e3)}
        log(f"[bench] variants {name}: {out[name]}")
    if batch_members > 0:
        systems = W.batch_planted(0, count=batch_members)
        out[f"batch_first_{batch_members}"] = {}
        for v, kw in variants.items():
            params = [P.make_params(s.tol, max_boxes=100_000, **kw) for s in systems]
            P.ibb_solve_batch(ctx, systems, params)
            t = time.perf_counter()
            res = P.ibb_solve_batch(ctx, systems, params)
            dt = time.perf_counter() - t
            nodes = sum(r.stats["processed"] for r in res)
            out[f"batch_first_{batch_members}"][v] = {
                "completed": sum(1 for r in res if r.status == P.OK), "tree_nodes": nodes, "seconds": dt,
                "boxes_per_s": nodes / dt}
        log(f"[bench] variants batch: {out[f'batch_first_{batch_members}']}")
    return out


def single_solves(ctx, P, W, steps, log, cpu_nodes=100_000):
    """Per-solve latency and boxes/s of the circle/line system (n=2) and the
    banded n=12 system (seed 0, tol 1e-10), workspace resident on the device."""
    import numpy as np
    import torch
    out = {}
    for name, s in (("circle_line_n2", W.circle_line()), ("banded_n12_s0", W.banded(0))):
        r = P.solve(ctx, s)  # sizes the buffers; the schedule autotuner times its candidates
        for _ in range(TUNE_SOLVES - 1):
            P.solve(ctx, s)
        fcap = 1
        while fcap < 4 * max(r.max_frontier, 256):
            fcap *= 2
        ocap = max(16, len(r.tag))
        ws = torch.empty(P.ibb_workspace_size(s.n, fcap, ocap), dtype=torch.uint8, device="cuda")
        olo = torch.empty(ocap * s.n, dtype=torch.float64, device="cuda")
        ohi = torch.empty_like(olo)
        otag = torch.empty(ocap, dtype=torch.uint8, device="cuda")
        info = torch.zeros(16, dtype=torch.int64, device="cuda")
        stream = torch.cuda.current_stream()
        params = P.make_params(s.tol)
        lat, kms = [], []
        for k in range(steps + 2):
            a = time.perf_counter()
            st = P.ibb_solve_async(ctx, s, params, ws, fcap, ocap, olo, ohi, otag, info, stream=stream)
            stream.synchronize()
            if k >= 2:
                lat.append(time.perf_counter() - a)
                kms.append(P.ibb_last_kernel_ms(ctx))
            assert st == P.OK
        inf = info.cpu().numpy()
        assert inf[0] == P.OK
        nodes = int(inf[2])
        out[name] = {"tree_nodes": nodes, "latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
                     "latency_ms_p99": float(np.percentile(lat, 99) * 1e3),
                     "kernel_ms_mean": float(np.mean(kms)), "boxes_per_s": nodes / float(np.median(lat)),
                     "same_as_solve": bool(dict(zip(P.STATS_FIELDS, (int(v) for v in inf[2:10]))) == r.stats)}
        if cpu_nodes > 0:
            # the oracle on one core: the whole solve, or its first cpu_nodes tree nodes
            import oracle
            t = time.perf_counter()
            o = oracle.solve(s, max_boxes=cpu_nodes)
            odt = time.perf_counter() - t
            done = o.stats["processed"] if o.status == 0 else cpu_nodes
            model, _ = host_cpu()
            out[name]["cpu_baseline"] = {"value": done / odt, "unit": "boxes/s", "cores": 1, "cpu": model,
                                         "kind": "oracle",
                                         "sample": ("the whole solve" if o.status == 0 else
                                                    f"first {done} tree nodes (last-in-first-out order)") +
                                                   f", one thread, {odt:.2f} s"}
        log(f"[bench] {name}: {out[name]}")
    return out


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1802_00330_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def measured_profile(system, nodes, kind):
    """A committed rocprofv3 counter summary of the search kernel on this
    workload (profiles/solve_kernel_<system>_<kind>.json), when it was taken
    on the current kernel source and the same tree; else None."""
    path = os.path.join(ROOT, "profiles", f"solve_kernel_{system}_{kind}.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("kernel_source") != kernel_source_hash() or t.get("tree_nodes") != nodes:
        return None
    return t


def measured_fp64(system, nodes, kernel_s):
    """FP64 vector FLOP/s the hardware issued in the search kernel: the
    wave-level FP64 add, multiply and fused multiply-add instructions of one
    launch (rocprofv3 counters) times 64 lanes (2 flops per FMA lane), over the
    launch time measured here; includes the directed-rounding and division
    emulation work and masked lanes, so it bounds the useful rate from above."""
    t = measured_profile(system, nodes, "valu")
    if t is None:
        return None
    c = t["counters"]
    flops = 64.0 * (c["SQ_INSTS_VALU_ADD_F64"] + c["SQ_INSTS_VALU_MUL_F64"] + 2.0 * c["SQ_INSTS_VALU_FMA_F64"])
    return {"flops_issued_per_launch": flops, "tflops": flops / kernel_s / 1e12,
            "frac": flops / kernel_s / FP64_PEAK, "counters": c}


def cpu_baseline(s, sample_nodes):
    import oracle
    t = time.perf_counter()
    r = oracle.solve(s, max_boxes=sample_nodes)
    dt = time.perf_counter() - t
    done = r.stats["processed"] if r.status == 0 else sample_nodes
    model, _ = host_cpu()
    return {"value": done / dt, "unit": "boxes/s", "cores": 1, "cpu": model, "kind": "oracle",
            "sample": f"first {done} tree nodes (last-in-first-out order) of the same solve, one thread, "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2,
                    help="untimed solves before the timed ones (after the set-up solves in which the schedule "
                         "autotuner times its two candidates)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--system", choices=("dense6", "banded12"), default="dense6",
                    help="workload of the timed solves: the dense n=6 system (tol 1e-8, the headline) or the "
                         "banded n=12 system (tol 1e-10)")
    ap.add_argument("--cpu-sample", type=int, default=300_000, help="tree nodes the oracle times (0 = skip)")
    ap.add_argument("--batch", type=int, default=4096, help="systems in the batched leg (0 = skip)")
    ap.add_argument("--batch-budget", type=int, default=100_000, help="tree nodes per system in the batch")
    ap.add_argument("--plain-sample", type=int, default=64,
                    help="batch members solved both by the plain solver and as a batch of their own")
    ap.add_argument("--batch-cpu-members", type=int, default=16,
                    help="batch members the oracle solves on all host cores (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="arrival window of the served leg (0 = skip)")
    ap.add_argument("--serve-drain", type=float, default=10.0,
                    help="seconds after the arrival window at which requests not yet admitted are cancelled")
    ap.add_argument("--serve-light-rate", type=float, default=100.0,
                    help="a second served run at an arrival rate the device keeps up with (0 = skip)")
    ap.add_argument("--serve-light-seconds", type=float, default=5.0)
    ap.add_argument("--serve-cpu-requests", type=int, default=32,
                    help="requests of the stream replayed on the oracle on all host cores (0 = skip)")
    ap.add_argument("--serve-cpu-nodes", type=int, default=20_000, help="tree nodes per replayed request")
    ap.add_argument("--singles", type=int, default=5, help="timed solves of the n=2 and banded n=12 systems")
    ap.add_argument("--variants", type=int, default=1, help="time the Krawczyk and mean-value variants (0 = skip)")
    ap.add_argument("--variants-batch", type=int, default=512, help="batch members solved with each variant")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="MiB copied by a plain device copy before the solves (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: one process drives one device and the search has "
              "no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1802_00330_amd as P
    import workloads as W

    assert torch.cuda.is_available(), "no GPU visible"
    dev = torch.device("cuda:0")
    ctx = P.Context(0)
    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {args.copy_probe} MiB read, {args.copy_probe} MiB written")
        del src, dst
    s = W.dense_planted(args.seed) if args.system == "dense6" else W.banded(args.seed)
    params = P.make_params(s.tol)
    stream = torch.cuda.current_stream(dev)

    # device buffers sized on a first (warm-up) solve
    fcap, ocap = 1 << 20, 1 << 10
    while True:
        ws = torch.empty(P.ibb_workspace_size(s.n, fcap, ocap), dtype=torch.uint8, device=dev)
        olo = torch.empty(ocap * s.n, dtype=torch.float64, device=dev)
        ohi = torch.empty_like(olo)
        otag = torch.empty(ocap, dtype=torch.uint8, device=dev)
        info = torch.zeros(16, dtype=torch.int64, device=dev)
        st = P.ibb_solve_async(ctx, s, params, ws, fcap, ocap, olo, ohi, otag, info, stream=stream)
        assert st == P.OK, P.ibb_strerror(st)
        stream.synchronize()
        inf = info.cpu().numpy()
        if inf[0] == P.ERR_QUEUE_OVERFLOW:
            fcap *= 4
            continue
        if inf[0] == P.ERR_OUTPUT_CAPACITY:
            ocap = int(inf[1])
            continue
        assert inf[0] == P.OK, P.ibb_strerror(int(inf[0]))
        break
    log(f"[bench] warm solve: {int(inf[2])} nodes, {int(inf[1])} boxes, {int(inf[10])} levels, "
        f"widest level {int(inf[11])}, frontier cap {fcap}")
    # set-up: the schedule autotuner times two launches of each schedule
    # (the sizing solve above was the first), then the warm-up solves
    for _ in range(TUNE_SOLVES - 1):
        P.ibb_solve_async(ctx, s, params, ws, fcap, ocap, olo, ohi, otag, info, stream=stream)
        stream.synchronize()
    for _ in range(args.warmup):
        P.ibb_solve_async(ctx, s, params, ws, fcap, ocap, olo, ohi, otag, info, stream=stream)
        stream.synchronize()
    torch.cuda.synchronize()

    lat, kms = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        a = time.perf_counter()
        P.ibb_solve_async(ctx, s, params, ws, fcap, ocap, olo, ohi, otag, info, stream=stream)
        stream.synchronize()
        lat.append(time.perf_counter() - a)
        kms.append(P.ibb_last_kernel_ms(ctx))
        log(f"[bench] step {k}: {lat[-1] * 1e3:.2f} ms (search kernel {kms[-1]:.2f} ms)")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    inf = info.cpu().numpy()
    assert inf[0] == P.OK
    nodes = int(inf[2])
    elapsed = t1 - t0
    value = nodes * args.steps / elapsed

    # bit-exactness against the stored oracle result of the same solve
    exact = None
    gold = os.path.join(ROOT, "tests", "golden", f"expected_{args.system}_s{args.seed}.json")
    if os.path.exists(gold):
        g = json.load(open(gold))
        m = int(inf[1])
        lo = olo[: m * s.n].view(m, s.n).cpu().numpy()
        hi = ohi[: m * s.n].view(m, s.n).cpu().numpy()
        tag = otag[:m].cpu().numpy()
        exp_lo = np.array([[float.fromhex(v) for v in row] for row in g["lo"]]).reshape(-1, s.n)
        exp_hi = np.array([[float.fromhex(v) for v in row] for row in g["hi"]]).reshape(-1, s.n)
        stats = dict(zip(P.STATS_FIELDS, (int(v) for v in inf[2:10])))
        exact = bool(g["status"] == 0 and stats == g["stats"] and lo.shape == exp_lo.shape
                     and np.array_equal(lo.view(np.uint64), exp_lo.view(np.uint64))
                     and np.array_equal(hi.view(np.uint64), exp_hi.view(np.uint64))
                     and tag.tolist() == g["tag"])

    f_eval, f_hs, f32 = flop_model(s)
    excl = int(inf[3])
    contracted = nodes - excl
    flops = excl * f_eval + contracted * f_hs + contracted * f32 / 2.0  # FP32 at twice the FP64 rate
    kmean = float(np.mean(kms)) / 1e3
    achieved = flops / kmean
    G = 2 if s.n <= 2 else 4 if s.n <= 4 else 8 if s.n <= 8 else 16
    bytes_alg = nodes * (16 * G + 4) + (int(inf[7]) * 2 + int(inf[6])) * (16 * G + 4)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "boxes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.system],
                   "seed": args.seed, "tree_nodes": nodes, "output_boxes": int(inf[1]),
                   "tree_levels": int(inf[10]), "widest_level": int(inf[11]), "split": "widest"},
        "solves_per_s": args.steps / elapsed,
        "latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
        "latency_ms_p99": float(np.percentile(lat, 99) * 1e3),
        "kernel_ms_mean": kmean * 1e3,
        "kernel_source": kernel_source_hash(),
        "bit_exact_vs_oracle": exact,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": FP64_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK,
                     "traffic": (measured_profile(args.system, nodes, "traffic") or {}).get("hbm_bytes_per_launch"),
                     "algorithmic_bytes_per_launch": bytes_alg,
                     "fp64_issued": measured_fp64(args.system, nodes, kmean)},
    }
    if args.batch > 0:
        out["batched"] = batched_leg(ctx, P, W, args.batch, args.batch_budget, args.plain_sample,
                                     args.batch_cpu_members, log)
        log(f"[bench] batched: {out['batched']}")
    if args.serve_seconds > 0:
        gold = served_gold()
        out["served"] = served_leg(ctx, P, W, args.serve_rate, args.serve_seconds, args.serve_drain, log, gold)
        log(f"[bench] served: {out['served']}")
        if args.serve_light_rate > 0:
            out["served_within_capacity"] = served_leg(ctx, P, W, args.serve_light_rate, args.serve_light_seconds,
                                                       args.serve_drain, log, gold)
            log(f"[bench] served within capacity: {out['served_within_capacity']}")
        if args.serve_cpu_requests > 0:
            sv = out["served"]
            done = sv["completed"] + sum(sv["failed"].values())
            mean_nodes = sv["boxes_per_s"] * sv["seconds"] / max(1, done)
            out["served"]["cpu_baseline"] = served_cpu_baseline(W, args.serve_rate, args.serve_seconds,
                                                                args.serve_cpu_requests, args.serve_cpu_nodes,
                                                                mean_nodes, log)
    if args.singles > 0:
        out["single_solves"] = single_solves(ctx, P, W, args.singles, log)
    if args.variants:
        out["variants"] = variants_leg(ctx, P, W, args.variants_batch, log)
    if args.cpu_sample > 0:
        log(f"[bench] timing the oracle on {args.cpu_sample} nodes")
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_sample)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
