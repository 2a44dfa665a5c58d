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
FP64_PEAK = 78.6e12  # MI355X FP64 vector, FLOP/s
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


def batched_leg(ctx, P, W, count, budget, plain_sample, log):
    """4096 planted systems (n 2..12, degree 2..4) in one batched pass vs the
    plain per-system solver on a sample of the same systems."""
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
    done = sum(1 for r in res if r.status == 0)
    # plain solver, one system per call, on the first systems of the batch
    t = time.perf_counter()
    pn = 0
    plain = []
    for s, p in zip(systems[:plain_sample], params[:plain_sample]):
        r = P.ibb_solve(ctx, s, p)
        pn += r.stats["processed"]
        plain.append(r)
    pdt = time.perf_counter() - t
    # members that finished both ways must agree bit for bit (a budget error
    # stops the two schedules at different points, so their partial counts differ)
    agree = all(a.stats == b.stats and np.array_equal(a.lo, b.lo) and np.array_equal(a.hi, b.hi)
                for a, b in zip(plain, res[:plain_sample]) if a.status == 0 and b.status == 0)
    agree = agree and all((a.status == 0) == (b.status == 0) for a, b in zip(plain, res[:plain_sample]))
    # the same batch recorded once and replayed from its graph
    plan = P.BatchPlan(ctx, systems, params)
    plan.run()  # first replay
    t = time.perf_counter()
    rres = plan.run()
    rdt = time.perf_counter() - t
    rkms = P.ibb_last_kernel_ms(ctx)
    plan.close()
    same = all(a.status == b.status and a.stats == b.stats and np.array_equal(a.lo, b.lo)
               and np.array_equal(a.hi, b.hi) and np.array_equal(a.tag, b.tag) for a, b in zip(rres, res))
    return {"systems": count, "budget_nodes_per_system": budget, "completed": done,
            "autotune": {"seconds": tune_s, "sample_per_class": 128,
                         "classes": [{k: c[k] for k in ("lanes", "tiles_per_claim", "blocks_per_cu", "ms")}
                                     for c in tuned]},
            "over_budget": count - done, "tree_nodes": nodes, "seconds": dt, "first_call_seconds": first_dt,
            "kernel_ms": kms,
            "boxes_per_s": nodes / dt, "solves_per_s": count / dt,
            "plain": {"systems": plain_sample, "tree_nodes": pn, "seconds": pdt, "boxes_per_s": pn / pdt,
                      "solves_per_s": plain_sample / pdt},
            "batched_vs_plain_boxes_per_s": (nodes / dt) / (pn / pdt) if pn else None,
            "plain_equals_batch": bool(agree),
            "graph_replay": {"seconds": rdt, "device_ms": rkms, "boxes_per_s": nodes / rdt,
                             "solves_per_s": count / rdt, "identical_to_batch": bool(same)}}


def served_leg(ctx, P, W, rate, duration, log):
    """Poisson arrivals (banded n=12 and products of quadratics, tol 1e-8)
    through the continuous-batching server; latency = arrival to result."""
    import numpy as np
    stream = W.served_stream(0, rate=rate, duration=duration)
    log(f"[bench] served: {len(stream)} requests over {duration} s at {rate}/s")
    srv = P.Server(ctx, max_slots=1024, frontier_cap=1 << 21, reserve_per_solve=1 << 11, levels_per_quantum=8)
    t0 = time.perf_counter()
    i = 0
    live = {}
    lat = []
    nodes = 0
    while i < len(stream) or live:
        now = time.perf_counter() - t0
        while i < len(stream) and stream[i][0] <= now:
            live[srv.submit(stream[i][1])] = stream[i][0]
            i += 1
        if not live:
            time.sleep(max(0.0, stream[i][0] - now))
            continue
        srv.step()
        now = time.perf_counter() - t0
        for rid in list(live):
            r = srv.poll(rid)
            if r is not None:
                lat.append(now - live.pop(rid))
                nodes += r.stats["processed"]
    total = time.perf_counter() - t0
    srv.close()
    lat = np.array(lat)
    return {"requests": len(stream), "offered_rate_per_s": rate, "seconds": total,
            "solves_per_s": len(stream) / total, "boxes_per_s": nodes / total,
            "latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
            "latency_ms_p99": float(np.percentile(lat, 99) * 1e3)}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1802_00330_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(nodes):
    """HBM bytes per launch of the search kernel from the committed rocprofv3
    counter summary, when it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "solve_kernel_dense6_traffic.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("kernel_source") != kernel_source_hash() or t.get("tree_nodes") != nodes:
        return None
    return t["hbm_bytes_per_launch"]


def cpu_baseline(s, sample_nodes):
    import oracle
    t = time.perf_counter()
    r = oracle.solve(s, max_boxes=sample_nodes)
    dt = time.perf_counter() - t
    done = r.stats["processed"] if r.status == 0 else sample_nodes
    return {"value": done / dt, "unit": "boxes/s", "cores": 1, "kind": "oracle",
            "sample": f"first {done} tree nodes (last-in-first-out order) of the same solve, one thread, "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2,
                    help="solves before the timed ones (the schedule autotuner times its two candidates here)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=300_000, help="tree nodes the oracle times (0 = skip)")
    ap.add_argument("--batch", type=int, default=4096, help="systems in the batched leg (0 = skip)")
    ap.add_argument("--batch-budget", type=int, default=100_000, help="tree nodes per system in the batch")
    ap.add_argument("--plain-sample", type=int, default=64)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=1.0, help="arrival window of the served leg (0 = skip)")
    ap.add_argument("--serve-light-rate", type=float, default=100.0,
                    help="a second served run at an arrival rate the device keeps up with (0 = skip)")
    ap.add_argument("--serve-light-seconds", type=float, default=2.0)
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
    s = W.dense_planted(args.seed)
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
    for _ in range(max(0, args.warmup - 1)):
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
    gold = os.path.join(ROOT, "tests", "golden", f"expected_dense6_s{args.seed}.json")
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
        "config": {"workload": "dense planted polynomial system, n=6, 20 monomials of degree 1..3 + constant "
                               "per equation, box [-2,2]^6, tol 1e-8, one solve per step",
                   "seed": args.seed, "tree_nodes": nodes, "output_boxes": int(inf[1]),
                   "tree_levels": int(inf[10]), "widest_level": int(inf[11]), "split": "widest"},
        "solves_per_s": args.steps / elapsed,
        "latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
        "latency_ms_p99": float(np.percentile(lat, 99) * 1e3),
        "kernel_ms_mean": kmean * 1e3,
        "kernel_source": kernel_source_hash(),
        "bit_exact_vs_oracle": exact,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": FP64_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK, "traffic": measured_traffic(nodes),
                     "algorithmic_bytes_per_launch": bytes_alg},
    }
    if args.batch > 0:
        out["batched"] = batched_leg(ctx, P, W, args.batch, args.batch_budget, args.plain_sample, log)
        log(f"[bench] batched: {out['batched']}")
    if args.serve_seconds > 0:
        out["served"] = served_leg(ctx, P, W, args.serve_rate, args.serve_seconds, log)
        log(f"[bench] served: {out['served']}")
        if args.serve_light_rate > 0:
            out["served_within_capacity"] = served_leg(ctx, P, W, args.serve_light_rate, args.serve_light_seconds,
                                                       log)
            log(f"[bench] served within capacity: {out['served_within_capacity']}")
    if args.cpu_sample > 0:
        log(f"[bench] timing the oracle on {args.cpu_sample} nodes")
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_sample)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
