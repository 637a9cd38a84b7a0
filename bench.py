#!/usr/bin/env python3
"""Benchmark: CFPQ closure throughput on one MI355X.

A step is one full relational closure (matrix initialisation, every product,
union and change check until the fixpoint) of the Dyck grammar on a seeded
G(16384, 65536) graph with labels a/b, edges already in device memory.  The
value is closure Gbit-op/s: 2 npad^3 Boolean operations (one AND and one OR per
(i, k, j)) per executed product, divided by the wall time of the closure, with
every product dense (the autotuned kernel).  The "hybrid" object times the
same closure with the per-product choice between the dense kernel and the
sparse-operand products (the library default), whose sparse products are
not counted as bit-operations: its figure is time to the fixpoint.

Prints one JSON line.  ``--gpus`` above 1 is refused: this build runs on one
GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "closure Gbitop/s at n=16384; batched queries/s + p50/p99 latency vs plain"
# MI355X peaks used for the roofline fraction.
PEAK_INT8_TOPS = 5000.0  # dense int8 MFMA, 5.0 POP/s (1 MAC = 2 ops = AND + OR here)
PEAK_FP4_TOPS = 10100.0  # dense fp4 (e2m1) MFMA, 10.1 PFLOP/s
# VALU: 256 CUs x 64 lanes per clock x 2.4 GHz x 64 bit-operations per v_and_or_b32
PEAK_VALU_BITOPS_T = 256 * 64 * 2.4e9 * 64 / 1e12
# The fp4 product's kernel variants: tile 2 or 3 = one workgroup per output
# tile with that many pipeline stages, 5 = the persistent kernel (the default).
FP4_DEFAULT_TILE = 5


def fp4_kernel_name(tile):
    return "mfma4_persistent_kernel" if tile == 5 else f"mfma_product_kernel<true, {tile}>"


def _blas_product_rate(inst, seconds_target=4.0):
    """The oracle's own Boolean product (oracle/alg1.py, float64 BLAS) timed on
    a bounded row block of the first product of the same workload."""
    import numpy as np
    from oracle import alg1
    try:
        from threadpoolctl import threadpool_info
        threads = max([int(i.get("num_threads", 1)) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    t0 = alg1.initial_matrix(inst.n, inst.edges, inst.grammar)
    b, c = t0[inst.grammar.nt("A")], t0[inst.grammar.nt("B")]
    n = inst.n
    rows, reps, dt = min(n, 1024), 0, 0.0
    t = time.perf_counter()
    alg1.bool_product(b[:rows], c)
    probe = time.perf_counter() - t
    rows = int(min(n, max(rows, rows * seconds_target / max(probe, 1e-6))))
    while dt < seconds_target:
        t = time.perf_counter()
        alg1.bool_product(b[:rows], c)
        dt += time.perf_counter() - t
        reps += 1
    return {"value": round(2.0 * rows * n * n * reps / dt / 1e9, 3), "unit": "Gbitop/s", "threads": threads,
            "sample": f"Boolean product (float64 BLAS) of rows 0..{rows - 1} of T_A by T_B at n={n}, "
                      f"{reps} time(s), {dt:.1f} s"}


def _bitset_closure_rate(inst, closure_bitops):
    """Algorithm 1 on bit-packed rows (oracle/cfpq_bitset.c, OpenMP over the
    rows of each product) on the whole benchmark workload, all host cores: the
    plain multi-core CPU closure.  Its result is checked against the worklist
    oracle's stored digest for this workload."""
    import hashlib
    import json as _json
    import numpy as np
    from oracle import bitset
    threads = len(os.sched_getaffinity(0))
    bitset.closure(64, inst.edges[:0], inst.grammar, threads=threads)  # loads the library
    t = time.perf_counter()
    bits, loops, rc = bitset.closure(inst.n, inst.edges, inst.grammar, threads=threads)
    dt = time.perf_counter() - t
    gold = _json.load(open(os.path.join(ROOT, "tests", "golden", "digests.json"))).get(inst.tag, {})
    digest = hashlib.sha256(np.ascontiguousarray(bits).astype("<u8").tobytes()).hexdigest()
    return {"value": round(closure_bitops / dt / 1e9, 3), "unit": "Gbitop/s", "threads": threads,
            "time_to_solution_s": round(dt, 3), "jacobi_loops": loops, "n": inst.n,
            "identical_to_oracle_digest": digest == gold.get("sha256") if gold else None,
            "sample": f"bit-packed Algorithm 1 (Jacobi, OpenMP over rows), whole closure of {inst.tag} on "
                      f"{threads} threads: {dt:.2f} s; value = the dense GPU closure's {closure_bitops:.3e} "
                      f"bit-ops / that time"}


def cpu_baseline(cfpq, torch, inst, sample_n=8192, closure_bitops=None):
    """The C worklist oracle's time to the fixpoint, single-threaded, on the
    same recipe (ER Dyck, seed 3) at n = sample_n, a bounded sample of the
    n = 16384 workload (about 15-90 s of CPU work, by the host).  ``value`` puts it in the
    metric's unit: the bit-operations the GPU's dense closure executes on that
    instance (2 npad^3 per product, as for the headline) divided by the
    oracle's time to the same relations.  The full-size oracle time comes from
    the digest run that stored the n = 16384 result.  Separate figures: the
    oracle's float64 BLAS product rate, and the bit-packed Algorithm 1 on all
    host cores over the whole workload (``closure_bitops``: the GPU closure's
    bit-operations on it)."""
    import json as _json
    from oracle import worklist
    from workloads import configs
    sample = configs.config3(sample_n, seed=3)
    worklist.closure(64, sample.edges[:0], sample.grammar)  # loads the oracle library
    t = time.perf_counter()
    want = worklist.closure(sample.n, sample.edges, sample.grammar)
    dt = time.perf_counter() - t
    res = cfpq.closure(sample.n, torch.from_numpy(sample.edges).cuda(), sample.grammar, hybrid=0)
    same = bool((cfpq.result_bits(res) == want).all())
    full = _json.load(open(os.path.join(ROOT, "tests", "golden", "digests.json"))).get("er16384_dyck", {})
    return {"value": round(res.stats["bitops"] / dt / 1e9, 3), "unit": "Gbitop/s", "cores": 1,
            "kind": "oracle_closure",
            "sample": f"C worklist oracle (one thread), closure of the ER Dyck recipe at n={sample.n}, "
                      f"{len(sample.edges)} edges: {dt:.2f} s; value = the dense GPU closure's "
                      f"{res.stats['bitops']:.3e} bit-ops on that instance / that time",
            "time_to_solution_s": round(dt, 3), "sample_n": sample.n, "identical_to_gpu": same,
            "host_nproc": len(os.sched_getaffinity(0)),
            "full_size": {"n": inst.n, "time_to_solution_s": full.get("oracle_seconds"),
                          "where": full.get("oracle_host", "digest run on the build host"),
                          "date": full.get("oracle_date")},
            "blas_product": _blas_product_rate(inst),
            "bitset_closure": _bitset_closure_rate(inst, closure_bitops) if closure_bitops else None}


def profiled_traffic(profile_md, kernel, sources):
    """HBM bytes per launch from a committed rocprofv3 summary, or None when
    the summary is of another kernel or the kernel's sources changed since the
    counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", profile_md)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.split(":", 1)[0] in ("traffic_bytes_per_launch", "source_sha256", "kernel"):
            k, v = line.split(":", 1)
            vals[k] = v.strip()
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if vals.get("source_sha256") != h.hexdigest() or "traffic_bytes_per_launch" not in vals:
        return None
    if vals.get("kernel") != kernel:
        return None
    return float(vals["traffic_bytes_per_launch"])


def bench_batch(cfpq, torch, steps=3):
    """Batched closure of the 512-instance workload (sizes log-uniform in
    [64, 2048], hierarchy or G(n, 3n), same-generation or Dyck) against the
    same queries run one at a time with the plain closure (no batching, no
    captured loops).  Edges are in device memory for both.  The engine's route
    per padded side (resident workgroup, or the tile work list with 256 or 128
    tiles) comes from the batch autotuner run on this workload first; the
    batch is also timed with the untuned default routes."""
    from workloads import configs
    insts = configs.config4()
    items = [(i.n, torch.from_numpy(i.edges).cuda(), i.grammar) for i in insts]
    torch.cuda.synchronize()

    def timed(outs):
        t0 = time.perf_counter()
        for _ in range(steps):
            res = cfpq.batch_closure(items, outs=outs)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, res

    cfpq.tune_clear()
    res = cfpq.batch_closure(items)  # warmup + buffers
    outs = [r.bits.view(-1) for r in res]
    t_default, _ = timed(outs)
    t0 = time.perf_counter()
    table = cfpq.batch_autotune(items, max_per_bucket=0, reps=3)
    t_tune = time.perf_counter() - t0
    cfpq.batch_closure(items, outs=outs)
    t_batch, res = timed(outs)
    bitops = sum(r.stats["bitops"] for r in res)
    print(f"[bench] batch of {len(items)}: {t_batch * 1e3:.2f} ms tuned, {t_default * 1e3:.2f} ms default routes "
          f"(tuning {t_tune:.2f} s)", file=sys.stderr, flush=True)
    for it, o in zip(items[:8], outs[:8]):  # warm the plain path
        cfpq.closure(*it, capture=0, out=o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it, o in zip(items, outs):
        cfpq.closure(*it, capture=0, out=o)
    torch.cuda.synchronize()
    t_serial = time.perf_counter() - t0
    print(f"[bench] serial plain: {t_serial * 1e3:.1f} ms", file=sys.stderr, flush=True)
    routes = {str(e["npad"]): (e["route"] if e["route"] == "resident" else f"tiles{e['tile']}") for e in table}
    return {"workload": "batch512_seed4", "instances": len(items),
            "queries_per_s": round(len(items) / t_batch, 1), "ms_per_batch": round(t_batch * 1e3, 3),
            "Gbitop_per_s": round(bitops / t_batch / 1e9, 1),
            "serial_plain_queries_per_s": round(len(items) / t_serial, 1),
            "speedup_vs_serial_plain": round(t_serial / t_batch, 2),
            "route_table": {"source": "cfpq_batch_autotune on this workload", "tuning_s": round(t_tune, 2),
                            "routes_by_npad": routes,
                            "candidates_ms_by_npad": {str(e["npad"]): e["candidates_ms"] for e in table}},
            "default_routes_ms_per_batch": round(t_default * 1e3, 3)}


def bench_hybrid_only(cfpq, torch, steps=5):
    """Only the hybrid closure of the n = 16384 workload (library defaults),
    `steps` times after one warm-up: a kernel trace of this section holds the
    hybrid closure's kernels alone."""
    from workloads import configs
    inst = configs.config3(16384)
    edges = torch.from_numpy(inst.edges).cuda()
    res = cfpq.closure(inst.n, edges, inst.grammar)
    out = res.bits.view(-1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = cfpq.closure(inst.n, edges, inst.grammar, out=out)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    st = res.stats
    return {"workload": inst.tag, "ms_per_closure": round(t * 1e3, 3), "loops": st["iterations"],
            "products": st["products"], "sparse_products": st["sparse_products"],
            "delta_products": st["delta_products"]}


def bench_hybrid(cfpq, torch, inst, edges, dense_out, args, dense_s):
    """The same closure with the hybrid product choice (host-driven loop, no
    per-product events); its result must equal the dense closure's bits."""
    kw = dict(path=args.path, schedule=args.schedule, hybrid=1)
    res = cfpq.closure(inst.n, edges, inst.grammar, **kw)
    out = res.bits.view(-1)
    for _ in range(args.warmup):
        res = cfpq.closure(inst.n, edges, inst.grammar, out=out, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = cfpq.closure(inst.n, edges, inst.grammar, out=out, **kw)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    same = bool(torch.equal(out, dense_out))
    st = res.stats
    # one more closure with per-product events: the sparse products' time and
    # algorithmic bytes (rows gathered at the set bits of the sparse operand,
    # its bit scan, and the read and write of the result) give their roofline
    prof = cfpq.closure(inst.n, edges, inst.grammar, out=out, profile=True, **kw).stats
    sp_gbs = prof["sparse_bytes"] / (prof["sparse_ms"] / 1e3) / 1e9 if prof["sparse_ms"] else 0.0
    print(f"[bench] hybrid: {t * 1e3:.1f} ms per closure ({st['products'] - st['sparse_products']} dense + "
          f"{st['sparse_products']} sparse products), identical bits: {same}", file=sys.stderr, flush=True)
    return {"ms_per_closure": round(t * 1e3, 3), "speedup_vs_dense": round(dense_s / t, 2),
            "closures_per_s": round(1.0 / t, 2), "dense_products": st["products"] - st["sparse_products"],
            "sparse_products": st["sparse_products"], "loops": st["iterations"], "identical_to_dense": same,
            "roofline": {"bound": "hbm", "kernels": "sparse products (rowor_kernel, rowor_heavy_kernel, "
                                                    "transpose_or_kernel and their transposes)",
                         "achieved": round(sp_gbs, 1), "peak": 8000.0, "unit": "GB/s",
                         "frac": round(sp_gbs / 8000.0, 4), "bytes_per_closure": prof["sparse_bytes"],
                         "ms_per_closure": round(prof["sparse_ms"], 3)}}


# VALU: 256 CUs x 64 lanes per clock x 2.4 GHz integer instructions.  A
# 32-bit min-plus term needs at least 1.5 of them (one v_add_u32 per term, one
# v_min3_u32 per two terms): 26.2 T terms/s.  The narrow kernel, which the
# library runs while every length fits 14 bits (its first 14 steps: a step's
# lengths are at most twice the last one's), takes two terms per
# v_pk_add_u16 and v_pk_min_u16: one instruction per term, 39.3 T terms/s.
PEAK_VALU_INT32_T = 256 * 64 * 2.4e9 / 1e12
PEAK_MINPLUS_TERMS_T = PEAK_VALU_INT32_T / 1.5
PEAK_MINPLUS_NARROW_TERMS_T = PEAK_VALU_INT32_T
NARROW_MINPLUS_STEPS = 14


def bench_single_path(cfpq, torch, n=4096, steps=2):
    """Single-path lengths (section 5) on the ER Dyck recipe at n = 4096: time
    per closure, and the min-plus kernel's rate in (i, j, k) terms against the
    VALU roofline of the variant that ran (1.5 integer instructions per term at
    least, or one with 16-bit pairs)."""
    from workloads import configs
    inst = configs.config3(n)
    edges = torch.from_numpy(inst.edges).cuda()
    res, L = cfpq.single_path(n, edges, inst.grammar)  # warm-up and buffers
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res, L = cfpq.single_path(n, edges, inst.grammar)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    st = res.stats
    achieved = st["minplus_terms"] / (st["product_ms"] / 1e3) / 1e12 if st["product_ms"] else 0.0
    # every step of this closure ran the narrow kernel when it took at most 14
    narrow = st["iterations"] <= NARROW_MINPLUS_STEPS
    peak = PEAK_MINPLUS_NARROW_TERMS_T if narrow else PEAK_MINPLUS_TERMS_T
    print(f"[bench] single path n={n}: {t * 1e3:.1f} ms, {st['iterations']} loops, min-plus "
          f"{st['minplus_terms']:.3e} terms in {st['product_ms']:.1f} ms", file=sys.stderr, flush=True)
    return {"workload": inst.tag, "n": n, "ms_per_closure": round(t * 1e3, 3), "loops": st["iterations"],
            "minplus_terms": st["minplus_terms"], "minplus_ms": round(st["product_ms"], 3),
            "roofline": {"bound": "alu", "kernel": "minplus_kernel<true>" if narrow else "minplus_kernel<false>",
                         "achieved": round(achieved, 2), "peak": round(peak, 1),
                         "unit": ("T terms/s (16-bit add + min per (i, j, k), two per instruction)" if narrow
                                  else "T terms/s (int32 add + min per (i, j, k))"),
                         "frac": round(achieved / peak, 4)}}


def bench_conjunctive(cfpq, torch, n=8192, steps=3):
    """Conjunctive closure (Dyck conjoined with a^n b^n at the start rules) on
    the ER recipe at n = 8192 with the library's default products (fp4 MFMA,
    and ROWS for conjuncts whose left operand is an edge matrix): time per
    closure and Gbit-op/s of its dense products (2 npad^3 each)."""
    from workloads import configs, grammars
    inst = configs.config3(n)
    g = grammars.dyck_and_anbn()
    edges = torch.from_numpy(inst.edges).cuda()
    res = cfpq.conjunctive_closure(n, edges, g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = cfpq.conjunctive_closure(n, edges, g)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    st = res.stats
    print(f"[bench] conjunctive n={n}: {t * 1e3:.1f} ms, {st['iterations']} loops, {st['products']} products",
          file=sys.stderr, flush=True)
    return {"workload": f"er{n}_dyck_and_anbn", "n": n, "ms_per_closure": round(t * 1e3, 3),
            "loops": st["iterations"], "products": st["products"], "sparse_products": st["sparse_products"],
            "Gbitop_per_s": round(st["bitops"] / t / 1e9, 1)}


def bench_small_configs(cfpq, torch, reps=5):
    """The two small workloads: the two-cycle graph with a^n b^n (126 nodes,
    launch/latency bound: 8065 loops under Algorithm 1's simultaneous step,
    4033 in place) and the 4096-node hierarchy with same-generation, both
    reversed and as generated.  Median of `reps` closures each, edges on the
    device, default options (captured loops)."""
    import statistics
    from workloads import configs
    out = {}
    cases = [("two_cycles_anbn_inplace", configs.config1(), "inplace"),
             ("two_cycles_anbn_jacobi", configs.config1(), "jacobi"),
             ("hierarchy4096_samegen", configs.config2(), "inplace"),
             ("hierarchy4096_rev_samegen", configs.config2(reverse=True), "inplace")]
    for name, inst, sched in cases:
        e = torch.from_numpy(inst.edges).cuda()
        res = cfpq.closure(inst.n, e, inst.grammar, schedule=sched)
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = cfpq.closure(inst.n, e, inst.grammar, schedule=sched)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        t = statistics.median(times)
        loops = res.stats["iterations"]
        out[name] = {"n": inst.n, "ms": round(t * 1e3, 3), "loops": loops,
                     "us_per_loop": round(t * 1e6 / max(loops, 1), 2),
                     "Gbitop_per_s": round(res.stats["bitops"] / t / 1e9, 1)}
    print(f"[bench] small configs: {out}", file=sys.stderr, flush=True)
    return out


def bench_end_to_end(cfpq, torch, inst, steps=3):
    """The headline closure with host edges: the edge upload (PCIe) and its
    validation on the host are inside the timed region."""
    res = cfpq.closure(inst.n, inst.edges, inst.grammar, hybrid=0)
    out = res.bits.view(-1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = cfpq.closure(inst.n, inst.edges, inst.grammar, hybrid=0, out=out)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    return {"ms_per_closure": round(t * 1e3, 3), "Gbitop_per_s": round(res.stats["bitops"] / t / 1e9, 1),
            "edges_from": "host"}


def _pct(xs, q):
    import numpy as np
    return round(float(np.percentile(np.asarray(xs), q)), 3) if xs else None


def bench_serve(cfpq, torch, warm=100, measured=500, loads=(1.5, 0.5), hybrid_lanes=None):
    """Serving stream (sizes log-uniform in [128, 8192], hierarchy or G(n, 4n),
    a^n b^n / same-generation / Dyck), host edges as a request would bring them.
    The first `warm` requests measure the serial plain closure's service rate
    mu; the next `measured` arrive as a Poisson process at lambda = load * mu
    and are served (a) by the continuous-batching server and (b) one at a time,
    in arrival order, by the plain closure (no batching, no captured loops; the
    library's default product choice, as for any single query).  After both
    timed runs every served result is compared with the serial closure's bits
    for the same request (``results_differing_from_serial``)."""
    from workloads import configs
    insts, gaps = configs.config5(count=warm + measured)
    warm_set, meas = insts[:warm], insts[warm:]
    for i in warm_set[:5]:
        cfpq.closure(i.n, i.edges, i.grammar, capture=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in warm_set:
        cfpq.closure(i.n, i.edges, i.grammar, capture=0)
    torch.cuda.synchronize()
    mu = warm / (time.perf_counter() - t0)

    def spin_until(t):
        while True:
            d = t - time.perf_counter()
            if d <= 0:
                return
            if d > 2e-4:
                time.sleep(d - 1e-4)

    def run(load):
        lam = load * mu
        arrivals = [0.0]
        for g in gaps[warm + 1:warm + measured]:
            arrivals.append(arrivals[-1] + g / lam)
        print(f"[bench] serving: mu={mu:.1f}/s lambda={lam:.1f}/s over {measured} requests", file=sys.stderr,
              flush=True)
        # (a) server
        with cfpq.Server(hbm_budget=32 << 30, max_slots=512, capture=4, hybrid_lanes=hybrid_lanes) as srv:
            for t in [srv.submit(i.n, i.edges, i.grammar) for i in warm_set[:20]]:  # warm its code paths
                srv.wait(t)
            start = time.perf_counter()
            tickets = []
            for a, i in zip(arrivals, meas):
                spin_until(start + a)
                tickets.append(srv.submit(i.n, i.edges, i.grammar))
            infos = [srv.wait(t) for t in tickets]
            end = time.perf_counter()
        lat_srv = [x["latency_ms"] for x in infos]
        bad = sum(1 for x in infos if x["status"] != 0)
        # what the tail is made of: the server's slowest 1% of requests, and the
        # percentiles of the requests its hybrid lanes take (padded side >= 4096)
        # and of those the batched engine takes
        lane = [cfpq.padded_rows(i.n) >= 4096 for i in meas]
        slow = sorted(range(measured), key=lambda q: -lat_srv[q])[:max(1, measured // 100)]
        tail = {"slowest_1pct": [{"n": int(meas[q].n), "grammar": meas[q].grammar.name,
                                  "latency_ms": round(lat_srv[q], 3)} for q in slow],
                "lanes": {"requests": sum(lane), "p50_ms": _pct([x for x, ln in zip(lat_srv, lane) if ln], 50),
                          "p99_ms": _pct([x for x, ln in zip(lat_srv, lane) if ln], 99)},
                "engine": {"requests": measured - sum(lane),
                           "p50_ms": _pct([x for x, ln in zip(lat_srv, lane) if not ln], 50),
                           "p99_ms": _pct([x for x, ln in zip(lat_srv, lane) if not ln], 99)}}
        qps_srv = measured / (end - start)
        # (b) serial plain closure on the same trace
        start = time.perf_counter()
        lat_ser, ser = [], []
        for a, i in zip(arrivals, meas):
            spin_until(start + a)
            ser.append(cfpq.closure(i.n, i.edges, i.grammar, capture=0))
            lat_ser.append((time.perf_counter() - (start + a)) * 1e3)
        end = time.perf_counter()
        qps_ser = measured / (end - start)
        # after the timed runs: every served result against the serial closure's bits
        differ = sum(1 for x, r in zip(infos, ser) if not torch.equal(x["result"].bits, r.bits))
        del infos, ser
        print(f"[bench] server {qps_srv:.1f} q/s p50 {_pct(lat_srv, 50)} p99 {_pct(lat_srv, 99)} ms; serial "
              f"{qps_ser:.1f} q/s p50 {_pct(lat_ser, 50)} p99 {_pct(lat_ser, 99)} ms", file=sys.stderr, flush=True)
        return {"lambda_per_s": round(lam, 1), "load_vs_serial": load,
                "queries_per_s": round(qps_srv, 1), "p50_ms": _pct(lat_srv, 50), "p99_ms": _pct(lat_srv, 99),
                "serial_plain_queries_per_s": round(qps_ser, 1), "serial_plain_p50_ms": _pct(lat_ser, 50),
                "serial_plain_p99_ms": _pct(lat_ser, 99), "failed": bad,
                "results_differing_from_serial": differ, "server_tail": tail}

    out = {"workload": f"serve_seed5_{measured}req", "arrival": "poisson",
           "serial_service_rate_per_s": round(mu, 1)}
    out.update(run(loads[0]))
    for ld in loads[1:]:
        out[f"at_load_{ld}"] = run(ld)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--path", default="auto", choices=["auto", "bits", "mfma", "fp4"])
    ap.add_argument("--schedule", default="inplace", choices=["inplace", "jacobi"])
    ap.add_argument("--tile", type=int, default=0,
                    help="kernel variant of the dense path (VALU strip width; fp4: 2 or 3 pipeline stages, 5 persistent); "
                         "0 = the default or the autotuned one")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-closure section")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving section")
    ap.add_argument("--no-next", action="store_true", help="skip the single-path and conjunctive sections")
    ap.add_argument("--section", choices=["single_path", "conjunctive", "small_configs", "batch", "serving",
                                          "hybrid"],
                    help="run only this section and print its JSON object (for profiling a kernel that the "
                         "section runs; no headline line)")
    ap.add_argument("--headline-only", action="store_true",
                    help="time the dense closure only (every other section off), so that a kernel trace of "
                         "the command holds exactly the timed products")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (3 times) and exit; used to "
                         "scale the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.headline_only:
        args.no_next = args.no_batch = args.no_serve = args.no_cpu_baseline = True
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; this build runs on a single GPU "
              "(one GPU's throughput is the value)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration_mib:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "launches": 3}), flush=True)
        return

    import paper_1707_01007_amd as cfpq
    from workloads import configs

    torch.cuda.set_device(0)
    if args.section:
        fn = {"single_path": bench_single_path, "conjunctive": bench_conjunctive,
              "small_configs": bench_small_configs, "batch": bench_batch, "serving": bench_serve,
              "hybrid": bench_hybrid_only}[args.section]
        print(json.dumps({"section": args.section, args.section: fn(cfpq, torch)}), flush=True)
        return
    inst = configs.config3(args.n)
    g = inst.grammar
    edges = torch.from_numpy(inst.edges).cuda()
    tuned = cfpq.autotune(inst.n) if args.path == "auto" else None
    if tuned:
        print(f"[bench] autotune n={inst.n}: {tuned}", file=sys.stderr, flush=True)
    # Every closure here uses the same options as the timed ones: per-product
    # HIP events on the library's stream (host-driven loop, no skipped launches).
    kw = dict(path=args.path, schedule=args.schedule, profile=True, hybrid=0, tile=args.tile)
    res = cfpq.closure(inst.n, edges, g, **kw)  # sizes buffers
    out = res.bits.view(-1)
    print(f"[bench] warmup {args.warmup} x closure n={inst.n} path={args.path}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        res = cfpq.closure(inst.n, edges, g, out=out, **kw)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        res = cfpq.closure(inst.n, edges, g, out=out, **kw)
        stats.append(res.stats)
        print(f"[bench] step {k}: {res.stats['device_ms']:.1f} ms, {res.stats['iterations']} loops, "
              f"{res.stats['products']} products", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    bitops = sum(s["bitops"] for s in stats)
    products = sum(s["products"] for s in stats)
    prod_ms = sum(s["product_ms"] for s in stats)
    path_used = {1: "bits", 2: "mfma", 5: "fp4"}[stats[-1]["path_used"]]
    assert all(s["sparse_products"] == 0 for s in stats)
    npad = cfpq.padded_rows(inst.n)
    per_launch = 2.0 * npad ** 3
    achieved_t = per_launch / (prod_ms / products / 1e3) / 1e12 if products else 0.0
    if path_used in ("mfma", "fp4"):
        peak = PEAK_FP4_TOPS if path_used == "fp4" else PEAK_INT8_TOPS
        roof = {"bound": "mfma", "achieved": round(achieved_t, 1), "peak": peak, "unit": "TOP/s",
                "frac": round(achieved_t / peak, 4), "traffic": None}
    else:
        roof = {"bound": "alu", "achieved": round(achieved_t, 1), "peak": round(PEAK_VALU_BITOPS_T, 1),
                "unit": "TOP/s", "frac": round(achieved_t / PEAK_VALU_BITOPS_T, 4), "traffic": None}
    fp4_tile = args.tile or (tuned or {}).get("tile") or FP4_DEFAULT_TILE if path_used == "fp4" else 0
    roof["kernel"] = {"mfma": "mfma_product_kernel<false, 2>",
                      "fp4": fp4_kernel_name(fp4_tile)}.get(path_used, "bits_product_kernel")
    if path_used in ("mfma", "fp4"):
        roof["traffic"] = profiled_traffic(f"{path_used}_product_er16384_dyck.md", roof["kernel"],
                                           ["paper_1707_01007_amd/csrc/mfma_tile.h",
                                            "paper_1707_01007_amd/csrc/kernels_mfma.hip"])
    roof["per_launch_bitops"] = per_launch
    line = {
        "metric": METRIC,
        "value": round(bitops / wall / 1e9, 1),
        "unit": "Gbitop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mfma": "i8", "fp4": "fp4"}.get(path_used, "u32"),
        "data": "synthetic",
        "config": {"workload": inst.tag, "n": inst.n, "edges": int(len(inst.edges)), "grammar": g.name,
                   "path": path_used, "schedule": args.schedule,
                   "loops_per_closure": stats[-1]["iterations"], "products_per_closure": stats[-1]["products"],
                   "autotune": tuned},
        "roofline": roof,
    }
    if not args.headline_only:
        line["hybrid"] = bench_hybrid(cfpq, torch, inst, edges, out, args, wall / args.steps)
        line["end_to_end"] = bench_end_to_end(cfpq, torch, inst)
    if not args.no_next:
        line["small_configs"] = bench_small_configs(cfpq, torch)
    if not args.no_next:
        line["single_path"] = bench_single_path(cfpq, torch)
        line["conjunctive"] = bench_conjunctive(cfpq, torch)
    if not args.no_batch:
        line["batch"] = bench_batch(cfpq, torch)
    if not args.no_serve:
        line["serving"] = bench_serve(cfpq, torch)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfpq, torch, inst, closure_bitops=res.stats["bitops"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
