"""Benchmark of the negacyclic NTT hot path on one MI355X.

One step = one pass of the whole hot path over a batch of RNS polynomials at
N = 2^14 with 8 limbs of 50-bit primes (q = 1 mod 2N):
    acc = acc + InvNTT( NTT(a) (.) NTT(b) )   per limb: forward(a) 1->4;
                                              forward(b) 1->4 fused with the
                                              element-wise modmul (factor 4);
                                              inverse 1->1 fused with the
                                              element-wise add into acc
The reported value is forward limb-NTTs per second of whole-step throughput
(2 forward transforms per limb-product; the inverse, the multiply and the add
run inside the same timed step).  Inputs are seeded synthetic uniform
coefficients, resident in device memory before timing starts.

Also reported, on the same JSON line:
  roofline      the dominant kernel of the step (the fused per-limb product:
                forward(b), multiply, inverse, accumulate), algorithmic bytes /
                average duration (HIP events on the launch stream) against 8 TB/s,
                with the VALU issue share beside it; roofline_fwd gives the same
                for the forward transform of the other operand;
  roofline_alu  the same two kernels against the VALU's peak (the bound that
                binds them): measured VALU lane instructions per second over
                256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz;
  cpu_baseline  the CPU oracle (O(N^2) direct forward transform) on a bounded
                sample, timed on this host's cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0

# Per-launch hardware counters of the two kernels of the step (N = 2^14, 4096 limbs), from
# rocprofv3 --pmc runs of this benchmark, mean over the dispatches of each kernel:
#   fetch_kib, write_kib   FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each later scaled by the
#                          same counter's reading for a plain 1 GiB device copy (FETCH_SIZE read
#                          524300 KiB for 1048576 KiB copied: x2.0; WRITE_SIZE 1048576 KiB: x1.0);
#   valu_insts             SQ_INSTS_VALU (wave-level VALU instructions per dispatch).
# Valid only for the kernel sources they were taken with, identified by the SHA-256 of these files.
COUNTERS_N16384 = {
    "sources": ["ntt_onchip.hip", "ntt_onchip.h", "ntt_common.h", "modarith.h", "internal.h", "ntt_kernels.hip"],
    "sha256": "081aafeb2850f1786c03544fc47790fbf1888847fb7cf0b76e47424e4560a928",
    "fetch_scale": 2.0, "write_scale": 1.0,
    "product": {"fetch_kib": 886963.8, "write_kib": 540672.0, "valu_insts": 394428416},
    "forward": {"fetch_kib": 294642.5, "write_kib": 581632.0, "valu_insts": 145195008},
}

# VALU issue capacity: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4 cycles at 2.4 GHz
VALU_WAVE_INSTS_PER_S = 256 * 4 * 2.4e9 / 4
# the same capacity in 32-bit lane operations: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (39.3 T/s)
VALU_LANE_OPS_PER_S = 256 * 4 * 16 * 2.4e9


def counters_valid(c):
    """True while the kernel sources are the ones the stored counters were taken with."""
    import hashlib
    h = hashlib.sha256()
    for f in c["sources"]:
        with open(os.path.join(ROOT, "paper_2103_16400_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest() == c["sha256"]


def measured_traffic(c, kernel):
    """HBM bytes per launch from the stored counters, or None once the kernel sources changed."""
    k = c[kernel]
    if not counters_valid(c) or k["fetch_kib"] is None:
        return None
    return int((k["fetch_kib"] * c["fetch_scale"] + k["write_kib"] * c["write_scale"]) * 1024)


def alu_roofline(c, kernel, avg_ms, desc):
    """The kernel against the VALU's peak: its measured VALU lane instructions (SQ_INSTS_VALU x 64)
    per second over 39.3 T lane-ops/s; None once the kernel sources changed."""
    k = c[kernel]
    if not counters_valid(c) or k["valu_insts"] is None:
        return None
    a = k["valu_insts"] * 64 / (avg_ms * 1e-3)
    return {"bound": "alu", "achieved": round(a / 1e12, 3), "peak": round(VALU_LANE_OPS_PER_S / 1e12, 3),
            "unit": "T lane-op/s", "frac": round(a / VALU_LANE_OPS_PER_S, 4), "kernel": desc,
            "avg_ms": round(avg_ms, 4), "valu_lane_ops": k["valu_insts"] * 64,
            "source": "SQ_INSTS_VALU per launch (rocprofv3 --pmc) x 64 lanes"}


def valu_share(c, kernel, avg_ms):
    """Fraction of the chip's VALU issue slots the kernel's instructions fill over its duration."""
    k = c[kernel]
    if not counters_valid(c) or k["valu_insts"] is None:
        return None
    return round(k["valu_insts"] / (avg_ms * 1e-3 * VALU_WAVE_INSTS_PER_S), 4)


def load_primes():
    with open(os.path.join(ROOT, "tests", "golden", "primes.json")) as f:
        return json.load(f)


def gen_operand(tag, N, moduli, B):
    from synthetic import uniform_mod, unit_seed
    L = len(moduli)
    out = np.empty(B * L * N, dtype=np.uint64)
    for p in range(B):
        for l, q in enumerate(moduli):
            out[(p * L + l) * N:(p * L + l + 1) * N] = uniform_mod(unit_seed(tag, p, l, q), N, q)
    return out


def cpu_baseline(N, moduli, psis, budget_s=12.0):
    """Oracle forward transform (O(N^2) direct sums) over a bounded sample of limbs."""
    import oracle
    from synthetic import uniform_mod, unit_seed
    threads = max(1, min(os.cpu_count() or 1, 16))
    done, t0 = 0, time.perf_counter()
    while True:
        l = done % len(moduli)
        a = uniform_mod(unit_seed(7, done, moduli[l]), N, moduli[l])
        oracle.ntt_forward(a, moduli[l], psis[l], threads=threads)
        done += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return {"value": done / el, "unit": "NTT/s", "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": "%d limb forward transforms (N=%d, first %d of the 8 primes), O(N^2) direct "
                      "definition, %d threads, %.1f s" % (done, N, min(done, len(moduli)), threads, el)}


def time_large_ring(nt, torch, primes, reps=20, batches=(1, 2, 8)):
    """Forward and inverse NTT of 32-limb polynomials at N = 2^16 (60-bit primes), one
    launch sequence per batch of B polynomials, rotating over 16 distinct polynomials
    (256 MiB) so coefficients come from HBM rather than the 256 MB MALL.  Out of place, into
    an output pool of the same size, so every call reads canonical inputs (factor 1) and
    its writes rotate through HBM as well."""
    p3 = primes["large_65536"]
    N, moduli = p3["N"], p3["moduli"]
    L = len(moduli)
    pool = 16
    dev = torch.device("cuda:0")
    data = torch.from_numpy(gen_operand(3, N, moduli, pool).view(np.int64)).to(dev)
    dst = torch.empty_like(data)
    stream = torch.cuda.current_stream()
    out = {}
    for B in batches:
        views = [(data[i * L * N:(i + B) * L * N], dst[i * L * N:(i + B) * L * N])
                 for i in range(0, pool - B + 1, B)]
        res = {}
        res["autotune_variant_fwd_inv"] = list(nt.autotune(N, moduli, B, stream=stream))
        for name, fn in (("fwd", lambda v: nt.ntt_forward_rns(v[1], v[0], N, moduli, B, 1, 4, stream=stream)),
                         ("fwd_canon", lambda v: nt.ntt_forward_rns(v[1], v[0], N, moduli, B, 1, 1, stream=stream)),
                         ("inv", lambda v: nt.ntt_inverse_rns(v[1], v[0], N, moduli, B, 1, 2, stream=stream))):
            for v in views[:2]:
                fn(v)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for r in range(reps):
                fn(views[r % len(views)])
            e1.record(stream)
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / reps
            alg = B * 16 * N * L + 16 * N * L          # coefficients read+written + one table per prime
            res[name + "_us"] = round(us, 2)
            res[name + "_hbm_frac"] = round(alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
        res["limb_ntts_per_s_fwd"] = round(B * L / (res["fwd_us"] * 1e-6), 1)
        out["B%d" % B] = res
    out["alg_bytes_B1"] = 16 * N * L + 16 * N * L
    return out


def time_uneven_batch(nt, torch, primes, reps=10):
    """256 RNS polynomials, N uniform in {2^12..2^15}, limb counts uniform in [2, 16], 50-bit
    primes (limb l uses the l-th prime of the pool): forward (1 -> 4) and inverse (1 -> 1) of
    every limb as one persistent launch (plain and hipGraph-replayed, grid autotuned) versus
    one launch per limb-transform."""
    from synthetic import uniform_int, uniform_mod, unit_seed
    pool = primes["uneven"]["moduli"]
    P = 256
    logNs = uniform_int(unit_seed(4, 0), P, 12, 15)
    Ls = uniform_int(unit_seed(4, 1), P, 2, 16)
    dev = torch.device("cuda:0")
    limbs = [(int(logNs[p]), pool[l]) for p in range(P) for l in range(int(Ls[p]))]
    total = sum(1 << n for n, _ in limbs)
    src = torch.empty(total, dtype=torch.int64, device=dev)
    dst = torch.empty(total, dtype=torch.int64, device=dev)
    off, views = 0, []
    host = np.empty(total, dtype=np.uint64)
    for k, (n, q) in enumerate(limbs):
        N = 1 << n
        host[off:off + N] = uniform_mod(unit_seed(5, k, q), N, q)
        views.append((src[off:off + N], dst[off:off + N], N, q))
        off += N
    src.copy_(torch.from_numpy(host.view(np.int64)))
    stream = torch.cuda.current_stream()
    batch = nt.Batch(len(limbs))
    res = {"limbs": len(limbs), "coefficients": total}
    plans = {(N, q) for _, _, N, q in views}
    alg = 16 * total + 16 * sum(N for N, _ in plans)
    for name, op in (("fwd", nt.BATCH_FWD_LAZY), ("inv", nt.BATCH_INV)):
        items, cnt = nt.Batch.make_items([(op, d, s_, None, None, N, q) for s_, d, N, q in views])
        res[name + "_grid"] = batch.autotune(items, cnt, stream=stream)
        res[name + "_shape"] = batch.config()[1]
        for mode in ("batched", "graph"):
            batch.run(items, cnt, stream=stream, graph=(mode == "graph"))
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                batch.run(items, cnt, stream=stream, graph=(mode == "graph"))
            e1.record(stream)
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / reps
            res["%s_%s_us" % (name, mode)] = round(us, 1)
            res["%s_%s_limb_ntts_per_s" % (name, mode)] = round(len(limbs) / (us * 1e-6), 1)
            res["%s_%s_hbm_frac" % (name, mode)] = round(alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
        # plain form: one launch per limb-transform
        fn = (lambda s_, d, N, q: nt.ntt_forward(d, s_, N, q, 1, 4, stream=stream)) if name == "fwd" else \
             (lambda s_, d, N, q: nt.ntt_inverse(d, s_, N, q, 1, 1, stream=stream))
        for v in views:
            fn(*v)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for v in views:
            fn(*v)
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3
        res["%s_per_call_us" % name] = round(us, 1)
        res["%s_per_call_limb_ntts_per_s" % name] = round(len(limbs) / (us * 1e-6), 1)
    batch.close()
    return res


def time_batch_one_size(nt, torch, primes, logN, polys=320, reps=10):
    """5120 limbs of one ring degree (320 polynomials x the 16 primes of the uneven pool), forward
    1 -> 4: the persistent batch (plain launches, grid of two workgroups per CU; unit shape 0,
    then 1) against one
    `ntt_forward_rns` launch over the same limbs.  Event-timed calls include the host's
    preparation of each batch; a kernel trace of this mode gives the kernels' own durations."""
    from synthetic import uniform_mod, unit_seed
    pool = primes["uneven"]["moduli"][:16]
    N, L = 1 << logN, len(pool)
    dev = torch.device("cuda:0")
    host = np.concatenate([uniform_mod(unit_seed(7, p, l), N, pool[l]) for p in range(polys) for l in range(L)])
    src = torch.from_numpy(host.view(np.int64)).to(dev)
    dst = torch.empty_like(src)
    items, cnt = nt.Batch.make_items([(nt.BATCH_FWD_LAZY, dst[k * N:(k + 1) * N], src[k * N:(k + 1) * N], None,
                                       None, N, pool[k % L]) for k in range(polys * L)])
    batch = nt.Batch(polys * L)
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return round(e0.elapsed_time(e1) * 1e3 / reps, 1)
    res = {"logN": logN, "limbs": polys * L,
           "batch_us": timed(lambda: batch.run(items, cnt, stream=stream))}
    batch.set_shape(1)
    res["batch_shape1_us"] = timed(lambda: batch.run(items, cnt, stream=stream))
    res["rns_us"] = timed(lambda: nt.ntt_forward_rns(dst, src, N, pool, polys, 1, 4, stream=stream))
    batch.close()
    return res


SERVE_RATES = (1000, 2000, 5000, 10000, 20000, 30000, 40000, 50000)


class OperandPool:
    """Resident operands for the serving stream: for every N in 2^12..2^17, `per_n` pairs of
    [40][N] arrays whose limb l is uniform in [0, q_l) for the l-th prime of the 40-prime serving
    pool; a request with L limbs reads the first L*N words (contiguous [L][N])."""

    def __init__(self, torch, moduli, per_n=2):
        from synthetic import uniform_mod, unit_seed
        self.bufs = {}
        dev = torch.device("cuda:0")
        for logN in range(12, 18):
            N = 1 << logN
            for p in range(per_n):
                for op in range(2):
                    h = np.empty(len(moduli) * N, dtype=np.uint64)
                    for l, q in enumerate(moduli):
                        h[l * N:(l + 1) * N] = uniform_mod(unit_seed(6, logN, p, op, l), N, q)
                    self.bufs[(logN, p, op)] = torch.from_numpy(h.view(np.int64)).to(dev)
        self.per_n = per_n

    def pick(self, logN, k):
        p = k % self.per_n
        return self.bufs[(logN, p, 0)], self.bufs[(logN, p, 1)]


def serve_schedule(rate, n):
    """n requests of a Poisson stream at `rate` req/s: N uniform in {2^12..2^17}, L uniform in [1, 40]."""
    from synthetic import exponential, uniform_int, unit_seed
    gaps = exponential(unit_seed(7, rate, 0), n, 1e9 / rate)
    offs = np.cumsum(gaps).astype(np.int64)
    logNs = uniform_int(unit_seed(7, rate, 1), n, 12, 17)
    Ls = uniform_int(unit_seed(7, rate, 2), n, 1, 40)
    return offs, logNs, Ls


def run_served(nt, pool, moduli, mode, rate, n, streams=2, wide_min=0, wide_max=0):
    """One open-loop run; latency = completion seen by the scheduler - scheduled arrival."""
    offs, logNs, Ls = serve_schedule(rate, n)
    srv = nt.Server(mode=mode, streams=streams, release_on_completion=True, wide_min_log_degree=wide_min,
                    wide_max_inflight=wide_max)
    for logN in range(12, 18):                   # warm-up: plans of every (N, q) and the kernels
        a, b = pool.pick(logN, 0)
        srv.submit(a, b, 1 << logN, moduli)
    srv.drain(timeout_s=60)
    t0 = nt.now_ns() + 30_000_000 + n * 40_000   # every request is handed over before the first arrival
    tickets = [srv.submit(*pool.pick(int(logNs[k]), k), 1 << int(logNs[k]), moduli[:int(Ls[k])],
                          arrival_ns=t0 + int(offs[k])) for k in range(n)]
    late = nt.now_ns() - t0
    srv.drain(timeout_s=600)
    infos = srv.query(tickets)
    st = srv.stats()
    srv.close()
    lat = np.array([i.done_ns - i.arrival_ns for i in infos], dtype=np.float64) / 1e6
    end = max(i.done_ns for i in infos)
    ok = all(i.state == nt.REQ_DONE for i in infos)
    return {"rate": rate, "requests": n, "ok": ok, "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3), "mean_ms": round(float(lat.mean()), 3),
            "throughput_rps": round(n / ((end - t0) / 1e9), 1),
            "limb_products_per_s": round(float(Ls.sum()) / ((end - t0) / 1e9), 1),
            "launches": st["launches"], "tasks_per_launch": round(st["tasks"] / max(1, st["launches"]), 1),
            "submit_margin_ms": round(-late / 1e6, 1)}


def time_serving(nt, torch, primes, rates=SERVE_RATES, max_requests=20000, seconds=2.0,
                 modes=("batched", "batched_persistent_only", "fifo", "fifo_per_limb")):
    """Open-loop sweep over arrival rates for each serving form: min(max_requests, rate x seconds)
    requests per rate, so 20k requests from 10k req/s up; the per-limb FIFO form (about 900
    req/s at best) is swept only up to 5k req/s with at most 2000 requests, where it is already
    saturated."""
    moduli = primes["serving"]["moduli"]
    pool = OperandPool(torch, moduli)
    code = {"batched": (nt.SERVE_BATCHED, 0, 0), "batched_persistent_only": (nt.SERVE_BATCHED, 18, 0),
            "fifo": (nt.SERVE_FIFO, 0, 0), "fifo_per_limb": (nt.SERVE_FIFO_PER_LIMB, 0, 0)}
    for m in modes:
        if m.startswith("batched_cap"):
            code[m] = (nt.SERVE_BATCHED, 0, int(m[len("batched_cap"):]))
    res = {"workload": "Poisson stream of negacyclic products, N ~ U{2^12..2^17}, L ~ U[1,40] "
                       "(50-60-bit primes), operands resident",
           "requests_per_rate": "min(%d, rate x %.1f s)" % (max_requests, seconds)}
    for m in modes:
        runs = []
        for r in rates:
            if m == "fifo_per_limb" and r > 5000:
                continue
            n = int(min(max_requests if m != "fifo_per_limb" else 2000, r * seconds))
            runs.append(run_served(nt, pool, moduli, code[m][0], r, n, wide_min=code[m][1], wide_max=code[m][2]))
            print("serve %s rate %d: p50 %.2f ms p99 %.2f ms, %.0f req/s" %
                  (m, r, runs[-1]["p50_ms"], runs[-1]["p99_ms"], runs[-1]["throughput_rps"]), file=sys.stderr,
                  flush=True)
        ok10 = [x["rate"] for x in runs if x["p99_ms"] <= 10.0 and x["throughput_rps"] >= 0.9 * x["rate"]]
        res[m] = {"runs": runs, "max_rate_p99_le_10ms": max(ok10) if ok10 else None}
    del pool
    torch.cuda.empty_cache()
    return res


def time_small_primes(nt, torch, primes, key="small_16384", B=512, steps=100, warmup=30):
    """The step of the headline (forward of a, then the fused product into acc) at word size
    2^32: N = 2^14 or 2^15 (on chip) or 2^16 (two passes per transform), 8 limbs of primes
    below 2^30, 4-byte coefficients."""
    p = primes[key]
    N, moduli = p["N"], p["moduli"]
    L = len(moduli)
    dev = torch.device("cuda:0")
    a = torch.from_numpy(gen_operand(11, N, moduli, B).astype(np.uint32).view(np.int32)).to(dev)
    b = torch.from_numpy(gen_operand(12, N, moduli, B).astype(np.uint32).view(np.int32)).to(dev)
    c = torch.empty_like(a)
    acc = torch.zeros_like(a)
    ws = torch.empty_like(a) if N > (1 << 15) else None
    stream = torch.cuda.current_stream()
    ev = []

    def step(record):
        es = [torch.cuda.Event(enable_timing=True) for _ in range(3)] if record else None
        if record:
            es[0].record(stream)
        nt.ntt_forward_rns32(c, a, N, moduli, B, 1, 4, stream=stream)
        if record:
            es[1].record(stream)
        nt.poly_mul_acc_ntt_rns32(acc, c, b, N, moduli, B, ws, stream=stream)
        if record:
            es[2].record(stream)
            ev.append(es)

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    fwd_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    prod_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    limbs = B * L
    fwd_bytes = 8 * N * limbs + 16 * N * L         # 4-byte coefficients read + written; 16-byte twiddle pairs
    prod_bytes = 16 * N * limbs + 32 * N * L       # b, NTT(a), acc read, acc written; both directions' pairs
    return {"N": N, "limbs": L, "polys": B, "moduli_bits": 30, "word_bits": 32,
            "forward_ntts_per_s": round(2 * limbs / wall, 1), "ms_per_step": round(wall * 1e3, 4),
            "fwd_lazy_ms": round(fwd_ms, 4), "fwd_hbm_frac": round(fwd_bytes / (fwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "product_ms": round(prod_ms, 4),
            "product_hbm_frac": round(prod_bytes / (prod_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "fwd_limb_ntts_per_s": round(limbs / (fwd_ms * 1e-3), 1)}


def time_plain_step(nt, torch, a, b, N, moduli, B, reps=2):
    """The headline step in the plain per-call form: for every limb, forward(a) 1 -> 4,
    forward(b) 1 -> 4, the element-wise multiply (input factor 4) and the inverse 1 -> 1, each
    its own launch on one stream (4 launches per limb), then the add into acc."""
    L = len(moduli)
    stream = torch.cuda.current_stream()
    fa, fb = torch.empty_like(a), torch.empty_like(a)
    acc = torch.zeros_like(a)

    views = []
    for p in range(B):
        for l, q in enumerate(moduli):
            s = slice((p * L + l) * N, (p * L + l + 1) * N)
            views.append((q, a[s], b[s], fa[s], fb[s], acc[s]))

    def step():
        for q, av, bv, fav, fbv, accv in views:
            nt.ntt_forward(fav, av, N, q, 1, 4, stream=stream)
            nt.ntt_forward(fbv, bv, N, q, 1, 4, stream=stream)
            nt.eltwise_mult_mod(fav, fav, fbv, N, q, 4, stream=stream)
            nt.ntt_inverse(fav, fav, N, q, 1, 1, stream=stream)
            nt.eltwise_add_mod(accv, accv, fav, N, q, stream=stream)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    return {"form": "one launch per limb-transform and per element-wise op (5 per limb), one stream",
            "ms_per_step": round(ms, 2), "forward_ntts_per_s": round(2 * B * L / (ms * 1e-3), 1),
            "launches_per_step": 5 * B * L}


def time_eltwise(nt, torch, a, b, N, moduli, B, reps=20):
    """eltwise_mult_mod (input factor 1) and eltwise_add_mod over the headline's arrays
    (B x 8 limbs of N = 2^14): 24 algorithmic bytes per element (two reads, one write)."""
    stream = torch.cuda.current_stream()
    c = torch.empty_like(a)
    n = a.numel()
    out = {}
    for name, fn in (("eltwise_mult_mod", lambda: nt.eltwise_mult_mod_rns(c, a, b, N, moduli, B, 1, stream=stream)),
                     ("eltwise_add_mod", lambda: nt.eltwise_add_mod_rns(c, a, b, N, moduli, B, stream=stream))):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = 24 * n / (ms * 1e-3) / 1e9
        out[name] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "avg_ms": round(ms, 4), "elements": n,
                     "alg_bytes": 24 * n}
    del c
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def time_copy(torch, words=1 << 27, reps=10):
    """Achieved streaming rate of a plain 1 GiB device-to-device copy (bytes read + written / time):
    the practical HBM ceiling beside the 8 TB/s peak."""
    src = torch.ones(words, dtype=torch.int64, device="cuda:0")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2 * words * 8 / (ms * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes_moved": 2 * words * 8, "ms": round(ms, 4), "gbs": round(gbs, 1),
            "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}


def time_single_1024(nt, torch, primes, reps=200):
    """Per-call latency of one forward and one inverse NTT at N = 1024 (single limb)."""
    p1 = primes["single_1024"]
    N, q = p1["N"], p1["moduli"][0]
    from synthetic import uniform_mod, unit_seed
    dev = torch.device("cuda:0")
    a = torch.from_numpy(uniform_mod(unit_seed(1, 1), N, q).view(np.int64)).to(dev)
    o = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    res = {}
    for name, fn in (("fwd", lambda: nt.ntt_forward(o, a, N, q, 1, 1, stream=stream)),
                     ("inv", lambda: nt.ntt_inverse(o, a, N, q, 1, 1, stream=stream))):
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        res[name + "_us_per_call"] = round(e0.elapsed_time(e1) * 1e3 / reps, 3)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the chip's clocks settle within about 20 steps; the timing protocol asks for at least
    # 10 warm-up launches and 100 timed iterations
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--polys", type=int, default=512, help="RNS polynomials per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary measurements")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving sweep")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving sweep (full size)")
    ap.add_argument("--serve-requests", type=int, default=20000, help="cap on requests per arrival rate")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="arrival window per rate")
    ap.add_argument("--serve-modes", default="batched,batched_persistent_only,fifo,fifo_per_limb",
                    help="comma-separated serving forms (batched_capK: batched with K wide launches per stream)")
    ap.add_argument("--large-ring-only", type=int, default=0, metavar="B",
                    help="only time the N = 2^16 x 32-limb forward and inverse at B polynomials per launch "
                         "(for profiling the two-pass kernels)")
    ap.add_argument("--uneven-only", action="store_true",
                    help="only time the uneven batch (256 polynomials, N in 2^12..2^15) as one persistent launch")
    ap.add_argument("--batch-one-size", type=int, default=0, metavar="LOGN",
                    help="only time a batch of 5120 limbs of N = 2^LOGN against the per-size kernels")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 4 times (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; the path shards over GPUs by limbs "
              "with no exchange, but no multi-GPU run is part of it (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2103_16400_amd as nt

    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.int64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_dispatch": src.numel() * 8}), flush=True)
        return

    if args.large_ring_only:
        print(json.dumps({"large_ring_n65536_l32": time_large_ring(nt, torch, load_primes(),
                                                                   batches=(args.large_ring_only,))}), flush=True)
        return

    if args.uneven_only:
        print(json.dumps({"uneven_batch_256polys": time_uneven_batch(nt, torch, load_primes())}), flush=True)
        return

    if args.batch_one_size:
        print(json.dumps({"batch_one_size": time_batch_one_size(nt, torch, load_primes(), args.batch_one_size)}),
              flush=True)
        return

    if args.serve_only:
        print(json.dumps({"serving": time_serving(nt, torch, load_primes(), max_requests=args.serve_requests,
                                                  seconds=args.serve_seconds,
                                                  modes=tuple(args.serve_modes.split(",")))}), flush=True)
        return

    primes = load_primes()["rns_16384"]
    N, moduli, psis = primes["N"], primes["moduli"], primes["psi"]
    L, B = len(moduli), args.polys
    dev = torch.device("cuda:0")

    def up(x):
        return torch.from_numpy(x.view(np.int64)).to(dev)

    a = up(gen_operand(1, N, moduli, B))
    b = up(gen_operand(2, N, moduli, B))
    c = torch.empty_like(a)
    ws = torch.empty_like(a)
    acc = torch.zeros_like(a)
    stream = torch.cuda.current_stream()

    ev = []

    def step(record):
        if record:
            es = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            es[0].record(stream)
        nt.ntt_forward_rns(c, a, N, moduli, B, 1, 4, stream=stream)             # c = NTT(a), lazy [0, 4q)
        if record:
            es[1].record(stream)
        # acc += InvNTT(NTT(b) (.) c): one launch, each limb kept on chip
        nt.poly_mul_acc_ntt_rns(acc, c, b, N, moduli, B, ws, stream=stream)
        if record:
            es[2].record(stream)
            ev.append(es)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    fwd_all = np.array([es[0].elapsed_time(es[1]) for es in ev])
    prod_all = np.array([es[1].elapsed_time(es[2]) for es in ev])
    step_all = np.array([es[0].elapsed_time(es[2]) for es in ev])
    fwd_ms = float(fwd_all.mean())
    prod_ms = float(prod_all.mean())

    def pct(x):
        return [round(float(v), 4) for v in np.percentile(x, [10, 50, 90])]

    limbs = B * L
    fwd_per_step = 2 * limbs
    value = fwd_per_step / (wall / args.steps)
    # forward: coefficients read + written, one direction's twiddle pairs per prime
    fwd_bytes = 16 * N * limbs + 16 * N * L
    # product: b, NTT(a), acc read and acc written; both directions' twiddle pairs per prime
    prod_bytes = 32 * N * limbs + 32 * N * L
    counted = (N, limbs) == (16384, 4096)

    def roof(kernel, desc, alg, ms):
        a = alg / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": round(a, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(a / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(COUNTERS_N16384, kernel) if counted else None,
                "kernel": desc, "avg_ms": round(ms, 4), "alg_bytes": alg,
                "valu_issue_frac": valu_share(COUNTERS_N16384, kernel, ms) if counted else None}

    out = {
        "metric": "forward NTTs/s at N=2^14 (RNS product pipeline, 8 x 50-bit limbs)",
        "value": round(value, 1),
        "unit": "NTT/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "rns_product_n16384_l8", "N": N, "limbs": L, "polys_per_step": B,
                   "step": "fwd(a) 1->4; then per limb on chip: fwd(b) 1->4, modmul f=4, inv 1->1, acc add",
                   "forward_ntts_per_step": fwd_per_step},
        "roofline": roof("product", "ntt_onchip_product_kernel<N=2^14>: per limb forward(b), multiply, "
                         "inverse, accumulate; %d limbs, one launch" % limbs, prod_bytes, prod_ms),
        "roofline_fwd": roof("forward", "ntt_onchip_kernel<fwd, N=2^14>: forward NTT of %d limbs, one launch"
                             % limbs, fwd_bytes, fwd_ms),
        "roofline_alu": alu_roofline(COUNTERS_N16384, "product", prod_ms,
                                     "ntt_onchip_product_kernel<N=2^14> (the binding bound of the dominant kernel)")
        if counted else None,
        "roofline_alu_fwd": alu_roofline(COUNTERS_N16384, "forward", fwd_ms, "ntt_onchip_kernel<fwd, N=2^14>")
        if counted else None,
        "step_kernels_ms": {"fwd_lazy": round(fwd_ms, 4), "fwd_mul_inv_acc_fused": round(prod_ms, 4)},
        "p10_p50_p90_ms": {"step_events": pct(step_all), "fwd_lazy": pct(fwd_all),
                           "fwd_mul_inv_acc_fused": pct(prod_all)},
        "fwd_ntt_rate": round(limbs / (fwd_ms * 1e-3), 1),
        "products_per_s": round(limbs / (wall / args.steps), 1),
    }
    if not args.no_extra:
        out["eltwise_n16384_l8x%d" % B] = time_eltwise(nt, torch, a, b, N, moduli, B)
        out["plain_per_call_step"] = time_plain_step(nt, torch, a, b, N, moduli, B)
        del a, b, c, ws, acc
        torch.cuda.empty_cache()
        out["hbm_copy"] = time_copy(torch)
        out["large_ring_n65536_l32"] = time_large_ring(nt, torch, load_primes())
        out["single_n1024"] = time_single_1024(nt, torch, load_primes())
        out["small_primes_n16384_l8"] = time_small_primes(nt, torch, load_primes())
        out["small_primes_n32768_l8"] = time_small_primes(nt, torch, load_primes(), "small_32768", B=256)
        out["small_primes_n65536_l8"] = time_small_primes(nt, torch, load_primes(), "small_65536", B=128)
        out["uneven_batch_256polys"] = time_uneven_batch(nt, torch, load_primes())
        if not args.no_serve:
            out["serving"] = time_serving(nt, torch, load_primes(), max_requests=args.serve_requests,
                                          seconds=args.serve_seconds, modes=tuple(args.serve_modes.split(",")))
    out["summary"] = summary(out)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(N, moduli, psis, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def summary(out):
    """The secondary figures in one short object near the end of the line, where a reader of the
    output's tail sees them: the forward-only batched launch and its roofline, the plain
    per-call step, the large ring against its 50%-of-HBM target, the uneven batch, the word-size
    2^32 steps, the element-wise rooflines and the serving forms' best rates at p99 <= 10 ms."""
    s = {"forward_only_launch": {"limb_ntts_per_s": out.get("fwd_ntt_rate"),
                                 "hbm_frac": (out.get("roofline_fwd") or {}).get("frac"),
                                 "avg_ms": (out.get("roofline_fwd") or {}).get("avg_ms")}}
    if "plain_per_call_step" in out:
        p = out["plain_per_call_step"]
        s["plain_per_call_step"] = {"ms_per_step": p["ms_per_step"], "forward_ntts_per_s": p["forward_ntts_per_s"],
                                    "batched_step_speedup": round(p["ms_per_step"] / out["ms_per_step"], 1)}
    lr = out.get("large_ring_n65536_l32")
    if lr:
        s["large_ring_n65536_l32"] = {k: {"fwd_us_per_launch": v["fwd_us"], "fwd_hbm_frac": v["fwd_hbm_frac"],
                                          "inv_us_per_launch": v["inv_us"]}
                                      for k, v in lr.items() if k.startswith("B")}
        s["large_ring_n65536_l32"]["target"] = "B1 forward <= 16.8 us (0.50 of 8 TB/s on 64 MiB)"
    ub = out.get("uneven_batch_256polys")
    if ub:
        s["uneven_batch_256polys"] = {k: ub[k] for k in ("fwd_batched_us", "fwd_graph_us", "fwd_batched_hbm_frac",
                                                         "fwd_per_call_us", "inv_batched_us") if k in ub}
    for k in ("small_primes_n16384_l8", "small_primes_n32768_l8", "small_primes_n65536_l8"):
        if k in out:
            s[k] = {"forward_ntts_per_s": out[k]["forward_ntts_per_s"], "ms_per_step": out[k]["ms_per_step"]}
    e = [k for k in out if k.startswith("eltwise_")]
    if e:
        s["eltwise"] = {n: {"frac": v["frac"], "achieved_gbs": v["achieved"]} for n, v in out[e[0]].items()}
    sv = out.get("serving")
    if sv:
        s["serving_max_rate_p99_le_10ms"] = {m: v["max_rate_p99_le_10ms"] for m, v in sv.items() if isinstance(v, dict)}
    return s


if __name__ == "__main__":
    main()
