"""GPU tests of the continuous-batching server (ntt_server_* in include/ntt_hip.h).

Each request is the negacyclic product a * b mod (X^N + 1, q_l) per limb (the
Section 4 product listing; limbs independent, Section 5).  A result must be the
same word for word whether the request ran alone or in a mix, in every serving
mode, and equal to the oracle's schoolbook product (in full for small N, at
sampled coefficients for large N)."""
import json
import os
import time

import numpy as np
import pytest

import oracle
from synthetic import uniform_int, uniform_mod, unit_seed
from gpu_util import empty_dev, from_dev, have_gpu, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a ROCm GPU")]

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PRIMES = json.load(open(os.path.join(ROOT, "tests", "golden", "primes.json")))
POOL = PRIMES["serving"]["moduli"]          # 40 primes = 1 mod 2^18, 50..60 bits


@pytest.fixture(scope="module")
def nt():
    import paper_2103_16400_amd as nt
    return nt


def _request(seed, logN, L):
    N = 1 << logN
    mods = POOL[:L]
    a = np.concatenate([uniform_mod(unit_seed(seed, 0, l), N, q) for l, q in enumerate(mods)]).astype(np.uint64)
    b = np.concatenate([uniform_mod(unit_seed(seed, 1, l), N, q) for l, q in enumerate(mods)]).astype(np.uint64)
    return {"N": N, "mods": mods, "a": a, "b": b, "da": to_dev(a), "db": to_dev(b)}


def _mix(seed, count):
    logNs = uniform_int(unit_seed(seed, 0), count, 10, 17)
    Ls = uniform_int(unit_seed(seed, 1), count, 1, 6)
    return [_request(unit_seed(seed, 2, k), int(logNs[k]), int(Ls[k])) for k in range(count)]


def _alone(nt, r):
    """The product of one request through poly_mul_rns (no server)."""
    N, L = r["N"], len(r["mods"])
    out = empty_dev(N * L)
    ws = empty_dev(N * L) if N > (1 << 14) else None
    nt.poly_mul_rns(out, r["da"], r["db"], N, r["mods"], 1, ws)
    return from_dev(out)


def _oracle_check(r, got, seed):
    N = r["N"]
    for l, q in enumerate(r["mods"]):
        a = r["a"][l * N:(l + 1) * N]
        b = r["b"][l * N:(l + 1) * N]
        g = got[l * N:(l + 1) * N]
        if N <= 2048:
            assert np.array_equal(g, oracle.negacyclic_mul(a, b, q)), (N, l)
        elif l in (0, len(r["mods"]) - 1):
            idx = np.unique(np.concatenate([uniform_mod(unit_seed(seed, l, N), 6, N).astype(np.uint64),
                                            np.array([0, N - 1], dtype=np.uint64)]))
            assert np.array_equal(g[idx], oracle.negacyclic_mul_at(a, b, idx, q)), (N, l)


def _serve(nt, reqs, mode, stagger_us=0, **kw):
    srv = nt.Server(mode=mode, **kw)
    t0 = nt.now_ns() + 1_000_000
    tickets = [srv.submit(r["da"], r["db"], r["N"], r["mods"], arrival_ns=t0 + k * stagger_us * 1000 if stagger_us else 0)
               for k, r in enumerate(reqs)]
    srv.drain(timeout_s=120)
    outs = []
    for t, r in zip(tickets, reqs):
        info = srv.poll(t)
        assert info.state == nt.REQ_DONE and info.status == 0
        assert info.done_ns >= info.launch_ns >= info.admit_ns >= info.arrival_ns
        dst = empty_dev(r["N"] * len(r["mods"]))
        srv.read(t, dst)
        outs.append(from_dev(dst))
        srv.release(t)
    _settle(srv)
    st = srv.stats()
    srv.close()
    return outs, st


def _settle(srv, timeout_s=10.0):
    """Released ranges that were read return to the arena once the copies have run, which the
    scheduler observes shortly after: wait for that."""
    deadline = time.time() + timeout_s
    while srv.stats()["arena_in_use"] and time.time() < deadline:
        time.sleep(0.005)


def test_server_mix_matches_alone_and_oracle(nt):
    reqs = _mix(300, 24)
    print("server mix:", [(r["N"], len(r["mods"])) for r in reqs], flush=True)
    outs, st = _serve(nt, reqs, nt.SERVE_BATCHED, stagger_us=150)
    assert st["completed"] == len(reqs) and st["failed"] == 0 and st["arena_in_use"] == 0
    for k, (r, got) in enumerate(zip(reqs, outs)):
        assert np.array_equal(got, _alone(nt, r)), k
        _oracle_check(r, got, 301 + k)
    # one request of the mix served alone gives the same words
    solo, _ = _serve(nt, [reqs[3]], nt.SERVE_BATCHED)
    assert np.array_equal(solo[0], outs[3])


@pytest.mark.parametrize("mode", ["fifo", "per_limb", "graph", "persistent_only", "all_wide"])
def test_server_modes_agree(nt, mode):
    reqs = _mix(310, 10)
    ref, _ = _serve(nt, reqs, nt.SERVE_BATCHED)
    if mode == "graph":
        got, st = _serve(nt, reqs, nt.SERVE_BATCHED, use_graph=True, streams=3)
    elif mode == "persistent_only":
        got, st = _serve(nt, reqs, nt.SERVE_BATCHED, wide_min_log_degree=18)
    elif mode == "all_wide":
        got, st = _serve(nt, reqs, nt.SERVE_BATCHED, wide_min_log_degree=10)
    else:
        got, st = _serve(nt, reqs, nt.SERVE_FIFO if mode == "fifo" else nt.SERVE_FIFO_PER_LIMB)
    assert st["completed"] == len(reqs)
    for k in range(len(reqs)):
        assert np.array_equal(got[k], ref[k]), (mode, k)


def test_server_backpressure_small_budget(nt):
    reqs = [_request(unit_seed(320, k), 14, 4) for k in range(12)]
    fp = (1 << 14) * 4 * 8                      # result footprint; no workspace at N = 2^14
    srv = nt.Server(hbm_budget=3 * fp, streams=2)
    tickets = [srv.submit(r["da"], r["db"], r["N"], r["mods"]) for r in reqs]
    for t, r in zip(tickets, reqs):             # results hold the arena until released
        srv.wait(t, timeout_s=60)
        dst = empty_dev(r["N"] * 4)
        srv.read(t, dst)
        got = from_dev(dst)
        srv.release(t)
        assert np.array_equal(got, _alone(nt, r))
    _settle(srv)
    st = srv.stats()
    assert st["completed"] == 12 and st["deferred"] > 0
    assert st["arena_peak"] <= 3 * fp and st["arena_in_use"] == 0
    srv.close()
    # release on completion: the same stream drains by itself
    srv = nt.Server(hbm_budget=3 * fp, release_on_completion=True)
    for r in reqs:
        srv.submit(r["da"], r["db"], r["N"], r["mods"])
    srv.drain(timeout_s=60)
    st = srv.stats()
    assert st["completed"] == 12 and st["arena_peak"] <= 3 * fp
    srv.close()


def test_server_large_ring_workspace(nt):
    # N = 2^17 products need a workspace as large as the result: footprint 2 L N 8
    reqs = [_request(unit_seed(330, k), 17, 2) for k in range(3)]
    fp = 2 * (1 << 17) * 2 * 8
    outs, st = _serve(nt, reqs, nt.SERVE_BATCHED, hbm_budget=2 * fp)
    for k, (r, got) in enumerate(zip(reqs, outs)):
        assert np.array_equal(got, _alone(nt, r))
        _oracle_check(r, got, 331 + k)


def test_server_rejects_malformed(nt):
    r = _request(340, 12, 2)
    srv = nt.Server(hbm_budget=1 << 20, max_queue=2)
    bad = [
        ((r["da"], r["db"], 4096, POOL[:1] * 0), -7),            # no limbs
        ((r["da"], r["db"], 4096, POOL[:1] * 65), -7),           # too many limbs
        ((r["da"], r["db"], 512, POOL[:1]), -1),                 # N below 2^10
        ((r["da"], r["db"], 3000, POOL[:1]), -1),                # not a power of two
        ((r["da"], r["db"], 1 << 18, POOL[:1]), -1),             # above 2^17
        ((r["da"], r["db"], 4096, [12289]), -2),                 # 12289 != 1 mod 8192
        ((r["da"], r["db"], 4096, [(1 << 50) + 1]), -2),         # not prime
        ((None, r["db"], 4096, POOL[:1]), -5),
        ((r["da"], r["db"], 1 << 17, POOL[:8]), -9),             # footprint above the whole budget
    ]
    for args, want in bad:
        st, t = srv.submit_status(*args)
        assert st == want and t == 0, (args[2:], st)
    far = nt.now_ns() + 60_000_000_000                           # arrives in a minute: stays queued
    t1 = srv.submit(r["da"], r["db"], 4096, r["mods"], arrival_ns=far)
    t2 = srv.submit(r["da"], r["db"], 4096, r["mods"], arrival_ns=far)
    st, t3 = srv.submit_status(r["da"], r["db"], 4096, r["mods"], arrival_ns=far)
    assert st == -11 and t3 == 0                                 # queue of two is full
    assert srv.poll(t1).state == nt.REQ_WAITING
    with pytest.raises(nt.NttError) as e:
        srv.wait(t2, timeout_s=0.05)
    assert e.value.status == -12
    with pytest.raises(nt.NttError) as e:
        srv.release(t1)                                          # still queued
    assert e.value.status == -11
    s = srv.stats()
    assert s["rejected"] == len(bad) + 1 and s["submitted"] == 2 and s["waiting"] == 2
    t0 = time.time()
    srv.close()                                                  # cancels the queued requests at once
    assert time.time() - t0 < 10


def test_server_read_then_release_without_sync(nt):
    """read() enqueues the copy on the caller's stream and release() follows at once, with no
    synchronisation, while the next request waits for exactly that arena range (the budget
    holds one result).  The caller's stream is kept busy first, so the copies run late; the
    range must not be handed to the next request before its copy has run."""
    import torch
    reqs = [_request(unit_seed(350, k), 14, 4) for k in range(6)]
    want = [_alone(nt, r) for r in reqs]
    fp = (1 << 14) * 4 * 8
    srv = nt.Server(hbm_budget=fp, streams=1)
    side = torch.cuda.Stream()
    busy = torch.zeros(1 << 27, dtype=torch.int64, device="cuda:0")
    dsts = [empty_dev(r["N"] * 4) for r in reqs]
    torch.cuda.synchronize()
    tickets = [srv.submit(r["da"], r["db"], r["N"], r["mods"]) for r in reqs]
    for t, dst in zip(tickets, dsts):
        srv.wait(t, timeout_s=60)
        with torch.cuda.stream(side):
            for _ in range(8):
                busy.add_(1)                 # delays the copy enqueued behind it
        srv.read(t, dst, stream=side)
        srv.release(t)                       # no synchronisation between read and release
    srv.drain(timeout_s=60)
    torch.cuda.synchronize()
    for k, (dst, w) in enumerate(zip(dsts, want)):
        assert np.array_equal(from_dev(dst), w), k
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["deferred"] > 0
    _settle(srv)
    assert srv.stats()["arena_in_use"] == 0
    srv.close()
