"""Writes tests/golden/primes.json: the moduli and default roots of the synthetic
workloads.  Calls only the oracle (its Miller-Rabin prime search and its minimal
primitive 2N-th root), never the GPU library.

Workloads (the paper fixes none of these primes; it only asks q = 1 mod 2N,
q prime, q < 2^62 and quotes timings on an unspecified 50-bit modulus):
  single_1024   largest prime < 2^50 that is 1 mod 2048 (N = 1024, one limb)
  rns_16384     8 largest primes < 2^50 that are 1 mod 2^15 (N = 2^14, 8 limbs)
  large_65536   32 largest primes < 2^60 that are 1 mod 2^17 (N = 2^16, 32 limbs)
  uneven        16 largest primes < 2^50 that are 1 mod 2^16 (N up to 2^15)
  serving       40 primes that are 1 mod 2^18 (valid for every N <= 2^17):
                prime i is the (i // 11)-th largest below 2^(50 + i % 11),
                so bit lengths run over 50..60
  edge          smallest primes just above 2^(Q-1), Q = 30..62, that are 1 mod
                2^18 (Barrett's quotient estimate is weakest there)
  small_16384   8 largest primes < 2^30 that are 1 mod 2^15 (N = 2^14, 8 limbs,
                for the word-size-2^32 path, which needs 4q < 2^32)
  small_32768   8 largest primes < 2^30 that are 1 mod 2^16 (N = 2^15, 8 limbs)
  small_65536   8 largest primes < 2^30 that are 1 mod 2^17 (N = 2^16, 8 limbs, two passes)
Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def main():
    out = {}
    q1 = oracle.find_primes(50, 2048, 1)
    out["single_1024"] = {"N": 1024, "moduli": q1, "psi": [oracle.min_root(1024, q) for q in q1]}
    q2 = oracle.find_primes(50, 1 << 15, 8)
    out["rns_16384"] = {"N": 16384, "moduli": q2, "psi": [oracle.min_root(16384, q) for q in q2]}
    q3 = oracle.find_primes(60, 1 << 17, 32)
    out["large_65536"] = {"N": 65536, "moduli": q3, "psi": [oracle.min_root(65536, q) for q in q3]}
    q4 = oracle.find_primes(50, 1 << 16, 16)
    out["uneven"] = {"N_max": 32768, "moduli": q4}
    per_bits = {b: oracle.find_primes(b, 1 << 18, 4) for b in range(50, 61)}
    q5 = [per_bits[50 + (i % 11)][i // 11] for i in range(40)]
    out["serving"] = {"N_max": 131072, "moduli": q5}
    edge = {}
    for Q in range(30, 63):
        edge[str(Q)] = oracle.find_primes_up(Q, 1 << 18, 2)
    out["edge"] = {"N_max": 131072, "by_bits": edge}
    q6 = oracle.find_primes(30, 1 << 15, 8)
    out["small_16384"] = {"N": 16384, "moduli": q6, "psi": [oracle.min_root(16384, q) for q in q6]}
    q7 = oracle.find_primes(30, 1 << 16, 8)
    out["small_32768"] = {"N": 32768, "moduli": q7, "psi": [oracle.min_root(32768, q) for q in q7]}
    q8 = oracle.find_primes(30, 1 << 17, 8)
    out["small_65536"] = {"N": 65536, "moduli": q8, "psi": [oracle.min_root(65536, q) for q in q8]}
    path = os.path.join(HERE, "primes.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
