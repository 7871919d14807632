"""Writes c2_fingerprint.json: the oracle's whole-graph summary of the
n = 1e6, average degree 10, gamma 2.7, seed 2 graph (every pair i < j tested
by brute force).  Calls only the oracle.  About half an hour on 8 cores:

    python tests/golden/make_c2_fingerprint.py [threads]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402

N, KBAR, GAMMA, SEED = 1_000_000, 10.0, 2.7, 2


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    import hashlib
    a, R = O.solve_R(N, KBAR, GAMMA)
    r, t, hard = O.sample(SEED, a, R, N, nthreads=threads)
    assert hard == 0
    t0 = time.time()
    deg, fs, fx, quad, ties = O.pair_scan(r, t, R, nthreads=threads)
    wall = time.time() - t0
    out = {
        "workload": "rhg n=1000000 avg_degree=10 gamma=2.7 seed=2",
        "n": N, "avg_degree": KBAR, "gamma": GAMMA, "seed": SEED,
        "alpha": a, "R": R, "R_hex": float(R).hex(),
        "undirected_edges": int(deg.sum()) // 2,
        "degree_sha256": hashlib.sha256(np.ascontiguousarray(deg, dtype=np.int32).tobytes()).hexdigest(),
        "max_degree": int(deg.max()),
        "fingerprint_sum": "%016x" % fs, "fingerprint_xor": "%016x" % fx,
        "binary128_fallbacks": quad, "ties": ties,
        "pairs_tested": N * (N - 1) // 2, "wall_s": round(wall, 1), "threads": O.threads(),
        "made_by": "tests/golden/make_c2_fingerprint.py (oracle only)",
    }
    with open(os.path.join(HERE, "c2_fingerprint.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
