#!/usr/bin/env python3
"""Write the FP64 oracle's results for the two full-size workloads whose oracle
runs take minutes, so that the GPU tests and the benchmark can compare every
result without re-running it:

  batched_4096_oracle.json      Q and A = (1/n) sum |f| of all 4096 integrands of
                                the batched workload (plain rule, eq. 1.2 with the
                                points of eq. 2.1, one Korobov lattice each)
  adjoint_d50_osc_oracle.json   Q, A and the 51-component gradient of all 64
                                oscillatory parameter sets of the adjoint workload
                                (derivative of eq. 1.2 term by term)

Only ``oracle/`` computes anything here; ``paper_2404_08867_amd.workloads`` only
draws the seeded inputs.  Each oracle call stays single-threaded and literal; the
calls for different integrands (or parameter sets) run side by side in a thread
pool (the oracle's C functions release the interpreter lock while they run).

Usage:  python tests/golden/make_oracle_cache.py [--jobs N] [--only batched|adjoint]
About 70 core-minutes for the batched workload and 10 for the adjoint one.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2404_08867_amd import workloads as W  # noqa: E402

BATCHED_FILE = os.path.join(HERE, "batched_4096_oracle.json")
ADJOINT_FILE = os.path.join(HERE, "adjoint_d50_osc_oracle.json")


def _batched_one(p):
    z = O.korobov(p.d, p.n, p.a)
    return O.lattice_sum(z, p.n, p.family, p.params)


def make_batched(jobs: int) -> None:
    batch = W.batched_4096()
    probs = batch.problems
    # longest first, so that the pool's tail is short
    order = sorted(range(len(probs)), key=lambda i: -probs[i].n * probs[i].d)
    q = [None] * len(probs)
    a = [None] * len(probs)
    t0 = time.time()
    done = 0
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {ex.submit(_batched_one, probs[i]): i for i in order}
        for f in cf.as_completed(futs):
            i = futs[f]
            q[i], a[i] = f.result()
            done += 1
            if done % 256 == 0:
                print(f"batched_4096: {done}/{len(probs)} integrands, {time.time() - t0:.0f} s", flush=True)
    out = {
        "workload": batch.name,
        "what": "FP64 oracle Q and A = (1/n) sum_i |f(x_i)| of every integrand, in workload order",
        "generator": "tests/golden/make_oracle_cache.py (oracle.lattice_sum on workloads.batched_4096())",
        "count": len(probs),
        "d": [p.d for p in probs],
        "n": [p.n for p in probs],
        "a": [p.a for p in probs],
        "family": [p.family for p in probs],
        "q": q,
        "abs_mean": a,
    }
    with open(BATCHED_FILE + ".tmp", "w") as f:
        json.dump(out, f)
    os.replace(BATCHED_FILE + ".tmp", BATCHED_FILE)
    print(f"wrote {BATCHED_FILE} in {time.time() - t0:.0f} s", flush=True)


def _adjoint_one(z, n, family, params):
    qg, g = O.lattice_grad(z, n, family, params)
    q, a = O.lattice_sum(z, n, family, params)
    return q, a, [float(v) for v in g], qg


def make_adjoint(jobs: int) -> None:
    w = W.adjoint_d50_osc()
    z = O.korobov(w.d, w.n, w.a)
    nsets = w.params.shape[0]
    q = [None] * nsets
    a = [None] * nsets
    g = [None] * nsets
    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {ex.submit(_adjoint_one, z, w.n, w.family, w.params[s]): s for s in range(nsets)}
        for f in cf.as_completed(futs):
            s = futs[f]
            q[s], a[s], g[s], qg = f.result()
            # the value computed beside the gradient is the same Neumaier sum
            assert qg == q[s], (s, qg, q[s])
    out = {
        "workload": w.name,
        "what": "FP64 oracle Q, A = (1/n) sum_i |f(x_i)| and dQ/dparams (u first, then c_j) per set",
        "generator": "tests/golden/make_oracle_cache.py (oracle.lattice_grad and oracle.lattice_sum on "
                     "workloads.adjoint_d50_osc())",
        "d": w.d, "n": w.n, "a": w.a, "nsets": nsets,
        "q": q, "abs_mean": a, "grad": g,
    }
    with open(ADJOINT_FILE + ".tmp", "w") as f:
        json.dump(out, f)
    os.replace(ADJOINT_FILE + ".tmp", ADJOINT_FILE)
    print(f"wrote {ADJOINT_FILE} in {time.time() - t0:.0f} s", flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--jobs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", choices=["batched", "adjoint"], default=None)
    args = ap.parse_args()
    if args.only in (None, "adjoint"):
        make_adjoint(args.jobs)
    if args.only in (None, "batched"):
        make_batched(args.jobs)


if __name__ == "__main__":
    main()
