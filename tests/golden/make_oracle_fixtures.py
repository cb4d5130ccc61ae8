"""Write oracle results for a slice of a seeded workload to a JSON fixture (calls only oracle/ and the
seeded input generator). The GPU tests and the benchmark's agreement figure read these files; nothing in
them comes from the HIP path.

    python tests/golden/make_oracle_fixtures.py --workload d17 --d 17 --p 0.10 --block 6 --chi 32 \
        --count 4096 --chunk 4 --procs 7 --out tests/golden/d17_p010_k6_chi32.json

An existing file with the same parameters is extended (records already present are kept), so a long run can
be resumed. The committed d=17 file holds all 4096 syndromes of the benchmark batch (about 21 hours of oracle
time summed over the worker processes).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)


def _run(args):
    d, p, block, chi, max_iter, eta, workload_name, p_index, start, count, fixed = args
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    from threadpoolctl import threadpool_limits

    from oracle import blockbp
    from paper_2402_04834_amd import workload

    _, syn = workload.make_batch(d, p, count, workload=workload_name, p_index=p_index, start=start)
    with threadpool_limits(1):
        t0 = time.time()
        r = blockbp.decode(d, p, syn, block=(block, block), chi=chi, max_iter=max_iter, eta=eta,
                           fixed_iters=fixed)
        dt = time.time() - t0
    out = []
    for i in range(count):
        out.append(dict(index=start + i, loglik=[float(v) for v in r["loglik"][i]],
                        delta=[float(v) for v in r["delta"][i]], iters=[int(v) for v in r["iters"][i]],
                        coset=int(r["coset"][i])))
    return out, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="d17")
    ap.add_argument("--d", type=int, default=17)
    ap.add_argument("--p", type=float, default=0.10)
    ap.add_argument("--p-index", type=int, default=0)
    ap.add_argument("--block", type=int, default=6)
    ap.add_argument("--chi", type=int, default=32)
    ap.add_argument("--max-iter", type=int, default=20)
    ap.add_argument("--eta", type=float, default=0.1)
    ap.add_argument("--fixed", action="store_true")
    ap.add_argument("--start", type=int, default=0)
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--chunk", type=int, default=2)
    ap.add_argument("--procs", type=int, default=4)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    meta = dict(workload=a.workload, d=a.d, p=a.p, p_index=a.p_index, block=a.block, chi=a.chi,
                max_iter=a.max_iter, eta=a.eta, delta0=1e-4, delta1=1e-2, fixed_iters=a.fixed,
                source="oracle.blockbp.decode (float64)")
    records = {}
    if os.path.exists(a.out):
        old = json.load(open(a.out))
        if {k: old["meta"].get(k) for k in meta} == meta:
            records = {r["index"]: r for r in old["records"]}
    todo = [i for i in range(a.start, a.start + a.count) if i not in records]
    tasks = []
    for j in range(0, len(todo), a.chunk):
        idx = todo[j:j + a.chunk]
        if idx != list(range(idx[0], idx[0] + len(idx))):
            for i in idx:
                tasks.append((a.d, a.p, a.block, a.chi, a.max_iter, a.eta, a.workload, a.p_index, i, 1, a.fixed))
        else:
            tasks.append((a.d, a.p, a.block, a.chi, a.max_iter, a.eta, a.workload, a.p_index, idx[0], len(idx),
                          a.fixed))
    cpu = 0.0
    with Pool(a.procs) as pool:
        for out, dt in pool.imap_unordered(_run, tasks):
            cpu += dt
            for r in out:
                records[r["index"]] = r
            recs = [records[k] for k in sorted(records)]
            tmp = a.out + ".tmp"
            json.dump(dict(meta=meta, records=recs), open(tmp, "w"))
            os.replace(tmp, a.out)
            print(f"{len(recs)} records, {cpu:.0f} s of oracle time", flush=True)


if __name__ == "__main__":
    main()
