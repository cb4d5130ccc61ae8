"""Write oracle results for a slice of a seeded workload to a JSON fixture (calls only oracle/ and the
seeded input generator). The GPU tests and the benchmark's agreement figure read these files; nothing in
them comes from the HIP path.

    python tests/golden/make_oracle_fixtures.py --workload d17 --d 17 --p 0.10 --block 6 --chi 32 \
        --count 4096 --chunk 4 --procs 7 --out tests/golden/d17_p010_k6_chi32.json

An existing file with the same parameters is extended (records already present are kept), so a long run can
be resumed. The committed d=17 file holds all 4096 syndromes of the benchmark batch (about 21 hours of oracle
time summed over the worker processes); the d=11 files hold all 1024 syndromes of each p.

Truncating block sweeps on the benchmark's d=17 batch (its first syndromes; chi binds inside the blocks):

    python tests/golden/make_oracle_fixtures.py --workload d17 --d 17 --p 0.10 --block 6 --chi 8 --count 64 \
        --chunk 2 --procs 7 --out tests/golden/d17_p010_k6_chi8_first64.json
    python tests/golden/make_oracle_fixtures.py --workload d17 --d 17 --p 0.10 --block 8 --chi 16 --count 32 \
        --chunk 1 --procs 7 --out tests/golden/d17_p010_k8_chi16_first32.json

Mixed-distance workload (8192 syndromes, each with its own d in {9, 13, 17, 21} and p in [0.05, 0.15]; chi 16
for d <= 13 and 32 above, 6x6 blocks): the first --per-d syndromes of every distance, each decoded at its own p:

    python tests/golden/make_oracle_fixtures.py --mixed 8192 --per-d 64 --procs 7 \
        --out tests/golden/mixed_8192_first64_per_d.json
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


MIXED_CHI = {9: 16, 13: 16, 17: 32, 21: 32}


def _run_mixed(args):
    """One syndrome of the mixed-distance workload at its own d and p (oracle only)."""
    count, index = args
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    from threadpoolctl import threadpool_limits

    from oracle import blockbp
    from paper_2402_04834_amd import workload

    d, p, _, syn = workload.mixed_batch(index + 1)[index]
    with threadpool_limits(1):
        t0 = time.time()
        r = blockbp.decode(d, p, syn[None], block=(6, 6), chi=MIXED_CHI[d], max_iter=20, eta=0.1)
        dt = time.time() - t0
    return [dict(index=index, d=d, p=p, chi=MIXED_CHI[d], loglik=[float(v) for v in r["loglik"][0]],
                 delta=[float(v) for v in r["delta"][0]], iters=[int(v) for v in r["iters"][0]],
                 coset=int(r["coset"][0]))], dt


def mixed_main(a):
    from paper_2402_04834_amd import workload
    meta = dict(workload="mixed", count=a.mixed, per_d=a.per_d, block=6, chi=MIXED_CHI, max_iter=20, eta=0.1,
                delta0=1e-4, delta1=1e-2, fixed_iters=False, source="oracle.blockbp.decode (float64)")
    meta = json.loads(json.dumps(meta))
    records = {}
    if os.path.exists(a.out):
        old = json.load(open(a.out))
        if {k: old["meta"].get(k) for k in meta if k != "per_d"} == {k: v for k, v in meta.items() if k != "per_d"}:
            records = {r["index"]: r for r in old["records"]}
    items = workload.mixed_batch(a.mixed)
    want = []
    for d in sorted(MIXED_CHI):
        want += [i for i, it in enumerate(items) if it[0] == d][:a.per_d]
    todo = [(a.mixed, i) for i in sorted(want) if i not in records]
    # the largest distances first, so that the pool ends on short tasks
    todo.sort(key=lambda t: -items[t[1]][0])
    cpu = 0.0
    with Pool(a.procs) as pool:
        for out, dt in pool.imap_unordered(_run_mixed, todo):
            cpu += dt
            for r in out:
                records[r["index"]] = r
            recs = [records[k] for k in sorted(records)]
            tmp = a.out + ".tmp"
            json.dump(dict(meta=meta, records=recs), open(tmp, "w"))
            os.replace(tmp, a.out)
            print(f"{len(recs)} records, {cpu:.0f} s of oracle time", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mixed", type=int, default=0, metavar="COUNT",
                    help="write the mixed-distance fixture of a COUNT-syndrome mixed workload instead")
    ap.add_argument("--per-d", type=int, default=64, help="mixed fixture: syndromes per distance")
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
    if a.mixed:
        return mixed_main(a)
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
