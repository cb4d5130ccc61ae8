"""Train the warm-start network on the GPU and save its weights.

  python -m paper_2402_04834_amd.train_warm [--count 50000] [--steps 8000] [--batch 16] [--lr 1e-3]

Training set: `count` synthetic syndromes (code-capacity depolarizing noise), d uniform over
{13, 15, 17, 19, 21} and p uniform over [0.05, 0.15], each decoded cold (uniform start) by the library;
the final messages of the converged coset jobs are the targets. Adam on the library's loss gradient with a
cosine-decayed learning rate. Writes weights/warmstart_d13-21.npy and a JSON summary beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import time


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--count", type=int, default=50000)
    ap.add_argument("--steps", type=int, default=8000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--max-iter", type=int, default=40)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)

    import torch
    import paper_2402_04834_amd as bbp
    from paper_2402_04834_amd import warm

    if not torch.cuda.is_available():
        raise SystemExit("training runs on the GPU")
    dev = torch.device("cuda:0")
    opts = bbp.default_opts(block=6, chi=32, max_iter=a.max_iter)
    log = lambda *x: print(*x, flush=True)
    t0 = time.time()
    pool = warm.make_training_set(a.count, opts, dev, log=log)
    t_pool = time.time() - t0
    theta, hist = warm.train(pool, opts, steps=a.steps, batch=a.batch, lr=a.lr, seed=a.seed, log=log, every=250)
    out = a.out or warm.WEIGHTS_PATH
    warm.save(theta.cpu().numpy(), out)
    summary = dict(count=a.count, steps=a.steps, batch=a.batch, lr=a.lr, max_iter=a.max_iter, seed=a.seed,
                   distances=list(warm.TRAIN_DISTANCES), p_range=list(warm.TRAIN_P),
                   pool={int(d): dict(syndromes=int(P["syn"].shape[0]), converged_jobs=int(P["use"].sum()))
                         for d, P in pool.items()},
                   loss_first=float(hist[:50].mean()), loss_last=float(hist[-250:].mean()),
                   pool_seconds=round(t_pool, 1), train_seconds=round(time.time() - t0 - t_pool, 1))
    with open(os.path.splitext(out)[0] + ".json", "w") as f:
        json.dump(summary, f, indent=1)
    log(json.dumps(summary))


if __name__ == "__main__":
    main()
