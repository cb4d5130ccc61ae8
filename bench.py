"""Throughput benchmark of the blockBP decoder on one MI355X.

Workload (one "step"): decode 4096 seeded syndromes of the d=17 planar surface code under i.i.d.
depolarizing noise p=0.10 (X, Y, Z each p/3) -- blocks of 6x6 tensors, chi=32, at most 20 BP iterations
with early exit (delta0 1e-4, delta1 1e-2, damping 0.1), the contractions on the matrix cores in BF16 with
FP32 accumulation and FP64 log-likelihoods (precision mode 1); the same decode in plain FP32 is timed beside
it. The syndromes are resident in HBM before the timed region starts. Prints one JSON line.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "syndromes decoded/s at d=17, chi=32 (1 GPU); agreement vs FP64 oracle"
PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector: 256 CU x 2.4 GHz x 256 flop/clk (packed dual FMA)
PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector
GOLDEN = os.path.join(ROOT, "tests", "golden", "d17_p010_k6_chi32.json")
TRAFFIC = os.path.join(ROOT, "profiles", "sweep_kernel_d17_b4096_traffic.txt")
BMPS_TRAFFIC = os.path.join(ROOT, "profiles", "bmps_kernel_d17_b4096_traffic.txt")


def traffic(kernel, path=TRAFFIC):
    """HBM bytes per launch of `kernel` from a committed FETCH_SIZE / WRITE_SIZE counter summary (each
    scaled by what the counter reads for a 1 GiB copy), or None when no summary covers it or the kernel
    sources changed since the counters were taken."""
    import hashlib
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    h = hashlib.sha256()
    for f in t["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    k = t["kernels"].get(kernel)
    if h.hexdigest() != t["source_sha256"] or k is None:
        return None
    return 1024.0 * (k["fetch_kib"] * t["fetch_scale"] + k["write_kib"] * t["write_scale"])


TRAFFIC_SOURCES = ["paper_2402_04834_amd/csrc/geom.hpp", "paper_2402_04834_amd/csrc/sweep_launch.hpp",
                   "paper_2402_04834_amd/csrc/wave_sweep.hpp", "paper_2402_04834_amd/csrc/sweep_kernel.hip"]
BMPS_TRAFFIC_SOURCES = ["paper_2402_04834_amd/csrc/bmps_launch.hpp", "paper_2402_04834_amd/csrc/bmps.hip",
                        "paper_2402_04834_amd/csrc/wave_mps.hpp"]


def _short_kernel_name(name):
    """'void bbp::(anonymous namespace)::sweep_kernel<false, 6, true, true, false, true, false>(...)' ->
    'sweep_kernel<6, true, true, false, true>' (FP32 depolarizing kernels; the first template argument true
    gives 'sweep_kernel_bf16<...>', as _lib.sweep_kernel_name names them); 'bmps_kernel'; other kernels
    keep their name."""
    import re
    m = re.search(r"sweep_kernel<(true|false), (\d+(?:, (?:true|false)){4}), false>", name)
    if m:
        return f"sweep_kernel{'_bf16' if m.group(1) == 'true' else ''}<{m.group(2)}>"
    m = re.search(r"trunc_sweep_kernel<(true|false)>", name)
    if m:
        return f"trunc_sweep_kernel<{m.group(1)}>"
    return "bmps_kernel" if re.search(r"bmps_kernel\b", name) and "decide" not in name else name


def write_traffic_summary(fetch_csv, write_csv, copy_mib=1024, target="sweep"):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of every FP32 sweep kernel (target "sweep") or of the
    boundary-MPS kernel (target "bmps") from two rocprofv3 --pmc counter CSVs of `bench.py --calibrate-copy
    MIB`, with the scale factors that make the calibration copy read and write exactly its size; stamped
    with the hash of the kernel sources."""
    sources, path, prefix = ((TRAFFIC_SOURCES, TRAFFIC, "sweep_kernel") if target == "sweep" else
                             (BMPS_TRAFFIC_SOURCES, BMPS_TRAFFIC, "bmps_kernel"))
    import collections
    import csv
    import hashlib

    def load(path, counter):
        per = collections.defaultdict(lambda: collections.defaultdict(float))
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                per[r["Kernel_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
        return per
    fetch, write = load(fetch_csv, "FETCH_SIZE"), load(write_csv, "WRITE_SIZE")
    # the calibration copy is the largest single dispatch of a copy kernel
    cf = max((v for k, d in fetch.items() if "copy" in k.lower() for v in d.values()), default=0.0)
    cw = max((v for k, d in write.items() if "copy" in k.lower() for v in d.values()), default=0.0)
    assert cf > 0 and cw > 0, "no calibration copy in the counter files"
    fetch = {k: (sum(d.values()) / len(d), len(d)) for k, d in fetch.items()}
    write = {k: (sum(d.values()) / len(d), len(d)) for k, d in write.items()}
    size_kib = copy_mib * 1024.0
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    kernels = {}
    for k, (v, n) in fetch.items():
        short = _short_kernel_name(k)
        if short.startswith(prefix) and k in write:
            kernels[short] = dict(fetch_kib=v, write_kib=write[k][0], dispatches=n)
    out = dict(source_sha256=h.hexdigest(), sources=sources, fetch_scale=round(size_kib / cf, 4),
               write_scale=round(size_kib / cw, 4),
               calibration=f"plain device copy of {copy_mib} MiB (bench.py --calibrate-copy {copy_mib}): FETCH_SIZE "
                           f"{cf:.0f} KiB, WRITE_SIZE {cw:.0f} KiB",
               kernels=kernels)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    return out


def _oracle_worker_init():
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    os.environ["MKL_NUM_THREADS"] = "1"


def _oracle_one(args):
    """One syndrome of the workload through the FP64 oracle in this worker (one BLAS thread)."""
    d, p, block, chi, max_iter, index = args
    from threadpoolctl import threadpool_limits

    from oracle import blockbp
    from paper_2402_04834_amd import workload

    _, syn = workload.make_batch(d, p, 1, workload="d17", start=index)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        blockbp.decode(d, p, syn, block=(block, block), chi=chi, max_iter=max_iter)
        return time.perf_counter() - t0


def host_cores():
    """Worker count for the CPU baseline: the cores this process may run on, at most 16 (a one-GPU share of
    the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(d, p, block, chi, max_iter):
    """The FP64 oracle on the host's cores: a process pool of one worker per core (one BLAS thread each), one
    syndrome of the workload per worker. Must run before anything in this process touches the GPU (the
    workers are forked)."""
    import multiprocessing as mp

    cores = host_cores()
    tasks = [(d, p, block, chi, max_iter, i) for i in range(cores)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores, initializer=_oracle_worker_init) as pool:
        per = pool.map(_oracle_one, tasks, chunksize=1)
    wall = time.perf_counter() - t0
    return dict(value=cores / wall, unit="syndromes/s", cores=cores, kind="oracle", cpu=cpu_model(),
                per_core=dict(value=len(per) / sum(per), unit="syndromes/s"),
                sample=f"syndromes 0..{cores - 1} of the d={d} p={p} workload, one per worker process, all 4 "
                       f"cosets, {block}x{block} blocks, chi={chi}, <= {max_iter} iterations with early exit, "
                       f"float64, one BLAS thread per worker; {wall:.1f} s wall")


def wilson(k, n, z=1.959964):
    """95 % Wilson score interval of a binomial proportion k / n."""
    if n == 0:
        return None
    ph = k / n
    den = 1 + z * z / n
    mid = (ph + z * z / (2 * n)) / den
    half = z * ((ph * (1 - ph) / n + z * z / (4 * n * n)) ** 0.5) / den
    return [max(0.0, mid - half), min(1.0, mid + half)]


def agreement(out, batch, errors=None, d=17):
    if not os.path.exists(GOLDEN):
        return None
    g = json.load(open(GOLDEN))
    recs = [r for r in g["records"] if r["index"] < batch]
    if not recs:
        return None
    import numpy as np
    cos = out["coset"].cpu().numpy()
    ll = out["loglik"].cpu().numpy()
    it = out["iters"].cpu().numpy()
    eq = sum(int(cos[r["index"]] == r["coset"]) for r in recs)
    every = np.array([abs(ll[r["index"], k] - r["loglik"][k]) for r in recs for k in range(4)
                      if np.isfinite(r["loglik"][k])])
    diffs = [abs(ll[r["index"], k] - r["loglik"][k]) for r in recs for k in range(4)
             if it[r["index"], k] == r["iters"][k] and np.isfinite(r["loglik"][k])]
    same_it = sum(int(it[r["index"], k] == r["iters"][k]) for r in recs for k in range(4))
    fin = every[np.isfinite(every)]
    logical = None
    if errors is not None:
        # logical failure against the sampled error: GPU from its correction; the oracle's correction differs
        # from the GPU's by the logical of the coset difference (coset bits (x, z) of I, X, Y, Z)
        idx = np.array([r["index"] for r in recs])
        corr = out["correction"].cpu().numpy()
        xs, zs = logical_class(d, errors[idx], corr[idx])
        bits = np.array([(0, 0), (1, 0), (1, 1), (0, 1)])
        go, orc = bits[cos[idx]], bits[np.array([r["coset"] for r in recs])]
        f_gpu = (xs | zs).astype(bool)
        f_orc = ((xs ^ go[:, 0] ^ orc[:, 0]) | (zs ^ go[:, 1] ^ orc[:, 1])).astype(bool)
        allx, allz = logical_class(d, errors[:batch], corr[:batch])
        n_all = int(((allx | allz) != 0).sum())
        logical = dict(
            gpu_fixture=dict(failures=int(f_gpu.sum()), rate=float(f_gpu.mean()), ci95=wilson(int(f_gpu.sum()), len(idx))),
            oracle_fixture=dict(failures=int(f_orc.sum()), rate=float(f_orc.mean()),
                                ci95=wilson(int(f_orc.sum()), len(idx))),
            discordant=dict(gpu_only=int((f_gpu & ~f_orc).sum()), oracle_only=int((f_orc & ~f_gpu).sum())),
            gpu_batch=dict(syndromes=int(batch), failures=n_all, rate=n_all / batch, ci95=wilson(n_all, batch)))
    return dict(syndromes=len(recs), decisions_equal=eq, frac=eq / len(recs), logical_failure=logical,
                cosets=4 * len(recs), cosets_same_iterations=same_it,
                abs_dlnz_all_cosets=dict(max=float(fin.max()), p99=float(np.percentile(fin, 99)),
                                         median=float(np.median(fin)), nonfinite=int(every.size - fin.size))
                if fin.size else None,
                max_abs_dlnz_same_iterations=float(max(diffs)) if diffs else None,
                median_abs_dlnz_same_iterations=float(np.median(diffs)) if diffs else None,
                oracle=os.path.relpath(GOLDEN, ROOT))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32-comparison", action="store_true",
                    help="skip the plain-FP32 decode timed beside the headline (precision 1)")
    ap.add_argument("--precision", type=int, choices=(0, 1), default=1,
                    help="1 (default): the middle-site contractions on the matrix cores in BF16 with FP32 "
                         "accumulation, FP32 elsewhere; 0: FP32 throughout")
    ap.add_argument("--workload", choices=("d17", "mixed", "warm", "biased", "bmps", "schedule", "trunc"),
                    default="d17",
                    help="d17: the headline workload (default); mixed: 8192 syndromes of mixed distance; warm: "
                         "learned warm start against the uniform start at d=25, p=0.10; biased: d=17 under "
                         "Z-biased Pauli noise (p=0.10, bias 10); bmps: the single-block limit (boundary-MPS "
                         "decoder, chi 16) on the d17 syndromes; schedule: iteration and threshold variants "
                         "at d=17, p=0.05 and 0.10, against the bMPS reference; trunc: block sweeps with a "
                         "binding chi (6x6 blocks at chi 8, 8x8 blocks at chi 16) on the first --trunc-batch "
                         "d17 syndromes")
    ap.add_argument("--trunc-batch", type=int, default=256,
                    help="syndromes of the trunc workload (default 256, the first of the d17 batch)")
    ap.add_argument("--block", type=int, default=6, choices=range(1, 7),
                    help="block size k of the d17 workload (default 6; 1 = plain BP between single tensors)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the launch-variant autotuner (job-major items, one stream): for profiler runs, "
                         "whose kernel statistics should hold the timed decodes only")
    ap.add_argument("--warm-d", type=int, default=25, help="distance of the warm-start comparison (default 25)")
    ap.add_argument("--bmps-d", type=int, default=17,
                    help="distance of the single-block (bMPS) workload (default 17, the d17 syndromes; other "
                         "distances draw their own seeded syndromes at p=0.10)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one plain device-to-device copy of MIB MiB (a known-size reference dispatch "
                         "for hardware byte counters)")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM traffic summary of the sweep kernels from two rocprofv3 counter files "
                         "(FETCH_SIZE and WRITE_SIZE runs of this benchmark with --calibrate-copy 1024) and exit")
    ap.add_argument("--traffic-target", choices=("sweep", "bmps"), default="sweep",
                    help="kernels the traffic summary covers: the sweep kernels (default) or the bMPS kernel")
    a = ap.parse_args()
    if a.traffic_summary:
        out = write_traffic_summary(*a.traffic_summary, target=a.traffic_target)
        print(json.dumps({k: v for k, v in out.items() if k != "kernels"}))
        return
    if a.gpus != 1:
        print("bench.py: this decoder runs on one GPU; only --gpus 1 is supported", file=sys.stderr)
        sys.exit(2)
    # the CPU baseline forks its worker processes, so it runs before anything here touches the GPU
    cpu = None
    if a.workload == "d17" and a.block == 6 and not a.no_cpu_baseline:
        cpu = cpu_baseline(17, 0.10, 6, 32, 20)

    import torch

    import paper_2402_04834_amd as bbp
    from paper_2402_04834_amd import _lib, workload

    if a.calibrate_copy > 0:
        n = a.calibrate_copy << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if a.workload == "mixed":
        return mixed_main(a)
    if a.workload == "warm":
        return warm_main(a)
    if a.workload == "biased":
        return biased_main(a)
    if a.workload == "bmps":
        return bmps_main(a)
    if a.workload == "schedule":
        return schedule_main(a)
    if a.workload == "trunc":
        return trunc_main(a)

    d, p, block, chi, max_iter = 17, 0.10, a.block, 32, 20
    errors, syn = workload.make_batch(d, p, a.batch, workload="d17")
    dev = torch.device("cuda:0")
    syn_dev = torch.from_numpy(syn).to(dev)
    head = d17_leg(a, d, p, block, chi, max_iter, syn_dev, a.precision)
    other = None if a.no_fp32_comparison or a.precision == 0 else d17_leg(a, d, p, block, chi, max_iter, syn_dev, 0)
    r = head
    cls, (dom_ms, dom_launches, dom_flops) = max(r["top"].items(), key=lambda kv: kv[1][0])
    achieved = dom_flops / (dom_ms * 1e-3) / 1e12 if dom_ms > 0 else 0.0
    kname = _lib.sweep_kernel_name(cls, a.precision)
    all_achieved = r["upd_flops"] / (r["upd_ms"] * 1e-3) / 1e12 if r["upd_ms"] > 0 else 0.0
    tune = r["tune"]
    precision_text = ("FP32 products and sums",
                      "the contractions with the side messages' middle sites on the matrix cores in BF16 "
                      "(v_mfma_f32_4x4x4_16b_bf16) with FP32 accumulation, the other products FP32, "
                      "FP64 convergence distance and log-likelihoods")[a.precision]
    line = dict(
        metric=METRIC, value=r["value"], unit="syndromes/s", n_gpus=1, steps=a.steps, warmup=a.warmup,
        ms_per_step=1e3 * r["elapsed"] / a.steps, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype=("f32", "bf16/f32")[a.precision], data="synthetic",
        config=dict(workload=f"planar surface code d={d}, depolarizing p={p}, {a.batch} seeded syndromes, "
                             f"{block}x{block} blocks, chi={chi}, <= {max_iter} BP iterations, early exit",
                    d=d, p=p, batch=a.batch, block=block, chi=chi, max_iter=max_iter, delta0=1e-4, delta1=1e-2,
                    damping=0.1, precision=precision_text, parallelism="single GPU"),
        roofline=dict(bound="alu", achieved=achieved, peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                      frac=achieved / PEAK_FP32_TFLOPS, traffic=traffic(kname),
                      kernel=kname, avg_launch_ms=dom_ms / max(dom_launches, 1),
                      flops_per_launch=dom_flops / max(dom_launches, 1), launches=dom_launches,
                      all_sweep_kernels=dict(achieved=all_achieved, frac=all_achieved / PEAK_FP32_TFLOPS,
                                             ms_per_step=r["upd_ms"] / a.steps,
                                             launches_per_step=r["launches"] / a.steps)),
        kernel_ms_per_step=dict(update=r["upd_ms"] / a.steps, bethe=r["bethe_ms"] / a.steps,
                                other=r["other_ms"] / a.steps),
        mean_iterations_per_coset=r["out"]["iters"].double().mean().item(),
        launch_tuning=dict(order=("sweep-major", "job-major")[tune.order], timed_streams=tune.streams,
                           timed_as=("eager launches" if r["events_in_timed"] else "one HIP graph per step"),
                           tuning_decode_ms=tune.ms,
                           roofline_measured_on=("the timed decodes" if r["events_in_timed"] else
                                                 f"{a.steps} separate single-stream decodes")),
        plan=dict(messages_per_coset=r["info"].num_messages, exact_sweeps=bool(r["info"].exact_sweeps),
                  max_cut_rank=r["info"].max_cut_rank),
        agreement=agreement(r["out"], a.batch, errors, d) if block == 6 else None,
    )
    if other is not None:
        ocls, (oms, ol, ofl) = max(other["top"].items(), key=lambda kv: kv[1][0])
        line["fp32_comparison"] = dict(
            value=other["value"], unit="syndromes/s", ms_per_step=1e3 * other["elapsed"] / a.steps,
            speedup=r["value"] / other["value"], kernel=_lib.sweep_kernel_name(ocls, 0),
            avg_launch_ms=oms / max(ol, 1), achieved_tflops=ofl / (oms * 1e-3) / 1e12 if oms > 0 else 0.0,
            mean_iterations_per_coset=other["out"]["iters"].double().mean().item(),
            agreement=agreement(other["out"], a.batch, errors, d) if block == 6 else None,
            note="the same workload and launch set-up in plain FP32 (precision 0), timed right after the headline")
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


def d17_leg(a, d, p, block, chi, max_iter, syn_dev, precision):
    """Autotune, warm up and time a.steps decodes of the d17 batch at `precision`; kernel rates from HIP events
    (in the timed decodes when the tuned variant is one stream, else from as many single-stream decodes after
    the timed region)."""
    import torch

    import paper_2402_04834_amd as bbp

    dev = syn_dev.device
    opts = bbp.default_opts(block=block, chi=chi, max_iter=max_iter, delta0=1e-4, delta1=1e-2, damping=0.1,
                            precision=precision)
    info = bbp.plan_query(d, opts)
    ws = torch.empty(bbp.workspace_size(d, a.batch, opts), dtype=torch.uint8, device=dev)
    # The library's autotuner picks the launch variant for (d, blocks, chi) on this batch (untimed set-up), and
    # the timed steps run that variant. Per-kernel rates need every launch timed alone, so the roofline
    # figure comes from separate single-stream decodes with HIP events after the timed region (with
    # --no-autotune, or when the tuned variant is single-stream, the timed decodes carry the events).
    if a.no_autotune:   # profiling runs: only the timed single-stream decodes, job-major items
        tune = bbp.bbp_tuning(1, 1, 0.0)
    else:
        tune = bbp.autotune(d, p, syn_dev, opts, workspace=ws)
    bbp.set_tuning(d, opts, tune.order, tune.streams)
    events_in_timed = tune.streams == 1
    # With the tuned multi-stream variant the timed steps replay the decode as one HIP graph (captured by the
    # library on the first call, on a stream of its own): no host work per launch.
    timed_opts, timed_stream = opts, None
    if not events_in_timed:
        timed_opts = bbp.default_opts(block=block, chi=chi, max_iter=max_iter, delta0=1e-4, delta1=1e-2,
                                      damping=0.1, precision=precision, graph=1)
        timed_stream = torch.cuda.Stream()
    out = bbp.decode_device(d, p, syn_dev, timed_opts, workspace=ws, stream=timed_stream)
    for _ in range(a.warmup):
        out = bbp.decode_device(d, p, syn_dev, timed_opts, workspace=ws, stream=timed_stream, out=out)
    torch.cuda.synchronize()
    r = dict(upd_ms=0.0, upd_flops=0.0, bethe_ms=0.0, other_ms=0.0, launches=0, top={}, tune=tune, info=info,
             events_in_timed=events_in_timed)

    def account(tm):
        r["upd_ms"] += tm.update_ms
        r["upd_flops"] += tm.update_flops
        r["bethe_ms"] += tm.bethe_ms
        r["other_ms"] += tm.other_ms
        r["launches"] += tm.update_launches
        t = r["top"].setdefault(tm.top_class, [0.0, 0, 0.0])
        t[0] += tm.top_ms
        t[1] += tm.top_launches
        t[2] += tm.top_flops

    t0 = time.perf_counter()
    for _ in range(a.steps):
        if events_in_timed:
            res = bbp.decode_device(d, p, syn_dev, opts, workspace=ws, timing=True)
            account(res["timing"])
        else:
            out = bbp.decode_device(d, p, syn_dev, timed_opts, workspace=ws, stream=timed_stream, out=out)
    torch.cuda.synchronize()
    r["elapsed"] = time.perf_counter() - t0
    r["value"] = a.batch * a.steps / r["elapsed"]
    if events_in_timed:
        out = res
    else:
        bbp.set_tuning(d, opts, tune.order, 1)
        for _ in range(a.steps):
            res = bbp.decode_device(d, p, syn_dev, opts, workspace=ws, timing=True)
            account(res["timing"])
        torch.cuda.synchronize()
    r["out"] = out
    del ws
    return r


def mixed_main(a):
    """Mixed-distance workload: 8192 syndromes, per syndrome d uniform over {9, 13, 17, 21} and p uniform
    over [0.05, 0.15], chi 16 for d <= 13 and 32 above, 6x6 blocks, <= 20 iterations with early exit. The
    timed steps replay one HIP graph that holds the whole decode of all four distances, in --precision (1,
    the BF16 matrix-core contractions, by default) and, for precision 1, once more in plain FP32 (the batched
    BF16 decode against plain FP32 on the same GPU); an eager pass with per-launch HIP events then gives the
    kernel rates."""
    import numpy as np
    import torch

    import paper_2402_04834_amd as bbp
    from paper_2402_04834_amd import _lib, workload

    count = 8192
    items = workload.mixed_batch(count)
    chi_of = {9: 16, 13: 16, 17: 32, 21: 32}
    dev = torch.device("cuda:0")
    groups = []
    for d in (9, 13, 17, 21):
        sel = [(p, s) for dd, p, _, s in items if dd == d]
        groups.append((d, torch.tensor([p for p, _ in sel], dtype=torch.float64, device=dev),
                       torch.from_numpy(np.stack([s for _, s in sel])).to(dev), chi_of[d]))
    # launch variant: tuned on the group with the most work (d=21), which the decode of the mix then uses
    big = groups[-1]
    tune_opts = bbp.default_opts(block=6, chi=big[3], max_iter=20, delta0=1e-4, delta1=1e-2, damping=0.1,
                                 precision=a.precision)
    tune = bbp.autotune(big[0], 0.10, big[2], tune_opts)

    def timed(precision):
        opts = bbp.default_opts(block=6, chi=32, max_iter=20, delta0=1e-4, delta1=1e-2, damping=0.1, graph=1,
                                precision=precision)
        st = torch.cuda.Stream(dev)
        with torch.cuda.stream(st):
            outs, ws, _ = bbp.decode_groups(groups, opts, stream=st)          # capture
            for _ in range(a.warmup):
                outs, ws, _ = bbp.decode_groups(groups, opts, stream=st, workspace=ws, outs=outs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(st):
            for _ in range(a.steps):
                outs, ws, _ = bbp.decode_groups(groups, opts, stream=st, workspace=ws, outs=outs)
        torch.cuda.synchronize()
        return outs, ws, time.perf_counter() - t0

    outs, ws, elapsed = timed(a.precision)
    value = count * a.steps / elapsed
    fp32 = None
    if a.precision == 1 and not a.no_fp32_comparison:
        # the same mix, graph and launch set-up in plain FP32: the batched BF16 decode against plain FP32
        o32, _, e32 = timed(0)
        same = [float((o["coset"] == q["coset"]).double().mean()) for o, q in zip(outs, o32)]
        fp32 = dict(value=count * a.steps / e32, ms_per_step=1e3 * e32 / a.steps,
                    decisions_equal_to_bf16={g[0]: f for g, f in zip(groups, same)},
                    speedup_of_bf16=e32 / elapsed)
    eager = bbp.default_opts(block=6, chi=32, max_iter=20, delta0=1e-4, delta1=1e-2, damping=0.1,
                             precision=a.precision)
    bbp.set_tuning(big[0], tune_opts, tune.order, 1)   # kernel rates: every launch timed alone
    _, _, tm = bbp.decode_groups(groups, eager, workspace=ws, timing=True)
    achieved = tm.top_flops / (tm.top_ms * 1e-3) / 1e12 if tm.top_ms > 0 else 0.0
    line = dict(
        metric="syndromes decoded/s, mixed d in {9, 13, 17, 21} (1 GPU)", value=value, unit="syndromes/s",
        n_gpus=1, steps=a.steps, warmup=a.warmup, ms_per_step=1e3 * elapsed / a.steps, higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype=("f32", "bf16/f32")[a.precision], data="synthetic",
        config=dict(workload="8192 syndromes, d uniform in {9, 13, 17, 21}, p uniform in [0.05, 0.15], chi 16 "
                             "(d <= 13) / 32, 6x6 blocks, <= 20 BP iterations, early exit, one HIP graph per step",
                    batch=count, per_distance={g[0]: int(g[2].shape[0]) for g in groups}, parallelism="single GPU"),
        roofline=dict(bound="alu", achieved=achieved, peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                      frac=achieved / PEAK_FP32_TFLOPS, traffic=None, kernel=_lib.sweep_kernel_name(tm.top_class, a.precision),
                      avg_launch_ms=tm.top_ms / max(tm.top_launches, 1),
                      measured_on="one eager decode on one stream"),
        mean_iterations_per_coset={g[0]: float(o["iters"].double().mean()) for g, o in zip(groups, outs)},
        launch_tuning=dict(order=("sweep-major", "job-major")[tune.order], streams=tune.streams,
                           tuned_on=f"d={big[0]}, {int(big[2].shape[0])} syndromes"),
    )
    if fp32 is not None:
        line["fp32_comparison"] = fp32
    print(json.dumps(line), flush=True)


def biased_main(a):
    """d=17 under Z-biased Pauli noise: p=0.10 with bias p_Z / (p_X + p_Y) = 10 (p_X = p_Y), 4096 syndromes,
    6x6 blocks, chi 32, <= 20 iterations with early exit; the qubit entries take the four probabilities.
    Eager decodes with per-launch HIP events, as the headline workload."""
    import numpy as np
    import torch

    import paper_2402_04834_amd as bbp
    from paper_2402_04834_amd import _lib, workload

    d, count = 17, a.batch
    probs = workload.biased_probs(0.10, 10.0)
    errors, syn = workload.make_batch_pauli(d, probs, count, p_index=17)
    dev = torch.device("cuda:0")
    s = torch.from_numpy(syn).to(dev)
    opts = bbp.default_opts(block=6, chi=32, max_iter=20, delta0=1e-4, delta1=1e-2, damping=0.1)
    bbp.set_tuning(d, opts, 1, 1)
    outs, ws, _ = bbp.decode_groups([(d, probs, s)], opts)
    for _ in range(a.warmup):
        outs, ws, _ = bbp.decode_groups([(d, probs, s)], opts, workspace=ws, outs=outs)
    torch.cuda.synchronize()
    top_ms = top_flops = 0.0
    top_launches, top_class = 0, -1
    t0 = time.perf_counter()
    for _ in range(a.steps):
        outs, ws, tm = bbp.decode_groups([(d, probs, s)], opts, workspace=ws, outs=outs, timing=True)
        top_ms += tm.top_ms
        top_flops += tm.top_flops
        top_launches += tm.top_launches
        top_class = tm.top_class
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    achieved = top_flops / (top_ms * 1e-3) / 1e12 if top_ms > 0 else 0.0
    o = outs[0]
    line = dict(
        metric="syndromes decoded/s at d=17, chi=32, Z-biased noise (1 GPU)", value=count * a.steps / elapsed,
        unit="syndromes/s", n_gpus=1, steps=a.steps, warmup=a.warmup, ms_per_step=1e3 * elapsed / a.steps,
        higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload=f"{count} syndromes, d=17, Pauli noise (I, X, Z, Y) = "
                             f"({probs[0]:.4f}, {probs[1]:.5f}, {probs[2]:.5f}, {probs[3]:.5f}), 6x6 blocks, "
                             "chi 32, <= 20 BP iterations, early exit", batch=count, parallelism="single GPU"),
        roofline=dict(bound="alu", achieved=achieved, peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                      frac=achieved / PEAK_FP32_TFLOPS, traffic=None, kernel=_lib.sweep_kernel_name(top_class),
                      avg_launch_ms=top_ms / max(top_launches, 1)),
        mean_iterations_per_coset=float(o["iters"].double().mean()),
        logical_failure_rate=float(logical_failures(d, errors, o["correction"].cpu().numpy()).mean()),
    )
    print(json.dumps(line), flush=True)


def bmps_flops(d, chi=16):
    """Algorithmic FP64 flops of one coset contraction by the boundary-MPS decoder at the actual bond sizes:
    compressed bond j of the L-row chain b_j = min(chi, 2^j, 2^(L-j)), after a column is absorbed
    w_j = min(2 b_j, 2^j, 2^(L-j)). Per row r of every column but the last, with the row's matrix M of
    m = 2 w_r rows (left bond, leg) and n = w_{r+1} columns:
      absorption  M = R (A (x) T): 2 m n (2 b_r) (the old left bond and the up leg summed per entry);
      QR          Householder, 2 m n^2 - 2 n^3 / 3 (m >= n; mirrored otherwise), rows but the last;
      Q C         the reflections applied to the carry from below (n x b_{r+1}): 4 m b_{r+1} min(m, n);
      SVD         one-sided Jacobi of N (w_r x 2 b_{r+1}) with its right singular vectors, counted by the
                  Golub-Van Loan figure 21 k^3, k = min(w_r, 2 b_{r+1}), plus C = N V: 2 w_r (2 b_{r+1}) b_r.
    The kernel executes every matrix at the padded size 2 chi = 32; these are the method's own flops."""
    L = 2 * d - 1
    b = [min(chi, 2 ** j, 2 ** (L - j)) for j in range(L + 1)]
    w = [min(2 * b[j], 2 ** j, 2 ** (L - j)) for j in range(L + 1)]
    per_col = 0.0
    for r in range(L):
        m, n = 2 * w[r], w[r + 1]
        per_col += 2 * m * n * 2 * b[r]
        if r < L - 1:
            lo, hi = min(m, n), max(m, n)
            per_col += 2 * hi * lo * lo - 2 * lo ** 3 / 3
            per_col += 4 * m * b[r + 1] * lo
        k = min(w[r], 2 * b[r + 1])
        per_col += 21 * k ** 3 + 2 * w[r] * 2 * b[r + 1] * b[r]
    return (L - 1) * per_col


def bmps_main(a):
    """The single-block limit of blockBP -- the boundary-MPS decoder, chi 16 -- on the 4096 syndromes of the
    d=17, p=0.10 workload. One decode per step; the contraction kernel is timed with HIP events on its
    stream. Reports decision agreement with the blockBP decoder (6x6 blocks, chi 32) on the same syndromes
    and both logical failure rates."""
    import numpy as np
    import torch

    import paper_2402_04834_amd as bbp
    from paper_2402_04834_amd import workload

    d, p, chi, count = a.bmps_d, 0.10, 16, a.batch
    errors, syn = workload.make_batch(d, p, count, workload="d17")
    dev = torch.device("cuda:0")
    s = torch.from_numpy(syn).to(dev)
    out = bbp.bmps_decode(d, p, s, chi)
    ws = out["workspace"]
    for _ in range(a.warmup):
        out = bbp.bmps_decode(d, p, s, chi, workspace=ws)
    torch.cuda.synchronize()
    kms = 0.0
    t0 = time.perf_counter()
    for _ in range(a.steps):
        out = bbp.bmps_decode(d, p, s, chi, workspace=ws, timing=True)
        kms += out["kernel_ms"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    avg_ms = kms / a.steps
    flops = bmps_flops(d, chi) * 4 * count
    achieved = flops / (avg_ms * 1e-3) / 1e12
    opts = bbp.default_opts(block=6, chi=32, max_iter=20, delta0=1e-4, delta1=1e-2, damping=0.1)
    ref = bbp.decode_device(d, p, s, opts)
    torch.cuda.synchronize()
    cb = out["coset"].cpu().numpy()
    cr = ref["coset"].cpu().numpy()
    fb = logical_failures(d, errors, out["correction"].cpu().numpy())
    fr = logical_failures(d, errors, ref["correction"].cpu().numpy())
    line = dict(
        metric=f"syndromes decoded/s at d={d} by the single-block limit (bMPS, chi 16; 1 GPU)",
        value=count * a.steps / elapsed, unit="syndromes/s", n_gpus=1, steps=a.steps, warmup=a.warmup,
        ms_per_step=1e3 * elapsed / a.steps, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64", data="synthetic",
        config=dict(workload=f"{count} syndromes, d={d}, p=0.10 (seeded, the d17 workload's generator), one "
                             "block = the whole network, boundary MPS chi 16, FP64", batch=count,
                    parallelism="single GPU"),
        roofline=dict(bound="alu", achieved=achieved, peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                      frac=achieved / PEAK_FP64_TFLOPS,
                      traffic=traffic("bmps_kernel", BMPS_TRAFFIC) if d == 17 and count == 4096 else None,
                      kernel="bmps_kernel",
                      avg_launch_ms=avg_ms, flops_per_launch=flops),
        decisions_equal_to_blockbp=float((cb == cr).mean()),
        logical_failures=dict(bmps=[int(fb.sum()), count, list(wilson(int(fb.sum()), count))],
                              blockbp=[int(fr.sum()), count, list(wilson(int(fr.sum()), count))]),
    )
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = bmps_cpu_baseline(d, p, chi)
    print(json.dumps(line), flush=True)


def _trunc_oracle_agreement(block, chi, out, count):
    """Decisions, iteration counts and ln Z of a truncating decode of the d=17 batch against the committed
    oracle fixture of its first syndromes (tests/golden/d17_p010_k{block}_chi{chi}_first*.json), or None."""
    import glob

    import numpy as np
    paths = sorted(glob.glob(os.path.join(ROOT, "tests", "golden", f"d17_p010_k{block}_chi{chi}_first*.json")))
    if not paths:
        return None
    g = json.load(open(paths[0]))
    rec = [r for r in g["records"] if r["index"] < count]
    if not rec:
        return None
    idx = np.array([r["index"] for r in rec])
    ref_ll = np.array([r["loglik"] for r in rec])
    ref_it = np.array([r["iters"] for r in rec])
    ref_cs = np.array([r["coset"] for r in rec])
    it, ll, cs = (out[k].cpu().numpy()[idx] for k in ("iters", "loglik", "coset"))
    same = (it == ref_it) & np.isfinite(ref_ll)
    err = np.abs(ll[same] - ref_ll[same])
    return dict(syndromes=len(rec), decisions_equal=int((cs == ref_cs).sum()),
                cosets_same_iterations=int((it == ref_it).sum()), cosets=int(it.size),
                max_abs_dlnz_same_iterations=float(err.max()) if err.size else None,
                oracle=os.path.relpath(paths[0], ROOT))


def trunc_main(a):
    """Block sweeps with a binding chi (Sec. III.D): the first --trunc-batch syndromes of the d=17, p=0.10
    workload decoded with (i) 6x6 blocks at chi 8 -- the sweeps whose boundary rank (16) exceeds chi run the
    truncating kernel, the others the exact dense kernels -- and (ii) 8x8 blocks at chi 16, where every sweep
    truncates. Per variant: syndromes/s over --steps decodes (each with HIP events per launch), the truncating
    kernel's FP64 rate (flops of the QR, reflection and SVD work at the padded sizes it executes, see
    plan.cpp), decisions against the headline decoder (6x6 blocks, chi 32, exact) and logical failures."""
    import numpy as np
    import torch

    import paper_2402_04834_amd as bbp
    from paper_2402_04834_amd import _lib, workload

    d, p, count = 17, 0.10, a.trunc_batch
    errors, syn = workload.make_batch(d, p, 4096, workload="d17")
    errors, syn = errors[:count], syn[:count]
    dev = torch.device("cuda:0")
    s = torch.from_numpy(np.ascontiguousarray(syn)).to(dev)
    base = dict(max_iter=20, delta0=1e-4, delta1=1e-2, damping=0.1)
    ref = bbp.decode_device(d, p, s, bbp.default_opts(block=6, chi=32, **base))
    torch.cuda.synchronize()
    cref = ref["coset"].cpu().numpy()
    fref = logical_failures(d, errors, ref["correction"].cpu().numpy())
    legs = []
    for block, chi in [(6, 8), (8, 16)]:
        # progress on stderr: each configuration takes tens of seconds
        print(f"[trunc] {block}x{block} blocks, chi {chi}: {count} syndromes, 1 + {a.warmup} + {a.steps} decodes",
              file=sys.stderr, flush=True)
        opts = bbp.default_opts(block=block, chi=chi, **base)
        info = bbp.plan_query(d, opts)
        ws = torch.empty(bbp.workspace_size(d, count, opts), dtype=torch.uint8, device=dev)
        out = bbp.decode_device(d, p, s, opts, workspace=ws)
        for _ in range(a.warmup):
            out = bbp.decode_device(d, p, s, opts, workspace=ws)
        torch.cuda.synchronize()
        tms = tfl = 0.0
        tl = 0
        kname = "trunc_sweep_kernel"
        t0 = time.perf_counter()
        for _ in range(a.steps):
            out = bbp.decode_device(d, p, s, opts, workspace=ws, timing=True)
            tm = out["timing"]
            if _lib.is_trunc_class(tm.top_class):
                kname = _lib.sweep_kernel_name(tm.top_class)
                tms += tm.top_ms
                tl += tm.top_launches
                tfl += tm.top_flops
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        c = out["coset"].cpu().numpy()
        f = logical_failures(d, errors, out["correction"].cpu().numpy())
        ach = tfl / (tms * 1e-3) / 1e12 if tms > 0 else 0.0
        legs.append(dict(
            block=block, chi=chi, value=count * a.steps / elapsed, unit="syndromes/s",
            ms_per_step=1e3 * elapsed / a.steps, truncating_sweeps=info.truncating_sweeps,
            message_stride=info.message_stride, max_cut_rank=info.max_cut_rank,
            mean_iterations_per_coset=out["iters"].double().mean().item(),
            kernel=dict(name=kname, bound="alu", achieved=ach, peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                        frac=ach / PEAK_FP64_TFLOPS, avg_launch_ms=tms / max(tl, 1), launches=tl,
                        flops_per_launch=tfl / max(tl, 1)),
            decisions_equal_to_exact_chi32=float((c == cref).mean()),
            logical_failures=[int(f.sum()), count, list(wilson(int(f.sum()), count))],
            oracle_agreement=_trunc_oracle_agreement(block, chi, out, count)))
        del ws
    line = dict(
        metric=f"syndromes decoded/s at d={d} with truncating block sweeps (1 GPU)",
        value=legs[0]["value"], unit="syndromes/s", n_gpus=1, steps=a.steps, warmup=a.warmup,
        ms_per_step=legs[0]["ms_per_step"], higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64 (truncating sweeps) / f32 (exact sweeps, messages)", data="synthetic",
        config=dict(workload=f"the first {count} syndromes of the d17 workload (d={d}, p={p}); blockBP with 6x6 "
                             "blocks at chi 8 (value) and 8x8 blocks at chi 16, <= 20 iterations, early exit",
                    batch=count, parallelism="single GPU"),
        variants=legs,
        exact_chi32_logical_failures=[int(fref.sum()), count, list(wilson(int(fref.sum()), count))],
    )
    print(json.dumps(line), flush=True)


SCHEDULE_VARIANTS = [
    # (label, block, max_iter, delta0, delta1, fixed_iters, gate)
    ("paper: <= 20 iterations, early exit at 1e-4", 6, 20, 1e-4, 1e-2, 0, 0.0),
    ("<= 10 iterations", 6, 10, 1e-4, 1e-2, 0, 0.0),
    ("<= 5 iterations", 6, 5, 1e-4, 1e-2, 0, 0.0),
    ("<= 3 iterations", 6, 3, 1e-4, 1e-2, 0, 0.0),
    ("early exit at 1e-3", 6, 20, 1e-3, 1e-2, 0, 0.0),
    ("early exit at 1e-2", 6, 20, 1e-2, 1e-2, 0, 0.0),
    ("trust threshold 1e-1", 6, 20, 1e-4, 1e-1, 0, 0.0),
    ("20 iterations, no early exit", 6, 20, 1e-4, 1e-2, 1, 0.0),
    ("residual gate 1e-7", 6, 20, 1e-4, 1e-2, 0, 1e-7),
    ("residual gate 1e-6", 6, 20, 1e-4, 1e-2, 0, 1e-6),
    ("residual gate 1e-5", 6, 20, 1e-4, 1e-2, 0, 1e-5),
    ("residual gate 1e-6, early exit at 1e-2", 6, 20, 1e-2, 1e-2, 0, 1e-6),
    ("blocks 4x4", 4, 20, 1e-4, 1e-2, 0, 0.0),
    ("blocks 3x3", 3, 20, 1e-4, 1e-2, 0, 0.0),
    ("blocks 2x2", 2, 20, 1e-4, 1e-2, 0, 0.0),
    ("blocks 1x1 (plain BP)", 1, 20, 1e-4, 1e-2, 0, 0.0),
]


def schedule_main(a):
    """Iteration, threshold, schedule and block-size variants of the blockBP decoder (chi 32, eta 0.1) on 4096
    syndromes at d=17 for p = 0.05 and 0.10, each judged against the single-block limit (bMPS, chi 16) on the
    same syndromes: throughput of one eager decode after a warm-up, mean iterations per coset, decisions
    equal to the reference, logical failures against the sampled errors."""
    import numpy as np
    import torch

    import paper_2402_04834_amd as bbp
    from paper_2402_04834_amd import workload

    d, count = 17, a.batch
    dev = torch.device("cuda:0")
    rows = []
    for pi, p in enumerate((0.05, 0.10)):
        errors, syn = workload.make_batch(d, p, count, workload="d17", p_index=pi + 1)
        s = torch.from_numpy(syn).to(dev)
        ref = bbp.bmps_decode(d, p, s, 16)
        torch.cuda.synchronize()
        ref_coset = ref["coset"].cpu().numpy()
        fr = logical_failures(d, errors, ref["correction"].cpu().numpy())
        rows.append(dict(p=p, variant="reference: single block (bMPS, chi 16)",
                         logical_failures=int(fr.sum())))
        del ref
        for label, block, max_iter, d0, d1, fixed, gate in SCHEDULE_VARIANTS:
            opts = bbp.default_opts(block=block, chi=32, max_iter=max_iter, delta0=d0, delta1=d1, damping=0.1,
                                    fixed_iters=fixed, gate=gate)
            out = bbp.decode_device(d, p, s, opts)
            ws = out["workspace"]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = bbp.decode_device(d, p, s, opts, workspace=ws)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            c = out["coset"].cpu().numpy()
            f = logical_failures(d, errors, out["correction"].cpu().numpy())
            rows.append(dict(p=p, variant=label, syndromes_per_s=round(count / dt, 1),
                             mean_iterations=round(float(out["iters"].double().mean()), 2),
                             decisions_equal_to_reference=round(float((c == ref_coset).mean()), 5),
                             logical_failures=int(f.sum())))
    line = dict(metric="blockBP iteration and threshold variants at d=17 against the single-block limit",
                unit="syndromes/s", n_gpus=1, batch=count, dtype="f32", data="synthetic",
                config=dict(workload=f"{count} syndromes per p, d=17, p in (0.05, 0.10), 6x6 blocks, chi 32, "
                                     "eta 0.1; reference bMPS chi 16 (FP64)", parallelism="single GPU"),
                rows=rows)
    print(json.dumps(line), flush=True)


def bmps_cpu_baseline(d, p, chi, count=8):
    """The FP64 bMPS oracle on the first `count` syndromes of the same workload, one thread."""
    from threadpoolctl import threadpool_limits

    from oracle import bmps, network
    from paper_2402_04834_amd import workload

    _, syn = workload.make_batch(d, p, count, workload="d17")
    with threadpool_limits(1):
        t0 = time.perf_counter()
        bmps.bmps_coset_loglik(d, syn, network.depolarizing(p), chi)
        dt = time.perf_counter() - t0
    return dict(value=count / dt, unit="syndromes/s", cores=1, kind="oracle",
                sample=f"syndromes 0..{count - 1} of the d={d} p={p} workload, all 4 cosets, chi={chi}, "
                       f"float64, one thread ({dt:.1f} s)")


def logical_class(d, errors, corrections):
    """Logical components (x, z) of error * correction (no syndrome): the product anticommutes with Z on the
    column-0 horizontal edges iff it has an X logical component, with X on row 0 iff a Z component."""
    import numpy as np
    from paper_2402_04834_amd import workload
    q = workload.qubit_coords(d)
    prod = np.bitwise_xor(errors, corrections)
    col0 = (q[:, 1] == 0) & (q[:, 0] % 2 == 0)
    row0 = (q[:, 0] == 0)
    xs = np.bitwise_xor.reduce(prod[:, col0] & 1, axis=1)
    zs = np.bitwise_xor.reduce((prod[:, row0] >> 1) & 1, axis=1)
    return xs, zs


def logical_failures(d, errors, corrections):
    """1 where the correction differs from the sampled error by a logical operator."""
    import numpy as np
    xs, zs = logical_class(d, errors, corrections)
    return (xs | zs).astype(np.float64)


def warm_main(a):
    """Learned warm start against the uniform (cold) start: 4096 syndromes at d=25 (--warm-d), p=0.10, 6x6 blocks,
    chi 32, early exit at delta0 1e-4 within at most 60 iterations (so that iterations to convergence are
    measured, not the cap). The warm decode is the network's forward, the decode from its messages and the
    cold rerun of the syndromes whose final distance stays at or above delta1 or whose decided coset was not
    the fastest to converge; each is timed whole. Outside the distances the committed network was trained on
    (13..21) the library decodes the whole batch cold ('warm'); 'unguarded' is the network used there anyway,
    the measurement of what it would do."""
    import numpy as np
    import torch

    import paper_2402_04834_amd as bbp
    from paper_2402_04834_amd import warm, workload

    d, p, count, max_iter = a.warm_d, 0.10, a.batch, 60
    dev = torch.device("cuda:0")
    errors, syn = workload.make_batch(d, p, count, workload="warm", p_index=10)
    s = torch.from_numpy(syn).to(dev)
    opts = bbp.default_opts(block=6, chi=32, max_iter=max_iter, delta0=1e-4, delta1=1e-2, damping=0.1)
    theta = torch.from_numpy(warm.load()).to(dev)

    def timed(fn):
        out = None
        for _ in range(a.warmup):
            out = fn(out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            out = fn(out)
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t0) / a.steps

    ws = torch.empty(bbp.workspace_size(d, count, opts), dtype=torch.uint8, device=dev)
    cold, t_cold = timed(lambda o: bbp.decode_device(d, p, s, opts, workspace=ws, out=o))
    wws = [None]

    def warm_step(o, trained=None):
        r = warm.decode(d, p, s, opts, theta, workspace=wws[0], out=o, trained=trained)
        wws[0] = r["workspace"]
        return r
    hot, t_warm = timed(warm_step)
    lo, hi = warm.trained_range()
    unguarded = None
    if not lo <= d <= hi:
        hu, t_u = timed(lambda o: warm_step(o, trained=(0, 0)))
        uwi = hu["iters"].double()
        unguarded = dict(value=count / t_u, ms_per_step=1e3 * t_u, mean_iterations_per_coset=float(uwi.mean()),
                         fallback_syndromes=int(hu["fallback"]),
                         decision_agreement_with_cold=float((hu["coset"] == cold["coset"]).double().mean()),
                         logical_failure_rate=logical_failures(d, errors, hu["correction"].cpu().numpy()).mean())
    pred_ws = torch.empty(warm.workspace_size(d, count, opts, False), dtype=torch.uint8, device=dev)
    _, t_pred = timed(lambda o: warm.predict(d, p, s, opts, theta, workspace=pred_ws))
    ci, wi = cold["iters"].double(), hot["iters"].double()
    line = dict(
        metric=f"syndromes decoded/s at d={d}, p=0.10 with the learned warm start (1 GPU)",
        value=count / t_warm, unit="syndromes/s", n_gpus=1, steps=a.steps, warmup=a.warmup,
        ms_per_step=1e3 * t_warm, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
        data="synthetic",
        config=dict(workload=f"{count} syndromes, d={d}, p=0.10, 6x6 blocks, chi 32, <= {max_iter} BP iterations, "
                             "early exit at delta0 1e-4; warm = network forward + decode from its messages + cold "
                             "rerun where delta >= delta1", batch=count, parallelism="single GPU"),
        cold=dict(value=count / t_cold, ms_per_step=1e3 * t_cold,
                  mean_iterations_per_coset=float(ci.mean()),
                  mean_iterations_per_syndrome_max=float(ci.max(dim=1).values.mean()),
                  converged_cosets=float((cold["delta"] < opts.delta0).double().mean())),
        warm=dict(value=count / t_warm, ms_per_step=1e3 * t_warm, forward_ms=1e3 * t_pred,
                  mean_iterations_per_coset=float(wi.mean()),
                  mean_iterations_per_syndrome_max=float(wi.max(dim=1).values.mean()),
                  converged_cosets=float((hot["delta"] < opts.delta0).double().mean()),
                  fallback_syndromes=int(hot["fallback"])),
        decision_agreement_with_cold=float((hot["coset"] == cold["coset"]).double().mean()),
        logical_failure_rate=dict(cold=logical_failures(d, errors, cold["correction"].cpu().numpy()).mean(),
                                  warm=logical_failures(d, errors, hot["correction"].cpu().numpy()).mean()),
        speedup=t_cold / t_warm, trained_distances=[lo, hi], unguarded=unguarded,
    )
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
