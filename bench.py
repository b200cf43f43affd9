"""Benchmark: ADMM outer iterations per second on a 512x512 fan-beam luggage slice.

One step is one outer iteration of the splitting scheme (CG x-update with R and
R^T, per-ray LM decomposition, shrinkage/nonnegativity/dual updates, rho
adaptation) on a synthetic 512x512 FP32 slice, 720 views x 1024 bins, with the
measurements already resident in device memory.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 50] [--warmup 5] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 compute units x 64 VALU lanes x 2.4 GHz = one lane-operation per lane
# per clock (an FMA counts as one operation; packed FP32 is not used).
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "admm_fan512_hbm_traffic.txt")
KERNEL_SOURCES = ["tomo.hip", "udm.hip", "admm.hip", "kernels.h", "common.h", "epilogue.h", "tv.h",
                  "reduce.h", "projidx.h"]


def kernel_source_hash() -> str:
    """Hash of the kernel sources without their // comments and blank lines, so that
    an edit of a comment does not retire counters taken on the same code."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1905_00934_amd", "csrc", f), encoding="utf-8") as fh:
            for line in fh:
                code = re.sub(r"//.*$", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def counted_traffic() -> dict:
    """HBM bytes per dispatch from the committed FETCH_SIZE/WRITE_SIZE summary,
    only while the kernel sources are the ones the counters were taken on."""
    if not os.path.exists(TRAFFIC_FILE):
        return {}
    meta, table = {}, {}
    for line in open(TRAFFIC_FILE):
        parts = line.split()
        if not parts or parts[0].startswith("#"):
            continue
        if parts[0] == "kernel":
            table[parts[1]] = int(parts[-1])
        else:
            meta[parts[0]] = parts[1]
    return table if meta.get("source_hash") == kernel_source_hash() else {}


COUNTERS_FILE = os.path.join(ROOT, "profiles", "admm_fan512_counters.txt")


def binding_unit(kernel: str) -> dict | None:
    """Busy fractions of the VALU and the texture addresser (the vector-memory path)
    of a kernel from the committed counter summary, while the kernel sources are the
    ones the counters were taken on."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    meta, rows = {}, {}
    for line in open(COUNTERS_FILE):
        parts = line.split()
        if not parts:
            continue
        if parts[0] == "#" and len(parts) >= 3 and parts[1] == "source_hash":
            meta["source_hash"] = parts[2]
        elif parts[0].startswith("k_") and len(parts) >= 9:
            rows[parts[0]] = {"valu_busy": float(parts[4]), "ta_busy": float(parts[6])}
    if meta.get("source_hash") != kernel_source_hash():
        return None
    # The FP32 ADMM instantiations (two channels, quarter-turn symmetry, quad records;
    # the transposes' q and dual epilogues with single-precision sums).
    pick = {"project": ("k_project<float,2,4,true,", ">"),
            "backproject_q": ("k_backproject<float,2,4,true,2,", ",float>"),
            "backproject_dual": ("k_backproject<float,2,4,true,3,", ",float>")}.get(kernel)
    for k, v in rows.items():
        if pick and k.startswith(pick[0]) and k.endswith(pick[1]):
            unit = "texture addresser (vector-memory path)" if v["ta_busy"] >= v["valu_busy"] \
                else "VALU issue"
            return {**v, "busiest": unit, "source": os.path.relpath(COUNTERS_FILE, ROOT)}
    return None


def algorithmic_bytes(N: int, M: int, cg_iters: int, elem: int = 4) -> dict:
    """Compulsory HBM bytes per launch of each kernel of the FP32 iteration: every
    array it must read or write once (images N pixels, sinograms M rays, two
    channels).  The tracked images h = R^T (a - R x) and u = R^T u^a are FP64: one
    of their values counts as two FP32 words."""
    extra = 2 * N if cg_iters > 1 else 0
    return {k: v * elem for k, v in {
        "rhs": 28 * N + extra,                      # h, u in, u out; x, y, u^y, z, u^z; p (and r)
        "backproject_q": 2 * M + 4 * N + extra,     # R p; p; R^T R p (and q)
        # da; dy, dz; h in and out; the last CG step: x in and out, p, R^T R p; u in and out
        "backproject_dual": 2 * M + 30 * N,
        "project": 2 * N + 2 * M,                   # p; R p
        "orbit": 2 * N + 16 * N,                    # p; its orbit image and the transpose
        "rhs_orbit": 28 * N + extra + 16 * N,       # the right-hand side and r0's orbit images
        # a-update: m, w, a, R x, R p, u^a, f cache in; a, u^a, R x, da, cache out; with
        # the TV/z/dual blocks: x, y, u^y, z, u^z in; y, u^y, dy, z, u^z, dz out
        "udm": 32 * M + 32 * N,
        "settle": 4 * M + 20 * N,                   # once per call, after a change of rho: u^a, u, u^y, u^z in and out
        "cg_vector": 16 * N,                        # x in and out, p, R^T R p, h in and out
    }.items()}


def table1_workload(dect, torch, plan, meas, steps: int = 3) -> list:
    """Operator applications per outer iteration of both schemes for several (m, n),
    counted from the launches the library records, beside Table 1's formulas, and the
    time per iteration on the same slice.  A two-channel launch applies R (or R^T) to
    both bases, so it counts as two."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rows = []
    for m, n in ((1, 1), (1, 2), (2, 1), (3, 4)):
        prm = dect.AdmmParams(lm_iters=m, cg_iters=n)
        for scheme in ("UDM-CG", "LMxCG"):
            if scheme == "UDM-CG":
                st = plan.new_state()
                plan.admm_init(meas, st, prm)
                run = lambda k: plan.admm_iterate(meas, st, prm, k)
            else:
                st = plan.new_lmcg_state()
                plan.lmcg_init(meas, st, prm)
                run = lambda k: plan.lmcg_iterate(meas, st, prm, k)
            run(1)
            torch.cuda.synchronize()
            e0.record()
            run(steps)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            dect.profile_start()
            run(steps)
            kt = dect.profile_stop()
            cnt = lambda k: kt[k][1] / steps if k in kt else 0.0
            if scheme == "UDM-CG":
                # The transpose of the a-change serves both the dual residual and the
                # next right-hand side (R^T t is tracked), so it is one of Table 1's 2(n+1).
                got = {"R": 2 * cnt("project"),
                       "RT": 2 * (cnt("backproject_q") + cnt("backproject_dual"))}
                want = {"R": 2 * n, "RT": 2 * (n + 1)}
            else:
                got = {"R": cnt("project"), "RT": cnt("backproject")}
                want = {"R": 2 * m * (n + 1), "RT": 2 * m * (n + 1)}
            rows.append({"scheme": scheme, "m": m, "n": n, "measured": got, "table1": want,
                         "ms_per_iter": round(ms, 4)})
    return rows


def _gen(job):
    """Counts of one synthetic slice (runs in a worker process)."""
    from paper_1905_00934_amd import synth
    kind, idx = job
    pr = (synth.slice_problem(idx, with_image=False) if kind == "stack"
          else synth.uneven_problem(idx, with_image=False))
    return kind, idx, pr.geom, pr.i0, pr.counts_high.astype("float32"), pr.counts_low.astype("float32")


def generate(jobs, workers):
    """Seeded inputs of many slices, in parallel, before the GPU is touched."""
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        return list(ex.map(_gen, jobs))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=2)
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-slice stack and the 96-slice uneven batch")
    ap.add_argument("--batch-steps", type=int, default=20,
                    help="timed iterations of the batched workloads")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="Poisson arrivals per s")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="arrival window, s")
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-queue", type=int, default=256,
                    help="queue bound of the 200 req/s run (requests beyond it are shed)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device-to-device copy (reference for "
                         "hardware byte counters)")
    ap.add_argument("--launch", default=None, metavar="BP,PJ[,VIEWS,CHUNK]",
                    help="fix the launch shapes instead of tuning them (waves per workgroup "
                         "of the transpose and the projector, 2, 4 or 8; the projector's "
                         "views per wave and XCD chunk), e.g. for counter passes")
    return ap.parse_args()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_admm_rate(O, pr, iters: int):
    """ADMM iterations/s of the FP64 oracle on one problem, after its initialisation."""
    orc = O.Oracle(pr.geom, pr.spec)
    mh, wh = O.ingest(pr.counts_high, pr.i0)
    ml, wl = O.ingest(pr.counts_low, pr.i0)
    prm = O.Params()
    st = orc.admm_init(mh, ml, wh, wl, prm)
    t0 = time.perf_counter()
    orc.admm_iterate(st, mh, ml, wh, wl, prm, iters)
    dt = time.perf_counter() - t0
    return iters / dt, dt


def cpu_baseline(pr, iters: int):
    """The FP64 oracle on the host cores: `iters` ADMM iterations of the same 512x512
    slice on all threads (the reported value) and one iteration on one thread, the tiny
    64x64 parallel-beam problem in full (20 iterations) on both, and 2 iterations of
    each size class of the uneven mix on all threads."""
    import oracle as O
    from paper_1905_00934_amd import synth
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    O.set_threads(threads)
    rate, dt = _oracle_admm_rate(O, pr, iters)
    tiny = synth.tiny_problem(0)
    tiny_all, tiny_all_s = _oracle_admm_rate(O, tiny, 20)
    # The uneven batch's and the server's three size classes (slices 0, 1, 2 of the
    # uneven mix): 2 iterations each on all threads, and the oracle's latency per request
    # at the server's 100-iteration cap projected from that rate (stated as such).
    per_size = {}
    for idx in (0, 1, 2):
        up = synth.uneven_problem(idx, with_image=False)
        r, d = _oracle_admm_rate(O, up, 2)
        g = up.geom
        per_size[f"{g['nx']}x{g['ny']}/{g['n_views']}x{g['n_det']}"] = {
            "iter_per_s": round(r, 3), "measured_s": round(d, 2), "iterations": 2,
            "latency_s_at_100_iterations_projected": round(100.0 / r, 1)}
    O.set_threads(1)
    rate1, dt1 = _oracle_admm_rate(O, pr, 1)
    tiny_1, tiny_1_s = _oracle_admm_rate(O, tiny, 20)
    O.set_threads(threads)
    return {"value": round(rate, 4), "unit": "iter/s", "cores": threads, "kind": "oracle",
            "sample": f"{iters} ADMM iterations (UDM1-CG1, adaptive rho, FP64) of the same "
                      f"512x512 slice after its initialisation, {threads} threads: {dt:.1f} s",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "one_thread": {"value": round(rate1, 4), "unit": "iter/s",
                           "sample": f"1 iteration of the 512x512 slice: {dt1:.1f} s"},
            "tiny64_full": {"iterations": 20, "all_threads_iter_per_s": round(tiny_all, 3),
                            "all_threads_s": round(tiny_all_s, 2),
                            "one_thread_iter_per_s": round(tiny_1, 3),
                            "one_thread_s": round(tiny_1_s, 2),
                            "workload": "64x64 parallel beam, 90 views x 95 bins, FP64, "
                                        "20 ADMM iterations (the whole tiny configuration)"},
            "per_size_all_threads": per_size}


def batch_workload(dect, torch, dev, items, params, steps, warmup):
    """Plain one-slice-at-a-time launches against one batch (HIP graph) of the same
    slices; both start from the same initial states."""
    from paper_1905_00934_amd import synth
    spec = synth.default_spectra()
    plans, slices, tuned_shapes = {}, [], {}
    for _, _, geom, i0, ch, cl in items:
        key = (geom["nx"], geom["ny"], geom["n_views"], geom["n_det"])
        if key not in plans:
            plans[key] = dect.Plan(geom, spec, torch.float32, device=dev)
            t = plans[key].tune()
            tuned_shapes[key] = {k: (round(v, 2) if isinstance(v, float) else v)
                                 for k, v in t.items()}
        plan = plans[key]
        c = [torch.from_numpy(x).to(dev) for x in (ch, cl)]
        meas = list(plan.ingest(c[0], c[1], i0))
        sa, sb = plan.new_state(), plan.new_state()
        plan.admm_init(meas, sa, params)
        plan.admm_init(meas, sb, params)
        slices.append((plan, meas, sa, sb))
    batch = dect.Batch([(p, m, sb) for p, m, _, sb in slices], params, graph=True)

    def plain(n):
        for plan, meas, sa, _ in slices:
            plan.admm_iterate(meas, sa, params, n)

    plain(warmup)
    batch.iterate(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    out = {}
    for name, fn in (("plain", plain), ("batched_graph", batch.iterate)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        rate = len(slices) * steps / (ms / 1e3)
        out[name] = {"slice_iters_per_s": round(rate, 1),
                     "slices_per_s_at_50_iters": round(rate / 50, 3),
                     "ms_per_batch_iter": round(ms / steps, 4)}
    identical = all(torch.equal(sa.buf, sb.buf) for _, _, sa, sb in slices)
    dect.profile_start()
    batch.iterate(2)
    kt = dect.profile_stop()
    batch.close()
    out["speedup"] = round(out["batched_graph"]["slice_iters_per_s"] /
                           out["plain"]["slice_iters_per_s"], 4)
    out["identical_states"] = identical
    out["groups"] = len(plans)
    out["launch"] = {f"{k[0]}x{k[1]}/{k[2]}x{k[3]}": tuned_shapes[k] for k in plans}
    out["kernels_per_batch_iter_us"] = {k: round(1e3 * v[0] / 2, 2) for k, v in kt.items()}
    return out


def serve_workload(dect, torch, dev, items, args):
    """Requests drawn from the uneven mix's 96 slices (relative objective change 1e-4, at
    most 100 iterations, checks every 5): plain one-slice-at-a-time processing against
    the continuous-batching server, all at once and with Poisson arrivals: at the
    configured 200 req/s (above capacity: the server's queue is bounded, so it sheds
    load; throughput is the saturated capacity and the latency that of served requests)
    and at 70 % of the measured capacity, each over a window of --serve-seconds."""
    import numpy as np
    from paper_1905_00934_amd import synth
    spec = synth.default_spectra()
    plans = {}
    reqs = []
    for _, _, geom, i0, ch, cl in items:
        key = (geom["nx"], geom["ny"], geom["n_views"], geom["n_det"])
        if key not in plans:
            plans[key] = dect.Plan(geom, spec, torch.float32, device=dev)
            plans[key].tune()
        reqs.append((plans[key], i0, ch, cl))
    params = dect.AdmmParams()
    tol, max_iters, step = 1e-4, 100, 5

    def plain_one(plan, i0, ch, cl):
        c = [torch.from_numpy(x).to(dev) for x in (ch, cl)]
        meas = list(plan.ingest(c[0], c[1], i0))
        st = plan.new_state()
        plan.admm_init(meas, st, params)
        it, phis, rels = 0, [], []
        while True:
            n = min(step, max_iters - it)
            log = plan.admm_iterate(meas, st, params, n, log=True)
            it += n
            phis += [e["data"] + e["tv"] for e in log]
            rel = abs(phis[-1] - phis[-2]) / abs(phis[-1]) if len(phis) >= 2 else math.inf
            rels.append(rel)
            if rel <= tol or it >= max_iters:
                return st.x.cpu().numpy(), it, rels

    n_plain = len(reqs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = [plain_one(*r) for r in reqs]
    t_plain = time.perf_counter() - t0
    iters = np.array([p[1] for p in plain])
    last_rel = np.array([p[2][-1] for p in plain])
    out = {"requests": n_plain, "pool": "the 96 uneven slices (256^2, 384^2, 512^2 in "
                                        "ratio 1:1:1), each request one of them in turn",
           "tol": tol, "max_iters": max_iters, "check_every": step,
           "plain": {"slices_per_s": round(n_plain / t_plain, 3),
                     "mean_iters": round(float(iters.mean()), 2)},
           "stop_rule": {"stopped_by_tol": int((iters < max_iters).sum()),
                         "stopped_at_max_iters": int((iters >= max_iters).sum()),
                         "iters_histogram": {str(k): int(v) for k, v in
                                             zip(*np.unique(iters, return_counts=True))},
                         "rel_change_at_last_check_quantiles": [
                             float("%.3g" % q) for q in np.quantile(last_rel, [0.1, 0.5, 0.9])],
                         "rel_change_per_check_slice0": [float("%.3g" % r)
                                                         for r in plain[0][2]]}}

    def run(arrivals, slots, window, max_queue=0):
        """Submit at the given arrival times; with a window, results are taken at its
        end (requests still queued or running then are dropped and counted), else all
        are awaited."""
        srv = dect.Server(max_slots=slots, step_iters=step, max_queue=max_queue)
        t0 = time.perf_counter()
        tickets, shed = [], 0
        for k, ta in enumerate(arrivals):
            wait = ta - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            plan, i0, ch, cl = reqs[k % n_plain]
            try:
                tickets.append((ta, srv.submit(plan, ch, cl, i0, params=params, tol=tol,
                                               max_iters=max_iters)))
            except dect.DectError as e:
                if e.status != -6:
                    raise
                shed += 1
        if window is None:
            res = [(ta, srv.wait(t, 600000)) for ta, t in tickets]
            span = time.perf_counter() - t0
            if any(r is None for _, r in res):
                raise RuntimeError("a served request did not finish within 600 s")
        else:
            left = window - (time.perf_counter() - t0)
            if left > 0:
                time.sleep(left)
            res = [(ta, srv.poll(t)) for ta, t in tickets]
            span = window
        st = srv.stats()
        srv.close()
        done = [r for _, r in res if r is not None]
        lat = np.array([r[1]["latency_s"] for r in done]) if done else np.zeros(1)
        rec = {"offered": len(arrivals), "admitted_to_queue": len(tickets), "shed": shed,
               "completed": len(done), "unfinished_at_end": len(res) - len(done),
               "slices_per_s": round(len(done) / span, 3),
               "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
               "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
               "mean_queue_s": round(float(np.mean([r[1]["queue_s"] for r in done])), 4)
               if done else None,
               "mean_iters": round(float(np.mean([r[1]["iters"] for r in done])), 2)
               if done else None,
               "peak_in_flight": st["peak_in_flight"], "steps": st["steps"]}
        return res, rec

    res, closed = run([0.0] * n_plain, args.serve_slots, None)
    closed["identical_to_plain"] = all(
        r is not None and np.array_equal(r[0], p[0]) and r[1]["iters"] == p[1]
        for (_, r), p in zip(res, plain))
    out["served_closed"] = closed
    rng = np.random.default_rng(2024)

    def poisson(rate, seconds):
        t = np.cumsum(rng.exponential(1.0 / rate, int(rate * seconds * 2) + 16))
        return t[t < seconds]

    print(f"[bench] serving: Poisson {args.serve_rate} req/s for {args.serve_seconds} s",
          file=sys.stderr, flush=True)
    _, over = run(poisson(args.serve_rate, args.serve_seconds), args.serve_slots,
                  args.serve_seconds, max_queue=args.serve_queue)
    over["offered_req_per_s"] = args.serve_rate
    over["arrival_window_s"] = args.serve_seconds
    over["max_queue"] = args.serve_queue
    out["served_poisson"] = over
    rate = 0.7 * closed["slices_per_s"]
    print(f"[bench] serving: Poisson {rate:.1f} req/s (70 % of capacity) for "
          f"{args.serve_seconds} s", file=sys.stderr, flush=True)
    _, under = run(poisson(rate, args.serve_seconds), args.serve_slots, None)
    under["offered_req_per_s"] = round(rate, 3)
    under["arrival_window_s"] = args.serve_seconds
    out["served_poisson_70pct"] = under
    out["speedup_closed_vs_plain"] = round(closed["slices_per_s"] / out["plain"]["slices_per_s"], 3)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(slices are independent and would shard across GPUs without communication)",
              file=sys.stderr)
        sys.exit(2)
    batch_items = {}
    if not args.no_batch:
        workers = min(16, os.cpu_count() or 1)
        jobs = [("stack", k) for k in range(64)] + [("uneven", k) for k in range(96)]
        for item in generate(jobs, workers):
            batch_items.setdefault(item[0], []).append(item)
    import numpy as np
    import torch

    from paper_1905_00934_amd import dect, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pr = synth.slice_problem(0, with_image=True)
    plan = dect.Plan(pr.geom, pr.spec, torch.float32, device=dev)
    if args.launch:
        vals = [int(v) for v in args.launch.split(",")]
        plan.set_launch(*vals)
        tuned = plan.launch()
        tuned_by = "fixed by --launch"
    else:
        tuned = plan.tune()
        tuned_by = "dect_plan_tune (timed on this device)"
    counts = [torch.from_numpy(c).to(dev, torch.float32) for c in (pr.counts_high, pr.counts_low)]
    meas = list(plan.ingest(counts[0], counts[1], pr.i0))
    params = dect.AdmmParams()
    st = plan.new_state()
    plan.admm_init(meas, st, params)
    plan.admm_iterate(meas, st, params, args.warmup)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    plan.admm_iterate(meas, st, params, args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / args.steps

    # Per-kernel times, live, with HIP events on the stream the kernels run on.
    dect.profile_start()
    plan.admm_iterate(meas, st, params, args.steps)
    kt = dect.profile_stop()
    log = plan.admm_iterate(meas, st, params, 1, log=True)
    x = st.x.double().cpu().numpy()
    xi = [20 * math.log10(np.linalg.norm(x[..., b] - pr.x_true[b]) / np.linalg.norm(pr.x_true[b]))
          for b in range(2)]

    # UDM1-PCG1: the same slice with the ramp-preconditioned x-update, as many
    # iterations as the CG run above, timed over the same number of steps.
    pparams = dect.AdmmParams(precond=dect.PRECOND_RAMP)
    pst = plan.new_state()
    plan.admm_init(meas, pst, pparams)
    plan.admm_iterate(meas, pst, pparams, args.warmup)
    torch.cuda.synchronize()
    e0.record(stream)
    plan.admm_iterate(meas, pst, pparams, args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    pms = e0.elapsed_time(e1) / args.steps
    dect.profile_start()
    plan.admm_iterate(meas, pst, pparams, args.steps)
    pkt = dect.profile_stop()
    plog = plan.admm_iterate(meas, pst, pparams, 1, log=True)
    px_ = pst.x.double().cpu().numpy()
    pxi = [20 * math.log10(np.linalg.norm(px_[..., b] - pr.x_true[b]) / np.linalg.norm(pr.x_true[b]))
           for b in range(2)]
    # The same with the transposes summing in double precision (dect_rt_sums F64), which
    # keeps the single-precision PCG iterates near double-precision arithmetic.
    dparams = dect.AdmmParams(precond=dect.PRECOND_RAMP, rt_sums=dect.RT_SUMS_F64)
    dst = plan.new_state()
    plan.admm_init(meas, dst, dparams)
    plan.admm_iterate(meas, dst, dparams, args.warmup)
    torch.cuda.synchronize()
    e0.record(stream)
    plan.admm_iterate(meas, dst, dparams, args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    dms = e0.elapsed_time(e1) / args.steps
    pcg = {"method": "UDM1-PCG1 (ramp filter max(|w|, 1/P) by 2-D FFT on the zero-padded image)",
           "value": round(1e3 / pms, 3), "unit": "iter/s", "ms_per_step": round(pms, 4),
           "precond_us": round(1e3 * pkt["precond"][0] / pkt["precond"][1], 2),
           "accuracy": {"xi_c_db": round(pxi[0], 3), "xi_p_db": round(pxi[1], 3),
                        "iterations": args.warmup + 2 * args.steps + 1,
                        "rho": plog[-1]["rho"]},
           "double_sums": {"value": round(1e3 / dms, 3), "unit": "iter/s",
                           "ms_per_step": round(dms, 4),
                           "note": "the transposes' sums in double precision (rt_sums F64)"}}

    # CDM-FBP: the projection-wise baseline (constrained decomposition of every ray,
    # then FBP of both bases) and the initial image of the iterations built from it.
    cdm_iters = 20
    a_cdm, img_cdm, x0 = plan.cdm_fbp_start(meas, cdm_iters)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        a_cdm, img_cdm, x0 = plan.cdm_fbp_start(meas, cdm_iters)
    e1.record(stream)
    torch.cuda.synchronize()
    cms = e0.elapsed_time(e1) / args.steps
    dect.profile_start()
    plan.cdm_fbp_start(meas, cdm_iters)
    ckt = dect.profile_stop()
    img = img_cdm.double().cpu().numpy()
    cxi = [20 * math.log10(np.linalg.norm(img[..., b] - pr.x_true[b]) / np.linalg.norm(pr.x_true[b]))
           for b in range(2)]
    # UDM1-PCG1 started from the CDM-FBP image, as many iterations as the run above.
    n_same = args.warmup + 2 * args.steps + 1
    sst = plan.new_state()
    plan.admm_init(meas, sst, pparams, x0=x0)
    slog = plan.admm_iterate(meas, sst, pparams, n_same, log=True)
    sx = sst.x.double().cpu().numpy()
    sxi = [20 * math.log10(np.linalg.norm(sx[..., b] - pr.x_true[b]) / np.linalg.norm(pr.x_true[b]))
           for b in range(2)]
    cdm_fbp = {"method": f"CDM (a >= 0, {cdm_iters} projected LM iterations) then Ram-Lak FBP "
                         "of both bases, and the start image (x_c, s x_c)",
               "value": round(1e3 / cms, 3), "unit": "slices/s", "ms_per_slice": round(cms, 4),
               "cdm_us": round(1e3 * ckt["cdm"][0] / ckt["cdm"][1], 2),
               "fbp_us": round(1e3 * ckt["fbp"][0] / ckt["fbp"][1], 2),
               "accuracy": {"xi_c_db": round(cxi[0], 3), "xi_p_db": round(cxi[1], 3)},
               "pcg_from_cdm_fbp": {"xi_c_db": round(sxi[0], 3), "xi_p_db": round(sxi[1], 3),
                                    "iterations": n_same, "rho": slog[-1]["rho"]}}

    # LM1xCG1: the baseline splitting of Eqs. (7)-(8) on the same slice, same rho rule,
    # timed over the same number of iterations; operator launches counted per iteration.
    lparams = dect.AdmmParams()
    lst = plan.new_lmcg_state()
    plan.lmcg_init(meas, lst, lparams)
    plan.lmcg_iterate(meas, lst, lparams, args.warmup)
    torch.cuda.synchronize()
    e0.record(stream)
    plan.lmcg_iterate(meas, lst, lparams, args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    lms = e0.elapsed_time(e1) / args.steps
    dect.profile_start()
    plan.lmcg_iterate(meas, lst, lparams, args.steps)
    lkt = dect.profile_stop()
    llog = plan.lmcg_iterate(meas, lst, lparams, 1, log=True)
    lx = lst.x.double().cpu().numpy()
    lxi = [20 * math.log10(np.linalg.norm(lx[b] - pr.x_true[b]) / np.linalg.norm(pr.x_true[b]))
           for b in range(2)]
    per = lambda k: lkt[k][1] / args.steps if k in lkt else 0.0
    avg = lambda k: round(1e3 * lkt[k][0] / lkt[k][1], 2) if k in lkt else None
    lmcg = {"method": "LM1xCG1 (Eqs. (7)-(8): x_c then x_p by 1 LM iteration each, its "
                      "Gauss-Newton system by 1 CG step with single-channel R and R^T)",
            "value": round(1e3 / lms, 3), "unit": "iter/s", "ms_per_step": round(lms, 4),
            "udm1_cg1_speedup": round(lms / ms_per_step, 3),
            "operators_per_iter": {"R": per("project"), "RT": per("backproject"),
                                   "f_per_ray": 2 * per("lm_eval")},
            "table1": {"R": 4, "RT": 4, "f": 4},
            "kernel_us": {"project": avg("project"), "backproject": avg("backproject"),
                          "lm_eval": avg("lm_eval")},
            "accuracy": {"xi_c_db": round(lxi[0], 3), "xi_p_db": round(lxi[1], 3),
                         "iterations": args.warmup + 2 * args.steps + 1,
                         "rho": llog[-1]["rho"]}}

    table1 = table1_workload(dect, torch, plan, meas)

    info = plan.info()
    N, M = info["n_pixels"], info["n_rays"]
    # Algorithmic VALU operations of one two-channel R or R^T application: per Joseph
    # sample of a base view the position (fma), floor and fraction, shared by the
    # `symmetry` rotated views that reuse it; per sample and channel the difference,
    # the interpolating fma and the accumulation.
    sym = info["symmetry"]
    ops_apply = 3 * info["samples"] // sym + 3 * 2 * info["samples"]
    alg = algorithmic_bytes(N, M, params.cg_iters)
    counted = counted_traffic()
    total = sum(t for t, _ in kt.values())
    per_kernel = {}
    for k, (t_ms, n) in kt.items():
        avg_s = t_ms / n / 1e3
        e = {"avg_us": round(avg_s * 1e6, 3), "launches": n, "share": round(t_ms / total, 4)}
        if k in alg:
            e["hbm_alg_bytes"] = alg[k]
            e["hbm_alg_frac"] = round(alg[k] / avg_s / 1e9 / HBM_PEAK_GBS, 4)
        if k in counted:
            e["hbm_counted_bytes"] = counted[k]
            e["hbm_counted_gbs"] = round(counted[k] / avg_s / 1e9, 1)
        per_kernel[k] = e
    dominant = max(kt, key=lambda k: kt[k][0])
    avg_s = kt[dominant][0] / kt[dominant][1] / 1e3
    achieved = ops_apply / avg_s / 1e12
    roofline = {"kernel": dominant, "bound": "alu", "achieved": round(achieved, 3),
                "peak": round(VALU_PEAK_TOPS, 2), "unit": "TOP/s",
                "frac": round(achieved / VALU_PEAK_TOPS, 4),
                "traffic": counted.get(dominant),
                "ops_per_launch": ops_apply,
                "ops_rule": f"3 per base-view sample (shared by {sym} rotated views) + 3 per "
                            "sample and channel",
                "samples_per_launch": info["samples"], "symmetry": sym,
                "avg_launch_us": round(avg_s * 1e6, 2),
                "hbm_alg_bytes_per_launch": alg.get(dominant),
                "hbm_alg_frac": per_kernel[dominant].get("hbm_alg_frac"),
                "binding_unit": binding_unit(dominant)}

    out = {
        "metric": "ADMM iters/s on 512² fan-beam slice",
        "value": round(1e3 / ms_per_step, 3),
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single fan-beam slice, 512x512 at 0.1 cm, 720 views x 1024 "
                               "bins, luggage phantom (30 objects, 2 steel), I0 2e5, "
                               "UDM1-CG1, adaptive rho, lambda 1e-5, rho0 1e-3",
                   "slices": 1, "image": 512, "views": 720, "bins": 1024,
                   "lm_iters": 1, "cg_iters": 1},
        "roofline": roofline,
        "launch": {**{k: tuned[k] for k in ("bp_waves", "proj_waves", "proj_views",
                                             "proj_chunk")},
                   **{k: round(tuned[k], 2) for k in ("bp_us", "proj_us", "bp_us_default",
                                                      "proj_us_default") if k in tuned},
                   "tuned_by": tuned_by},
        "kernels": per_kernel,
        "accuracy": {"xi_c_db": round(xi[0], 3), "xi_p_db": round(xi[1], 3),
                     "iterations": args.warmup + 2 * args.steps + 1,
                     "rho": log[-1]["rho"]},
        "wall_s": round(wall, 4),
        "pcg": pcg,
        "cdm_fbp": cdm_fbp,
        "lmcg": lmcg,
        "table1": table1,
    }
    if batch_items:
        params_b = dect.AdmmParams()
        out["batched"] = {
            "stack64": {"workload": "64 independent 512x512 fan-beam luggage slices, 720 "
                                    "views x 1024 bins, UDM1-CG1, adaptive rho",
                        **batch_workload(dect, torch, dev, batch_items["stack"], params_b,
                                         args.batch_steps, 2)},
            "uneven96": {"workload": "96 slices, 256x256/360x512, 384x384/540x768 and "
                                     "512x512/720x1024 in ratio 1:1:1, 10-40 objects, 0-3 "
                                     "steel, UDM1-CG1, adaptive rho",
                         **batch_workload(dect, torch, dev, batch_items["uneven"], params_b,
                                          args.batch_steps, 2)},
        }
    if batch_items and not args.no_serve:
        out["serving"] = serve_workload(dect, torch, dev, batch_items["uneven"], args)
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = src.numel() * 4
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pr, args.cpu_iters)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
