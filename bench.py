"""Benchmark: parallel NN-chain HAC on one MI355X.

One step = the whole hot path over one synthetic input resident in HBM:
Ward and complete linkage HAC of n = 1,000,000 points in 2-D drawn from a
mixture of 50 isotropic Gaussians (sigma 0.01, centres uniform in [0,1]^2,
equal weights), seeded. ``value`` is points clustered per second over the
step (both linkages); linkage-distance evaluations per second are reported
beside it.

Also reported (one JSON line):
  roofline      the step's dominant kernel, measured live with HIP events on
                the library's stream: algorithmic work per launch / average
                launch time, against MI355X's published peak
  cpu_baseline  the FP64 oracle (sequential NN-chain, accelerated mode) timed
                on this host on the first points of the same input
Extra, outside the timed steps: the 10,000,000-point Ward run of the same law;
one run each of the d = 10 (1M uniform, average) and d = 128 (200K unit
vectors, Ward / complete / average / avg-2) workloads with their dominant
kernel's roofline; one run each on the paper's own synthetic laws (2U1M, 2G1M,
5U1M, 5G1M, 2U10M, 2G10M) beside its 48-core times; range-query pruning on /
off and the cluster-pair cache size (0, 16, 64, 256 slots per cluster); the
serving leg (a trace of requests of uneven n, d and linkage: one at a time,
open loop at 0.8 x the one-at-a-time capacity with p50/p99 latency, all at
once); the BF16 and FP32 forms of the screening tiles beside the FP16 default at
d = 10 and d = 128.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

def log(msg):
    """Progress line on stderr (stdout carries the one JSON result line)."""
    print("[bench %s] %s" % (time.strftime("%H:%M:%S"), msg), file=sys.stderr, flush=True)


PEAK_HBM_GBS = 8000.0
PEAK_FP64_VEC_TFLOPS = 78.6
PEAK_FP16_MFMA_TFLOPS = 2500.0

# Algorithmic unit costs.
#   search kernels: per candidate visited, the fields a range query has to
#   read: the FP64 centroid (8 d bytes), size and cluster ID (4 + 4 bytes),
#   plus the float32 box (8 d bytes) for complete / average and the FP64
#   spread term (8 bytes) for avg-2; the kernels are gathers, so they are
#   priced against HBM bandwidth (40 bytes per visit for complete at d = 2,
#   24 for Ward).
#   complete tiles: 6 FP64 flops per point pair at d = 2 (2 sub, 2 mul, 1 add,
#   1 max), priced against the FP64 vector peak.
def visit_bytes(link, d=2):
    return 8 * d + 4 + 4 + {"ward": 0, "avgsq": 8}.get(link, 8 * d)


COMPLETE_PAIR_FLOPS = 6
KERNEL_NAMES = ("ring_search", "block_search", "pair_tiles", "ring_emit")

LINKS = ("ward", "complete")


def gram_kp(d):
    """MFMA depth of the Gram tiles for dimension d (d plus two augmented
    coordinates, in steps of 16)."""
    for kp in (16, 32, 64, 80, 128):
        if d + 2 <= kp:
            return kp
    return 144


def point_kp(d):
    """MFMA depth of the interval screening's point tiles (d alone: their norm
    terms are added outside the MFMA)."""
    for kp in (16, 32, 64, 80):
        if d <= kp:
            return kp
    return 128


def roofline(kname, link, d, ms, nl, sts):
    """Roofline entry of the step's dominant kernel: algorithmic work per
    launch (unit cost x units counted by the library) / average launch time
    (HIP events on the library's stream), against MI355X's published peak."""
    avg_ms = ms / nl
    gram = 4 <= d <= 128
    visits = sum(s["kernels"][kname]["visits"] for s in sts)
    if kname == "pair_tiles":
        # exact tiles: FP64 flops per point pair (d sub, d mul, d add, + max or sqrt/add)
        flops = COMPLETE_PAIR_FLOPS if d == 2 else 3 * d + 1
        work = sum(s["point_pair_evals"] for s in sts) * flops / nl
        achieved = work / (avg_ms / 1000.0) / 1e12
        r = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VEC_TFLOPS, "unit": "TFLOP/s",
             "note": "exact FP64 point-pair tiles; work = point pairs x FP64 flops per pair"}
    elif link in ("ward", "avgsq") and 3 <= d <= 5 and kname == "ring_search":
        # the slot holds the box-tree walk (gathers) of the rounds with many
        # active clusters and Gram pass 0 (MFMA pairs) of the later ones, and
        # its visit count adds both: no single unit prices it
        r = {"bound": None, "achieved": None, "peak": None, "unit": None,
             "note": "box-tree walk and Gram pass 0 share this timing slot; not priced"}
        r.update({"frac": None, "traffic": None, "kernel": kname, "linkage": link, "avg_launch_ms": avg_ms,
                  "launches": nl, "work_per_launch": None})
        return r
    elif gram and kname in ("ring_search", "ring_emit", "block_search"):
        # Gram passes (centroid pairs, K = d + 2 padded) and interval tiles
        # (point pairs, K = d padded): FP16 MFMA, 2 x K flops per pair
        kp = point_kp(d) if kname == "block_search" else gram_kp(d)
        work = visits * 2 * kp / nl
        achieved = work / (avg_ms / 1000.0) / 1e12
        r = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP16_MFMA_TFLOPS, "unit": "TFLOP/s",
             "note": "FP16 MFMA tiles; work = pairs x 2K flops (K = %d)" % kp}
    else:
        work = visits * visit_bytes(link, d) / nl
        achieved = work / (avg_ms / 1000.0) / 1e9
        r = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
             "note": "search kernels gather candidate records; work = visits x record bytes"}
    r["frac"] = r["achieved"] / r["peak"]
    r["traffic"] = measured_traffic(kname, link, d)
    if r["traffic"] is not None and r["unit"] == "GB/s":
        # the same launches priced by the HBM bytes the counters measured
        r["measured_gbs"] = r["traffic"] / (avg_ms / 1000.0) / 1e9
        r["measured_frac"] = r["measured_gbs"] / PEAK_HBM_GBS
    r.update({"kernel": kname, "linkage": link, "avg_launch_ms": avg_ms, "launches": nl,
              "work_per_launch": work})
    return r


def measured_traffic(kname, link, d):
    """HBM bytes per launch of the kernel from the committed rocprofv3 PMC
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration),
    or None when there is none or the kernel source changed since."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "blob50_1m_d2_%s_%s_traffic.md" % (link, kname))
    if d != 2 or not os.path.exists(path):
        return None
    src = os.path.join(ROOT, "paper_2106_04727_amd", "csrc", "pc_round.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != sha:
        return None
    return float(vals["hbm_bytes_per_launch"])


def workload_leg(pc, synth, torch, ctx, stream, wl, link):
    """One timed run of another configuration (after a small warm-up of the
    same dimension), inputs resident on the device; with its dominant kernel's
    roofline entry."""
    x = synth.WORKLOADS[wl]()
    n, d = x.shape
    dev = torch.device("cuda:0")
    w = torch.from_numpy(synth.blobs(4000, d, 20, 0.03, 3)).to(dev)
    pc.hac_device(w, link, ctx=ctx, stream=stream)
    xt = torch.from_numpy(x).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = pc.hac_device(xt, link, ctx=ctx, stream=stream, timing="kernels")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    best = max(KERNEL_NAMES, key=lambda k: st["kernels"][k]["ms"])
    roof = roofline(best, link, d, st["kernels"][best]["ms"], max(st["kernels"][best]["launches"], 1), [st])
    del xt
    return {"n": int(n), "d": int(d), "linkage": link, "s": wall, "points_per_s": n / wall,
            "rounds": st["rounds"], "cluster_evals": st["cluster_evals"], "refined": st["refined"],
            "fp64_fallbacks": st["fp64_fallbacks"],
            "point_pair_evals": st["point_pair_evals"], "cache_hits": st["cache_hits"],
            "cache_derived": st["cache_derived"], "kernels": st["kernels"], "roofline": roof}


# The paper's 48-core (two-way hyper-threaded) running times in seconds on its
# own synthetic sets (Sec. 6, table of running times), for context only:
# another machine, and inputs drawn here from the same laws, not the same files.
PAPER_48H_S = {
    ("2U1M", "ward"): 0.50, ("2G1M", "ward"): 0.52, ("5U1M", "ward"): 1.95, ("5G1M", "ward"): 2.69,
    ("2U10M", "ward"): 5.69, ("2G10M", "ward"): 5.20,
    ("2U1M", "complete"): 1.34, ("2G1M", "complete"): 1.61, ("2U10M", "complete"): 19.01,
    ("2G10M", "complete"): 21.29,
    ("2U1M", "average"): 23.59, ("2G1M", "average"): 26.83, ("5U1M", "average"): 38.10,
    ("5G1M", "average"): 45.27,
    ("2U1M", "avgsq"): 0.47, ("2G1M", "avgsq"): 0.49, ("5U1M", "avgsq"): 1.65, ("5G1M", "avgsq"): 2.27,
    ("2U10M", "avgsq"): 5.30, ("2G10M", "avgsq"): 4.80,
}


def precision_leg(pc, synth, torch, ctx, stream, base):
    """The screening tiles' element type (pc_precision) at the d = 10 and
    d = 128 workloads: BF16 and FP32 operands beside the FP16 default (whose
    run is in `base`); every form refines what its tiles cannot rule out in
    FP64, so the rows must equal the FP16 form's (reported, with the largest
    relative height difference) while the time and the number of refined
    candidates differ."""
    import numpy as np

    from paper_2106_04727_amd import parchain

    out = {}
    dev = torch.device("cuda:0")
    for wl, link in (("u1m_d10", "average"), ("blob100_1m_d10", "average"),
                     ("vmf1000_200k_d128", "complete"), ("vmf1000_200k_d128", "average")):
        key = "%s_%s" % (wl, link)
        log("precision forms: %s, %s linkage" % (wl, link))
        try:
            x = synth.WORKLOADS[wl]()
            xt = torch.from_numpy(x).to(dev)
            w = torch.from_numpy(synth.blobs(4000, x.shape[1], 20, 0.03, 3)).to(dev)
            row = {"fp16": {k: base[key][k] for k in ("s", "refined", "fp64_fallbacks") if k in base.get(key, {})}}
            ref = None
            for prec in ("fp16", "bf16", "fp32"):
                pc.hac_device(w, link, ctx=ctx, stream=stream, precision=prec)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rows, st = pc.hac_device(xt, link, ctx=ctx, stream=stream, precision=prec)
                torch.cuda.synchronize()
                sec = time.perf_counter() - t0
                Z = parchain.rows_to_Z(rows)
                if prec == "fp16":
                    ref = Z
                    row["fp16"].update({"s_rerun": sec, "refined": st["refined"],
                                        "fp64_fallbacks": st["fp64_fallbacks"]})
                    continue
                rel = np.abs(Z[:, 2] - ref[:, 2]) / np.maximum(np.abs(ref[:, 2]), 1e-300)
                row[prec] = {"s": sec, "refined": st["refined"], "fp64_fallbacks": st["fp64_fallbacks"],
                             "tree_equal_fp16": bool(np.array_equal(Z[:, [0, 1, 3]], ref[:, [0, 1, 3]])),
                             "max_rel_height_diff_vs_fp16": float(rel.max()),
                             "median_rel_height_diff_vs_fp16": float(np.median(rel))}
            del xt
            out[key] = row
        except Exception as e:  # reported, never hidden
            out[key] = {"error": str(e)}
    return out


def paper_leg(pc, synth, torch, ctx, stream):
    """One run each on the paper's synthetic laws (UniformFill, GaussianDisc)
    beside the paper's 48-core time for the same set name."""
    out = {}
    for (wl, link), ref in PAPER_48H_S.items():
        log("paper set %s, %s linkage" % (wl, link))
        try:
            r = workload_leg(pc, synth, torch, ctx, stream, wl, link)
            out["%s_%s" % (wl, link)] = {"s": r["s"], "rounds": r["rounds"], "paper_48h_s": ref,
                                         "ratio_paper_over_ours": ref / r["s"]}
        except Exception as e:  # reported, never hidden
            out["%s_%s" % (wl, link)] = {"error": str(e)}
    return out


def ablation_leg(pc, synth, torch, ctx, stream):
    """The paper's two ablations, on its GaussianDisc law in 2-D (Sec. 6):
    the range-query pruning of Alg. 3 on and off (its "no range query"
    comparison), at sizes where the unpruned search still finishes; and
    the cluster-pair cache size s in {0, 16, 64, 256} slots per cluster
    (Sec. 5; the paper uses s = 64) for average and complete linkage on 2G1M."""
    dev = torch.device("cuda:0")

    def run(x, link, **kw):
        xt = torch.from_numpy(x).to(dev)
        pc.hac_device(xt[:4000].contiguous(), link, ctx=ctx, stream=stream, **kw)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = pc.hac_device(xt, link, ctx=ctx, stream=stream, **kw)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, st

    out = {"pruning": {}, "cache": {}}
    for link in ("ward", "avgsq", "complete", "average"):
        log("ablation: range-query pruning on / off, %s linkage" % link)
        # the unpruned search evaluates every pair: O(n^2) centroid pairs per
        # round for Ward / avg-2, O(n^2) point pairs for complete / average
        x = synth.gaussian_disc(100_000 if link in ("ward", "avgsq") else 20_000, 2, 71)
        row = {"n": int(x.shape[0])}
        for prune in (True, False):
            sec, st = run(x, link, prune=prune)
            row["on" if prune else "off"] = {"s": sec, "cluster_evals": st["cluster_evals"],
                                             "point_pair_evals": st["point_pair_evals"]}
        row["speedup"] = row["off"]["s"] / row["on"]["s"]
        out["pruning"][link] = row
    x = synth.WORKLOADS["2G1M"]()
    for link in ("average", "complete"):
        log("ablation: cache sizes, %s linkage" % link)
        row = {}
        for slots in (0, 16, 64, 256):
            sec, st = run(x, link, cache_slots=slots)
            row[str(slots)] = {"s": sec, "hits": st["cache_hits"], "inserts": st["cache_inserts"],
                               "derived": st["cache_derived"], "point_pair_evals": st["point_pair_evals"]}
        out["cache"][link] = row
    return out


def serve_bench(num, slots, n_max):
    """Serving leg: a Poisson trace of clustering requests of uneven n, d and
    linkage (the serving law of ``synth.serving_trace``), first solved one at
    a time on one context (the measured one-at-a-time capacity C, requests
    per second), then submitted at their Poisson arrival times to a server
    with ``slots`` slots at rate 0.8 C (open loop; latency = completion -
    arrival, p50/p99), then all at once (closed loop: throughput against one
    at a time)."""
    import numpy as np

    import paper_2106_04727_amd as pc
    import synth

    log("serving: %d requests, one at a time first" % num)
    trace = synth.serving_trace(num, 1.0, seed=41, n_max=n_max)
    xs = [synth.request_points(r) for r in trace]
    ctx = pc.Context(0)
    outs = [np.zeros((max(r["n"] - 1, 1), 4), np.int64) for r in trace]
    # warm the device code paths once on small requests of each shape class
    for d in (2, 3, 10, 64):
        for link in ("complete", "average", "ward"):
            w = synth.blobs(300, d, 5, 0.02, 7)
            o = np.zeros((299, 4), np.int64)
            ctx.hac(w.ctypes.data, 300, d, link, o.ctypes.data, points_on_device=False, out_on_device=False)
    t0 = time.perf_counter()
    alone = []
    for i, (r, x, o) in enumerate(zip(trace, xs, outs)):
        ta = time.perf_counter()
        ctx.hac(x.ctypes.data, r["n"], r["d"], r["linkage"], o.ctypes.data, points_on_device=False,
                out_on_device=False)
        alone.append(time.perf_counter() - ta)
        if (i + 1) % 50 == 0:
            log("serving: %d of %d solved one at a time" % (i + 1, num))
    t_seq = time.perf_counter() - t0
    ctx.close()
    # arrival rate 0.8 x the measured one-at-a-time capacity
    rate = 0.8 * num / t_seq
    span = num / rate
    scale = span / max(trace[-1]["t"], 1e-9)
    arrivals = [r["t"] * scale for r in trace]
    lat = []
    log("serving: open loop at 0.8 x the one-at-a-time capacity (%.1f req/s)" % (num / span))
    with pc.Server(device=0, slots=slots) as srv:
        start = time.perf_counter()
        tickets = []
        for a, r, x in zip(arrivals, trace, xs):
            dt = a - (time.perf_counter() - start)
            if dt > 0:
                time.sleep(dt)
            tickets.append((srv.submit(x, r["linkage"]), time.perf_counter() - start))
            if len(tickets) % 50 == 0:
                log("serving: %d of %d submitted" % (len(tickets), num))
        slow = []
        for (t, at), ta in zip(tickets, alone):
            info = srv.wait(t)
            if info["status"] != 0:
                raise RuntimeError("request failed: %s" % info["error"])
            lat.append(info["t_done_ms"] - info["t_submit_ms"])
            slow.append(lat[-1] / max(1e3 * ta, 1e-3))
            srv.release(t)
        makespan = time.perf_counter() - start
        st = srv.stats()
        # closed loop: the whole trace submitted at once (throughput against
        # one-at-a-time solving of the same requests)
        log("serving: all requests at once")
        start = time.perf_counter()
        burst = [srv.submit(x, r["linkage"]) for r, x in zip(trace, xs)]
        for t in burst:
            info = srv.wait(t)
            if info["status"] != 0:
                raise RuntimeError("request failed: %s" % info["error"])
            srv.release(t)
        burst_s = time.perf_counter() - start
    return {
        "requests": num, "slots": slots, "n_max": n_max,
        "trace": "Poisson arrivals; n log-uniform [256, n_max], d uniform {2,3,10,64}, linkage uniform "
                 "{complete, average, ward}, 5-100 Gaussian blobs, sigma 0.01-0.05 (seed 41)",
        "one_at_a_time_s": t_seq, "one_at_a_time_req_per_s": num / t_seq,
        "offered_rate_req_per_s": num / span, "offered_load_vs_capacity": 0.8,
        "open_loop_makespan_s": makespan,
        "burst_makespan_s": burst_s, "burst_req_per_s": num / burst_s,
        "burst_speedup_vs_one_at_a_time": t_seq / burst_s,
        "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
        "latency_ms_max": float(np.max(lat)),
        # latency over the request's own one-at-a-time time (1 = no wait, no sharing)
        "slowdown_p50": float(np.percentile(slow, 50)), "slowdown_p99": float(np.percentile(slow, 99)),
        "alone_ms_p50": 1e3 * float(np.percentile(alone, 50)), "alone_ms_p99": 1e3 * float(np.percentile(alone, 99)),
        "requeued": st.get("requeued", 0),
        "peak_running": st["peak_running"], "peak_bytes_in_use": st["peak_bytes_in_use"],
        "budget_bytes": st["budget_bytes"],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--cpu-sample", type=int, default=100_000,
                    help="points of the headline input the CPU oracle baseline clusters")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 10M Ward run and the d=10 / d=128 workloads")
    ap.add_argument("--links", default=",".join(LINKS))
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests of the serving trace (0 skips the serving leg)")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-nmax", type=int, default=200_000)
    ap.add_argument("--workload", default="blob50_1m_d2",
                    help="named input of synth.WORKLOADS (the headline is blob50_1m_d2)")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the BF16 / FP32 screening forms at d = 10 and 128")
    ap.add_argument("--no-ablations", action="store_true",
                    help="skip the pruning on/off and cache-size ablations")
    ap.add_argument("--copy-probe", action="store_true",
                    help="copy 256 MiB on the device first (calibrates HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the method runs on a single MI355X here "
              "(--gpus %d requested); multi-GPU sharding is a design note, not a run." % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2106_04727_amd as pc
    import synth

    links = [l for l in args.links.split(",") if l]
    if args.workload == "blob50_1m_d2":
        x = synth.blobs(args.n, 2, 50, 0.01, 11)
    else:
        x = synth.WORKLOADS[args.workload]()
    n, d = x.shape
    dev = torch.device("cuda:0")
    xt = torch.from_numpy(x).to(dev)
    torch.cuda.synchronize()
    if args.copy_probe:
        src = torch.ones(1 << 26, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = pc.Context(0)
    stream = torch.cuda.current_stream(dev).cuda_stream

    def one_step(collect):
        # kernel events only (the roofline's launch times); the per-round
        # phase events would add host reads to every round of the timed steps
        for link in links:
            _, st = pc.hac_device(xt, link, ctx=ctx, stream=stream, timing="kernels")
            collect.setdefault(link, []).append(st)

    log("warm-up: %d steps of %s on %s" % (args.warmup, "+".join(links), args.workload))
    for _ in range(args.warmup):
        one_step({})
    torch.cuda.synchronize()
    per = {}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step(per)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1000.0 * wall / max(args.steps, 1)
    log("timed: %d steps, %.2f ms per step" % (args.steps, ms_step))

    # per-linkage summaries
    lk = {}
    tot_evals = 0
    for link, sts in per.items():
        ms = np.array([s["ms_total"] for s in sts])
        ce = sts[-1]["cluster_evals"]
        pp = sts[-1]["point_pair_evals"]
        tot_evals += ce * len(sts)
        lk[link] = {
            "ms_device_median": float(np.median(ms)),
            "ms_device_min": float(ms.min()),
            "points_per_s": n / (float(np.median(ms)) / 1000.0),
            "rounds": sts[-1]["rounds"],
            "terminals": sts[-1]["terminals"],
            "cluster_evals": ce,
            "point_pair_evals": pp,
            "cluster_evals_per_s": ce / (float(np.median(ms)) / 1000.0),
            "point_pair_evals_per_s": pp / (float(np.median(ms)) / 1000.0),
            "kernels": sts[-1]["kernels"],
        }

    # dominant kernel over the step (largest summed event time)
    cands = []
    for link, sts in per.items():
        for kname in KERNEL_NAMES:
            ms = sum(s["kernels"][kname]["ms"] for s in sts)
            nl = sum(s["kernels"][kname]["launches"] for s in sts)
            if nl:
                cands.append((ms, link, kname, nl, sts))
    cands.sort(key=lambda c: c[0], reverse=True)
    roof = None
    if cands:
        ms, link, kname, nl, sts = cands[0]
        roof = roofline(kname, link, d, ms, nl, sts)

    value = n * len(links) / (wall / max(args.steps, 1))
    out = {
        "metric": "points clustered/sec (+ linkage distance evals/sec) at n=1M",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (float32 inputs)",
        "data": "synthetic",
        "config": {"workload": ("blob50_1m_d2: n=1,000,000 d=2, 50 Gaussians sigma=0.01, seed 11; "
                                "Ward + complete linkage per step") if args.workload == "blob50_1m_d2"
                   else "%s (%s linkage per step)" % (args.workload, "+".join(links)),
                   "n": int(n), "d": int(d), "linkages": links, "parallelism": "single GPU"},
        "linkage_dist_evals_per_s": tot_evals / wall,
        "per_linkage": lk,
        "roofline": roof,
    }

    if not args.no_extra and "ward" in links:
        log("10M-point Ward run")
        try:
            x10 = synth.blobs(10_000_000, 2, 50, 0.01, 12)
            x10t = torch.from_numpy(x10).to(dev)
            del x10
            pc.hac_device(x10t, "ward", ctx=ctx, stream=stream)  # warm
            _, st = pc.hac_device(x10t, "ward", ctx=ctx, stream=stream)
            out["ward_10m"] = {"ms_device": st["ms_total"], "points_per_s": 1e7 / (st["ms_total"] / 1000.0),
                               "rounds": st["rounds"], "cluster_evals": st["cluster_evals"]}
            del x10t
        except Exception as e:  # reported, never hidden
            out["ward_10m"] = {"error": str(e)}

    if not args.no_extra and args.workload == "blob50_1m_d2":
        out["workloads"] = {}
        for wl, link in (("u1m_d10", "average"), ("blob100_1m_d10", "average"), ("vmf1000_200k_d128", "ward"),
                         ("vmf1000_200k_d128", "complete"), ("vmf1000_200k_d128", "average"),
                         ("vmf1000_200k_d128", "avgsq")):
            log("workload %s, %s linkage" % (wl, link))
            try:
                out["workloads"]["%s_%s" % (wl, link)] = workload_leg(pc, synth, torch, ctx, stream, wl, link)
            except Exception as e:  # reported, never hidden
                out["workloads"]["%s_%s" % (wl, link)] = {"error": str(e)}

    if not args.no_extra and not args.no_precision and args.workload == "blob50_1m_d2":
        out["precision_forms"] = precision_leg(pc, synth, torch, ctx, stream, out.get("workloads", {}))

    if not args.no_extra and args.workload == "blob50_1m_d2":
        out["paper_sets"] = paper_leg(pc, synth, torch, ctx, stream)

    if not args.no_ablations and args.workload == "blob50_1m_d2":
        try:
            out["ablations"] = ablation_leg(pc, synth, torch, ctx, stream)
        except Exception as e:  # reported, never hidden
            out["ablations"] = {"error": str(e)}

    if args.serve_requests > 0:
        try:
            out["serving"] = serve_bench(args.serve_requests, args.serve_slots, args.serve_nmax)
        except Exception as e:  # reported, never hidden
            out["serving"] = {"error": str(e)}

    if not args.no_cpu:
        import oracle

        # the FP64 oracle (sequential NN-chain, accelerated mode: grid-pruned
        # exact queries) on the first points of the headline input itself
        cores = os.cpu_count() or 1
        m = min(args.cpu_sample, n)
        log("CPU oracle baseline on the first %d points" % m)
        xs = np.ascontiguousarray(x[:m])
        tt, detail = 0.0, {}
        for link in links:
            t = time.perf_counter()
            _, cert = oracle.nnchain(xs, link, accel=True)
            dt = time.perf_counter() - t
            tt += dt
            detail[link] = {"n": m, "s": dt, "points_per_s": m / dt, "cand_evals": cert["cand_evals"],
                            "point_pair_evals": cert["pair_evals"]}
        out["cpu_baseline"] = {
            "value": m * len(links) / tt, "unit": "points/s", "cores": cores, "kind": "oracle",
            "sample": "FP64 NN-chain oracle (accelerated mode) on the first %d points of the headline "
                      "input, %s linkage; the chain is sequential (one thread), only large complete-"
                      "linkage pair maxima use the %d host threads" % (m, " + ".join(links), cores),
            "detail": detail,
        }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
