#!/usr/bin/env python3
"""FITrig hot-path benchmark on one MI355X.

One step = one fitrig_detect call over a resident synthetic stack: the whole
path (index pass, per-triple spread, N-sigma selection, 8-connected
candidates, image-frequency branch, result copies to the host).

Prints ONE JSON line: whole-job throughput in detected snapshot Mpix/s
(n * H * W / step time), p50 / p99 step latency, the roofline of the
dominant kernel (the streaming index kernel; its duration comes from HIP
events the library records on the stream it launches on) and the FP64 CPU
oracle timed on a bounded sample of the same workload.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
BYTES_IN = {"f32": 4, "f16": 2, "bf16": 2}
WORKLOAD_TEXT = {
    "c0": "256x256 px x 32 snapshots fp32, 7x7 window, tau 6",
    "c1": "4096x4096 px x 64 snapshots fp32, 7x7 window, tau 6",
    "c2": "16384x16384 px x 32 snapshots fp32, 9x9 window, tau 6",
    "c3": "50000x50000 px x 16 snapshots fp16, 9x9 window, tau 6",
}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("fitrig_device.h", "fitrig_launch.hip", "fitrig_kernels.hip", "fitrig_api.hip", "fitrig_internal.h"):
        with open(os.path.join(ROOT, "paper_2509_21754_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(workload: str):
    """HBM bytes per launch of the streaming kernel from the committed
    rocprofv3 counter summary, only if it was taken on the current source."""
    p = os.path.join(ROOT, "profiles", "k_stream_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("source_hash") != kernel_source_hash() or d.get("workload") != workload:
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_model() -> str:
    """CPU model name of this host (lscpu, else /proc/cpuinfo)."""
    import subprocess

    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(spec_name: str) -> dict:
    """The oracle as it stands, timed on bounded samples of the same recipe:
    on every host thread the process may use (the reported value) and on one
    thread (a smaller sample, scaled to the same unit)."""
    import synth
    from oracle import ref

    base = synth.WORKLOADS[spec_name]

    def run(H, W, n, threads):
        spec = synth.spec(spec_name, H=H, W=W, n=n) if (H, W, n) != (base.H, base.W, base.n) else base
        X = synth.make_stack(spec).float().numpy()
        used = ref.set_threads(threads)
        t0 = time.perf_counter()
        ref.detect(X, tau=spec.taus[0], window=spec.window, keep_maps=False)
        dt = time.perf_counter() - t0
        return n * H * W / dt / 1e6, dt, used, spec

    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = int(os.environ.get("OMP_NUM_THREADS") or threads)
    big = (4096, 2048, 12) if base.H >= 4096 else (base.H, base.W, base.n)
    small = (2048, 2048, 12) if base.H >= 4096 else (base.H, base.W, base.n)
    v_all, dt_all, used_all, spec = run(*big, threads)
    v_one, dt_one, _, _ = run(*small, 1)
    ref.set_threads(threads)
    return {"value": round(v_all, 3), "unit": "Mpix/s", "cores": used_all, "kind": "oracle",
            "sample": f"{big[0]}x{big[1]} px x {big[2]} snapshots of the {spec_name} recipe (window {spec.window}), "
                      f"full detect incl. frequency branch, {dt_all:.2f} s on {used_all} threads",
            "cpu_model": cpu_model(),
            "single_thread": {"value": round(v_one, 3), "unit": "Mpix/s", "cores": 1,
                              "sample": f"{small[0]}x{small[1]} px x {small[2]} snapshots, same recipe, "
                                        f"{dt_one:.2f} s on 1 thread"}}


def pulsar_recall(cands, spec) -> dict:
    """Share of (pulsar, trigger triple) pairs with an image-branch candidate
    whose box (grown by 2 px) holds the pulsar: a pulse in frame p triggers
    triples p-2 and p."""
    import numpy as np

    import synth

    sky = synth.sky_model(spec)
    img = cands[cands["branch"] == 1]
    by_t = {}
    for t in np.unique(img["triple"]):
        sel = img[img["triple"] == t]
        by_t[int(t)] = (sel["y0"] - 2, sel["x0"] - 2, sel["y1"] + 2, sel["x1"] + 2)
    hit = tot = 0
    for i in range(len(sky.pulsar_amp)):
        y, x = int(sky.pulsar_yx[i, 0]), int(sky.pulsar_yx[i, 1])
        for p in np.nonzero(sky.pulsar_w[i] > 0)[0]:
            for t in (int(p) - 2, int(p)):
                if 0 <= t <= spec.n - 3:
                    tot += 1
                    b = by_t.get(t)
                    if b is not None and bool(np.any((b[0] <= y) & (y <= b[2]) & (b[1] <= x) & (x <= b[3]))):
                        hit += 1
    return {"pulsar_triggers": tot, "detected": hit, "recall": round(hit / tot, 4) if tot else None}


def time_detect(ctx, stack, tau, steps, warmup, stream):
    import gc

    import torch

    # Python's cyclic collector runs before the warmup, not inside the timed
    # region (a full collection after the host-side checks of a previous leg
    # took about 40 ms in one step)
    gc.collect()
    gc.disable()
    try:
        for _ in range(warmup):
            ctx.detect(stack, tau, stream=stream, as_dicts=False)
        torch.cuda.synchronize()
        step_ms, phases = [], []
        t0 = time.perf_counter()
        for _ in range(steps):
            ts = time.perf_counter()
            cands, stats, rc = ctx.detect(stack, tau, stream=stream, as_dicts=False)
            step_ms.append((time.perf_counter() - ts) * 1e3)
            phases.append(ctx.phase_times())
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
    finally:
        gc.enable()
    return total * 1e3 / steps, step_ms, phases, cands, stats


def pctl(v, p):
    srt = sorted(v)
    return srt[min(len(srt) - 1, int(round(p * (len(srt) - 1))))]


CROP = 2048
N_CROPS = 64


def crop_origins(H: int, W: int) -> list:
    """Seeded crop origins (seeds 0..63), multiples of 16 so that the block
    structure of the window sums in a crop run lines up with the full image
    and interior q values are the full image's bit for bit."""
    import numpy as np

    out = []
    for i in range(N_CROPS):
        rng = np.random.default_rng(i)
        out.append((16 * int(rng.integers(0, (H - CROP) // 16 + 1)), 16 * int(rng.integers(0, (W - CROP) // 16 + 1))))
    return out


def _component_at(q2, mu, sg, tau, py, px):
    """The oracle's 8-connected component of {z > tau} holding (py, px)."""
    import numpy as np
    from scipy import ndimage

    from oracle import ref

    comps, mask = ref.components(q2, mu, sg, tau, with_mask=True)
    if not mask[py, px]:
        return None
    lab, _ = ndimage.label(mask, structure=np.ones((3, 3)))
    first = int(np.flatnonzero(lab.ravel() == lab[py, px])[0])
    return next(d for d in comps if d["label"] == first)


def precision_report(spec, stack, raw, origins, stats, cands) -> dict:
    """Error of the FP16-storage path against the FP64 oracle on seeded
    crops, stated twice: algorithmic (oracle on the same decoded FP16 input)
    and total (oracle on the values before rounding to FP16). q is compared on
    crop-interior cells; candidates of the full-image run that lie inside a
    crop's interior are compared with the oracle's components built with the
    full-image mean and std."""
    import numpy as np
    import torch

    from oracle import ref
    from paper_2509_21754_amd import Context

    h = spec.window // 2
    tau = spec.taus[0]
    n = spec.n
    lo, hi = h, CROP - h
    alg_rel, tot_rel = [], []
    alg_bad = 0
    cells = 0
    cand_cmp = {"checked": 0, "identical_alg": 0, "near_threshold_skipped": 0, "found_in_total": 0}
    img = cands[cands["branch"] == 1]
    t0 = time.perf_counter()
    with Context(window=spec.window) as ctx:
        for i, (oy, ox) in enumerate(origins):
            sub = stack[:, oy:oy + CROP, ox:ox + CROP].contiguous()
            qg = torch.empty((n - 2, CROP, CROP), dtype=torch.float32, device=sub.device)
            ctx.detect(sub, tau, index_map=qg, as_dicts=False)
            qg = qg[:, lo:hi, lo:hi].cpu().numpy().astype(np.float64)
            dec = sub.float().cpu().numpy()
            pre = raw[i].cpu().numpy()
            qd = ref.index_maps(dec, window=spec.window)[:, lo:hi, lo:hi]
            qt = ref.index_maps(pre, window=spec.window)[:, lo:hi, lo:hi]
            for s in range(n - 2):
                atol = 1e-7 * float(qd[s].mean())
                e_alg = np.abs(qg[s] - qd[s]) / (np.abs(qd[s]) + atol)
                e_tot = np.abs(qg[s] - qt[s]) / (np.abs(qt[s]) + atol)
                alg_bad += int(np.count_nonzero(np.abs(qg[s] - qd[s]) > 1e-5 * np.abs(qd[s]) + atol))
                alg_rel.append(np.quantile(e_alg, [0.5, 0.99, 1.0]))
                tot_rel.append(np.quantile(e_tot, [0.5, 0.99, 1.0]))
                cells += qd[s].size
            # candidates of the full-image run inside this crop's interior
            inside = img[(img["y0"] >= oy + lo + 1) & (img["y1"] < oy + hi - 1) &
                         (img["x0"] >= ox + lo + 1) & (img["x1"] < ox + hi - 1)]
            for c in inside:
                s = int(c["triple"])
                mu, sg = stats["mu"][s], stats["sigma"][s]
                # the candidate's box grown by one cell, in interior coordinates
                y0, y1 = int(c["y0"]) - oy - lo - 1, int(c["y1"]) - oy - lo + 2
                x0, x1 = int(c["x0"]) - ox - lo - 1, int(c["x1"]) - ox - lo + 2
                if np.any(np.abs((qd[s][y0:y1, x0:x1] - mu) / sg - tau) <= 1e-4):
                    cand_cmp["near_threshold_skipped"] += 1
                    continue
                cand_cmp["checked"] += 1
                py, px = int(c["peak_y"]) - oy - lo - y0, int(c["peak_x"]) - ox - lo - x0
                d = _component_at(qd[s][y0:y1, x0:x1], mu, sg, tau, py, px)
                if d is not None and (d["n_pix"], d["y0"] + y0, d["x0"] + x0, d["y1"] + y0, d["x1"] + x0,
                                      d["peak_y"], d["peak_x"]) == (
                        int(c["n_pix"]), int(c["y0"]) - oy - lo, int(c["x0"]) - ox - lo, int(c["y1"]) - oy - lo,
                        int(c["x1"]) - ox - lo, py, px):
                    cand_cmp["identical_alg"] += 1
                if _component_at(qt[s][y0:y1, x0:x1], mu, sg, tau, py, px) is not None:
                    cand_cmp["found_in_total"] += 1
            if (i + 1) % 8 == 0:
                print(f"[bench] precision report: {i + 1}/{len(origins)} crops, {time.perf_counter() - t0:.0f} s",
                      file=sys.stderr, flush=True)
    A = np.array(alg_rel)
    T = np.array(tot_rel)
    return {
        "crops": f"{len(origins)} seeded {CROP}x{CROP} crops (seeds 0..{len(origins) - 1}), interior cells",
        "cells": cells,
        "q_algorithmic_rel_err": {"median": float(np.median(A[:, 0])), "p99": float(np.max(A[:, 1])),
                                  "max": float(np.max(A[:, 2])), "cells_outside_tolerance": alg_bad},
        "q_total_rel_err": {"median": float(np.median(T[:, 0])), "p99": float(np.max(T[:, 1])),
                            "max": float(np.max(T[:, 2]))},
        "candidates": cand_cmp,
    }


def serving_replay(n_req: int, slots: int, rate_hz: float, budget_gib: float, dev, freq_window: int = 30) -> dict:
    """The serving workload: Poisson arrivals of snapshot stacks of 16 fields
    (size class 2048^2 / 4096^2 / 8192^2 and storage dtype fixed per field,
    16 / 32 / 128 snapshots per request) replayed in real time through the
    server, then the same requests submitted at once (capacity). Each
    request's frequency branch covers its field's last freq_window triples."""
    import numpy as np
    import torch

    import synth
    from paper_2509_21754_amd import Server

    reqs = synth.serving_requests(n_req, rate_hz=rate_hz)
    n_pool = max(r["n"] for r in reqs)
    pools = {}
    for i, size in enumerate(sorted({r["size"] for r in reqs})):
        sp = synth.scaled(synth.WORKLOADS["c1"], size, size, n=n_pool, seed=1004 * 10 + i)
        base = synth.make_stack(sp, device=dev)
        for dt in sorted({r["dtype"] for r in reqs if r["size"] == size}):
            pools[(size, dt)] = base if dt == "f32" else base.to(torch.float16)
        if ("f32" not in {r["dtype"] for r in reqs if r["size"] == size}):
            del base
    torch.cuda.synchronize()
    print(f"[bench] serving pools ready: {sorted(pools)}", file=sys.stderr, flush=True)
    max_px = max(r["size"] for r in reqs) ** 2

    def run(realtime: bool):
        cursor = {}
        with Server(n_slots=slots, max_fields=32, mem_budget=int(budget_gib * (1 << 30)), window=7,
                    max_pixels=max_px, max_snap=n_pool + 2, freq_window=freq_window) as srv:
            # warm every slot and size class outside the timed part (fields 100+)
            for j, key in enumerate(sorted(pools)):
                tk = srv.submit(100 + j, pools[key][:3], 6.0)
                srv.poll(tk)
                srv.release(tk)
            tickets = []
            t0 = time.perf_counter()
            for r in reqs:
                if realtime:
                    dt = t0 + r["t"] - time.perf_counter()
                    if dt > 0:
                        time.sleep(dt)
                pool = pools[(r["size"], r["dtype"])]
                c = cursor.get(r["field"], 0)
                if c + r["n"] > n_pool:
                    c = 0
                cursor[r["field"]] = c + r["n"]
                tickets.append((srv.submit(r["field"], pool[c:c + r["n"]], 6.0), r))
            res = []
            for tk, r in tickets:
                o = srv.poll(tk, as_dicts=False)
                res.append((o, r))
                srv.release(tk)
            wall = time.perf_counter() - t0
        return res, wall

    out = {"requests": n_req, "rate_hz": rate_hz, "slots": slots, "mem_budget_gib": budget_gib,
           "fields": 16, "window": 7, "tau": 6.0, "freq_window": freq_window}
    for mode in ("realtime", "saturated"):
        res, wall = run(mode == "realtime")
        bad = [o["status"] for o, _ in res if o["status"] not in (0, -4)]
        lat = [(o["t_done_ns"] - o["t_submit_ns"]) / 1e6 for o, _ in res]
        wait = [(o["t_start_ns"] - o["t_submit_ns"]) / 1e6 for o, _ in res]
        first = min(o["t_submit_ns"] for o, _ in res)
        last = max(o["t_done_ns"] for o, _ in res)
        px = sum(r["n"] * r["size"] ** 2 for _, r in res)
        d = {"mpix_s": round(px / ((last - first) / 1e9) / 1e6, 1), "wall_s": round(wall, 3),
             "p50_ms": round(pctl(lat, 0.5), 3), "p99_ms": round(pctl(lat, 0.99), 3),
             "queue_wait_p50_ms": round(pctl(wait, 0.5), 3), "errors": len(bad),
             "freq_branch_runs": sum(1 for o, _ in res if o["freq_triples"] > 0),
             "graph_replays": sum(1 for o, _ in res if o.get("replayed"))}
        for dt in ("f16", "f32"):
            l2 = [x for x, (_, r) in zip(lat, res) if r["dtype"] == dt]
            pxd = [r["n"] * r["size"] ** 2 for _, r in res if r["dtype"] == dt]
            if l2:
                d[dt] = {"requests": len(l2), "p50_ms": round(pctl(l2, 0.5), 3), "p99_ms": round(pctl(l2, 0.99), 3),
                         "mean_mpix": round(float(np.mean(pxd)) / 1e6, 1)}
        out[mode] = d
        print(f"[bench] serving {mode}: {d}", file=sys.stderr, flush=True)
    del pools
    torch.cuda.empty_cache()
    return out


def localisation(ctx, stack, tau: float, spec, stream) -> dict:
    """Sub-cell localisation of the frequency-branch candidates on the eta map
    (spline, 1/16-cell grid), timed with events on the launch stream; one
    detect call outside the timed steps supplies eta and the candidates."""
    import numpy as np
    import torch

    from paper_2509_21754_amd import INTERP_SPLINE, interp_peaks

    tile = ctx.cfg.tile
    eta = torch.zeros(((spec.H + tile - 1) // tile, (spec.W + tile - 1) // tile), dtype=torch.float32,
                      device=stack.device)
    cands, _, _ = ctx.detect(stack, tau, eta_map=eta, as_dicts=False)
    fq = cands[cands["branch"] == 2]
    peaks = np.stack([fq["peak_y"], fq["peak_x"]], axis=1) if len(fq) else np.zeros((0, 2), np.int32)
    with torch.cuda.stream(stream):
        interp_peaks(eta, peaks, method=INTERP_SPLINE, sub=16, stream=stream)
        ms = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            interp_peaks(eta, peaks, method=INTERP_SPLINE, sub=16, stream=stream)
            e1.record(stream)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
    return {"peaks": int(len(peaks)), "method": "spline", "grid": "1/16 cell", "map": f"eta {tuple(eta.shape)}",
            "ms_per_call": round(statistics.median(ms), 4),
            "us_per_peak": round(statistics.median(ms) * 1e3 / max(len(peaks), 1), 3)}


def paper_workload(dev, harm: int) -> dict:
    """The shape of the paper's real-data run (Sec. 3.2: 1500 snapshots of
    4096 x 4096, tiles of 32, the image-frequency branch with a harmonic sum,
    spline localisation of the frequency candidates), on a synthetic stack
    resident in HBM: wall time of one detect call plus the localisation."""
    import numpy as np
    import torch

    import synth
    from paper_2509_21754_amd import INTERP_SPLINE, Context, interp_peaks

    spec = synth.StackSpec("paper", 4096, 4096, 1500, "f32", 9, (6.0,), n_steady=200, n_pulsar=10,
                           pulsar_kind="periodic", period_range=(20, 60), seed=1010)
    print("[bench] generating the paper-shaped stack: 1500x4096x4096 f32", file=sys.stderr, flush=True)
    stack = synth.make_stack(spec, device=dev)
    torch.cuda.synchronize()
    n, H, W, tile = spec.n, spec.H, spec.W, 32
    ctx = Context(window=spec.window, profile=1, max_pixels=H * W, max_snap=n, mode=1, tile=tile, branches=3,
                  harm=harm)
    eta = torch.zeros(((H + tile - 1) // tile, (W + tile - 1) // tile), dtype=torch.float32, device=dev)
    tau = spec.taus[0]

    def once():
        t0 = time.perf_counter()
        cands, stats, rc = ctx.detect(stack, tau, eta_map=eta, as_dicts=False)
        t1 = time.perf_counter()
        fq = cands[cands["branch"] == 2]
        peaks = np.stack([fq["peak_y"], fq["peak_x"]], axis=1) if len(fq) else np.zeros((0, 2), np.int32)
        loc = interp_peaks(eta, peaks, method=INTERP_SPLINE, sub=16)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1, cands, stats, rc, len(peaks)

    print("[bench] timing the paper-shaped run", file=sys.stderr, flush=True)
    once()  # warm
    runs = [once() for _ in range(3)]
    td = statistics.median(r[0] for r in runs)
    tl = statistics.median(r[1] for r in runs)
    _, _, cands, stats, rc, npk = runs[-1]
    ph = ctx.phase_times()
    # the same run from pageable host memory (the stack cannot be page-locked
    # whole): chunks of 8 frames staged and copied over PCIe under the path
    hp = stack.cpu()
    del stack
    torch.cuda.empty_cache()
    print("[bench] timing the paper-shaped run from pageable host memory", file=sys.stderr, flush=True)
    th = []
    for _ in range(2):
        t0 = time.perf_counter()
        ch, sth, rch = ctx.detect_host(hp, tau, 8, eta_map=eta, as_dicts=False)
        fq = ch[ch["branch"] == 2]
        pk = np.stack([fq["peak_y"], fq["peak_x"]], axis=1) if len(fq) else np.zeros((0, 2), np.int32)
        interp_peaks(eta, pk, method=INTERP_SPLINE, sub=16)
        torch.cuda.synchronize()
        th.append(time.perf_counter() - t0)
    del hp
    ctx.close()
    px = n * H * W
    torch.cuda.empty_cache()
    return {"workload": "1500 x 4096 x 4096 fp32 snapshots (synthetic, 10 periodic pulsars of 20-60 frames), "
                        f"tiles of 32, image + frequency branches, harmonic sum of {harm}, spline localisation",
            "stack_gb": round(px * 4 / 1e9, 2), "ms_detect": round(td * 1e3, 2),
            "ms_localise": round(tl * 1e3, 3), "ms_end_to_end": round((td + tl) * 1e3, 2),
            "mpix_s": round(px / (td + tl) / 1e6, 1), "status": rc, "n_candidates": stats["n_cand"],
            "frequency_candidates_localised": npk,
            "phase_ms": {k: round(v, 3) for k, v in ph.items()} if isinstance(ph, dict) else ph,
            "from_pageable_host": {"ms_end_to_end": round(min(th) * 1e3, 1), "status": rch,
                                   "n_candidates": sth["n_cand"], "same_candidates": sth["n_cand"] == stats["n_cand"],
                                   "h2d_gbs": round(px * 4 / min(th) / 1e9, 2)},
            "note": "stack resident in HBM (and, separately, in pageable host memory); the paper's 6.34 s (H100) "
                    "is timed from image loading to positions"}


# largest stack the host-streaming measurement copies into page-locked memory
HOST_STREAM_MAX_GIB = 48


def host_stream(ctx, stack, tau: float, chunk: int, steps: int, ref_n_cand: int) -> dict:
    """The same stack from page-locked host memory, streamed to the device in
    chunks of frames (the copy of the next chunk overlaps the path over the
    current one), against the plain host-to-device copy rate of the link."""
    import torch

    n, H, W = stack.shape
    h = torch.empty(stack.shape, dtype=stack.dtype, pin_memory=True)
    h.copy_(stack)
    torch.cuda.synchronize()
    # ceiling: plain pinned host-to-device copies of one chunk
    d = torch.empty((chunk, H, W), dtype=stack.dtype, device=stack.device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    d.copy_(h[:chunk], non_blocking=True)
    e0.record()
    reps = max(1, n // chunk)
    for i in range(reps):
        d.copy_(h[i * chunk:(i + 1) * chunk], non_blocking=True)
    e1.record()
    torch.cuda.synchronize()
    chunk_bytes = chunk * H * W * stack.element_size()
    ceil_gbs = reps * chunk_bytes / (e0.elapsed_time(e1) / 1e3) / 1e9
    del d
    ctx.detect_host(h, tau, chunk, as_dicts=False)  # warm
    times, ncand = [], None
    for _ in range(steps):
        t0 = time.perf_counter()
        c, st, rc = ctx.detect_host(h, tau, chunk, as_dicts=False)
        times.append(time.perf_counter() - t0)
        ncand = st["n_cand"]
    t = statistics.median(times)
    total = n * H * W * stack.element_size()
    del h
    torch.cuda.synchronize()
    # the same stack in pageable memory: staged by the library's host threads
    hp = stack.cpu()
    ctx.detect_host(hp, tau, chunk, as_dicts=False)  # warm
    tp, ncp = [], None
    for _ in range(steps):
        t0 = time.perf_counter()
        c, st, rc = ctx.detect_host(hp, tau, chunk, as_dicts=False)
        tp.append(time.perf_counter() - t0)
        ncp = st["n_cand"]
    del hp
    tpm = statistics.median(tp)
    return {"value": round(n * H * W / t / 1e6, 1), "unit": "Mpix/s", "ms_per_step": round(t * 1e3, 2),
            "chunk_frames": chunk, "steps": steps, "h2d_gbs": round(total / t / 1e9, 2),
            "h2d_copy_ceiling_gbs": round(ceil_gbs, 2), "frac_of_copy_ceiling": round(total / t / 1e9 / ceil_gbs, 3),
            "n_candidates": ncand, "same_candidate_count_as_device": ncand == ref_n_cand,
            "pageable": {"value": round(n * H * W / tpm / 1e6, 1), "ms_per_step": round(tpm * 1e3, 2),
                         "h2d_gbs": round(total / tpm / 1e9, 2), "same_candidate_count_as_device": ncp == ref_n_cand,
                         "note": "pageable host memory, staged through page-locked buffers by host threads"},
            "note": "stack in page-locked host memory; wall time of fitrig_detect_host (median)"}


def prefix_report(ctx, stack, tau: float, window: int, n_cells: int = 2000) -> dict:
    """The window sums of the headline stack read from full-image prefix sums
    (FP64 and FP32 integral images, the comparison variant) against the
    direct sums of the timed path, both against the FP64 oracle at seeded
    sampled cells (each evaluated on a crop holding its clipped window)."""
    import numpy as np
    import torch

    from oracle import ref
    from paper_2509_21754_amd import index_prefix

    n, H, W = stack.shape
    h = window // 2
    rng = np.random.default_rng(77)
    cells = np.stack([rng.integers(0, n - 2, n_cells), rng.integers(0, H, n_cells), rng.integers(0, W, n_cells)], 1)
    cells[:4] = [[0, 0, 0], [n - 3, H - 1, W - 1], [0, 0, W - 1], [n - 3, H - 1, 0]]
    want = []
    for s, y, x in cells:
        ya, yb, xa, xb = max(0, y - h), min(H, y + h + 1), max(0, x - h), min(W, x + h + 1)
        X = stack[s:s + 3, ya:yb, xa:xb].float().cpu().numpy()
        want.append(ref.index_cells(X, [[0, y - ya, x - xa]], window=window)[0])
    want = np.array(want)
    q = torch.empty((n - 2, H, W), dtype=torch.float32, device=stack.device)
    out = {"cells": f"{n_cells} seeded cells (corners and random), oracle on crops holding each window"}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for name in ("direct_fp32", "prefix_fp64", "prefix_fp32"):
        for rep in range(2):  # the second run is timed (the first sizes scratch)
            e0.record()
            if name == "direct_fp32":
                ctx.detect(stack, tau, index_map=q)
            else:
                index_prefix(stack, window, 64 if name == "prefix_fp64" else 32, out=q)
            e1.record()
            torch.cuda.synchronize()
        torch.cuda.synchronize()
        g = q[torch.from_numpy(cells[:, 0]).to(q.device), torch.from_numpy(cells[:, 1]).to(q.device),
              torch.from_numpy(cells[:, 2]).to(q.device)].double().cpu().numpy()
        rel = np.abs(g - want) / np.maximum(np.abs(want), 1e-30)
        out[name] = {"ms_whole_call": round(e0.elapsed_time(e1), 2), "rel_err_median": float(np.median(rel)),
                     "rel_err_p99": float(np.quantile(rel, 0.99)), "rel_err_max": float(rel.max()),
                     "cells_over_1e-5": int((rel > 1e-5).sum())}
    del q
    torch.cuda.empty_cache()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sigma-est", default="mean_std", choices=("mean_std", "median_mad"))
    ap.add_argument("--mode", default="sliding", choices=("sliding", "tiles"),
                    help="sliding window (per pixel) or the paper's tiles")
    ap.add_argument("--tile", type=int, default=32, help="tile size (tile mode and frequency branch)")
    ap.add_argument("--no-fp16-form", action="store_true", help="skip the FP16-storage run of the same stack")
    ap.add_argument("--freq-pixel", action="store_true",
                    help="add the per-pixel frequency branch (spectrum of every pixel's q series)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving replay")
    ap.add_argument("--no-precision-report", action="store_true",
                    help="skip the crop error report of an FP16 / BF16 workload")
    ap.add_argument("--serving-requests", type=int, default=200)
    ap.add_argument("--serving-slots", type=int, default=4)
    ap.add_argument("--serving-budget-gib", type=float, default=48.0)
    ap.add_argument("--serving-freq-window", type=int, default=30,
                    help="triples of a field's history the frequency branch covers (0 = the request's own)")
    ap.add_argument("--prefix-report", action="store_true",
                    help="also compare the window sums from FP64 / FP32 prefix sums with the direct ones")
    ap.add_argument("--no-host-stream", action="store_true",
                    help="skip the run of the same stack streamed from host memory")
    ap.add_argument("--host-chunk", type=int, default=4, help="frames per host-to-device chunk")
    ap.add_argument("--paper-workload", type=int, default=0, metavar="HARM",
                    help="also time the paper's real-data run shape (1500 x 4096^2, tiles of 32, frequency branch "
                         "with a harmonic sum of HARM terms, spline localisation)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (scale for rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        return 2

    import torch

    import synth
    from paper_2509_21754_amd import Context

    spec = synth.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print(f"[bench] generating {args.workload}: {spec.n}x{spec.H}x{spec.W} {spec.dtype}", file=sys.stderr,
          flush=True)
    raw = origins = None
    if spec.dtype != "f32" and not args.no_precision_report:
        # keep crops of the values before rounding to the storage dtype
        origins = crop_origins(spec.H, spec.W)
        raw = torch.empty((len(origins), spec.n, CROP, CROP), dtype=torch.float32, device=dev)

        def grab(k, frame):
            for i, (oy, ox) in enumerate(origins):
                raw[i, k].copy_(frame[oy:oy + CROP, ox:ox + CROP])
    stack = synth.make_stack(spec, device=dev, on_frame=grab if raw is not None else None)
    torch.cuda.synchronize()
    if args.calibrate_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    tau = spec.taus[0]
    n, H, W = spec.n, spec.H, spec.W
    est = {"mean_std": 0, "median_mad": 1}[args.sigma_est]
    mode = {"sliding": 0, "tiles": 1}[args.mode]
    branches = 3 | (4 if args.freq_pixel else 0)
    ctx = Context(window=spec.window, profile=1, max_pixels=H * W, max_snap=n, sigma_est=est, mode=mode,
                  tile=args.tile, branches=branches)
    stream = torch.cuda.current_stream(dev)
    print(f"[bench] timing {args.steps} steps after {args.warmup} warmup", file=sys.stderr, flush=True)
    ms_per_step, step_ms, phases, cands, stats = time_detect(ctx, stack, tau, args.steps, args.warmup, stream)
    kern_ms = [p["index_pass"] for p in phases]
    px = n * H * W
    value = px / (ms_per_step / 1e3) / 1e6
    kmean = statistics.mean(kern_ms)
    alg_bytes = px * BYTES_IN[spec.dtype]
    achieved = alg_bytes / (kmean / 1e3) / 1e9
    traffic = stored_traffic(args.workload) if args.mode == "sliding" else None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "k_stream (streaming index pass)" if args.mode == "sliding" else "k_tile (tile-mode pass)",
            "kernel_ms": round(kmean, 4),
            "alg_bytes_per_launch": alg_bytes}
    phase_mean = {k: round(statistics.mean(p[k] for p in phases), 4) for k in phases[0]}
    out = {
        "metric": "detected snapshot Mpix/s",
        "value": round(value, 1),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": spec.dtype,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOAD_TEXT[args.workload]}", "n_snap": n, "H": H, "W": W,
                   "window": spec.window, "tau": tau, "branches": "image+freq" + ("+freq_pixel" if args.freq_pixel else ""), "sigma_est": args.sigma_est,
                   "mode": args.mode, "tile": args.tile},
        "hbm_peak_frac_whole_step": round(px * BYTES_IN[spec.dtype] / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "p50_ms": round(statistics.median(step_ms), 4),
        "p99_ms": round(pctl(step_ms, 0.99), 4),
        "phase_ms": phase_mean,
        "n_candidates": stats["n_cand"],
        "roofline": roof,
    }
    if spec.dtype == "f32" and not args.no_fp16_form:
        # the precision form on the same stack: FP16 storage (round to nearest
        # even), FP32 arithmetic; detection accuracy on the injected pulsars
        acc32 = pulsar_recall(cands, spec)
        s16 = stack.to(torch.float16)
        torch.cuda.synchronize()
        print("[bench] timing the FP16-storage form", file=sys.stderr, flush=True)
        ms16, st16, ph16, c16, stats16 = time_detect(ctx, s16, tau, args.steps, args.warmup, stream)
        k16 = statistics.mean(p["index_pass"] for p in ph16)
        a16 = px * 2 / (k16 / 1e3) / 1e9
        keys32 = set(zip(cands["branch"].tolist(), cands["triple"].tolist(), cands["label"].tolist()))
        keys16 = set(zip(c16["branch"].tolist(), c16["triple"].tolist(), c16["label"].tolist()))
        out["fp16_form"] = {
            "value": round(px / (ms16 / 1e3) / 1e6, 1), "unit": "Mpix/s", "ms_per_step": round(ms16, 4),
            "p50_ms": round(statistics.median(st16), 4), "p99_ms": round(pctl(st16, 0.99), 4),
            "roofline": {"bound": "hbm", "achieved": round(a16, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(a16 / HBM_PEAK_GBS, 4), "kernel_ms": round(k16, 4)},
            "n_candidates": stats16["n_cand"], "pulsar_recall_fp32": acc32,
            "pulsar_recall_fp16": pulsar_recall(c16, spec),
            "candidates_shared_with_fp32": len(keys32 & keys16),
        }
        del s16
    if args.mode == "sliding":
        out["localisation"] = localisation(ctx, stack, tau, spec, stream)
    if args.prefix_report and args.mode == "sliding":
        print("[bench] prefix-sum comparison", file=sys.stderr, flush=True)
        out["prefix_report"] = prefix_report(ctx, stack, tau, spec.window)
    stack_gib = stack.numel() * stack.element_size() / 2**30
    if not args.no_host_stream and stack_gib > HOST_STREAM_MAX_GIB:
        out["host_stream"] = {"skipped": f"stack of {stack_gib:.1f} GiB exceeds the {HOST_STREAM_MAX_GIB} GiB "
                                         "page-locked host copy this run allocates"}
    elif not args.no_host_stream:
        print("[bench] streaming the stack from host memory", file=sys.stderr, flush=True)
        out["host_stream"] = host_stream(ctx, stack, tau, args.host_chunk, 3, stats["n_cand"])
    if raw is not None:
        print("[bench] precision report on crops", file=sys.stderr, flush=True)
        out["precision_report"] = precision_report(spec, stack, raw, origins, stats, cands)
        del raw
    ctx.close()
    del stack
    torch.cuda.empty_cache()
    if args.paper_workload > 0:
        out["paper_workload"] = paper_workload(dev, args.paper_workload)
    if not args.no_serving:
        print("[bench] serving replay", file=sys.stderr, flush=True)
        out["serving"] = serving_replay(args.serving_requests, args.serving_slots, 40.0, args.serving_budget_gib, dev,
                                        args.serving_freq_window)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
