"""Throughput of the SFFT differencing hot path on one MI355X.

A step is one pass of the whole path over one synthetic DECam-CCD-shaped
pair (2048 x 4096 FP32 images, L = 11, DK = 2, DB = 2, N = 732 unknowns):
sfft_build_system + sfft_solve (FP64, 1 refinement step) + sfft_subtract
with the chi2 judge. Inputs are resident in HBM before the timed region.

The plain form is timed twice: one pair at a time (serial_pairs_per_s, the
per-pair latency, and the per-kernel events behind phase_us and the
rooflines), then over a queue of different pairs with three in flight on
separate streams (value: the throughput of differencing a queue of CCD
pairs, as the paper's pipeline does per GPU). `--serial` skips the second.

The default run prints one JSON line for the plain form and adds, measured in
the same process, the precision form (FP32 spectra), the batched form (one
exposure of 60 CCD pairs and 40 cutouts from one HIP graph), the stamp form
and the learned form (gated network inference with the chi2 fallback), each
counted only when every pair it differenced ends at chi2 <= 1.05.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "CCD pairs differenced/sec (2048×4096, L=11, DK=2) plain vs batched/surrogate"
# pairs in flight and solve team of the pipelined plain path (measured best
# on MI355X among depths 1..3 and teams 16..128)
PIPE_DEPTH, PIPE_TEAM = 3, 32
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VALU_TFLOPS = 78.6        # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
W, H, L, DK, DB = 2048, 4096, 11, 2, 2


# ---------------------------------------------------------------------------
# HIP events through the runtime's C API (timings on the library's stream)
# ---------------------------------------------------------------------------
def _loaded_hip_runtime() -> str:
    """Path of the HIP runtime already mapped into this process (the one torch
    and the SFFT library use), so that events live in the same runtime."""
    with open("/proc/self/maps") as f:
        for line in f:
            path = line.split()[-1]
            if "libamdhip64.so" in path:
                return path
    return "libamdhip64.so"


class HipEvents:
    def __init__(self):
        self.hip = ctypes.CDLL(_loaded_hip_runtime())
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                 ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.made = []

    def create(self):
        e = ctypes.c_void_p()
        rc = self.hip.hipEventCreate(ctypes.byref(e))
        if rc != 0:
            raise RuntimeError(f"hipEventCreate failed ({rc})")
        self.made.append(e)
        return e

    def elapsed_ms(self, a, b):
        ms = ctypes.c_float()
        rc = self.hip.hipEventElapsedTime(ctypes.byref(ms), a, b)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return float(ms.value)

    def close(self):
        for e in self.made:
            self.hip.hipEventDestroy(e)
        self.made = []


# ---------------------------------------------------------------------------
# algorithmic work per launch at this workload
# ---------------------------------------------------------------------------
def n_unknowns():
    return (DK + 1) * (DK + 2) // 2 * L * L + (DB + 1) * (DB + 2) // 2


def algorithmic_work(fp32=False):
    """Algorithmic bytes and flops per launch; fp32: the precision form's
    FP32 spectra (half the spectra bytes)."""
    npix = W * H
    nkx = W // 2 + 1
    nsig = DK + 2
    nk = (DK + 1) * (DK + 2) // 2
    npairs = nk * (nk + 1) // 2 + nk
    h = L - 1
    T = 128 - 2 * h
    nblocks = -(-H // T)
    cplx64 = 16
    cspec = 8 if fp32 else 16
    N = n_unknowns()
    row_bytes = 2 * npix * 4 + nsig * H * nkx * cspec
    row_flops = H * (-(-nsig // 2)) * 5 * W * 11
    col_bytes = nsig * H * nkx * cspec + npairs * (2 * h + 1) * nkx * cplx64
    col_flops = nkx * (nblocks * ((2 * nk + 1) * 5 * 128 * 7 + npairs * 128 * 8) + npairs * 5 * 128 * 7)
    sub_bytes = 3 * npix * 4
    sub_flops = npix * 2 * (L * L * (DK + 1))
    # Cholesky N^3/3, two triangular solves and one refinement step
    # (residual product + two triangular solves): N^3/3 + 6 N^2 flops; reads G
    solve_flops = N ** 3 // 3 + 6 * N * N
    solve_bytes = N * N * 8 + 3 * N * 8
    return {
        "row_pass": dict(bytes=row_bytes, flops=row_flops, bound="hbm"),
        "col_pass": dict(bytes=col_bytes, flops=col_flops, bound="alu"),
        "solve": dict(bytes=solve_bytes, flops=solve_flops, bound="mfma"),
        "subtract": dict(bytes=sub_bytes, flops=sub_flops, bound="alu"),
    }


def roofline_entry(name, avg_s, traffic, fp32=False):
    w = algorithmic_work(fp32)[name]
    base = {"kernel": name, "traffic": traffic, "avg_us": round(avg_s * 1e6, 2), "alg_bytes": w["bytes"],
            "alg_flops": w["flops"]}
    if w["bound"] == "hbm":
        ach = w["bytes"] / avg_s / 1e9
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), **base}
    ach = w["flops"] / avg_s / 1e12
    out = {"bound": w["bound"], "achieved": round(ach, 3), "peak": FP64_VALU_TFLOPS, "unit": "TFLOP/s",
           "frac": round(ach / FP64_VALU_TFLOPS, 5), **base}
    if name == "solve":
        # FP64 tile products on the matrix cores (their FP64 peak equals the
        # vector one); the kernel is bound by its chain of N dependent pivots
        out["note"] = (f"latency-bound: {n_unknowns()} dependent pivot steps; HBM floor "
                       f"{w['bytes'] / HBM_PEAK_GBS / 1e3:.2f} us, FP64 floor "
                       f"{w['flops'] / FP64_VALU_TFLOPS / 1e6:.2f} us")
    return out


def build_roofline(build_s, fp32=False):
    """The whole system build (sfft_build_system, every kernel from the row
    moments to the gather) against the HBM roofline: algorithmic bytes =
    images read once, row spectra written and read back, column strips
    written and read back, normal matrix written."""
    npix = W * H
    nkx = W // 2 + 1
    nsig = DK + 2
    nk = (DK + 1) * (DK + 2) // 2
    npairs = nk * (nk + 1) // 2 + nk
    N = n_unknowns()
    cspec = 8 if fp32 else 16
    b = (2 * npix * 4 + 2 * nsig * H * nkx * cspec + 2 * npairs * (2 * (L - 1) + 1) * nkx * 16
         + N * N * 8)
    ach = b / build_s / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "alg_bytes": b, "build_us": round(build_s * 1e6, 2)}


def load_traffic(kernel):
    """HBM bytes per launch from committed rocprofv3 counter summaries, or
    None when absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        rec = json.load(open(path))[kernel]
    except Exception:
        return None
    src = os.path.join(ROOT, "paper_2603_08593_amd", "csrc", rec["source"])
    try:
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    return rec["bytes_per_launch"] if digest == rec.get("source_sha256_16") else None


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on a bounded sample of the same workload
# ---------------------------------------------------------------------------
def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return {i.get("internal_api", "?"): i.get("num_threads") for i in threadpool_info()}
    except Exception:
        return None


def cpu_baseline(pair, reps=3):
    """Median of `reps` runs of each oracle step: FFT normal equations and
    Cholesky on the full pair, direct subtraction on a 2048 x 256 crop scaled
    to the full height."""
    import statistics
    import numpy as np
    import oracle as O
    rows = 256
    Rc = np.ascontiguousarray(pair.R[:rows])
    Sc = np.ascontiguousarray(pair.S[:rows])
    tb, ts, tsub = [], [], []
    t_start = time.perf_counter()
    for _ in range(reps):
        t0 = time.perf_counter()
        G, h = O.build_fft64(pair.R, pair.S, L, DK, DB)
        t1 = time.perf_counter()
        theta, _ = O.solve_cholesky64(G, h, refine=1)
        t2 = time.perf_counter()
        O.subtract64(Rc, Sc, theta, L, DK, DB)
        t3 = time.perf_counter()
        tb.append(t1 - t0)
        ts.append(t2 - t1)
        tsub.append(t3 - t2)
    b, s, u = statistics.median(tb), statistics.median(ts), statistics.median(tsub)
    per_pair = b + s + u * (H / rows)
    aff = len(os.sched_getaffinity(0))
    return {"value": round(1.0 / per_pair, 5), "unit": "CCD pairs/s", "cores": aff,
            "kind": "oracle",
            "sample": (f"FP64 oracle on the 2048x4096 pair, median of {reps}: FFT normal equations {b:.2f} s "
                       f"and Cholesky + 1 refinement step {s:.2f} s on the full pair, direct 121-tap "
                       f"subtraction on a 2048x{rows} crop {u:.2f} s scaled x{H // rows}"),
            "cpu_model": _cpu_model(), "os_cpu_count": os.cpu_count(), "affinity_cpus": aff,
            "fft_workers": os.cpu_count(), "blas_threads": _blas_threads(),
            "seconds_measured": round(time.perf_counter() - t_start, 2)}


def _ok(info_status, chis):
    return info_status == 0 and all(c <= 1.05 for c in chis)


# ---------------------------------------------------------------------------
# forms
# ---------------------------------------------------------------------------
def run_plain(R, S, pair, steps, warmup, compute="fp64"):
    """Plain (FP64 build and solve) or precision (compute="fp32": FP32
    spectra with the FP64 image means as pedestals) form on one pair."""
    import numpy as np
    import torch
    import paper_2603_08593_amd as sf
    peds = (0.0, 0.0)
    if compute == "fp32":
        peds = (float(np.mean(pair.R, dtype=np.float64)), float(np.mean(pair.S, dtype=np.float64)))
    d = sf.Differencer(W, H, L, DK, DB, image_dtype="float32", compute=compute,
                       ref_pedestal=peds[0], sci_pedestal=peds[1])
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        d.run(R, S, max_refine=1, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        d.run(R, S, max_refine=1, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-kernel durations: the same steps again with the library recording
    # HIP events around each kernel on the launch stream
    ev = HipEvents()
    slots = {"row_pass": 1, "col_pass": 2, "xinv": 3, "subtract": 4, "solve": 5, "build": 6}
    evs = {k: [(ev.create(), ev.create()) for _ in range(steps)] for k in slots}
    lib = sf.lib()
    for k in range(steps):
        for name, slot in slots.items():
            a, b = evs[name][k]
            lib.sfft_profile_events(d.handle.ptr, slot, a, b)
        d.run(R, S, max_refine=1, stream=stream)
    torch.cuda.synchronize()
    for slot in slots.values():
        lib.sfft_profile_events(d.handle.ptr, slot, None, None)
    avg = {name: sum(ev.elapsed_ms(a, b) for a, b in evs[name]) / steps / 1e3 for name in slots}
    ev.close()
    info = d.info()
    chi2 = float(d.buf.chi2.item())
    d.close()
    ok = _ok(info.status, [chi2])
    return dict(value=(steps / (t1 - t0)) if ok else 0.0, ms=(t1 - t0) * 1e3 / steps, avg=avg, chi2=chi2,
                info=info, peds=peds)


def run_pipelined(inputs, steps, warmup, compute="fp64", depth=PIPE_DEPTH, team=PIPE_TEAM):
    """The plain (or precision) path over a queue of pairs with `depth` pairs
    in flight: each slot has its own stream, handle, workspace and buffers,
    and the solves run with a team of `team` workgroups so that the other
    slots' builds and subtracts use the rest of the chip. inputs: list of
    (R, S, pedestals) resident on the device; step k differences input
    k % len(inputs) (so with len(inputs) == depth every slot always sees the
    same pair, and its final results stand for every step of that slot)."""
    import torch
    import paper_2603_08593_amd as sf
    pipe = sf.PairPipeline(W, H, L, DK, DB, depth=depth, solve_team=team, image_dtype="float32",
                           compute=compute)
    n = len(inputs)

    def step(k):
        R, S, peds = inputs[k % n]
        pipe.submit(R, S, max_refine=1, pedestals=peds)

    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    chis = [float(pipe.buffers(k).chi2.item()) for k in range(min(depth, steps))]
    infos = [pipe.info(k) for k in range(min(depth, steps))]
    pipe.close()
    ok = all(_ok(i.status, [c]) for i, c in zip(infos, chis))
    return dict(value=(steps / (t1 - t0)) if ok else 0.0, ms=(t1 - t0) * 1e3 / steps, chi2=max(chis),
                depth=depth, team=team)


def pipeline_inputs(pairs, compute):
    """(R, S, pedestals) on the device for each pair (pedestals: the FP64
    image means for the FP32-spectra form, else none)."""
    import numpy as np
    import torch
    out = []
    for p in pairs:
        peds = None
        if compute == "fp32":
            peds = (float(np.mean(p.R, dtype=np.float64)), float(np.mean(p.S, dtype=np.float64)))
        out.append((torch.from_numpy(p.R).cuda(), torch.from_numpy(p.S).cuda(), peds))
    return out


def run_batch(steps, warmup):
    """Batched form: one exposure of 60 CCD pairs (2048x4096) and 40 uneven
    cutouts, L in {11, 15}, FP32 spectra with per-item FP64-mean pedestals,
    every phase one launch, replayed from one HIP graph; tunables from the
    autotuner."""
    import numpy as np
    import torch
    import synth.gpu as sg
    import paper_2603_08593_amd as sf
    shapes = sg.batch_shapes()
    ccd_equiv = sum(w * h for w, h, _ in shapes) / float(W * H)
    b = sf.Batch(shapes, dk=DK, db=DB, max_refine=1)
    for k, (w, h, l) in enumerate(shapes):
        pr = sg.make_batch_pair(k, w, h, l)
        b.load(k, pr["R"], pr["S"])
        del pr
    torch.cuda.synchronize()
    rpb, team = b.tune()
    knobs = b.knobs()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            b.run_graph(stream)
    stream.synchronize()
    # phase timings on one eager run (events around each batched launch)
    ev = HipEvents()
    slots = {"row_pass": 1, "col_pass": 2, "xinv": 3, "subtract": 4, "solve": 5, "build": 6}
    pairs = {k: (ev.create(), ev.create()) for k in slots}
    lib = sf.lib()
    for name, slot in slots.items():
        lib.sfft_profile_events(b.handle.ptr, slot, pairs[name][0], pairs[name][1])
    b.run(stream)
    stream.synchronize()
    for slot in slots.values():
        lib.sfft_profile_events(b.handle.ptr, slot, None, None)
    phase = {k: ev.elapsed_ms(*pairs[k]) * 1e3 for k in slots}
    ev.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(steps):
            b.run_graph(stream)
    stream.synchronize()
    t1 = time.perf_counter()
    chis = np.array([float(x.chi2.item()) for x in b.bufs])
    stat = [int(b.info(k).status) for k in range(len(shapes))]
    b.close()
    ok = all(s == 0 for s in stat) and bool(np.all(chis <= 1.05))
    t_step = (t1 - t0) / steps
    return dict(value=round(ccd_equiv / t_step, 3) if ok else 0.0, ms=t_step * 1e3, items=len(shapes),
                ccd_equiv=ccd_equiv, items_per_s=len(shapes) / t_step, max_chi2=float(chis.max()),
                rpb=rpb, team=team, knobs=knobs, phase=phase, steps=steps)


def run_stamps(pair, R, S, steps, warmup):
    """Precision form: stamp-restricted build (64 stamps of 41 x 41, FP32
    operands split into three bfloat16 terms, six term products per operand
    pair on the matrix cores, FP64 image means as pedestals) +
    FP64 solve + full-image subtract and chi2 on the 2048x4096 pair."""
    import numpy as np
    import torch
    import synth
    import paper_2603_08593_amd as sf
    c = synth.pick_stamps(pair, 64, 41)
    C = torch.from_numpy(c).to(R.device)
    peds = (float(np.mean(pair.R, dtype=np.float64)), float(np.mean(pair.S, dtype=np.float64)))
    d = sf.Differencer(W, H, L, DK, DB, image_dtype="float32", stamps=(len(c), 41),
                       ref_pedestal=peds[0], sci_pedestal=peds[1])
    stream = torch.cuda.current_stream()

    def step():
        d.build_stamps(R, S, C, 41, stream=stream)
        d.solve(max_refine=1, stream=stream)
        d.subtract(R, S, stream=stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ev = HipEvents()
    slots = {"stamp_gram": 7, "solve": 5, "subtract": 4}
    evs = {k: [(ev.create(), ev.create()) for _ in range(steps)] for k in slots}
    lib = sf.lib()
    for k in range(steps):
        for name, slot in slots.items():
            lib.sfft_profile_events(d.handle.ptr, slot, evs[name][k][0], evs[name][k][1])
        step()
    torch.cuda.synchronize()
    for slot in slots.values():
        lib.sfft_profile_events(d.handle.ptr, slot, None, None)
    avg = {n: sum(ev.elapsed_ms(a, b) for a, b in evs[n]) / steps / 1e3 for n in slots}
    ev.close()
    info = d.info()
    chi2 = float(d.buf.chi2.item())
    d.close()
    ok = _ok(info.status, [chi2])
    K = len(c) * 41 * 41
    N = n_unknowns()
    flops = 6.0 * K * (N + 1) * (N + 2)          # upper triangle of the augmented Gram, 6 split-term products
    ach = flops / avg["stamp_gram"] / 1e12
    roof = {"kernel": "stamp_gram", "bound": "mfma", "achieved": round(ach, 2), "peak": 2500.0,
            "unit": "TFLOP/s", "frac": round(ach / 2500.0, 4), "traffic": None,
            "avg_us": round(avg["stamp_gram"] * 1e6, 2), "alg_flops": flops}
    return dict(value=steps / (t1 - t0) if ok else 0.0, ms=(t1 - t0) * 1e3 / steps, chi2=chi2, avg=avg,
                roofline=roof, steps=steps)


def run_learned(n_pairs, warmup, batch, depth=PIPE_DEPTH, team=PIPE_TEAM):
    """Learned form (gated inference) against the plain path on held-out
    pairs of the learned-form workload (seeds never used in training). Each
    pair: stamps -> bf16 network -> background refit -> subtract + chi2
    judge, full build + solve + subtract when the judge rejects; the network
    runs on `batch` pairs per launch with one host read of their chi2 values,
    and `depth` pairs are refitted, subtracted (and, if rejected, fitted) in
    flight. The plain path runs build + solve + subtract on the same pairs,
    also with `depth` pairs in flight (the gain is against that), and one at
    a time (reported beside it). The pairs are rendered into HBM before the
    timed loops."""
    import torch
    import synth
    import synth.gpu as sg
    from paper_2603_08593_amd.learned import GatedDifferencer, load_weights
    path = os.path.join(ROOT, "paper_2603_08593_amd", "weights", "surrogate_L11_DK2_DB2.npz")
    params, std, _ = load_weights(path)
    import paper_2603_08593_amd as sf
    g = GatedDifferencer(W, H, L, DK, DB, params, std, max_pairs=batch, in_flight=depth, solve_team=team)
    d = sf.Differencer(W, H, L, DK, DB, image_dtype="float32")
    pipe = sf.PairPipeline(W, H, L, DK, DB, depth=depth, solve_team=team, image_dtype="float32")
    pairs = []
    k = 8500
    while len(pairs) < n_pairs + warmup:
        pr = sg.make_learned_pair(k)
        c = synth.pick_centers(pr["xs"], pr["ys"], pr["flux"], W, H, 64, 32, 5)
        k += 1
        if len(c) < 64:
            continue
        pairs.append((pr["R"], pr["S"], torch.from_numpy(c).cuda()))
    warm, timed = pairs[:warmup], pairs[warmup:]
    for R, S, C in warm:
        g.run(R, S, C)
        d.run(R, S, max_refine=1)
        pipe.submit(R, S, max_refine=1)
    g.run_batch(warm[:batch])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    acc, finals = 0, []
    for i in range(0, len(timed), batch):
        ok, _, cf = g.run_batch(timed[i:i + batch])
        acc += sum(ok)
        finals += cf
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for R, S, C in timed:
        pipe.submit(R, S, max_refine=1)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for R, S, C in timed:
        d.run(R, S, max_refine=1)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    plain_chi = []
    for R, S, C in timed:                      # chi2 of the plain path (outside the timing)
        d.run(R, S, max_refine=1)
        plain_chi.append(float(d.buf.chi2.item()))
    d.close()
    pipe.close()
    g.close()
    n = len(timed)
    ok_all = max(finals) <= 1.05 and max(plain_chi) <= 1.05
    gated = n / (t1 - t0)
    plain = n / (t2 - t1)
    serial = n / (t3 - t2)
    return dict(value=gated if ok_all else 0.0, ms=(t1 - t0) * 1e3 / n, n=n, accept=acc / n,
                max_final=max(finals), plain=plain if ok_all else 0.0, gain=gated / plain if ok_all else 0.0,
                plain_serial=serial if ok_all else 0.0, max_plain=max(plain_chi), batch=batch, depth=depth)


def run_multi(steps, warmup, n_temp=5):
    """Multi-template form: one 2048x4096 science image differenced against
    n_temp templates (FP64 build and solve, the science row spectrum and
    moments taken once), each difference brought to the science zero point
    and median-combined; then the 5-sigma limiting magnitude of the combined
    image from 1024 background apertures of radius 3 px and forced
    photometry at the planted transients. Throughput in science images per
    second and template pairs per second; counted only when every
    template's chi2 <= 1.05 (the planted transients stay in the chi2 sum)."""
    import numpy as np
    import torch
    import synth
    import paper_2603_08593_amd as sf
    mt = synth.make_multi_template(W, H, n_temp, seed=synth.seed_for(6, 0), n_transients=20,
                                   transient_flux=(3e3, 3e4))
    refs = [torch.from_numpy(t).cuda() for t in mt.templates]
    sci = torch.from_numpy(mt.S).cuda()
    md = sf.MultiDifferencer(W, H, L, DK, DB, n_temp)
    zps = [mt.zp_sci] * n_temp
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        md.run(refs, sci, zps, mt.zp_sci, max_refine=1, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        md.run(refs, sci, zps, mt.zp_sci, max_refine=1, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    chis = md.chi2s.cpu().numpy()
    stat = [int(md.info(t).status) for t in range(n_temp)]
    # the median combine alone (HBM-bound: n reads + 1 write per pixel)
    ev = HipEvents()
    a, b = ev.create(), ev.create()
    hip = ev.hip
    hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    reps = 20
    hip.hipEventRecord(a, ctypes.c_void_p(stream.cuda_stream))
    desc = sf.image_desc(sci)
    for _ in range(reps):
        sf.sfft_median_combine(md.handle, desc, md.diffs, zps, mt.zp_sci, md.combined, stream)
    hip.hipEventRecord(b, ctypes.c_void_p(stream.cuda_stream))
    torch.cuda.synchronize()
    comb_s = ev.elapsed_ms(a, b) / reps / 1e3
    ev.close()
    comb_bytes = (n_temp + 1) * W * H * 4
    # photometry on the combined image
    xy = synth.background_positions(W, H, 1024, 3.0, seed=synth.seed_for(6, 1), avoid=mt.transients,
                                    avoid_radius=15.0)
    xyd = torch.from_numpy(xy).cuda()
    flux = torch.zeros(1024, dtype=torch.float64, device="cuda")
    res = torch.zeros(3, dtype=torch.float64, device="cuda")
    sf.sfft_limiting_magnitude(md.handle, desc, md.combined, xyd, 3.0, mt.zp_sci, flux, res, stream=stream)
    td = torch.from_numpy(np.ascontiguousarray(mt.transients[:, :2])).cuda()
    ff = torch.zeros(len(td), dtype=torch.float64, device="cuda")
    mm = torch.zeros_like(ff)
    sf.sfft_forced_photometry(md.handle, desc, md.combined, td, 3.0, mt.zp_sci, res[0:1], ff, mm, stream=stream)
    torch.cuda.synchronize()
    r = res.cpu().numpy()
    det = int(np.sum(ff.cpu().numpy() > 5.0 * r[0]))
    md.close()
    ok = all(x == 0 for x in stat) and bool(np.all(chis <= 1.05))
    t_step = (t1 - t0) / steps
    # science images in flight: PIPE_DEPTH differencers (own handle,
    # workspace, buffers and stream; solve team PIPE_TEAM), each with its own
    # synthetic science image and templates
    sets = [(refs, sci, mt)] + [None] * (PIPE_DEPTH - 1)
    for k in range(1, PIPE_DEPTH):
        m2 = synth.make_multi_template(W, H, n_temp, seed=synth.seed_for(6, 10 + k), n_transients=20,
                                       transient_flux=(3e3, 3e4))
        sets[k] = ([torch.from_numpy(t).cuda() for t in m2.templates], torch.from_numpy(m2.S).cuda(), m2)
    mds = [sf.MultiDifferencer(W, H, L, DK, DB, n_temp, solve_team=PIPE_TEAM) for _ in range(PIPE_DEPTH)]
    streams = [torch.cuda.Stream() for _ in range(PIPE_DEPTH)]

    def pstep(k):
        j = k % PIPE_DEPTH
        rj, sj, mj = sets[j]
        mds[j].run(rj, sj, [mj.zp_sci] * n_temp, mj.zp_sci, max_refine=1, stream=streams[j])

    torch.cuda.synchronize()
    for k in range(warmup * PIPE_DEPTH):
        pstep(k)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for k in range(steps * PIPE_DEPTH):
        pstep(k)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    pchis = np.concatenate([m.chi2s.cpu().numpy() for m in mds])
    pstat = [int(m.info(t).status) for m in mds for t in range(n_temp)]
    for m in mds:
        m.close()
    pok = ok and all(x == 0 for x in pstat) and bool(np.all(pchis <= 1.05))
    tp = (t3 - t2) / (steps * PIPE_DEPTH)
    return dict(value=(1.0 / tp) if pok else 0.0, pairs=(n_temp / tp) if pok else 0.0, ms=tp * 1e3,
                serial_value=(1.0 / t_step) if ok else 0.0, serial_ms=t_step * 1e3,
                n_temp=n_temp, max_chi2=float(max(chis.max(), pchis.max())), comb_us=comb_s * 1e6,
                comb_gbs=comb_bytes / comb_s / 1e9, comb_bytes=comb_bytes, sigma=float(r[0]), mlim=float(r[1]),
                detected=det, n_transients=len(td), steps=steps)


def rb_flops_per_candidate():
    """Multiply-adds x 2 of the scorer's convolutions (no padding terms), four
    rotated copies: stem 32x32x32x27, block 1 2 x 32x32x32x288, block 2
    16x16x64x(288 + 576 + 32), block 3 8x8x128x(576 + 1152 + 64)."""
    macs = (32 * 32 * 32 * 27 + 2 * 32 * 32 * 32 * 288 + 16 * 16 * 64 * (288 + 576 + 32)
            + 8 * 8 * 128 * (576 + 1152 + 64))
    return 4 * 2 * macs


def run_realbogus(steps, warmup, n=4096):
    """Real-bogus scorer on n candidates of the 2048x4096 pair's difference
    image (random positions), seeded random weights: stamp extraction + the
    network, candidates per second, and the network's matrix-core rate
    against the bf16 peak."""
    import numpy as np
    import torch
    import synth
    import paper_2603_08593_amd as sf
    pair = synth.make_cfg2(0)
    R = torch.from_numpy(pair.R).cuda()
    S = torch.from_numpy(pair.S).cuda()
    d = sf.Differencer(W, H, L, DK, DB)
    d.run(R, S, max_refine=1)
    c = torch.from_numpy(synth.rb_candidates((H, W), n, seed=synth.seed_for(8, 0))).cuda()
    params = torch.from_numpy(synth.rb_init(1)).cuda()
    stamps = torch.zeros((n, 3, 32, 32), dtype=torch.float32, device="cuda")
    logits = torch.zeros(n, dtype=torch.float32, device="cuda")
    probs = torch.zeros(n, dtype=torch.float32, device="cuda")
    ws = torch.empty(sf.sfft_rb_workspace_size(n), dtype=torch.uint8, device="cuda")
    desc = sf.image_desc(S)
    stream = torch.cuda.current_stream()

    def step():
        sf.sfft_rb_extract(d.handle, desc, S, R, d.buf.diff, c, (1000.0, 1000.0, 0.0), (0.01, 0.01, 0.05), stamps,
                           stream)
        sf.sfft_rb_score(d.handle, params, stamps, logits, probs, ws, stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ev = HipEvents()
    a, b = ev.create(), ev.create()
    ev.hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    ev.hip.hipEventRecord(a, ctypes.c_void_p(stream.cuda_stream))
    for _ in range(steps):
        sf.sfft_rb_score(d.handle, params, stamps, logits, probs, ws, stream)
    ev.hip.hipEventRecord(b, ctypes.c_void_p(stream.cuda_stream))
    torch.cuda.synchronize()
    score_s = ev.elapsed_ms(a, b) / steps / 1e3
    ev.close()
    fin = bool(torch.isfinite(logits).all().item())
    d.close()
    t_step = (t1 - t0) / steps
    fl = rb_flops_per_candidate() * n
    ach = fl / score_s / 1e12
    return dict(value=n / t_step if fin else 0.0, ms=t_step * 1e3, n=n, steps=steps, score_us=score_s * 1e6,
                roofline={"kernel": "rb_score (7 conv GEMMs + head)", "bound": "mfma", "achieved": round(ach, 2),
                          "peak": 2500.0, "unit": "TFLOP/s", "frac": round(ach / 2500.0, 4), "traffic": None,
                          "avg_us": round(score_s * 1e6, 2), "alg_flops": fl})


# ---------------------------------------------------------------------------
# JSON lines
# ---------------------------------------------------------------------------
BASE_KEYS = dict(unit="CCD pairs/s", n_gpus=1, higher_is_better=True, scaling="weak", vs_baseline=None,
                 data="synthetic")


def plain_line(args, res, compute, traffic_ok=True, pipe=None):
    """One JSON object for the plain (or precision) form. With `pipe` (the
    pipelined run), value and ms_per_step are its throughput and the serial
    run (one pair at a time) is reported beside it; phase_us and the
    rooflines always come from the serial run's per-kernel events."""
    fp32 = compute == "fp32"
    kern = {k: res["avg"][k] for k in ("row_pass", "col_pass", "solve", "subtract")}
    dominant = max(kern, key=kern.get)
    # the committed counters were taken on the FP64 kernels only
    roof_all = {k: roofline_entry(k, kern[k], load_traffic(k) if (traffic_ok and not fp32) else None, fp32)
                for k in kern}
    info = res["info"]
    label = ("plain SFFT, one DECam CCD pair 2048x4096 FP32, Moffat PSF, L=11 DK=2 DB=2 (N=732), FP64 "
             "build+solve (1 refinement step), FP64-accumulated subtract") if not fp32 else \
        ("precision form, one DECam CCD pair 2048x4096 FP32, Moffat PSF, L=11 DK=2 DB=2 (N=732), FP32 "
         "spectra and products with FP32 accumulation, FP64 image-mean pedestals, FP64 solve "
         "(1 refinement step), FP64-accumulated subtract")
    cfg = {"workload": label, "form": "plain" if not fp32 else "precision-fp32", "parallelism": "single GPU"}
    top = res
    extra = {}
    if pipe is not None:
        top = pipe
        cfg["workload"] = label + (f"; a queue of {pipe['depth']} different synthetic pairs differenced with "
                                   f"{pipe['depth']} pairs in flight (one HIP stream, handle and workspace "
                                   f"each; solve team {pipe['team']} workgroups)")
        cfg["pipeline"] = {"pairs_in_flight": pipe["depth"], "solve_team": pipe["team"]}
        extra = {"serial_pairs_per_s": round(res["value"], 3), "serial_ms_per_pair": round(res["ms"], 4)}
    return {
        "metric": METRIC, "value": round(top["value"], 3), **BASE_KEYS, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(top["ms"], 4),
        "dtype": "f64" if not fp32 else "f32",
        "config": cfg, **extra,
        "chi2_nu": round(res["chi2"], 5), "solve_status": int(info.status), "backward_err": info.backward_err,
        "phase_us": {k: round(v * 1e6, 2) for k, v in res["avg"].items()},
        "roofline": dict(roof_all[dominant]),
        "roofline_kernels": roof_all,
        "build_roofline": build_roofline(res["avg"]["build"], fp32),
    }


def batch_line(args, r):
    return {
        "metric": METRIC, "value": r["value"], **BASE_KEYS, "steps": r["steps"], "warmup": args.warmup,
        "ms_per_step": round(r["ms"], 4), "dtype": "f32",
        "config": {"workload": "batched SFFT: one exposure of 60 CCD pairs 2048x4096 + 40 cutouts "
                               "({2,3,5}-smooth 512..1536 x 512..2048), L in {11,15}, DK=2 DB=2, FP32 "
                               "spectra with FP64-mean pedestals, FP64 solve, one launch per phase, HIP graph",
                   "form": "batched", "parallelism": "single GPU", "items": r["items"],
                   "ccd_equivalents": round(r["ccd_equiv"], 2), "tuned_rows_per_workgroup": r["rpb"],
                   "tuned_solve_team": r["team"], "tuned_knobs": r["knobs"]},
        "items_per_s": round(r["items_per_s"], 2), "max_chi2_nu": round(r["max_chi2"], 5),
        "phase_us_eager": {k: round(v, 1) for k, v in r["phase"].items()},
    }


def stamps_line(args, r):
    return {
        "metric": METRIC, "value": round(r["value"], 3), **BASE_KEYS, "steps": r["steps"], "warmup": args.warmup,
        "ms_per_step": round(r["ms"], 4), "dtype": "bf16x6",
        "config": {"workload": "precision form: 2048x4096 FP32 pair, 64 stamps of 41x41, L=11 DK=2 DB=2, "
                               "split-product Gram on matrix cores (three bf16 terms per FP32 operand, six term "
                               "products, FP32 runs flushed to FP64) with FP64-mean pedestals, FP64 solve, "
                               "FP64 subtract", "form": "stamps", "parallelism": "single GPU"},
        "chi2_nu": round(r["chi2"], 5), "phase_us": {k: round(v * 1e6, 2) for k, v in r["avg"].items()},
        "roofline": r["roofline"],
    }


def learned_line(args, r):
    return {
        "metric": METRIC, "value": round(r["value"], 3), **BASE_KEYS, "steps": r["n"], "warmup": args.warmup,
        "ms_per_step": round(r["ms"], 4), "dtype": "bf16+f64",
        "config": {"workload": "learned form: held-out 2048x4096 FP32 pairs with random PSF FWHM 2.5-6 px and "
                               "gradients, 64 star-stamp pairs of 32x32, bf16 network on batches of pairs + "
                               "background refit, chi2 judge at 1.05 with fallback to the FP64 build + solve, "
                               "L=11 DK=2 DB=2; pairs in flight as in the plain line it is compared with",
                   "form": "learned", "parallelism": "single GPU"},
        "accept_rate": round(r["accept"], 4), "max_final_chi2_nu": round(r["max_final"], 5),
        "plain_pairs_per_s": round(r["plain"], 3), "gain_vs_plain": round(r["gain"], 4),
        "plain_serial_pairs_per_s": round(r["plain_serial"], 3),
        "max_plain_chi2_nu": round(r["max_plain"], 5), "network_batch_pairs": r["batch"],
        "pairs_in_flight": r["depth"],
    }


def multi_line(args, r):
    return {
        "metric": METRIC, "value": round(r["pairs"], 3), **BASE_KEYS, "steps": r["steps"], "warmup": args.warmup,
        "ms_per_step": round(r["ms"], 4), "dtype": "f64",
        "config": {"workload": f"multi-template differencing: one 2048x4096 FP32 science image against "
                               f"{r['n_temp']} templates (Gaussian PSFs, different seeing, flux scales and skies), "
                               "L=11 DK=2 DB=2, FP64 build (science spectrum reused) and solve, per-template "
                               "subtract, zero-point normalisation and pixelwise median; "
                               f"{PIPE_DEPTH} different science images in flight (one stream, handle and "
                               f"workspace each; solve team {PIPE_TEAM})",
                   "form": "multi-template", "parallelism": "single GPU",
                   "pipeline": {"science_images_in_flight": PIPE_DEPTH, "solve_team": PIPE_TEAM}},
        "science_images_per_s": round(r["value"], 3),
        "serial_science_images_per_s": round(r["serial_value"], 3), "serial_ms_per_science_image":
            round(r["serial_ms"], 4),
        "max_chi2_nu": round(r["max_chi2"], 5),
        "median_combine": {"avg_us": round(r["comb_us"], 2), "bound": "hbm",
                           "achieved": round(r["comb_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(r["comb_gbs"] / HBM_PEAK_GBS, 4), "alg_bytes": r["comb_bytes"]},
        "limiting_mag_5sigma": round(r["mlim"], 4), "aperture_sigma": round(r["sigma"], 3),
        "transients_detected_5sigma": f"{r['detected']}/{r['n_transients']}",
    }


def rb_line(args, r):
    return {
        "metric": "real-bogus candidates scored/sec", "value": round(r["value"], 1), "unit": "candidates/s",
        "n_gpus": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "data": "synthetic",
        "steps": r["steps"], "warmup": args.warmup, "ms_per_step": round(r["ms"], 4), "dtype": "bf16",
        "config": {"workload": f"real-bogus scorer: {r['n']} candidates of a 2048x4096 difference image, "
                               "3x32x32 stamps, 4 rotated copies through a residual CNN (stem 32, blocks 32/64/128),"
                               " seeded random weights, bf16 matrix cores with FP32 accumulation",
                   "form": "realbogus", "parallelism": "single GPU"},
        "roofline": r["roofline"],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="plain form only (no precision/batched/learned keys)")
    ap.add_argument("--serial", action="store_true",
                    help="one pair at a time only (no pipelined run; the command the kernel profiles use)")
    ap.add_argument("--compute", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (counter calibration)")
    ap.add_argument("--form", choices=["plain", "batch", "stamps", "learned", "multi", "realbogus"], default="plain")
    ap.add_argument("--learned-batch", type=int, default=10, help="pairs per network launch (learned form)")
    ap.add_argument("--learned-pairs", type=int, default=60, help="held-out pairs timed (learned form)")
    ap.add_argument("--batch-steps", type=int, default=10, help="graph replays timed (batched form)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by CCD pair with no exchange between GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.form == "batch":
        print(json.dumps(batch_line(args, run_batch(args.steps, args.warmup))), flush=True)
        return
    if args.form == "realbogus":
        print(json.dumps(rb_line(args, run_realbogus(args.steps, args.warmup))), flush=True)
        return
    if args.form == "multi":
        print(json.dumps(multi_line(args, run_multi(args.steps, args.warmup))), flush=True)
        return
    if args.form == "learned":
        print(json.dumps(learned_line(args, run_learned(args.steps, args.warmup, args.learned_batch))), flush=True)
        return
    pair = synth.make_cfg2(0)
    dev = torch.device("cuda:0")
    R = torch.from_numpy(pair.R).to(dev)
    S = torch.from_numpy(pair.S).to(dev)
    if args.form == "stamps":
        print(json.dumps(stamps_line(args, run_stamps(pair, R, S, args.steps, args.warmup))), flush=True)
        return
    res = run_plain(R, S, pair, args.steps, args.warmup, args.compute)
    pipe = None
    if not args.serial:
        others = [synth.make_cfg2(i) for i in range(1, PIPE_DEPTH)]
        inputs = pipeline_inputs([pair] + others, args.compute)
        pipe = run_pipelined(inputs, args.steps, args.warmup, args.compute)
    if args.copy_calib_mib:
        n = args.copy_calib_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    out = plain_line(args, res, args.compute, pipe=pipe)
    if not args.no_forms and args.compute == "fp64":
        ksteps = min(args.steps, 20)
        p32 = run_plain(R, S, pair, ksteps, args.warmup, "fp32")
        p32_pipe = None
        if not args.serial:
            del inputs
            inputs32 = pipeline_inputs([pair] + others, "fp32")
            p32_pipe = run_pipelined(inputs32, ksteps, args.warmup, "fp32")
            del inputs32
        st = run_stamps(pair, R, S, ksteps, args.warmup)
        del R, S
        torch.cuda.empty_cache()
        bt = run_batch(args.batch_steps, 2)
        torch.cuda.empty_cache()
        ln = run_learned(args.learned_pairs, 3, args.learned_batch)
        torch.cuda.empty_cache()
        mu = run_multi(min(args.steps, 5), 1)
        torch.cuda.empty_cache()
        rb = run_realbogus(min(args.steps, 10), 2)
        torch.cuda.empty_cache()
        out["precision_fp32_pairs_per_s"] = round((p32_pipe or p32)["value"], 3)
        out["batched_ccd_equiv_per_s"] = bt["value"]
        out["batched_items_per_s"] = round(bt["items_per_s"], 2) if bt["value"] else 0.0
        out["stamps_pairs_per_s"] = round(st["value"], 3)
        out["learned_pairs_per_s"] = round(ln["value"], 3)
        out["learned_accept_rate"] = round(ln["accept"], 4)
        out["learned_gain_vs_plain"] = round(ln["gain"], 4)
        out["multi_template_pairs_per_s"] = round(mu["pairs"], 3)
        out["multi_template_science_per_s"] = round(mu["value"], 3)
        out["realbogus_candidates_per_s"] = round(rb["value"], 1)
        out["forms"] = {
            "precision_fp32": plain_line(args, p32, "fp32", pipe=p32_pipe),
            "batched": batch_line(args, bt),
            "stamps": stamps_line(args, st),
            "learned": learned_line(args, ln),
            "multi_template": multi_line(args, mu),
            "realbogus": rb_line(args, rb),
        }
        for v in out["forms"].values():
            for k in ("metric", "unit", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data"):
                v.pop(k, None)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pair)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
