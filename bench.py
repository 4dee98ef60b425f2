#!/usr/bin/env python3
"""Benchmark: batched log-likelihood evaluations per second on one MI355X.

One step = one pass of the library's forward path (per-point set-up, bin loop, epilogue) over
the full parameter batch of the chosen workload; inputs are resident in HBM before timing.
Default workload: 3 detectors, 8 s, 20-2048 Hz (16225 bins per detector), 65536 prior draws,
mixed precision. Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--config 1|2|3|4] [--no-cpu-baseline]

The CPU baseline times the FP64 oracle on a bounded sample of the same workload on the
host's cores before the GPU is touched.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import multiprocessing as mp
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# ---- peaks (MI355X: 256 CUs at 2.4 GHz) --------------------------------------------------
PEAK_FP64 = 78.6e12    # FP64 vector FLOP/s (published)
PEAK_FP32 = 157.3e12   # FP32 vector FLOP/s (published; needs packed FMA)
# transcendental VALU ops (v_sin_f32 / v_cos_f32): half the FP32 lane rate on gfx950,
# 256 CU x 64 lanes/clk x 2.4 GHz / 2
PEAK_TRANS = 256 * 64 * 2.4e9 / 2
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_eval_mixed_c1.txt")
# tile shapes measured on an MI355X by the library's autotuner (gwl_autotune / gwl_multi_autotune);
# loaded so that timed launches use a fixed, tuned shape; --retune measures them again
TUNE_FILE = os.path.join(ROOT, "paper_1909_11873_amd", "tuning_gfx950.json")
KERNEL_SOURCES = ["paper_1909_11873_amd/csrc/k_bins.hip", "paper_1909_11873_amd/csrc/gwl_bins.h",
                  "paper_1909_11873_amd/csrc/gwl_common.h", "paper_1909_11873_amd/csrc/gwl_device.h",
                  "paper_1909_11873_amd/csrc/gwl_epilogue.h", "paper_1909_11873_amd/csrc/gwl_launch.h"]


def work_per_point_bin(ndet: int, mixed: bool, grad: bool = False):
    """Algorithmic work per (point, frequency bin): (fp64 flops, fp32 flops, transcendental ops).

    FMA counts 2 flops. Phase polynomial: 7 FMA + 2 MUL in float64 (16 flops). Per detector:
    the f T_det shift (1 FMA), the reduction to one cycle (1 op), the phasor (sin + cos) and the
    complex multiply-accumulate u (cos - i sin) (4 FMA). In the float64 kernel sin and cos have
    no hardware instruction; their work is the table-and-polynomial evaluation, with the phase
    in units of 1/2048 cycle (the table index n = rint of it is the reduction, 1 op; y = phase - n,
    y^2, 3 FMA + 1 MUL for the two short series, 2 FMA + 2 MUL to rotate: 16 flops in all).
    The adjoint replaces the multiply-accumulate by the explicit product w = u p (2 MUL + 2 FMA),
    its sum (2 ADD), y_det = Im(c_det w) (MUL + FMA), the f-weighted sum of y_det (FMA) and the
    sum over detectors (ADD, one fewer than detectors): 14 flops per detector - 1; then the 8
    basis moments (8 FMA).

    A coarser planning count, 2M(11 + N_det) float64 flops per evaluation (28 per point-bin at
    three detectors), prices the phase at 11 FMA and each detector's shift at one FMA; the kernels'
    Horner form in x = f^(1/3) with the log terms folded in needs 7 FMA + 2 MUL, and the count here
    adds one operation per detector for the reduction to one cycle: 25 at three detectors. The
    fraction is taken against the work the kernels' algorithm needs, so it is the smaller count.
    """
    if grad:
        moments = 14 * ndet - 1 + 16
        if mixed:
            return 16 + ndet * (2 + 1), moments, ndet * 2
        return 16 + ndet * (2 + 16) + moments, 0, 0
    if mixed:
        return 16 + ndet * (2 + 1), ndet * 8, ndet * 2
    return 16 + ndet * (2 + 16 + 8), 0, 0


def roofline(ndet: int, mixed: bool, nbins: float, npoints: float, seconds: float, grad: bool = False):
    f64, f32, tr = work_per_point_bin(ndet, mixed, grad)
    units = float(nbins) * npoints
    ops = (f64 + f32 + tr) * units
    tmin = units * (f64 / PEAK_FP64 + f32 / PEAK_FP32 + tr / PEAK_TRANS)
    achieved = ops / seconds
    peak = ops / tmin
    return achieved / 1e12, peak / 1e12, achieved / peak


def NPARAM_ALL(nd: int, nodes: int) -> int:
    return 11 + 2 * nodes * nd


def kernel_hash() -> str:
    """Hash of the evaluation kernel's sources with comments and blank lines removed, so that a
    counter summary stays matched to the code it measured across edits of comments only."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
        h.update(code.encode())
    return h.hexdigest()[:16]


def read_traffic(layout: str):
    """HBM bytes per evaluation launch from the committed counter summary, if it was taken with the
    same kernel source and the same launch layout (waves per workgroup, workgroups per point group,
    set-up inside the kernel)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    m_hash = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    m_shape = re.search(r"launch_layout:\s*(\S+)", text)
    if not (m_hash and m_bytes and m_shape) or m_hash.group(1) != kernel_hash() or m_shape.group(1) != layout:
        return None
    return float(m_bytes.group(1))


def layout_key(shape) -> str:
    return f"W{shape['waves']}G{shape['groups']}S{int(bool(shape['setup']))}"


def kernel_name(nd: int, mixed: bool, grad: bool, shape) -> str:
    """The evaluation kernel's name as the profiler prints it: k_eval<ND, MIXED, GRAD, SETUP, CUT,
    ROT> (no ISCO cut; the float64 loop on the workloads' uniform grids rotates the phasors)."""
    b = lambda x: "true" if x else "false"
    return f"gwl::k_eval<{nd}, {b(mixed)}, {b(grad)}, {b(shape['setup'])}, false, {b(not mixed)}>"


WARM_S = 0.3


def warm_up(fn, n: int, min_s: float = WARM_S) -> None:
    """At least n untimed calls, continued until min_s seconds have passed: the first launches of
    a fresh process run slower (up to 2.5x for about a quarter second) than the steady state."""
    import torch
    t0 = time.perf_counter()
    i = 0
    while i < n or time.perf_counter() - t0 < min_s:
        fn()
        i += 1
        if i >= n:
            torch.cuda.synchronize()


def load_or_tune(tune_out):
    """Use the committed tile shapes unless asked to measure them again."""
    from paper_1909_11873_amd import gwlike as gw
    if tune_out is None and os.path.exists(TUNE_FILE):
        gw.autotune_load(TUNE_FILE)
        return False
    return True


# ---- CPU baseline (FP64 oracle) ----------------------------------------------------------
_W = {}


def _worker_init(data, psd, dets, f, df):
    import torch
    torch.set_num_threads(1)
    _W.update(data=data, psd=psd, dets=dets, f=f, df=df)


def _worker_eval(theta_rows):
    from oracle import gw_oracle as o
    return o.logl(theta_rows, _W["data"], _W["psd"], _W["dets"], _W["f"], _W["df"]).numpy()


def cpu_baseline(cfg: int, target_s: float):
    import numpy as np
    import torch

    from oracle import gw_oracle as o
    from paper_1909_11873_amd import synth

    spec = synth.event_spec(cfg)
    f, psd, nz, dets = synth.event_arrays(spec)
    data = nz + o.strain_all(spec.theta0, dets, f).numpy()
    theta = synth.theta_batch(spec)
    torch.set_num_threads(1)
    t0 = time.perf_counter()
    o.logl(theta[:4], data, psd, dets, f, spec.df)
    per_point = (time.perf_counter() - t0) / 4
    workers = max(1, min(16, os.cpu_count() or 1))
    n = int(min(len(theta), max(workers, target_s * workers / per_point)))
    n = max(workers, n // workers * workers)
    chunks = np.array_split(theta[:n], workers * 4)
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers, initializer=_worker_init, initargs=(data, psd, dets, f, spec.df)) as pool:
        t0 = time.perf_counter()
        parts = pool.map(_worker_eval, chunks)
        wall = time.perf_counter() - t0
    ref = np.concatenate(parts)
    return {
        "value": n / wall, "unit": "evals/s", "cores": workers, "kind": "oracle", "value_1core": 1.0 / per_point,
        "sample": f"first {n} of the {len(theta)} prior draws of the same workload, FP64 torch-CPU oracle, "
                  f"{workers} single-threaded processes, {wall:.1f} s wall",
    }, (theta[:n], ref, data, psd, dets, f, spec.df)


def _rb_oracle_sample(cfg: int, eps: float):
    """A function that evaluates the oracle's relative binning (same event data as the CPU
    baseline, fiducial theta0) on a few points; the summary data are built here, on the host."""
    import numpy as np

    from oracle import gw_oracle as o
    from oracle import rb_oracle as rbo
    from paper_1909_11873_amd import synth
    spec = synth.event_spec(cfg)
    f, psd, nz, dets = synth.event_arrays(spec)
    data = nz + o.strain_all(spec.theta0, dets, f).numpy()
    summ = rbo.summary(data, psd, dets, f, spec.df, spec.theta0, eps)

    def run(theta):
        return theta, rbo.logl(theta, summ, psd, dets, f, spec.df).numpy()
    run.sum_abs_v = float(np.abs(summ["V"]).sum())
    return run, data


# ---- GPU leg --------------------------------------------------------------------------------
def gpu_leg(cfg: int, steps: int, warmup: int, parity_inputs, tune_out=None, rb_eps=0.1, rb_inputs=None,
            cal_nodes=10):
    import numpy as np
    import torch

    from paper_1909_11873_amd import gwlike as gw
    from paper_1909_11873_amd import synth

    dev = torch.device("cuda:0")
    spec = synth.event_spec(cfg)
    f, psd, nz, dets = synth.event_arrays(spec)
    ft = torch.tensor(f, device=dev)
    # injection from the library's own waveform at theta0
    h0 = gw.waveform(torch.tensor(spec.theta0[None], device=dev), dets, ft)[0]
    data = torch.tensor(nz, device=dev) + h0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev = gw.Event(data, torch.tensor(psd, device=dev), dets, ft, spec.df)
    prep_ms = (time.perf_counter() - t0) * 1e3
    theta = torch.tensor(synth.theta_batch(spec), device=dev)
    B, M, nd = theta.shape[0], len(f), spec.ndet
    # tile shapes for the timed launches: the committed autotuner results, or measured now (not timed)
    t_tune = time.perf_counter()
    if load_or_tune(tune_out):
        for prec in ("mixed", "fp64"):
            gw.autotune(ev, B, prec, with_grad=False, cache_path=tune_out)
            gw.autotune(ev, min(B, 16384), prec, with_grad=True, cache_path=tune_out)
    t_tune = time.perf_counter() - t_tune
    shapes = {}
    for key, (bb, prec, gr) in {"mixed": (B, "mixed", False), "fp64": (B, "fp64", False),
                                "mixed_grad": (min(B, 16384), "mixed", True),
                                "fp64_grad": (min(B, 16384), "fp64", True)}.items():
        nchunk, chunk = gw.launch_shape(ev, bb, prec, gr)
        waves, groups, setup = gw.launch_layout(ev, bb, prec, gr)
        shapes[key] = {"nchunk": nchunk, "chunk_bins": chunk, "waves": waves, "groups": groups, "setup": setup}

    def timed(fn, k, w):
        """(wall seconds of k calls, mean bin-loop kernel seconds over k more calls). The wall clock
        runs with nothing added to the calls; in the second pass the bin-loop launches are
        bracketed by HIP events on the stream they run on (two events and two records per call,
        which would otherwise count in a short call's wall time)."""
        warm_up(fn, w)
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gw.profile_read()
        gw.profile_enable(True)
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        gw.profile_enable(False)
        n, kms = gw.profile_read()
        return wall, kms / max(n, 1) / 1e3

    def kernel_median(fn, reps=50):
        """Median over `reps` launches of the bin-loop kernel's duration (HIP events on its
        stream, read after every call) and of the whole call (torch events on the same stream)."""
        ks, calls = [], []
        gw.profile_read()
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            gw.profile_enable(True)
            a.record()
            fn()
            b.record()
            gw.profile_enable(False)
            n, kms = gw.profile_read()
            b.synchronize()
            ks.append(kms / max(n, 1) / 1e3)
            calls.append(a.elapsed_time(b) / 1e3)
        return float(np.median(ks)), float(np.median(calls))

    out = {}
    # the configuration's headline precision takes the full step count, the other the quarter
    head64 = cfg == 0
    k_mixed = max(3, steps // 4) if head64 else steps
    k_64 = steps if head64 else max(3, steps // 4)
    wall, kern_s = timed(lambda: gw.logl(theta, ev, "mixed"), k_mixed, warmup if not head64 else 2)
    out["mixed"] = (wall, kern_s, k_mixed) + kernel_median(lambda: gw.logl(theta, ev, "mixed"))
    wall64, kern64 = timed(lambda: gw.logl(theta, ev, "fp64"), k_64, warmup if head64 else 2)
    out["fp64"] = (wall64, kern64, k_64) + kernel_median(lambda: gw.logl(theta, ev, "fp64"))
    # adjoint at the gradient workload's batch (same shapes, 16384 points)
    tg = theta[:16384]
    BG = int(tg.shape[0])
    k_g = steps if cfg == 3 else max(3, steps // 4)
    wg, kg = timed(lambda: gw.logl_grad(tg, ev, "mixed"), k_g, 2)
    kg_med = kernel_median(lambda: gw.logl_grad(tg, ev, "mixed"))
    wg64, kg64 = timed(lambda: gw.logl_grad(tg, ev, "fp64"), 3, 1)

    # relative binning against theta0 (the injection) on the same event: cost and accuracy
    rb = None
    if rb_eps > 0:
        rev = gw.Event(data, torch.tensor(psd, device=dev), dets, ft, spec.df, fiducial=spec.theta0, rb_eps=rb_eps)
        if tune_out is not None:      # both precisions run the float64 edge loop on this event
            gw.autotune(rev, B, "fp64", with_grad=False, cache_path=tune_out)
        rng = np.random.default_rng(77)
        # offsets of the order of the posterior width: a binary black hole (c1, c3), or the long
        # low-mass signal (c2), whose chirp mass is measured some hundred times more finely
        step = (np.array([0.05, 0.01, 0.02, 0.02, 10.0, 0.01, 0.01, 0.02, 0.02, 0.05, 1e-4]) if spec.mc_range[1] > 5
                else np.array([2e-4, 0.005, 0.005, 0.005, 5.0, 0.005, 0.005, 0.01, 0.01, 0.02, 2e-5])) * 0.3
        near = torch.tensor(spec.theta0 + step * rng.standard_normal((B, 11)), device=dev)
        wr, kr = timed(lambda: gw.logl(near, rev, "mixed"), steps, warmup)
        wr64, kr64 = timed(lambda: gw.logl(near, rev, "fp64"), steps, warmup)
        a = gw.logl(near, rev, "fp64").cpu().numpy()
        b = gw.logl(near, ev, "fp64").cpu().numpy()
        am = gw.logl(near, rev, "mixed").cpu().numpy()
        rb = {"eps": rb_eps, "edges": rev.rb_edges, "bins": M, "mixed_evals_per_s": B * steps / wr,
              "fp64_evals_per_s": B * steps / wr64, "mixed_kernel_ms": kr * 1e3, "fp64_kernel_ms": kr64 * 1e3,
              "points": "theta0 plus Gaussian offsets of standard deviation " + ", ".join(f"{x:.3g}" for x in step),
              "max_abs_dlogl_vs_full_fp64": float(np.abs(a - b).max()),
              "median_abs_dlogl_vs_full_fp64": float(np.median(np.abs(a - b))),
              "max_abs_dlogl_mixed_vs_fp64": float(np.abs(am - a).max())}
        rev.close()
        if rb_inputs is not None:       # the oracle's relative binning on the oracle-injected data
            run, pdata = rb_inputs
            pev = gw.Event(torch.tensor(pdata, device=dev), torch.tensor(psd, device=dev), dets, ft, spec.df,
                           fiducial=spec.theta0, rb_eps=rb_eps)
            th_s, ref_rb = run(near[:16].cpu().numpy())
            got = gw.logl(torch.tensor(th_s, device=dev), pev, "mixed").cpu().numpy()
            got64 = gw.logl(torch.tensor(th_s, device=dev), pev, "fp64").cpu().numpy()
            # mixed runs the float64 edge loop on a relative-binning event: both within 1e-3 absolute,
            # the float64 one within 1e-9 relative
            rb["parity_vs_rb_oracle"] = {"points": len(th_s), "max_abs_dlogl_mixed": float(np.abs(got - ref_rb).max()),
                                         "max_abs_dlogl_fp64": float(np.abs(got64 - ref_rb).max()),
                                         "tolerance_mixed": 1e-3,
                                         "tolerance_fp64": 1e-9 * float(np.abs(ref_rb).max())}
            pev.close()

    # detector calibration model: cal_nodes amplitude and phase nodes per detector, node values
    # N(0, 0.05) (the relative amplitude and the phase in radians), on the same batch
    cal = None
    if cal_nodes > 0:
        cev = gw.Event(data, torch.tensor(psd, device=dev), dets, ft, spec.df, calibration_nodes=cal_nodes)
        crng = np.random.default_rng(5)
        cth = torch.cat([theta, torch.tensor(crng.normal(0.0, 0.05, (B, 2 * cal_nodes * nd)), device=dev)], dim=1)
        wc, _ = timed(lambda: gw.logl(cth, cev, "mixed"), max(3, steps // 4), 2)
        wc64, _ = timed(lambda: gw.logl(cth, cev, "fp64"), 3, 1)
        cg = cth[:min(B, 16384)]
        wcg, _ = timed(lambda: gw.logl_grad(cg, cev, "mixed"), 3, 1)
        cal = {"nodes": cal_nodes, "parameters": NPARAM_ALL(nd, cal_nodes),
               "mixed_evals_per_s": B * max(3, steps // 4) / wc, "fp64_evals_per_s": B * 3 / wc64,
               "mixed_grad_evals_per_s": int(cg.shape[0]) * 3 / wcg, "grad_batch": int(cg.shape[0])}
        if parity_inputs is not None:
            from oracle import cal_oracle as co
            th_s, _, pdata, ppsd, pdets, pf, pdf = parity_inputs
            pev = gw.Event(torch.tensor(pdata, device=dev), torch.tensor(ppsd, device=dev), pdets,
                           torch.tensor(pf, device=dev), pdf, calibration_nodes=cal_nodes)
            cs = np.concatenate([th_s[:8], crng.normal(0.0, 0.05, (8, 2 * cal_nodes * nd))], axis=1)
            ref_c = co.logl(cs, pdata, ppsd, pdets, pf, pdf, cal_nodes).numpy()
            got_c = gw.logl(torch.tensor(cs, device=dev), pev, "mixed").cpu().numpy()
            got_c64 = gw.logl(torch.tensor(cs, device=dev), pev, "fp64").cpu().numpy()
            cal["parity_vs_cal_oracle"] = {"points": 8, "max_abs_dlogl_mixed": float(np.abs(got_c - ref_c).max()),
                                           "max_abs_dlogl_fp64": float(np.abs(got_c64 - ref_c).max()),
                                           "tolerance": 1e-3}
            pev.close()
        cev.close()

    parity = None
    if parity_inputs is not None:
        th_s, ref, pdata, ppsd, pdets, pf, pdf = parity_inputs
        pev = gw.Event(torch.tensor(pdata, device=dev), torch.tensor(ppsd, device=dev), pdets,
                       torch.tensor(pf, device=dev), pdf)
        got = gw.logl(torch.tensor(th_s, device=dev), pev, "mixed").cpu().numpy()
        got64 = gw.logl(torch.tensor(th_s, device=dev), pev, "fp64").cpu().numpy()
        err = np.abs(got - ref)
        err64 = np.abs(got64 - ref)
        parity = {"points": int(len(ref)), "max_abs_dlogl": float(err.max()),
                  "p99_abs_dlogl": float(np.quantile(err, 0.99)), "tolerance": 1e-3,
                  "max_abs_dlogl_fp64": float(err64.max()), "p99_abs_dlogl_fp64": float(np.quantile(err64, 0.99)),
                  "tolerance_fp64": 1e-6}
        pev.close()
    ev.close()
    res = {
        "B": B, "M": M, "ndet": nd, "prep_ms": prep_ms, "parity": parity, "autotune_s": t_tune,
        "shapes": shapes,
        "mixed_wall": out["mixed"][0], "mixed_kern": out["mixed"][1], "mixed_steps": out["mixed"][2],
        "mixed_kern_median": out["mixed"][3], "mixed_call_median": out["mixed"][4],
        "fp64_wall": out["fp64"][0], "fp64_kern": out["fp64"][1], "fp64_steps": out["fp64"][2],
        "fp64_kern_median": out["fp64"][3], "fp64_call_median": out["fp64"][4],
        "fp64_evals": B * out["fp64"][2] / out["fp64"][0],
        "grad_mixed_evals": BG * k_g / wg, "grad_fp64_evals": BG * 3 / wg64, "grad_batch": BG, "grad_steps": k_g,
        "grad_mixed_wall": wg, "grad_mixed_kern": kg, "grad_mixed_kern_median": kg_med[0],
        "grad_mixed_call_median": kg_med[1], "grad_fp64_kern": kg64, "rb": rb, "cal": cal,
    }
    return res


def _worker_value_grad(args):
    """Oracle value and gradient of a few points of one event, in points of 8; compute seconds."""
    import numpy as np

    from oracle import gw_oracle as o
    th, data, psd, dets, f, df = args
    t0 = time.perf_counter()
    vs, gs = [], []
    for i in range(0, len(th), 8):
        v, g = o.logl_grad(th[i:i + 8], data, psd, dets, f, df)
        vs.append(v.numpy())
        gs.append(g.numpy())
    return np.concatenate(vs), np.concatenate(gs), time.perf_counter() - t0


def multi_inputs(nevents: int, oracle_injection: bool):
    """Per event: (spec, fgrid, psd, data or noise, dets, theta). With oracle_injection the data
    carry the FP64 oracle's signal at the event's theta0; otherwise the caller injects."""
    from paper_1909_11873_amd import synth
    out = []
    for e in range(nevents):
        spec = synth.event_spec(4, e)
        f, psd, nz, dets = synth.event_arrays(spec)
        if oracle_injection:
            from oracle import gw_oracle as o
            nz = nz + o.strain_all(spec.theta0, dets, f).numpy()
        out.append((spec, f, psd, nz, dets, synth.theta_batch(spec)))
    return out


def cpu_baseline_multi(inputs, target_s: float):
    """The FP64 oracle's value and gradient on the first k points of every event, k sized to about
    target_s seconds on the host's cores; projected to the whole workload per event."""
    import torch

    from oracle import gw_oracle as o
    torch.set_num_threads(1)
    big = max(inputs, key=lambda x: len(x[1]))
    t0 = time.perf_counter()
    o.logl(big[5][:1], big[3], big[2], big[4], big[1], big[0].df)
    per_bin = 3.0 * (time.perf_counter() - t0) / len(big[1])   # value + gradient: about 3x the value
    # torch's autograd engine opens the GPU in every process that runs a backward pass: the
    # gradient workers stay one below the box's limit of 16 GPU processes, and this process
    # runs no backward pass itself
    workers = max(1, min(15, os.cpu_count() or 1))
    mbins = sum(len(x[1]) for x in inputs)
    k = max(1, min(64, int(target_s * workers / (per_bin * mbins))))
    order = sorted(range(len(inputs)), key=lambda e: -len(inputs[e][1]))   # longest first
    tasks = [(inputs[e][5][:k], inputs[e][3], inputs[e][2], inputs[e][4], inputs[e][1], inputs[e][0].df)
             for e in order]
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers, initializer=_worker_init, initargs=(None, None, None, None, None)) as pool:
        t0 = time.perf_counter()
        res = pool.map(_worker_value_grad, tasks, chunksize=1)
        wall = time.perf_counter() - t0
    refs = [None] * len(inputs)
    full_s = 0.0
    for e, (v, g, sec) in zip(order, res):
        refs[e] = (v, g)
        full_s += sec * inputs[e][0].batch / k
    total = sum(x[0].batch for x in inputs)
    sampled = k * len(inputs)
    return {
        "value": total / (full_s / workers), "unit": "evals/s", "cores": workers, "kind": "oracle",
        "sample": f"value and gradient of the first {k} points of each of the {len(inputs)} events ({sampled} points, "
                  f"FP64 torch-CPU oracle, {workers} single-threaded processes, {wall:.1f} s wall); each event's "
                  f"compute time scaled by B_e/{k} and the sum divided over the {workers} processes",
    }, (k, refs)


def multi_leg(steps: int, warmup: int, inputs, cpu=None, refs=None, tune_out=None):
    """All events of the uneven workload in one persistent mixed-precision launch, forward + gradient."""
    import numpy as np
    import torch

    from paper_1909_11873_amd import gwlike as gw

    dev = torch.device("cuda:0")
    events, thetas, batches, bins, devdata = [], [], [], [], []
    for spec, f, psd, data, dets, th in inputs:
        ft = torch.tensor(f, device=dev)
        dt = torch.tensor(data, device=dev)
        if refs is None:   # no oracle data: inject with the library's own waveform at theta0
            dt = dt + gw.waveform(torch.tensor(spec.theta0[None], device=dev), dets, ft)[0]
        pt = torch.tensor(psd, device=dev)
        devdata.append((dt, pt, ft))
        events.append(gw.Event(dt, pt, dets, ft, spec.df))
        thetas.append(torch.tensor(th, device=dev))
        batches.append(spec.batch)
        bins.append(len(f))
    t_tune = time.perf_counter()
    if load_or_tune(tune_out):                                       # plan shape for this workload
        gw.multi_autotune(events, batches, "mixed", with_grad=True, cache_path=tune_out)
    t_tune = time.perf_counter() - t_tune
    plan = gw.MultiPlan(events, batches, "mixed", with_grad=True)
    chunk, desc, items = plan.info()
    warm_up(lambda: plan.launch(thetas), warmup)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.launch(thetas)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    logls, grads, lat = plan.launch(thetas, latency=True)
    lat = np.array(lat)
    # the other queue order: per-event latency against launch time
    other = "ascending" if desc else "descending"
    plan_o = gw.MultiPlan(events, batches, "mixed", with_grad=True, order=other)
    warm_up(lambda: plan_o.launch(thetas), 1)
    ko = max(2, steps // 2)
    t0 = time.perf_counter()
    for _ in range(ko):
        plan_o.launch(thetas)
    torch.cuda.synchronize()
    wall_o = time.perf_counter() - t0
    _, _, lat_o = plan_o.launch(thetas, latency=True)
    lat_o = np.array(lat_o)
    plan_o.close()
    other_order = {"queue": f"{other} work", "ms_per_step": wall_o / ko * 1e3,
                   "latency_us": {"p50": float(np.percentile(lat_o, 50)), "p99": float(np.percentile(lat_o, 99)),
                                  "max": float(lat_o.max())}}
    total = int(sum(batches))
    pb = float(np.dot(batches, bins))
    parity = None
    if refs is not None:
        k, ref = refs
        dl, ge, gv = [], [], []
        w = np.array(WIDTHS)
        for (v, g), l, gg in zip(ref, logls, grads):
            got = gg[:k].cpu().numpy()
            dl.append(np.abs(l[:k].cpu().numpy() - v))
            ge.append(scaled_grad_error(got, g))
            gv.append(np.linalg.norm((got - g) * w, axis=1) / np.linalg.norm(g * w, axis=1))
        dl, ge, gv = np.concatenate(dl), np.concatenate(ge), np.concatenate(gv)
        gmax = ge.max(axis=1)
        parity = {"points": int(len(dl)), "max_abs_dlogl": float(dl.max()),
                  "p99_abs_dlogl": float(np.quantile(dl, 0.99)), "tolerance": 1e-3,
                  "max_scaled_grad_error": float(gmax.max()), "p99_scaled_grad_error": float(np.quantile(gmax, 0.99)),
                  "median_scaled_grad_error": float(np.median(gmax)),
                  "max_grad_vector_rel_error": float(gv.max())}
    plan.close()

    # the same workload through a float64 plan (its gradient meets the 1e-4 per-component bound
    # that the mixed adjoint misses on a few components of long events)
    plan64 = gw.MultiPlan(events, batches, "fp64", with_grad=True)
    warm_up(lambda: plan64.launch(thetas), 1)
    k64 = max(2, steps // 2)
    t0 = time.perf_counter()
    for _ in range(k64):
        plan64.launch(thetas)
    torch.cuda.synchronize()
    wall64 = time.perf_counter() - t0
    fp64 = {"value": total * k64 / wall64, "ms_per_step": wall64 / k64 * 1e3}
    if refs is not None:
        k, ref = refs
        l64, g64, _ = plan64.launch(thetas)
        ge64 = np.concatenate([scaled_grad_error(gg[:k].cpu().numpy(), g) for (v, g), gg in zip(ref, g64)])
        fp64["max_scaled_grad_error"] = float(ge64.max())
        fp64["max_abs_dlogl"] = float(max(np.abs(l[:k].cpu().numpy() - v).max() for (v, g), l in zip(ref, l64)))
    plan64.close()

    # calibrated events (10 nodes per detector, 71 parameters) in one plan: their own kernels run
    # after the persistent launch
    ncal = 10
    rng = np.random.default_rng(404)
    cal_events, cal_thetas = [], []
    for (spec, f, psd, data, dets, th), (dt, pt, ft), t in zip(inputs, devdata, thetas):
        cal_events.append(gw.Event(dt, pt, dets, ft, spec.df, calibration_nodes=ncal))
        c = torch.tensor(rng.normal(0.0, 0.05, (t.shape[0], 2 * ncal * 3)), device=dev)
        cal_thetas.append(torch.cat([t, c], dim=1).contiguous())
    planc = gw.MultiPlan(cal_events, batches, "mixed", with_grad=True)
    warm_up(lambda: planc.launch(cal_thetas), 1)
    kc = max(2, steps // 2)
    t0 = time.perf_counter()
    for _ in range(kc):
        planc.launch(cal_thetas)
    torch.cuda.synchronize()
    wallc = time.perf_counter() - t0
    calibrated = {"nodes_per_detector": ncal, "parameters": 11 + 2 * ncal * 3, "value": total * kc / wallc,
                  "ms_per_step": wallc / kc * 1e3}
    planc.close()
    for ev in cal_events:
        ev.close()
    for ev in events:
        ev.close()
    ach, peak, frac = roofline(3, True, pb, 1.0, wall / steps, grad=True)
    return {
        "metric": "total logL+gradient evals/s, 64 uneven events in one persistent launch (mixed)",
        "value": total * steps / wall, "unit": "evals/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": wall / steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"c4: {len(inputs)} events, 3 detectors, durations {min(bins)}-{max(bins)} bins, "
                               f"{total} points in total", "events": len(inputs), "points": total,
                   "point_bins": pb, "precision": "mixed", "gradient": True, "chunk_bins": chunk,
                   "queue": "descending work" if desc else "ascending work", "items": items,
                   "autotune_s": t_tune},
        "roofline": {"bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": frac, "traffic": None,
                     "kernel": "whole graph launch (set-up, k_multi_bins<3,mixed,grad>, epilogue)"},
        "latency_us": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max())},
        "cpu_baseline": cpu,
        "parity_vs_oracle": parity,
        "fp64": fp64,
        "calibrated": calibrated,
        "other_queue_order": other_order,
    }


# prior widths scale the gradient components before their error is taken
WIDTHS = (50.0, 0.8, 1.8, 1.8, 1900.0, 2 * math.pi, math.pi, math.pi, math.pi, 2 * math.pi, 0.2)


def scaled_grad_error(g, gref):
    """Per-component error of width-scaled gradients, relative to max(|g_i|, 1e-3 max_i |g_i|)."""
    import numpy as np
    w = np.array(WIDTHS)
    gs, rs = np.asarray(g) * w, np.asarray(gref) * w
    scale = np.maximum(np.abs(rs), 1e-3 * np.max(np.abs(rs), axis=-1, keepdims=True))
    return np.abs(gs - rs) / scale


def _trace_marker(dev, k: int) -> None:
    """One gwl_slice_list_init launch of k * 256 chains: a kernel of that grid marks a point in a
    profiler's kernel trace (synchronised, so nothing overlaps it)."""
    import torch
    from paper_1909_11873_amd import gwlike as gw
    torch.cuda.synchronize()
    gw.slice_list_init(k * 256, dev)
    torch.cuda.synchronize()


def ns_leg(cfg: int, nlive: int, batches, eps: float, proposal: str = "slice", snr: float = 20.0, seed: int = 1,
           tune_out=None):
    """Static parallel nested sampling on one event through the mixed-precision kernels, once per
    batch size. The injection sits at the event's theta0 moved in distance to an optimal SNR of
    `snr`. Reports iterations, accepted candidates per iteration, the paper's speed-up
    S = K ln(1 + n/K) at the mean number n accepted per iteration (which the volume estimate
    reproduces: K ln(1/X_end) / iterations), wall time, likelihood calls and ln Z."""
    import numpy as np
    import torch

    from paper_1909_11873_amd import gwlike as gw
    from paper_1909_11873_amd import nested
    from paper_1909_11873_amd import synth

    dev = torch.device("cuda:0")
    spec = synth.event_spec(cfg)
    f, psd, nz, dets = synth.event_arrays(spec)
    ft, pt = torch.tensor(f, device=dev), torch.tensor(psd, device=dev)
    th0 = spec.theta0.copy()
    h0 = gw.waveform(torch.tensor(th0[None], device=dev), dets, ft)[0]
    quiet = gw.Event(h0, pt, dets, ft, spec.df)           # noiseless data: logL(theta0) = SNR^2 / 2
    snr0 = math.sqrt(2.0 * float(gw.logl(torch.tensor(th0[None], device=dev), quiet, "fp64")[0]))
    quiet.close()
    th0[4] *= snr0 / snr
    data = torch.tensor(nz, device=dev) + gw.waveform(torch.tensor(th0[None], device=dev), dets, ft)[0]
    ev = gw.Event(data, pt, dets, ft, spec.df)
    l0 = float(gw.logl(torch.tensor(th0[None], device=dev), ev, "fp64")[0])
    transform = nested.gw_prior_transform(mc_range=spec.mc_range, spins=spec.spins)
    if load_or_tune(tune_out):
        # the likelihood batches a slice-sampling run makes: the live points, then per move the
        # m - 1 stepping-out ends and the groups of shrinkage draws of every chain
        m = 4                                              # the sampler's default stepping-out limit
        shapes = {nlive} | {k * n for n in batches for k in (m - 1,) + tuple(set(nested.SLICE_GROUPS))}
        for b in sorted(shapes):
            gw.autotune(ev, b, "mixed", cache_path=tune_out)
    rows = []
    for n in batches:
        kw = dict(device=dev, seed=seed, prior_transform=transform, proposal=proposal,
                  loglike_live=lambda th, live: gw.logl_live(th, live, ev, "mixed"))
        if proposal == "gmc":
            kw.update(loglike_grad=lambda th: gw.logl_grad(th, ev, "mixed"), gmc_steps=10)
        last = None
        smp = nested.ParallelNestedSampler(lambda th: gw.logl(th, ev, "mixed"), 11, nlive, n, **kw)
        smp.run(eps=1e3, max_iter=2)           # warm-up (kernels, allocator)
        torch.cuda.synchronize()
        _trace_marker(dev, 97)                 # a launch a kernel trace can find: the timed run starts
        res = smp.run(eps=eps, max_iter=20000)
        _trace_marker(dev, 89)                 # ... and ends
        w = np.exp(res.log_w)
        mc = float(np.sum(w * res.theta[:, 0]))
        nbar = float(res.n_accepted.mean()) if res.niter else 0.0
        rows.append({"batch": n, "iterations": res.niter, "mean_accepted": nbar,
                     "speedup_measured": res.speedup(), "speedup_law": nested.speedup_law(nbar, nlive) if nbar else 0.0,
                     "seconds": res.seconds, "ms_per_iteration": res.seconds / max(res.niter, 1) * 1e3,
                     "calls": res.ncall, "calls_per_s": res.ncall / res.seconds, "logz": res.logz,
                     "logz_err": res.logz_err, "information": res.information, "mc_mean": mc,
                     "max_logl": float(res.logl.max())})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
        last = res
    # an evidence estimate independent of nested sampling: importance sampling with a proposal
    # fitted to the last run's posterior
    wl = np.exp(last.log_w)
    post = last.u[np.random.default_rng(0).choice(len(wl), size=20000, p=wl / wl.sum())]
    lz_is, rel_is, ess_is = nested.importance_logz(post, lambda th: gw.logl(th, ev, "mixed"), transform, dev)
    print(json.dumps({"importance_sampling_logz": lz_is, "relative_error": rel_is, "ess": ess_is}),
          file=sys.stderr, flush=True)
    ev.close()
    best = min(rows, key=lambda r: r["seconds"])
    return {
        "metric": "static parallel nested sampling wall time to convergence (one event, mixed-precision likelihood)",
        "value": best["seconds"], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": best["seconds"] * 1e3, "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"c{cfg}: {spec.ndet} detectors, {len(f)} bins, injection at theta0 with the distance "
                               f"set for optimal SNR {snr}, {nlive} live points, {proposal} proposals, eps {eps}",
                   "nlive": nlive, "batches": list(batches), "logl_theta0": l0, "injected_mc": float(th0[0])},
        "runs": rows,
        "importance_sampling_check": {"logz": lz_is, "logz_err": rel_is, "ess": ess_is,
                                      "proposal": "16-component Gaussian mixture fitted to 20,000 draws from the last "
                                                  "run's posterior, with copies widened 1.5, 2.5 and 4 times; 8.0e6 draws"},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=1, choices=[0, 1, 2, 3, 4])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--ns", action="store_true",
                    help="time static parallel nested sampling on the chosen event (configs 0-3) for several batch sizes")
    ap.add_argument("--nlive", type=int, default=1000)
    ap.add_argument("--ns-batches", default="128,256,512,1024,2048")
    ap.add_argument("--ns-eps", type=float, default=0.1)
    ap.add_argument("--ns-proposal", default="slice", choices=["slice", "gmc", "ellipsoid", "prior"])
    ap.add_argument("--retune", metavar="CACHE", default=None,
                    help="measure the tile shapes again (written to CACHE) instead of loading " + TUNE_FILE)
    ap.add_argument("--rb-eps", type=float, default=0.1,
                    help="also time relative binning against theta0 with this edge spacing (0: skip)")
    ap.add_argument("--cal-nodes", type=int, default=10,
                    help="also time the detector calibration model with this many nodes per detector (0: skip)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also run one plain device-to-device copy of this many bytes (a known-size reference "
                         "for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path is single-GPU; "
              f"batch sharding across GPUs needs no exchange and is not measured here)", file=sys.stderr)
        sys.exit(2)

    if args.ns:
        batches = [int(x) for x in args.ns_batches.split(",") if x]
        print(json.dumps(ns_leg(args.config if args.config != 4 else 1, args.nlive, batches, args.ns_eps,
                                args.ns_proposal, tune_out=args.retune)))
        return

    if args.config == 4:
        inputs = multi_inputs(64, not args.no_cpu_baseline)
        cpu, refs = None, None
        if not args.no_cpu_baseline:
            cpu, refs = cpu_baseline_multi(inputs, args.cpu_seconds)
        print(json.dumps(multi_leg(args.steps, args.warmup, inputs, cpu, refs, args.retune)))
        return

    cpu, parity_inputs = None, None
    if not args.no_cpu_baseline:
        cpu, parity_inputs = cpu_baseline(args.config, args.cpu_seconds)

    if args.copy_bytes > 0:
        import torch
        n = args.copy_bytes // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    rb_inputs = None
    if parity_inputs is not None and args.rb_eps > 0:
        rb_inputs = _rb_oracle_sample(args.config, args.rb_eps)
    r = gpu_leg(args.config, args.steps, args.warmup, parity_inputs, args.retune, args.rb_eps, rb_inputs,
                args.cal_nodes)
    B, M, nd = r["B"], r["M"], r["ndet"]
    spec = __import__("paper_1909_11873_amd.synth", fromlist=["synth"]).event_spec(args.config)
    band = f"{nd} det, {spec.duration:g} s, {spec.f_lo:g}-{spec.f_hi:g} Hz"
    ach, peak, frac = roofline(nd, True, M, B, r["mixed_kern_median"])
    a64, p64, f64 = roofline(nd, False, M, B, r["fp64_kern_median"])
    agm, pgm, fgm = roofline(nd, True, M, r["grad_batch"], r["grad_mixed_kern_median"], True)
    sh = r["shapes"]
    traffic = read_traffic(layout_key(sh["mixed"])) if args.config == 1 else None
    mixed_line = {"value": B * r["mixed_steps"] / r["mixed_wall"], "kernel": kernel_name(nd, True, False, sh["mixed"]),
                  "kernel_ms_median": r["mixed_kern_median"] * 1e3, "kernel_ms_mean": r["mixed_kern"] * 1e3,
                  "call_ms_median": r["mixed_call_median"] * 1e3,
                  "roofline": {"bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": frac}}
    fp64_line = {"value": r["fp64_evals"], "kernel": kernel_name(nd, False, False, sh["fp64"]),
                 "kernel_ms_median": r["fp64_kern_median"] * 1e3, "kernel_ms_mean": r["fp64_kern"] * 1e3,
                 "call_ms_median": r["fp64_call_median"] * 1e3,
                 "roofline": {"bound": "alu", "achieved": a64, "peak": p64, "unit": "TFLOP/s", "frac": f64}}
    if args.config == 0:       # a float64 workload: the float64 kernel is the headline
        metric = f"logL evals/sec ({band}) FP64; frac VALU FP64 peak"
        head, other, other_name = fp64_line, mixed_line, "mixed"
        steps_head, wall_head, dtype, prec = r["fp64_steps"], r["fp64_wall"], "f64", "fp64"
    elif args.config == 3:     # the gradient workload: forward + adjoint, mixed
        metric = f"logL+gradient evals/sec ({band}, 11 parameters) mixed vs FP64; frac VALU peak"
        head = {"value": r["grad_mixed_evals"], "kernel": kernel_name(nd, True, True, sh["mixed_grad"]),
                "kernel_ms_median": r["grad_mixed_kern_median"] * 1e3, "kernel_ms_mean": r["grad_mixed_kern"] * 1e3,
                "call_ms_median": r["grad_mixed_call_median"] * 1e3,
                "roofline": {"bound": "alu", "achieved": agm, "peak": pgm, "unit": "TFLOP/s", "frac": fgm}}
        other, other_name = mixed_line, "forward_mixed"
        steps_head, wall_head, dtype, prec = r["grad_steps"], r["grad_mixed_wall"], "f64+f32", "mixed"
        B = r["grad_batch"]
    else:
        metric = ("logL evals/sec (3 det, 8 s, 20-2048 Hz) mixed vs FP64; frac VALU peak" if args.config == 1 else
                  f"logL evals/sec ({band}) mixed vs FP64; frac VALU peak")
        head, other, other_name = mixed_line, fp64_line, "fp64"
        steps_head, wall_head, dtype, prec = r["mixed_steps"], r["mixed_wall"], "f64+f32", "mixed"
    roof = dict(head["roofline"])
    roof.update({"traffic": traffic if prec == "mixed" and args.config == 1 else None, "kernel": head["kernel"],
                 "kernel_ms": head["kernel_ms_median"], "kernel_ms_mean": head["kernel_ms_mean"],
                 "timing": ("median over 50 launches of HIP events on its stream around the evaluation kernel and, "
                           "where the launch shape has one, its value-epilogue kernel")})
    line = {
        "metric": metric,
        "value": head["value"], "unit": "evals/s", "n_gpus": 1, "steps": steps_head, "warmup": args.warmup,
        "ms_per_step": wall_head / steps_head * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": f"c{args.config}: {nd} detectors, {M} bins per detector, {B} prior draws per batch",
                   "ndet": nd, "nbins": M, "batch": B, "precision": prec, "gradient": args.config == 3},
        "roofline": roof,
        "call_ms_median": head["call_ms_median"],
        "cpu_baseline": cpu,
        other_name: other,
        "grad": {"batch": r["grad_batch"], "mixed_evals_per_s": r["grad_mixed_evals"],
                 "fp64_evals_per_s": r["grad_fp64_evals"],
                 "mixed_kernel_ms": r["grad_mixed_kern_median"] * 1e3, "fp64_kernel_ms": r["grad_fp64_kern"] * 1e3,
                 "mixed_roofline": {"achieved": agm, "peak": pgm, "frac": fgm},
                 "fp64_roofline": dict(zip(("achieved", "peak", "frac"), roofline(nd, False, M, r["grad_batch"],
                                                                                 r["grad_fp64_kern"], True)))},
        "event_prep_ms": r["prep_ms"], "autotune_s": r["autotune_s"], "shapes": r["shapes"],
        "relative_binning": r["rb"], "calibration": r["cal"],
        "parity_vs_oracle": r["parity"],
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
