"""Benchmark of the frequency-domain EMRI mode sum on one MI355X.

One step = one FP64 waveform of the realistic-size workload (M=2e6, mu=20,
p0=13, e0=0.45, T=2 yr at dt=10 s: 3842 (l,m,n) modes, 200 knots, 3155816
bins) through the C ABI: spline coefficients, mode constants and piece
table, and the bin-major gather.  Inputs are resident in HBM before the
timed region.  Prints one JSON line; besides the headline it measures the
mixed-precision batch of 512 draws (one persistent launch, replayed from a
HIP graph) and the forward+adjoint of 64 draws, each with the roofline of
its dominant kernel, and the FP64 oracle on this host's cores.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--batch B] [--adjoint A]
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

METRIC = "waveforms/s + mode·bin evals/s (fwd, fwd+adjoint) at stated error vs FP64"
# Algorithmic work of one mode-bin evaluation (one root of Eq. cubic_equation,
# the per-root factor of Eq. extendedspa1, the phase, the amplitude spline and
# the two complex accumulations): about 150 arithmetic operations (a fused
# multiply-add counts 2) plus one sine/cosine pair, two divisions and one
# reciprocal square root, each of these four counted as one.
FLOPS_PER_EVAL = 154
# Rows with the same (m, n) share the voice frequency, hence the pieces, the
# roots, the factor of Eq. extendedspa1 and the phase, and the sum over such
# a group of c_t A_t(t(f)) E is one cubic per polarization, (sum_t c_t A_t)
# times E, whose coefficients the set-up combines once per segment.  The
# gather's algorithmic work is therefore counted per (group, piece, bin):
# the 154 flops above (for a group of two or more rows: two cubics of
# combined coefficients and two products with E, 40 flops, in place of one
# cubic, one product with E and two polarization products, 34; the lower
# count is used).  fdemri_last_group_eval_count gives those evaluations; for
# ungrouped tables it equals the mode-bin count.
# The adjoint per (voice group, piece, bin): the shared forward terms (root,
# derivatives, factor, phase and E: 120), the products conj(g) E for both
# polarizations with their sign fold (14), u = tau / h and its powers to u^6
# (6), and the moment sums of four values over seven powers of u (52); the
# group's Im Z sums and every row's gradient terms follow from the moments
# once per (group, segment), not per bin.
ADJ_FLOPS_PER_GROUP_EVAL = 192
PEAK_FP64_VALU = 78.6e12


def algorithmic_flops(evals, group_evals):
    """Algorithmic flops of a gather launch from its evaluation counts (the
    mode-bin count `evals` is the metric's unit and not used here)."""
    return FLOPS_PER_EVAL * group_evals


def progress(msg):
    """A line on stderr as each stage of a long measurement ends."""
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--batch", type=int, default=512,
                    help="waveforms in the batched mixed-precision measurement (0: skip)")
    ap.add_argument("--adjoint", type=int, default=64,
                    help="waveforms in the forward+adjoint measurement (0: skip)")
    ap.add_argument("--batch-reps", type=int, default=2,
                    help="timed graph replays of the batch (counter runs use 1)")
    ap.add_argument("--only", choices=["batch", "adjoint", "small"], default=None,
                    help="run only this secondary measurement after the headline (profiling runs)")
    ap.add_argument("--headline-only", action="store_true",
                    help="skip the secondary measurements (used for counter runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one device-to-device copy of 256 MiB, whose HBM byte counters "
                         "calibrate the gather kernel's")
    return ap.parse_args()


def _oracle_worker_init():
    """Each pool worker computes with one thread."""
    from threadpoolctl import threadpool_limits
    global _THREAD_LIMIT
    _THREAD_LIMIT = threadpool_limits(limits=1)


def _oracle_worker_probe(_):
    return os.getpid()


def _row_subset(w, j, P):
    """The workload restricted to the mode rows j, j + P, j + 2P, ..."""
    import dataclasses
    return dataclasses.replace(w, l=w.l[j::P], m=w.m[j::P], n=w.n[j::P], A=w.A[j::P])


def _oracle_rows(args):
    """The oracle waveform of the mode rows j::P of w on its whole grid (one
    pool task); the waveform is the sum of these parts (it is linear in the
    voices)."""
    w, j, P = args
    import oracle
    t0 = time.perf_counter()
    hp, hc = oracle.waveform(_row_subset(w, j, P))
    return j, hp, hc, time.perf_counter() - t0


def pool_cores():
    """Worker processes for the oracle's multiprocess leg: the cores this
    process may run on, held to 16 (the host share of one GPU here)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def cpu_baseline(w, gpu_hp, gpu_hc, evals_full, small, sample_stride=32):
    """The FP64 oracle timed on this host's cores.
    * value: multiprocess, full size.  The oracle's cost is per voice (a mask
      over the whole grid and a vectorised bisection per monotonic piece,
      then the per-root terms), so the work is split by voices: worker j of
      P computes the mode rows j::P on the whole grid and the parts are
      summed.  The result is compared with the GPU waveform on every bin.
    * single_process: every sample_stride-th mode row on the whole grid on
      one core, scaled by sample_stride (flagged as extrapolated).
    * full_size_single_process: the two 20-mode workloads (full DFT grid and
      log grid), small = [(name, workload, GPU seconds per waveform)]."""
    import multiprocessing as mp
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle

    P = pool_cores()
    res = {"kind": "oracle", "unit": "waveforms/s", "affinity_cores": len(os.sched_getaffinity(0))}
    with mp.get_context("spawn").Pool(P, initializer=_oracle_worker_init) as pool:
        pool.map(_oracle_worker_probe, range(P))  # every worker up before the clock starts
        t0 = time.perf_counter()
        parts = pool.map(_oracle_rows, [(w, j, P) for j in range(P)])
        t_pool = time.perf_counter() - t0
    op = np.zeros(w.Nf, np.complex128)
    oc = np.zeros(w.Nf, np.complex128)
    for _, hp, hc, _ in parts:
        op += hp
        oc += hc
    err_full = max(float(np.linalg.norm(gpu_hp - op) / np.linalg.norm(op)),
                   float(np.linalg.norm(gpu_hc - oc) / np.linalg.norm(oc)))
    progress(f"cpu baseline: oracle on {P} processes, whole 3842-mode waveform in {t_pool:.1f} s "
             f"(GPU rel L2 against it {err_full:.2e})")
    res.update({
        "value": 1.0 / t_pool, "cores": P,
        "sample": (f"full size: the whole 3842-mode waveform ({w.Nf} bins, {evals_full} mode-bin evals) on "
                   f"{P} worker processes, mode rows dealt round-robin, parts summed; {t_pool:.1f} s per "
                   f"waveform (slowest worker {max(x[3] for x in parts):.1f} s)"),
        "evals_per_s": evals_full / t_pool,
        "gpu_rel_l2_vs_oracle_all_bins": err_full,
    })
    with threadpool_limits(limits=1):
        sub = _row_subset(w, 0, sample_stride)
        t0 = time.perf_counter()
        oracle.waveform(sub)
        t_s = time.perf_counter() - t0
        t_full = t_s * sample_stride
        res["single_process"] = {
            "value": 1.0 / t_full, "cores": 1, "extrapolated": True,
            "sample": (f"one mode row in {sample_stride} ({sub.Nm} of {w.Nm}) on the whole grid: {t_s:.1f} s, "
                       f"scaled by {sample_stride}: {t_full:.0f} s per waveform"),
        }
        progress(f"cpu baseline: single process sample {t_s:.1f} s")
        full_small = {}
        for name, wl, gpu_s in small:
            t0 = time.perf_counter()
            oracle.waveform(wl)
            ts = time.perf_counter() - t0
            full_small[name] = {"oracle_s_per_waveform": ts, "gpu_s_per_waveform": gpu_s,
                                "bins": wl.Nf, "cores": 1}
        res["full_size_single_process"] = full_small
    return res


def device_noise(f, df, seed, dev, dtype):
    """Complex Gaussian noise per channel with Re, Im ~ N(0, S/(4 df)) drawn
    on the device (torch's seeded generator), the distribution of
    workloads.noise_draw without its host cost at batch size."""
    import numpy as np
    import torch
    S = W_psd(f)
    sig = torch.as_tensor(np.sqrt(np.where(np.isfinite(S), S, 0.0) / (4.0 * df)), device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    out = []
    for _ in range(2):
        re = torch.randn(sig.numel(), generator=g, device=dev, dtype=torch.float64)
        im = torch.randn(sig.numel(), generator=g, device=dev, dtype=torch.float64)
        out.append(torch.complex(sig * re, sig * im).to(dtype))
    return out


def W_psd(f):
    import workloads as W
    return W.psd_closed_form(f)


def batch_measure(ctx, W, fd, dev, B, with_loglike=True, reps=2):
    """Mixed-precision batch of B draws from the batched distribution (M
    log-U[1e5,1e7], mu U[1,100], e0 U[0.05,0.5], p0 U[10,16], T U[0.5,4] yr,
    dt = 10 s, full DFT grids): one eager profiled call gives the persistent
    gather kernel's own duration (its roofline); the timed calls are replays
    of the captured batch (a context with batch graphs); each waveform's error
    against the FP64 batch; then the same batch with the Hann-windowed Whittle
    likelihood fused in (no waveform written)."""
    import torch
    ws = [W.batch_workload(prm) for prm in W.batch_params(B, 4)]
    dws = [fd.DeviceWaveform.from_workload(w, device=dev) for w in ws]
    bins = sum(w.Nf for w in ws)
    progress(f"batch: {B} waveforms, {bins} bins on the device")
    outs = [(torch.empty(d.Nf, dtype=torch.complex64, device=dev),
             torch.empty(d.Nf, dtype=torch.complex64, device=dev)) for d in dws]
    # eager, profiled: the gather kernel's duration and the evaluation count
    ctx.profile(True, classes=["gather"])
    ctx.profile_read()
    ctx.waveform_batch(dws, "mixed", outs=outs)
    g_ms, g_n = ctx.profile_read()["gather"]
    ctx.profile(False)
    assert ctx.sync_flags() == 0
    evals = ctx.last_eval_count()
    group_evals = ctx.last_group_eval_count()
    progress(f"batch: eager mixed batch, gather {g_ms:.0f} ms ({evals} evals, {group_evals} group evals)")
    # graph path: capture on the first call, then replays
    gctx = fd.Context(dev.index if dev.index is not None else 0, graphs=True)
    gctx.waveform_batch(dws, "mixed", outs=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        gctx.waveform_batch(dws, "mixed", outs=outs)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    progress(f"batch: mixed {sec:.3f} s per batch (graph replays)")
    gctx.close()
    ref = ctx.waveform_batch(dws, "fp64")
    torch.cuda.synchronize()
    errs = []
    for (mp, mc), (rp, rc) in zip(outs, ref):
        for x, y in ((mp, rp), (mc, rc)):
            nb = float(torch.linalg.vector_norm(y))
            if nb > 0:
                errs.append(float(torch.linalg.vector_norm(x.to(torch.complex128) - y)) / nb)
    progress("batch: FP64 reference done")
    g_avg = g_ms / max(g_n, 1) * 1e-3
    achieved = algorithmic_flops(evals, group_evals) / g_avg
    res = {"waveforms": B, "bins": bins, "evals": evals, "group_evals": group_evals, "seconds_per_batch": sec,
           "path": "hipGraph replay (captured on the first call, FDEMRI_CTX_BATCH_GRAPHS)",
           "waveforms_per_s": B / sec, "evals_per_s": evals / sec,
           "rel_l2_vs_fp64_max": max(errs), "rel_l2_vs_fp64_median": sorted(errs)[len(errs) // 2],
           "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                        "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU,
                        "traffic": profile_traffic(BATCH_TRAFFIC_FILE, "gather_batch_kernel<true, 1, 4, false>"),
                        # no batch autotune runs here: the default block shape, 1 tile per wave
                        "kernel": "gather_batch_kernel<true, 1, 4, false>", "kernel_ms": g_avg * 1e3,
                        "flops_per_group_eval": FLOPS_PER_EVAL,
                        "mode_bin_evals_per_s_in_kernel": evals / g_avg,
                        "peak_note": ("without packed FP32 (off in this build) FP32 and FP64 vector instructions "
                                      "issue at the same rate, so the FP64 vector peak bounds the mixed path")}}
    del outs
    if with_loglike:
        # data = FP64 waveform + device noise of the closed-form PSD, Hann-windowed comparison
        import numpy as np
        dps, dcs, wss = [], [], []
        for i, (w, (rp, rc)) in enumerate(zip(ws, ref)):
            S = W.psd_closed_form(w.f)
            df = float(w.f[1] - w.f[0])
            wss.append(torch.as_tensor(np.where(np.isfinite(S), 4.0 * df / np.where(np.isfinite(S), S, 1.0), 0.0),
                                       device=dev))
            n_p, n_c = device_noise(w.f, df, 31 + i, dev, torch.complex128)
            dps.append((rp + n_p).to(torch.complex64).contiguous())
            dcs.append((rc + n_c).to(torch.complex64).contiguous())
        del ref
        progress("batch: likelihood data on the device")
        llo = ctx.loglike_batch(dws, dps, dcs, wss, prec="mixed", hann=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.loglike_batch(dws, dps, dcs, wss, prec="mixed", hann=True, out=llo)
        torch.cuda.synchronize()
        sec_ll = time.perf_counter() - t0
        progress(f"batch: fused likelihood {sec_ll:.3f} s per batch")
        del dps, dcs, wss
        res["loglike_fused_hann"] = {"seconds_per_batch": sec_ll, "waveforms_per_s": B / sec_ll,
                                     "evals_per_s": evals / sec_ll, "waveform_bytes_not_written": bins * 16}
    return res


def small_workloads(W):
    """The latency-bound workloads: 20 modes on the full DFT grid and on 1e4
    log-spaced bins."""
    return (("inspiral_20_modes_fp64", W.inspiral_20_modes()),
            ("inspiral_20_modes_log_grid_fp64", W.inspiral_20_modes_log_grid()))


def small_latency(ctx, fd, dev, wl, reps=200):
    """Microseconds per FP64 waveform for back-to-back eager calls (host
    launch work included) and per replay of the call captured in a graph."""
    import torch
    d2 = fd.DeviceWaveform.from_workload(wl, device=dev)
    o2 = (torch.empty(d2.Nf, dtype=torch.complex128, device=dev),
          torch.empty(d2.Nf, dtype=torch.complex128, device=dev))
    for _ in range(5):
        ctx.waveform_dev(d2, "fp64", out=o2)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(reps):
        ctx.waveform_dev(d2, "fp64", out=o2)
    torch.cuda.synchronize()
    return {"us_per_waveform": (time.perf_counter() - ts) / reps * 1e6,
            "us_per_waveform_graph_replay": graph_latency(fd, d2)}


def graph_latency(fd, dw, reps=50):
    """Microseconds per FP64 waveform when the call is captured once into a
    HIP graph (torch's capture of the current stream) and replayed: the
    launch-bound small workloads without per-call host launch work.  The
    graph holds its context's workspace, so it gets a context of its own."""
    import torch
    gctx = fd.Context(dw.device.index if dw.device.index is not None else 0)
    out = (torch.empty(dw.Nf, dtype=torch.complex128, device=dw.device),
           torch.empty(dw.Nf, dtype=torch.complex128, device=dw.device))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(3):
            gctx.waveform_dev(dw, "fp64", out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gctx.waveform_dev(dw, "fp64", out=out)
    for _ in range(3):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    us = (time.perf_counter() - t0) / reps * 1e6
    del g
    gctx.close()
    return us


def adjoint_measure(ctx, W, fd, dev, B):
    """Forward plus adjoint of the Whittle log-likelihood for B draws of the
    batched distribution (seed 1) in mixed precision: the forward of all B
    templates in one persistent launch, then per draw the cotangent
    wS (d - h) and fdemri_vjp, all enqueued before one synchronisation.
    Data: the FP64 waveform at the drawn parameters plus device noise of the
    closed-form PSD; template: the same source with perturbed amplitudes,
    phase offset and inclination, so that the residual carries signal as well
    as noise.  Errors against the FP64 forward+adjoint are reported per
    gradient group, end to end (mixed forward and mixed adjoint) and for the
    adjoint alone (the FP64 cotangent rounded to complex64).  The adjoint
    kernel's duration comes from HIP events around its launches in a
    separate (warm-up) pass."""
    import dataclasses
    import numpy as np
    import torch
    ws = [W.batch_workload(prm) for prm in W.batch_params(B, 1)]
    keys = ("gA_knots", "gPhi_knots", "g_scalars")
    dws, data = [], []
    for i, w in enumerate(ws):
        dw_true = fd.DeviceWaveform.from_workload(w, device=dev)
        traj = dataclasses.replace(w.traj, Phiphi=w.traj.Phiphi + 0.3)
        tpl = dataclasses.replace(w, traj=traj, A=w.A * (1.02 * np.exp(0.05j)), theta=w.theta + 0.01)
        dws.append(fd.DeviceWaveform.from_workload(tpl, device=dev))
        df = float(w.f[1] - w.f[0])
        S = W.psd_closed_form(w.f)
        wS = torch.as_tensor(np.where(np.isfinite(S), 4.0 * df / np.where(np.isfinite(S), S, 1.0), 0.0), device=dev)
        tp, tc = ctx.waveform_dev(dw_true, "fp64")
        n1, n2 = device_noise(w.f, df, 7 + i, dev, torch.complex128)
        data.append((tp + n1, tc + n2, wS))
        del tp, tc, dw_true
    torch.cuda.synchronize()
    progress(f"forward+adjoint: data of {B} draws on the device")
    mouts = [(torch.empty(d.Nf, dtype=torch.complex64, device=dev),
              torch.empty(d.Nf, dtype=torch.complex64, device=dev)) for d in dws]

    def adjoints():
        grads = []
        for dw, (mp, mc), (dp, dc, wS) in zip(dws, mouts, data):
            gp = (wS * (dp - mp.to(torch.complex128))).to(torch.complex64)
            gc = (wS * (dc - mc.to(torch.complex128))).to(torch.complex64)
            grads.append(ctx.vjp_dev(dw, gp, gc, "mixed", coef=False))
        return grads

    def run():
        ctx.waveform_batch(dws, "mixed", outs=mouts)
        return adjoints()

    # warm-up pass: the forward's evaluation count, then the adjoints with
    # their bin work (plan, scan, chunks, sums) bracketed
    ctx.waveform_batch(dws, "mixed", outs=mouts)
    evals = ctx.last_eval_count()
    group_evals = ctx.last_group_eval_count()
    ctx.profile(True, classes=["vjp"])
    ctx.profile_read()
    adjoints()
    v_ms, v_n = ctx.profile_read()["vjp"]
    ctx.profile(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grads = run()
    torch.cuda.synchronize()
    tot = time.perf_counter() - t0
    progress(f"forward+adjoint: {B} draws in {tot:.2f} s ({evals} forward evals)")

    def rel(a, b):
        nb = float(torch.linalg.vector_norm(b))
        return float(torch.linalg.vector_norm(a.to(b.dtype) - b)) / nb if nb > 0 else 0.0

    e2e = {k: 0.0 for k in keys}
    vjp_only = {k: 0.0 for k in keys}
    fwd_err = 0.0
    for dw, (mp, mc), (dp, dc, wS), g in zip(dws, mouts, data, grads):
        hp, hc = ctx.waveform_dev(dw, "fp64")
        g64p = wS * (dp - hp)
        g64c = wS * (dc - hc)
        ref = ctx.vjp_dev(dw, g64p, g64c, "fp64", coef=False)
        only = ctx.vjp_dev(dw, g64p.to(torch.complex64), g64c.to(torch.complex64), "mixed", coef=False)
        fwd_err = max(fwd_err, rel(mp, hp), rel(mc, hc))
        for k in keys:
            e2e[k] = max(e2e[k], rel(g[k], ref[k]))
            vjp_only[k] = max(vjp_only[k], rel(only[k], ref[k]))
    progress("forward+adjoint: FP64 references done")
    achieved = group_evals * ADJ_FLOPS_PER_GROUP_EVAL / (v_ms * 1e-3)
    return {"waveforms": B, "evals_forward": evals, "group_evals_forward": group_evals, "seconds": tot,
            "waveforms_per_s": B / tot,
            "evals_per_s_forward_plus_adjoint": evals / tot,
            "forward_rel_l2_vs_fp64_max": fwd_err,
            "vjp_kernel_ms_per_waveform": v_ms / max(v_n, 1),
            "grad_rel_l2_vs_fp64_max": e2e, "adjoint_only_rel_l2_vs_fp64_max": vjp_only,
            "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                         "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU,
                         "traffic": profile_traffic(VJP_TRAFFIC_FILE, "vjp_chunk_kernel<true>"),
                         "kernel": "vjp_chunk_kernel<true>", "kernel_ms_total": v_ms,
                         "launches": v_n, "flops_per_group_eval": ADJ_FLOPS_PER_GROUP_EVAL}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the mode sum is measured on a single MI355X", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2307_12585_amd as fd
    import workloads as W

    dev = torch.device("cuda", 0)
    w = W.inspiral_3842_modes()
    ctx = fd.Context(0)
    dw = fd.DeviceWaveform.from_workload(w, device=dev)
    hp = torch.empty(dw.Nf, dtype=torch.complex128, device=dev)
    hc = torch.empty_like(hp)
    out = (hp, hc)

    bpl = None
    if not args.no_autotune:
        bpl = ctx.autotune([dw], "fp64", outs=[out])
        ctx.autotune([dw], "mixed")
    for _ in range(args.warmup):
        ctx.waveform_dev(dw, "fp64", out=out)
    torch.cuda.synchronize()
    assert ctx.sync_flags() == 0
    evals = ctx.last_eval_count()
    group_evals = ctx.last_group_eval_count()

    # timed region: only the gather is bracketed by events (its duration is
    # the roofline's); an event pair around every kernel would add its own
    # gaps to the step
    ctx.profile(True, classes=["gather"])
    ctx.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.waveform_dev(dw, "fp64", out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    sec = (t1 - t0) / args.steps
    g_ms, g_n = prof["gather"]
    g_avg = g_ms / max(g_n, 1) * 1e-3
    achieved = algorithmic_flops(evals, group_evals) / g_avg
    # the set-up kernels' durations, from a few more steps with every class bracketed
    ctx.profile(True)
    for _ in range(10):
        ctx.waveform_dev(dw, "fp64", out=out)
    setup = ctx.profile_read()
    ctx.profile(False)
    for k in ("spline", "pieces"):
        prof[k] = setup[k]

    # secondary measurements (not the headline): mixed precision on the same
    # workload and the latency of the small and sparse-grid workloads
    secondary = {}
    if args.calibrate_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        secondary["copy_calibration_bytes"] = src.numel() * 8
    if args.headline_only or args.only:
        if args.only == "batch":
            secondary["batch_mixed"] = batch_measure(ctx, W, fd, dev, args.batch, with_loglike=False,
                                                     reps=args.batch_reps)
        elif args.only == "adjoint":
            secondary["forward_adjoint"] = adjoint_measure(ctx, W, fd, dev, args.adjoint)
        elif args.only == "small":
            for name, wl in small_workloads(W):
                secondary[name] = small_latency(ctx, fd, dev, wl)
        line = headline(args, w, evals, group_evals, sec, prof, achieved, bpl, secondary)
        print(json.dumps(line), flush=True)
        ctx.close()
        return
    hpm = torch.empty(dw.Nf, dtype=torch.complex64, device=dev)
    hcm = torch.empty_like(hpm)
    for _ in range(3):
        ctx.waveform_dev(dw, "mixed", out=(hpm, hcm))
    torch.cuda.synchronize()
    ts = time.perf_counter()
    nmix = max(5, args.steps // 2)
    for _ in range(nmix):
        ctx.waveform_dev(dw, "mixed", out=(hpm, hcm))
    torch.cuda.synchronize()
    smix = (time.perf_counter() - ts) / nmix
    mix_err = max(float(torch.linalg.vector_norm(hpm.to(torch.complex128) - hp) / torch.linalg.vector_norm(hp)),
                  float(torch.linalg.vector_norm(hcm.to(torch.complex128) - hc) / torch.linalg.vector_norm(hc)))
    secondary["mixed_same_workload"] = {"waveforms_per_s": 1.0 / smix, "ms": smix * 1e3,
                                        "rel_l2_vs_fp64": mix_err}
    secondary["loglike_fused_fp64"] = loglike_measure(ctx, W, dw, hp, hc, dev, max(5, args.steps // 2))
    secondary["td_vs_fd_fp64"] = td_measure(ctx, W, dw, hp, hc, dev, sec)
    # adaptive downsampled grid (Sec. 3.3) for the same source, tol 1e-3 on <h|h>
    from paper_2307_12585_amd.downsample import adaptive_grid, hh_on_grid
    ts = time.perf_counter()
    grid, hist = adaptive_grid(ctx, w, W.psd_closed_form, tol=1e-3, n0=256)
    ds_ms = (time.perf_counter() - ts) * 1e3
    hh_full = hh_on_grid(ctx, w, w.f, W.psd_closed_form)
    secondary["downsampled_grid"] = {"bins": int(grid.size - 1), "full_grid_bins": int(w.f.size),
                                     "hh_downsampled": hist[-2][1], "hh_full_grid": hh_full,
                                     "levels": len(hist), "selection_ms": ds_ms}
    # trajectories on the device: 512 draws of the batch distribution, K = 100
    prms = W.batch_params(512, 77)
    tp = [dict(M=P["M"], mu=P["mu"], p0=P["p0"], e0=P["e0"], T=P["T"]) for P in prms]
    ctx.trajectory(tp[:4], 100)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    ctx.trajectory(tp, 100)
    torch.cuda.synchronize()
    secondary["trajectory_batch"] = {"waveforms": len(tp), "knots": 100,
                                     "ms_per_batch": (time.perf_counter() - ts) * 1e3,
                                     "integrator": "Dormand-Prince 5(4), rtol 1e-12, one thread per waveform"}
    # mode selection on the device: the unselected 3843-row table of the same source
    full = W.inspiral_3842_modes(eps=0.0)
    At = torch.as_tensor(full.A, device=dev)
    ctx.select_modes(At, 1e-5)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(20):
        kept = ctx.select_modes(At, 1e-5)
    secondary["mode_selection"] = {"rows": int(full.l.size), "knots": int(full.traj.t.size), "kept": int(kept.numel()),
                                   "us_per_call": (time.perf_counter() - ts) / 20 * 1e6,
                                   "note": "includes the device-to-host read of the kept count"}
    if args.batch > 0:
        secondary["batch_mixed"] = batch_measure(ctx, W, fd, dev, args.batch, reps=args.batch_reps)
    if args.adjoint > 0:
        secondary["forward_adjoint"] = adjoint_measure(ctx, W, fd, dev, args.adjoint)
    small = []
    for name, wl in small_workloads(W):
        secondary[name] = small_latency(ctx, fd, dev, wl)
        small.append((name, wl, secondary[name]["us_per_waveform"] * 1e-6))

    line = headline(args, w, evals, group_evals, sec, prof, achieved, bpl, secondary)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, hp.cpu().numpy(), hc.cpu().numpy(), evals, small)
    print(json.dumps(line), flush=True)
    ctx.close()


def td_measure(ctx, W, dw, hp, hc, dev, fd_sec):
    """The paper's FD/TD comparison on the same source: the time-domain voice
    sum (fdemri_td_waveform) on the full 10 s grid plus the Hann-windowed
    rfft of both channels, against the FD step; and the mismatch (R12)
    between the windowed TD transform and the FD sum with the matching
    three-tap kernel."""
    import numpy as np
    import torch
    w = W.inspiral_3842_modes()
    dt = w.meta["dt"]
    Nt = 2 * (w.f.size - 1)
    out = (torch.empty(Nt, dtype=torch.float64, device=dev), torch.empty(Nt, dtype=torch.float64, device=dev))
    win = 0.5 - 0.5 * torch.cos(2 * np.pi * torch.arange(Nt, dtype=torch.float64, device=dev) / Nt)
    ctx.td_waveform_dev(dw, 0.0, dt, Nt, out=out)
    torch.fft.rfft(out[0] * win)  # FFT plan set up outside the timed region
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(3):
        torch.fft.rfft(out[0] * win)
    torch.cuda.synchronize()
    fft_ms = (time.perf_counter() - ts) / 3 * 1e3
    ctx.profile(True)
    ctx.profile_read()
    reps = 3
    ts = time.perf_counter()
    for _ in range(reps):
        ctx.td_waveform_dev(dw, 0.0, dt, Nt, out=out)
        tp = dt * torch.conj(torch.fft.rfft(out[0] * win))
        tc = dt * torch.conj(torch.fft.rfft(out[1] * win))
    torch.cuda.synchronize()
    td_sec = (time.perf_counter() - ts) / reps
    k_ms, k_n = ctx.profile_read()["gather"]
    ctx.profile(False)

    def hw(h):
        g = 0.5 * h.clone()
        g[:-1] -= 0.25 * h[1:]
        g[1:] -= 0.25 * h[:-1]
        g[0] -= 0.25 * torch.conj(h[1])
        return g
    S = torch.as_tensor(W.psd_closed_form(w.f), device=dev)
    wts = torch.full_like(S, float(w.f[1] - w.f[0]))
    good = torch.isfinite(S)
    wS = torch.where(good, 4.0 * wts / torch.where(good, S, torch.ones_like(S)), torch.zeros_like(S))
    ip = lambda a, b: float(torch.sum(wS * torch.real(torch.conj(a) * b)))
    fp, fc = hw(hp), hw(hc)
    ab = ip(fp, tp) + ip(fc, tc)
    mm = 1.0 - ab / np.sqrt((ip(fp, fp) + ip(fc, fc)) * (ip(tp, tp) + ip(tc, tc)))
    k_avg = k_ms / max(k_n, 1) * 1e-3
    return {"samples": Nt, "td_kernel_ms": k_avg * 1e3, "rfft_ms_per_channel": fft_ms,
            "td_plus_rfft_ms": td_sec * 1e3,
            "fd_step_ms": fd_sec * 1e3, "fd_speedup_over_td": td_sec / fd_sec,
            "mode_sample_pairs_per_s": w.l.size * Nt / k_avg, "mismatch_fd_vs_windowed_td": mm}


def loglike_measure(ctx, W, dw, hp, hc, dev, steps):
    """Fused Whittle log-likelihood (fdemri_loglike) on the same workload, with
    and without the Hann kernel: time per waveform and the relative difference
    from the same sums taken (in torch, FP64) over the stored FP64 waveform."""
    import numpy as np
    import torch
    f = W.inspiral_3842_modes().f
    S = W.psd_closed_form(f)
    df = float(f[1] - f[0])
    wS = torch.as_tensor(np.where(np.isfinite(S), 4.0 * df / np.where(np.isfinite(S), S, 1.0), 0.0), device=dev)
    n_p, n_c = W.noise_draw(f, df, 21)
    dp = (complex(1.1 * np.exp(0.3j)) * hp + torch.as_tensor(n_p, device=dev)).contiguous()
    dc = (complex(0.9 * np.exp(-0.2j)) * hc + torch.as_tensor(n_c, device=dev)).contiguous()
    res = {}
    for hann in (False, True):
        out = ctx.loglike_dev(dw, dp, dc, wS, hann=hann)
        for _ in range(2):
            ctx.loglike_dev(dw, dp, dc, wS, hann=hann, out=out)
        torch.cuda.synchronize()
        ctx.profile(True)
        ctx.profile_read()
        ts = time.perf_counter()
        for _ in range(steps):
            ctx.loglike_dev(dw, dp, dc, wS, hann=hann, out=out)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - ts) / steps
        g_ms, g_n = ctx.profile_read()["gather"]
        ctx.profile(False)
        # the same sums over the stored waveform
        gp, gc = hp, hc
        if hann:
            def win(h):
                g = 0.5 * h.clone()
                g[:-1] -= 0.25 * h[1:]
                g[1:] -= 0.25 * h[:-1]
                g[0] -= 0.25 * torch.conj(h[1])
                return g
            gp, gc = win(hp), win(hc)
        ref_ll = -0.5 * float(torch.sum(wS * (torch.abs(dp - gp) ** 2 + torch.abs(dc - gc) ** 2)))
        got = out.cpu().numpy()
        res["hann" if hann else "plain"] = {
            "waveforms_per_s": 1.0 / sec, "ms": sec * 1e3, "gather_plus_reduction_ms": g_ms / max(g_n, 1),
            "loglike": float(got[0]), "rel_diff_vs_stored_waveform": abs(float(got[0]) - ref_ll) / abs(ref_ll)}
    # the unfused route for comparison: store the waveform, then the sum in torch
    for _ in range(2):
        ctx.waveform_dev(dw, "fp64", out=(hp, hc))
        float(torch.sum(wS * (torch.abs(dp - hp) ** 2 + torch.abs(dc - hc) ** 2)))
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(steps):
        ctx.waveform_dev(dw, "fp64", out=(hp, hc))
        ll_t = -0.5 * torch.sum(wS * (torch.abs(dp - hp) ** 2 + torch.abs(dc - hc) ** 2))
    torch.cuda.synchronize()
    res["unfused_plain"] = {"ms": (time.perf_counter() - ts) / steps * 1e3,
                            "what": "fdemri_waveform into HBM, then the weighted sum in torch (FP64)"}
    res["note"] = ("log L of data = scaled, phase-shifted model + noise of the closed-form PSD; the model is "
                   "reduced in the gather epilogue and never stored (no 101 MB output write)")
    return res


# HBM bytes per launch of a kernel from rocprofv3 FETCH_SIZE/WRITE_SIZE
# passes (each scaled by what the same counter reads for a device copy of
# known size), recorded with a digest of the kernel's sources; a figure is
# reported only while the sources and the launched instantiation are those
# the counters were taken on (else null).
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gather_fp64_3842modes_hbm_traffic.txt")
BATCH_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gather_batch_mixed_512waveforms_hbm_traffic.txt")
VJP_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "vjp_mixed_64waveforms_hbm_traffic.txt")
GATHER_SOURCES = ["paper_2307_12585_amd/csrc/gather.hip", "paper_2307_12585_amd/csrc/evalcore.hpp",
                  "paper_2307_12585_amd/csrc/spa.hpp", "paper_2307_12585_amd/csrc/w_table.inc",
                  "paper_2307_12585_amd/csrc/fdemri_internal.hpp"]


def sources_digest(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_traffic(path, kernel, key="traffic_bytes_per_launch"):
    """The recorded figure `key` of `kernel` from a counter summary, or None."""
    rec = {}
    try:
        with open(path) as fh:
            for ln in fh:
                if "=" in ln and not ln.lstrip().startswith("#"):
                    k, v = ln.split("=", 1)
                    rec[k.strip()] = v.strip()
        files = [x.strip() for x in rec.get("sources", ",".join(GATHER_SOURCES)).split(",") if x.strip()]
        digest = sources_digest(files)
    except (OSError, KeyError):
        return None
    if digest != rec.get("kernel_sources_sha256") or rec.get("kernel") != kernel or key not in rec:
        return None
    return float(rec[key])


def gather_traffic(bpl):
    return profile_traffic(TRAFFIC_FILE, f"gather_kernel<false, {bpl}, 4, false>")


def headline(args, w, evals, group_evals, sec, prof, achieved, bpl, secondary):
    bpl = bpl or 1  # without the autotuner: the default block shape, 1 tile per wave
    return {
        "metric": METRIC,
        "value": 1.0 / sec,
        "unit": "waveforms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": ("FP64 single waveform, Peters-type toy inspiral M=2e6 mu=20 "
                                "p0=13 e0=0.45, T=2 yr, dt=10 s; l=2..10, m=0..l, n=-30..30 at 1e-5 "
                                "power: 3842 modes, K=200 knots, 3155816 bins"),
                   "modes": w.Nm, "knots": w.K, "bins": w.Nf, "evals": evals, "group_evals": group_evals,
                   "bins_per_lane": bpl},
        "evals_per_s": evals / sec,
        "kernel_ms": {k: (v[0] / max(v[1], 1)) for k, v in prof.items() if v[1]},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU, "traffic": gather_traffic(bpl),
                     "traffic_unit": "HBM bytes per launch (read + write)",
                     "kernel": f"gather_kernel<false, {bpl}, 4, false>", "flops_per_group_eval": FLOPS_PER_EVAL,
                     "mode_bin_evals_per_s_in_kernel": evals / (prof["gather"][0] / max(prof["gather"][1], 1) * 1e-3),
                     "issued_fp64_flops_per_group_eval": profile_traffic(
                         TRAFFIC_FILE, f"gather_kernel<false, {bpl}, 4, false>", "issued_fp64_flops_per_group_eval")},
        "secondary": secondary,
    }


if __name__ == "__main__":
    main()
