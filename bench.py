#!/usr/bin/env python
"""Benchmark: templates/s of the semi-coherent time-frequency statistic on one MI355X.

Workload (the full-size configuration): two years of TDI A+E at dt = 5 s, Nt = 6144
tranches of M = 2048 samples (12,582,912 samples per channel), PSD modulated by +-20 %
on a one-year sinusoid, 7-h gaps every 14 days; bank of 1,000,020 non-spinning
templates (Mc log-uniform in [10, 60] Msun, f0 uniform in [10, 40] mHz, isotropic sky,
uniform polarisation and inclination, plus 20 exact-injection templates), adaptive
N_seg from 16 to 256.  Data and bank are seeded and synthetic.

One step = tfsc_transform (data -> pixels) + tfsc_segment_layout + tfsc_processing_order +
tfsc_bank_statistic over the whole bank, with inputs resident in HBM.  Prints one JSON line.
The WAVE schedule's launch shape comes from the autotuner (timed on a separate 65,536-template
tuning bank, cached per device and workload shape).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

METRIC = "templates/s, semi-coherent stat (2-yr A+E), chosen vs plain @1e-4; HBM roofline %"
HBM_PEAK_GBS = 8000.0
NF = 21


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--templates", type=int, default=1_000_000)
    p.add_argument("--chosen-store", default="f32", choices=["f32", "f16", "bf16", "i16"])
    p.add_argument("--chosen-layout", default="layer_ci", choices=["layer_ci", "layer"],
                   help="pixel layout of the chosen form (channels of a cell adjacent, or one block per channel)")
    p.add_argument("--plain-steps", type=int, default=2)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--block-waves", type=int, default=0, help="fix the launch shape (0 = autotune)")
    p.add_argument("--groups-per-cu", type=int, default=0)
    p.add_argument("--no-order", action="store_true", help="process the bank in its own order")
    p.add_argument("--no-batching", action="store_true",
                   help="skip the batching workload (4M wide-range templates over 16 noise realisations replayed "
                        "from one HIP graph) and the differentiation workload that follows it")
    p.add_argument("--no-follow-up", action="store_true",
                   help="skip the differentiation workload (one VJP and 50 Adam steps on the top 65,536 "
                        "templates of the batching bank)")
    p.add_argument("--no-precision", action="store_true",
                   help="skip the 16-bit pixel stores (FP16, BF16) of the precision form")
    p.add_argument("--no-harmonics", action="store_true",
                   help="skip the multi-harmonic leg (harmonics 1, 2, 3 of the orbital phase on the same data and bank)")
    p.add_argument("--no-links", action="store_true",
                   help="skip the unequal-arm leg (the chosen form with six link light times per tranche on the "
                        "same data and bank)")
    p.add_argument("--interleave", type=int, default=2, choices=[0, 2, 4],
                   help="also time the batching workload with 2 or 4 realisations interleaved cell by cell in one "
                        "store and evaluated in one pass over the bank (0: skip)")
    p.add_argument("--interleave-store", default="i16", choices=["f32", "i16"],
                   help="pixel type of the interleaved batching store (i16: int16 fixed point, per-layer scale)")
    p.add_argument("--eight-per-pass", action="store_true",
                   help="also time the several-realisation pass (eight realisations per pass over the bank)")
    p.add_argument("--background", action="store_true",
                   help="also build the background of the batching workload: per-tile maxima of the 16 "
                        "realisations on an 8 x 8 (Mc, f0) tile grid, power-law and Gumbel tail fits")
    p.add_argument("--ladder", action="store_true",
                   help="also run the segment ladder N_seg 16 -> 8 -> 4 -> 2 -> 1 (20 ascent steps per stage) "
                        "on the top 65,536 templates of the batching bank")
    p.add_argument("--psd-tf", action="store_true",
                   help="also time the chosen form with a PSD that varies between tranches in a general way "
                        "(per-pixel whitening and weights), with sampled parity against the oracle")
    p.add_argument("--aet", action="store_true",
                   help="also time the chosen form on three channels (A, E and the null channel T) of the same "
                        "2-yr grid and bank, with sampled parity against the oracle")
    p.add_argument("--copy-calibration", action="store_true",
                   help="copy 256 MiB device-to-device once, so profiler byte counters can be calibrated")
    p.add_argument("--summarize-counters", nargs="+", metavar="DIR",
                   help="no GPU run: write profiles/k_stat_wave_counters.txt from rocprofv3 --pmc CSV directories "
                        "of this bench's chosen statistic launch (with --templates, --chosen-store, "
                        "--chosen-layout, --block-waves, --groups-per-cu as profiled)")
    p.add_argument("--vjp-profile", action="store_true",
                   help="only the differentiation kernels, for profiling: on the 2-yr grid, the first 65,536 "
                        "templates of the bench's bank, one FP32 statistic (with z_n) and --steps launches each of "
                        "the statistic, the FP64 VJP and the FP32 VJP; prints one JSON line of event timings")
    p.add_argument("--batching-profile", action="store_true",
                   help="only the batching kernels, for profiling: the first 1,000,000 templates of the batching bank "
                        "over 4 noise realisations, one graph replay each of one FP32 launch per realisation, FP32 "
                        "pairs and int16 pairs interleaved per store; prints one JSON line of timings")
    p.add_argument("--fetch-factor", type=float, default=2.0,
                   help="bytes per FETCH_SIZE KiB / 1024 from the copy calibration")
    p.add_argument("--write-factor", type=float, default=1.0,
                   help="bytes per WRITE_SIZE KiB / 1024 from the copy calibration")
    return p.parse_args()


def main():
    args = parse()
    if args.summarize_counters:
        n = args.templates + 20
        summarize_counters(args.summarize_counters, n, args.chosen_store, args.chosen_layout,
                           "bank" if args.no_order else "f0 bin, ln Mc", f"{args.block_waves}x{args.groups_per_cu}",
                           args.fetch_factor, args.write_factor)
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}): templates shard across GPUs with no "
              f"exchange in the hot loop, and the benchmark measures one GPU's throughput only", file=sys.stderr)
        sys.exit(2)
    import torch
    import tfsc_inputs as ti
    noise_jobs = None
    if not (args.no_batching or args.vjp_profile or args.batching_profile):
        # the batching workload's 16 noise realisations are drawn on the host by worker processes forked
        # here, before this process touches the GPU; they run while the GPU works on the rest
        import multiprocessing as mp
        from concurrent.futures import ProcessPoolExecutor
        workers = max(1, min(8, len(os.sched_getaffinity(0)) // 2))
        pool = ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork"))
        noise_jobs = (pool, [pool.submit(_noise_realisation, r) for r in range(16)], workers)
    import paper_2510_19047_amd as tfsc
    tfsc.lib()
    dev = torch.device("cuda:0")
    g = ti.FULL
    grid = tfsc.GridSpec(g.n_channels, g.tranche_len, g.n_tranches, g.dt, 0.1)
    if args.vjp_profile:
        vjp_profile_run(args, tfsc, ti, g, grid, dev)
        return
    if args.batching_profile:
        batching_profile_run(tfsc, ti, g, grid, dev)
        return

    log("generating synthetic data (noise, gaps, modulation) and bank")
    x = (ti.noise(g) * ti.sample_keep_mask(g)[None, :]).astype(np.float32)
    psd, mu, keep = ti.psd_on_bins(g), ti.tranche_psd_scale(g), ti.tranche_keep(g)
    bank_h = ti.full_bank(args.templates)
    n = len(bank_h)
    x_d = torch.from_numpy(x).to(dev)
    psd_d, mu_d = torch.from_numpy(psd).to(dev), torch.from_numpy(mu).to(dev)
    keep_d = torch.from_numpy(keep).to(dev)
    bank = tfsc.BankTensors.from_host(bank_h, dev)

    if args.copy_calibration:
        a_ = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        b_ = torch.empty_like(a_)
        torch.cuda.synchronize()
        b_.copy_(a_)
        torch.cuda.synchronize()
        log("copy calibration: 268435456 bytes read, 268435456 bytes written")
        del a_, b_

    # first pass: layout with total read-back, allocations reused by every timed step
    seg = tfsc.segment_layout(grid, bank)
    pix_chosen = tfsc.transform(grid, x_d, psd_d, mu_d, keep_d, dtype=args.chosen_store, layout=args.chosen_layout)
    pix_plain = tfsc.transform(grid, x_d, psd_d, mu_d, keep_d, dtype="f32", layout="tranche")
    res = tfsc.bank_statistic(grid, pix_chosen, bank, seg, precision="f32", schedule="wave", want_active=True)
    torch.cuda.synchronize()
    n_active = res.n_active.cpu().numpy().astype(np.int64)
    b_pix = {"f32": 8, "f16": 4, "bf16": 4, "i16": 4}[args.chosen_store]
    pix_cols = int(n_active.sum())
    alg_bytes = pix_cols * NF * g.n_channels * b_pix + n * 56 + 8 * (seg.total + n)
    alg_bytes_f32 = pix_cols * NF * g.n_channels * 8 + n * 56 + 8 * (seg.total + n)
    log(f"bank {n} templates, mean active tranches {n_active.mean():.0f}, segments {seg.total}, "
        f"algorithmic bytes {alg_bytes / 1e12:.3f} TB")

    order = None if args.no_order else tfsc.processing_order(grid, bank)
    if args.block_waves > 0:
        shape = (args.block_waves, args.groups_per_cu if args.groups_per_cu > 0 else 4)
    else:
        from paper_2510_19047_amd import batching
        tune_h = ti.random_bank(65536, 5, mc_range=(10.0, 60.0), f0_range=(0.010, 0.040), stream=77)
        tune = tfsc.BankTensors.from_host(tune_h, dev)
        tune_seg = tfsc.segment_layout(grid, tune)
        shape = batching.autotune(grid, pix_chosen, tune, tune_seg, precision="f32",
                                  order=None if args.no_order else tfsc.processing_order(grid, tune))
        del tune, tune_seg
    kw = dict(block_waves=shape[0], groups_per_cu=shape[1])
    log(f"launch shape: {shape[0]} waves per block, {shape[1]} blocks per CU; "
        f"order: {'bank order' if order is None else 'by f0 bin, then ln Mc class (device counting sort)'}")

    def step(store_dtype, layout, schedule, pix_out, res_out):
        tfsc.transform(grid, x_d, psd_d, mu_d, keep_d, dtype=store_dtype, layout=layout, out=pix_out)
        tfsc.segment_layout(grid, bank, out=seg, read_total=False)
        if schedule == "wave":
            o = None if order is None else tfsc.processing_order(grid, bank, out=order)
            return tfsc.bank_statistic(grid, pix_out, bank, seg, precision="f32", schedule=schedule, out=res_out,
                                       order=o, **kw)
        return tfsc.bank_statistic(grid, pix_out, bank, seg, precision="f32", schedule=schedule, out=res_out)

    # ---------------- chosen form: wave-per-template schedule
    res_c = tfsc.StatResult(torch.empty(n, dtype=torch.float64, device=dev),
                            torch.empty(seg.total, dtype=torch.float64, device=dev),
                            torch.empty(n, dtype=torch.int32, device=dev))
    for i in range(args.warmup):
        step(args.chosen_store, args.chosen_layout, "wave", pix_chosen, res_c)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.chosen_store, args.chosen_layout, "wave", pix_chosen, res_c)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    value = n / (ms_step / 1e3)
    log(f"chosen: {ms_step:.2f} ms/step, {value / 1e6:.3f} M templates/s")

    # kernel-only timing of the statistic launch (events on the launch stream)
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ks = []
    for i in range(max(args.steps, 3)):
        ev[0].record(st)
        tfsc.bank_statistic(grid, pix_chosen, bank, seg, precision="f32", schedule="wave", out=res_c, order=order,
                            **kw)
        ev[1].record(st)
        torch.cuda.synchronize()
        ks.append(ev[0].elapsed_time(ev[1]))
    k_ms = float(np.median(ks))
    achieved = alg_bytes / (k_ms / 1e3) / 1e9
    log(f"chosen statistic kernel: {k_ms:.2f} ms, {achieved:.0f} GB/s algorithmic ({100 * achieved / HBM_PEAK_GBS:.1f}% of 8 TB/s)")

    # ---------------- plain form: one thread per template (the paper's mapping), tranche-major store
    res_p = tfsc.StatResult(torch.empty(n, dtype=torch.float64, device=dev),
                            torch.empty(seg.total, dtype=torch.float64, device=dev),
                            torch.empty(n, dtype=torch.int32, device=dev))
    step("f32", "tranche", "thread", pix_plain, res_p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.plain_steps):
        step("f32", "tranche", "thread", pix_plain, res_p)
        torch.cuda.synchronize()
        log(f"plain step {i + 1}/{args.plain_steps} done")
    plain_ms = 1e3 * (time.perf_counter() - t0) / args.plain_steps
    plain_value = n / (plain_ms / 1e3)
    log(f"plain: {plain_ms:.2f} ms/step, {plain_value / 1e6:.3f} M templates/s")
    ev[0].record(st)
    tfsc.bank_statistic(grid, pix_plain, bank, seg, precision="f32", schedule="thread", out=res_p)
    ev[1].record(st)
    torch.cuda.synchronize()
    plain_k_ms = ev[0].elapsed_time(ev[1])

    # agreement of the two forms
    sc, sp = res_c.stat.cpu().numpy(), res_p.stat.cpu().numpy()
    rel_cp = float(np.max(np.abs(sc - sp) / np.maximum(np.abs(sp), 1.0)))

    # ---------------- the roofs: vector-ALU issue binds; HBM and algorithmic bytes reported beside it
    prof = measured_profile(n, args.chosen_store, args.chosen_layout, "bank" if order is None else "f0 bin, ln Mc")
    k_s = k_ms / 1e3
    roofline = alu_roofline(prof, k_s)
    traffic = None if prof is None else prof.get("traffic_bytes")
    roofline.update({
        "traffic": traffic,
        "kernel": "k_stat_wave",
        "kernel_ms": round(k_ms, 3),
        "profile_launch_shape": None if prof is None else prof.get("launch_shape"),
        "alg_bytes_per_launch": alg_bytes,
        "alg_gbs": round(achieved, 1),
        "alg_bytes_over_hbm_peak": round(achieved / HBM_PEAK_GBS, 4),
        "alg_bytes_note": "algorithmic gathered bytes per launch / kernel time / 8 TB/s; the 100 MB pixel store "
                          "is reused by the templates in flight and served from L2 and the Infinity Cache, so this "
                          "ratio is not an HBM fraction",
        "hbm": None if traffic is None else {
            "beyond_l2_bytes": traffic, "gbs": round(traffic / k_s / 1e9, 1),
            "frac_of_8tbs": round(traffic / k_s / 1e9 / HBM_PEAK_GBS, 4),
            "note": "calibrated FETCH_SIZE + WRITE_SIZE (bytes beyond L2, Infinity-Cache hits included)"},
    })
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "templates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "2-yr TDI A+E, dt 5 s, Nt 6144 x M 2048, PSD +-20% 1-yr modulation, 7-h gaps every 14 d; "
                        f"{n} non-spinning 2PN templates, adaptive Nseg 16-256",
            "n_templates": n,
            "pixel_store": args.chosen_store,
            "pixel_layout": args.chosen_layout,
            "schedule": "wave-per-template persistent",
            "launch_shape": {"block_waves": kw["block_waves"], "groups_per_cu": kw["groups_per_cu"]},
            "order": "bank" if order is None else "f0 bin, ln Mc",
            "step": "transform + segment layout + processing order + bank statistic",
        },
        "roofline": roofline,
        "forms": {
            "chosen": {"templates_per_s": round(value, 1), "kernel_ms": round(k_ms, 3),
                       "store": f"{args.chosen_store} {args.chosen_layout}",
                       "arith": "f32 (track f64)"},
            "plain": {"templates_per_s": round(plain_value, 1), "ms_per_step": round(plain_ms, 3),
                      "kernel_ms": round(plain_k_ms, 3), "store": "f32 tranche-major", "arith": "f32 (track f64)",
                      "schedule": "thread-per-template"},
            "chosen_over_plain": round(value / plain_value, 3),
            "max_rel_diff_chosen_vs_plain": rel_cp,
        },
    }

    # ---------------- accuracy against the FP64 oracle (outside the timed region): 10k-template subsample
    log("oracle: transform of the same data and the plain-C FP64 statistic on a 10,000-template subsample")
    from oracle import cpu as ocpu
    from oracle import transform as otf
    pix_o, u_o, wm_o = otf.transform(x.astype(np.float64), g, psd, mu, keep, 0.1, "rfft")
    sub_idx = ti.subsample_indices(n, min(10_000, n), must_include=np.arange(max(0, n - 20), n), cfg_id=13)
    threads = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    ref = ocpu.statistic(pix_o, u_o, wm_o, bank_h.subset(sub_idx), g, threads=threads)
    log(f"oracle: {len(sub_idx)} templates in {time.perf_counter() - t0:.1f} s on {threads} threads")
    flags_c = res_c.flags.cpu().numpy()
    out["forms"]["chosen"]["vs_oracle"] = accuracy(sc[sub_idx], flags_c[sub_idx], ref)
    out["forms"]["plain"]["vs_oracle"] = accuracy(sp[sub_idx], res_p.flags.cpu().numpy()[sub_idx], ref)
    log(f"chosen vs oracle: {out['forms']['chosen']['vs_oracle']}")

    # ---------------- multi-harmonic templates on the same store and bank
    if not args.no_harmonics:
        out["harmonics"] = harmonics_run(args, tfsc, grid, g, pix_chosen, bank, bank_h, seg, order, kw, k_ms, pix_o,
                                         u_o, wm_o)

    # ---------------- unequal arms: six link light times per tranche on the same store and bank
    if not args.no_links:
        out["links"] = links_run(args, tfsc, grid, g, pix_chosen, bank, bank_h, seg, order, kw, k_ms, pix_o, u_o,
                                 wm_o)

    # ---------------- precision form: 16-bit pixel stores with a per-layer FP32 scale
    if not args.no_precision:
        del pix_plain
        out["forms"]["precision"] = precision_run(args, tfsc, grid, x_d, psd_d, mu_d, keep_d, bank, seg, order, kw,
                                                  res_c, sub_idx, ref, value)

    if args.aet:
        out["aet"] = aet_run(args, tfsc, ti, g, psd_d, mu_d, keep_d, bank, bank_h, seg, order, kw, pix_cols, value,
                             k_ms)
    if args.psd_tf:
        out["psd_tf"] = psd_tf_run(args, tfsc, ti, grid, g, x, x_d, keep_d, bank, bank_h, seg, order, kw, pix_cols,
                                   value, k_ms)
    if not args.no_batching:
        del res, res_c, res_p
        torch.cuda.empty_cache()
        out["forms"]["batching"] = batching_run(args, tfsc, ti, grid, g, psd_d, mu_d, keep_d, kw, k_ms / n, noise_jobs)
    # ---------------- CPU baseline: the oracle on host cores, bounded samples
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, pix_o, u_o, wm_o, bank_h, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def harmonics_run(args, tfsc, grid, g, pix, bank, bank_h, seg, order, kw, k_ms_one, pix_o, u_o, wm_o):
    """Templates of harmonics 1, 2 and 3 of the orbital phase (seeded complex factors per template: |a_1| = 0.3,
    a_2 = 1, |a_3| = 0.4, random phases) on the chosen form's store and bank: the statistic kernel timed with
    events, and sampled templates against the oracle's harmonic statistic."""
    import torch
    from oracle import harmonics as oh
    n = bank.n
    hs = [1, 2, 3]
    rng = np.random.default_rng(23)
    amps = np.stack([0.3 * np.exp(2j * np.pi * rng.random(n)), np.ones(n, dtype=np.complex128),
                     0.4 * np.exp(2j * np.pi * rng.random(n))], axis=1)
    amp_d = torch.from_numpy(amps).to(bank.device)
    res = tfsc.bank_statistic_harmonics(grid, pix, bank, seg, hs, amp_d, precision="f32", order=order, **kw)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    ks = []
    for _ in range(3):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(st)
        tfsc.bank_statistic_harmonics(grid, pix, bank, seg, hs, amp_d, precision="f32", order=order, out=res, **kw)
        ev[1].record(st)
        torch.cuda.synchronize()
        ks.append(ev[0].elapsed_time(ev[1]))
    k_ms = float(np.median(ks))
    s = res.stat.cpu().numpy()
    idx = sorted(set(np.argsort(-np.nan_to_num(s, nan=-1.0))[:3].tolist()) |
                 set(np.random.default_rng(29).choice(n, 9, replace=False).tolist()))
    ref = oh.statistic(pix_o, u_o, wm_o, bank_h.subset(idx), g, hs, amps[idx])
    r = np.abs(s[idx] - ref.stat) / np.maximum(np.abs(ref.stat), 1.0)
    flags_ok = bool(np.array_equal(res.flags.cpu().numpy()[idx], ref.flags))
    log(f"harmonics {hs}: statistic kernel {k_ms:.2f} ms ({n / (k_ms / 1e3) / 1e6:.3f} M templates/s, "
        f"{k_ms / k_ms_one:.2f}x the single-harmonic kernel); {len(idx)} sampled templates vs oracle max rel "
        f"{r.max():.2e}, flags equal {flags_ok}")
    return {"workload": "same 2-yr grid, store and bank; harmonics 1, 2, 3 with seeded complex factors "
                        "(|a1| 0.3, a2 1, |a3| 0.4)", "harmonics": hs, "kernel_ms": round(k_ms, 3),
            "templates_per_s_kernel": round(n / (k_ms / 1e3), 1), "kernel_over_single": round(k_ms / k_ms_one, 4),
            "store": f"f32 {args.chosen_layout}", "arith": "f32 (track f64)",
            "sampled_parity": {"templates": len(idx), "max_rel_vs_oracle": float(r.max()), "flags_equal": flags_ok}}


def links_run(args, tfsc, grid, g, pix, bank, bank_h, seg, order, kw, k_ms_eq, pix_o, u_o, wm_o):
    """The chosen form with a caller's link light times (unequal arms): the analytic orbit's |p_r - p_s|
    (tfsc_link_lengths), arm a flexing by +-1% over a year (phase 2 pi a / 3) and each reverse link 1e-5 longer
    (a point-ahead scale difference).  The statistic kernel timed with events against the equal-arm kernel, and
    sampled templates against the oracle's unequal-arm statistic."""
    import dataclasses
    import torch
    from oracle import o2
    from oracle import track as otrk
    n = bank.n
    lk = tfsc.link_lengths(grid)
    t = torch.arange(g.n_tranches, dtype=torch.float64, device=lk.device) * g.tranche_dur
    yr = 31557600.0
    flex = torch.stack([0.01 * torch.sin(2.0 * np.pi * t / yr + 2.0 * np.pi * a / 3.0) for a in range(3)])
    lk = (lk * (1.0 + torch.cat([flex, flex])) * torch.tensor([1, 1, 1, 1 + 1e-5, 1 + 1e-5, 1 + 1e-5],
                                                               dtype=torch.float64, device=lk.device)[:, None])
    lk = lk.contiguous()
    store = dataclasses.replace(pix, links=lk)
    res = tfsc.bank_statistic(grid, store, bank, seg, precision="f32", schedule="wave", order=order, **kw)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    ks = []
    for _ in range(3):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(st)
        tfsc.bank_statistic(grid, store, bank, seg, precision="f32", schedule="wave", out=res, order=order, **kw)
        ev[1].record(st)
        torch.cuda.synchronize()
        ks.append(ev[0].elapsed_time(ev[1]))
    k_ms = float(np.median(ks))
    s = res.stat.cpu().numpy()
    # the second TDI generation on the same geometry: kernel time only
    store2 = dataclasses.replace(store, tdi_generation=2)
    res2 = tfsc.bank_statistic(grid, store2, bank, seg, precision="f32", schedule="wave", order=order, **kw)
    ks2 = []
    for _ in range(3):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(st)
        tfsc.bank_statistic(grid, store2, bank, seg, precision="f32", schedule="wave", out=res2, order=order, **kw)
        ev[1].record(st)
        torch.cuda.synchronize()
        ks2.append(ev[0].elapsed_time(ev[1]))
    k2_ms = float(np.median(ks2))
    del res2
    idx = sorted(set(np.argsort(-np.nan_to_num(s, nan=-1.0))[:3].tolist()) |
                 set(np.random.default_rng(31).choice(n, 5, replace=False).tolist()))
    sub = bank_h.subset(idx)
    ref = o2.statistic(pix_o, u_o, wm_o, sub, g, layout=otrk.Layout(sub, g), links=lk.cpu().numpy())
    r = np.abs(s[idx] - ref.stat) / np.maximum(np.abs(ref.stat), 1.0)
    flags_ok = bool(np.array_equal(res.flags.cpu().numpy()[idx], ref.flags))
    log(f"links: statistic kernel {k_ms:.2f} ms ({n / (k_ms / 1e3) / 1e6:.3f} M templates/s, {k_ms / k_ms_eq:.3f}x "
        f"the equal-arm kernel; second TDI generation {k2_ms:.2f} ms); {len(idx)} sampled templates vs oracle max "
        f"rel {r.max():.2e}, flags equal {flags_ok}")
    return {"workload": "same 2-yr grid, store and bank; link light times |p_r - p_s| of the analytic orbit, arms "
                        "flexing +-1% over a year, reverse links 1e-5 longer",
            "kernel_ms": round(k_ms, 3), "templates_per_s_kernel": round(n / (k_ms / 1e3), 1),
            "kernel_over_equal_arm": round(k_ms / k_ms_eq, 4), "kernel_ms_tdi2": round(k2_ms, 3),
            "kernel_over_equal_arm_tdi2": round(k2_ms / k_ms_eq, 4), "store": f"f32 {args.chosen_layout}",
            "arith": "f32 (track and f k.p FP64)",
            "sampled_parity": {"templates": len(idx), "max_rel_vs_oracle": float(r.max()), "flags_equal": flags_ok}}


def batching_profile_run(tfsc, ti, g, grid, dev):
    """One statistic launch per realisation against realisations interleaved in pairs (FP32 and int16) on 1M
    templates of the batching bank and 4 realisations, each as a replayed graph timed by wall clock (the run
    rocprofv3 profiles for the interleaved kernel)."""
    import torch
    from paper_2510_19047_amd import batching
    R = 4
    keep = ti.sample_keep_mask(g)[None, :]
    xs = torch.stack([torch.from_numpy((ti.noise(g, realisation=r) * keep).astype(np.float32))
                      for r in range(R)]).to(dev)
    psd, mu, kp = (torch.from_numpy(a).to(dev) for a in (ti.psd_on_bins(g), ti.tranche_psd_scale(g),
                                                           ti.tranche_keep(g)))
    bank = tfsc.BankTensors.from_host(ti.batching_bank(1_000_000), dev)
    seg = tfsc.segment_layout(grid, bank)
    order = tfsc.processing_order(grid, bank)
    kw = dict(block_waves=4, groups_per_cu=4)

    def timed(rg, reps=3):
        rg.replay()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            rg.replay()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    out = {"workload": "first 1,000,000 templates of the batching bank x 4 noise realisations of the 2-yr A+E data",
           "templates": bank.n, "realisations": R}
    rg = batching.RealisationGraph(grid, xs, psd, mu, kp, bank, seg, store="f32", layout="layer_ci", precision="f32",
                                   order=order, **kw)
    out["one_per_launch_ms"] = round(1e3 * timed(rg), 2)
    log(f"batching profile: one launch per realisation {out['one_per_launch_ms']:.1f} ms per replay")
    for st in ("f32", "i16"):
        rgi = batching.RealisationGraph(grid, xs, psd, mu, kp, bank, seg, store=st, layout="layer_ci",
                                        precision="f32", order=order, interleave=2, **kw)
        ms = 1e3 * timed(rgi)
        d = max(float(torch.max(torch.abs(rgi.results[r].stat - rg.results[r].stat)
                                / torch.clamp(rg.results[r].stat.abs(), min=1.0))) for r in range(R))
        out[f"pairs_{st}_ms"] = round(ms, 2)
        out[f"pairs_{st}_max_rel_vs_fp32"] = d
        log(f"batching profile: {st} pairs {ms:.1f} ms per replay ({out['one_per_launch_ms'] / ms:.3f}x); max rel {d:.1e}")
        del rgi
    print(json.dumps(out), flush=True)


def vjp_profile_run(args, tfsc, ti, g, grid, dev):
    """Statistic and both VJP arithmetics on 65,536 templates of the 2-yr workload, timed with events on the
    launch stream (the run rocprofv3 profiles for the VJP kernel)."""
    import torch
    x = (ti.noise(g) * ti.sample_keep_mask(g)[None, :]).astype(np.float32)
    psd, mu, keep = ti.psd_on_bins(g), ti.tranche_psd_scale(g), ti.tranche_keep(g)
    pix = tfsc.transform(grid, torch.from_numpy(x).to(dev), torch.from_numpy(psd).to(dev),
                         torch.from_numpy(mu).to(dev), torch.from_numpy(keep).to(dev), dtype="f32", layout="layer_ci")
    bank = tfsc.BankTensors.from_host(ti.full_bank(65536 - 20), dev)
    seg = tfsc.segment_layout(grid, bank)
    fw = tfsc.bank_statistic(grid, pix, bank, seg, precision="f32", want_zn=True)
    ones = torch.ones(bank.n, dtype=torch.float64, device=dev)
    g64 = tfsc.statistic_vjp(grid, pix, bank, seg, fw.seg_zn, g_stat=ones, precision="f64")
    g32 = tfsc.statistic_vjp(grid, pix, bank, seg, fw.seg_zn, g_stat=ones, precision="f32")
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    t = {"statistic": [], "vjp_f64": [], "vjp_f32": []}
    for i in range(args.steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(st)
        tfsc.bank_statistic(grid, pix, bank, seg, precision="f32", want_zn=True, out=fw)
        ev[1].record(st)
        tfsc.statistic_vjp(grid, pix, bank, seg, fw.seg_zn, g_stat=ones, precision="f64", out=g64)
        ev[2].record(st)
        tfsc.statistic_vjp(grid, pix, bank, seg, fw.seg_zn, g_stat=ones, precision="f32", out=g32)
        ev[3].record(st)
        torch.cuda.synchronize()
        for k, (a, b) in zip(t, ((0, 1), (1, 2), (2, 3))):
            t[k].append(ev[a].elapsed_time(ev[b]))
        log(f"vjp profile step {i + 1}/{args.steps}: statistic {t['statistic'][-1]:.2f} ms, VJP FP64 "
            f"{t['vjp_f64'][-1]:.2f} ms, FP32 {t['vjp_f32'][-1]:.2f} ms")
    med = {k: float(np.median(v)) for k, v in t.items()}
    a, b = g64.cpu().numpy(), g32.cpu().numpy()
    floor = 1e-3 * np.max(np.abs(a), axis=0, keepdims=True)
    r = np.abs(b - a) / np.maximum(np.abs(a), np.maximum(floor, 1e-300))
    print(json.dumps({"workload": "2-yr A+E, first 65,536 templates of the bench bank", "templates": bank.n,
                      "median_ms": med, "f64_over_statistic": round(med["vjp_f64"] / med["statistic"], 3),
                      "f32_over_statistic": round(med["vjp_f32"] / med["statistic"], 3),
                      "f32_vs_f64_max_rel": float(r.max()), "f32_vs_f64_median_rel": float(np.median(r))}),
          flush=True)


def accuracy(stat, flags, ref):
    """|Upsilon - Upsilon_oracle| / max(Upsilon_oracle, 1) over a sample, and whether the flags agree."""
    r = np.abs(stat - ref.stat) / np.maximum(np.abs(ref.stat), 1.0)
    return {"templates": int(r.size), "max_rel": float(r.max()), "p99_rel": float(np.quantile(r, 0.99)),
            "median_rel": float(np.median(r)), "flags_equal": bool(np.array_equal(flags, ref.flags))}


def precision_run(args, tfsc, grid, x_d, psd_d, mu_d, keep_d, bank, seg, order, kw, res_c, sub_idx, ref, value_f32):
    """FP16, BF16 and int16 fixed-point stores (per-layer FP32 scale, FP32 accumulation, FP64 track): templates/s
    of the same step and the error of every template of the 10k subsample against the FP64 oracle."""
    import torch
    out = {}
    n = bank.n
    for dt in ("f16", "bf16", "i16"):
        pix = tfsc.transform(grid, x_d, psd_d, mu_d, keep_d, dtype=dt, layout=args.chosen_layout)

        def step():
            tfsc.transform(grid, x_d, psd_d, mu_d, keep_d, dtype=dt, layout=args.chosen_layout, out=pix)
            tfsc.segment_layout(grid, bank, out=seg, read_total=False)
            o = None if order is None else tfsc.processing_order(grid, bank, out=order)
            return tfsc.bank_statistic(grid, pix, bank, seg, precision="f32", schedule="wave", out=res_c, order=o,
                                       **kw)

        step()
        torch.cuda.synchronize()
        reps = max(2, args.steps // 2)
        t0 = time.perf_counter()
        for _ in range(reps):
            step()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        st = torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(st)
        tfsc.bank_statistic(grid, pix, bank, seg, precision="f32", schedule="wave", out=res_c, order=order, **kw)
        ev[1].record(st)
        torch.cuda.synchronize()
        s = res_c.stat.cpu().numpy()
        acc = accuracy(s[sub_idx], res_c.flags.cpu().numpy()[sub_idx], ref)
        out[dt] = {"templates_per_s": round(n / (ms / 1e3), 1), "ms_per_step": round(ms, 3),
                   "kernel_ms": round(ev[0].elapsed_time(ev[1]), 3), "over_f32": round(n / (ms / 1e3) / value_f32, 4),
                   "store": f"{dt} {args.chosen_layout} + per-layer f32 scale" + (" (step = layer max / 32767)"
                                                                                   if dt == "i16" else ""),
                   "arith": "f32 (track f64)",
                   "vs_oracle": acc}
        log(f"precision {dt}: {ms:.2f} ms/step, {n / (ms / 1e3) / 1e6:.3f} M templates/s; vs oracle {acc}")
        del pix
    return out


def aet_run(args, tfsc, ti, g, psd_d, mu_d, keep_d, bank, bank_h, seg, order, kw, pix_cols, value_ae, k_ms_ae):
    """The chosen form on three channels (A, E, T) of the same 2-yr grid: transform + layout + order + statistic
    per step, the statistic kernel timed alone, and sampled templates checked against the oracle."""
    import torch
    from oracle import o2
    from oracle import track as otrk
    from oracle import transform as otf
    dev = psd_d.device
    n = bank.n
    g3 = ti.GridSpec("full-aet", g.cfg_id, 3, g.dt, g.tranche_len, g.n_tranches, g.modulated, g.gapped)
    grid3 = tfsc.GridSpec(3, g.tranche_len, g.n_tranches, g.dt, 0.1)
    x3 = (ti.noise(g3) * ti.sample_keep_mask(g3)[None, :]).astype(np.float32)
    x3_d = torch.from_numpy(x3).to(dev)
    layout = args.chosen_layout
    pix = tfsc.transform(grid3, x3_d, psd_d, mu_d, keep_d, dtype="f32", layout=layout)
    res = tfsc.StatResult(torch.empty(n, dtype=torch.float64, device=dev),
                          torch.empty(seg.total, dtype=torch.float64, device=dev),
                          torch.empty(n, dtype=torch.int32, device=dev))

    def step():
        tfsc.transform(grid3, x3_d, psd_d, mu_d, keep_d, dtype="f32", layout=layout, out=pix)
        tfsc.segment_layout(grid3, bank, out=seg, read_total=False)
        o = None if order is None else tfsc.processing_order(grid3, bank, out=order)
        tfsc.bank_statistic(grid3, pix, bank, seg, precision="f32", schedule="wave", out=res, order=o, **kw)

    step()
    torch.cuda.synchronize()
    log("aet: warmup done")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_step = 1e3 * (time.perf_counter() - t0) / args.steps
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ks = []
    for _ in range(3):
        ev[0].record(st)
        tfsc.bank_statistic(grid3, pix, bank, seg, precision="f32", schedule="wave", out=res, order=order, **kw)
        ev[1].record(st)
        torch.cuda.synchronize()
        ks.append(ev[0].elapsed_time(ev[1]))
    k_ms = float(np.median(ks))
    alg_bytes = pix_cols * NF * 3 * 8 + n * 56 + 8 * (seg.total + n)
    value = n / (ms_step / 1e3)
    log(f"aet: {ms_step:.2f} ms/step, {value / 1e6:.3f} M templates/s; statistic kernel {k_ms:.2f} ms "
        f"({k_ms / k_ms_ae:.3f}x the A+E kernel's)")
    s = res.stat.cpu().numpy()
    rng = np.random.default_rng(19)
    idx = sorted(set(np.argsort(-np.nan_to_num(s, nan=-1.0))[:3].tolist()) | set(rng.choice(n, 5, replace=False).tolist()))
    pix_o, u, wm = otf.transform(x3.astype(np.float64), g3, ti.psd_on_bins(g3), ti.tranche_psd_scale(g3),
                                 ti.tranche_keep(g3), 0.1, "rfft")
    sub = bank_h.subset(idx)
    ref = o2.statistic(pix_o, u, wm, sub, g3, layout=otrk.Layout(sub, g3))
    r = np.abs(s[idx] - ref.stat) / np.maximum(np.abs(ref.stat), 1.0)
    log(f"aet: sampled parity on {len(idx)} templates, max rel {r.max():.2e}")
    return {"workload": "same 2-yr grid and bank, three channels A, E, T (noise of the A/E model in each)",
            "templates_per_s": round(value, 1), "ms_per_step": round(ms_step, 3), "kernel_ms": round(k_ms, 3),
            "kernel_over_ae": round(k_ms / k_ms_ae, 4), "value_over_ae": round(value / value_ae, 4),
            "alg_bytes_per_launch": alg_bytes, "alg_gbs": round(alg_bytes / (k_ms / 1e3) / 1e9, 1),
            "store": f"f32 {layout}, 3 channels",
            "sampled_parity": {"templates": len(idx), "max_rel_vs_oracle": float(r.max())}}


def psd_tf_run(args, tfsc, ti, grid, g, x, x_d, keep_d, bank, bank_h, seg, order, kw, pix_cols, value_sep, k_ms_sep):
    """The chosen form with a locally stationary PSD that is not separable in time and frequency (a spectral
    tilt drifting over the orbit): transform_tf + layout + order + statistic per step, the statistic kernel
    timed alone, and sampled templates checked against the oracle's per-pixel weights."""
    import torch
    from oracle import o2
    from oracle import track as otrk
    from oracle import transform as otf
    dev = x_d.device
    n = bank.n
    S = ti.tranche_psd_tf(g)
    S_d = torch.from_numpy(S).to(dev)
    layout = args.chosen_layout
    pix = tfsc.transform_tf(grid, x_d, S_d, keep_d, dtype="f32", layout=layout)
    res = tfsc.StatResult(torch.empty(n, dtype=torch.float64, device=dev),
                          torch.empty(seg.total, dtype=torch.float64, device=dev),
                          torch.empty(n, dtype=torch.int32, device=dev))

    def step():
        tfsc.transform_tf(grid, x_d, S_d, keep_d, dtype="f32", layout=layout, out=pix)
        tfsc.segment_layout(grid, bank, out=seg, read_total=False)
        o = None if order is None else tfsc.processing_order(grid, bank, out=order)
        tfsc.bank_statistic(grid, pix, bank, seg, precision="f32", schedule="wave", out=res, order=o, **kw)

    step()
    torch.cuda.synchronize()
    log("psd_tf: warmup done")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_step = 1e3 * (time.perf_counter() - t0) / args.steps
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ks = []
    for _ in range(3):
        ev[0].record(st)
        tfsc.bank_statistic(grid, pix, bank, seg, precision="f32", schedule="wave", out=res, order=order, **kw)
        ev[1].record(st)
        torch.cuda.synchronize()
        ks.append(ev[0].elapsed_time(ev[1]))
    k_ms = float(np.median(ks))
    alg_bytes = pix_cols * NF * (g.n_channels * 8 + 4) + n * 56 + 8 * (seg.total + n)
    value = n / (ms_step / 1e3)
    log(f"psd_tf: {ms_step:.2f} ms/step, {value / 1e6:.3f} M templates/s; statistic kernel {k_ms:.2f} ms "
        f"({k_ms / k_ms_sep:.3f}x the separable PSD's)")
    # sampled parity: the three largest statistics and five seeded others, FP64 oracle with per-pixel weights
    s = res.stat.cpu().numpy()
    rng = np.random.default_rng(17)
    idx = sorted(set(np.argsort(-np.nan_to_num(s, nan=-1.0))[:3].tolist()) | set(rng.choice(n, 5, replace=False).tolist()))
    pix_o, wt = otf.transform_tf(x.astype(np.float64), g, S, ti.tranche_keep(g), 0.1, "rfft")
    sub = bank_h.subset(idx)
    ref = o2.statistic(pix_o, None, None, sub, g, layout=otrk.Layout(sub, g), weight_tf=wt)
    r = np.abs(s[idx] - ref.stat) / np.maximum(np.abs(ref.stat), 1.0)
    log(f"psd_tf: sampled parity on {len(idx)} templates, max rel {r.max():.2e}")
    return {"workload": "same data and bank; PSD S_m(f_k) = mu_m S0(f_k) (f_k / 10 mHz)^(0.3 sin(2 pi t_m / 0.5 yr + 0.7))",
            "templates_per_s": round(value, 1), "ms_per_step": round(ms_step, 3), "kernel_ms": round(k_ms, 3),
            "kernel_over_separable": round(k_ms / k_ms_sep, 4), "value_over_separable": round(value / value_sep, 4),
            "alg_bytes_per_launch": alg_bytes, "alg_gbs": round(alg_bytes / (k_ms / 1e3) / 1e9, 1),
            "store": f"f32 {layout} + f32 rho[K][Nt]",
            "sampled_parity": {"templates": len(idx), "max_rel_vs_oracle": float(r.max())}}


def _noise_realisation(r):
    """Realisation r of the full-size noise with the gaps applied, FP32 (a worker process's job)."""
    import tfsc_inputs as ti
    g = ti.FULL
    return (ti.noise(g, realisation=r) * ti.sample_keep_mask(g)[None, :]).astype(np.float32)


def batching_run(args, tfsc, ti, grid, g, psd_d, mu_d, keep_d, kw, chosen_ms_per_template, noise_jobs):
    """4M wide-range templates x 16 realisations in one HIP graph; then the differentiation workload."""
    import torch
    from paper_2510_19047_amd import batching
    dev = psd_d.device
    pool, jobs, workers = noise_jobs
    R = len(jobs)
    log("batching: 4M-template bank and 16 noise realisations")
    bank_h = ti.batching_bank()
    bank = tfsc.BankTensors.from_host(bank_h, dev)
    seg = tfsc.segment_layout(grid, bank)
    order = tfsc.processing_order(grid, bank)
    xs = torch.empty((R, g.n_channels, g.n_samples), dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    for r, job in enumerate(jobs):
        xs[r] = torch.from_numpy(job.result()).to(dev)
    pool.shutdown()
    log(f"batching: {R} realisations in device memory after {time.perf_counter() - t0:.1f} s more "
        f"({workers} host processes)")
    evals = bank.n * R

    def timed_replay(rg, reps=3):
        """Median wall time of ``reps`` replays after one warm-up replay."""
        rg.replay()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            rg.replay()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    # one statistic launch per realisation (the reference for the paired path)
    rg = batching.RealisationGraph(grid, xs, psd_d, mu_d, keep_d, bank, seg, store="f32", layout=args.chosen_layout,
                                   precision="f32", order=order, **kw)
    wall = timed_replay(rg)
    log(f"batching: one replay {wall * 1e3:.1f} ms (median of 3), {evals / wall / 1e6:.3f} M template-realisations/s "
        f"(one statistic launch per realisation)")

    def max_rel_vs_single(rgx):
        worst = 0.0
        for r in range(R):
            a, b = rgx.results[r].stat, rg.results[r].stat
            ok = torch.isfinite(b)
            if bool(ok.any()):
                worst = max(worst, float((torch.abs(a - b)[ok] / torch.clamp(b.abs(), min=1.0)[ok]).max()))
        return worst

    # the batching path: realisations paired cell by cell in one FP32 store, one pass over the bank per pair, with
    # each realisation's own arithmetic (compared with its single launch below)
    rgp = batching.RealisationGraph(grid, xs, psd_d, mu_d, keep_d, bank, seg, store="f32", layout="layer_ci",
                                    precision="f32", order=order, interleave=2, **kw)
    wp = timed_replay(rgp)
    dp = max_rel_vs_single(rgp)
    del rgp
    torch.cuda.empty_cache()
    log(f"batching: one replay {wp * 1e3:.1f} ms (median of 3), {evals / wp / 1e6:.3f} M template-realisations/s "
        f"(realisations paired in FP32 stores, one pass per pair); every realisation within {dp:.1e} of its own "
        f"launch; {wall / wp:.3f}x one launch per realisation")
    rec = {"workload": "4M templates (Mc log-U[5, 100], f0 U[5, 50] mHz, 48% merging in the window) x 16 noise "
                       "realisations of the 2-yr A+E data",
           "templates": bank.n, "realisations": R, "ms_per_replay": round(wp * 1e3, 2),
           "template_realisations_per_s": round(evals / wp, 1),
           "path": "realisations paired cell by cell in FP32 channel-interleaved stores, one pass over the bank "
                   "per pair",
           "graph": "transform + interleave + statistic per pair, 8 pairs", "store": "f32 layer_ci, 2 realisations",
           "arith": "f32 (track f64)", "max_rel_vs_one_launch_per_realisation": dp,
           "one_launch_per_realisation": {"ms_per_replay": round(wall * 1e3, 2),
                                          "template_realisations_per_s": round(evals / wall, 1)},
           "paired_over_one_launch_per_realisation": round(wall / wp, 4)}
    if args.interleave:
        NR = args.interleave
        rgi = batching.RealisationGraph(grid, xs, psd_d, mu_d, keep_d, bank, seg, store=args.interleave_store,
                                        layout="layer_ci", precision="f32", order=order, interleave=NR, **kw)
        wi = timed_replay(rgi)
        d0, n_over, big, n_all = 0.0, 0, 0.0, 0
        for r in range(R):
            a, b = rgi.results[r].stat, rg.results[r].stat
            ok = torch.isfinite(b)
            e = torch.abs(a - b)[ok] / torch.clamp(b.abs(), min=1.0)[ok]
            d0 = max(d0, float(e.max()))
            n_over += int((e > 1e-4).sum())
            n_all += int(e.numel())
            loud = b[ok] >= 10.0
            if bool(loud.any()):
                big = max(big, float(e[loud].max()))
        log(f"batching: one replay {wi * 1e3:.1f} ms (median of 3), {evals / wi / 1e6:.3f} M template-realisations/s "
            f"({NR} realisations interleaved per {args.interleave_store} store and pass); every realisation within "
            f"{d0:.1e} of its own FP32 launch")
        log(f"batching: against the FP32 launches, {n_over} of {n_all} template-realisations deviate by more than "
            f"1e-4 of max(Upsilon, 1); largest deviation where Upsilon >= 10: {big:.1e}")
        rec["interleaved"] = {"realisations_per_pass": NR, "store": args.interleave_store,
                              "ms_per_replay": round(wi * 1e3, 2),
                              "vs_fp32_launches": {"max_rel": d0, "n_above_1e-4": n_over, "n": n_all,
                                                   "max_rel_upsilon_ge_10": big},
                              "template_realisations_per_s": round(evals / wi, 1),
                              "over_one_per_launch": round(wall / wi, 4), "max_rel_diff_vs_one_per_launch": d0}
        del rgi
        torch.cuda.empty_cache()
    if args.eight_per_pass:
        # the several-realisation alternative: eight realisations per pass over the bank
        rgm = batching.RealisationGraph(grid, xs, psd_d, mu_d, keep_d, bank, seg, store="f32",
                                        layout=args.chosen_layout, precision="f32", order=order, multi=True, group=8,
                                        **kw)
        wm = timed_replay(rgm, reps=1)
        d0 = float(torch.max(torch.abs(rgm.results[0].stat - rg.results[0].stat)
                             / torch.clamp(rg.results[0].stat.abs(), min=1.0)))
        log(f"batching: one replay {wm * 1e3:.1f} ms, {evals / wm / 1e6:.3f} M template-realisations/s "
            f"(eight realisations per pass over the bank); realisation 0 agrees to {d0:.1e}")
        rec["eight_per_pass"] = {"ms_per_replay": round(wm * 1e3, 2),
                                 "template_realisations_per_s": round(evals / wm, 1),
                                 "max_rel_diff_vs_one_per_launch": d0}
        del rgm
        torch.cuda.empty_cache()
    if args.background:
        from paper_2510_19047_amd import background as bg
        n_m, n_f = 8, 8
        tiles = bg.tile_ids(bank_h.mc, bank_h.f0, np.geomspace(5.0, 100.0, n_m + 1), np.linspace(0.005, 0.050, n_f + 1))
        B = bg.Background(tiles, n_m * n_f, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in range(R):
            B.add(rg.results[r].stat)
        wall = time.perf_counter() - t0
        pl, gb = B.fits()
        mx = B.maxima
        log(f"background: per-tile maxima of {R} realisations x {n_m * n_f} tiles in {wall * 1e3:.1f} ms; "
            f"Gumbel mu {gb.mu:.2f} beta {gb.beta:.3f}; power law delta {pl.delta:.2f} above {pl.u:.2f}")
        rec["background"] = {"realisations": R, "tiles": n_m * n_f, "tile_grid": "8 log-Mc x 8 f0",
                             "ms_tile_max_all_realisations": round(wall * 1e3, 3),
                             "max_median": round(float(np.median(mx)), 3), "max_max": round(float(mx.max()), 3),
                             "gumbel": {"mu": round(gb.mu, 4), "beta": round(gb.beta, 4)},
                             "power_law": {"delta": round(pl.delta, 4), "u": round(pl.u, 4), "q": pl.q},
                             "fap_at_max": {"gumbel": float(bg.fap_gumbel(mx.max(), gb)),
                                            "power_law": float(bg.fap_power_law(mx.max(), pl))}}
    if args.ladder:
        from paper_2510_19047_amd import search
        stat0 = rg.results[0].stat
        top = torch.topk(torch.nan_to_num(stat0, nan=-1.0), 65536).indices
        sub = tfsc.BankTensors(*(getattr(bank, k)[top].contiguous() for k in tfsc.BankTensors.FIELDS))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lad = search.segment_ladder(grid, rg.stores[0], sub, steps=20, lr_scale=0.5, precision="f32")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        u1 = lad.upsilon1.cpu().numpy()
        stages = [{"nseg": ns, "start_median": round(float(a.median().item()), 3),
                   "best_median": round(float(b.median().item()), 3)} for ns, a, b in zip(lad.nseg, lad.start, lad.best)]
        log(f"ladder: N_seg {'->'.join(str(v) for v in lad.nseg)}, 20 steps each, on 65536 templates in {wall:.2f} s; "
            f"Upsilon_1 median {np.median(u1):.2f}")
        rec["ladder"] = {"templates": 65536, "steps_per_stage": 20, "wall_s": round(wall, 3), "stages": stages,
                         "upsilon1_median": round(float(np.median(u1)), 3), "upsilon1_p90": round(float(np.quantile(u1, 0.9)), 3)}
    if not args.no_follow_up:
        stat0 = rg.results[0].stat
        top = torch.topk(torch.nan_to_num(stat0, nan=-1.0), 65536).indices
        sub = tfsc.BankTensors(*(getattr(bank, k)[top].contiguous() for k in tfsc.BankTensors.FIELDS))
        # the candidates in processing order (f0 bin, then ln Mc), as the follow-up runs them
        perm = tfsc.processing_order(grid, sub).long()
        sub = tfsc.BankTensors(*(getattr(sub, k)[perm].contiguous() for k in tfsc.BankTensors.FIELDS))
        store0 = rg.stores[0]
        # one forward and one VJP on the candidates, each timed with events on the launch stream
        sseg = tfsc.segment_layout(grid, sub)
        st = torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        fw = tfsc.bank_statistic(grid, store0, sub, sseg, precision="f32", want_zn=True)
        ones = torch.ones(sub.n, dtype=torch.float64, device=dev)
        gp = tfsc.statistic_vjp(grid, store0, sub, sseg, fw.seg_zn, g_stat=ones, precision="f64")
        gp32 = tfsc.statistic_vjp(grid, store0, sub, sseg, fw.seg_zn, g_stat=ones, precision="f32")
        torch.cuda.synchronize()
        ev[0].record(st)
        tfsc.bank_statistic(grid, store0, sub, sseg, precision="f32", want_zn=True, out=fw)
        ev[1].record(st)
        tfsc.statistic_vjp(grid, store0, sub, sseg, fw.seg_zn, g_stat=ones, precision="f64", out=gp)
        ev[2].record(st)
        tfsc.statistic_vjp(grid, store0, sub, sseg, fw.seg_zn, g_stat=ones, precision="f32", out=gp32)
        ev[3].record(st)
        torch.cuda.synchronize()
        f_ms, v_ms, v32_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3])
        # the FP32 VJP against the FP64 one, per component relative to max(|g|, 1e-3 x the column's largest |g|)
        g64 = gp.cpu().numpy()
        floor = 1e-3 * np.max(np.abs(g64), axis=0, keepdims=True)
        rel32 = np.abs(gp32.cpu().numpy() - g64) / np.maximum(np.abs(g64), np.maximum(floor, 1e-300))
        log(f"follow-up candidates: statistic {f_ms:.1f} ms, VJP {v_ms:.1f} ms FP64 and {v32_ms:.1f} ms FP32 for "
            f"65536 templates; FP32 vs FP64 gradient max rel {rel32.max():.2e}, median {np.median(rel32):.2e}")
        rec["vjp"] = {"templates": 65536, "statistic_ms": round(f_ms, 3),
                      "f64": {"vjp_ms": round(v_ms, 3), "vjp_over_statistic": round(v_ms / f_ms, 3),
                              "vjp_over_chosen_per_template": round(v_ms / 65536 / chosen_ms_per_template, 3),
                              "vjp_templates_per_s": round(65536 / v_ms * 1e3, 1)},
                      "f32": {"vjp_ms": round(v32_ms, 3), "vjp_over_statistic": round(v32_ms / f_ms, 3),
                              "vjp_over_chosen_per_template": round(v32_ms / 65536 / chosen_ms_per_template, 3),
                              "vjp_templates_per_s": round(65536 / v32_ms * 1e3, 1),
                              "vs_f64": {"max_rel": float(rel32.max()), "median_rel": float(np.median(rel32))}}}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        first, best, _ = tfsc.follow_up(grid, store0, sub, steps=50, lr_scale=0.5, precision="f32",
                                        vjp_precision="f32")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gain = (best - first).cpu().numpy()
        log(f"follow-up: 50 Adam steps on 65536 templates in {wall:.2f} s; gain median {np.median(gain):.2f}, "
            f"p90 {np.quantile(gain, 0.9):.2f}")
        rec["follow_up"] = {"workload": "top 65,536 templates of realisation 0 of the batching workload",
                            "templates": 65536, "steps": 50, "wall_s": round(wall, 3), "statistic": "f32",
                            "vjp": "f32",
                            "gain_median": round(float(np.median(gain)), 3),
                            "gain_p90": round(float(np.quantile(gain, 0.9)), 3),
                            "start_median": round(float(first.median().item()), 3)}
    return rec


PROFILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "k_stat_wave_counters.txt")
STAT_SOURCES = ("tfsc_stat.hip", "tfsc_stat_common.hpp", "tfsc_device.hpp", "tfsc_kernels.hpp")
SIMDS = 1024                  # 256 CUs x 4 SIMDs
NOMINAL_CLOCK_HZ = 2.4e9
CYCLES_PER_VALU = 4           # a wave64 instruction on a 16-lane SIMD


def stat_source_sha256():
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in STAT_SOURCES:
        with open(os.path.join(root, "paper_2510_19047_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_profile(n, store, layout, order):
    """Per-launch hardware counters of the chosen k_stat_wave launch from the committed rocprofv3 runs
    (written by ``bench.py --summarize-counters``): calibrated bytes beyond L2, VALU instructions, the shader
    clock (GRBM_GUI_ACTIVE over the dispatch time) and the FP32/FP64 operation counts.

    Only valid while the kernel source, the bank, the store, its layout and the processing order are the ones
    that were profiled; otherwise None.
    """
    if not os.path.exists(PROFILE):
        return None
    rec = {}
    with open(PROFILE) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#") and ":" in line:
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    same = (rec.get("source_sha256") == stat_source_sha256() and rec.get("n_templates") == str(n)
            and rec.get("pixel_store") == store and rec.get("pixel_layout") == layout and rec.get("order") == order)
    if not same:
        return None
    out = {}
    for k, v in rec.items():
        try:
            out[k] = float(v)
        except ValueError:
            out[k] = v
    return out


def alu_roofline(prof, k_s):
    """The binding roof of the chosen kernel: vector-ALU issue.

    achieved = VALU wave instructions per launch outside the transcendental pipe (counters of the same source
    and workload) / the launch time measured here; peak = the chip's issue rate at its rated 2.4 GHz clock,
    1,024 SIMDs x 2.4e9 / 4 cycles per wave64 instruction = 614.4 G instructions/s.  Under sustained load the
    shader clock runs below 2.4 GHz; the clock of the counter run (GRBM_GUI_ACTIVE, summed over the eight XCDs,
    per dispatch time) and the fraction at that clock are reported beside it.  Counting every VALU instruction
    at 4 cycles exceeds the cycles the launch had (valu_all_over_profile_clock_peak), so the transcendental
    instructions (rcp, rsq, sqrt, sin, cos, exp, log) overlap the others and are left out of the issue count.
    The FP32/FP64 operation rate is reported against the non-packed vector peak (64 FMA lanes per CU and cycle
    for FP32 and FP64 alike: 78.6 TFLOP/s at 2.4 GHz)."""
    peak = SIMDS * NOMINAL_CLOCK_HZ / CYCLES_PER_VALU
    rec = {"bound": "alu", "unit": "G VALU instr/s", "achieved": None, "peak": round(peak / 1e9, 2), "frac": None}
    if prof is None or "valu_insts" not in prof:
        rec["note"] = "no counter profile of this kernel source and workload; run the rocprofv3 passes"
        return rec
    clock = prof.get("clock_hz", NOMINAL_CLOCK_HZ)
    peak_clk = SIMDS * clock / CYCLES_PER_VALU
    issue = prof.get("valu_nontrans_insts", prof["valu_insts"])
    ach = issue / k_s
    rec.update({"achieved": round(ach / 1e9, 2), "frac": round(ach / peak, 4),
                "peak_note": "1,024 SIMDs x 2.4 GHz rated clock / 4 cycles per wave64 instruction",
                "profile_clock_ghz": round(clock / 1e9, 4), "peak_at_profile_clock": round(peak_clk / 1e9, 2),
                "frac_at_profile_clock": round(ach / peak_clk, 4),
                "valu_insts_per_launch": prof["valu_insts"], "valu_issue_insts_per_launch": issue,
                "valu_all_over_profile_clock_peak": round(prof["valu_insts"] / k_s / peak_clk, 4),
                "issue_note": "issue count excludes the transcendental VALU instructions, which overlap the others"})
    if prof.get("dispatch_ns_counter_run"):
        # the counter run's own issue fraction: its instructions, its dispatch time and its clock
        rec["issue_in_profile_run"] = round(issue / (prof["dispatch_ns_counter_run"] * 1e-9) / peak_clk, 4)
        rec["profile_note"] = ("frac_at_profile_clock divides this run's rate by the counter run's clock; "
                               "issue_in_profile_run is the counter run's own fraction (above 1: some counted "
                               "instructions take fewer than 4 cycles)")
    if "flops" in prof:
        tf = prof["flops"] / k_s / 1e12
        peak_tf = SIMDS * 16 * 2 * NOMINAL_CLOCK_HZ / 1e12
        rec["flops"] = {"per_launch": prof["flops"], "tflops": round(tf, 3), "peak_tflops": round(peak_tf, 2),
                        "frac": round(tf / peak_tf, 4),
                        "note": "64 x (ADD + MUL + 2 FMA + TRANS) over the FP32 and FP64 VALU instructions, "
                                "against the non-packed vector peak at 2.4 GHz"}
    return rec


def summarize_counters(dirs, n, store, layout, order, shape, fetch_factor, write_factor):
    """Write profiles/k_stat_wave_counters.txt from rocprofv3 --pmc CSV outputs (one directory per pass):
    the median per dispatch of each counter over the chosen k_stat_wave launches after the first."""
    import csv
    import glob
    vals = {}
    durs = []
    copy = {}
    for d in dirs:
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(path) as fh:
                rows = list(csv.DictReader(fh))
            by_disp = {}
            for row in rows:
                name = row.get("Kernel_Name", "")
                if "copyBuffer" in name and row["Counter_Name"] in ("FETCH_SIZE", "WRITE_SIZE"):
                    # the 256 MiB device copy of --copy-calibration (the largest copy dispatch): bytes per KiB
                    k = row["Counter_Name"]
                    copy[k] = max(copy.get(k, 0.0), float(row["Counter_Value"]))
                if "k_stat_wave<2, float, float, 2, false>" not in name:
                    continue
                by_disp.setdefault(int(row["Dispatch_Id"]), []).append(row)
            for disp in sorted(by_disp)[1:]:
                for row in by_disp[disp]:
                    vals.setdefault(row["Counter_Name"], []).append(float(row["Counter_Value"]))
                r0 = by_disp[disp][0]
                if "Start_Timestamp" in r0 and "End_Timestamp" in r0:
                    durs.append(float(r0["End_Timestamp"]) - float(r0["Start_Timestamp"]))
    med = {k: float(np.median(v)) for k, v in vals.items()}
    lines = ["# Read by bench.py: per-launch counters of the chosen k_stat_wave launch (median over the dispatches",
             "# after the first), valid only for this kernel source and workload; written by",
             "# python bench.py --summarize-counters <rocprofv3 --pmc output directories>",
             "kernel: k_stat_wave<2, float, float, 2, false>",
             f"source_sha256: {stat_source_sha256()}", f"n_templates: {n}", f"pixel_store: {store}",
             f"pixel_layout: {layout}", f"order: {order}", f"launch_shape: {shape}"]
    for k in sorted(med):
        lines.append(f"{k}: {med[k]:.6e}")
    if durs:
        dur = float(np.median(durs))
        lines.append(f"dispatch_ns_counter_run: {dur:.6e}")
        if "GRBM_GUI_ACTIVE" in med:
            clk = med["GRBM_GUI_ACTIVE"] / (dur * 1e-9)
            # GRBM_GUI_ACTIVE is summed over the eight XCDs when the profiler reports it per device
            if clk > 4e9:
                clk /= 8.0
            lines.append(f"clock_hz: {clk:.6e}")
    if "SQ_INSTS_VALU" in med:
        lines.append(f"valu_insts: {med['SQ_INSTS_VALU']:.6e}")
        if "SQ_INSTS_VALU_TRANS_F32" in med and "SQ_INSTS_VALU_TRANS_F64" in med:
            nt = med["SQ_INSTS_VALU"] - med["SQ_INSTS_VALU_TRANS_F32"] - med["SQ_INSTS_VALU_TRANS_F64"]
            lines.append(f"valu_nontrans_insts: {nt:.6e}")
    if copy.get("FETCH_SIZE", 0) > 0 and copy.get("WRITE_SIZE", 0) > 0:
        fetch_factor = 268435456.0 / (copy["FETCH_SIZE"] * 1024.0)
        write_factor = 268435456.0 / (copy["WRITE_SIZE"] * 1024.0)
        lines += [f"copy_calibration_fetch_kib: {copy['FETCH_SIZE']:.6e}",
                  f"copy_calibration_write_kib: {copy['WRITE_SIZE']:.6e}"]
    if "FETCH_SIZE" in med and "WRITE_SIZE" in med:
        tb = med["FETCH_SIZE"] * 1024 * fetch_factor + med["WRITE_SIZE"] * 1024 * write_factor
        lines += [f"fetch_factor: {fetch_factor:.3f}", f"write_factor: {write_factor:.3f}", f"traffic_bytes: {tb:.6e}"]
    ops = [k for k in med if k.startswith("SQ_INSTS_VALU_") and (k.endswith("_F32") or k.endswith("_F64"))]
    if ops:
        fl = 0.0
        for k in ops:
            w = 2.0 if "_FMA_" in k else 1.0
            fl += 64.0 * w * med[k]
        lines.append(f"flops: {fl:.6e}")
    with open(PROFILE, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, pix, u, wm, bank_h, seconds):
    """The FP64 oracle on the host: the plain-C O2 statistic on all cores and on one core (the paper's own CPU
    comparison is one core), on bounded samples of the same bank, and O1 (the definition: time-domain
    synthesis and direct DFT) on two templates over a 256-tranche span, extrapolated by samples."""
    import torch
    from oracle import cpu as ocpu
    import tfsc_inputs as ti
    threads = len(os.sched_getaffinity(0))

    def timed(n_s, nthreads, cfg_id):
        idx = ti.subsample_indices(len(bank_h), n_s, cfg_id=cfg_id)
        t0 = time.perf_counter()
        ocpu.statistic(pix, u, wm, bank_h.subset(idx), g, threads=nthreads)
        return time.perf_counter() - t0

    t_cal = timed(256, threads, 12)
    n_all = int(min(len(bank_h), max(256, 256 * seconds / max(t_cal, 1e-3))))
    log(f"cpu baseline: {n_all} templates on {threads} threads")
    t_all = timed(n_all, threads, 12)
    n_one = int(max(16, 256 * (seconds / 3) / max(t_cal * threads, 1e-3)))
    log(f"cpu baseline: {n_one} templates on 1 thread")
    t_one = timed(n_one, 1, 14)
    # O1 on a 256-tranche span of the same grid (its cost grows with the samples synthesised)
    from oracle import o1
    from oracle import track as otrk
    span = 256
    gs = ti.GridSpec("full-span", g.cfg_id, g.n_channels, g.dt, g.tranche_len, span, g.modulated, g.gapped)
    idx = ti.subsample_indices(len(bank_h), 2, cfg_id=15)
    sub = bank_h.subset(idx)
    lay = otrk.Layout(sub, gs)
    t0 = time.perf_counter()
    for i in range(len(idx)):
        Y = o1.template_pixels(sub, i, gs, u, wm[:span])
        o1.statistic_from_pixels(pix[:, :, :span], Y, o1.bin_mask(gs, lay, i), int(lay.nseg[i]), span)
    t_o1 = (time.perf_counter() - t0) / len(idx)
    per_tpl_o1 = t_o1 * g.n_tranches / span
    return {"value": round(n_all / t_all, 1), "unit": "templates/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{n_all} templates drawn from the same bank (seeded permutation), plain-C FP64 O2 oracle with "
                      f"OpenMP over templates, statistic only (pixels from the oracle's own transform), {t_all:.1f} s",
            "one_core": {"value": round(n_one / t_one, 2), "unit": "templates/s", "cores": 1,
                         "us_per_template": round(1e6 * t_one / n_one, 1),
                         "sample": f"{n_one} other templates of the same bank on one thread, {t_one:.1f} s"},
            "o1_definition": {"s_per_template": round(per_tpl_o1, 2), "threads": torch.get_num_threads(),
                              "sample": f"2 templates, time-domain synthesis of A and E plus direct DFT over the "
                                        f"first {span} of {g.n_tranches} tranches ({t_o1:.2f} s each), scaled by "
                                        f"{g.n_tranches / span:.0f} to the 2-yr span"},
            "paper_context": "paper: 1-10 us per statistic evaluation on one A100 (about 1e5-1e6 per s), 2680 tiles x "
                             "1e8 evaluations in 11 days on 4 A100 (about 7e4 per s per GPU end to end), a search "
                             "within a day on about 40 GPUs; its CPU comparison is one core of a 2.4 GHz Xeon "
                             "Platinum"}


if __name__ == "__main__":
    main()
