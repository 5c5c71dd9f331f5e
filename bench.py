#!/usr/bin/env python3
"""Throughput of Bluebild standard synthesis on one MI355X.

Workload (default): the LOFAR-like single-channel configuration -- 512
stations over 50 km, 100 epochs over 6 h of Earth rotation, 1024 x 1024
pixels over 10 degrees, all 512 eigenpairs in 8 positive + 1 negative
k-means levels, complex64 contraction with FP64 phase arguments.  Inputs are
synthetic (seeded sims), built on the host; the eigenpairs come from the
library's own FP64 GPU pre-step before the timed region.

A step is one pass of the synthesis hot path over the whole job (staging of
every epoch plus one batched synthesis launch over all 100 epochs), with all
inputs resident in HBM.  Prints one JSON line on stdout; progress goes to
stderr.

    python bench.py [--steps K] [--warmup W] [--precision fp32|bf16x3]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

FP32_PEAK_TFLOPS = 157.3      # MI355X dense FP32 matrix
BF16_PEAK_TFLOPS = 2516.6     # MI355X dense BF16 matrix

# HBM-side bytes per launch of the synthesis kernel on this workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) scaled by the same counters of a
# 256 MiB device copy; valid only for the kernel source they were taken on
# (sha256 of csrc/synth_kernels.hip), reported as null otherwise.
MEASURED_TRAFFIC = {
    "fp32_3m": {"bytes": 8.7692e+10,
                "kernel_source_sha256": "32ff6b0bc86e4020d0512878d3b20f9d513c6fd20f4c841d2f061c3925f6f748"},
}


def measured_traffic(mode):
    import hashlib
    rec = MEASURED_TRAFFIC.get(mode)
    if rec is None:
        return None
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2310_09200_amd", "csrc",
                       "synth_kernels.hip")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["kernel_source_sha256"]:
            return None
    return rec["bytes"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def build_inputs(args, torch, dev):
    from paper_2310_09200_amd import StandardSynthesis, Context
    from sims import configs
    from sims.levels import kmeans1d_intervals

    w = configs.c2(n_steps=args.epochs, n_side=args.n_side)
    ctx = Context(0)
    t0 = time.time()
    insts = [w.instance(i) for i in range(args.epochs)]
    log(f"simulated {len(insts)} visibility matrices in {time.time() - t0:.1f}s")
    probe = StandardSynthesis(ctx, w.pix[:1], 1, 1, 512, 512)
    _, lam0, _, _ = probe.prestep(insts[0].x, insts[0].wl, insts[0].V, 512, np.array([[-np.inf, np.inf]]))
    intervals = kmeans1d_intervals(lam0.cpu().numpy(), 8, negative_level=True)
    probe.close()
    pre = StandardSynthesis(ctx, w.pix[:1], intervals.shape[0], 1, 512, 512)
    items = []
    t0 = time.time()
    for i, inst in enumerate(insts):
        W, lam, d, lev = pre.prestep(inst.x, inst.wl, inst.V, 512, intervals)
        items.append((0, inst.x, inst.wl, W.clone(), d.clone(), lev.clone()))
    torch.cuda.synchronize()
    log(f"GPU FP64 pre-step (Gram + zhegvd) for {len(items)} epochs in {time.time() - t0:.1f}s")
    pre.close()
    return ctx, w, intervals, items, insts


def measure_phase_peak(torch, ctx, w, items, reps=4, steps=3):
    """Peak phase-generation rate of this device: the probe kernel evaluates every (antenna, pixel) phase of
    the workload's first epoch with the synthesis kernel's arithmetic and no contraction beside it.
    Returns (pairs per second, ms per probe call, pairs per call)."""
    from paper_2310_09200_amd import phase_probe
    _, x, wl = items[0][:3]
    pix = torch.as_tensor(w.pix).to(ctx.device)  # the per-call column-major copy stays on the device
    out = phase_probe(ctx, x, wl, pix, reps)  # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        phase_probe(ctx, x, wl, pix, reps, out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    pairs = float(x.shape[0]) * w.n_pix * reps
    return pairs / (ms / 1000.0), ms, pairs


def time_modes(args, torch, ctx, w, items, modes, n_levels):
    """Time every contraction mode, interleaved step by step (same thermal / power state for all).

    Returns {mode: (ms per step, synthesis kernel ms, staging ms, products per pixel)}.
    """
    from paper_2310_09200_amd import Batch, StandardSynthesis
    batch = Batch(items, ctx.device)
    handles = {m: StandardSynthesis(ctx, w.pix, n_levels, 1, 512, 512, m) for m in modes}
    for _ in range(args.warmup):
        for m in modes:
            handles[m].collect_eig_batched(batch)
    torch.cuda.synchronize()
    wall = {m: [] for m in modes}
    kern = {m: [] for m in modes}
    for _ in range(args.steps):
        for m in modes:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            handles[m].collect_eig_batched(batch)
            torch.cuda.synchronize()
            wall[m].append((time.perf_counter() - t0) * 1000.0)
            kern[m].append(handles[m].timings())
    out = {}
    for m in modes:
        handles[m].sync()
        handles[m].close()
        ms = float(np.mean(wall[m]))
        stage = float(np.mean([k[1] for k in kern[m]]))
        synth = float(np.mean([k[2] for k in kern[m]]))
        log(f"{m}: {ms:.1f} ms/step, synthesis kernel {synth:.1f} ms, staging {stage:.2f} ms")
        out[m] = (ms, synth, stage, batch.products)
    return out


def measure_c4(args, torch, ctx):
    """Batched uneven instances (a6): 64 channels x 32 epochs, L 200..512, K 16..128, 512^2 pixels, one call."""
    from paper_2310_09200_amd import Batch, StandardSynthesis
    from sims import configs
    w = configs.c4()
    items = []
    for i in range(w.n_instances()):
        inst = w.instance(i)
        items.append((inst.slot, inst.x, inst.wl, inst.W.astype(np.complex64), inst.lam.astype(np.float32),
                      inst.level_of))
    batch = Batch(items, ctx.device)
    s = StandardSynthesis(ctx, w.pix, 4, 64, 512, 128, args.precision)
    s.collect_eig_batched(batch)
    torch.cuda.synchronize()
    ms = []
    for _ in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.collect_eig_batched(batch)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1000.0)
    kern = s.timings()[2]
    s.close()
    prods = batch.products * w.n_pix
    log(f"C4 batched: {np.mean(ms):.1f} ms/call, synthesis {kern:.1f} ms, {prods / (np.mean(ms) / 1e3):.3e} products/s")
    return {"workload": "2048 uneven instances (64 channels x 32 epochs, L 200..512, K 16..128, 4 levels), "
                        "512x512 pixels, one batched call", "contraction": args.precision,
            "products": prods, "ms_per_call": float(np.mean(ms)), "synthesis_kernels_ms": kern,
            "value": prods / (np.mean(ms) / 1e3), "unit": "products/s",
            "fp32_equivalent_mfma_fraction": 8.0 * prods / (np.mean(ms) / 1e3) / (FP32_PEAK_TFLOPS * 1e12)}


def measure_c5_backward(args, torch, ctx):
    """Backward (a7): L=256, K=64, 512^2 pixels, 4 levels; forward image and gradients w.r.t. W, d, x."""
    from paper_2310_09200_amd import StandardSynthesis
    from sims import configs
    from sims.levels import kmeans1d_intervals
    w = configs.c5()
    inst = w.instance(0)
    s = StandardSynthesis(ctx, w.pix, 4, 1, 256, 64, "fp32")
    probe = StandardSynthesis(ctx, w.pix[:1], 1, 1, 256, 256)
    _, lam, _, _ = probe.prestep(inst.x, inst.wl, inst.V, 64, np.array([[-np.inf, np.inf]]))
    probe.close()
    iv = kmeans1d_intervals(lam.cpu().numpy(), 4, negative_level=False)
    W, lam, d, lev = s.prestep(inst.x, inst.wl, inst.V, 64, iv)
    gimg = torch.as_tensor(w.meta["loss_weights"](), dtype=torch.float32, device=ctx.device)
    s.eig_backward(inst.x, inst.wl, W, d, lev, gimg)
    s.collect_eig(0, inst.x, inst.wl, W, d, lev)
    torch.cuda.synchronize()
    fwd, bwd = [], []
    for _ in range(5):
        s.collect_eig(0, inst.x, inst.wl, W, d, lev)
        fwd.append(s.timings()[2])
        s.eig_backward(inst.x, inst.wl, W, d, lev, gimg)
        bwd.append(s.timings()[2])
    s.close()
    prods = 256 * 64 * w.n_pix
    f_ms, b_ms = float(np.median(fwd)), float(np.median(bwd))
    log(f"C5: forward {f_ms:.3f} ms, backward {b_ms:.3f} ms")
    return {"workload": "L=256, K=64, 512x512 pixels, 4 levels, loss weights N(0,1) per level and pixel",
            "forward_ms": f_ms, "backward_ms": b_ms, "products": prods,
            "backward_note": "E recompute (FP32 MFMA) + dd/M, dW = 2 B M^T and H = conj(W) M on FP32 MFMA (one fused "
                             "kernel at K <= 64) -> dx; about 3x the forward's complex MACs",
            "backward_fp32_mfma_fraction": 3 * 8.0 * prods / (b_ms / 1e3) / (FP32_PEAK_TFLOPS * 1e12)}


def measure_nufft(args, torch, ctx):
    """NUFFT synthesis next to standard synthesis on the paper's performance setup.

    SKA-Low-like array (C3: 512 stations, 65 km), 50 epochs over 6 h, 4 arcsec
    pixels, 8 + 1 k-means levels, every eigenpair kept; eigenpairs from the GPU
    FP64 pre-step.  Both syntheses image the same eigenpairs; the NUFFT image
    is compared with the standard one level by level.
    """
    from paper_2310_09200_amd import Batch, NufftSynthesis, StandardSynthesis
    from sims import configs, tangent_basis
    from sims.levels import kmeans1d_intervals
    side = args.nufft_side
    fov = side * 4.0 / 3600.0
    w = configs.c3(n_steps=50, n_side=side, fov_deg=fov)
    insts = [w.instance(i) for i in range(w.n_steps)]
    probe = StandardSynthesis(ctx, w.pix[:1], 1, 1, 512, 512)
    _, lam0, _, _ = probe.prestep(insts[0].x, insts[0].wl, insts[0].V, 512, np.array([[-np.inf, np.inf]]))
    probe.close()
    iv = kmeans1d_intervals(lam0.cpu().numpy(), 8, negative_level=True)
    n_levels = iv.shape[0]
    pre = StandardSynthesis(ctx, w.pix[:1], n_levels, 1, 512, 512)
    items = []
    for inst in insts:
        W, lam, d, lev = pre.prestep(inst.x, inst.wl, inst.V, 512, iv)
        items.append((0, inst.x, inst.wl, W.clone(), d.clone(), lev.clone()))
    pre.close()
    batch = Batch(items, ctx.device)
    frame = np.array(tangent_basis(w.dec0_deg))
    uvw = np.zeros(3)
    for inst in insts:
        li, mi = np.triu_indices(inst.x.shape[0], k=1)
        b = (inst.x[li] - inst.x[mi]) @ frame.T / inst.wl
        uvw = np.maximum(uvw, np.max(np.abs(b), axis=0))
    uvw = uvw * 1.001

    s = StandardSynthesis(ctx, w.pix, n_levels, 1, 512, 512, args.precision)
    plan = NufftSynthesis(ctx, w.pix, n_levels, 512, 512, args.nufft_eps, frame, uvw, transform=args.nufft_transform,
                          partitions=args.nufft_partitions)
    N, M, kw = plan.shape
    s.collect_eig_batched(batch)
    plan.collect_eig_batched(batch)
    plan.emit()
    torch.cuda.synchronize()
    s.reset()
    plan.images.zero_()
    std_ms, nu_ms, spread_ms, emit_ms = [], [], [], []
    for _ in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.collect_eig_batched(batch)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plan.collect_eig_batched(batch)
        plan.emit()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        std_ms.append((t1 - t0) * 1e3)
        nu_ms.append((t2 - t1) * 1e3)
        a, b = plan.timings()
        spread_ms.append(a)
        emit_ms.append(b)
    plan.sync()
    s.sync()
    std_img = s.images[0].double()
    nu_img = plan.images.double()
    errs = []
    for lv in range(n_levels):
        peak = float(std_img[lv].abs().max())
        if peak > 0:
            errs.append(float((nu_img[lv] - std_img[lv]).abs().max()) / peak)
    s.close()
    plan.close()
    prods = batch.products * w.n_pix
    log(f"NUFFT {side}^2 ({args.nufft_partitions}x{args.nufft_partitions} partitions): standard {np.mean(std_ms):.1f} ms, NUFFT {np.mean(nu_ms):.1f} ms "
        f"(spread {np.mean(spread_ms):.1f}, emit {np.mean(emit_ms):.1f}), grid {N} fft {M} w={kw}, "
        f"max level diff {max(errs):.2e}")
    return {"workload": f"SKA-Low-like 512 stations (65 km), 50 epochs over 6 h, {side}x{side} pixels of 4 arcsec "
                        f"({fov * 60:.1f} arcmin), 8+1 k-means levels, all 512 eigenpairs (GPU FP64 pre-step)",
            "epsilon": args.nufft_eps, "spread_grid": list(N), "fft_grid": list(M), "kernel_width": kw,
            "standard_ms": float(np.mean(std_ms)), "standard_contraction": args.precision,
            "nufft_ms": float(np.mean(nu_ms)), "nufft_spread_ms": float(np.mean(spread_ms)),
            "nufft_emit_ms": float(np.mean(emit_ms)), "speedup_nufft_over_standard": float(np.mean(std_ms) / np.mean(nu_ms)),
            "products": prods, "standard_products_per_s": prods / (np.mean(std_ms) / 1e3),
            "partitions": args.nufft_partitions,
            "transform": {"auto": "pruned, own LDS line FFTs where every axis fits, else rocFFT",
                          "rocfft": "pruned, rocFFT"}[args.nufft_transform],
            "max_level_diff_nufft_vs_standard": max(errs)}


def spot_error(args, torch, ctx, w, items, precision, n_levels, sel, ref_img):
    """Per-level max error (peak-normalised) of one epoch on the oracle's sample pixels."""
    from paper_2310_09200_amd import StandardSynthesis
    s = StandardSynthesis(ctx, w.pix, n_levels, 1, 512, 512, precision)
    _, x, wl, W, d, lev = items[0]
    s.collect_eig(0, x, wl, W, d, lev)
    s.sync()
    got = s.images[0][:, torch.as_tensor(sel, device=ctx.device)].double().cpu().numpy()
    s.close()
    errs = []
    for a, b in zip(got, ref_img):
        if np.max(np.abs(b)) > 0:
            errs.append(float(np.max(np.abs(a - b)) / np.max(np.abs(b))))
    return max(errs)


def cpu_baseline(args, w, items, n_levels):
    """The FP64 oracle (numpy/BLAS, all host threads) on a bounded sample of epoch 0."""
    import oracle as ref
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    _, x, wl, W, d, lev = items[0]
    Wn = W.cpu().numpy().astype(np.complex128)
    dn = d.cpu().numpy().astype(np.float64)
    member = ref.membership_from_level_of(lev.cpu().numpy(), n_levels)
    sel = np.arange(0, w.n_pix, args.cpu_stride)
    t0 = time.perf_counter()
    img = ref.synthesize_blas(Wn, dn, member, x, w.pix[sel], wl)
    dt = time.perf_counter() - t0
    prods = sel.size * Wn.shape[0] * Wn.shape[1]
    log(f"oracle: {sel.size} pixels x 1 epoch in {dt:.1f}s -> {prods / dt:.3e} products/s on {threads} threads")
    return {"value": prods / dt, "unit": "products/s", "cores": int(threads), "kind": "oracle",
            "sample": f"epoch 0 of the workload, every {args.cpu_stride}th pixel ({sel.size} pixels), "
                      f"L=512, K=512, FP64 numpy/BLAS, {dt:.1f} s"}, sel, img


MODES = ("fp32_3m", "fp32", "bf16x3", "bf16x3_3m")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32_3m", choices=MODES,
                    help="contraction of the headline line: fp32_3m (FP32, three real products per complex "
                         "product), fp32 (FP32, four), bf16x3 (BF16 hi/lo, three bf16 products per real product, "
                         "four real products), bf16x3_3m (BF16 hi/lo, three real products)")
    ap.add_argument("--epochs", type=int, default=100)
    ap.add_argument("--n-side", type=int, default=1024)
    ap.add_argument("--cpu-stride", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="time only the headline contraction mode")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the batched (C4), backward (C5) and NUFFT-synthesis measurements")
    ap.add_argument("--nufft-side", type=int, default=1024, help="image side of the NUFFT comparison (4 arcsec pixels)")
    ap.add_argument("--nufft-eps", type=float, default=1e-5)
    ap.add_argument("--nufft-transform", choices=["auto", "rocfft"], default="auto",
                    help="type-2 transform of the NUFFT comparison")
    ap.add_argument("--nufft-partitions", type=int, default=1,
                    help="image-domain partitions per axis of the NUFFT comparison")
    ap.add_argument("--only-nufft", action="store_true",
                    help="print only the NUFFT-vs-standard measurement (for profiling it alone)")
    ap.add_argument("--calibration-copy-mb", type=int, default=0,
                    help="before timing, copy this many MiB device-to-device once (a kernel of known traffic "
                         "for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (instances or pixel tiles would be "
              "sharded across GPUs with one final all-reduce of the images). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda", 0)

    if args.calibration_copy_mb > 0:
        n = args.calibration_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calibration_copy_mb} MiB read + {args.calibration_copy_mb} MiB written")
        del src, dst
    if args.only_nufft:
        from paper_2310_09200_amd import Context
        print(json.dumps({"nufft_vs_standard": measure_nufft(args, torch, Context(0))}), flush=True)
        return
    ctx, w, intervals, items, insts = build_inputs(args, torch, dev)
    n_levels = intervals.shape[0]
    modes = [args.precision] + ([] if args.no_compare else [m for m in MODES if m != args.precision])

    timing = time_modes(args, torch, ctx, w, items, modes, n_levels)
    ms, kern, stage, products = timing[args.precision]
    total_products = products * w.n_pix
    value = total_products / (ms / 1000.0)

    cpu, sel, ref_img = (None, None, None)
    if not args.no_cpu_baseline:
        cpu, sel, ref_img = cpu_baseline(args, w, items, n_levels)

    # executed MFMA work per product: 8 flop (four real MACs), 6 (three); BF16 x3 three times that in bf16
    exec_flop = {"fp32": 8.0, "fp32_3m": 6.0, "bf16x3": 24.0, "bf16x3_3m": 18.0}
    peak = {"fp32": FP32_PEAK_TFLOPS, "fp32_3m": FP32_PEAK_TFLOPS, "bf16x3": BF16_PEAK_TFLOPS,
            "bf16x3_3m": BF16_PEAK_TFLOPS}
    flops = exec_flop[args.precision] * total_products
    achieved = flops / (kern / 1000.0) / 1e12
    out = {
        "metric": "pixel*antenna*eigvec products/s for standard synthesis; compensated vs plain FP32 at 1e-4",
        "value": value,
        "unit": "products/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3" if args.precision.startswith("bf16") else "f32",
        "data": "synthetic",
        "config": {"workload": f"LOFAR-like single channel: L=512 stations (50 km), K=512 eigenpairs, "
                               f"{w.n_side}x{w.n_side} pixels over 10 deg, {args.epochs} epochs over 6 h, "
                               f"{n_levels - 1}+1 k-means levels, FP64 phase arguments",
                   "n_ant": 512, "n_eig": 512, "n_pix": w.n_pix, "n_instances": args.epochs,
                   "n_levels": n_levels, "contraction": args.precision,
                   "launch": "batched: one synthesis launch over all epochs per step"},
        "fp32_equivalent_mfma_fraction": 8.0 * value / (FP32_PEAK_TFLOPS * 1e12),
        "kernel_ms_per_step": kern,
        "staging_ms_per_step": stage,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak[args.precision], "unit": "TFLOP/s",
                     "frac": achieved / peak[args.precision], "traffic": measured_traffic(args.precision),
                     "kernel": "synth_fwd_kernel",
                     "flops_per_launch": flops,
                     "flop_per_product": exec_flop[args.precision]},
    }
    modes_out = {}
    for m in modes:
        ms_m, kern_m, _, _ = timing[m]
        modes_out[m] = {"value": total_products / (ms_m / 1000.0), "ms_per_step": ms_m, "kernel_ms": kern_m,
                        "fp32_equivalent_mfma_fraction": 8.0 * total_products / (kern_m / 1000.0)
                        / (FP32_PEAK_TFLOPS * 1e12),
                        "mfma_fraction_of_own_peak": exec_flop[m] * total_products / (kern_m / 1000.0)
                        / (peak[m] * 1e12)}
    out["modes"] = modes_out
    # phase generation (FP64 argument and reduction, hardware sin/cos) against its own peak on this device:
    # the synthesis kernel evaluates every phase once per K pass of its tile (256 eigenpairs for K > 128)
    peak_pairs, probe_ms, probe_pairs = measure_phase_peak(torch, ctx, w, items)
    n_ant, n_eig, eig_per_pass = 512, 512, 256
    n_pass = -(-n_eig // eig_per_pass)
    alg_pairs = float(n_ant) * w.n_pix * args.epochs
    gen_pairs = n_pass * alg_pairs
    out["phase_generation"] = {
        "peak_pairs_per_s": peak_pairs, "probe": f"bb_phase_probe: {probe_pairs:.3e} pairs in {probe_ms:.3f} ms",
        "pairs_per_launch": alg_pairs, "passes": n_pass,
        "achieved_pairs_per_s": alg_pairs / (kern / 1000.0),
        "frac": alg_pairs / (kern / 1000.0) / peak_pairs,
        "generated_frac": gen_pairs / (kern / 1000.0) / peak_pairs,
        "note": "pairs_per_launch = N_pix * L * epochs; generated_frac counts every pass's evaluation: the share "
                "of the launch that phase generation would take at its own peak"}
    log(f"phase generation: probe peak {peak_pairs:.3e} pairs/s; synthesis {alg_pairs / (kern / 1000.0):.3e} "
        f"pairs/s ({100 * alg_pairs / (kern / 1000.0) / peak_pairs:.1f} % of peak; with {n_pass} passes "
        f"{100 * gen_pairs / (kern / 1000.0) / peak_pairs:.1f} %)")
    # compensated (BF16 x3) forms against the plain FP32 forms, whole-step times
    comp = {}
    for cm in ("bf16x3", "bf16x3_3m"):
        for pm in ("fp32", "fp32_3m"):
            if cm in timing and pm in timing:
                comp[f"speedup_{cm}_over_{pm}"] = timing[pm][0] / timing[cm][0]
    if comp:
        out["compensated_vs_fp32"] = comp
    if not args.no_extra:
        out["batched_c4"] = measure_c4(args, torch, ctx)
        out["backward_c5"] = measure_c5_backward(args, torch, ctx)
        out["nufft_vs_standard"] = measure_nufft(args, torch, ctx)
    if cpu is not None:
        out["cpu_baseline"] = cpu
        out["max_level_error_vs_oracle"] = {
            m: spot_error(args, torch, ctx, w, items, m, n_levels, sel, ref_img) for m in modes}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
