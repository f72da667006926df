#!/usr/bin/env python3
"""Throughput of the fine-registration hot path on one MI355X.

One step = sfoc_register_cps on the 2048 x 2048 scene pair: dense SFOC of
both images, float64 integral images of the reference, Fast-NCC_SFOC for the
400 interest points (20 x 20 grid, template 64, search +-32), peak fit and
consistency check.  Inputs are resident in HBM before the timed region.
The "batched" object reports the batching workload (64 uneven pairs, one
autotuned plan replayed as a hipGraph) against per-pair calls.

Prints one JSON line.  --gpus must be 1: this build runs on a single GPU.
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

PEAK_FP32_VALU = 157.3e12       # published FP32 vector rate: 256 CU x 4 SIMD x 32 lanes/cycle x 2 (FMA) x 2.4 GHz
PEAK_HBM = 8.0e12
PEAK_BF16_MFMA = 2.5e15         # published dense BF16 / FP16 matrix rate


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_scene2048_rectify10000.md")
KERNEL_SOURCES = {"describe": "sfoc_describe.hip", "describe_reference": "sfoc_describe.hip",
                  "integral": "sfoc_describe.hip", "match": "sfoc_match.hip", "rectify": "sfoc_rectify.hip"}


def stored_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary:
    (FETCH_SIZE * fetch_scale + WRITE_SIZE * write_scale) KiB, the scales
    measured on a plain device copy of known size.  None when the summary
    has no line for the kernel or was taken on a different kernel source."""
    import hashlib
    src = os.path.join(ROOT, "paper_2202_13347_amd", "csrc", KERNEL_SOURCES[kernel])
    if not os.path.exists(TRAFFIC_FILE) or not os.path.exists(src):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for line in open(TRAFFIC_FILE):
        f = line.strip().strip("`").split()
        if len(f) < 3 or f[0] != "traffic" or f[1] != kernel:
            continue
        kv = dict(x.split("=", 1) for x in f[2:] if "=" in x)
        if kv.get("sha256") != digest:
            return None
        return 1024.0 * (float(kv["fetch_kib"]) * float(kv["fetch_scale"]) +
                         float(kv["write_kib"]) * float(kv["write_scale"]))
    return None


def timed_and_traced(S, torch, step, steps: int):
    """Runs `steps` steps twice: untimed by events (the step time), then
    with the library's per-kernel HIP events on (the kernel durations).  The
    event pairs act as barriers between kernels and add about 4 % to a step,
    so the step time comes from the first pass.  Returns (seconds per step,
    seconds per step with events, {kernel: (ms, launches)}, last output)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    S.trace_enable(True)
    S.trace_collect()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = step()
    torch.cuda.synchronize()
    dt_traced = (time.perf_counter() - t0) / steps
    kt = S.trace_collect()
    S.trace_enable(False)
    return dt, dt_traced, kt, out


def sfoc_fma_per_px(p) -> float:
    """Algorithmic FMAs per output pixel of SFOC in separable form, counting
    every tap as one FMA: per sigma a (2R+1)-tap row pass for each of g, d
    (and dd when the second order uses the sigma) and a column pass for each
    basis map it feeds (2 first-order, 3 second-order); steering 2 per
    first-order and 3 per second-order channel; the dilated smoothing a
    separable (2K+1) + (2K+1) per rate and channel; normalisation 2 per
    channel plus one root per order.  Baseline (N 8, sigma 1/2/3): 312 + 40
    + 288 + 34 = 674."""
    sig = {}
    for s in p.s1[:p.n_s1]:
        sig[s] = sig.get(s, 0) | 1
    if p.second_order:
        for s in p.s2[:p.n_s2]:
            sig[s] = sig.get(s, 0) | 2
    conv = 0.0
    for s, use in sig.items():
        R = math.ceil(p.trunc * s - 1e-9)
        rows = 3 if use & 2 else 2
        cols = (2 if use & 1 else 0) + (3 if use & 2 else 0)
        conv += (rows + cols) * (2 * R + 1)
    N = p.n_orient
    orders = 2 if p.second_order else 1
    z = N * orders
    steer = 2 * N + (3 * N if p.second_order else 0)
    smooth = z * p.n_dil * 2 * (2 * p.K + 1)
    norm = 2 * z + orders
    return conv + steer + smooth + norm


def sfoc_flops_per_px(p) -> float:
    """Two flops per algorithmic FMA: 1348 at the baseline."""
    return 2.0 * sfoc_fma_per_px(p)


def sfoc_bytes_per_px(es: int, z: int) -> float:
    """Bytes SFOC must move per pixel: the float32 input and the stored
    descriptor (z channels of es bytes): 68 at float32, 36 at bfloat16 /
    float16 for z = 16."""
    return 4.0 + z * es


INTEGRAL_BYTES_PER_PX = 24.0   # two float32 channel sums in, two float64 prefix sums out


def fastncc_flops_per_ip(M: int, z: int, V: int) -> float:
    """Algorithmic flops per interest point of Fast-NCC_SFOC with FFT side
    L = M (Eq. 13): 2z forward real 2-D FFTs and one inverse at
    2.5 L^2 log2(L^2) flops each, the spectrum product summed over channels
    (8 flops per half-spectrum bin per channel) and the NCC assembly of
    Eq. 9 (about 20 flops per offset, V^2 offsets): 20.07 M for m 64, r 32."""
    L = M
    fft = 2.5 * L * L * math.log2(L * L)
    return (2 * z + 1) * fft + z * L * (L // 2 + 1) * 8 + 20.0 * V * V


def fastncc_bytes_per_ip(m: int, M: int, z: int, es: int) -> float:
    """Bytes the matching must move per interest point: the template and
    search windows of every channel (655 KB at bfloat16 for m 64, M 128)."""
    return float(z * es * (m * m + M * M))


def roof_entry(name, ms, flops, nbytes, launches=1):
    """Per-kernel figures: achieved rates from the algorithmic flops and
    bytes per launch and the measured duration, against the FP32 VALU and
    HBM peaks, and against the binding roof min(peak, HBM x intensity)."""
    if not ms or ms <= 0:
        return None
    t = ms * 1e-3
    ach_f = flops / t
    ach_b = nbytes / t
    roof = min(PEAK_FP32_VALU, PEAK_HBM * flops / nbytes) if flops > 0 else PEAK_HBM
    return {"ms_per_launch": ms, "launches_per_step": launches,
            "algorithmic_flop": flops, "algorithmic_bytes": nbytes,
            "achieved_tflops": ach_f / 1e12, "achieved_gbs": ach_b / 1e9,
            "frac_valu_peak": ach_f / PEAK_FP32_VALU, "frac_hbm_peak": ach_b / PEAK_HBM,
            "binding_roof": "hbm" if flops <= 0 or PEAK_HBM * flops / nbytes < PEAK_FP32_VALU else "valu",
            "frac_binding_roof": (ach_f / roof) if flops > 0 else ach_b / PEAK_HBM}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pr, ips, m, r, budget_s: float):
    """The FP64 oracle as it stands, on the host cores: every CP of the same
    scene (SFOC of the template and search crops + Eq. 9-16 + peak) over a
    pool of worker processes, and a bounded single-core sample."""
    from oracle import sfoc_oracle as O
    from tests.oracle_pool import oracle_cps, pool_workers
    p = O.Params()
    workers = pool_workers()
    t0 = time.perf_counter()
    oracle_cps(pr.ref, pr.sen, ips, m, r, p, keep_surfaces=False, workers=workers)
    dt_pool = time.perf_counter() - t0
    t0 = time.perf_counter()
    done = 0
    order = list(range(0, len(ips), 7)) + [i for i in range(len(ips)) if i % 7]
    for k in order:
        O.match_one_region(pr.ref, pr.sen, ips[k], m, r, p)
        done += 1
        if time.perf_counter() - t0 >= budget_s and done >= 2:
            break
    dt1 = time.perf_counter() - t0
    return {"value": len(ips) / dt_pool, "unit": "CPs/s", "cores": workers, "kind": "oracle",
            "sample": f"all {len(ips)} CPs of the same scene, each computed from its template and search crops "
                      f"(FP64 SFOC with reflect-101 halo, FFT NCC with integral images, peak) over a pool of "
                      f"{workers} worker processes, {dt_pool:.1f} s including their start-up",
            "single_core": {"value": done / dt1, "unit": "CPs/s", "cores": 1,
                            "sample": f"{done} of the {len(ips)} CPs in one process, {dt1:.1f} s"},
            "os_cpu_count": os.cpu_count(), "cpu_model": cpu_model()}


def parity_vs_stored_oracle(S, name, cps, kind="o64", ref_kind=None):
    """The GPU's CPs against the oracle's stored decisions for the same
    seeded workload (tests/golden/make_oracle_cps.py): integer CPs equal,
    tie-set answers, largest score and sub-pixel differences."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"oracle_cps_{name}.npz")
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        rec, flags, ties = z[kind + "_rec"], z[kind + "_flags"], z[kind + "_ties"]
        base = z[(ref_kind or kind) + "_rec"]
    g = S.cps_to_numpy(cps)
    tie = {}
    for i, dy, dx in ties:
        tie.setdefault(int(i), set()).add((int(dy), int(dx)))
    bad = S.OOB | S.FLAT_T | S.FLAT_S | S.NONFINITE
    ok = (flags & bad) == 0
    same = ok & (g["dy"] == rec[:, 0]) & (g["dx"] == rec[:, 1])
    taken = [i for i in np.nonzero(ok & ~same)[0] if (int(g["dy"][i]), int(g["dx"][i])) in tie.get(int(i), ())]
    other = int(ok.sum() - same.sum()) - len(taken)
    out = {"oracle": kind, "cps": int(len(g)), "compared": int(ok.sum()), "integer_equal": int(same.sum()),
           "ambiguous": len(tie), "ambiguous_other_index": len(taken), "mismatched": other,
           "max_score_err": float(np.max(np.abs(g["score"][same] - rec[same, 4]))) if same.any() else None,
           "max_subpx_err": float(np.max(np.abs(np.stack([g["sub_dy"][same] - rec[same, 2],
                                                         g["sub_dx"][same] - rec[same, 3]])))) if same.any() else None}
    if ref_kind:
        tot_g = np.stack([g["dy"] + g["sub_dy"], g["dx"] + g["sub_dx"]], 1).astype(np.float64)
        tot_o = np.stack([base[:, 0] + base[:, 2], base[:, 1] + base[:, 3]], 1)
        e = np.abs(tot_g - tot_o).max(axis=1)[ok]
        s64 = ok & (g["dy"] == base[:, 0]) & (g["dx"] == base[:, 1])
        out["vs_" + ref_kind] = {"integer_equal": int(s64.sum()),
                                 "max_score_err": float(np.max(np.abs(g["score"][s64] - base[s64, 4]))),
                                 "max_offset_err_px": float(e.max()), "median_offset_err_px": float(np.median(e))}
    return out


def described_px(S, ips, m, r, H, W):
    """Pixels the describe launch of a register step covers: the whole
    reference image and the sensed image's tiles under the templates, both
    in one launch.  The pair call describes each IP's own template tiles (a
    tile two IPs share is described twice), so the tiles are counted per IP,
    each clipped to the image."""
    import numpy as np
    sen_px = 0.0
    for k in range(len(ips)):
        t = S.sensed_tiles(ips[k:k + 1], m, r, H, W, H, W)
        sen_px += float((np.minimum(32, H - t[:, 0]) * np.minimum(32, W - t[:, 1])).sum())
    return H * W + sen_px, sen_px


def kernel_table(kt, steps, p, H, W, n, m, r, desc_px=None):
    """Roof entries of the describe, integral and match launches of one
    register step (HIP-event durations from the library's trace); desc_px is
    the pixel count of a describe launch (H W if not given)."""
    z = p.z
    es = 4 if p.desc_dtype == 0 else 2
    avg = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in kt.items()}
    per = {k: kt[k][1] / steps for k in kt}
    M, V = m + 2 * r, 2 * r + 1
    dpx = H * W if desc_px is None else desc_px
    return {
        "describe": roof_entry("describe", avg["describe"], sfoc_flops_per_px(p) * dpx,
                               sfoc_bytes_per_px(es, z) * dpx, per["describe"]),
        "integral": roof_entry("integral", avg["integral"], 0.0, INTEGRAL_BYTES_PER_PX * H * W, per["integral"]),
        "match": roof_entry("match", avg["match"], fastncc_flops_per_ip(M, z, V) * n,
                            fastncc_bytes_per_ip(m, M, z, es) * n, per["match"]),
    }


def run_integral_alone(args, S, torch, p, ref):
    """sfoc_describe with integral images on the scene's reference image:
    the describe launch, then the integral-image kernels on the same stream
    with nothing beside them (in the register step they share the GPU with
    the sensed image's describe)."""
    H, W = ref.shape
    z = p.z
    desc = torch.empty((z, H, W), dtype=torch.float32, device=ref.device)
    i1 = torch.empty((H + 1, W + 1), dtype=torch.float64, device=ref.device)
    i2 = torch.empty_like(i1)
    wsb = S.describe_workspace(H, W, p)
    ws = torch.empty(wsb, dtype=torch.uint8, device=ref.device)
    fn = S.lib().sfoc_describe
    import ctypes

    def step():
        rc = fn(ref.data_ptr(), H, W, ref.stride(0), ctypes.byref(p), desc.data_ptr(), i1.data_ptr(),
                i2.data_ptr(), ws.data_ptr(), wsb, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == 0, rc

    for _ in range(args.warmup):
        step()
    _, _, kt, _ = timed_and_traced(S, torch, step, args.steps)
    ms = kt["integral"][0] / max(1, kt["integral"][1])
    return {"workload": f"sfoc_describe with integral images of the {H}x{W} reference image",
            "integral_ms_per_call": ms, "describe_ms_per_call": kt["describe"][0] / max(1, kt["describe"][1]),
            "kernels": {"integral": roof_entry("integral", ms, 0.0, INTEGRAL_BYTES_PER_PX * H * W, 1)}}


def run_precision(args, S, synth, torch, dev, scene):
    """Descriptor storage in bfloat16 and float16 (FFT in float32, integral
    images and variance in float64): the scene step and the 10000 x 10000
    precision workload (5000 IPs, m 64, r 48), with per-kernel roofs at the
    2-byte storage and every CP against the oracle's stored decisions on the
    same rounded descriptors (O64q) and on unrounded ones (O64)."""
    import numpy as np
    out = {}
    pr, ips, m, r = scene
    H, W = pr.ref.shape
    ref = torch.from_numpy(pr.ref).to(dev)
    sen = torch.from_numpy(pr.sen).to(dev)
    dips = torch.from_numpy(ips).to(dev)
    for kind, dt in (("bf16", S.DTYPE_BF16), ("f16", S.DTYPE_F16)):
        p = S.preset("baseline", dtype=dt)
        R = S.Registrar(H, W, H, W, len(ips), m, r, p, device=dev)
        for _ in range(args.warmup):
            R(ref, sen, dips)
        dts, _, kt, cps = timed_and_traced(S, torch, lambda: R(ref, sen, dips), args.steps)
        d_ms = kt["describe"][0] / max(1, kt["describe"][1])
        dpx = described_px(S, ips, m, r, H, W)[0]
        out["scene_" + kind] = {
            "value": len(ips) / dts, "unit": "CPs/s", "ms_per_step": 1e3 * dts,
            "sfoc_mpixel_per_s": dpx / (d_ms * 1e-3) / 1e6 if d_ms > 0 else None,
            "kernels": kernel_table(kt, args.steps, p, H, W, len(ips), m, r, dpx),
            "parity": parity_vs_stored_oracle(S, "scene", cps, kind, ref_kind="o64")}
        del R
    del ref, sen, dips
    if args.large:
        t0 = time.perf_counter()
        lp, lips, lm, lr = synth.workload(synth.LARGE, 0)
        gen_s = time.perf_counter() - t0
        H, W = lp.ref.shape
        ref = torch.from_numpy(lp.ref).to(dev)
        sen = torch.from_numpy(lp.sen).to(dev)
        dips = torch.from_numpy(lips).to(dev)
        for kind, dt in (("bf16", S.DTYPE_BF16), ("f16", S.DTYPE_F16)):
            p = S.preset("baseline", dtype=dt)
            R = S.Registrar(H, W, H, W, len(lips), lm, lr, p, device=dev)
            R(ref, sen, dips)
            torch.cuda.synchronize()
            dts, _, kt, cps = timed_and_traced(S, torch, lambda: R(ref, sen, dips), args.large_steps)
            d_ms = kt["describe"][0] / max(1, kt["describe"][1])
            dpx = described_px(S, lips, lm, lr, H, W)[0]
            out["large_" + kind] = {
                "workload": f"one {H}x{W} seeded pair (speckled sensed image), {len(lips)} IPs (71x71 grid truncated), "
                            f"template {lm}, search +-{lr}, N=8, sigma 1/2/3, {kind} descriptors, float32 FFT, "
                            f"float64 integral images and variance; whole images resident in HBM",
                "value": len(lips) / dts, "unit": "CPs/s", "ms_per_step": 1e3 * dts, "steps": args.large_steps,
                "sfoc_mpixel_per_s": dpx / (d_ms * 1e-3) / 1e6 if d_ms > 0 else None,
                "kernels": kernel_table(kt, args.large_steps, p, H, W, len(lips), lm, lr, dpx),
                "parity": parity_vs_stored_oracle(S, "large", cps, kind, ref_kind="o64"),
                "generate_s": gen_s}
            if kind == "bf16":
                out["large_streamed_bf16"] = run_streamed(args, S, torch, p, ref, sen, lips, lm, lr, cps, R.wsb)
            del R
            torch.cuda.empty_cache()
        del ref, sen, dips
        torch.cuda.empty_cache()
    return out


def run_batched(args, S, synth, torch, p, dev):
    """The batching workload: 64 uneven pairs as one autotuned plan replayed
    as a hipGraph, against the plain path (one sfoc_register_cps per pair on
    preallocated workspaces) on the same resident inputs.  Both describe
    only the sensed tiles under the templates, so the gain is that of
    batching alone."""
    import numpy as np
    t0 = time.perf_counter()
    work = synth.batch_workload(args.seed, workers=min(16, os.cpu_count() or 1))
    gen_s = time.perf_counter() - t0
    dp, regs = [], []
    for spec, pr, ips in work:
        q = dict(ref=torch.from_numpy(pr.ref).to(dev), sen=torch.from_numpy(pr.sen).to(dev),
                 ips=torch.from_numpy(ips).to(dev), m=spec["m"], r=spec["r"])
        dp.append(q)
        H, W = pr.ref.shape
        regs.append(S.Registrar(H, W, H, W, len(ips), spec["m"], spec["r"], p, device=dev))
    n_ips = sum(len(w[2]) for w in work)
    mpx = sum(w[1].ref.size for w in work) / 1e6

    def plain():
        for q, R in zip(dp, regs):
            R(q["ref"], q["sen"], q["ips"])

    for _ in range(args.batched_warmup):
        plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batched_steps):
        plain()
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / args.batched_steps

    def time_plan(flags, pp):
        t0 = time.perf_counter()
        plan = S.Plan(dp, pp, flags=flags)
        create_s = time.perf_counter() - t0
        for _ in range(args.batched_warmup):
            plan()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batched_steps):
            plan()
        torch.cuda.synchronize()
        return plan, (time.perf_counter() - t0) / args.batched_steps, create_s

    def correct(cps_list):
        n_ok = n_valid = 0
        for (spec, pr, _), c in zip(work, cps_list):
            g = S.cps_to_numpy(c)
            v = (g["flags"] & S.VALID) != 0
            e = np.hypot(g["dy"] + g["sub_dy"] - pr.shift[0], g["dx"] + g["sub_dx"] - pr.shift[1])
            n_valid += int(v.sum())
            n_ok += int((e[v] <= 1.5).sum())
        return {"valid": n_valid, "correct_1p5px": n_ok}

    plain_cps = [R.cps.clone() for R in regs]
    plan, batch_s, create_s = time_plan(S.PLAN_GRAPH | S.PLAN_AUTOTUNE, p)
    info = plan.info()
    # pairs whose tuned transform side is the per-pair call's default must
    # give identical records; on another side the NCC values round
    # differently, so the integer CPs and the VALID decisions are compared
    same = n_same_side = same_int = 0
    for k, (spec, _, _) in enumerate(work):
        a, b = plan.cps[k].cpu().numpy(), regs[k].cps.cpu().numpy()
        if (info["fft_side"][k], info["blocks"][k]) == S.match_candidates(spec["m"], spec["r"])[0]:
            n_same_side += len(a)
            same += int((a == b).all(axis=1).sum())
        same_int += int(((a[:, 2] == b[:, 2]) & (a[:, 3] == b[:, 3]) & ((a[:, 7] & S.VALID) == (b[:, 7] & S.VALID))).sum())
    classes = {}
    for (spec, _, _), L, nb in zip(work, info["fft_side"], info["blocks"]):
        classes[f"m{spec['m']}_r{spec['r']}"] = f"L{L}x{nb * nb}"
    plan.close()
    # bfloat16 descriptor storage in the plan, against the plain float32 calls
    pb = S.preset("baseline", dtype=S.DTYPE_BF16)
    plan_b, bf16_s, _ = time_plan(S.PLAN_GRAPH | S.PLAN_AUTOTUNE, pb)
    same_b = 0
    for k, c in enumerate(plain_cps):
        a, b = plan_b.cps[k].cpu().numpy(), c.cpu().numpy()
        same_b += int(((a[:, 2] == b[:, 2]) & (a[:, 3] == b[:, 3])).sum())
    acc_b = correct(plan_b.cps)
    plan_b.close()
    return {"workload": f"{len(work)} seeded pairs, square sides U{{512..4096}} ({mpx:.0f} Mpx per image set), "
                        f"{n_ips} uniform IPs (50..500 per pair), m in {{48,64,96}}, r in {{16,32,64}}, "
                        f"every second sensed image speckled; one autotuned plan replayed as a hipGraph",
            "value": n_ips / batch_s, "unit": "CPs/s", "ms_per_step": 1e3 * batch_s,
            "plain_value": n_ips / plain_s, "plain_ms_per_step": 1e3 * plain_s, "gain": plain_s / batch_s,
            "identical_cps": same, "cps_on_default_side": n_same_side, "integer_cps_and_valid_equal": same_int,
            "ips": n_ips, "steps": args.batched_steps,
            "accuracy_plain": correct(plain_cps),
            "sides": classes, "persistent": info["persistent"], "describe_tiles": info["describe_tiles"],
            "describe_config": info["describe_config"],
            "match_items": info["match_items"],
            "tuned_classes": info["tuned_classes"], "plan_create_s": create_s, "generate_s": gen_s,
            "device_gb": info["device_bytes"] / 2 ** 30,
            "bf16": {"value": n_ips / bf16_s, "ms_per_step": 1e3 * bf16_s, "gain_vs_plain_f32": plain_s / bf16_s,
                     "integer_cps_equal_to_plain_f32": same_b, "accuracy": acc_b}}


def run_learned(args, S, synth, torch, p, dev, ref, sen, dips, m, r):
    """The learned head on the scene workload: describe + match (with NCC
    surfaces) + head features + head inference per step, against the plain
    step; and its accuracy against the plain peak fit and consistency check
    on held-out seeded pairs."""
    from paper_2202_13347_amd import head as HD
    head = S.Head(HD.load_params(), device=dev)
    H, W = ref.shape
    n = dips.shape[0]

    def step():
        d_ref, i1, i2 = S.describe(ref, p)
        d_sen, _, _ = S.describe(sen, p, integrals=False)
        cps, ncc = S.fastncc_match(d_sen, d_ref, i1, i2, dips, m, r, want_ncc=True)
        crops, stats = S.head_features(d_sen, d_ref, i1, i2, dips, m, r, ncc, cps)
        head.infer(crops, stats, cps)
        return cps

    for _ in range(args.warmup):
        step()
    dt, _, kt, _ = timed_and_traced(S, torch, step, args.steps)
    res = HD.evaluate(head, range(HD.TEST_SEED0, HD.TEST_SEED0 + args.learned_pairs),
                      workers=min(16, os.cpu_count() or 1))
    return {"workload": f"the scene step with NCC surfaces kept, then head features and inference for its {n} "
                        f"CPs; accuracy on {args.learned_pairs} held-out 512x512 pairs (m 64, r 32, 30% with "
                        f"occlusion patches)",
            "value": n / dt, "unit": "CPs/s", "ms_per_step": 1e3 * dt,
            "head_ms_per_step": (kt["head_features"][0] + kt["head_forward"][0]) / args.steps,
            "accuracy": res}


RANSAC_HYP = 2048


def ransac_flops_per_eval(model: int) -> float:
    """FP64 flops of one inlier test (one hypothesis against one candidate):
    projective: denominator 4, two numerators 8, minus X w and Y w 4, squared
    distance 3, threshold times w^2 2 = 21; affine: numerators 8, minus X
    and Y 2, squared distance 3 = 13."""
    return 21.0 if model == 8 else 13.0


def run_ransac(args, S, synth, torch, p, dev):
    """Registration of a pair related by a projective map (rotation, scale,
    shift, perspective; occlusion patches on the sensed image): the scene
    step followed by projective RANSAC over its CPs, against the same step
    with the median-translation check; accuracy against the known map."""
    import numpy as np
    rec = synth.WARP
    w = synth.make_warp_pair(args.seed, rec)
    size, m, r = rec["size"], rec["m"], rec["r"]
    ips = synth.grid_ips(size, size, rec["n_side"], (m + 1) // 2 + r)
    n = len(ips)
    ref = torch.from_numpy(w.ref).to(dev)
    sen = torch.from_numpy(w.sen).to(dev)
    dips = torch.from_numpy(ips).to(dev)
    Rg = S.Registrar(size, size, size, size, n, m, r, p, device=dev)
    rp = S.ransac_params(S.MODEL_PROJECTIVE, RANSAC_HYP, (size, size, size, size), 1.5, 2)
    RS = S.Ransac(n, rp, device=dev)
    words = torch.from_numpy(synth.ransac_words(args.seed, RANSAC_HYP, 4).view(np.int32)).to(dev)
    plain = S.cps_to_numpy(Rg(ref, sen, dips)).copy()

    def step():
        cps = Rg(ref, sen, dips)
        RS(cps, words)
        return cps

    for _ in range(args.warmup):
        step()
    dt, _, kt, cps = timed_and_traced(S, torch, step, args.steps)
    got = S.cps_to_numpy(cps)
    info = RS.info.cpu().numpy()
    model = RS.model.cpu().numpy().reshape(3, 3)
    src = np.stack([plain["sen_row"], plain["sen_col"]], 1).astype(np.float64)
    pred = src + np.stack([plain["dy"] + plain["sub_dy"].astype(np.float64),
                           plain["dx"] + plain["sub_dx"].astype(np.float64)], 1)
    correct = np.hypot(*(pred - synth.apply_model(w.model, src)).T) <= 1.5
    elig = (plain["flags"] & (S.VALID | S.INCONSISTENT)) != 0

    def pr(flags):
        v = (flags & S.VALID) != 0
        tp = int((v & correct).sum())
        return {"valid": int(v.sum()), "precision": tp / max(1, int(v.sum())),
                "recall": tp / max(1, int((elig & correct).sum()))}

    grid = np.stack(np.meshgrid(np.linspace(0, size - 1, 9), np.linspace(0, size - 1, 9)), -1).reshape(-1, 2)
    ms_r = kt["ransac"][0] / max(1, kt["ransac"][1])
    evals = int(info[0]) * RANSAC_HYP
    return {"workload": f"one seeded {size}x{size} pair related by a projective map (rotation 0.375-0.75 deg, "
                        f"scale 0.2-0.4 %, shift <= 5 px, perspective <= 1e-6/px; sensed speckled, 4-8 occlusion "
                        f"patches), {n} IPs on a grid, m {m}, r {r}; describe + match + projective RANSAC "
                        f"({RANSAC_HYP} hypotheses, 2 refits, 1.5 px)",
            "value": n / dt, "unit": "CPs/s", "ms_per_step": 1e3 * dt, "ransac_ms_per_call": ms_r,
            "hypothesis_tests_per_s": evals / (ms_r * 1e-3) if ms_r > 0 else None,
            "fp64_tflops_hypotheses": evals * ransac_flops_per_eval(8) / (ms_r * 1e-3) / 1e12 if ms_r > 0 else None,
            "candidates": int(info[0]), "inliers": int(info[1]),
            "model_error_px": float(np.abs(synth.apply_model(model, grid) - synth.apply_model(w.model, grid)).max()),
            "accuracy": {"correct_candidates": int((elig & correct).sum()), "ransac": pr(got["flags"]),
                         "median_check": pr(plain["flags"])}}


RECT_SIDE = 10000
RECT_BYTES_PER_PX = 8.0   # one float32 written, one float32 of sensed image read (each sensed pixel once)


def run_rectify(args, S, torch, dev):
    """Rectification of a 10000 x 10000 float32 image (seeded uniform
    values) through a projective map (rotation 0.5 deg, scale 1.002,
    perspective 1e-7 / px), HIP-event time per launch against the HBM roof
    at 8 algorithmic bytes per output pixel."""
    import numpy as np
    n = RECT_SIDE
    gen = torch.Generator(device=dev).manual_seed(args.seed)
    sen = torch.rand((n, n), dtype=torch.float32, device=dev, generator=gen)
    out = torch.empty_like(sen)
    a = np.deg2rad(0.5)
    c = 0.5 * (n - 1)
    M = np.array([[1.002 * np.cos(a), -1.002 * np.sin(a), 0.0], [1.002 * np.sin(a), 1.002 * np.cos(a), 0.0],
                  [1e-7, -1e-7, 1.0]])
    C = np.array([[1, 0, c], [0, 1, c], [0, 0, 1.0]])
    Ci = np.array([[1, 0, -c], [0, 1, -c], [0, 0, 1.0]])
    M = C @ M @ Ci
    model = torch.from_numpy((M / M[2, 2]).reshape(9)).to(dev)
    for _ in range(args.warmup):
        S.rectify(sen, model, (n, n), out=out)
    torch.cuda.synchronize()
    S.trace_enable(True)
    S.trace_collect()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        S.rectify(sen, model, (n, n), out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    kt = S.trace_collect()
    S.trace_enable(False)
    ms = kt["rectify"][0] / max(1, kt["rectify"][1])
    gbs = n * n * RECT_BYTES_PER_PX / (ms * 1e-3) / 1e9
    return {"workload": f"{n}x{n} float32 image rectified through a projective map (rotation 0.5 deg, scale 1.002, "
                        f"perspective 1e-7/px) into a {n}x{n} reference grid, bilinear",
            "ms_per_call": ms, "wall_ms_per_call": 1e3 * dt, "gpx_per_s": n * n / (ms * 1e-3) / 1e9,
            "roofline": {"kernel": "rectify", "bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
                         "frac": gbs / 8000.0, "traffic": stored_traffic("rectify"),
                         "algorithmic_bytes_per_px": RECT_BYTES_PER_PX}}


FAST_OPS_PER_PX = 176.0   # 16 differences, 3 x 32 pairwise min / max, 16 x 4 to close the arcs
# The published FP32 vector rate (157.3 TFLOP/s) counts an FMA as two flops:
# non-fused lane operations (add, min, max) at the same issue rate.
PEAK_FP32_OPS = PEAK_FP32_VALU / 2


def run_fast(args, S, synth, torch, dev):
    """Block-based FAST: on the scene's sensed image (20 x 20 blocks, one
    interest point each, matching margin) followed by registration from
    those points; and on a 10000 x 10000 image (seeded uniform values,
    Gaussian-smoothed on the device by a 5 x 5 box twice) for throughput."""
    import numpy as np
    pr, _, m, r = synth.workload(synth.SCENE, args.seed)
    margin = (m + 1) // 2 + r
    sen = torch.from_numpy(pr.sen).to(dev)
    ref = torch.from_numpy(pr.ref).to(dev)
    D = S.Detector(sen.shape[0], sen.shape[1], 20, 20, 1, 0.05, margin, device=dev)
    Rg = S.Registrar(ref.shape[0], ref.shape[1], sen.shape[0], sen.shape[1], 400, m, r, S.preset("baseline"),
                     device=dev)

    def step():
        ips, _, _, n = D(sen)
        return Rg(ref, sen, ips[:400])

    for _ in range(args.warmup):
        step()
    dt, _, kt, cps = timed_and_traced(S, torch, step, args.steps)
    n = int(D.n_out.item())
    c = S.cps_to_numpy(cps)[:n]
    v = (c["flags"] & S.VALID) != 0
    err = np.hypot(c["dy"] + c["sub_dy"] - pr.shift[0], c["dx"] + c["sub_dx"] - pr.shift[1])
    ms_scene = kt["fast"][0] / max(1, kt["fast"][1])
    # throughput image
    side = 10000
    gen = torch.Generator(device=dev).manual_seed(args.seed)
    big = torch.rand((1, 1, side, side), dtype=torch.float32, device=dev, generator=gen)
    box = torch.full((1, 1, 5, 5), 1.0 / 25.0, dtype=torch.float32, device=dev)
    big = torch.nn.functional.conv2d(torch.nn.functional.conv2d(big, box, padding=2), box, padding=2)[0, 0].contiguous()
    Db = S.Detector(side, side, 71, 71, 1, 0.002, 80, device=dev)
    for _ in range(args.warmup):
        Db(big)
    torch.cuda.synchronize()
    S.trace_enable(True)
    S.trace_collect()
    for _ in range(args.steps):
        Db(big)
    torch.cuda.synchronize()
    kt = S.trace_collect()
    S.trace_enable(False)
    ms_big = kt["fast"][0] / max(1, kt["fast"][1])
    ach = side * side * FAST_OPS_PER_PX / (ms_big * 1e-3)
    return {"workload": f"block-based FAST on the scene's 2048x2048 sensed image (20x20 blocks, 1 IP each, "
                        f"threshold 0.05, margin {margin}), then registration of the pair from those IPs; and "
                        f"on a {side}x{side} smoothed-noise image (71x71 blocks, margin 80)",
            "value": n / dt, "unit": "CPs/s", "ms_per_step": 1e3 * dt, "detect_ms_2048": ms_scene,
            "ips": n, "valid": int(v.sum()), "correct_1p5px": int((err[v] <= 1.5).sum()),
            "detect_ms_10000": ms_big, "mpx_per_s_10000": side * side / (ms_big * 1e-3) / 1e6,
            "roofline": {"kernel": "fast", "bound": "alu", "achieved": ach / 1e12, "peak": PEAK_FP32_OPS / 1e12,
                         "unit": "Tops/s", "frac": ach / PEAK_FP32_OPS, "ops_per_px": FAST_OPS_PER_PX,
                         "ips_10000": int(Db.n_out.item())}}


def run_sweep(args, S, torch):
    """Noise sensitivity and the F-SFOC ablation at the paper's noise
    levels on seeded pairs (CMR per level), with the GPU time it took."""
    from paper_2202_13347_amd import sweep as W
    t0 = time.perf_counter()
    res = W.run(args.sweep_pairs)
    res["wall_s"] = time.perf_counter() - t0
    res["workload"] = (f"{args.sweep_pairs} seeded {res['size']}x{res['size']} pairs (shift up to 16 px), "
                       f"Gaussian white noise v = 0..0.01 and speckle v = 0..0.1 on the sensed image, "
                       f"{res['ips_per_pair']} block-FAST IPs per pair, 80x80 templates, r {res['radius']}, "
                       f"paper preset (N 6); SFOC and F-SFOC (first-order channels only)")
    return res


def run_streamed(args, S, torch, p, ref, sen, ips, m, r, whole_cps, whole_ws, band_rows=1024):
    """The 10000 x 10000 precision workload streamed over bands of 1024 IP
    rows (sfoc_register_cps_streamed, IPs sorted by row): one band's
    descriptors, integral images and scratch resident at a time.  Step time
    (the call synchronises twice to plan its bands on the host), workspace
    against the whole-image call's, integer CPs and flags equal to the
    whole-image records, and parity against the stored oracle."""
    import numpy as np
    order = np.argsort(ips[:, 0], kind="stable")
    sips = torch.from_numpy(np.ascontiguousarray(ips[order])).to(ref.device)
    H, W = ref.shape
    R = S.StreamedRegistrar(H, W, H, W, len(ips), m, r, p, band_rows=band_rows, device=ref.device)
    R(ref, sen, sips)
    torch.cuda.synchronize()
    dts, _, kt, cps = timed_and_traced(S, torch, lambda: R(ref, sen, sips), args.large_steps)
    g = np.empty((len(ips), 8), np.int32)
    g[order] = cps.cpu().numpy()
    w = S.cps_to_numpy(whole_cps)
    gg = S.cps_to_numpy(g)
    bands, y0 = 0, None
    for y in ips[order, 0]:   # the library's band rule: a band starts at the first IP row past the last band
        if y0 is None or y >= y0 + band_rows:
            bands, y0 = bands + 1, int(y)
    out = {"band_rows": band_rows, "bands": bands,
           "value": len(ips) / dts, "unit": "CPs/s", "ms_per_step": 1e3 * dts, "steps": args.large_steps,
           "workspace_gb": R.wsb / 1e9, "whole_image_workspace_gb": whole_ws / 1e9,
           "integer_cps_equal_to_whole": int(np.sum((gg["dy"] == w["dy"]) & (gg["dx"] == w["dx"]))),
           "flags_equal_to_whole": int(np.sum(gg["flags"] == w["flags"])), "ips": int(len(ips)),
           "max_score_diff_to_whole": float(np.abs(gg["score"] - w["score"]).max()),
           "parity": parity_vs_stored_oracle(S, "large", g, "bf16", ref_kind="o64")}
    del R
    return out


def run_small_windows(args, S, synth, torch, dev):
    """FFT or matrix cores for small windows: the scene pair and its 400 IPs
    with the small configuration's template (32) and search radius (10) at
    bfloat16 storage, matched by the FFT of side 64, by the direct form
    (R_ST summed in space as 32 x 32 x 16 MFMAs), and by an autotuned plan.
    The scene's shift (up to 30 px) exceeds the radius, so every IP gets the
    rounded true shift as its prior, as a coarse registration would give.
    Plans with one pair each; per-launch match times from the library's
    events.  The direct form's rates: useful flops 2 V^2 m^2 z per IP and
    the MFMA flops it issues, 2 x 32 x 32 x 16 per MFMA, ceil(M / 16) m z
    MFMAs per IP, against the dense BF16 peak."""
    import numpy as np
    pr, ips, _, _ = synth.workload(synth.SCENE, args.seed)
    m, r = 32, 10
    V, M = 2 * r + 1, m + 2 * r
    p = S.preset("baseline", dtype=S.DTYPE_BF16)
    prior = np.tile(np.round(np.asarray(pr.shift)).astype(np.int32), (len(ips), 1))
    d = dict(ref=torch.from_numpy(pr.ref).to(dev), sen=torch.from_numpy(pr.sen).to(dev),
             ips=torch.from_numpy(ips).to(dev), prior=torch.from_numpy(prior).to(dev), m=m, r=r)
    n = len(ips)
    out = {"workload": f"scene pair ({pr.ref.shape[0]}x{pr.ref.shape[1]}), {n} IPs, template {m}, search +-{r} "
                       f"around the rounded true shift as prior, N=8, sigma 1/2/3, bfloat16 descriptors"}
    got = {}
    for name, side, flags in (("fft64", 64, 0), ("direct", S.MATCH_DIRECT, 0), ("autotuned", 0, S.PLAN_AUTOTUNE)):
        d["fft_side"] = side
        plan = S.Plan([d], p, flags=flags)
        for _ in range(3):
            plan()
        dt, _, kt, _ = timed_and_traced(S, torch, plan, args.steps)
        ms = kt["match"][0] / max(1, kt["match"][1])
        got[name] = S.cps_to_numpy(plan.cps[0]).copy()
        out[name] = {"form": plan.info()["fft_side"][0], "match_us": 1e3 * ms, "ms_per_step": 1e3 * dt,
                     "cps_per_s": n / dt}
        plan.close()
    useful = 2.0 * V * V * m * m * p.z * n
    issued = 2.0 * 32 * 32 * 16 * ((M + 15) // 16) * m * p.z * n
    t = out["direct"]["match_us"] * 1e-6
    out["direct"]["useful_tflops"] = useful / t / 1e12
    out["direct"]["mfma_tflops"] = issued / t / 1e12
    out["direct"]["frac_bf16_mfma_peak"] = issued / t / PEAK_BF16_MFMA
    out["speedup_direct_vs_fft64"] = out["fft64"]["match_us"] / out["direct"]["match_us"]
    a, b = got["fft64"], got["direct"]
    bad = S.OOB | S.FLAT_T | S.FLAT_S | S.EDGE_PEAK | S.NONFINITE
    ok = ((a["flags"] & bad) == 0) & ((b["flags"] & bad) == 0)
    err = np.hypot(prior[:, 0] + b["dy"] + b["sub_dy"] - pr.shift[0], prior[:, 1] + b["dx"] + b["sub_dx"] - pr.shift[1])
    valid = (b["flags"] & S.VALID) != 0
    out["direct"]["accuracy"] = {"valid": int(valid.sum()), "correct_1p5px": int((err[valid] <= 1.5).sum())}
    out["direct_vs_fft64"] = {"integer_cps_equal": int(np.sum((a["dy"] == b["dy"]) & (a["dx"] == b["dx"]) & ok)),
                              "compared": int(ok.sum()),
                              "max_score_diff": float(np.abs(a["score"][ok] - b["score"][ok]).max()) if ok.any()
                              else None}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds for the oracle baseline (0: skip)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--batched-steps", type=int, default=5, help="timed steps of the batching workload (0: skip)")
    ap.add_argument("--batched-warmup", type=int, default=2)
    ap.add_argument("--learned-pairs", type=int, default=100, help="held-out pairs for the head (0: skip)")
    ap.add_argument("--ransac", type=int, default=1, help="warped-pair registration with RANSAC (0: skip)")
    ap.add_argument("--rectify", type=int, default=1, help="10000^2 rectification (0: skip)")
    ap.add_argument("--fast", type=int, default=1, help="block-based FAST detection (0: skip)")
    ap.add_argument("--sweep-pairs", type=int, default=4, help="pairs of the noise-sensitivity sweep (0: skip)")
    ap.add_argument("--precision", type=int, default=1, help="bfloat16 / float16 storage sections (0: skip)")
    ap.add_argument("--large", type=int, default=1, help="the 10000^2 precision workload (0: skip)")
    ap.add_argument("--large-steps", type=int, default=3)
    ap.add_argument("--small-windows", type=int, default=1,
                    help="FFT vs matrix-core matching for small windows (0: skip)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2202_13347_amd import sfoc as S
    from paper_2202_13347_amd import synth

    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(1)
    S.lib()
    pr, ips, m, r = synth.workload(synth.SCENE, args.seed)
    H, W = pr.ref.shape
    n = len(ips)
    p = S.preset("baseline")
    dev = torch.device("cuda:0")
    ref = torch.from_numpy(pr.ref).to(dev)
    sen = torch.from_numpy(pr.sen).to(dev)
    dips = torch.from_numpy(ips).to(dev)
    R = S.Registrar(H, W, H, W, n, m, r, p, device=dev)
    stream = torch.cuda.current_stream()

    if args.copy_mb > 0:
        src = torch.empty(args.copy_mb << 18, dtype=torch.float32, device=dev).uniform_()
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        R(ref, sen, dips)
    dt, dt_traced, kt, _ = timed_and_traced(S, torch, lambda: R(ref, sen, dips), args.steps)
    elapsed = dt * args.steps
    ms_step = 1e3 * dt
    cps_s = n / dt

    g = S.cps_to_numpy(R.cps)
    err = np.hypot(g["dy"] + g["sub_dy"] - pr.shift[0], g["dx"] + g["sub_dx"] - pr.shift[1])
    valid = (g["flags"] & S.VALID) != 0

    z = p.z
    avg = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in kt.items()}   # ms per launch
    d_ms = avg["describe"]
    px, sen_px = described_px(S, ips, m, r, H, W)
    sfoc_mpix = px / (d_ms * 1e-3) / 1e6 if d_ms > 0 else None
    per_step = {k: kt[k][0] / args.steps for k in kt}
    kernels = kernel_table(kt, args.steps, p, H, W, n, m, r, px)
    for k in kernels:   # measured HBM bytes per launch (counters of this configuration)
        if kernels[k] is not None:
            kernels[k]["traffic"] = stored_traffic(k)
    # the dominant kernel: the largest share of a step's kernel time
    dom = max(("describe", "match"), key=lambda k: per_step[k])
    ke = kernels[dom]
    out = {
        "metric": "matched CPs/s + SFOC Mpixel/s",
        "value": cps_s,
        "unit": "CPs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_with_kernel_events": 1e3 * dt_traced,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"scene: one {H}x{W} seeded multimodal pair (speckled sensed image), {n} IPs on a "
                               f"20x20 grid, template {m}, search +-{r}, N=8 orientations, sigma 1/2/3, float32 "
                               f"descriptors, float64 integral images",
                   "image": [H, W], "ips": n, "template": m, "radius": r, "z": z, "fft_side": 128},
        "sfoc_mpixel_per_s": sfoc_mpix,
        "sfoc_mpixel_per_s_step": px * args.steps / elapsed / 1e6,
        "described_px": {"reference": H * W, "sensed_tiles": sen_px},
        "kernel_ms_per_launch": avg,
        "kernel_ms_per_step": per_step,
        "roofline": {"kernel": dom, "bound": "alu", "achieved": ke["achieved_tflops"],
                     "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s", "frac": ke["frac_valu_peak"],
                     "traffic": stored_traffic(dom),
                     "algorithmic": {"sfoc_flop_per_px": sfoc_flops_per_px(p),
                                     "fastncc_flop_per_ip": fastncc_flops_per_ip(m + 2 * r, z, 2 * r + 1),
                                     "units_per_launch": px if dom == "describe" else n,
                                     "flop_per_launch": ke["algorithmic_flop"]},
                     "frac_binding_roof": ke["frac_binding_roof"]},
        "kernels": kernels,
        "accuracy": {"valid": int(valid.sum()), "correct_1p5px": int((err[valid] <= 1.5).sum()),
                     "rmse_valid_px": float(np.sqrt(np.mean(err[valid] ** 2))) if valid.any() else None},
        "parity": parity_vs_stored_oracle(S, "scene", R.cps),
    }
    out["integral_standalone"] = run_integral_alone(args, S, torch, p, ref)
    # The step's describe launch covers both images (the reference image's
    # grid tiles and the sensed template tiles); the same kernel on the
    # reference image alone, with the counters of that launch, is reported
    # as the kernel's roofline, and the step's launch beside it.
    d_alone = out["integral_standalone"]["describe_ms_per_call"]
    if dom == "describe" and d_alone > 0:
        fl = sfoc_flops_per_px(p) * H * W
        rf = out["roofline"]
        rf["in_step"] = {"note": "the step's one describe launch: the reference image's grid tiles and the "
                                 "sensed image's template tiles",
                         "ms_per_launch": d_ms, "achieved": rf["achieved"], "frac": rf["frac"]}
        rf.update({"launch": f"the {H}x{W} reference image's describe, timed with HIP events on its stream "
                             f"with nothing beside it (the same kernel and tiles as in the step)",
                   "ms_per_launch": d_alone, "achieved": fl / (d_alone * 1e-3) / 1e12,
                   "frac": fl / (d_alone * 1e-3) / PEAK_FP32_VALU,
                   "frac_binding_roof": fl / (d_alone * 1e-3) / PEAK_FP32_VALU,
                   "traffic": stored_traffic("describe_reference")})
        rf["algorithmic"] = dict(rf["algorithmic"], units_per_launch=H * W, flop_per_launch=fl)
    if args.ransac:
        out["ransac"] = run_ransac(args, S, synth, torch, p, dev)
    if args.rectify:
        out["rectify"] = run_rectify(args, S, torch, dev)
    if args.fast:
        out["fast"] = run_fast(args, S, synth, torch, dev)
    if args.sweep_pairs > 0:
        out["noise_sweep"] = run_sweep(args, S, torch)
    if args.learned_pairs > 0:
        out["learned"] = run_learned(args, S, synth, torch, p, dev, ref, sen, dips, m, r)
    if args.precision:
        out["precision"] = run_precision(args, S, synth, torch, dev, (pr, ips, m, r))
    if args.small_windows:
        out["small_windows"] = run_small_windows(args, S, synth, torch, dev)
    if args.batched_steps > 0:
        del R
        torch.cuda.empty_cache()
        out["batched"] = run_batched(args, S, synth, torch, p, dev)
    if args.cpu_budget > 0:
        out["cpu_baseline"] = cpu_baseline(pr, ips, m, r, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
