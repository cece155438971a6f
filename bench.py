#!/usr/bin/env python3
"""Throughput of the batched HEALPix SHT: IQU map triples per second through
alm2map + map2alm (one step = both directions over the whole batch).

Default workload: nside 512, lmax 1535, 1000 IQU map triples with Gaussian
random a_lm (C_l^TT = 1/(l+1)^2, C^EE = 0.1 C^TT, C^BB = 0.01 C^TT, TE correlation
0.5), inputs resident in HBM before timing.  FP64 is the headline `value`; the
mixed-precision contractions are reported beside it on the same GPU.

Prints one JSON line.  Only N = 1 GPU is supported (the build targets one GPU).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

# Request buffers of the serving leg come and go in sizes from kilobytes to tens of
# gigabytes; growable segments keep torch's cache from splitting HBM into pieces
# too small for the next large request (set before torch is imported).
os.environ.setdefault("PYTORCH_ALLOC_CONF", "expandable_segments:True")

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "IQU maps/s (alm2map+map2alm) nside 512, FP64 vs mixed; serve p50/p99 ms"
# split BF16 forms each product from six bf16 MFMA products, so its peak in
# products is a sixth of the BF16 matrix peak
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0 / 6.0}
PEAK_HBM_GBS = 8000.0


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def compact_scale(lmax: int):
    """sqrt of the per-entry variance of a unit-C_l Gaussian field in the compact
    (lmax+1)^2 storage: 1 for Re at m = 0, 1/2 for Re and Im at m > 0; and the l
    of every entry."""
    import torch
    L1 = lmax + 1
    idx = torch.arange(L1 * L1, dtype=torch.int64)
    col, row = idx // L1, idx % L1
    is_re = row >= col
    l = torch.where(is_re, row, row + L1 - col)
    m = torch.where(is_re, col, L1 - col)
    cl = 1.0 / (l.double() + 1.0) ** 2
    cl[l < 2] = 0.0
    return torch.sqrt(cl) * torch.where(m == 0, 1.0, math.sqrt(0.5)).double()


def fill_alm(alm, lmax: int, seed: int, block: int = 25) -> None:
    """Seeded Gaussian IQU a_lm written block by block on the device."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    s = compact_scale(lmax).to("cuda")
    n = alm.shape[0]
    rho = 0.5
    for k0 in range(0, n, block):
        k1 = min(n, k0 + block)
        z = torch.randn((k1 - k0, 3, s.numel()), generator=g, device="cuda", dtype=torch.float64)
        alm[k0:k1, 0] = s * z[:, 0]
        alm[k0:k1, 1] = math.sqrt(0.1) * s * (rho * z[:, 0] + math.sqrt(1 - rho * rho) * z[:, 1])
        alm[k0:k1, 2] = math.sqrt(0.01) * s * z[:, 2]
        del z


def leg_flops(nside: int, lmax: int, spin: int, nmaps: int) -> float:
    """Algorithmic flops of one direction of the Legendre contraction for nmaps map
    sets, with the two hemispheres folded (north rings incl. the equator, rn =
    2 nside): spin 0: 4 rn sum_m (L+1-m); spin 2 (E/B or Q/U): 16 rn sum_m (L+1-max(m,2))."""
    rn = 2 * nside
    if spin == 0:
        rows = sum(lmax + 1 - m for m in range(lmax + 1))
        return 4.0 * rn * rows * nmaps
    rows = sum(lmax + 1 - max(m, 2) for m in range(lmax + 1))
    return 16.0 * rn * rows * nmaps


def paper_form_flops(nside: int, lmax: int) -> float:
    """The paper-form count per IQU triple and direction (all rings, 4 real products
    for Q/U): 5 * 2 R (L+1)(L+2), R = 4 nside - 1."""
    return 5 * 2.0 * (4 * nside - 1) * (lmax + 1) * (lmax + 2)


def cl_index(lmax: int, device):
    """l and weight of every entry of the compact (lmax+1)^2 storage: entry (row i,
    col j) holds Re a_{i,j} (i >= j, weight 1 for m = 0, else 2) or Im a_{l,m} with
    m = lmax+1-j, l = i+m (i < j, weight 2), so C_l = sum w a^2 / (2l+1)."""
    import torch
    n = lmax + 1
    i = torch.arange(n, device=device).repeat(n)          # row (fast index, column-major)
    j = torch.arange(n, device=device).repeat_interleave(n)
    re = i >= j
    ell = torch.where(re, i, i + n - j)
    w = torch.where(re & (j == 0), 1.0, 2.0).to(torch.float64)
    return ell, w


def accuracy(sht, args, prec, alm, maps, alm_out, ref):
    """Mixed-precision error statistics on the first IQU triple against the FP64
    results of the same inputs (the paper gives no mixed-precision bar beyond what
    is reported here): relative RMS of the synthesised maps and of the analysed
    a_lm (worst component), the largest relative error of the power spectrum
    C_l (l >= 2) of the analysed a_lm, and the round-trip residual
    |m - Y A m| / |m| of this precision."""
    import torch
    L = args.lmax
    ell, w = cl_index(L, alm.device)

    def cl(a):
        c = torch.zeros((3, L + 1), dtype=torch.float64, device=a.device)
        c.index_add_(1, ell, w * a * a)
        return c / (2 * torch.arange(L + 1, device=a.device, dtype=torch.float64) + 1)

    def rel(x, y):
        return float(((x - y).norm(dim=-1) / y.norm(dim=-1)).max().item())

    out = {"maps_rel_rms": rel(maps[0], ref["maps"]), "alm_rel_rms": rel(alm_out[0], ref["alm"])}
    c, c0 = cl(alm_out[0]), cl(ref["alm"])
    out["cl_max_rel_err"] = float(((c - c0).abs() / c0)[:, 2:].max().item())
    p = sht.Plan(args.nside, L, 2, 1, precision=prec)
    rt = torch.empty_like(maps[:1])
    p.alm2map(alm_out[:1], rt)
    p.sync()
    p.close()
    out["roundtrip_residual"] = rel(rt[0], maps[0])
    return {k: float(f"{v:.3e}") for k, v in out.items()}


def run_precision(sht, args, prec, alm, maps, alm_out):
    import torch
    nside, lmax, n = args.nside, args.lmax, args.nmaps
    t0 = time.perf_counter()
    p = sht.Plan(nside, lmax, 2, n, precision=prec, chunk=args.chunk)
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t0
    log(f"{prec}: plan {init_s:.2f}s, workspace {p.workspace_bytes() / 1e9:.1f} GB, tables {p.table_bytes() / 1e9:.2f} GB")
    stream = torch.cuda.current_stream()
    for w in range(args.warmup):
        p.alm2map(alm, maps, stream)
        p.map2alm(maps, alm_out, stream)
        torch.cuda.synchronize()
        log(f"{prec}: warmup {w + 1}/{args.warmup} done")
    p.set_profiling(True)
    p.profile(reset=True)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    evs[0].record(stream)
    for k in range(args.steps):
        p.alm2map(alm, maps, stream)
        p.map2alm(maps, alm_out, stream)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = evs[0].elapsed_time(evs[-1])
    per = sorted(evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps))
    prof = p.profile(reset=True)
    p.set_profiling(False)
    rows = p.ring_rows()
    p.close()
    del p
    per_step = ms / args.steps
    log(f"{prec}: {per_step:.1f} ms/step ({wall:.2f}s wall for {args.steps} steps)")
    return {"ms_per_step": per_step, "value": n * 1000.0 / per_step, "init_s": init_s, "stages": prof,
            "ring_rows": rows, "step_ms": {"median": per[len(per) // 2], "min": per[0], "max": per[-1]}}


def eb_leg(sht, args, precs, alm, maps, alm_out):
    """Separate E / B transforms and pixel-domain E/B separation on the first
    `--eb-nmaps` triples of the resident workload: eb_split throughput per
    precision, and the spin-2 contraction time of E-only against E and B
    (one profiled call each of alm2map_sel and map2alm_sel)."""
    import torch
    ne = min(args.eb_nmaps, args.nmaps)
    x, a = maps[:ne], alm_out[:ne]
    me, mb = torch.empty_like(x), torch.empty_like(x)
    stream = torch.cuda.current_stream()
    out = {"map_triples": ne, "chunk": args.chunk}
    for prec in precs:
        p = sht.Plan(args.nside, args.lmax, 2, ne, precision=prec, chunk=args.chunk)
        p.eb_split(x, a, me, mb, stream)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(args.steps):
            p.eb_split(x, a, me, mb, stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        p.set_profiling(True)
        half = {}
        for name, fn, src, dst, stage in (("alm2map", p.alm2map_sel, alm[:ne], me, "a2m_spin2"),
                                          ("map2alm", p.map2alm_sel, x, a, "m2a_spin2")):
            t = {}
            for sel in ("EB", "E", "B"):
                p.profile(reset=True)
                fn(sel, src, dst, stream)
                t[sel] = p.profile(reset=True)[stage][0]
            half[name] = {"spin2_contraction_ms": {k: round(v, 2) for k, v in t.items()},
                          "e_only_over_eb": round(t["E"] / t["EB"], 3)}
        p.close()
        out[prec] = {"eb_split_ms": round(ms, 2), "eb_split_triples_per_s": round(ne * 1000.0 / ms, 2), **half}
        log(f"{prec}: eb_split {ms:.1f} ms for {ne} triples; E-only/EB contraction "
            f"{half['alm2map']['e_only_over_eb']} (alm2map), {half['map2alm']['e_only_over_eb']} (map2alm)")
    del me, mb
    return out


# Sources each Legendre kernel family is built from: a committed counter record
# applies only while the family's sources hash to the profiled version.
LEG_COMMON = ["paper_2208_10154_amd/csrc/leg_rec.h", "paper_2208_10154_amd/csrc/leg_common.h",
              "paper_2208_10154_amd/csrc/sht_internal.h"]
LEG_SOURCES = {"fp": ["paper_2208_10154_amd/csrc/k_leg.hip"] + LEG_COMMON,
               "bf": ["paper_2208_10154_amd/csrc/k_leg_bf16.hip"] + LEG_COMMON}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
MFMA_FILE = os.path.join(ROOT, "profiles", "mfma.json")


def leg_family(kernel: str) -> str:
    return "bf" if "_bf" in kernel else "fp"


def leg_source_hash(family: str = "fp") -> str:
    import hashlib
    h = hashlib.sha256()
    for f in LEG_SOURCES[family]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_record(path: str, kernel: str, nside: int, lmax: int, per_launch_maps: int):
    """The committed counter record of `kernel`, if it was taken on the kernel's
    current sources at this workload (else None)."""
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    e = rec.get(kernel)
    if not e or e.get("source_hash") != leg_source_hash(leg_family(kernel)):
        return None
    if (e.get("nside"), e.get("lmax"), e.get("maps_per_launch")) != (nside, lmax, per_launch_maps):
        return None
    return e


def measured_traffic(kernel: str, nside: int, lmax: int, per_launch_maps: int):
    """HBM bytes per launch of `kernel` from the committed counter summary."""
    e = counter_record(TRAFFIC_FILE, kernel, nside, lmax, per_launch_maps)
    return e.get("bytes_per_launch") if e else None


def roofline(args, prec, res):
    """Dominant Legendre kernel's achieved FLOP rate from the live stage timings.

    `achieved` counts the folded work (both hemispheres folded, every ring): an
    effective rate, since the kernels skip the ring chunks where the Legendre
    values are negligible.  `executed` divides the MFMA instructions the kernel
    actually issues per launch (committed counter record, current sources only)
    by the same live time, which is the occupancy of the matrix pipe."""
    st = res["stages"]
    cand = {k: v for k, v in st.items() if k.startswith(("m2a", "a2m")) and v[1] > 0}
    name = max(cand, key=lambda k: cand[k][0])
    ms, launches = cand[name]
    spin = 0 if name.endswith("spin0") else 2
    flops_per_step = leg_flops(args.nside, args.lmax, spin, args.nmaps)
    achieved = flops_per_step * args.steps / (ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec]
    kname = "k_" + name + {"fp64": "<double>", "fp32": "<float>", "bf16x3": "_bf"}[prec]
    out = {
        "kernel": kname,
        "bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
        "frac": round(achieved / peak, 4),
        "traffic": measured_traffic(kname, args.nside, args.lmax, args.chunk),
        "launches": launches, "avg_launch_ms": round(ms / launches, 3),
        "flops_per_launch": flops_per_step * args.steps / launches,
        "achieved_counts": "folded flops (all rings of a hemisphere) per launch / live launch time",
    }
    e = counter_record(MFMA_FILE, kname, args.nside, args.lmax, args.chunk)
    if e and args.nmaps % args.chunk == 0:
        ex = e["mfma_insts_per_launch"] * e["flops_per_inst"] / (ms / launches * 1e-3) / 1e12
        out["executed"] = {"flops_per_launch": e["mfma_insts_per_launch"] * e["flops_per_inst"],
                           "achieved": round(ex, 2), "frac": round(ex / peak, 4),
                           "mfma_busy_profiled": e["mfma_busy"], "source": e["summary"]}
    return out


def layout_rate(args, prec, res):
    """Coefficient layout stage (compact a_lm <-> m-major rows, both directions):
    algorithmic HBM bytes (the compact FP64 side and the operand rows, each
    moved once) over its measured time."""
    es = 8 if prec == "fp64" else 4
    L, n = args.lmax, args.nmaps
    c = min(args.chunk, n)
    ldx = 64 if c <= 32 else 2 * ((c + 63) // 64 * 64)
    rows0 = (L + 1) * (L + 2) // 2
    rows2 = sum(L + 1 - max(m, 2) for m in range(L + 1))
    per_dir = 8 * (L + 1) ** 2 * 3 * n + (rows0 + 2 * rows2) * ldx * es * (n // c)
    tot = 2 * per_dir * args.steps
    ms, k = res["stages"]["alm_layout"]
    if not k:
        return None
    gbs = tot / (ms * 1e-3) / 1e9
    return {"GB/s": round(gbs, 1), "frac_hbm": round(gbs / PEAK_HBM_GBS, 3),
            "bytes_per_step": per_dir * 2,
            "counters": "profiles/k_layout_nside512_x125_hbm_counters.md"}


def fft_rate(args, prec, res):
    """Ring-FFT stages: algorithmic HBM bytes (maps in/out + the (m, ring) rows
    of ring coefficients the mapping writes/reads once, `ring_rows` of them per
    component map after the ring cut) over their measured time."""
    es = 8 if prec == "fp64" else 4
    npix = 12 * args.nside ** 2
    per_map = 8 * npix + 2 * es * res["ring_rows"]
    tot = 3 * args.nmaps * per_map * args.steps
    out = {"ring_rows": res["ring_rows"], "ring_rows_uncut": (4 * args.nside - 1) * (args.lmax + 1)}
    for k in ("fft_fwd", "fft_inv"):
        ms, n = res["stages"][k]
        if n:
            out[k] = {"GB/s": round(tot / (ms * 1e-3) / 1e9, 1), "frac_hbm": round(tot / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 3)}
    return out


def cpu_baseline(args):
    """The oracle on a bounded stratified sample of the same workload: one IQU
    triple, every `stride`-th ring (alm2map) and every `stride`-th m (map2alm)."""
    import numpy as np
    import oracle
    from paper_2208_10154_amd import synth
    stride = args.cpu_stride
    a = synth.gaussian_alm(args.lmax, 1, True, workload=3)[0]
    m = synth.white_maps(12 * args.nside ** 2, 1, 3, workload=3)[0]
    t_a2m, t_m2a = oracle.timing_sample_iqu(args.nside, args.lmax, a, m, stride)
    sec_per_triple = stride * (t_a2m + t_m2a)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), model)
    except OSError:
        pass
    return {"value": round(1.0 / sec_per_triple, 6), "unit": "IQU map triples/s", "cores": oracle.num_threads(),
            "cpu_model": model, "nproc": os.cpu_count(),
            "kind": "oracle",
            "sample": (f"1 IQU triple at nside {args.nside}, lmax {args.lmax}: alm2map on every {stride}th ring, "
                       f"map2alm on every {stride}th m ({t_a2m + t_m2a:.1f} s measured), scaled by {stride}"),
            "seconds_per_triple": round(sec_per_triple, 1)}


def iteration_leg(args):
    """Config 4: map2alm_iter with N_iter = 3 on nside 1024, lmax 2047, 200 IQU
    triples (Gaussian a_lm synthesised in FP64 plus white noise at 1e-2 of each
    map's RMS), contraction in each requested precision, residual in FP64.  Reports
    seconds per run at N_iter 0, 3 and 9 with the fit of t0 + (2 N_iter + 1) t1,
    the per-iteration cost, triples/s and the RMS residual after every iteration."""
    import torch
    from paper_2208_10154_amd import sht
    nside, n, niter = args.iter_nside, args.iter_nmaps, 3
    L = 2 * nside - 1
    t0 = time.perf_counter()
    p = sht.Plan(nside, L, 2, n, chunk=args.iter_chunk)
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t0
    alm = torch.empty((n, 3, (L + 1) ** 2), dtype=torch.float64, device="cuda")
    fill_alm(alm, L, seed=220810154 + 4)
    maps = torch.empty((n, 3, 12 * nside * nside), dtype=torch.float64, device="cuda")
    p.alm2map(alm, maps)
    g = torch.Generator(device="cuda")
    g.manual_seed(4)
    maps += 1e-2 * maps.std(dim=2, keepdim=True) * torch.randn(maps.shape, generator=g, dtype=torch.float64,
                                                                device="cuda")
    out = torch.empty_like(alm)
    torch.cuda.synchronize()
    log(f"iteration: nside {nside} lmax {L} {n} IQU triples, plan {init_s:.1f}s, inputs ready")
    res = {}
    stream = torch.cuda.current_stream()
    for prec in args.iter_precisions.split(","):
        p.set_precision(prec)
        p.map2alm_iter(maps, out, 0)  # warm-up (work lists, iteration buffers)
        torch.cuda.synchronize()
        times, resid = {}, {}
        for k in (0, 9, niter):  # the N_iter = 3 run last, so `out` holds its result
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            resid[k] = p.map2alm_iter(maps, out, k, residuals=True)
            e1.record(stream)
            torch.cuda.synchronize()
            times[k] = e0.elapsed_time(e1) / 1e3
        err = float(((out - alm).norm() / alm.norm()).item())
        # the paper's cost model t = t0 + (2 N_iter + 1) t1 (Appendix B), least squares over N_iter 0, 3, 9
        ks = sorted(times)
        xs = [2 * k + 1 for k in ks]
        xm, ym = sum(xs) / 3, sum(times[k] for k in ks) / 3
        t1 = sum((x - xm) * (times[k] - ym) for x, k in zip(xs, ks)) / sum((x - xm) ** 2 for x in xs)
        t0 = ym - t1 * xm
        res[prec] = {"s_niter0": round(times[0], 3), f"s_niter{niter}": round(times[niter], 3),
                     "s_niter9": round(times[9], 3),
                     "s_per_iteration": round((times[niter] - times[0]) / niter, 3),
                     "fit_t0_s": round(t0, 4), "fit_t1_s": round(t1, 4),
                     "triples_per_s": round(n / times[niter], 2),
                     "residual_rms": [float(f"{x:.6e}") for x in resid[niter]],
                     "residual_rms_niter9": [float(f"{x:.6e}") for x in resid[9]],
                     "rel_err_vs_input_alm": float(f"{err:.4e}")}
        log(f"iteration {prec}: {res[prec]}")
    p.close()
    del alm, maps, out
    torch.cuda.empty_cache()
    return {"workload": f"healpix_iqu_nside{nside}_lmax{L}_x{n}_map2alm_iter{niter}", "plan_init_s": round(init_s, 2),
            "chunk": args.iter_chunk, "noise": "white, 1e-2 of each map's RMS", "by_precision": res}


def spin0_leg(args):
    """Spin-0 workload: nside 128, lmax 383, 1000 T maps, FP64 (Gaussian a_lm with
    C_l = 1/(l+1)^2, seeded on the device), alm2map + map2alm per step, the whole
    batch resident in HBM.  Reports T maps/s and the stage times."""
    import torch
    from paper_2208_10154_amd import sht
    nside, L, n = 128, 383, 1000
    p = sht.Plan(nside, L, 0, n)
    g = torch.Generator(device="cuda")
    g.manual_seed(220810154 + 2)
    alm = compact_scale(L).to("cuda") * torch.randn((n, 1, (L + 1) ** 2), generator=g, device="cuda",
                                                     dtype=torch.float64)
    maps = torch.empty((n, 1, 12 * nside * nside), dtype=torch.float64, device="cuda")
    out = torch.empty_like(alm)
    stream = torch.cuda.current_stream()
    for _ in range(max(1, args.warmup)):
        p.alm2map(alm, maps, stream)
        p.map2alm(maps, out, stream)
    torch.cuda.synchronize()
    p.set_profiling(True)
    p.profile(reset=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        p.alm2map(alm, maps, stream)
        p.map2alm(maps, out, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    prof = p.profile(reset=True)
    p.close()
    del alm, maps, out
    torch.cuda.empty_cache()
    res = {"workload": f"healpix_t_nside{nside}_lmax{L}_x{n}", "dtype": "f64", "ms_per_step": round(ms, 3),
           "t_maps_per_s": round(n * 1000.0 / ms, 1),
           "stages_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in prof.items() if v[1]}}
    log(f"spin 0 nside {nside}: {res}")
    return res


def immediate_leg(args):
    """Immediate iteration (Sec. 4, Algorithm 3) against the traditional one on the
    comparison of Fig. 3: maps band limited to lmax = 3 nside - 1 (Gaussian a_lm
    synthesised in FP64, no noise), nside 512, lmax 1535, `--imm-nmaps` IQU
    triples in one chunk, N_iter = 3.  Reports seconds per run, the RMS residual
    after every round and the relative error against the input a_lm for both
    modes, and the immediate run's stage times."""
    import torch
    from paper_2208_10154_amd import sht
    nside, n, niter = args.nside, args.imm_nmaps, 3
    L = 3 * nside - 1
    p = sht.Plan(nside, L, 2, n, chunk=n)
    alm = torch.empty((n, 3, (L + 1) ** 2), dtype=torch.float64, device="cuda")
    fill_alm(alm, L, seed=220810154 + 6)
    maps = torch.empty((n, 3, 12 * nside * nside), dtype=torch.float64, device="cuda")
    p.alm2map(alm, maps)
    out = torch.empty_like(alm)
    stream = torch.cuda.current_stream()
    res = {}
    for prec in args.imm_precisions.split(","):
        p.set_precision(prec)
        p.map2alm_immediate(maps, out, 1)  # warm-up (schedule, work lists, iteration buffers)
        torch.cuda.synchronize()
        r = {}
        for mode, fn in (("traditional", p.map2alm_iter), ("immediate", p.map2alm_immediate)):
            p.set_profiling(mode == "immediate")
            p.profile(reset=True)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            rr = fn(maps, out, niter, residuals=True)
            e1.record(stream)
            torch.cuda.synchronize()
            prof = p.profile(reset=True)
            p.set_profiling(False)
            err = float(((out - alm).norm() / alm.norm()).item())
            r[mode] = {"s": round(e0.elapsed_time(e1) / 1e3, 3), "residual_rms": [float(f"{x:.6e}") for x in rr],
                       "rel_err_vs_input_alm": float(f"{err:.4e}")}
            if mode == "immediate":
                r[mode]["stages_ms"] = {k: round(v[0], 2) for k, v in prof.items() if v[1]}
                r[mode]["stage_records"] = int(sum(v[1] for v in prof.values()))
        r["residual_ratio_immediate_over_traditional"] = round(r["immediate"]["residual_rms"][-1] /
                                                               r["traditional"]["residual_rms"][-1], 4)
        res[prec] = r
        log(f"immediate {prec}: {r}")
    p.close()
    del alm, maps, out
    torch.cuda.empty_cache()
    return {"workload": f"healpix_iqu_nside{nside}_lmax{L}_x{n}_bandlimited_iter{niter}", "by_precision": res}


def small_batch_leg(args):
    """Small batches (the BLAS2 regime): latency of alm2map + map2alm of 1, 8 and
    9 IQU triples at nside 512 / lmax 1535 and nside 1024 / lmax 2047, FP64 and
    split BF16, inputs resident in HBM, median over repetitions.  Up to 8 map sets
    run the narrow Legendre tiles; 9 run the 64-column tile (32 map sets wide)."""
    import torch
    from paper_2208_10154_amd import sht
    out = {}
    stream = torch.cuda.current_stream()
    for nside, L in ((512, 1535), (1024, 2047)):
        p = sht.Plan(nside, L, 2, 9)
        alm = torch.empty((9, 3, (L + 1) ** 2), dtype=torch.float64, device="cuda")
        fill_alm(alm, L, seed=220810154 + 8, block=9)
        maps = torch.empty((9, 3, 12 * nside * nside), dtype=torch.float64, device="cuda")
        back = torch.empty_like(alm)
        res = {}
        for prec in ("fp64", "bf16x3"):
            p.set_precision(prec)
            for n in (1, 8, 9):
                p.set_nmaps(n)
                p.alm2map(alm[:n], maps[:n], stream)
                p.map2alm(maps[:n], back[:n], stream)
                torch.cuda.synchronize()
                ts = []
                for _ in range(max(3, args.steps)):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    p.alm2map(alm[:n], maps[:n], stream)
                    p.map2alm(maps[:n], back[:n], stream)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    ts.append(e0.elapsed_time(e1))
                ms = sorted(ts)[len(ts) // 2]
                res[f"{prec}_x{n}"] = {"ms": round(ms, 3), "triples_per_s": round(n * 1000.0 / ms, 1)}
        p.close()
        del alm, maps, back
        torch.cuda.empty_cache()
        out[f"nside{nside}_lmax{L}"] = res
        log(f"small batches nside {nside}: {res}")
    return out


def part_leg(args):
    """One GPU's share of the split by m at the resolution beyond one GPU's memory
    (Sec. 5): a plan owning part 0 of 8 of the orders m at nside 2048 / lmax 6143,
    IQU, FP64, `--part-nmaps` map sets: Legendre (K_LEG) and ring-FFT time per
    call, from the library's stage timers.  The exchange between the ring and m
    layouts that would join the parts across GPUs is not part of this build."""
    import torch
    from paper_2208_10154_amd import sht
    nside, L, nparts, n = 2048, 6143, 8, args.part_nmaps
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    p = sht.Plan(nside, L, 2, n, part=0, nparts=nparts)
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t0
    alm = torch.empty((n, 3, (L + 1) ** 2), dtype=torch.float64, device="cuda")
    fill_alm(alm, L, seed=220810154 + 9, block=max(1, n))
    maps = torch.empty((n, 3, 12 * nside * nside), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    p.alm2map(alm, maps, stream)
    p.map2alm(maps, alm, stream)
    torch.cuda.synchronize()
    p.set_profiling(True)
    p.profile(reset=True)
    reps = max(1, min(3, args.steps))
    for _ in range(reps):
        p.alm2map(alm, maps, stream)
        p.map2alm(maps, alm, stream)
    prof = p.profile(reset=True)
    out = {"workload": f"healpix_iqu_nside{nside}_lmax{L}_x{n}_mpart0of{nparts}", "dtype": "f64",
           "owned_m": len(sht.part_orders(L, 0, nparts)), "plan_init_s": round(init_s, 2),
           "table_gb": round(p.table_bytes() / 1e9, 2), "workspace_gb": round(p.workspace_bytes() / 1e9, 2),
           "ms_per_call": {k: round(v[0] / reps, 3) for k, v in prof.items() if v[1]}}
    leg = sum(v for k, v in out["ms_per_call"].items() if k.startswith(("m2a", "a2m")))
    out["k_leg_ms_per_call_pair"] = round(leg, 3)
    p.close()
    del alm, maps
    torch.cuda.empty_cache()
    log(f"m part: {out}")
    return out


def serving(args):
    """Config 5: a seeded mix of requests (nside 64..1024, lmax = 3 nside - 1, T or
    IQU, both directions, FP64 or the mixed precision, log-normal map counts with
    median 16 capped at 512 map sets, no other cap) through the batching server:
    a saturated pass (all requests at once) gives the capacity, a Poisson pass at
    80% of it gives p50/p99 latency, and the baseline serves the same Poisson
    arrivals in FP64 one request at a time, first come first served, on one
    stream.  The callers hold at most --serve-live-gb of request inputs and outputs
    in HBM at a time: a request that would exceed it is created once earlier ones
    finish (its latency still counts from its arrival), later requests that fit go
    ahead of it until it has waited 2 s (independent callers, no starvation).
    Plan creation happens in a warm-up pass, timed separately."""
    import torch
    from paper_2208_10154_amd import serve
    N = args.serve_requests
    base = serve.request_mix(N, rate_hz=1.0, seed=7, mixed=args.serve_mixed)
    live = args.serve_live_gb * 1e9

    def make_io(d):
        nside, spin, n = d["nside"], d["spin"], d["nmaps"]
        L, nc = 3 * nside - 1, (1 if spin == 0 else 3)
        a_shape, m_shape = (n, nc, (L + 1) ** 2), (n, nc, 12 * nside * nside)
        ish, osh = (a_shape, m_shape) if d["direction"] == "alm2map" else (m_shape, a_shape)
        for attempt in (0, 1):
            try:
                inp = torch.randn(ish, dtype=torch.float64, device="cuda")
                out = torch.empty(osh, dtype=torch.float64, device="cuda")
                break
            except torch.OutOfMemoryError:
                # freed request tensors cached by torch in pieces too small for this one
                if attempt:
                    raise
                inp = out = None
                torch.cuda.empty_cache()
        ev = torch.cuda.Event()
        ev.record()
        return inp, out, ev

    def warm_up(srv, precisions):
        t0 = time.perf_counter()
        warm = [dict(arrival=0.0, nside=k[0], spin=k[1], direction=k[2], precision=k[3], nmaps=1)
                for k in sorted({(d["nside"], d["spin"], d["direction"], p) for d in base for p in precisions})]
        serve.replay(srv, warm, make_io)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def rebased(srv, mix, scale):
        now = srv.now()
        return [dict(d, arrival=now + 0.05 + d["arrival"] * scale) for d in mix]

    srv = serve.Server(args.serve_budget_gb * 1e9, max_slots=512, depth=2, slot_bytes_per_plan=args.serve_slot_gb * 1e9,
                       executor=serve.Executor(nstreams=4, graphs=args.serve_graphs))
    init_s = warm_up(srv, sorted({d["precision"] for d in base}))
    log(f"serve: warm-up (plans for {len(srv.plans)} keys) {init_s:.1f}s, {srv.used / 1e9:.1f} GB held")
    def churn(srv, since):
        return {"plans_created": srv.plans_created - since[0], "plans_evicted": srv.plans_evicted - since[1],
                "plan_create_s": round(srv.plan_create_s - since[2], 1)}

    def mark(srv):
        return (srv.plans_created, srv.plans_evicted, srv.plan_create_s)

    m0 = mark(srv)
    sat = serve.replay(srv, rebased(srv, [dict(d, arrival=0.0) for d in base], 0.0), make_io, max_live_bytes=live)
    st_sat = serve.latency_stats(sat)
    st_sat.update(churn(srv, m0))
    cap_req = N / st_sat["makespan_s"]
    rate = 0.8 * cap_req
    log(f"serve: saturated {st_sat}")
    m0 = mark(srv)
    poisson = serve.replay(srv, rebased(srv, base, 1.0 / rate), make_io, max_live_bytes=live)
    st_p = serve.latency_stats(poisson)
    st_p.update(churn(srv, m0))
    log(f"serve: poisson at {rate:.2f} req/s {st_p}")
    peak = srv.peak
    srv.close()
    del srv
    torch.cuda.empty_cache()
    # baseline: the same arrivals, FP64, one request per launch, in arrival order on one stream
    ser = serve.Server(args.serve_budget_gb * 1e9, max_slots=512, depth=1 << 20, batching=False,
                       slot_bytes_per_plan=args.serve_slot_gb * 1e9,
                       executor=serve.Executor(nstreams=1))
    warm_up(ser, ["fp64"])
    m0 = mark(ser)
    serial = serve.replay(ser, rebased(ser, [dict(d, precision="fp64") for d in base], 1.0 / rate), make_io,
                          max_live_bytes=live)
    st_s = serve.latency_stats(serial)
    st_s.update(churn(ser, m0))
    log(f"serve: serial fp64 fifo {st_s}")
    ser.close()
    del ser
    torch.cuda.empty_cache()
    sizes = sorted(d["nmaps"] for d in base)
    out = {"requests": N,
           "mix": f"nside 64-1024 (lmax 3 nside - 1), T/IQU, alm2map/map2alm, fp64/{args.serve_mixed}, "
                  "log-normal map sets (median 16, sigma_ln 1, cap 512), no byte cap",
           "map_sets_median_max": [sizes[len(sizes) // 2], sizes[-1]],
           "largest_request_gb": round(max(serve.request_bytes(d) for d in base) / 1e9, 1),
           "rate_req_per_s": round(rate, 3), "capacity_req_per_s": round(cap_req, 3),
           "p50_ms": st_p["p50_ms"], "p99_ms": st_p["p99_ms"], "maps_per_s": st_p["maps_per_s"],
           "by_nside": st_p["by_nside"],
           "plan_churn": {name: {k: st[k] for k in ("plans_created", "plans_evicted", "plan_create_s")}
                          for name, st in (("saturated", st_sat), ("poisson", st_p), ("serial", st_s))},
           "saturated_maps_per_s": st_sat["maps_per_s"],
           "serial_fp64_fifo": {"maps_per_s": st_s["maps_per_s"], "p50_ms": st_s["p50_ms"], "p99_ms": st_s["p99_ms"],
                                "by_nside": st_s["by_nside"],
                                "arrivals": "the same Poisson arrivals, one request per launch, first come first served"},
           "callers": "independent: at most live_request_gb of request buffers, first fit in arrival order, "
                      "no bypass of a request waiting more than 2 s",
           "graphs": bool(args.serve_graphs), "budget_gb": args.serve_budget_gb, "live_request_gb": args.serve_live_gb,
           "slot_gb_per_plan": args.serve_slot_gb,
           "peak_server_gb": round(peak / 1e9, 1), "init_s": round(init_s, 1)}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nside", type=int, default=512)
    ap.add_argument("--lmax", type=int, default=None)
    ap.add_argument("--nmaps", type=int, default=1000, help="IQU map triples per step")
    ap.add_argument("--chunk", type=int, default=125)
    ap.add_argument("--precisions", default="fp64,fp32,bf16x3")
    ap.add_argument("--cpu-stride", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg (config 5)")
    ap.add_argument("--no-iter", action="store_true", help="skip the iteration leg (config 4)")
    ap.add_argument("--no-eb", action="store_true", help="skip the E/B leg")
    ap.add_argument("--no-imm", action="store_true", help="skip the immediate-iteration leg")
    ap.add_argument("--no-spin0", action="store_true", help="skip the spin-0 nside 128 leg")
    ap.add_argument("--no-small", action="store_true", help="skip the small-batch latency leg")
    ap.add_argument("--no-part", action="store_true", help="skip the nside 2048 m-part leg")
    ap.add_argument("--part-nmaps", type=int, default=2, help="IQU map sets of the m-part leg")
    ap.add_argument("--imm-nmaps", type=int, default=64, help="IQU triples of the immediate-iteration leg")
    ap.add_argument("--imm-precisions", default="fp64,bf16x3")
    ap.add_argument("--eb-nmaps", type=int, default=250, help="IQU triples of the E/B leg")
    ap.add_argument("--iter-nside", type=int, default=1024)
    ap.add_argument("--iter-nmaps", type=int, default=200)
    ap.add_argument("--iter-chunk", type=int, default=64)
    ap.add_argument("--iter-precisions", default="bf16x3,fp32,fp64")
    ap.add_argument("--serve-requests", type=int, default=500)
    ap.add_argument("--serve-budget-gb", type=float, default=185.0, help="HBM the server may hold (plans, slots)")
    ap.add_argument("--serve-live-gb", type=float, default=65.0,
                    help="HBM the emulated callers hold for request inputs and outputs at a time")
    ap.add_argument("--serve-slot-gb", type=float, default=3.0,
                    help="batch slot buffers per plan and direction, GB (bounds the map sets one batched call holds)")
    ap.add_argument("--serve-mixed", default="bf16x3")
    ap.add_argument("--serve-graphs", action="store_true")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="run one plain device copy of this many GiB (counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the split over several GPUs "
              "(map batch or m range per GPU) is not built.", file=sys.stderr)
        sys.exit(2)
    if args.lmax is None:
        args.lmax = 3 * args.nside - 1
    import torch
    from paper_2208_10154_amd import sht
    sht.lib()
    if args.copy_probe_gib > 0:
        nbytes = int(args.copy_probe_gib * 2 ** 30)
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {nbytes} bytes read and written once")
        del src, dst
    n, L = args.nmaps, args.lmax
    log(f"workload nside {args.nside} lmax {L} nmaps {n} (IQU), chunk {args.chunk}")
    alm = torch.empty((n, 3, (L + 1) ** 2), dtype=torch.float64, device="cuda")
    fill_alm(alm, L, seed=220810154)
    maps = torch.empty((n, 3, 12 * args.nside ** 2), dtype=torch.float64, device="cuda")
    alm_out = torch.empty_like(alm)
    torch.cuda.synchronize()
    log(f"inputs resident: {(alm.numel() * 2 + maps.numel()) * 8 / 1e9:.1f} GB")
    results, ref, acc = {}, None, {}
    precs = args.precisions.split(",")
    precs = (["fp64"] if "fp64" in precs else []) + [q for q in precs if q != "fp64"]
    for prec in precs:
        results[prec] = run_precision(sht, args, prec, alm, maps, alm_out)
        if prec == "fp64":
            ref = {"maps": maps[0].clone(), "alm": alm_out[0].clone()}
            acc[prec] = accuracy(sht, args, prec, alm, maps, alm_out, ref)
        elif ref is not None:
            acc[prec] = accuracy(sht, args, prec, alm, maps, alm_out, ref)
        log(f"{prec}: accuracy {acc.get(prec)}")
    head = "fp64" if "fp64" in results else list(results)[0]
    r = results[head]
    line = {
        "metric": METRIC, "value": round(r["value"], 3), "unit": "IQU map triples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64" if head == "fp64" else head,
        "data": "synthetic (seeded Gaussian a_lm, C_l = 1/(l+1)^2 spectra)",
        "config": {"workload": f"healpix_iqu_nside{args.nside}_lmax{L}_x{n}", "nside": args.nside, "lmax": L,
                   "map_triples": n, "spin": 2, "chunk": args.chunk, "step": "alm2map+map2alm"},
        "by_precision": {k: {"value": round(v["value"], 3), "ms_per_step": round(v["ms_per_step"], 3),
                             "plan_init_s": round(v["init_s"], 2),
                             "component_maps_per_s": round(3 * v["value"], 2),
                             "step_ms_median_min_max": [round(v["step_ms"][q], 3) for q in ("median", "min", "max")],
                             "stages_ms_per_step": {s: round(t / args.steps, 3) for s, (t, c) in v["stages"].items() if c},
                             **({"accuracy_vs_fp64": acc[k]} if k in acc else {})}
                         for k, v in results.items()},
        "roofline": roofline(args, head, r),
        "paper_form_tflops_equiv": round(2 * paper_form_flops(args.nside, L) * n / (r["ms_per_step"] * 1e-3) / 1e12, 2),
        "fft_hbm": fft_rate(args, head, r),
        "layout_hbm": layout_rate(args, head, r),
    }
    if "fp64" in results:
        line["mixed_over_fp64"] = {k: round(v["value"] / results["fp64"]["value"], 3) for k, v in results.items() if k != "fp64"}
        for k in results:
            if k != head:
                line["by_precision"][k]["roofline"] = roofline(args, k, results[k])
    if not args.no_eb:
        line["eb"] = eb_leg(sht, args, precs, alm, maps, alm_out)
    del alm, maps, alm_out
    torch.cuda.empty_cache()
    if not args.no_iter:
        line["iteration"] = iteration_leg(args)
    if not args.no_spin0:
        line["spin0"] = spin0_leg(args)
    if not args.no_imm:
        line["immediate"] = immediate_leg(args)
    if not args.no_small:
        line["small_batch"] = small_batch_leg(args)
    if not args.no_part:
        line["m_part"] = part_leg(args)
    if not args.no_serve:
        line["serve"] = serving(args)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample) ...")
        line["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
