"""Benchmark of the short-range P3M pair force on one MI355X.

Workload (default): N = 128^3 clustered particles (Zel'dovich lattice plus
200 NFW-like halos holding 30 % of the particles), PM grid 256^3,
x_s = 1.25 cells, r_cut = 4.5 x_s, unit box, G*m = 1, all particles active.
Inputs are synthetic and seeded (see workloads/).

One step = one full short-range force evaluation through the C ABI: tile
keys, counting sort, receiver compaction, cluster/work-item planning and the
persistent pair kernel, with inputs already resident in HBM.  The headline
value is accepted ordered pair interactions per second of the FP32 path
(FP32 kernel shape, FP64 separations and accumulation); the FP64 path is
timed beside it.  Prints ONE JSON line.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--workload clustered128]
"""
import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_INTERACTION = 40          # forward pair, algorithmic convention
ADJOINT_FLOPS = 60                  # adjoint pair (the VJP of one interaction)
PEAK_FP32_TFLOPS = 157.3            # MI355X FP32 vector (packed) peak
PEAK_FP64_TFLOPS = 78.6             # MI355X FP64 vector peak
PEAK_HBM_TBPS = 8.0                 # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="clustered128")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--ns", type=int, default=0, help="fixed subtiles per tile (0 = autotune)")
    ap.add_argument("--target", type=int, default=0, help="fixed work-item size (0 = autotune)")
    ap.add_argument("--csize", type=int, default=0,
                    help="fixed cluster size 8/16/32/64 (0 = autotune)")
    ap.add_argument("--screen", type=int, default=-1,
                    help="fixed per-supplier box screen 0/1 (-1 = autotune)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 512 MiB device copy (HBM counter calibration)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-tiled", action="store_true",
                    help="skip the oracle's cell-list walk on the full uniform32, diff64 and "
                         "clustered128 sets (about 20 s on 16 host threads)")
    ap.add_argument("--legs", default="adjoint,batched,softened,long_range,kdk,shapes,deterministic,"
                                      "configs",
                    help="extra measured legs beside the forward force: adjoint, batched, "
                         "softened, long_range, kdk, shapes, deterministic; and, not run by "
                         "default, subtiles (fixed subtile counts against the autotuner)")
    ap.add_argument("--batched-workload", default="clustered256")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_steps(torch, ctx, pos, mass, wl, prec, steps, warmup):
    kw = dict(box=wl.box, x_s=wl.x_s, r_cut=wl.r_cut, precision=prec)
    out = torch.empty((wl.n, 3), dtype=torch.float64, device=pos.device)
    ctx.set_timing(False)
    for _ in range(warmup):
        ctx.force(pos, mass, None, out=out, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.force(pos, mass, None, out=out, **kw)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    # per-kernel durations from HIP events on the launch stream, same calls
    ctx.set_timing(True)
    pairs_ms, build_ms, sort_ms = [], [], []
    for _ in range(steps):
        ctx.force(pos, mass, None, out=out, **kw)
        st = ctx.stats()
        pairs_ms.append(st["ms_pairs"])
        build_ms.append(st["ms_build"])
        sort_ms.append(st["ms_sort"])
    ctx.set_timing(False)
    st = ctx.stats()
    st["ms_sort_median"] = statistics.median(sort_ms)
    return out, wall, st, statistics.median(pairs_ms), statistics.median(build_ms)


def time_calls(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def adjoint_leg(torch, ctx, pos, mass, wl, steps, warmup, tune=True):
    """Vector-Jacobian product of the force (60 algorithmic flops per pair),
    in the layout the autotuner picks for the adjoint itself."""
    gen = torch.Generator(device=pos.device).manual_seed(4003)
    w = torch.randn((wl.n, 3), dtype=torch.float64, device=pos.device, generator=gen)
    out = {}
    for prec in ("fp32", "fp64"):
        kw = dict(box=wl.box, x_s=wl.x_s, r_cut=wl.r_cut, precision=prec)
        if tune:
            ctx.autotune(pos, mass, None, level=2, adjoint=True, **kw)
        wall = time_calls(torch, lambda: ctx.force_backward(pos, mass, None, w, **kw),
                          max(2, steps // 4), 1)
        ctx.set_timing(True)
        ctx.force_backward(pos, mass, None, w, **kw)
        st = ctx.stats()
        ctx.set_timing(False)
        out[prec] = {"ms_per_call": wall * 1e3, "pair_kernel_ms": st["ms_pairs"],
                     "interactions": st["interactions"],
                     "value": st["interactions"] / wall,
                     "achieved_tflops": ADJOINT_FLOPS * st["interactions"] / (st["ms_pairs"] * 1e-3) / 1e12,
                     "layout": {k: st[k] for k in ("subtiles_per_dim", "item_target",
                                                   "cluster_size", "screen")}}
        log("adjoint", prec, "%.3f ms" % (wall * 1e3))
    return out


def softened_leg(torch, ctx, pos, mass, wl, steps, warmup):
    """The B-spline softened force (eps = 0.03 L / cbrt(N), eps_B = 2.8 eps) on
    the main workload, with the layouts the autotuner chose."""
    eps = 0.03 / round(wl.n ** (1.0 / 3.0))
    out = {"eps": eps, "eps_b": 2.8 * eps}
    ctx.set_softening(eps)
    try:
        for prec in ("fp32", "fp64"):
            _, wall, st, pairs_ms, _ = time_steps(torch, ctx, pos, mass, wl, prec,
                                                  max(2, steps // 2), warmup)
            out[prec] = {"ms_per_step": wall * 1e3, "pair_kernel_ms": pairs_ms,
                         "interactions": st["interactions"],
                         "value": st["interactions"] / wall,
                         "achieved_tflops": FLOPS_PER_INTERACTION * st["interactions"]
                         / (pairs_ms * 1e-3) / 1e12}
            log("softened", prec, "%.3f ms/step  pairs %.3f ms" % (wall * 1e3, pairs_ms))
    finally:
        ctx.set_softening(0.0)
    return out


def long_range_bytes(n_grid, n_part):
    """Algorithmic HBM bytes of each long-range stage: every grid read or
    written once per pass (real grid 8 B per node, half spectrum 16 B per
    complex value), particles read and written once per stage that uses
    them."""
    cells = n_grid ** 3
    half = (n_grid // 2 + 1) * n_grid * n_grid * 16
    return {
        # positions and masses in, node keys, ranks, histogram; sorted records out
        "sort": n_part * (24 + 8 + 4 + 4) + 2 * 4 * cells + n_part * (32 + 4 + 4 + 1),
        "deposit": 8 * cells + n_part * (32 + 4) + 8 * cells,   # clear, records, grid
        "fft_x_fwd": 8 * cells + half,
        "fft_y_fwd": 2 * half,
        "fft_z_conv": 2 * half,
        "fft_y_inv": 2 * half,
        "fft_x_inv": half + 8 * cells,
        "readout": 8 * cells + n_part * (32 + 4 + 4 + 1 + 24),
    }


def long_range_leg(torch, ctx, pos, mass, wl, steps, warmup, cpu=True):
    """The long-range PM half of the P3M force (p3m_lr_force) on the main
    workload's grid, with per-stage HIP-event times and the HBM roofline of
    the FFT passes; the CPU oracle (numpy FFT) of the same call beside it."""
    kw = dict(box=wl.box, n_grid=wl.n_pm, x_s=wl.x_s)
    out = torch.empty((wl.n, 3), dtype=torch.float64, device=pos.device)
    wall = time_calls(torch, lambda: ctx.force_long_range(pos, mass, None, out=out, **kw),
                      steps, warmup)
    ctx.set_timing(True)
    rows = []
    for _ in range(steps):
        ctx.force_long_range(pos, mass, None, out=out, **kw)
        rows.append(ctx.lr_stats())
    ctx.set_timing(False)
    stages = ("sort", "deposit", "fft_x_fwd", "fft_y_fwd", "fft_z_conv", "fft_y_inv", "fft_x_inv",
              "readout")
    ms = {k: sum(r["ms_" + k] for r in rows) / len(rows) for k in stages}
    nbytes = long_range_bytes(wl.n_pm, wl.n)
    fft = [k for k in stages if k.startswith("fft")]
    fft_ms = sum(ms[k] for k in fft)
    fft_gbs = sum(nbytes[k] for k in fft) / (fft_ms * 1e-3) / 1e9
    res = {"workload": "%s: N=%d, PM grid %d^3, x_s=1.25 cells, CIC, 2 deconvolutions, D4"
                       % (wl.name, wl.n, wl.n_pm),
           "ms_per_call": wall * 1e3,
           "stage_ms": ms,
           "stage_gbs": {k: nbytes[k] / (ms[k] * 1e-3) / 1e9 for k in stages},
           "fft_roofline": {"bound": "hbm", "achieved": fft_gbs, "peak": 8000.0, "unit": "GB/s",
                            "frac": fft_gbs / 8000.0, "bytes": sum(nbytes[k] for k in fft)}}
    log("long range %.3f ms per call, FFT passes %.3f ms at %.0f GB/s"
        % (wall * 1e3, fft_ms, fft_gbs))
    if cpu:
        from oracle import pm_oracle
        t0 = time.perf_counter()
        pm_oracle.pm_force(wl.pos, None if mass is None else wl.mass, wl.box, wl.n_pm, wl.x_s)
        dt = time.perf_counter() - t0
        res["cpu_oracle"] = {"ms_per_call": dt * 1e3, "cores": 1, "kind": "oracle",
                             "sample": "the whole call (numpy FFT, one thread)"}
    return res


def p3m_leg(torch, ctx, pos, mass, wl, steps, warmup):
    """The whole P3M acceleration in one call (p3m_force: FP32 short range
    and PM overlapped on two streams) against the two halves called one
    after the other on one stream."""
    kw = dict(box=wl.box, x_s=wl.x_s, r_cut=wl.r_cut)
    out = torch.empty((wl.n, 3), dtype=torch.float64, device=pos.device)
    lro = torch.empty_like(out)

    def seq():
        ctx.force(pos, mass, None, precision="fp32", out=out, **kw)
        ctx.force_long_range(pos, mass, None, box=wl.box, n_grid=wl.n_pm, x_s=wl.x_s, out=lro)

    both = time_calls(torch, lambda: ctx.force_total(pos, mass, None, n_grid=wl.n_pm,
                                                     precision="fp32", out=out, **kw),
                      steps, warmup)
    one_by_one = time_calls(torch, seq, steps, warmup)
    log("p3m force %.3f ms overlapped, %.3f ms one after the other"
        % (both * 1e3, one_by_one * 1e3))
    return {"ms_per_call": both * 1e3, "ms_sequential": one_by_one * 1e3,
            "interactions_per_s": ctx.stats()["interactions"] / both}


def shapes_leg(torch, ctx, pos, mass, wl, steps, warmup):
    """The tabulated FP32 kernel shapes (the paper's 2^12-entry NGP table on
    r^2 and a 1024-entry linearly interpolated one) against the polynomial,
    on the main workload with the layout the FP32 autotuner chose; their
    force errors are filled in from the CPU oracle sample afterwards."""
    out = {}
    for kind, size in (("poly", 0), ("table_ngp", 4096), ("table_linear", 1024)):
        ctx.set_shape(kind, size)
        try:
            acc, wall, st, pairs_ms, _ = time_steps(torch, ctx, pos, mass, wl, "fp32",
                                                    max(2, steps // 2), warmup)
        finally:
            ctx.set_shape("poly")
        key = kind if not size else "%s_%d" % (kind, size)
        out[key] = {"ms_per_step": wall * 1e3, "pair_kernel_ms": pairs_ms,
                    "achieved_tflops": FLOPS_PER_INTERACTION * st["interactions"]
                    / (pairs_ms * 1e-3) / 1e12, "_acc": acc.cpu().numpy()}
        log("shape", key, "pairs %.3f ms" % pairs_ms)
    return out


def kdk_leg(torch, ctx, pos, mass, wl, repeats=2):
    """One synchronised period (one global step) of the rung-hierarchical KDK
    scheme (p3m_kdk_step) on the main workload from rest: FP32 short range
    with B-spline softening eps = 0.03 L / cbrt(N), PM long range, eta =
    0.025, at most 8 rungs.  dt puts the particle with the median short-range
    acceleration on the boundary of rung 0 (eq. rung), so the halo cores fill
    the upper rungs."""
    eta = 0.025
    eps = 0.03 / round(wl.n ** (1.0 / 3.0))
    kw = dict(box=wl.box, x_s=wl.x_s, r_cut=wl.r_cut)
    ctx.set_softening(eps)
    try:
        acc = ctx.force(pos, mass, None, precision="fp32", **kw)
    finally:
        ctx.set_softening(0.0)
    amag = torch.linalg.norm(acc, dim=1)
    dt = math.sqrt(2.0 * eta * eps / float(amag.median()))
    z = dt * torch.sqrt(amag / (2.0 * eta * eps))
    start = torch.clamp(torch.ceil(torch.log2(torch.clamp(z, min=1e-300))), 0, 7).to(torch.int64)
    res = {"dt": dt, "eps": eps, "eta": eta,
           "start_rungs": torch.bincount(start, minlength=8).tolist()}
    times = []
    for _ in range(repeats):
        p = pos.clone()
        v = torch.zeros_like(pos)
        r = torch.zeros(wl.n, dtype=torch.uint8, device=pos.device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.kdk_step(p, v, mass, r, n_grid=wl.n_pm, dt=dt, n_steps=1, eta=eta, eps=eps,
                     precision="fp32", **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    st = ctx.kdk_stats()
    wall = min(times)
    res.update({"ms_per_period": wall * 1e3, "highest_rung": st["highest_rung"],
                "substeps": st["substeps"], "sr_calls": st["sr_calls"],
                "lr_calls": st["lr_calls"], "interactions": st["interactions"],
                "interactions_per_s": st["interactions"] / wall,
                "end_rungs": torch.bincount(r.to(torch.int64), minlength=8).tolist(),
                "ms_per_substep": wall * 1e3 / st["substeps"]})
    log("kdk period %.1f ms, %d sub-steps, %d short-range calls, %.3g interactions"
        % (wall * 1e3, st["substeps"], st["sr_calls"], st["interactions"]))
    return res


def deterministic_leg(torch, ctx, pos, mass, wl, steps, warmup):
    """The deterministic mode (p3m_sr_set_deterministic) against the default
    atomic mode in the same layout, the one a deterministic FP32 call takes
    (screen 2 cannot run there: after tuning, the fastest other layout):
    time per call, pair-kernel time, and whether two deterministic calls
    agree bit for bit."""
    keys = ("subtiles_per_dim", "item_target", "cluster_size", "screen")
    ctx.set_deterministic(True)
    ctx.force(pos, mass, None, box=wl.box, x_s=wl.x_s, r_cut=wl.r_cut, precision="fp32")
    torch.cuda.synchronize()
    layout = tuple(ctx.stats()[k] for k in keys)
    ctx.set_deterministic(False)
    out = {"layout": dict(zip(keys, layout))}
    ctx.set_config(*layout)
    try:
        for prec in ("fp32", "fp64"):
            res = {}
            for det in (False, True):
                ctx.set_deterministic(det)
                _, wall, st, pairs_ms, build_ms = time_steps(torch, ctx, pos, mass, wl, prec,
                                                             max(2, steps // 2), warmup)
                res["det" if det else "atomic"] = {"ms_per_step": wall * 1e3,
                                                   "pair_kernel_ms": pairs_ms,
                                                   "build_ms": build_ms}
            kw = dict(box=wl.box, x_s=wl.x_s, r_cut=wl.r_cut, precision=prec)
            a = ctx.force(pos, mass, None, **kw).cpu().numpy()
            b = ctx.force(pos, mass, None, **kw).cpu().numpy()
            res["bitwise_repeat"] = a.tobytes() == b.tobytes()
            ctx.set_deterministic(False)
            out[prec] = res
            log("deterministic", prec, res)
    finally:
        ctx.set_deterministic(False)
        ctx.set_config()
    return out


def subtiles_leg(torch, p3):
    """Fixed subtiles per tile dimension (1..4; items of 4096, 32-receiver
    clusters, screen 1, and screen 2 for the forward and the adjoint) against the
    autotuner's choice (section 2.1.3, "Subtiles"; the paper's subtile
    experiment), on the diff64 set (forward and adjoint) and the rung-batched
    clustered256 launch, FP32 and FP64.  Pair-kernel ms (HIP events, median)."""
    from workloads import make_workload
    dev = torch.device("cuda", 0)
    rows = []
    for name in ("diff64", "clustered256"):
        log("subtiles: generating", name)
        wl = make_workload(name, with_rungs=(name == "clustered256"))
        pos = torch.from_numpy(wl.pos).to(dev)
        ctx = p3.Context(0)
        if name == "clustered256":
            rung = torch.from_numpy(wl.rung).to(dev)
            thr = list(range(8))
            out = torch.empty((8, wl.n, 3), dtype=torch.float64, device=dev)
            calls = [("batched", prec) for prec in ("fp32", "fp64")]
        else:
            gen = torch.Generator(device=dev).manual_seed(4003)
            w = torch.randn((wl.n, 3), dtype=torch.float64, device=dev, generator=gen)
            out = torch.empty((wl.n, 3), dtype=torch.float64, device=dev)
            calls = [(k, prec) for k in ("forward", "adjoint") for prec in ("fp32", "fp64")]
        for kind, prec in calls:
            kw = dict(box=wl.box, x_s=wl.x_s, r_cut=wl.r_cut, precision=prec)
            if kind == "batched":
                fn, reps = (lambda: ctx.force_batched(pos, None, rung, thr, out=out, **kw)), 3
            elif kind == "forward":
                fn, reps = (lambda: ctx.force(pos, None, None, out=out, **kw)), 7
            else:
                fn, reps = (lambda: ctx.force_backward(pos, None, None, w, **kw)), 7

            def timed():
                fn()
                ctx.set_timing(True)
                ms = []
                for _ in range(reps):
                    fn()
                    ms.append(ctx.stats()["ms_pairs"])
                ctx.set_timing(False)
                st = ctx.stats()
                return statistics.median(ms), st

            for screen in ([1, 2] if kind in ("forward", "adjoint") else [1]):
                for ns in (1, 2, 3, 4):
                    ctx.set_config(ns, 4096, 32, screen)
                    ms, st = timed()
                    rows.append({"workload": name, "call": kind, "precision": prec, "ns": ns,
                                 "screen": screen, "pair_kernel_ms": ms})
                    log("subtiles", rows[-1])
            ctx.set_config()
            t0 = time.perf_counter()
            if kind == "batched":
                ctx.autotune_batched(pos, None, rung, thr, out=out, **kw)
            else:
                ctx.autotune(pos, None, None, level=2, adjoint=(kind == "adjoint"), **kw)
            tune_s = time.perf_counter() - t0
            ms, st = timed()
            rows.append({"workload": name, "call": kind, "precision": prec, "tuned": True,
                         "ns": st["subtiles_per_dim"], "item_target": st["item_target"],
                         "cluster_size": st["cluster_size"], "screen": st["screen"],
                         "pair_kernel_ms": ms, "tune_s": tune_s})
            log("subtiles", rows[-1])
        ctx.close()
        del pos, out
        torch.cuda.empty_cache()
    return rows


def batched_leg(torch, p3, name, steps, warmup, layouts=None, tune=True):
    """All 8 nested rung subsets (rung >= k, k = 0..7) in one persistent launch,
    in the layout the autotuner picks for this batched call on its own
    subsets (p3m_sr_autotune_batched), or in fixed `layouts` (precision ->
    (subtiles, item target, cluster size, screen)) when tuning is off."""
    from workloads import make_workload
    log("generating", name, "with rungs")
    wl = make_workload(name)
    dev = torch.device("cuda", 0)
    pos = torch.from_numpy(wl.pos).to(dev)
    mass = None if bool((wl.mass == 1.0).all()) else torch.from_numpy(wl.mass).to(dev)
    rung = torch.from_numpy(wl.rung).to(dev)
    ctx = p3.Context(0)
    thr = list(range(8))
    out = torch.empty((8, wl.n, 3), dtype=torch.float64, device=dev)
    res = {"workload": "%s: N=%d clustered, PM grid %d^3, k-NN density rungs 0-7, 8 nested "
                       "subsets rung>=k in one launch" % (name, wl.n, wl.n_pm),
           "subset_sizes": [int((wl.rung >= k).sum()) for k in thr]}
    for prec in ("fp32", "fp64"):
        kw = dict(box=wl.box, x_s=wl.x_s, r_cut=wl.r_cut, precision=prec)
        tune_s = 0.0
        if tune:
            t0 = time.perf_counter()
            ctx.autotune_batched(pos, mass, rung, thr, out=out, **kw)
            tune_s = time.perf_counter() - t0
            log("batched", prec, "tuned in %.1f s" % tune_s, ctx.tune_status())
        elif layouts and prec in layouts:
            ctx.set_config(*layouts[prec])
        wall = time_calls(torch, lambda: ctx.force_batched(pos, mass, rung, thr, out=out, **kw),
                          max(2, steps // 5), 1)
        ctx.set_timing(True)
        ctx.force_batched(pos, mass, rung, thr, out=out, **kw)
        st = ctx.stats()
        ctx.set_timing(False)
        if prec == "fp32":
            # interactions of each subset (untimed single calls): rung k
            # particles are kicked 2^k times per step of the rung hierarchy,
            # so a step needs sum_i 2^rung_i n_nb(i) = sum_k 2^k (I_k - I_k+1)
            inter_k = []
            for k in thr:
                ctx.force_batched(pos, mass, rung, [k], out=out[:1], **kw)
                inter_k.append(ctx.stats()["interactions"])
            per_step = sum((2 ** k) * (inter_k[k] - (inter_k[k + 1] if k + 1 < 8 else 0))
                           for k in thr)
            res["subset_interactions"] = inter_k
            res["interactions_per_global_step"] = per_step
        res[prec] = {"ms_per_call": wall * 1e3, "pair_kernel_ms": st["ms_pairs"],
                     "interactions": st["interactions"], "value": st["interactions"] / wall,
                     "achieved_tflops": 40 * st["interactions"] / (st["ms_pairs"] * 1e-3) / 1e12,
                     "subtiles_per_dim": st["subtiles_per_dim"], "items": st["items"],
                     "item_target": st["item_target"], "cluster_size": st["cluster_size"],
                     "screen": st["screen"], "layout_from": "autotune_batched" if tune
                     else "fixed", "tune_s": tune_s}
        log("batched", prec, "%.3f ms  interactions %d" % (wall * 1e3, st["interactions"]))
    ctx.close()
    return res


LAYOUT_KEYS = ("subtiles_per_dim", "item_target", "cluster_size", "screen")


def configs_leg(torch, p3, steps, warmup, scale=True):
    """The other configurations: uniform32 (plain method, FP64 and FP32
    forward, autotuned), diff64 (forward and adjoint in both precisions, the
    adjoint autotuned on its own) and scale512 (N = 512^3, 1000 halos: the
    all-active FP32 forward, the 8 rung subsets in one persistent launch and
    the FP32 adjoint, in fixed layouts, since one trial is seconds there).
    GPU rows of uniform32 (all of them) and of 64 sampled diff64 particles
    are kept for the oracle comparison made with the CPU baseline; scale512's
    parity is the 4096-receiver check of its GPU tests."""
    from workloads import make_workload
    from workloads.generators import gaussian_weights
    dev = torch.device("cuda", 0)
    res = {}
    ctx = p3.Context(0)
    try:
        # uniform32: every row is kept (32768 x 32768 brute force is cheap)
        wl = make_workload("uniform32")
        pos = torch.from_numpy(wl.pos).to(dev)
        r = {"n": wl.n}
        for prec in ("fp64", "fp32"):
            kw = dict(box=wl.box, x_s=wl.x_s, r_cut=wl.r_cut, precision=prec)
            ctx.autotune(pos, None, None, level=1, **kw)
            acc, wall, st, pairs_ms, _ = time_steps(torch, ctx, pos, None, wl, prec, steps,
                                                    warmup)
            r[prec] = {"value": st["interactions"] / wall, "ms_per_step": wall * 1e3,
                       "pair_kernel_ms": pairs_ms, "interactions": st["interactions"],
                       "layout": {k: st[k] for k in LAYOUT_KEYS}, "_acc": acc.cpu().numpy()}
            log("uniform32", prec, "%.4f ms/step  pairs %.4f ms" % (wall * 1e3, pairs_ms))
        res["uniform32"] = r
        # diff64: forward and adjoint (loss sum_i w_i . a_i, seeded Gaussian w)
        wl = make_workload("diff64")
        pos = torch.from_numpy(wl.pos).to(dev)
        mass = None if bool((wl.mass == 1.0).all()) else torch.from_numpy(wl.mass).to(dev)
        w = gaussian_weights(wl.n, wl.config_id)
        wd = torch.from_numpy(w).to(dev)
        from workloads import sample_indices
        idx = sample_indices(wl.n, 64, wl.config_id, salt=7)
        r = {"n": wl.n, "_idx": idx, "_w": w}
        for prec in ("fp64", "fp32"):
            kw = dict(box=wl.box, x_s=wl.x_s, r_cut=wl.r_cut, precision=prec)
            ctx.autotune(pos, mass, None, level=1, **kw)
            _, wall, st, pairs_ms, _ = time_steps(torch, ctx, pos, mass, wl, prec, steps, warmup)
            fwd = {"value": st["interactions"] / wall, "ms_per_step": wall * 1e3,
                   "pair_kernel_ms": pairs_ms, "interactions": st["interactions"],
                   "layout": {k: st[k] for k in LAYOUT_KEYS}}
            ctx.autotune(pos, mass, None, level=1, adjoint=True, **kw)
            call = lambda: ctx.force_backward(pos, mass, None, wd, **kw)
            wall_b = time_calls(torch, call, steps, warmup)
            ctx.set_timing(True)
            g = call()
            stb = ctx.stats()
            ctx.set_timing(False)
            r[prec] = {"forward": fwd,
                       "adjoint": {"ms_per_call": wall_b * 1e3, "pair_kernel_ms": stb["ms_pairs"],
                                   "value": stb["interactions"] / wall_b,
                                   "layout": {k: stb[k] for k in LAYOUT_KEYS}},
                       "_grad": g[torch.from_numpy(idx).to(dev)].cpu().numpy()}
            log("diff64", prec, "forward %.3f ms  adjoint %.3f ms" % (wall * 1e3, wall_b * 1e3))
        res["diff64"] = r
        del pos, mass, wd, g
    finally:
        ctx.close()
    torch.cuda.empty_cache()
    if scale:
        res["scale512"] = scale512_leg(torch, p3)
    return res


def scale512_leg(torch, p3):
    """scale512 (N = 512^3, 1000 halos hold 50 %, rungs 0-7 from grid counts)
    on one GPU: each call once after a warm-up call (the batched one once,
    after the forward has grown most of the workspace), HIP-event pair-kernel
    times beside the wall clock."""
    from workloads import make_workload
    from workloads.generators import gaussian_weights
    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    wl = make_workload("scale512")
    log("scale512 generated in %.1f s" % (time.perf_counter() - t0))
    pos = torch.from_numpy(wl.pos).to(dev)
    rung = torch.from_numpy(wl.rung).to(dev)
    kw = dict(box=wl.box, x_s=wl.x_s, r_cut=wl.r_cut, precision="fp32")
    thr = list(range(8))
    res = {"workload": "scale512: N=%d clustered (1000 halos hold 50%%), PM grid %d^3, "
                       "rungs 0-7 from grid counts" % (wl.n, wl.n_pm),
           "subset_sizes": [int((wl.rung >= k).sum()) for k in thr],
           "parity": "4096 receivers against the FP64 oracle in the GPU tests"}
    ctx = p3.Context(0)

    def once(name, fn, layout, warm=True, flops=FLOPS_PER_INTERACTION):
        ctx.set_config(*layout)
        if warm:
            fn()
        torch.cuda.synchronize()
        ctx.set_timing(True)
        t1 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        st = ctx.stats()
        ctx.set_timing(False)
        rec = {"ms_per_call": wall * 1e3, "pair_kernel_ms": st["ms_pairs"],
               "build_ms": st["ms_build"], "interactions": st["interactions"],
               "value": st["interactions"] / wall,
               "achieved_tflops": flops * st["interactions"] / (st["ms_pairs"] * 1e-3) / 1e12,
               "layout": {k: st[k] for k in LAYOUT_KEYS}}
        log("scale512", name, "%.1f ms  pairs %.1f ms  %.3g interactions"
            % (wall * 1e3, st["ms_pairs"], st["interactions"]))
        return rec

    try:
        out = torch.empty((wl.n, 3), dtype=torch.float64, device=dev)
        res["forward_fp32"] = once(
            "forward", lambda: ctx.force(pos, None, None, out=out, **kw), (1, 4096, 32, 2))
        del out
        out8 = torch.empty((8, wl.n, 3), dtype=torch.float64, device=dev)
        res["batched_fp32"] = once(
            "batched", lambda: ctx.force_batched(pos, None, rung, thr, out=out8, **kw),
            (2, 4096, 32, 1), warm=False)
        del out8
        wd = torch.from_numpy(gaussian_weights(wl.n, wl.config_id)).to(dev)
        res["adjoint_fp32"] = once(
            "adjoint", lambda: ctx.force_backward(pos, None, None, wd, **kw),
            (1, 4096, 32, 2), flops=ADJOINT_FLOPS)
        del wd
    finally:
        ctx.set_config()
        ctx.close()
    del pos, rung
    torch.cuda.empty_cache()
    return res


def configs_errors(cfg):
    """Force errors of the uniform32 rows (every row, against the oracle's
    brute force, with the exact pair count) and the VJP errors of the diff64
    sampled rows (against the oracle's cell-list VJP), filled into the
    configs leg's records; part of the CPU-baseline work."""
    import numpy as np

    import oracle
    from workloads import make_workload
    if "uniform32" in cfg:
        u = make_workload("uniform32")
        ref_u, cnt_u, absum_u = oracle.force_full(u.pos, None, u.box, u.x_s, u.r_cut)
        for prec in ("fp64", "fp32"):
            rec = cfg["uniform32"][prec]
            e = oracle.errors(rec["_acc"], ref_u, absum_u)
            rec["force_error"] = {"e_l2": e["e_l2"], "e_max_cond": e["e_max_cond"], "rows": u.n}
            rec["interactions_match_oracle"] = rec["interactions"] == int(cnt_u.sum())
    if "diff64" in cfg:
        d = make_workload("diff64")
        rd = cfg["diff64"]
        g_ref = oracle.vjp(d.pos, d.mass, None, rd["_w"], d.box, d.x_s, d.r_cut,
                           kidx=rd["_idx"], method="tiled")
        for prec in ("fp64", "fp32"):
            got = rd[prec]["_grad"]
            rd[prec]["adjoint"]["vjp_error"] = {
                "rel_l2": float(np.linalg.norm(got - g_ref) / np.linalg.norm(g_ref)),
                "max_row": float(np.max(np.linalg.norm(got - g_ref, axis=1))
                                 / np.max(np.linalg.norm(g_ref, axis=1))),
                "rows": int(rd["_idx"].size)}


def configs_strip(cfg):
    """Drop the configs leg's kept GPU rows before the line is printed."""
    for prec in ("fp64", "fp32"):
        cfg.get("uniform32", {}).get(prec, {}).pop("_acc", None)
        cfg.get("diff64", {}).get(prec, {}).pop("_grad", None)
    for k in ("_idx", "_w"):
        cfg.get("diff64", {}).pop(k, None)


def sort_record(st, n):
    """HBM rate of the counting sort (cell keys, scan, scatter, fine order)
    against its algorithmic bytes: each particle's position read once (24 B)
    and its sorted record (32 B) and original index (4 B) written once, plus
    the cell table counted and scanned (4 B per fine cell written, read and
    written again)."""
    cells = st["tiles_per_dim"] ** 3 * st["subtiles_per_dim"] ** 3
    nbytes = 60 * n + 12 * cells
    ms = st["ms_sort_median"]
    gbps = nbytes / (ms * 1e-3) / 1e9
    return {"ms": ms, "algorithmic_bytes": nbytes, "bytes_per_particle": 60,
            "bytes_per_cell": 12, "gb_per_s": gbps, "frac_hbm": gbps / (PEAK_HBM_TBPS * 1e3),
            "bound": "hbm"}


def cpu_tiled_leg():
    """The oracle's cell-list walk (FP64, OpenMP over receivers) on the full
    uniform32, diff64 and clustered128 sets: the fair CPU rate beside the GPU
    numbers, with the host threads it used."""
    import oracle
    from workloads import make_workload
    oracle.build(force=False)
    res = {"cores": oracle.threads(), "kind": "oracle (cell list, all N receivers)"}
    for name in ("uniform32", "diff64", "clustered128"):
        wl = make_workload(name, with_rungs=False)
        t0 = time.perf_counter()
        _, cnt, _ = oracle.force_full(wl.pos, None, wl.box, wl.x_s, wl.r_cut, method="tiled")
        dt = time.perf_counter() - t0
        res[name] = {"n": wl.n, "interactions": int(cnt.sum()), "seconds": dt,
                     "value": float(cnt.sum()) / dt, "unit": "interactions/s"}
        log("cpu tiled", name, "%.1f s  %.3e interactions/s" % (dt, cnt.sum() / dt))
    return res


def profiled_record(name, st):
    """The committed rocprofv3 counter record of the pair kernel in this
    call's decomposition (profiles/traffic.json holds one per profiled
    layout), or None when the kernel sources or the decomposition differ
    from the ones the counters were taken with."""
    import hashlib
    try:
        recs = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[name]
    except (OSError, KeyError, ValueError):
        return None
    if isinstance(recs, dict):
        recs = [recs]
    h = hashlib.sha256()
    for f in ("force.hip", "p3msr_internal.hpp", "gpoly.inc"):
        with open(os.path.join(ROOT, "paper_2112_01508_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    keys = ("subtiles_per_dim", "item_target", "cluster_size", "screen")
    for rec in recs:
        if h.hexdigest() == rec.get("kernel_sources_sha256") and all(
                rec.get(k) == st[k] for k in keys):
            return rec
    return None


def copy_probe():
    import torch
    n = 64 * 1024 * 1024                      # 64 Mi doubles = 512 MiB
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 8, "copies": 3}), flush=True)


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2112_01508_amd as p3
    from workloads import make_workload, sample_indices

    log("generating workload", args.workload)
    wl = make_workload(args.workload, with_rungs=False)
    dev = torch.device("cuda", 0)
    pos = torch.from_numpy(wl.pos).to(dev)
    # G*m = 1 for every particle: pass no mass array (the ABI's "all ones")
    mass = None if np.all(wl.mass == 1.0) else torch.from_numpy(wl.mass).to(dev)
    ctx = p3.Context(0)

    results = {}
    fixed = bool(args.ns or args.target or args.csize or args.screen >= 0)
    if fixed:
        ctx.set_config(args.ns, args.target, args.csize, args.screen)
    for prec in (["fp32"] if args.no_fp64 else ["fp32", "fp64"]):
        if not args.no_autotune and not fixed:
            log("autotuning", prec)
            ctx.autotune(pos, mass, None, box=wl.box, x_s=wl.x_s, r_cut=wl.r_cut,
                         precision=prec, level=2)
        log("timing", prec)
        out, wall, st, pairs_ms, build_ms = time_steps(torch, ctx, pos, mass, wl, prec,
                                                       args.steps, args.warmup)
        results[prec] = dict(out=out.cpu().numpy(), wall=wall, stats=st, pairs_ms=pairs_ms,
                             build_ms=build_ms)
        log(prec, "ms/step %.3f  pairs %.3f ms  build %.3f ms  interactions %d  ns %d target %d "
            "csize %d screen %d steps %d" % (wall * 1e3, pairs_ms, build_ms, st["interactions"],
                                             st["subtiles_per_dim"], st["item_target"],
                                             st["cluster_size"], st["screen"], st["steps"]))

    r32 = results["fp32"]
    inter = r32["stats"]["interactions"]
    value = inter / r32["wall"]
    achieved = FLOPS_PER_INTERACTION * inter / (r32["pairs_ms"] * 1e-3) / 1e12

    line = {
        "metric": "short-range pair interactions/s (FP32 vs FP64) at stated force error, "
                  "% VALU peak",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["wall"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: N=%d clustered (200 NFW halos hold 30%%), PM grid %d^3, "
                               "x_s=1.25 cells, r_cut=4.5 x_s, all active, G*m=1"
                               % (args.workload, wl.n, wl.n_pm),
                   "n": wl.n, "interactions_per_step": inter,
                   "tiles_per_dim": r32["stats"]["tiles_per_dim"],
                   "subtiles_per_dim": r32["stats"]["subtiles_per_dim"],
                   "item_target": r32["stats"]["item_target"],
                   "cluster_size": r32["stats"]["cluster_size"],
                   "screen": r32["stats"]["screen"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None},
        "pair_kernel_ms": r32["pairs_ms"],
        "build_ms": r32["build_ms"],
        "sort": sort_record(r32["stats"], wl.n),
    }
    prof = profiled_record("k_pairs_fwd_fp32_%s" % args.workload, r32["stats"])
    if prof:
        line["roofline"]["traffic"] = prof["traffic_bytes"]
        if "counter_fp32_tflops" in prof:
            # SQ_INSTS_VALU_FLOPS_FP32/_FP64 x 64 lanes over the traced kernel time;
            # masked lanes count as well
            line["roofline"]["counter"] = {
                "fp32_tflops": prof["counter_fp32_tflops"],
                "fp64_tflops": prof["counter_fp64_tflops"],
                "fp32_frac": prof["counter_fp32_tflops"] / PEAK_FP32_TFLOPS,
                "includes_masked_lanes": True}
    if "fp64" in results:
        r64 = results["fp64"]
        a64 = FLOPS_PER_INTERACTION * r64["stats"]["interactions"] / (r64["pairs_ms"] * 1e-3) / 1e12
        line["fp64"] = {"value": r64["stats"]["interactions"] / r64["wall"],
                        "ms_per_step": r64["wall"] * 1e3, "pair_kernel_ms": r64["pairs_ms"],
                        "achieved_tflops": a64, "frac_fp64_peak": a64 / PEAK_FP64_TFLOPS,
                        "layout": {k: r64["stats"][k] for k in
                                   ("subtiles_per_dim", "item_target", "cluster_size", "screen")}}

    legs = [l for l in args.legs.split(",") if l]
    if "adjoint" in legs:
        line["adjoint"] = adjoint_leg(torch, ctx, pos, mass, wl, args.steps, args.warmup,
                                      tune=not (args.no_autotune or fixed))
    if "softened" in legs:
        line["softened"] = softened_leg(torch, ctx, pos, mass, wl, args.steps, args.warmup)
    if "long_range" in legs:
        line["long_range"] = long_range_leg(torch, ctx, pos, mass, wl, args.steps, args.warmup,
                                            cpu=not args.no_cpu_baseline)
        line["long_range"]["p3m_step_ms_fp32"] = (line["ms_per_step"]
                                                  + line["long_range"]["ms_per_call"])
        line["long_range"]["p3m_force"] = p3m_leg(torch, ctx, pos, mass, wl, args.steps,
                                                  args.warmup)
    if "shapes" in legs:
        line["shapes"] = shapes_leg(torch, ctx, pos, mass, wl, args.steps, args.warmup)
    if "kdk" in legs:
        line["kdk"] = kdk_leg(torch, ctx, pos, mass, wl)
    if "deterministic" in legs:
        line["deterministic"] = deterministic_leg(torch, ctx, pos, mass, wl, args.steps,
                                                  args.warmup)
    if "subtiles" in legs:
        line["subtiles"] = subtiles_leg(torch, p3)
    if "configs" in legs:
        line["configs"] = configs_leg(torch, p3, args.steps, args.warmup,
                                      scale="noscale" not in legs)
    if "batched" in legs:
        layouts = {p: tuple(results[p]["stats"][k] for k in
                            ("subtiles_per_dim", "item_target", "cluster_size", "screen"))
                   for p in results}
        line["batched"] = batched_leg(torch, p3, args.batched_workload, args.steps, args.warmup,
                                      layouts=layouts, tune=not (args.no_autotune or fixed))

    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        # size the receiver sample for about args.cpu_seconds of oracle work
        probe = sample_indices(wl.n, 2048, wl.config_id, salt=1)
        t0 = time.perf_counter()
        oracle.force(wl.pos, wl.mass, wl.box, wl.x_s, wl.r_cut, recv=probe)
        per = (time.perf_counter() - t0) / probe.size
        m = int(max(256, min(wl.n, args.cpu_seconds / max(per, 1e-9))))
        idx = sample_indices(wl.n, m, wl.config_id)
        log("cpu oracle on %d receivers" % idx.size)
        t0 = time.perf_counter()
        ref, cnt, absum, _ = oracle.force(wl.pos, wl.mass, wl.box, wl.x_s, wl.r_cut, recv=idx)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {
            "value": float(cnt.sum()) / dt, "unit": "interactions/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": "FP64 brute force over all N suppliers for %d seeded receivers "
                      "(%d interactions, %.1f s)" % (idx.size, int(cnt.sum()), dt),
            "pair_tests_per_s": float(idx.size) * wl.n / dt}
        # the oracle's cell-list walk on the same receivers: the fair CPU rate
        t0 = time.perf_counter()
        _, cnt_t, _, _ = oracle.force(wl.pos, wl.mass, wl.box, wl.x_s, wl.r_cut, recv=idx,
                                      method="tiled")
        dt_t = time.perf_counter() - t0
        line["cpu_baseline"]["tiled"] = {"value": float(cnt_t.sum()) / dt_t,
                                         "unit": "interactions/s", "seconds": dt_t}
        errs = {}
        for prec, r in results.items():
            errs[prec] = oracle.errors(r["out"][idx], ref, absum)
        line["force_error"] = {p: {"e_l2": e["e_l2"], "e_max_cond": e["e_max_cond"],
                                   "p999": e["p999"]} for p, e in errs.items()}
        for key, rec in line.get("shapes", {}).items():
            e = oracle.errors(rec["_acc"][idx], ref, absum)
            rec["force_error"] = {"e_l2": e["e_l2"], "e_max_cond": e["e_max_cond"]}
        configs_errors(line.get("configs", {}))
        if not args.no_cpu_tiled:
            line["cpu_tiled"] = cpu_tiled_leg()
    for rec in line.get("shapes", {}).values():
        rec.pop("_acc", None)
    configs_strip(line.get("configs", {}))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
