#!/usr/bin/env python3
"""Benchmark of the hydrodynamics step on one MI355X.

Workload: the 3D spherical (phi, r, theta) adiabatic disk, 1536 x 512 x 128
active zones, FP64, orbital advection on, time step computed on the device
every step (the whole hot path: boundary fill, bulk velocity, CFL reduction,
source step, transport with integer shift and PPA residual, velocities).
Inputs are seeded and synthetic and already resident in HBM when the timed
region starts.

Prints one JSON line: cell-updates/s, ms/step, the roofline of the dominant
kernel (algorithmic bytes per launch over its average duration from HIP
events recorded on the launch stream during the timed steps) and the CPU
oracle timed on a bounded sample of the same workload.  The FP32-bulk
variant (FP32 state, FP64 time step, ring split and sums) is then timed on
the same workload and reported with its normwise error against the FP64 run
after the same number of steps from the same initial state.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s per full hydro step + HBM GB/s; FP32/batched vs FP64 at error"
HBM_PEAK_GBS = 8000.0
NGH = 3


def words_per_unit(p):
    """Algorithmic words (8 bytes in FP64, 4 in FP32 bulk) moved per zone by
    each kernel of the step (each input read once, each output written once),
    and the zones one launch processes."""
    d3 = p["nz"] > 1
    adi = 1 if p["eos"] == "adi" else 0
    nT = 5 + (2 if d3 else 0) + adi
    nvel = 3 if d3 else 2
    act = p["nx"] * p["ny"] * p["nz"]
    whole = p["nx"] * (p["ny"] + 2 * NGH) * ((p["nz"] + 2 * NGH) if d3 else 1)
    y_rows = p["nx"] * p["ny"] * ((p["nz"] + 4) if d3 else 1)
    return {
        # name: (words per zone, zones per launch)
        "cfl": (2 + nvel, act),                              # rho, cs|e, velocities
        "source": ((3 + nvel) + (nvel + adi), act),          # rho, cs|e, pot, v -> v'', e''
        "source_ghosts": (2 * (nvel + adi), whole - act),    # v, e -> v'', e'' in ghost zones
        "sweep_y": ((1 + nvel + adi) + nT, y_rows),          # rho, v'', e'' -> T (momenta formed on the fly)
        "sweep_z": ((2 * nT + 1) if d3 else 0, act),         # T, v_z -> T
        "ring_x": ((nT + 1) + (2 + adi + 2 + (2 if d3 else 0)), act),  # T, v_x -> rho, v_x, e, Pi_y, Pi_z
        "zx_ring": ((nT + 2 + 2 + adi + 4) if d3 else 0, act),   # Y-swept T, v_z, v_x -> rho, v_x, e, Pi_y, Pi_z
        "vel_yz": ((1 + 2 + (2 if d3 else 0)) + (nvel - 1), act),      # rho, Pi_y, Pi_z -> v_y, v_z
    }


# the source file of each kernel: a measured traffic figure is used only while
# the file (and the shared internal header) is unchanged since the counters
# were taken
KERNEL_SOURCES = {"cfl": "timestep.hip", "source": "source.hip", "source_ghosts": "source.hip",
                  "sweep_y": "transport.hip", "sweep_z": "transport.hip", "ring_x": "transport.hip",
                  "zx_ring": "transport.hip",
                  "vel_yz": "transport.hip"}


def source_hash(kernel):
    h = hashlib.sha256()
    for f in (KERNEL_SOURCES[kernel], "fargo_internal.h"):
        with open(os.path.join(ROOT, "paper_1602_02359_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, tag):
    """HBM bytes per launch of `kernel` from the rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary in profiles/ (copy-calibrated), or None if there is none or the
    kernel's source changed since."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_%s.md" % tag)
    if kernel not in KERNEL_SOURCES or not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) >= 6 and cells[0] == kernel:
                if cells[1] != source_hash(kernel):
                    return None
                try:
                    return float(cells[5])
                except ValueError:
                    return None
    return None


def compulsory_bytes(p):
    """Read every state and static field once, write the state once, plus the
    time-step pass the global dt forces (velocities and sound speed again)."""
    d3 = p["nz"] > 1
    adi = p["eos"] == "adi"
    nvel = 3 if d3 else 2
    state = 1 + nvel + (1 if adi else 0)
    static = 1 + (0 if adi else 1)  # pot, cs
    cfl = nvel + 2
    return 8 * (state + static + state + cfl)


def sample_problem(prob, ny_s, nz_s):
    """Rings [j0, j0+ny_s) x [k0, k0+nz_s) of a problem, whole X, with the
    real neighbouring zones as caller-fixed ghosts on cut sides."""
    from paper_1602_02359_amd import workloads as W
    p = prob.params
    sub = dict(p)
    bc = list(p["bc"])
    ja, jb = NGH, NGH + ny_s
    if jb != NGH + p["ny"]:
        bc[1] = "fixed"
    sub["ny"] = ny_s
    sub["ymin"] = p["ymin"][ja - NGH:jb + NGH + 1].copy()
    if p["nz"] > 1:
        mid = NGH + p["nz"] // 2 - nz_s // 2
        ka, kb = mid, mid + nz_s
        bc[2] = "fixed"
        bc[3] = "fixed"
        sub["nz"] = nz_s
        sub["zmin"] = p["zmin"][ka - NGH:kb + NGH + 1].copy()
        ks = slice(ka - NGH, kb + NGH)
    else:
        ks = slice(0, 1)
    sub["bc"] = tuple(bc)
    js = slice(ja - NGH, jb + NGH)
    f = {k: (None if v is None else v[ks, js, :].copy()) for k, v in prob.fields.items()}
    return W.Problem(prob.name + "_sample", sub, f, 1)


def cpu_baseline(prob, target_s=12.0):
    from oracle import oracle as O
    p = prob.params
    nz_s = 8 if p["nz"] > 1 else 1
    ny_s = 16
    s = sample_problem(prob, ny_s, nz_s)
    f = s.copy_fields()
    t0 = time.perf_counter()
    O.step(s.params, f)
    t_cal = time.perf_counter() - t0
    rate = s.active_cells / t_cal
    # scale the sample to about target_s of work, within the workload
    want = rate * target_s
    if p["nz"] > 1:
        nz_s = max(4, min(p["nz"], int(want / (p["nx"] * p["ny"]))))
        ny_s = p["ny"] if nz_s * p["nx"] * p["ny"] <= want else max(4, int(want / (p["nx"] * nz_s)))
    else:
        ny_s = max(4, min(p["ny"], int(want / p["nx"])))
    s = sample_problem(prob, ny_s, nz_s)
    f = s.copy_fields()
    t0 = time.perf_counter()
    O.step(s.params, f)
    el = time.perf_counter() - t0
    return {
        "value": s.active_cells / el,
        "unit": "cell-updates/s",
        "cores": O.num_threads(),
        "kind": "oracle",
        "sample": "one full step (CFL included) of %d x %d x %d zones of the same workload (rings cut "
                  "from the mesh, neighbours as fixed ghosts), %.1f s" % (p["nx"], s.params["ny"], s.params["nz"], el),
    }


def batch_variant(steps, warmup, tune=True):
    """The parameter sweep of 256 uneven viscous disks (N_r in 64..512,
    N_phi = 3 N_r, alpha viscosity): the plain FP64 step called disk by disk,
    then the FP32-bulk batch advanced by one captured graph per step with the
    autotuned graph width and sweep chunk.  Same disks, same number of steps."""
    import torch
    from paper_1602_02359_amd import fargo as F
    from paper_1602_02359_amd import workloads as W
    probs = W.disk_batch()
    cells = sum(p.active_cells for p in probs)
    print("disk batch: %d disks, %d cells" % (len(probs), cells), file=sys.stderr, flush=True)

    def timed(run_one, nsteps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            run_one()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    out = {}
    s64 = []
    for p in probs:
        s = F.Solver(p.params)
        s.upload(p.fields)
        s64.append(s)
    step64 = lambda: [s.fargo_step(0.0) for s in s64]
    for _ in range(warmup):
        step64()
    el = timed(step64, steps)
    for s in s64:
        s.fargo_check()
    out["fp64_disk_by_disk"] = {"value": cells * steps / el, "ms_per_step": 1e3 * el / steps}
    del s64
    torch.cuda.empty_cache()
    s32 = []
    for p in probs:
        s = F.Solver(dict(p.params, precision="fp32"))
        s.upload(p.fields)
        s32.append(s)
    b = F.Batch(s32, lanes=8)
    best = None
    if tune:
        best = b.fargo_batch_tune(lanes=(1, 4, 8, 16), chunks=(16, 32, 64), steps=10)
    for _ in range(warmup):
        b.fargo_batch_step()
    el = timed(b.fargo_batch_step, steps)
    for s in s32:
        s.fargo_check()
    out["fp32_batched_graph"] = {"value": cells * steps / el, "ms_per_step": 1e3 * el / steps,
                                 "tuned": {"lanes": best[0], "chunk": best[1]} if best else None}
    out["speedup"] = out["fp32_batched_graph"]["value"] / out["fp64_disk_by_disk"]["value"]
    out["disks"] = len(probs)
    out["active_cells"] = cells
    out["unit"] = "cell-updates/s"
    print("  fp64 disk by disk %.3e, fp32 batched graph %.3e cell-updates/s (x%.2f), tuned %s" % (
        out["fp64_disk_by_disk"]["value"], out["fp32_batched_graph"]["value"], out["speedup"], best),
        file=sys.stderr, flush=True)
    del b, s32
    torch.cuda.empty_cache()
    return out


MFMA_BF16_PEAK_TFLOPS = 2500.0  # MI355X dense bf16 matrix peak


def copy_bandwidth():
    """Bytes read plus written per second by a plain 1 GiB device copy
    (torch's copy kernel), timed with HIP events: the bandwidth a streaming
    kernel can reach on this GPU, for comparison with the 8 TB/s peak."""
    import torch
    src = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(10):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / 10
    del src, dst
    torch.cuda.empty_cache()
    return 2 * 2 ** 27 * 8 / (ms * 1e-3) / 1e9


def lfc_variant(iters=600):
    """The learned flux correction on the planet disks (coarse 768 x 256,
    fine 3072 x 1024): 40 samples along one fine trajectory (after 200 fine
    spin-up steps), 32 for training and 8 held out.  Adam steps are timed with
    per-kernel HIP events; the held-out error of the corrected coarse step
    (|drho - target| / |target|, 1 = the plain step) before and after."""
    import torch
    from paper_1602_02359_amd import learned as LN
    t0 = time.perf_counter()
    cp, samples = LN.make_samples(40, spinup=200)
    torch.cuda.synchronize()
    gen = time.perf_counter() - t0
    sc = LN.scales(cp, samples)
    tr = LN.Trainer(cp, sc)
    train, held = samples[:32], samples[32:]
    before = tr.evaluate(held)
    tr.train(train, 20, 3e-3, every=20)
    torch.cuda.synchronize()
    tr.feed.fargo_profile_enable(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tr.train(train, iters, 3e-3, every=iters)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    tim = tr.feed.fargo_timings()
    tr.feed.fargo_profile_enable(False)
    tr.train(train, iters, 1e-3, every=iters)
    after, after_train = tr.evaluate(held), tr.evaluate(train)
    # one guarded correction on a held-out state
    tr.load(held[0])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(50):
        tr.net.apply()
    torch.cuda.synchronize()
    apply_ms = 1e3 * (time.perf_counter() - t2) / 50
    npix = cp.params["nx"] * cp.params["ny"]
    # algorithmic flops of a training step (unpadded GEMM dimensions)
    fl = {"lfc_conv_fwd": 2.0 * npix * (36 * 32 + 288 * 32 + 288 * 2),
          "lfc_conv_bwd_w": 2.0 * npix * (36 * 32 + 288 * 32 + 288 * 2),
          "lfc_conv_bwd_data": 2.0 * npix * (18 * 32 + 288 * 32)}
    kern = {}
    for name, (cnt, tot) in tim.items():
        e = {"launches": cnt, "avg_ms": tot / cnt, "ms_per_train_step": tot / iters}
        if name in fl:
            e["TFLOPs"] = fl[name] * iters / (tot * 1e-3) / 1e12
        kern[name] = e
    dom = max((k for k in kern if "TFLOPs" in kern[k]), key=lambda k: kern[k]["ms_per_train_step"])
    out = {
        "workload": "learned flux correction, planet disk: coarse 768x256 (196608 zones), fine 3072x1024, "
                    "3 conv layers 4-32-32-2, bf16 MFMA",
        "ms_per_train_step": 1e3 * el / iters,
        "train_steps_per_s": iters / el,
        "ms_per_apply": apply_ms,
        "sample_generation_s": gen,
        "heldout_relative_error": {"before": before["relative_error"], "after": after["relative_error"]},
        "train_relative_error_after": after_train["relative_error"],
        "train_steps": 20 + 2 * iters,
        "kernels": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kern.items()},
        "roofline": {"bound": "mfma", "kernel": dom, "achieved": round(kern[dom]["TFLOPs"], 3),
                     "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": kern[dom]["TFLOPs"] / MFMA_BF16_PEAK_TFLOPS, "traffic": None},
    }
    print("  lfc: %.3f ms per training step, %.3f ms per apply; held-out error %.3f -> %.3f; %s %.2f TFLOP/s" % (
        out["ms_per_train_step"], apply_ms, before["relative_error"], after["relative_error"], dom,
        kern[dom]["TFLOPs"]), file=sys.stderr, flush=True)
    del tr, samples
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="sph3d", choices=["sph3d", "cyl3d_planet", "disk2d"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variant", action="store_true", help="skip the FP32-bulk and disk-batch variants")
    ap.add_argument("--no-batch", action="store_true", help="skip the disk-batch variant")
    ap.add_argument("--no-lfc", action="store_true", help="skip the learned-flux-correction variant")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one plain device copy of 2 GiB first (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library's step runs on one device; the multi-GPU slab "
              "decomposition is a design, not a measured path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1602_02359_amd import fargo as F
    from paper_1602_02359_amd import workloads as W

    if args.copy_probe:
        src = torch.ones(2 ** 28, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("copy probe: %d bytes read, %d bytes written" % (src.numel() * 8, dst.numel() * 8), file=sys.stderr)
        del src, dst
        torch.cuda.empty_cache()
    prob = W.make(args.config)
    p = prob.params
    wpu = words_per_unit(p)
    cells = prob.active_cells

    def run(precision):
        """Warm up, then time args.steps steps with per-kernel HIP events on
        the launch stream; returns the solver (state kept) and the figures."""
        print("workload %s %dx%dx%d %s, building state" % (args.config, p["nx"], p["ny"], p["nz"], precision),
              file=sys.stderr, flush=True)
        solver = F.Solver(dict(p, precision=precision))
        solver.upload(prob.fields)
        for _ in range(args.warmup):
            solver.fargo_step(0.0)
        solver.fargo_check()
        torch.cuda.synchronize()
        solver.fargo_profile_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            solver.fargo_step(0.0)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        timings = solver.fargo_timings()
        solver.fargo_profile_enable(False)
        solver.fargo_check()
        dt_last = solver.fargo_get_dt()
        value = cells * args.steps / el
        ms = 1e3 * el / args.steps
        print("timed %d steps: %.3f ms/step, %.3e cell-updates/s, dt %.6g" % (args.steps, ms, value, dt_last),
              file=sys.stderr, flush=True)
        wb = 4.0 if precision == "fp32" else 8.0
        kern = {}
        for name, (cnt, tot) in timings.items():
            avg = tot / cnt
            entry = {"launches": cnt, "avg_ms": avg}
            if name in wpu and wpu[name][0] > 0:
                b = wb * wpu[name][0] * wpu[name][1]
                entry["alg_bytes"] = b
                entry["GBs"] = b / (avg * 1e-3) / 1e9
            kern[name] = entry
            print("  %-16s %6d launches  %9.4f ms avg  %s" % (name, cnt, avg,
                  ("%.0f GB/s" % entry["GBs"]) if "GBs" in entry else ""), file=sys.stderr)
        dom = max((k for k in kern if "alg_bytes" in kern[k]),
                  key=lambda k: kern[k]["avg_ms"] * kern[k]["launches"])
        # the kernels that ran, each as often per step as it was launched
        step_alg = sum(e["alg_bytes"] * e["launches"] for e in kern.values() if "alg_bytes" in e) / args.steps
        return solver, {"value": value, "ms": ms, "kern": kern, "dom": dom, "step_alg": step_alg}

    copy_gbs = copy_bandwidth()
    print("device copy: %.0f GB/s (read + write)" % copy_gbs, file=sys.stderr, flush=True)
    solver, r64 = run("fp64")
    value, ms, kern, dom, step_alg = r64["value"], r64["ms"], r64["kern"], r64["dom"], r64["step_alg"]
    achieved = kern[dom]["GBs"]
    tag = "%s_%dx%dx%d_fp64" % (args.config, p["nx"], p["ny"], p["nz"])
    traffic = measured_traffic(dom, tag)
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "alg_bytes_per_launch": kern[dom]["alg_bytes"], "avg_launch_ms": kern[dom]["avg_ms"]}

    variants = {}
    if not args.no_variant:
        s32, r32 = run("fp32")
        # normwise error of the FP32-bulk state against the FP64 state after
        # the same warmup + timed steps (velocities scaled by the largest speed)
        nx = p["nx"]
        d3 = p["nz"] > 1
        ks = slice(NGH, NGH + p["nz"]) if d3 else slice(0, 1)
        js = slice(NGH, NGH + p["ny"])
        vnames = ("vx", "vy", "vz") if d3 else ("vx", "vy")
        vmax = max(float(solver.state[k][ks, js, :nx].abs().max()) for k in vnames)
        err = {}
        for k in ("rho", "e") + vnames:
            if solver.state.get(k) is None:
                continue
            a = s32.state[k][ks, js, :nx].double()
            b = solver.state[k][ks, js, :nx]
            den = vmax if k.startswith("v") else float(b.abs().max())
            err[k] = float((a - b).abs().max()) / den
            del a
        dk = r32["dom"]
        variants["fp32_bulk"] = {
            "value": r32["value"], "unit": "cell-updates/s", "ms_per_step": r32["ms"],
            "speedup_vs_fp64": r32["value"] / value,
            "error_vs_fp64": {k: float("%.3g" % v) for k, v in err.items()},
            "steps_compared": args.warmup + args.steps,
            "step_alg_bytes_per_cell": r32["step_alg"] / cells,
            "dominant_kernel": {"kernel": dk, "avg_ms": r32["kern"][dk]["avg_ms"],
                                "GBs": round(r32["kern"][dk]["GBs"], 1)},
            "kernels": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                        for k, v in r32["kern"].items()},
        }
        print("  fp32 bulk: %.3e cell-updates/s (x%.2f), error vs fp64 %s" % (
            r32["value"], r32["value"] / value, variants["fp32_bulk"]["error_vs_fp64"]), file=sys.stderr)
        del s32
    del solver
    torch.cuda.empty_cache()
    if not args.no_variant and not args.no_batch:
        variants["disk_batch"] = batch_variant(args.steps, args.warmup)
    if not args.no_variant and not args.no_lfc:
        variants["learned_flux_correction"] = lfc_variant()

    cpu = None
    if not args.no_cpu_baseline:
        print("timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(prob)
        print("  oracle %.3e cell-updates/s on %d threads" % (cpu["value"], cpu["cores"]), file=sys.stderr)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "%s: %s %dx%dx%d (phi, r, %s), %s, orbital advection %s, FP64, dt on device" % (
                args.config, p["geometry"], p["nx"], p["ny"], p["nz"], "theta" if p["geometry"] == "sph" else "z",
                "adiabatic" if p["eos"] == "adi" else "isothermal", "on" if p["fargo"] else "off"),
            "active_cells": cells,
            "parallelism": "single GPU",
        },
        "hbm": {
            "device_copy_GBs": copy_gbs,
            "step_alg_bytes_per_cell": step_alg / cells,
            "step_alg_GBs": value * step_alg / cells / 1e9,
            "compulsory_bytes_per_cell": compulsory_bytes(p),
            "effective_GBs": value * compulsory_bytes(p) / 1e9,
        },
        "kernels": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kern.items()},
        "roofline": roof,
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
