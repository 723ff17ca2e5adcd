#!/usr/bin/env python3
"""Benchmark of the hydrodynamics step on one MI355X.

Headline workload: the 3D cylindrical (phi, r, z) isothermal disk with a
fixed planet, 2048 x 768 x 96 active zones (151 M), FP64, orbital advection
on, time step computed on the device every step (the whole hot path:
boundary fill, bulk velocity, CFL reduction, source step, transport with
integer shift and PPA residual, velocities).  Inputs are seeded and synthetic
and already resident in HBM when the timed region starts.  The timed steps
run with per-kernel timing off; per-kernel HIP-event means come from a
separate pass over the same state.

Prints one JSON line: cell-updates/s and ms/step of the headline, the
roofline of its dominant kernel (algorithmic bytes per launch over its mean
duration), the CPU oracle timed on a bounded sample of the same workload on
one core and on all cores, and beside them:
  - the 3D spherical adiabatic disk 1536 x 512 x 128 and the 2D disk
    384 x 128, FP64 (same figures);
  - the FP32-bulk state (FP64 time step, ring split and sums) on both 3D
    disks: its rate, and its error against the FP64 run after 100 steps at
    equal times (the FP32 run takes the FP64 run's time steps);
  - physical time advanced per second with orbital advection on and off;
  - the HBM ceiling of a hand-written streaming copy;
  - the batch of 256 uneven viscous disks and the learned flux correction.
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
    and the zones one launch processes.  The potential is FP64 in both modes:
    two words of an FP32 state."""
    d3 = p["nz"] > 1
    pw = 2 if p.get("precision") == "fp32" else 1
    adi = 1 if p["eos"] == "adi" else 0
    nT = 5 + (2 if d3 else 0) + adi
    nvel = 3 if d3 else 2
    act = p["nx"] * p["ny"] * p["nz"]
    whole = p["nx"] * (p["ny"] + 2 * NGH) * ((p["nz"] + 2 * NGH) if d3 else 1)
    y_rows = p["nx"] * p["ny"] * ((p["nz"] + 4) if d3 else 1)
    return {
        # name: (words per zone, zones per launch)
        "cfl": (2 + nvel, act),                              # rho, cs|e, velocities
        "source": ((2 + pw + nvel) + (nvel + adi), act),     # rho, cs|e, pot, v -> v'', e''
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


def host_info():
    """CPU model and logical CPU count of the host."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(),
            "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(prob, target_s=10.0):
    """The FP64 oracle (built with -march=native on this host, no contraction,
    no fast-math) timed on one step of a bounded sample of the workload: whole
    rings of the mesh, the real neighbours as fixed ghosts, scaled to about
    target_s of work; on one thread, then on every thread OpenMP is allowed."""
    from oracle import oracle as O
    O.use_native()
    p = prob.params
    all_threads = O.num_threads()

    def timed(ny_s, nz_s):
        smp = sample_problem(prob, ny_s, nz_s)
        f = smp.copy_fields()
        t0 = time.perf_counter()
        O.step(smp.params, f)
        return smp, time.perf_counter() - t0

    def sized(rate):
        want = min(rate * target_s, 1.6e8)  # at most 160 M zones (some 50 GB of host memory for the oracle)
        if p["nz"] > 1:
            nz_s = max(4, min(p["nz"], int(want / (p["nx"] * p["ny"]))))
            ny_s = p["ny"] if nz_s * p["nx"] * p["ny"] <= want else max(4, int(want / (p["nx"] * nz_s)))
        else:
            nz_s, ny_s = 1, max(4, min(p["ny"], int(want / p["nx"])))
        return ny_s, nz_s

    out = {}
    for label, nth in (("one_core", 1), ("all_cores", all_threads)):
        O.set_num_threads(nth)
        cal, t_cal = timed(16, 8 if p["nz"] > 1 else 1)
        smp, el = timed(*sized(cal.active_cells / t_cal))
        out[label] = {
            "value": smp.active_cells / el, "unit": "cell-updates/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": "one full step (CFL included) of %d x %d x %d zones of the same workload (whole rings, "
                      "neighbours as fixed ghosts), %.1f s, oracle built -O3 -march=native -ffp-contract=off"
                      % (p["nx"], smp.params["ny"], smp.params["nz"], el)}
    O.set_num_threads(all_threads)
    res = dict(out["all_cores"])
    res["one_core"] = out["one_core"]
    res["host"] = host_info()
    return res


def field_errors(a, b, keys, owned):
    """Normwise L_inf errors of solver a against solver b over the slices
    owned(k): velocities scaled by b's largest speed; each velocity also by
    its own largest value (own_scale)."""
    vk = [k for k in keys if k.startswith("v")]
    vmax = max(float(b.field64(k)[owned(k)].abs().max()) for k in vk)
    err, own = {}, {}
    for k in keys:
        x, y = a.field64(k)[owned(k)], b.field64(k)[owned(k)]
        d, ymax = float((x - y).abs().max()), float(y.abs().max())
        err[k] = d / (vmax if k in vk else ymax)
        if k in vk:
            own[k] = d / ymax if ymax > 0 else d
        del x, y
    return err, own


def owned_slices(p):
    """What a step defines: active zones, and the owned Y/Z faces (interior
    faces; the radial and vertical sides of the disks are not periodic)."""
    d3 = p["nz"] > 1
    ks = slice(NGH, NGH + p["nz"]) if d3 else slice(0, 1)
    js = slice(NGH, NGH + p["ny"])
    reg = {"vy": (ks, slice(NGH + 1, NGH + p["ny"]), slice(None)),
           "vz": (slice(NGH + 1, NGH + p["nz"]), js, slice(None))}
    return lambda k: reg.get(k, (ks, js, slice(None)))


def batch_variant(steps, warmup, tune=True, err_steps=100):
    """The parameter sweep of 256 uneven viscous disks (N_r in 64..512,
    N_phi = 3 N_r, alpha viscosity), same disks and steps in six forms: the
    FP64 and FP32-bulk steps called disk by disk; both advanced by one captured
    graph of the disks' own steps per step (autotuned graph width and sweep
    chunk); and both in the fused form, each kernel of the step launched once
    over all disks (sweep chunk autotuned per size class); then the FP32 disks
    against the FP64 ones after err_steps steps at equal times (each FP32 disk
    takes its FP64 twin's time steps)."""
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

    def solvers(precision):
        out = []
        for p in probs:
            sv = F.Solver(dict(p.params, precision=precision))
            sv.upload(p.fields)
            out.append(sv)
        return out

    out = {}
    for prec in ("fp64", "fp32"):
        ss = solvers(prec)
        step = lambda: [sv.fargo_step(0.0) for sv in ss]
        for _ in range(warmup):
            step()
        el = timed(step, steps)
        out[prec + "_disk_by_disk"] = {"value": cells * steps / el, "ms_per_step": 1e3 * el / steps}
        b = F.Batch(ss, lanes=8)
        best = b.fargo_batch_tune(lanes=(1, 4, 8, 16), chunks=(16, 32, 64), steps=10) if tune else None
        for _ in range(warmup):
            b.fargo_batch_step()
        el = timed(b.fargo_batch_step, steps)
        for sv in ss:
            sv.fargo_check()
        out[prec + "_batched_graph"] = {"value": cells * steps / el, "ms_per_step": 1e3 * el / steps,
                                        "tuned": {"lanes": best[0], "chunk": best[1]} if best else None}
        del b
        # fused: every kernel of the step once over all disks
        b = F.Batch(ss, lanes=0)
        if tune:
            b.fargo_batch_tune(lanes=(0,), chunks=(8, 16, 32, 64), steps=10)
        ch = b.chunks()
        for _ in range(warmup):
            b.fargo_batch_step()
        el = timed(b.fargo_batch_step, steps)
        for sv in ss:
            sv.fargo_check()
        by_class = {}
        for p, c in zip(probs, ch):
            by_class.setdefault(int(math.floor(math.log2(p.params["ny"]))), c)
        out[prec + "_fused"] = {"value": cells * steps / el, "ms_per_step": 1e3 * el / steps,
                                "chunk_by_size_class": {"ny in [%d, %d)" % (2 ** k, 2 ** (k + 1)): c
                                                        for k, c in sorted(by_class.items())}}
        print("  %s: disk by disk %.3e, batched graph %.3e (tuned %s), fused %.3e cell-updates/s" % (
            prec, out[prec + "_disk_by_disk"]["value"], out[prec + "_batched_graph"]["value"], best,
            out[prec + "_fused"]["value"]), file=sys.stderr, flush=True)
        del b, ss
        torch.cuda.empty_cache()
    v = lambda k: out[k]["value"]
    out["speedup"] = {
        "fused_vs_disk_by_disk_fp64": v("fp64_fused") / v("fp64_disk_by_disk"),
        "fused_vs_disk_by_disk_fp32": v("fp32_fused") / v("fp32_disk_by_disk"),
        "fused_vs_graph_fp64": v("fp64_fused") / v("fp64_batched_graph"),
        "fused_vs_graph_fp32": v("fp32_fused") / v("fp32_batched_graph"),
        "precision_fused": v("fp32_fused") / v("fp64_fused"),
        "fp32_fused_vs_fp64_disk_by_disk": v("fp32_fused") / v("fp64_disk_by_disk"),
    }
    # FP32 against FP64 at equal times, disk by disk (a batch step equals the
    # disks' own steps bit for bit)
    worst = {}
    for d, p in enumerate(probs):
        a64 = F.Solver(dict(p.params, precision="fp64"))
        a64.upload(p.fields)
        a32 = F.Solver(dict(p.params, precision="fp32"))
        a32.upload(p.fields)
        for _ in range(err_steps):
            a64.fargo_step(0.0)
            a32.fargo_step(a64.fargo_get_dt())
        a64.fargo_check()
        a32.fargo_check()
        err, _ = field_errors(a32, a64, ("rho", "vx", "vy"), owned_slices(p.params))
        for k, e in err.items():
            worst[k] = max(worst.get(k, 0.0), e)
        del a64, a32
    torch.cuda.empty_cache()
    out["fp32_error_vs_fp64"] = {"steps": err_steps, "equal_times": True, "max_over_disks":
                                 {k: float("%.3g" % e) for k, e in worst.items()}}
    out["disks"] = len(probs)
    out["active_cells"] = cells
    out["unit"] = "cell-updates/s"
    print("  batch speedups %s, fp32 error %s" % (out["speedup"], out["fp32_error_vs_fp64"]),
          file=sys.stderr, flush=True)
    return out


MFMA_BF16_PEAK_TFLOPS = 2500.0  # MI355X dense bf16 matrix peak


def copy_bandwidth():
    """Bytes read plus written per second by a plain 1 GiB device copy, timed
    with HIP events: torch's copy kernel, and the library's hand-written
    streaming copy (16-byte vectors, four per thread per round over a grid of
    several sizes, or one per thread), the best of which is the practical
    HBM ceiling a kernel reaches on this GPU (the vendor peak is 8 TB/s)."""
    import torch
    from paper_1602_02359_amd import fargo as F
    src = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    nb = 2 * src.nbytes

    def rate(fn, reps=10):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return nb / (a.elapsed_time(b) / reps * 1e-3) / 1e9

    out = {"torch_copy_GBs": rate(lambda: dst.copy_(src))}
    grid = {}
    for blocks in (8192, 32768, 131072, 0):  # 0: one thread per 16-byte vector
        grid[blocks] = rate(lambda: F.fargo_hbm_copy(src, dst, blocks))
    best = max(grid, key=grid.get)
    out["hip_stream_copy_GBs"] = grid[best]
    out["hip_stream_copy_blocks"] = best
    out["hip_stream_copy_by_blocks"] = {str(k): round(v, 1) for k, v in grid.items()}
    assert torch.equal(src, dst)
    del src, dst
    torch.cuda.empty_cache()
    return out


def pattern_bandwidth(nx, ny, nz, nin, nout, reps=5):
    """Bytes read plus written per second by the library's access-pattern
    probe with a column sweep's field counts (nin FP64 fields read, nout
    written, nx * ny * nz each): one (x, y) column per thread walking the
    planes, as the sweeps walk theirs, and one element per thread for
    comparison.  The column walk's rate is the ceiling of the sweep's memory
    access pattern with none of its arithmetic."""
    import torch
    from paper_1602_02359_amd import fargo as F
    n = nx * ny * nz
    ins = [torch.ones(n, dtype=torch.float64, device="cuda") for _ in range(nin)]
    outs = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(nout)]
    nb = (nin + nout) * 8 * n

    def rate(march):
        F.fargo_hbm_streams(ins, outs, nx, ny, nz, march)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            F.fargo_hbm_streams(ins, outs, nx, ny, nz, march)
        b.record()
        torch.cuda.synchronize()
        return nb / (a.elapsed_time(b) / reps * 1e-3) / 1e9

    out = {"fields_read": nin, "fields_written": nout, "shape": [nx, ny, nz],
           "column_march_GBs": round(rate(1), 1), "flat_GBs": round(rate(0), 1)}
    assert bool((outs[0] == 2.0).all())
    del ins, outs
    torch.cuda.empty_cache()
    return out


LFC_BATCH = 8  # training samples per Adam step


def lfc_variant(iters=600, batch=LFC_BATCH):
    """The learned flux correction on the planet disks (coarse 768 x 256,
    fine 3072 x 1024): 40 samples along one fine trajectory (after 200 fine
    spin-up steps), 32 for training and 8 held out, `batch` samples per Adam
    step.  Adam steps are timed with per-kernel HIP events; the held-out error
    of the corrected coarse step (|drho - target| / |target|, 1 = the plain
    step) before and after."""
    import torch
    from paper_1602_02359_amd import learned as LN
    t0 = time.perf_counter()
    cp, samples = LN.make_samples(40, spinup=200, medium=True)
    torch.cuda.synchronize()
    gen = time.perf_counter() - t0
    sc = LN.scales(cp, samples)
    tr = LN.Trainer(cp, sc, batch=batch)
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
    # against the plain FP64 solver: the coarse step with and without the
    # correction, and the plain solver at twice the resolution (its result
    # averaged onto the coarse mesh), on the held-out intervals
    from paper_1602_02359_amd import fargo as F
    from paper_1602_02359_amd import workloads as W

    def step_ms(prob, nsteps=50):
        sv = F.Solver(prob.params)
        sv.upload(prob.fields)
        for _ in range(3):
            sv.fargo_step(0.0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(nsteps):
            sv.fargo_step(0.0)
        torch.cuda.synchronize()
        sv.fargo_check()
        return 1e3 * (time.perf_counter() - t) / nsteps

    med = LN.medium_error(held)
    msteps = sum(s["medium_steps"] for s in held) / len(held)
    cpp = cp.params
    t_coarse = step_ms(cp)
    t_medium = step_ms(W.disk2d_planet(nx=2 * cpp["nx"], ny=2 * cpp["ny"]))
    equal_error = {
        "metric": "relative error of the density after one coarse interval against the 4x-finer solution "
                  "averaged onto the coarse mesh (1 = the plain coarse step), held-out intervals",
        "plain_coarse": {"relative_error": 1.0, "ms_per_interval": t_coarse,
                         "coarse_cell_updates_per_s": npix / (t_coarse * 1e-3)},
        "corrected_coarse": {"relative_error": after["relative_error"], "ms_per_interval": t_coarse + apply_ms,
                             "coarse_cell_updates_per_s": npix / ((t_coarse + apply_ms) * 1e-3)},
        "plain_2x": {"relative_error": med["relative_error"], "steps_per_interval": msteps,
                     "ms_per_interval": msteps * t_medium,
                     "coarse_cell_updates_per_s": npix / (msteps * t_medium * 1e-3)},
    }
    print("  lfc equal error: corrected coarse %.3f at %.3f ms, plain 2x %.3f at %.3f ms per interval" % (
        after["relative_error"], t_coarse + apply_ms, med["relative_error"], msteps * t_medium),
        file=sys.stderr, flush=True)
    # algorithmic flops of each convolution of a training step over the
    # batch (unpadded GEMM dimensions: outputs x reduction length x 2)
    P = float(npix * batch)
    fl = {"lfc_fwd_l1": 2.0 * P * 32 * 36, "lfc_fwd_l2": 2.0 * P * 32 * 288, "lfc_fwd_l3": 2.0 * P * 2 * 288,
          "lfc_adj_l3": 2.0 * P * 32 * 18, "lfc_adj_l2": 2.0 * P * 32 * 288,
          "lfc_wgrad_l3": 2.0 * P * 2 * 288, "lfc_wgrad_l2": 2.0 * P * 32 * 288, "lfc_wgrad_l1": 2.0 * P * 32 * 36}
    # and their algorithmic bytes (each input read once, each output written
    # once): activations and layer gradients 2 bytes a channel, features and
    # the last layer's gradient 4 channels, the FP32 output 8 bytes a pixel
    by = {"lfc_fwd_l1": 8 + 64, "lfc_fwd_l2": 64 + 64, "lfc_fwd_l3": 64 + 8, "lfc_adj_l3": 8 + 64 + 64,
          "lfc_adj_l2": 64 + 64 + 64, "lfc_wgrad_l3": 8 + 64, "lfc_wgrad_l2": 64 + 64, "lfc_wgrad_l1": 64 + 8}
    kern = {}
    for name, (cnt, tot) in tim.items():
        e = {"launches": cnt, "avg_ms": tot / cnt, "ms_per_train_step": tot / iters}
        if name in fl:
            e["TFLOPs"] = fl[name] * iters / (tot * 1e-3) / 1e12
            e["GBs"] = P * by[name] * iters / (tot * 1e-3) / 1e9
            e["flop_per_byte"] = fl[name] / (P * by[name])
        kern[name] = e
    dom = max((k for k in kern if "TFLOPs" in kern[k]), key=lambda k: kern[k]["ms_per_train_step"])
    # the roof that binds: the matrix peak, or HBM bandwidth times the
    # kernel's arithmetic intensity (the bf16 ridge is 2500 / 8 = 312 flop/byte)
    hbm_bound = HBM_PEAK_GBS * 1e-3 * kern[dom]["flop_per_byte"] < MFMA_BF16_PEAK_TFLOPS
    out = {
        "workload": "learned flux correction, planet disk: coarse 768x256 (196608 zones), fine 3072x1024, "
                    "3 conv layers 4-32-32-2, bf16 MFMA, %d samples per training step" % batch,
        "batch": batch,
        "ms_per_train_step": 1e3 * el / iters,
        "train_steps_per_s": iters / el,
        "train_samples_per_s": iters * batch / el,
        "ms_per_apply": apply_ms,
        "sample_generation_s": gen,
        "heldout_relative_error": {"before": before["relative_error"], "after": after["relative_error"]},
        "train_relative_error_after": after_train["relative_error"],
        "against_plain_solver": equal_error,
        "train_steps": 20 + 2 * iters,
        "kernels": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kern.items()},
        "roofline": ({"bound": "hbm", "kernel": dom, "achieved": round(kern[dom]["GBs"], 1), "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "frac": kern[dom]["GBs"] / HBM_PEAK_GBS, "traffic": None,
                      "flop_per_byte": kern[dom]["flop_per_byte"], "TFLOPs": round(kern[dom]["TFLOPs"], 3),
                      "frac_of_bf16_mfma_peak": kern[dom]["TFLOPs"] / MFMA_BF16_PEAK_TFLOPS}
                     if hbm_bound else
                     {"bound": "mfma", "kernel": dom, "achieved": round(kern[dom]["TFLOPs"], 3),
                      "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                      "frac": kern[dom]["TFLOPs"] / MFMA_BF16_PEAK_TFLOPS, "traffic": None}),
    }
    print("  lfc: %.3f ms per training step, %.3f ms per apply; held-out error %.3f -> %.3f; %s %.2f TFLOP/s" % (
        out["ms_per_train_step"], apply_ms, before["relative_error"], after["relative_error"], dom,
        kern[dom]["TFLOPs"]), file=sys.stderr, flush=True)
    del tr, samples
    torch.cuda.empty_cache()
    return out


_PROBS = {}


def problem(name):
    """The seeded workload, generated once (its host arrays are kept)."""
    from paper_1602_02359_amd import workloads as W
    if name not in _PROBS:
        _PROBS[name] = W.make(name)
    return _PROBS[name]


def run_workload(name, precision, steps, warmup, fargo=None, kernel_steps=5, keep=False):
    """Upload the workload, warm up, time `steps` steps with kernel timing off,
    then `kernel_steps` more with per-kernel HIP events on the launch stream.
    Returns the figures (and the solver, if keep)."""
    import torch
    from paper_1602_02359_amd import fargo as F
    prob = problem(name)
    p = dict(prob.params, precision=precision)
    if fargo is not None:
        p["fargo"] = bool(fargo)
    cells = prob.active_cells
    print("workload %s %dx%dx%d %s fargo=%s" % (name, p["nx"], p["ny"], p["nz"], precision, p["fargo"]),
          file=sys.stderr, flush=True)
    solver = F.Solver(p)
    solver.upload(prob.fields)
    for _ in range(warmup):
        solver.fargo_step(0.0)
    solver.fargo_check()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        solver.fargo_step(0.0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    solver.fargo_check()
    value = cells * steps / el
    r = {"value": value, "ms_per_step": 1e3 * el / steps, "active_cells": cells,
         "dt_last": solver.fargo_get_dt()}
    # per-kernel means, in a pass of their own
    wpu = words_per_unit(p)
    wb = 4.0 if precision == "fp32" else 8.0
    solver.fargo_profile_enable(True)
    for _ in range(kernel_steps):
        solver.fargo_step(0.0)
    timings = solver.fargo_timings()
    solver.fargo_profile_enable(False)
    kern = {}
    for kname, (cnt, tot) in timings.items():
        e = {"launches": cnt, "avg_ms": tot / cnt}
        if kname in wpu and wpu[kname][0] > 0:
            e["alg_bytes"] = wb * wpu[kname][0] * wpu[kname][1]
            e["GBs"] = e["alg_bytes"] / (e["avg_ms"] * 1e-3) / 1e9
        kern[kname] = e
    dom = max((k for k in kern if "alg_bytes" in kern[k]), key=lambda k: kern[k]["avg_ms"] * kern[k]["launches"])
    step_alg = sum(e["alg_bytes"] * e["launches"] for e in kern.values() if "alg_bytes" in e) / kernel_steps
    r.update({"kernels": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                          for k, v in kern.items()},
              "dominant": dom, "step_alg_bytes_per_cell": step_alg / cells,
              "step_alg_GBs": value * step_alg / cells / 1e9})
    tag = "%s_%dx%dx%d_%s" % (name, p["nx"], p["ny"], p["nz"], precision)
    r["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": round(kern[dom]["GBs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(kern[dom]["GBs"] / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom, tag), "alg_bytes_per_launch": kern[dom]["alg_bytes"],
                     "avg_launch_ms": kern[dom]["avg_ms"]}
    print("  %.3f ms/step, %.3e cell-updates/s; dominant %s %.4f ms, %.0f GB/s" % (
        r["ms_per_step"], value, dom, kern[dom]["avg_ms"], kern[dom]["GBs"]), file=sys.stderr, flush=True)
    for kname, e in sorted(kern.items(), key=lambda kv: -kv[1]["avg_ms"] * kv[1]["launches"]):
        print("    %-16s %5d launches %9.4f ms avg  %s" % (kname, e["launches"], e["avg_ms"],
              ("%.0f GB/s" % e["GBs"]) if "GBs" in e else ""), file=sys.stderr)
    if keep:
        return r, solver
    del solver
    torch.cuda.empty_cache()
    return r, None


def fp32_error(name, nsteps=100):
    """FP32 bulk against FP64 after nsteps from the same FP64 initial state,
    at equal times (the FP32 run takes the FP64 run's time steps)."""
    import torch
    from paper_1602_02359_amd import fargo as F
    prob = problem(name)
    p = prob.params
    a64 = F.Solver(dict(p, precision="fp64"))
    a64.upload(prob.fields)
    a32 = F.Solver(dict(p, precision="fp32"))
    a32.upload(prob.fields)
    t_sim = 0.0
    for n in range(nsteps):
        a64.fargo_step(0.0)
        dt = a64.fargo_get_dt()
        t_sim += dt
        a32.fargo_step(dt)
        if n % 25 == 24:
            print("  fp32 vs fp64 %s: step %d" % (name, n + 1), file=sys.stderr, flush=True)
    a64.fargo_check()
    a32.fargo_check()
    keys = ("rho", "e", "vx", "vy", "vz") if p["eos"] == "adi" else ("rho", "vx", "vy", "vz")
    err, own = field_errors(a32, a64, keys, owned_slices(p))
    del a64, a32
    torch.cuda.empty_cache()
    out = {"steps": nsteps, "equal_times": True, "time_advanced": t_sim,
           "normwise": {k: float("%.3g" % v) for k, v in err.items()},
           "velocity_own_scale": {k: float("%.3g" % v) for k, v in own.items()}}
    print("  fp32 error after %d steps: %s" % (nsteps, out["normwise"]), file=sys.stderr, flush=True)
    return out


def physical_time_rate(name, steps, warmup, fargo):
    """Physical time advanced per second of wall time, with orbital advection
    on or off: the timed rate of whole steps times the mean time step of the
    same steps (read back after the timed region)."""
    import torch
    from paper_1602_02359_amd import fargo as F
    prob = problem(name)
    p = dict(prob.params, fargo=bool(fargo))
    s = F.Solver(p)
    s.upload(prob.fields)
    for _ in range(warmup):
        s.fargo_step(0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.fargo_step(0.0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    dts = []
    for _ in range(steps):
        s.fargo_step(0.0)
        dts.append(s.fargo_get_dt())
    s.fargo_check()
    del s
    torch.cuda.empty_cache()
    mdt = sum(dts) / len(dts)
    return {"ms_per_step": 1e3 * el / steps, "mean_dt": mdt, "time_per_s": mdt * steps / el}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="cyl3d_planet", choices=["cyl3d_planet", "sph3d", "disk2d"])
    ap.add_argument("--kernel-steps", type=int, default=5, help="steps of the per-kernel timing pass")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"],
                    help="state of the headline run (fp32: for profiling the FP32-bulk kernels)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-side", action="store_true", help="skip the other two FP64 workloads")
    ap.add_argument("--no-variant", action="store_true",
                    help="skip FP32 bulk, FARGO on/off, the disk batch and the learned correction")
    ap.add_argument("--no-batch", action="store_true", help="skip the disk-batch variant")
    ap.add_argument("--no-lfc", action="store_true", help="skip the learned-flux-correction variant")
    ap.add_argument("--fp32-steps", type=int, default=100, help="steps of the FP32-vs-FP64 comparison")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one plain device copy of 2 GiB first (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library's step runs on one device; the multi-GPU slab "
              "decomposition is a design, not a measured path", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe:
        src = torch.ones(2 ** 28, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("copy probe: %d bytes read, %d bytes written" % (src.numel() * 8, dst.numel() * 8), file=sys.stderr)
        del src, dst
        torch.cuda.empty_cache()
    hbm = copy_bandwidth()
    print("device copy: torch %.0f GB/s, hand-written %.0f GB/s (read + write)" % (
        hbm["torch_copy_GBs"], hbm["hip_stream_copy_GBs"]), file=sys.stderr, flush=True)

    head, _ = run_workload(args.config, args.precision, args.steps, args.warmup, kernel_steps=args.kernel_steps)
    p = problem(args.config).params
    cells = problem(args.config).active_cells
    ceiling = hbm["hip_stream_copy_GBs"]
    hbm.update({"step_alg_bytes_per_cell": head["step_alg_bytes_per_cell"], "step_alg_GBs": head["step_alg_GBs"],
                "step_alg_frac_of_peak": head["step_alg_GBs"] / HBM_PEAK_GBS,
                "step_alg_frac_of_copy_ceiling": head["step_alg_GBs"] / ceiling,
                "compulsory_bytes_per_cell": compulsory_bytes(p),
                "effective_GBs": head["value"] * compulsory_bytes(p) / 1e9})
    roof = head["roofline"]
    roof["frac_of_copy_ceiling"] = round(roof["achieved"] / ceiling, 4)
    if args.precision == "fp64" and "sweep_z" in head["kernels"] and "ring_x" in head["kernels"]:
        # the ceilings of the two largest kernels' own access patterns: the Z
        # sweep reads density, v_z and NQ conserved fields and writes density
        # and the NQ fields (2 NQ + 3 words a zone), one column per thread;
        # the X transport reads density, v_x and NQ fields and writes NQ (the
        # Y/Z momenta, e, density and v_x: 2 NQ + 2 words), consecutive zones
        # per wave
        kz, kx = head["kernels"]["sweep_z"], head["kernels"]["ring_x"]
        nqz = (round(kz["alg_bytes"] / (cells * 8)) - 3) // 2
        nqx = (round(kx["alg_bytes"] / (cells * 8)) - 2) // 2
        pats = {"sweep_z": dict(pattern_bandwidth(p["nx"], p["ny"], p["nz"], nqz + 2, nqz + 1), walk="column"),
                "ring_x": dict(pattern_bandwidth(p["nx"], p["ny"], p["nz"], nqx + 2, nqx), walk="flat")}
        for name, pat in pats.items():
            ceil_k = pat["column_march_GBs"] if pat["walk"] == "column" else pat["flat_GBs"]
            pat["kernel_GBs"] = head["kernels"][name]["GBs"]
            pat["kernel_frac"] = round(pat["kernel_GBs"] / ceil_k, 4)
            print("access pattern of %s (%d read, %d written): column walk %.0f GB/s, flat %.0f GB/s; "
                  "%s at %.3f of the %s walk" % (name, pat["fields_read"], pat["fields_written"],
                                                  pat["column_march_GBs"], pat["flat_GBs"], name, pat["kernel_frac"],
                                                  pat["walk"]), file=sys.stderr, flush=True)
        roof["pattern_ceilings"] = pats
        if roof["kernel"] in pats:
            roof["frac_of_pattern_ceiling"] = pats[roof["kernel"]]["kernel_frac"]

    side = {}
    if not args.no_side:
        for name in ("sph3d", "disk2d"):
            if name == args.config:
                continue
            r, _ = run_workload(name, "fp64", args.steps, args.warmup, kernel_steps=args.kernel_steps)
            side[name] = r

    variants = {}
    if not args.no_variant:
        fp32 = {}
        for name in ("cyl3d_planet", "sph3d"):
            r, _ = run_workload(name, "fp32", args.steps, args.warmup, kernel_steps=args.kernel_steps)
            fp64v = head["value"] if name == args.config else side.get(name, {}).get("value")
            r["speedup_vs_fp64"] = r["value"] / fp64v if fp64v else None
            r["error_vs_fp64"] = fp32_error(name, args.fp32_steps)
            fp32[name] = r
        variants["fp32_bulk"] = fp32
        on = physical_time_rate(args.config, args.steps, args.warmup, True)
        off = physical_time_rate(args.config, args.steps, args.warmup, False)
        variants["physical_time_per_s"] = {"workload": args.config, "fargo_on": on, "fargo_off": off,
                                           "gain": on["time_per_s"] / off["time_per_s"]}
        print("  physical time per second: fargo on %.4g, off %.4g (x%.1f)" % (
            on["time_per_s"], off["time_per_s"], on["time_per_s"] / off["time_per_s"]), file=sys.stderr, flush=True)
        if not args.no_batch:
            variants["disk_batch"] = batch_variant(args.steps, args.warmup)
        if not args.no_lfc:
            variants["learned_flux_correction"] = lfc_variant()

    cpu = None
    if not args.no_cpu_baseline:
        print("timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(problem(args.config))
        print("  oracle %.3e cell-updates/s on %d threads, %.3e on one" % (
            cpu["value"], cpu["cores"], cpu["one_core"]["value"]), file=sys.stderr)

    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 bulk (f64 time step, split, sums)",
        "data": "synthetic",
        "config": {
            "workload": "%s: %s %dx%dx%d (phi, r, %s), %s, orbital advection %s, dt on device" % (
                args.config, p["geometry"], p["nx"], p["ny"], p["nz"], "theta" if p["geometry"] == "sph" else "z",
                "adiabatic" if p["eos"] == "adi" else "isothermal", "on" if p["fargo"] else "off") +
                ("" if args.precision == "fp64" else " (FP32-bulk state)"),
            "active_cells": cells,
            "parallelism": "single GPU",
        },
        "hbm": hbm,
        "kernels": head["kernels"],
        "roofline": roof,
        "cpu_baseline": cpu,
        "other_workloads_fp64": side,
        "variants": variants,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
