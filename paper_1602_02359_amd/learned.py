"""Learned flux correction: training data, training and evaluation on the
coarse and fine planet disks.

Orchestration of fargo_lfc_* and fargo_step calls.  The fine disk (4 x the
coarse resolution in each direction) is advanced by the plain FP64 solver;
at every sample its state is averaged 4 x 4 onto the coarse mesh, the coarse
solver takes one step from it, and the fine disk is advanced by the same time
step; the target is the density change that takes the coarse step to the
averaged fine state.  The net sees the coarse state after the plain step, so
that at run time a step is `fargo_step` followed by `fargo_lfc_apply`.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np
import torch

from . import fargo as F
from . import workloads as W

NGH = F.NGH
EVOLVING = ("rho", "vx", "vy")


def _copy_state(dst: F.Solver, src: F.Solver):
    for k in EVOLVING:
        dst.state[k].copy_(src.state[k])


def make_samples(count: int, seed: int = 4000, coarse: Dict = None, fine: Dict = None,
                 spinup: int = 0, medium: bool = False) -> Tuple[W.Problem, List[Dict[str, torch.Tensor]]]:
    """`count` consecutive (coarse state after the plain step, target) pairs
    along one fine trajectory.  `coarse` and `fine` are keyword arguments of
    the planet-disk generator (the defaults are 768 x 256 and 3072 x 1024).
    With `medium`, the plain solver at twice the coarse resolution also
    covers each interval from the fine state averaged 2 x 2 onto its mesh, and
    its result averaged 2 x 2 onto the coarse mesh is kept ("medium_rho",
    with its step count "medium_steps"): the plain solver's own answer at the
    next resolution, for comparison with the corrected coarse step."""
    cp = W.make("lfc_coarse", seed=seed, **(coarse or {}))
    fp = W.make("lfc_fine", seed=seed, **(fine or {}))
    fs = F.Solver(fp.params)
    fs.upload(fp.fields)
    cin, run, ref = (F.Solver(cp.params) for _ in range(3))
    for s in (cin, run, ref):
        s.upload(cp.fields)
    ms = mc = None
    if medium:
        cpp = cp.params
        mp = W.disk2d_planet(nx=2 * cpp["nx"], ny=2 * cpp["ny"], seed=seed)
        ms, mc = F.Solver(mp.params), F.Solver(cp.params)
        ms.upload(mp.fields)
        mc.upload(cp.fields)
    for _ in range(spinup):
        fs.fargo_step(0.0)
    n = cp.params["nx"] * cp.params["ny"]
    out = []
    for _ in range(count):
        F.lfc_restrict(fs, cin)
        if ms is not None:
            F.lfc_restrict(fs, ms)
        dt = cin.fargo_cfl_dt()
        _copy_state(run, cin)
        run.fargo_step(dt)
        # the fine disk covers the same interval in equal steps within its own limit
        nsub = max(1, math.ceil(dt / fs.fargo_cfl_dt() * (1.0 + 1e-12)))
        for _ in range(nsub):
            fs.fargo_step(dt / nsub)
        F.lfc_restrict(fs, ref)
        t = torch.empty(n, dtype=torch.float64, device=run.device)
        F.lfc_target(ref, run, t)
        smp = {"rho": run.state["rho"].clone(), "vx": run.state["vx"].clone(), "vy": run.state["vy"].clone(),
               "target": t, "dt": dt}
        if ms is not None:
            msub = max(1, math.ceil(dt / ms.fargo_cfl_dt() * (1.0 + 1e-12)))
            for _ in range(msub):
                ms.fargo_step(dt / msub)
            F.lfc_restrict(ms, mc)
            tm = torch.empty(n, dtype=torch.float64, device=run.device)
            F.lfc_target(mc, run, tm)  # the medium run's density change relative to the plain coarse step
            smp["medium_drho"] = tm
            smp["medium_steps"] = msub
        out.append(smp)
    for s in [fs, cin, run, ref] + ([ms, mc] if ms is not None else []):
        s.fargo_check()
    return cp, out


def medium_error(samples) -> Dict[str, float]:
    """Relative error of the plain solver at twice the coarse resolution in
    the metric of Trainer.evaluate: |drho_medium - target| / |target|."""
    rel = [float(torch.linalg.vector_norm(s["medium_drho"] - s["target"]) / torch.linalg.vector_norm(s["target"]))
           for s in samples]
    return {"relative_error": float(np.mean(rel)), "min": float(np.min(rel)), "max": float(np.max(rel))}


def init_params(seed: int) -> np.ndarray:
    """He-scaled normal weights (the last layer scaled down by 10), zero
    biases, in the parameter order of fargo_lfc_set_params."""
    rng = np.random.default_rng(seed)
    parts = []
    for n, (ci, co) in enumerate(((4, 32), (32, 32), (32, 2)), 1):
        std = math.sqrt(2.0 / (9 * ci)) * (0.1 if n == 3 else 1.0)
        parts.append((rng.standard_normal(co * 9 * ci) * std).astype(np.float32))
        parts.append(np.zeros(co, dtype=np.float32))
    v = np.concatenate(parts)
    assert v.size == F.LFC_NPARAM
    return v


def scales(cp: W.Problem, samples) -> Dict[str, float]:
    """Feature and output scales: sigma = the RMS target, flux_scale = sigma
    times the mean zone volume (so that a unit net output moves about sigma)."""
    p = cp.params
    y = p["ymin"]
    a, b = y[NGH:NGH + p["ny"]], y[NGH + 1:NGH + p["ny"] + 1]
    dx = (p["xmax"] - p["xmin"]) / p["nx"]
    vol = 0.5 * (b * b - a * a) * dx
    sq = sum(float((s["target"] ** 2).mean()) for s in samples) / len(samples)
    sigma = math.sqrt(sq) if sq > 0 else 1.0
    r_in, r_out = float(y[NGH]), float(y[NGH + p["ny"]])
    return dict(rho_s=1.0, u_s=0.05, r_mid=0.5 * (r_in + r_out), r_span=0.5 * (r_out - r_in),
                flux_scale=sigma * float(vol.mean()), sigma=sigma)


class Trainer:
    """A net bound to a coarse solver whose state is loaded from samples."""

    def __init__(self, cp: W.Problem, sc: Dict[str, float], seed: int = 7, guard: float = 0.5, batch: int = 1):
        self.feed = F.Solver(cp.params)
        self.feed.upload(cp.fields)
        self.batch = int(batch)
        self.net = F.LFC(self.feed, sc["rho_s"], sc["u_s"], sc["r_mid"], sc["r_span"], sc["flux_scale"],
                         sc["sigma"], guard, max_batch=self.batch)
        self.net.set_params(init_params(seed))

    def load(self, s):
        for k in EVOLVING:
            self.feed.state[k].copy_(s[k])

    def train(self, samples, iters: int, lr: float, seed: int = 0, every: int = 50) -> List[float]:
        """iters Adam steps, each on the next `batch` samples of a fixed
        random permutation of `samples` (cyclically)."""
        order = np.random.default_rng(seed).permutation(len(samples))
        losses = []
        b = self.batch
        for it in range(iters):
            if b == 1:
                s = samples[order[it % len(samples)]]
                self.load(s)
                self.net.train_step(s["target"], lr)
            else:
                self.net.train_batch([samples[order[(it * b + k) % len(samples)]] for k in range(b)], lr)
            if it % every == 0 or it == iters - 1:
                losses.append(self.net.result()[0])
        return losses

    def evaluate(self, samples) -> Dict[str, float]:
        """Relative error of the corrected coarse step, |drho - target| /
        |target| (1 = the plain step's own error), averaged over samples."""
        rel = []
        for s in samples:
            self.load(s)
            self.net.forward()
            d = self.net.views()["drho"].reshape(-1)
            t = s["target"]
            rel.append(float(torch.linalg.vector_norm(d - t) / torch.linalg.vector_norm(t)))
        return {"relative_error": float(np.mean(rel)), "min": float(np.min(rel)), "max": float(np.max(rel))}
