"""Shared test helpers: running the oracle to a time, reading golden files,
normwise errors.  No arithmetic of the method lives here."""
import os

import numpy as np

from paper_1602_02359_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()[:2]
            out[k] = float(v)
    return out


def oracle_run_to(O, prob, t_end, fields=None, max_steps=100000):
    """Advance with the oracle's own time step until t_end; returns (fields, nsteps)."""
    f = prob.copy_fields() if fields is None else fields
    t, n = 0.0, 0
    while t < t_end * (1.0 - 1e-14) and n < max_steps:
        g = {k: (None if v is None else v.copy()) for k, v in f.items()}
        dt = min(O.cfl_dt(prob.params, g), t_end - t)
        O.step(prob.params, f, dt)
        t += dt
        n += 1
    return f, n


def active(prob, a):
    """Active-zone view of a (nz_g, ny_g, nx) array."""
    p = prob.params
    k0 = W.NGH if p["nz"] > 1 else 0
    return a[k0:k0 + p["nz"], W.NGH:W.NGH + p["ny"], :]


def normwise(a, b):
    """||a - b||_inf / ||b||_inf (0 if both vanish)."""
    den = np.max(np.abs(b))
    num = np.max(np.abs(a - b))
    if den == 0.0:
        return float(num)
    return float(num / den)
