"""The radial (Y) slab decomposition of several GPUs (Sect. 4.1, 4.3), shown
on one GPU: a 3D planet disk split into two slabs that each run as their own
context, with the global time step the minimum of the slabs' CFL steps (the
all-reduce of a multi-GPU run) and the rows next to each cut refreshed from
the slab that owns them after every step (the halo exchange, here device
copies).  Each slab covers its own rows plus H overlap rows past each cut,
and its cut sides are FIXED: their three ghost rows hold the neighbour's
values and no step writes them.  A step's Y dependency cone is a few rows
(the source step's two-zone stencil, the boundary face it leaves at v^n and
the v'' ghosts it copies from v^n, the Y sweep's two upwind zones), so the
owned rows, H rows away from the slab's edge, must come out bit for bit as in
the unsplit run, and the minimum of the slabs' time steps must be the unsplit
run's own (every ring is an interior ring of some slab).
"""
import sys

import numpy as np
import pytest

from paper_1602_02359_amd import workloads as W

pytestmark = pytest.mark.gpu

NG = W.NGH


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _slab(prob, a, b):
    """Active rows [a, b) of prob as a problem of its own: whole rings, the
    real neighbours in the ghost rows, FIXED radial sides."""
    p = prob.params
    sub = dict(p)
    sub["ny"] = b - a
    sub["ymin"] = p["ymin"][a:b + 2 * NG + 1].copy()
    sub["bc"] = ("fixed", "fixed") + tuple(p["bc"][2:])
    f = {k: (None if v is None else v[:, a:b + 2 * NG, :].copy()) for k, v in prob.fields.items()}
    return W.Problem(prob.name + "_slab", sub, f, 1)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("H", [4, 8])
def test_two_slabs_equal_the_unsplit_mesh(precision, H):
    import torch
    from paper_1602_02359_amd import fargo as F
    prob = W.make("cyl3d_planet", nx=128, ny=40, nz=10, noise=1e-2)
    ny = prob.params["ny"]
    cut = ny // 2
    own = [(0, cut), (cut, ny)]
    ext = [(max(0, a - H), min(ny, b + H)) for a, b in own]  # each slab's active rows (overlap included)
    _say("slabs", own, "with overlap", H, precision)
    full = F.Solver(dict(prob.params, precision=precision))
    full.upload(prob.fields)
    slabs = []
    for a, b in ext:
        s = F.Solver(dict(_slab(prob, a, b).params, precision=precision))
        s.upload(_slab(prob, a, b).fields)
        slabs.append(s)
    fields = [k for k in ("rho", "vx", "vy", "vz", "e") if full.state.get(k) is not None]

    def rows(solver, a, b, lo, hi):
        """storage rows of the active rows [lo, hi) (full-mesh numbering) in a
        solver whose active rows are [a, b)"""
        return slice(lo - a + NG, hi - a + NG)

    for n in range(4):
        dts = [s.fargo_cfl_dt() for s in slabs]
        dt = min(dts)
        full.fargo_step(0.0)
        assert full.fargo_get_dt() == dt, (n, full.fargo_get_dt(), dts)
        for s in slabs:
            s.fargo_step(dt)
        torch.cuda.synchronize()
        # the owned rows against the unsplit run, bit for bit
        for (a, b), (ea, eb), s in zip(own, ext, slabs):
            for k in fields:
                got = s.state[k][:, rows(s, ea, eb, a, b), :]
                ref = full.state[k][:, rows(full, 0, ny, a, b), :]
                if not torch.equal(got, ref):
                    bad = (got != ref).nonzero()
                    raise AssertionError("step %d, %s, rows [%d, %d): %d values differ, first row %d" % (
                        n + 1, k, a, b, bad.shape[0], a + int(bad[:, 1].min())))
        # the overlap rows next to a cut are not the unsplit run's after a
        # step (a FIXED side is not a neighbour): the exchange below is what
        # keeps the slabs right; the depth of the wrong rows is printed
        for (a, b), (ea, eb), s in zip(own, ext, slabs):
            lo, hi = (ea, a) if ea < a else (b, eb)
            depth = 0
            for j in range(lo, hi):
                same = all(torch.equal(s.state[k][:, rows(s, ea, eb, j, j + 1), :],
                                       full.state[k][:, rows(full, 0, ny, j, j + 1), :]) for k in fields)
                if not same:  # rows counted from the slab's FIXED edge inwards
                    depth = max(depth, (hi - j) if lo == b else (j - lo + 1))
            if n == 0:
                _say("  slab rows [%d, %d): overlap rows that differ before the exchange: %d of %d" % (
                    a, b, depth, hi - lo))
            assert depth > 0
        # halo exchange: every row a slab does not own (its overlap and the
        # ghost rows of its cut side) from the slab that owns it
        for (ea, eb), s in zip(ext, slabs):
            lo, hi = max(0, ea - NG), min(ny, eb + NG)  # rows of the full mesh this slab stores
            for (a, b), (oa, ob), o in zip(own, ext, slabs):
                x0, x1 = max(lo, a), min(hi, b)
                if o is s or x0 >= x1:
                    continue
                for k in fields:
                    s.state[k][:, rows(s, ea, eb, x0, x1), :] = o.state[k][:, rows(o, oa, ob, x0, x1), :]
        torch.cuda.synchronize()
    for s in slabs + [full]:
        s.fargo_check()
