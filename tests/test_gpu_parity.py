"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars: integer work (shift amounts, circular shifts) and the ring split are
bit-exact; the time step agrees within the bound derived in gpu_common
(32 units in the last place: the oracle writes Eq. cfl2 as printed, the
library through rates); floating-point state is within 1e-12 normwise after
one step, as the target states, both with velocities normalised by the
largest speed and with each velocity component normalised by its own
largest value.  The state is compared at the oracle's time step, imposed on
the library, so that both take the same shift amounts.
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1602_02359_amd import workloads as W
from gpu_common import NG, dt_close, errors, errors_own, gpu_solver, sub_problem

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cases():
    yield "disk2d_small", lambda: W.disk2d_cyl(nx=200, ny=37, noise=1e-2)
    yield "disk2d_rot", lambda: W.disk2d_cyl(nx=130, ny=21, noise=3e-2, omega=1.0)
    yield "disk2d_nofargo", lambda: W.disk2d_cyl(nx=96, ny=17, noise=1e-2, fargo=False)
    yield "sph3d_small", lambda: W.disk3d_sph(nx=136, ny=19, nz=11, noise=1e-2)
    yield "cyl3d_planet_small", lambda: W.disk3d_cyl_planet(nx=150, ny=23, nz=9, noise=1e-2)
    yield "cart_random_reflect", lambda: W.random_problem("cart", nx=70, ny=9, nz=7, eos="adi", seed=1)
    yield "cart_random_periodic", lambda: W.random_problem("cart", nx=33, ny=8, nz=6, eos="iso", seed=2,
                                                          bc=("periodic",) * 4)
    yield "cart_random_outflow", lambda: W.random_problem("cart", nx=65, ny=7, nz=5, eos="adi", seed=3,
                                                         bc=("outflow", "reflect", "outflow", "outflow"))
    yield "cyl_random_fargo", lambda: W.random_problem("cyl", nx=300, ny=6, nz=5, eos="iso", seed=4, fargo=True,
                                                      omega=0.5, bc=("fixed", "outflow", "periodic", "periodic"))
    yield "sph_random_fargo", lambda: W.random_problem("sph", nx=257, ny=5, nz=4, eos="adi", seed=5, fargo=True,
                                                      omega=-0.3, bc=("reflect", "fixed", "fixed", "reflect"))
    yield "cyl2d_random_mean", lambda: _with(W.random_problem("cyl", nx=64, ny=12, nz=1, eos="adi", seed=6,
                                                              fargo=True), v0_mode="mean")
    yield "sod_y_nx1", lambda: W.sod("y", n=64)
    yield "sod_z", lambda: W.sod("z", n=40)
    yield "ring_2048", lambda: W.random_problem("cyl", nx=2048, ny=4, nz=1, eos="iso", seed=7, fargo=True)
    # rings above 2048 zones: the time-step kernel's 512-thread form
    yield "ring_3072", lambda: W.random_problem("cyl", nx=3072, ny=4, nz=1, eos="iso", seed=9, fargo=True)
    # degenerate rings: a single zone (axisymmetric), and rings shorter than
    # the stencils, whose neighbours wrap onto the zone itself
    yield "ring_nx1_cyl", lambda: W.random_problem("cyl", nx=1, ny=9, nz=6, eos="adi", seed=12, fargo=True)
    yield "ring_nx2_cart", lambda: W.random_problem("cart", nx=2, ny=9, nz=6, eos="adi", seed=13, fargo=True)
    yield "ring_nx3_sph", lambda: W.random_problem("sph", nx=3, ny=9, nz=6, eos="adi", seed=14, fargo=True)
    # two chunks of planes in the Z sweep (the second ragged), two ring segments
    yield "cyl3d_chunks", lambda: W.random_problem("cyl", nx=130, ny=5, nz=70, eos="adi", seed=21, fargo=True)
    # rings longer than one workgroup of the time-step pass holds: segments of
    # 1024 zones, the last one ragged; v0 by min/max and by the mean; 3D
    yield "ring_8192", lambda: W.random_problem("cyl", nx=8192, ny=4, nz=1, eos="iso", seed=31, fargo=True)
    yield "ring_5000_mean", lambda: _with(W.random_problem("cyl", nx=5000, ny=3, nz=1, eos="adi", seed=32,
                                                           fargo=True), v0_mode="mean")
    yield "ring_4500_sph3d", lambda: W.random_problem("sph", nx=4500, ny=4, nz=3, eos="adi", seed=33, fargo=True,
                                                      omega=0.2)


def _with(prob, **kw):
    prob.params.update(kw)
    return prob


CASES = dict(_cases())


@pytest.mark.parametrize("name", list(CASES))
def test_one_step_matches_oracle(name):
    prob = CASES[name]()
    _say("case", name, prob.shape)
    ref = prob.copy_fields()
    dt_ref = O.step(prob.params, ref)
    s = gpu_solver(prob)
    dt_gpu = s.fargo_cfl_dt()
    assert dt_close(dt_gpu, dt_ref), (dt_gpu, dt_ref)
    s.fargo_step(dt_ref)
    s.fargo_check()
    got = s.download()
    err, own = errors(prob, got, ref), errors_own(prob, got, ref)
    _say(name, "dt", dt_gpu, dt_ref, "errors", err, "per component", own)
    for k, e in err.items():
        assert e <= TOL, (k, e)
    for k, e in own.items():
        assert e <= TOL, (k, e)


@pytest.mark.parametrize("name", ["disk2d_small", "sph3d_small", "cart_random_periodic", "sph_random_fargo"])
def test_several_steps_match_oracle(name):
    """Five steps, each side with its own time step."""
    prob = CASES[name]()
    _say("case", name, prob.shape)
    ref = prob.copy_fields()
    s = gpu_solver(prob)
    for n in range(5):
        dt_ref = O.step(prob.params, ref)
        s.fargo_step(0.0)
        dt = s.fargo_get_dt()
        if n == 0:
            assert dt_close(dt, dt_ref), (dt, dt_ref)
        else:
            # the states now differ by rounding, and so may the time steps
            assert abs(dt / dt_ref - 1.0) < 1e-12, (n, dt, dt_ref)
    s.fargo_check()
    err = errors(prob, s.download(), ref)
    _say(name, err)
    for k, e in err.items():
        assert e <= 10 * TOL, (k, e)


def test_imposed_dt_and_cfl_readback():
    prob = CASES["sph3d_small"]()
    ref = prob.copy_fields()
    dt_ref = O.cfl_dt(prob.params, ref)
    s = gpu_solver(prob)
    assert dt_close(s.fargo_cfl_dt(), dt_ref)
    got0 = s.download()
    for k in ("rho", "vx", "vy", "vz", "e"):  # box 2 on both sides, ghosts included
        assert np.array_equal(got0[k], ref[k]), k
    dt = 0.7 * dt_ref
    O.step(prob.params, ref, dt)
    s.fargo_step(dt)
    assert s.fargo_get_dt() == dt
    err = errors(prob, s.download(), ref)
    for k, e in err.items():
        assert e <= TOL, (k, e)


@pytest.mark.parametrize("name", ["disk2d_small", "sph3d_small", "cyl_random_fargo", "cyl2d_random_mean"])
def test_ring_split_bit_exact(name):
    """v0, N and xi of Eq. 29 are bit-exact."""
    import torch
    prob = CASES[name]()
    s = gpu_solver(prob)
    for dt in (0.013, 0.0371, 1e-3):
        v0, N, xi = O.ring_split(prob.params, prob.fields["vx"], dt)
        g0, gN, gxi = s.fargo_ring_split(s.state["vx"], dt)
        torch.cuda.synchronize()
        if prob.params.get("v0_mode") == "mean":
            # summation order differs: v0 within rounding, N exact away from ties
            assert np.allclose(g0.cpu().numpy(), v0.ravel(), rtol=1e-14, atol=1e-15)
            assert np.array_equal(gN.cpu().numpy(), N.ravel())
            assert np.allclose(gxi.cpu().numpy(), xi.ravel(), rtol=0, atol=1e-12)
            continue
        assert np.array_equal(g0.cpu().numpy(), v0.ravel())
        assert np.array_equal(gN.cpu().numpy(), N.ravel())
        assert np.array_equal(gxi.cpu().numpy(), xi.ravel())


def test_split_ties_and_signs():
    """Nearest-integer ties (D = k + 1/2) go away from zero on both sides."""
    import torch
    p = W.default_params(geometry="cart", nx=16, ny=3, nz=1, xmin=0.0, xmax=16.0,
                         ymin=W.uniform_faces(0.0, 3.0, 3), zmin=np.array([0.0, 1.0]), fargo=True)
    pr = W._blank(p)
    vals = [2.5, -2.5, 0.5]
    for j, v in enumerate(vals):
        pr.fields["vx"][0, NG + j, :] = v
    s = gpu_solver(pr)
    v0, N, xi = s.fargo_ring_split(s.state["vx"], 1.0)
    torch.cuda.synchronize()
    assert N.cpu().tolist() == [3, -3, 1]
    assert xi.cpu().tolist() == [-0.5, 0.5, -0.5]
    ov0, oN, oxi = O.ring_split(p, pr.fields["vx"], 1.0)
    assert oN.ravel().tolist() == [3, -3, 1]


@pytest.mark.parametrize("nx,precision", [(1, "fp64"), (7, "fp64"), (64, "fp64"), (200, "fp64"), (2048, "fp64"),
                                          (8192, "fp64"), (8193, "fp64"), (20000, "fp64"), (16385, "fp32")])
def test_shift_bit_exact(nx, precision):
    """Eq. 32 as a pure permutation, equal to the oracle's, ghosts untouched
    (rings beyond 64 KiB through the out-of-place form)."""
    import torch
    prob = W.random_problem("cart", nx=nx, ny=5, nz=4, seed=8)
    if precision == "fp32":  # values representable in FP32, so the oracle's shift compares exactly
        prob.fields["rho"] = prob.fields["rho"].astype(np.float32).astype(np.float64)
    from paper_1602_02359_amd import fargo as F
    s = F.Solver(dict(prob.params, precision=precision))
    s.upload(prob.fields)
    rng = np.random.default_rng(nx)
    N = rng.integers(-3 * nx, 3 * nx + 1, size=(4, 5)).astype(np.int32)
    f = s.state["rho"]
    s.fargo_shift(f, torch.from_numpy(N.ravel()).to(f.device))
    got = f[:, :, :nx].double().cpu().numpy()
    ref = prob.fields["rho"].copy()
    O.shift(prob.params, ref, N)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("name", ["disk2d_small", "sph3d_small", "cart_random_periodic", "cyl_random_fargo"])
def test_conserved_sums(name):
    prob = CASES[name]()
    ref = prob.copy_fields()
    O.cfl_dt(prob.params, ref)
    s = gpu_solver(prob)
    s.fargo_cfl_dt()
    g = s.fargo_conserved_sums()
    o, a = O.sums(prob.params, ref)
    for q in range(5):
        assert abs(g[q] - o[q]) <= 1e-14 * max(a[q], 1e-300), (q, g[q], o[q])


def test_deterministic():
    prob = CASES["sph3d_small"]()
    outs = []
    for _ in range(2):
        s = gpu_solver(prob)
        for _ in range(3):
            s.fargo_step(0.0)
        outs.append(s.download())
    for k in outs[0]:
        if outs[0][k] is not None:
            assert np.array_equal(outs[0][k], outs[1][k]), k


def test_errors_reported():
    from paper_1602_02359_amd import fargo as F
    prob = W.random_problem("cart", nx=16, ny=5, nz=4, seed=9)
    bad = dict(prob.params, ny=2)
    with pytest.raises(F.FargoError) as e:
        F.Solver(bad)
    assert e.value.code == -1
    f = prob.copy_fields()
    f["rho"][NG + 1, NG + 1, 3] = np.nan
    s = gpu_solver(W.Problem("nan", prob.params, f))
    s.fargo_step(0.0)
    with pytest.raises(F.FargoError) as e:
        s.fargo_check()
    assert e.value.code == -4
    # error word cleared after the report
    s2 = gpu_solver(prob)
    s2.fargo_step(0.0)
    s2.fargo_check()


# ---------------------------------------------------------------------------
# Full-size configurations, in the launch configuration the benchmark times:
# time step bit-exact over the whole mesh, state checked on sampled sub-blocks
# that the oracle recomputes with the real neighbouring data as ghosts.
# ---------------------------------------------------------------------------

MARGIN = 6


def _blocks(p):
    ny, nz = p["ny"], p["nz"]
    w = 10
    ys = [(NG, NG + w + MARGIN), (NG + ny // 2 - w // 2 - MARGIN, NG + ny // 2 + w // 2 + MARGIN),
          (NG + ny - w - MARGIN, NG + ny)]
    if nz == 1:
        return [(y, None) for y in ys]
    zs = [(NG, NG + w + MARGIN), (NG + nz // 2 - w // 2 - MARGIN, NG + nz // 2 + w // 2 + MARGIN),
          (NG + nz - w - MARGIN, NG + nz)]
    return [(ys[0], zs[1]), (ys[1], zs[0]), (ys[1], zs[1]), (ys[2], zs[2])]


def _inner(p, sub_p, jr, kr):
    """Slices of the sub-block result (and of the full arrays) that are exact."""
    ja, jb = jr
    lo = 0 if ja == NG else MARGIN
    hi = 0 if jb == NG + p["ny"] else MARGIN
    sj = slice(NG + lo, NG + sub_p["ny"] - hi)
    fj = slice(ja + lo, jb - hi)
    if p["nz"] == 1:
        return (slice(0, 1), sj), (slice(0, 1), fj)
    ka, kb = kr
    lo = 0 if ka == NG else MARGIN
    hi = 0 if kb == NG + p["nz"] else MARGIN
    return (slice(NG + lo, NG + sub_p["nz"] - hi), sj), (slice(ka + lo, kb - hi), fj)


@pytest.mark.parametrize("cfg", ["sph3d", "cyl3d_planet", "disk2d"])
def test_full_size_sampled(cfg):
    import torch
    prob = W.make(cfg)
    p = prob.params
    _say("full-size", cfg, prob.shape, "cells", prob.active_cells)
    f0 = prob.fields
    full = {k: (None if v is None else v.copy()) for k, v in f0.items()}
    dt_ref = O.cfl_dt(p, full)  # fills the ghosts of `full` (box 2)
    s = gpu_solver(prob)
    dt = s.fargo_cfl_dt()
    assert dt_close(dt, dt_ref), (dt, dt_ref)
    # v0, shift amounts and residuals of every ring at the library's time
    # step, against the oracle's split of the same velocities
    g0, gN, gxi = s.fargo_ring_split(s.state["vx"], dt)
    o0, oN, oxi = O.ring_split(p, full["vx"], dt)
    torch.cuda.synchronize()
    assert np.array_equal(g0.cpu().numpy(), o0.ravel())
    assert np.array_equal(gN.cpu().numpy(), oN.ravel())
    assert np.array_equal(gxi.cpu().numpy(), oxi.ravel())
    del g0, gN, gxi
    s.fargo_step(0.0)
    s.fargo_check()
    assert s.fargo_get_dt() == dt  # the step's own time step, formed on the device again
    got = s.download()
    del s
    torch.cuda.empty_cache()
    vmax = max(np.abs(full[k]).max() for k in ("vx", "vy", "vz") if full.get(k) is not None)
    worst = {}
    for jr, kr in _blocks(p):
        sub = sub_problem(prob, full, jr, kr)
        ref = sub.copy_fields()
        O.step(sub.params, ref, dt)
        (sk, sj), (fk, fj) = _inner(p, sub.params, jr, kr)
        for k in ("rho", "e", "vx", "vy", "vz"):
            if ref.get(k) is None:
                continue
            a = got[k][fk, fj, :]
            b = ref[k][sk, sj, :]
            den = vmax if k.startswith("v") else np.abs(full[k]).max()
            e = float(np.abs(a - b).max() / den)
            worst[k] = max(worst.get(k, 0.0), e)
    _say(cfg, "dt", dt, "sampled errors", worst)
    for k, e in worst.items():
        assert e <= TOL, (k, e)


def test_disk2d_full_ten_steps():
    """The 2D disk configuration at its full size (384 x 128) for the ten steps
    it is specified with, each side with its own time step."""
    prob = W.make("disk2d")
    _say("case disk2d full, 10 steps", prob.shape)
    ref = prob.copy_fields()
    s = gpu_solver(prob)
    for n in range(prob.steps):
        dt_ref = O.step(prob.params, ref)
        s.fargo_step(0.0)
        dt = s.fargo_get_dt()
        assert dt_close(dt, dt_ref) if n == 0 else abs(dt / dt_ref - 1.0) < 1e-12, (n, dt, dt_ref)
    s.fargo_check()
    err = errors(prob, s.download(), ref)
    _say("disk2d 10 steps", err)
    for k, e in err.items():
        assert e <= 10 * TOL, (k, e)


# Meshes of several thousand rings, so that the time-step pass runs many
# workgroups per compute unit and per XCD.  Its rings go in a logical order:
# logical ring L is in plane tile L // (16 ny), k fastest within the tile, and
# consecutive logical rings go to one XCD (about an eighth of them each).
def _many_ring_cases():
    yield "rings_cyl3d", "fp64", lambda: W.disk3d_cyl_planet(nx=256, ny=64, nz=66, noise=1e-2)
    yield "rings_cyl3d", "fp32", lambda: W.disk3d_cyl_planet(nx=256, ny=64, nz=66, noise=1e-2)
    yield "rings_2048", "fp64", lambda: W.random_problem("cyl", nx=2048, ny=40, nz=53, eos="iso", seed=11,
                                                         fargo=True)
    yield "rings_disk2d_visc", "fp64", lambda: W.disk2d_visc(nx=96, ny=4100)
    yield "rings_sph3d_mean", "fp64", lambda: _with(W.disk3d_sph(nx=320, ny=64, nz=70, noise=1e-2), v0_mode="mean")


def _logical_ring(L, ny, nz):
    tile, q = divmod(L, 16 * ny)
    kb = 16 * tile
    kt = min(16, nz - kb)
    return kb + q % kt, q // kt  # (k, j) counted from the first active plane and row


@pytest.mark.parametrize("name,precision,make", list(_many_ring_cases()),
                         ids=lambda v: v if isinstance(v, str) else "")
def test_cfl_many_rings(name, precision, make):
    """Every ring's v0 against the oracle (bit-exact for the min/max mode),
    and the time step with one zone's sound speed (or energy) raised 30-fold
    in rings at chosen places of the logical order (the first and last ring,
    both sides of the first XCD's share, one in the middle), so that each of
    those rings in turn sets dt: each ring's rate must come from its own
    zones."""
    prob = make()
    p = dict(prob.params, precision=precision)
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    nring = ny * nz
    r8 = (nring + 7) // 8
    qf = "cs" if p["eos"] == "iso" else "e"
    picks = [0, r8 - 1, r8, nring // 2 + 5, nring - 1]
    for L in picks:
        kk, jj = _logical_ring(L, ny, nz)
        _say(name, precision, "ring", L, "(j, k) =", (jj, kk))
        fields = prob.copy_fields()
        zk = NG + kk if nz > 1 else 0
        fields[qf][zk, NG + jj, nx // 3] *= 30.0
        from paper_1602_02359_amd import fargo as F
        s = F.Solver(p)
        s.upload(fields)
        dt = s.fargo_cfl_dt()
        full = s.download()  # the state as the library holds it, ghosts filled
        dt_ref = O.cfl_dt(p, full)
        assert dt_close(dt, dt_ref), (L, dt, dt_ref)
        if L == picks[0]:
            import torch
            g0, gN, gxi = s.fargo_ring_split(s.state["vx"], dt)
            torch.cuda.synchronize()
            v0, N, xi = O.ring_split(p, full["vx"], dt)
            if p.get("v0_mode") == "mean":
                assert np.allclose(g0.cpu().numpy(), v0.ravel(), rtol=1e-14, atol=1e-15)
            else:
                assert np.array_equal(g0.cpu().numpy(), v0.ravel())
        s.fargo_check()
