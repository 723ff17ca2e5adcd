"""FP32-bulk state (precision "fp32") through the C ABI.

What stays FP64 is checked exactly: the time step (formed in FP64 from the
stored FP32 values) and each ring's v0, N and xi equal the oracle's on the
same stored values in FP64; circular shifts are bit-exact permutations and
the conserved sums match the oracle's FP64 sums of the stored state.  The
bulk arithmetic is FP32: one step is compared with the oracle on the stored
input, and 100 steps with the plain FP64 GPU step from the same FP64 initial
state, normwise with velocities scaled by the largest speed (the error is
reported for every field, and per velocity component), within 1e-5.  The two
runs are compared at equal times: the FP32 run takes the time steps of the
FP64 run.  Left to its own CFL steps, the FP32 run drifts in time by a few
1e-6 relative (the artificial-viscosity term of the time step divides by
velocity differences), checked at 1e-4.

The FP32 state stores v_x, and transports the X momenta, as deviations from
an FP64 per-ring background (each ring's mean of the initial v_x).  Stored
in full, v_x would be rounded to eps v_K (eps = 6e-8) in every zone at every
step, an error that enters the divergence of the residual velocity scaled by
the step's full-velocity Courant number (about 6 under orbital advection):
some 4e-7 of density per step, 1e-5 to 6e-5 after 100 steps (measured
before the change).  As deviations, the rounding is relative to the
deviation, orders of magnitude smaller.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1602_02359_amd import workloads as W
from gpu_common import dt_close, errors, errors_own, owned

pytestmark = pytest.mark.gpu

TOL_100 = 1e-5     # FP32 bulk vs FP64 after 100 steps
# One step: a chain of some thirty FP32 roundings (unit 6e-8), amplified by at
# most ~50 where a gradient takes the difference of neighbouring values, and
# scaled by the step's relative change (< 1): a few 1e-7 at most.
TOL_ONE = 2e-6


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _solver(prob, precision):
    from paper_1602_02359_amd import fargo as F
    s = F.Solver(dict(prob.params, precision=precision))
    s.upload(prob.fields)
    return s


def _stored(s):
    """The FP32 state as stored, in FP64 (exact; v_x in full, background
    added in FP64 as the library does), with the FP64 potential."""
    return s.download()


def _small(name):
    if name == "sph3d":
        return W.disk3d_sph(nx=136, ny=19, nz=11, noise=1e-3)
    if name == "cyl3d_planet":
        return W.disk3d_cyl_planet(nx=150, ny=23, nz=9, noise=1e-3)
    if name == "disk2d":
        return W.disk2d_cyl(nx=200, ny=37, noise=1e-3)
    if name == "cart_random":
        return W.random_problem("cart", nx=70, ny=9, nz=7, eos="adi", seed=1)
    if name == "ring_2048":  # several ring segments per wave-group, FARGO shift
        return W.random_problem("cyl", nx=2048, ny=4, nz=1, eos="iso", seed=7, fargo=True)
    # 3D meshes go through the fused Z/X kernel: two chunks of planes (the
    # second ragged) and two ring segments with a ragged tail; then rings of
    # one and three zones
    if name == "cyl3d_chunks":
        return W.random_problem("cyl", nx=130, ny=5, nz=70, eos="adi", seed=21, fargo=True)
    if name == "ring_nx1_cyl3d":
        return W.random_problem("cyl", nx=1, ny=9, nz=6, eos="adi", seed=12, fargo=True)
    if name == "ring_nx3_sph3d":
        return W.random_problem("sph", nx=3, ny=9, nz=6, eos="adi", seed=14, fargo=True)
    if name == "ring_5000_cyl3d":  # the time-step pass in segments of a long ring
        return W.random_problem("cyl", nx=5000, ny=4, nz=3, eos="adi", seed=34, fargo=True)
    raise KeyError(name)


@pytest.mark.parametrize("name", ["sph3d", "cyl3d_planet", "disk2d", "cart_random", "ring_2048", "cyl3d_chunks",
                                  "ring_nx1_cyl3d", "ring_nx3_sph3d", "ring_5000_cyl3d"])
def test_fp32_one_step_vs_oracle(name):
    prob = _small(name)
    _say("fp32 one step", name, prob.params["nx"], prob.params["ny"], prob.params["nz"])
    s = _solver(prob, "fp32")
    up = _stored(s)
    ref = {k: (None if v is None else v.copy()) for k, v in up.items()}
    dt_ref = O.step(prob.params, ref)
    # box 6 runs in FP64 on the stored values: the oracle's step on the
    # upcast state, within the bound of the two codes' FP64 arithmetic
    dt = s.fargo_cfl_dt()
    assert dt_close(dt, dt_ref), (dt, dt_ref)
    s.fargo_step(dt_ref)
    s.fargo_check()
    got = s.download()
    err = errors(prob, got, ref)
    _say("  errors", err, "per component", errors_own(prob, got, ref))
    for k, e in err.items():
        assert e <= TOL_ONE, (k, e)


@pytest.mark.parametrize("name", ["sph3d", "cyl3d_planet", "disk2d"])
def test_fp32_hundred_steps_vs_fp64(name):
    prob = _small(name)
    _say("fp32 vs fp64, 100 steps", name)
    s64, s32, own = _solver(prob, "fp64"), _solver(prob, "fp32"), _solver(prob, "fp32")
    for _ in range(100):
        s64.fargo_step(0.0)
        s32.fargo_step(s64.fargo_get_dt())   # equal times
        own.fargo_step(0.0)                  # its own CFL steps
    for s in (s64, s32, own):
        s.fargo_check()
    b = s64.download()
    a = s32.download()
    err = errors(prob, a, b)
    err_own = errors(prob, own.download(), b)
    _say("  errors at equal times", err, "per component", errors_own(prob, a, b))
    _say("  errors with own time steps", err_own, "dt", own.fargo_get_dt(), s64.fargo_get_dt())
    for k, e in err.items():
        assert e <= TOL_100, (k, e)
    assert abs(own.fargo_get_dt() / s64.fargo_get_dt() - 1.0) < 1e-4


@pytest.mark.parametrize("name", ["sph3d", "disk2d"])
def test_fp32_ring_split_bit_exact(name):
    import torch
    prob = _small(name)
    s = _solver(prob, "fp32")
    vx = s.state["vx"]  # the stored deviation; the library adds the background
    up = s.download()["vx"]
    dt = 0.37 * O.cfl_dt(prob.params, _stored(s))
    v0, N, xi = s.fargo_ring_split(vx, dt)
    torch.cuda.synchronize()
    rv0, rN, rxi = O.ring_split(prob.params, up, dt)
    assert np.array_equal(N.cpu().numpy(), rN.ravel())
    assert np.array_equal(v0.cpu().numpy(), rv0.ravel())
    assert np.array_equal(xi.cpu().numpy(), rxi.ravel())


def test_fp32_shift_bit_exact():
    import torch
    prob = W.random_problem("cyl", nx=200, ny=6, nz=5, eos="iso", seed=11, fargo=True)
    s = _solver(prob, "fp32")
    p = prob.params
    rng = np.random.default_rng(5)
    nr = p["ny"] * p["nz"]
    N = rng.integers(-450, 450, size=nr).astype(np.int32)
    f = s.state["rho"].clone()
    before = f[:, :, :p["nx"]].double().cpu().numpy()
    s.fargo_shift(f, torch.from_numpy(N).to(f.device))
    torch.cuda.synchronize()
    after = f[:, :, :p["nx"]].double().cpu().numpy()
    O.shift(p, before, N.reshape(p["nz"], p["ny"]))
    assert np.array_equal(after, before)


@pytest.mark.parametrize("name", ["sph3d", "cyl3d_planet"])
def test_fp32_conserved_sums(name):
    prob = _small(name)
    s = _solver(prob, "fp32")
    s.fargo_cfl_dt()               # box 2 fill, as the oracle's sums expect
    got = s.fargo_conserved_sums()
    o, a = O.sums(prob.params, s.download())
    for q in range(5):
        assert abs(got[q] - o[q]) <= 1e-14 * max(a[q], 1e-300), (q, got[q], o[q])


def test_fp32_full_size_hundred_steps():
    """The 3D cylindrical planet disk at 2048x768x96: FP32 bulk vs the plain
    FP64 step after 100 steps, errors formed on the device."""
    import torch
    prob = W.make("cyl3d_planet")
    p = prob.params
    _say("fp32 vs fp64 full size", p["nx"], p["ny"], p["nz"])
    s64, s32 = _solver(prob, "fp64"), _solver(prob, "fp32")
    prob.fields = None  # host copy no longer needed
    for n in range(100):
        s64.fargo_step(0.0)
        s32.fargo_step(s64.fargo_get_dt())   # equal times
        if n % 25 == 24:
            torch.cuda.synchronize()
            _say("  step", n + 1)
    s64.fargo_check()
    s32.fargo_check()
    nx = p["nx"]
    vmax = max(float(s64.field64(k)[owned(prob, k)].abs().max()) for k in ("vx", "vy", "vz"))
    err, own = {}, {}
    for k in ("rho", "vx", "vy", "vz"):
        sl = owned(prob, k)
        a = s32.field64(k)[sl]
        b = s64.field64(k)[sl]
        bmax = float(b.abs().max())
        den = vmax if k.startswith("v") else bmax
        d = float((a - b).abs().max())
        err[k] = d / den
        if k.startswith("v"):
            own[k] = d / bmax
        del a, b
    _say("  errors", err, "per component", own, "dt", s32.fargo_get_dt(), s64.fargo_get_dt())
    for k, e in err.items():
        assert e <= TOL_100, (k, e)
