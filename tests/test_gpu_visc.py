"""Box 7d (kinematic viscosity, cylindrical 2D) and batches of uneven disks
through the C ABI.

The viscous step is compared with the FP64 oracle (time step within the bound
of gpu_common, state within 1e-12 normwise after one step at the oracle's
time step); the FP32-bulk form with the FP64 step
after 100 steps at 1e-5 (the FP32 bar of tests/test_gpu_fp32.py).  A batch step (one captured hipGraph over many disks)
must equal the disks' own steps bit for bit, and the autotuner must leave the
states as it found them.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1602_02359_amd import workloads as W
from gpu_common import dt_close, errors, errors_own

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


def _solver(prob, **kw):
    from paper_1602_02359_amd import fargo as F
    s = F.Solver(dict(prob.params, **kw))
    s.upload(prob.fields)
    return s


def _visc_disk(nx=96, ny=40, alpha=1e-2, seed=11, noise=1e-2):
    return W.disk2d_visc(nx=nx, ny=ny, alpha=alpha, seed=seed, noise=noise)


@pytest.mark.parametrize("shape", [(96, 40), (200, 37), (1, 50)])
def test_visc_one_step_matches_oracle(shape):
    prob = _visc_disk(*shape)
    _say("visc one step", shape)
    ref = prob.copy_fields()
    dt_ref = O.step(prob.params, ref)
    s = _solver(prob)
    assert dt_close(s.fargo_cfl_dt(), dt_ref)
    s.fargo_step(dt_ref)
    s.fargo_check()
    got = s.download()
    err, own = errors(prob, got, ref), errors_own(prob, got, ref)
    _say("  errors", err, "per component", own)
    for k, e in err.items():
        assert e <= TOL, (k, e)
    for k, e in own.items():
        assert e <= TOL, (k, e)


def test_visc_several_steps_match_oracle():
    prob = _visc_disk(128, 48, alpha=3e-2)
    ref = prob.copy_fields()
    s = _solver(prob)
    for n in range(5):
        dt_ref = O.step(prob.params, ref)
        s.fargo_step(0.0)
        dt = s.fargo_get_dt()
        assert dt_close(dt, dt_ref) if n == 0 else abs(dt / dt_ref - 1.0) < 1e-12
    s.fargo_check()
    err = errors(prob, s.download(), ref)
    _say("visc 5 steps", err)
    for k, e in err.items():
        assert e <= 10 * TOL, (k, e)


def test_visc_fp32_hundred_steps_vs_fp64():
    prob = _visc_disk(192, 64, alpha=1e-2, noise=1e-3)
    s64, s32 = _solver(prob), _solver(prob, precision="fp32")
    for _ in range(100):
        s64.fargo_step(0.0)
        s32.fargo_step(s64.fargo_get_dt())   # equal times
    s64.fargo_check()
    s32.fargo_check()
    a, b = s32.download(), s64.download()
    err = errors(prob, a, b)
    _say("visc fp32 vs fp64, 100 steps", err, "per component", errors_own(prob, a, b))
    for k, e in err.items():   # the FP32 bar of tests/test_gpu_fp32.py
        assert e <= 1e-5, (k, e)


def test_visc_unsupported_configurations():
    from paper_1602_02359_amd import fargo as F
    for prob in (W.disk3d_sph(nx=16, ny=6, nz=4), W.random_problem("cyl", nx=16, ny=6, nz=4, eos="iso"),
                 W.random_problem("cyl", nx=16, ny=6, nz=1, eos="adi")):
        with pytest.raises(F.FargoError) as e:
            F.fargo_layout(dict(prob.params, visc=True))
        assert e.value.code == -6


def _small_batch(count, precision):
    probs = W.disk_batch(count=count, nr_range=(16, 72), seed=5)
    return probs, [_solver(p, precision=precision) for p in probs]


@pytest.mark.parametrize("lanes", [3, 0])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_step_equals_individual_steps(precision, lanes):
    """A graph of the disks' own steps over three streams, and the fused form
    (each kernel once over all disks: lanes = 0), against every disk's own
    steps, bit for bit (odd and even ring lengths)."""
    from paper_1602_02359_amd import fargo as F
    probs, batch_solvers = _small_batch(7, precision)
    _, own = _small_batch(7, precision)
    assert len({p.params["nx"] % 2 for p in probs}) == 2
    b = F.Batch(batch_solvers, lanes=lanes)
    for _ in range(4):
        b.fargo_batch_step()
        for s in own:
            s.fargo_step(0.0)
    for s in batch_solvers + own:
        s.fargo_check()
    for p, a, c in zip(probs, batch_solvers, own):
        ga, gc = a.download(), c.download()
        assert a.fargo_get_dt() == c.fargo_get_dt(), p.name
        for k in ("rho", "vx", "vy"):
            assert np.array_equal(ga[k], gc[k]), (p.name, k)
    del b


@pytest.mark.parametrize("lanes", [3, 0])
def test_batch_fp64_matches_oracle(lanes):
    """Six uneven viscous disks advanced by one captured graph per step
    (each disk with its own device time step), every disk against the oracle
    after each of two steps: the time step within the bound of the two codes'
    FP64 arithmetic (32 units in the last place, then 1e-12 once the states
    differ by rounding) and the state within 1e-12 normwise.  The per-component
    errors are printed for information: a batch cannot be given the oracle's
    time step, and v_y, some 1e-3 of the orbital speed, carries the 1e-15
    relative difference of the two time steps at its own scale."""
    from paper_1602_02359_amd import fargo as F
    probs, solvers = _small_batch(6, "fp64")
    refs = [p.copy_fields() for p in probs]
    b = F.Batch(solvers, lanes=lanes)
    for n in range(2):
        b.fargo_batch_step()
        for p, sv, ref in zip(probs, solvers, refs):
            dt_ref = O.step(p.params, ref)
            dt = sv.fargo_get_dt()
            if n == 0:
                assert dt_close(dt, dt_ref), (p.name, dt, dt_ref)
            else:
                assert abs(dt / dt_ref - 1.0) < 1e-12, (p.name, dt, dt_ref)
            sv.fargo_check()
            got = sv.download()
            err, own = errors(p, got, ref), errors_own(p, got, ref)
            _say("batch step", n + 1, p.name, p.params["nx"], p.params["ny"], err, "per component", own)
            for k, e in err.items():
                assert e <= TOL, (p.name, k, e)
    del b


def test_batch_tune_keeps_states_and_picks_a_candidate():
    import torch
    from paper_1602_02359_amd import fargo as F
    probs, solvers = _small_batch(5, "fp32")
    b = F.Batch(solvers, lanes=1)
    b.fargo_batch_step()
    before = [s.download() for s in solvers]
    lanes, chunk = b.fargo_batch_tune(lanes=(1, 2, 4), chunks=(16, 64), steps=2)
    assert lanes in (1, 2, 4) and chunk in (16, 64)
    after = [s.download() for s in solvers]
    for x, y in zip(before, after):
        for k in ("rho", "vx", "vy"):
            assert np.array_equal(x[k], y[k]), k
    # the retuned batch still steps like the disks' own steps
    _, own = _small_batch(5, "fp32")
    for o in own:
        o.fargo_step(0.0)
    b.fargo_batch_step()
    torch.cuda.synchronize()
    for a, o in zip(solvers, own):
        o.fargo_step(0.0)
    for a, o in zip(solvers, own):
        ga, go = a.download(), o.download()
        for k in ("rho", "vx", "vy"):
            assert np.array_equal(ga[k], go[k]), k
    del b


def test_fused_batch_tunes_per_size_class():
    """The fused form's autotuner: a sweep chunk per size class of disks
    (floor(log2 ny)) from the candidates, the states left as found, and the
    tuned batch still steps like the disks' own steps."""
    import torch
    from paper_1602_02359_amd import fargo as F
    probs, solvers = _small_batch(6, "fp32")
    b = F.Batch(solvers, lanes=0)
    before = [s.download() for s in solvers]
    lanes, chunk = b.fargo_batch_tune(lanes=(1,), chunks=(8, 64), steps=2)
    assert lanes == 0 and chunk in (8, 64)
    ch = b.chunks()
    assert all(c in (8, 64) for c in ch)
    cls = [int(np.floor(np.log2(p.params["ny"]))) for p in probs]
    for c1, k1 in zip(ch, cls):
        for c2, k2 in zip(ch, cls):
            if k1 == k2:
                assert c1 == c2
    after = [s.download() for s in solvers]
    for x, y in zip(before, after):
        for k in ("rho", "vx", "vy"):
            assert np.array_equal(x[k], y[k]), k
    _, own = _small_batch(6, "fp32")
    for _ in range(2):
        b.fargo_batch_step()
        for o in own:
            o.fargo_step(0.0)
    torch.cuda.synchronize()
    for a, o in zip(solvers, own):
        ga, go = a.download(), o.download()
        for k in ("rho", "vx", "vy"):
            assert np.array_equal(ga[k], go[k]), k
    del b


def test_fused_batch_refuses_mixed_configurations():
    from paper_1602_02359_amd import fargo as F
    probs = W.disk_batch(count=2, nr_range=(16, 24), seed=6)
    mixed = [_solver(probs[0], precision="fp64"), _solver(probs[1], precision="fp32")]
    with pytest.raises(F.FargoError) as e:
        F.Batch(mixed, lanes=0)
    assert e.value.code == -6
    b = F.Batch(mixed, lanes=2)  # the graph of the disks' own steps takes them
    b.fargo_batch_step()
    for s in mixed:
        s.fargo_check()
    del b


def test_fused_batch_full_size():
    """The benchmark's batch: the 256 uneven viscous disks (N_r 64..512,
    70.7 M zones), FP64, in the fused form with the chunk tuned per size class
    as the benchmark does.  After two steps every disk equals its own
    fargo_step bit for bit (a property at any size), and four sampled disks,
    the smallest, the largest and two between, match the oracle after the
    first step (dt within the 32-ulp bound, state within 1e-12 normwise)."""
    import torch
    from paper_1602_02359_amd import fargo as F
    probs = W.disk_batch()
    sizes = [p.active_cells for p in probs]
    order = np.argsort(sizes)
    sample = [int(order[0]), int(order[len(order) // 3]), int(order[2 * len(order) // 3]), int(order[-1])]
    refs = {d: probs[d].copy_fields() for d in sample}
    fused = [_solver(p) for p in probs]
    b = F.Batch(fused, lanes=0)
    b.fargo_batch_tune(lanes=(0,), chunks=(8, 16, 32, 64), steps=2)
    _say("fused batch of %d disks, %d zones, chunks by disk %s" % (len(probs), sum(sizes), sorted(set(b.chunks()))))
    b.fargo_batch_step()
    torch.cuda.synchronize()
    for d in sample:
        p = probs[d]
        dt_ref = O.step(p.params, refs[d])
        sv = fused[d]
        dt = sv.fargo_get_dt()
        assert dt_close(dt, dt_ref), (p.name, dt, dt_ref)
        err = errors(p, sv.download(), refs[d])
        _say("  %s %dx%d against the oracle: %s" % (p.name, p.params["nx"], p.params["ny"], err))
        for k, e in err.items():
            assert e <= TOL, (p.name, k, e)
    b.fargo_batch_step()
    for sv in fused:
        sv.fargo_check()
    for d, p in enumerate(probs):
        own = _solver(p)
        own.fargo_step(0.0)
        own.fargo_step(0.0)
        a, c = fused[d], own
        assert a.fargo_get_dt() == c.fargo_get_dt(), p.name
        for k in ("rho", "vx", "vy"):
            assert torch.equal(a.state[k], c.state[k]), (p.name, k)
        del own
    del b
