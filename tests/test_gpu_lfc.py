"""Learned flux correction through the C ABI (fargo_lfc_*), against the
numpy oracle (oracle/lfc.py) on the same weights and inputs, element by
element.

Bars.  The features are formed in FP64 and rounded the same way on both
sides: bit-exact.  Every product takes bfloat16 operands (exact in FP32); the
GPU sums them in FP32, the oracle exactly.  Each layer is checked from the
GPU's own inputs: the oracle's exact pre-rounding value z, and the bound
delta = 2 depth u sum|terms| of an FP32 sum of that depth (oracle.lfc.
sum_bound), give the interval [q(z - delta), q(z + delta)] that the stored
bfloat16 value q must lie in (q is monotone; oracle.lfc.interval).  Where
the stored value differs from the oracle's q(z) (a bfloat16 rounding flipped
by the FP32 sum error, about one value in 10^4) it is counted, and the count
must stay under a budget of one in a thousand (at least 8); a wrong tap,
index or sign puts values outside their intervals.  The FP32 output and
the weight and bias gradients are checked the same way, without rounding;
the density change and loss against the oracle applied to the GPU's own net
output (FP64 on both sides), and the Adam step against the oracle applied to
the GPU's own gradient (FP32 against FP64, 1e-5).
"""
import sys

import numpy as np
import pytest

from oracle import lfc as L
from paper_1602_02359_amd import workloads as W

pytestmark = pytest.mark.gpu

NG = W.NGH
FLIP_FRACTION = 1e-3  # stored bfloat16 values allowed to differ from the oracle's rounding


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _inside(name, got, lo, hi):
    got = np.asarray(got, dtype=np.float64)
    bad = (got < lo) | (got > hi)
    if bad.any():
        idx = np.argwhere(bad)[:5]
        raise AssertionError("%s: %d values outside their bound, first at %s: got %s, bound [%s, %s]" % (
            name, int(bad.sum()), idx.tolist(), got[tuple(idx.T)], lo[tuple(idx.T)], hi[tuple(idx.T)]))


def _check_rounded(name, got, z, delta, relu=False, mask=None):
    """A stored bfloat16 layer against the interval of oracle.lfc.interval;
    returns the number of values that differ from the oracle's own rounding."""
    lo, mid, hi = L.interval(z, delta, relu=relu, mask=mask)
    _inside(name, got, lo, hi)
    flips = int(np.count_nonzero(np.asarray(got, dtype=np.float64) != mid))
    assert flips <= max(8, int(FLIP_FRACTION * mid.size)), (name, flips, mid.size)
    return flips


def _check_sum(name, got, ref, delta):
    """An FP32 sum against its exact value: within the sum bound plus the
    rounding of the result."""
    ref = np.asarray(ref, dtype=np.float64)
    _inside(name, got, ref - delta - L.U32 * np.abs(ref), ref + delta + L.U32 * np.abs(ref))


def _bw(P):
    return {k: L.bf16(P[k]) for k in ("W1", "W2", "W3")}


def _forward_layers(v, P):
    """Each layer of the GPU's forward pass from the GPU's own input to it:
    h1 from the features, h2 from the GPU's h1, o from the GPU's h2.
    Returns the flip counts."""
    Wb = _bw(P)
    f = v["f"].float().cpu().numpy().astype(np.float64)
    h1 = v["h1"].float().cpu().numpy().astype(np.float64)
    h2 = v["h2"].float().cpu().numpy().astype(np.float64)
    o = v["o"].double().cpu().numpy()
    flips = {}
    for name, x, w, b, got in (("h1", f, Wb["W1"], P["b1"], h1), ("h2", h1, Wb["W2"], P["b2"], h2)):
        K = 9 * x.shape[2]
        z = L.conv(x, w, b)
        d = L.sum_bound(K + 1, L.conv(np.abs(x), np.abs(w), np.abs(np.asarray(b, dtype=np.float64))))
        flips[name] = _check_rounded(name, got, z, d, relu=True)
    z = L.conv(h2, Wb["W3"], P["b3"])
    d = L.sum_bound(9 * 32 + 1, L.conv(np.abs(h2), np.abs(Wb["W3"]), np.abs(np.asarray(P["b3"], dtype=np.float64))))
    _check_sum("o", o, z, d)
    return flips


def _wdepth(nx, ny, nsamp):
    """Longest chain of FP32 additions behind a weight or bias gradient: the
    library's weight-gradient blocks (a 64-pixel strip of one sample over rpc
    rows, at most 512 blocks where the strips allow; the block layout of
    lfc_wblocks) each
    accumulate rpc x 64 pixels (an MFMA adds 32 products per k step of 32
    pixels, two k steps a row), the bias sums rpc values per thread and 64 in
    the block, then the partials of the nw blocks are summed."""
    strips = nsamp * (nx // 64)
    want = min(max(512 // strips, 1), ny)
    rpc = -(-ny // want)
    nw = strips * (-(-ny // rpc))
    return rpc * 64 + nw + 64


def _np(v, name):
    t = v[name]
    return t.double().cpu().numpy() if name in ("o", "drho") else t.float().cpu().numpy().astype(np.float64)


def _backward_layers(vs, P, grad, ts, sF, invV, sigma, depth):
    """The backward pass of a batch from the GPU's own values: for each
    sample (views vs[s], target ts[s]) g3 from the GPU's density change (the
    loss the mean over all zones of the batch), g2 and g1 from the GPU's g3
    and g2 (masked by the GPU's h2, h1); each weight and bias gradient, summed
    over the samples, from the GPU's layer gradients and activations.
    Returns the flip counts."""
    Wb = _bw(P)
    N = sum(t.size for t in ts)
    flips = {"g3": 0, "g2": 0, "g1": 0}
    ref, bnd = {}, {}

    def acc(k, r, d):
        ref[k] = ref.get(k, 0.0) + r
        bnd[k] = bnd.get(k, 0.0) + d

    for v, t in zip(vs, ts):
        f, h1, h2 = _np(v, "f"), _np(v, "h1"), _np(v, "h2")
        g3, g2, g1 = _np(v, "g3")[..., :2], _np(v, "g2"), _np(v, "g1")
        d = _np(v, "drho")
        # g3 = bf16(fp32(dL/dF)) from the density change: FP64 on both sides
        gg = 2.0 * (d - t) / (N * sigma * sigma)
        gD = -invV[:, None] * gg
        gFx = np.roll(gD, 1, axis=1) - gD
        gFy = np.zeros_like(gD)
        gFy[1:] = gD[:-1] - gD[1:]
        g3ref = np.stack([sF * gFx, sF * gFy], axis=-1)
        flips["g3"] += _check_rounded("g3", g3, g3ref, 1e-15 * np.abs(g3ref))
        flips["g2"] += _check_rounded("g2", g2, L.conv_t(g3, Wb["W3"]),
                                      L.sum_bound(9 * 2 + 1, L.conv_t(np.abs(g3), np.abs(Wb["W3"]))), mask=h2 > 0)
        flips["g1"] += _check_rounded("g1", g1, L.conv_t(g2, Wb["W2"]),
                                      L.sum_bound(9 * 32 + 1, L.conv_t(np.abs(g2), np.abs(Wb["W2"]))), mask=h1 > 0)
        for n, g, x in ((3, g3, h2), (2, g2, h1), (1, g1, f)):
            acc("W%d" % n, L.conv_w(g, x), L.conv_w(np.abs(g), np.abs(x)))
            acc("b%d" % n, g.sum(axis=(0, 1)), np.abs(g).sum(axis=(0, 1)))
    G = _unflat(grad)
    for k in ref:
        _check_sum(k, G[k], ref[k], L.sum_bound(depth, bnd[k]))
    return flips


def _nerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _flat(P):
    return np.concatenate([np.asarray(P[k], dtype=np.float32).ravel()
                           for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def _unflat(v):
    P, o = {}, 0
    for n, (ci, co) in enumerate(L.LAYERS, 1):
        w = 9 * ci * co
        P["W%d" % n] = v[o:o + w].reshape(co, 3, 3, ci).astype(np.float64)
        o += w
        P["b%d" % n] = v[o:o + co].astype(np.float64)
        o += co
    return P


def _geometry(p):
    y = p["ymin"]
    a, b = y[NG:NG + p["ny"]], y[NG + 1:NG + p["ny"] + 1]
    dx = (p["xmax"] - p["xmin"]) / p["nx"]
    rc = 0.5 * (a + b)
    invV = 2.0 / ((b * b - a * a) * dx)
    return rc, invV


def _setup(nx=64, ny=16, seed=11, sF=None, guard=0.5, max_batch=1):
    import torch
    from paper_1602_02359_amd import fargo as F
    prob = W.disk2d_planet(nx=nx, ny=ny, seed=4000 + seed, noise=0.05)
    rng = np.random.default_rng(seed)
    act = (0, slice(NG, NG + ny), slice(None))
    prob.fields["vy"][act] = 0.02 * rng.standard_normal((ny, nx))
    prob.fields["vx"][act] += 0.02 * rng.standard_normal((ny, nx))
    s = F.Solver(prob.params)
    s.upload(prob.fields)
    rc, invV = _geometry(prob.params)
    scales = (1.0, 0.05, 1.45, 1.05)
    sF = sF if sF is not None else 1e-4 / float(invV.mean())
    sigma = 1e-3
    net = F.LFC(s, *scales, flux_scale=sF, sigma=sigma, guard=guard, max_batch=max_batch)
    P = L.init_params(rng)
    for k in ("b1", "b2", "b3"):
        P[k] = (0.05 * rng.standard_normal(P[k].shape)).astype(np.float32)
    P["W3"] = (P["W3"] * 10.0).astype(np.float32)
    net.set_params(_flat(P))
    fields = {k: prob.fields[k][act].copy() for k in ("rho", "vx", "vy")}
    target = 1e-3 * rng.standard_normal((ny, nx))
    return dict(s=s, net=net, P=P, rc=rc, invV=invV, scales=scales, sF=sF, sigma=sigma, fields=fields,
                target=target, torch=torch, prob=prob, nx=nx, ny=ny)


def _samples(c, n, seed):
    """n batch samples on the mesh of setup c: the setup's state with
    different seeded perturbations of rho, v_x and v_y in the active zones,
    laid out as the solver's state, and a target each."""
    torch, s = c["torch"], c["s"]
    nx, ny = c["nx"], c["ny"]
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        smp, fields = {}, {}
        for name, amp in (("rho", 0.05), ("vx", 0.02), ("vy", 0.02)):
            t = s.state[name].clone()
            a = t[0, NG:NG + ny, :nx].cpu().numpy()
            a = a * (1.0 + amp * rng.standard_normal(a.shape)) if name == "rho" else a + amp * rng.standard_normal(a.shape)
            t[0, NG:NG + ny, :nx] = torch.from_numpy(a)
            smp[name] = t
            fields[name] = a
        tg = 1e-3 * (k + 1) * rng.standard_normal((ny, nx))
        smp["target"] = torch.from_numpy(np.ascontiguousarray(tg)).cuda()
        out.append((smp, fields, tg))
    return out


def test_forward_matches_oracle():
    c = _setup()
    net, torch = c["net"], c["torch"]
    _say("lfc forward 64 x 16")
    net.forward()
    v = net.views()
    fx = c["fields"]
    f = L.features(fx["rho"], fx["vx"], fx["vy"], c["rc"], c["scales"])
    assert np.array_equal(v["f"].float().cpu().numpy().astype(np.float64), f)
    flips = _forward_layers(v, c["P"])
    A = L.forward(f, c["P"])
    _say("  flipped roundings", flips, "end to end normwise (information)",
         {k: _nerr(v[k].float().cpu().numpy(), A[k]) for k in ("h1", "h2", "o")})
    # the density change from the GPU's own output: FP64 on both sides
    o_gpu = v["o"].double().cpu().numpy()
    d_ref = L.drho(o_gpu, c["sF"], c["invV"])
    d_gpu = v["drho"].cpu().numpy()
    assert np.abs(d_gpu - d_ref).max() <= 1e-14 * np.abs(d_ref).max()
    # and it conserves mass: sum V drho = 0
    Vs = (1.0 / c["invV"])[:, None]
    assert abs(np.sum(d_gpu * Vs)) <= 1e-13 * np.sum(np.abs(d_gpu * Vs))


def test_train_step_gradient_loss_and_adam():
    c = _setup(seed=12)
    net, torch = c["net"], c["torch"]
    _say("lfc train step 64 x 16")
    t_dev = torch.from_numpy(c["target"]).cuda()
    lr = 1e-3
    net.train_step(t_dev, lr)
    loss, _ = net.result()
    v = net.views()
    grad = net.get_grad()
    newp = net.get_params()
    fx = c["fields"]
    f = L.features(fx["rho"], fx["vx"], fx["vy"], c["rc"], c["scales"])
    Pd = {k: np.asarray(x, dtype=np.float64) for k, x in c["P"].items()}
    fwd = _forward_layers(v, c["P"])
    bwd = _backward_layers([v], c["P"], grad, [c["target"]], c["sF"], c["invV"], c["sigma"], _wdepth(64, 16, 1))
    d_gpu = v["drho"].cpu().numpy()
    loss_ref = L.loss(d_gpu, c["target"], c["sigma"])
    A = L.forward(f, c["P"])
    G = L.backward(A, Pd, c["target"], c["sF"], c["invV"], c["sigma"])
    Gg = _unflat(grad)
    _say("  loss", loss, loss_ref, "flipped roundings", fwd, bwd, "gradient end to end normwise (information)",
         {k: _nerr(Gg[k], G[k]) for k in G})
    assert abs(loss - loss_ref) <= 1e-12 * loss_ref
    # the padding channels of the last layer's gradient
    g3 = v["g3"].float().cpu().numpy()
    assert np.all(g3[..., 2:] == 0.0)
    # Adam on the GPU's own gradient: FP32 against FP64
    M0 = {k: np.zeros_like(x) for k, x in Pd.items()}
    Pn, _, _ = L.adam(Pd, Gg, M0, dict(M0), 1, lr)
    Pg = _unflat(newp)
    for k in Pn:
        assert np.allclose(Pg[k], Pn[k], rtol=1e-5, atol=1e-3 * lr), k


def test_forward_batch_equals_single_forwards():
    """A batch of three states through the net in one set of launches gives,
    sample by sample, bit for bit what the single-state forward gives."""
    c = _setup(seed=16, max_batch=3)
    net = c["net"]
    smps = _samples(c, 3, 161)
    _say("lfc forward batch of 3, 64 x 16")
    net.forward_batch([x[0] for x in smps])
    vb = net.views(3)
    for k, (smp, _, _) in enumerate(smps):
        net.forward_batch([smp])
        v1 = net.views()
        for name in ("f", "h1", "h2", "o", "drho"):
            assert c["torch"].equal(vb[name][k], v1[name]), (k, name)


@pytest.mark.parametrize("shape", [(64, 16, 3), (128, 13, 2)])
def test_train_batch_matches_oracle(shape):
    """One Adam step on a batch (three 64 x 16 samples; two 128 x 13, a
    ragged row tile): every sample's features, layers and layer gradients
    element by element, the summed weight and bias gradients within the FP32
    sum bound, the batch loss and the Adam step."""
    nx, ny, n = shape
    c = _setup(nx=nx, ny=ny, seed=17, max_batch=4)
    net, torch = c["net"], c["torch"]
    smps = _samples(c, n, 171)
    _say("lfc train batch of %d, %d x %d" % (n, nx, ny))
    lr = 1e-3
    net.train_batch([x[0] for x in smps], lr)
    loss, _ = net.result()
    vb = net.views(n)
    grad, newp = net.get_grad(), net.get_params()
    vs = [{k: vb[k][s] for k in vb} for s in range(n)]
    flips = {}
    for s, (_, fx, _) in enumerate(smps):
        f = L.features(fx["rho"], fx["vx"], fx["vy"], c["rc"], c["scales"])
        assert np.array_equal(_np(vs[s], "f"), f), s
        for k, x in _forward_layers(vs[s], c["P"]).items():
            flips[k] = flips.get(k, 0) + x
        d_ref = L.drho(_np(vs[s], "o"), c["sF"], c["invV"])
        assert np.abs(_np(vs[s], "drho") - d_ref).max() <= 1e-14 * np.abs(d_ref).max()
    ts = [x[2] for x in smps]
    bwd = _backward_layers(vs, c["P"], grad, ts, c["sF"], c["invV"], c["sigma"], _wdepth(nx, ny, n))
    loss_ref = L.loss_batch([_np(v, "drho") for v in vs], ts, c["sigma"])
    _say("  loss", loss, loss_ref, "flipped roundings", flips, bwd)
    assert abs(loss - loss_ref) <= 1e-12 * loss_ref
    Pd = {k: np.asarray(x, dtype=np.float64) for k, x in c["P"].items()}
    Gg = _unflat(grad)
    M0 = {k: np.zeros_like(x) for k, x in Pd.items()}
    Pn, _, _ = L.adam(Pd, Gg, M0, dict(M0), 1, lr)
    Pg = _unflat(newp)
    for k in Pn:
        assert np.allclose(Pg[k], Pn[k], rtol=1e-5, atol=1e-3 * lr), k


def test_batch_size_is_checked():
    c = _setup(seed=18, max_batch=2)
    from paper_1602_02359_amd import fargo as F
    smps = [x[0] for x in _samples(c, 3, 181)]
    with pytest.raises(F.FargoError):
        c["net"].forward_batch(smps)
    with pytest.raises(F.FargoError):
        c["net"].train_batch(smps, 1e-3)


def test_training_reduces_the_loss():
    """Adam on one fixed sample whose target the net can represent (the
    density change of a second, randomly drawn net on the same state): the
    loss falls well below its start."""
    c = _setup(seed=13)
    net, torch = c["net"], c["torch"]
    fx = c["fields"]
    f = L.features(fx["rho"], fx["vx"], fx["vy"], c["rc"], c["scales"])
    teacher = L.init_params(np.random.default_rng(99))
    teacher["W3"] = (teacher["W3"] * 10.0).astype(np.float32)
    target = L.drho(L.forward(f, teacher)["o"], c["sF"], c["invV"])
    t_dev = torch.from_numpy(np.ascontiguousarray(target)).cuda()
    losses = []
    for n in range(300):
        net.train_step(t_dev, 3e-3)
        if n % 50 == 0 or n == 299:
            losses.append(net.result()[0])
    _say("  losses", losses)
    assert losses[-1] < 0.5 * losses[0]


def test_apply_conserves_mass_and_guard_rejects():
    c = _setup(seed=14)
    s, net = c["s"], c["net"]
    rho0 = s.state["rho"][0, NG:NG + 16, :64].clone()
    net.apply()
    _, skipped = net.result()
    assert not skipped
    d = net.views()["drho"].cpu().numpy()
    rho1 = s.state["rho"][0, NG:NG + 16, :64].cpu().numpy()
    assert np.array_equal(rho1, rho0.cpu().numpy() + d)
    V = (1.0 / c["invV"])[:, None]
    m0 = np.sum(rho0.cpu().numpy() * V)
    assert abs(np.sum(rho1 * V) - m0) <= 1e-13 * m0
    # a huge flux scale makes the correction exceed the guard: no change
    c2 = _setup(seed=14, sF=1e3, guard=0.5)
    s2, net2 = c2["s"], c2["net"]
    before = s2.state["rho"].clone()
    net2.apply()
    _, skipped = net2.result()
    assert skipped
    assert c2["torch"].equal(before, s2.state["rho"])


@pytest.mark.parametrize("ratio", [4, 2])
def test_restriction_matches_oracle(ratio):
    from paper_1602_02359_amd import fargo as F
    fine = W.disk2d_planet(nx=256, ny=64, seed=4001, noise=0.05)
    coarse = W.disk2d_planet(nx=256 // ratio, ny=64 // ratio, seed=4002)
    rng = np.random.default_rng(21)
    act = (0, slice(NG, NG + 64), slice(None))
    fine.fields["vy"][act] = 0.01 * rng.standard_normal((64, 256))
    fine.fields["vx"][act] += 0.01 * rng.standard_normal((64, 256))
    sf, sc = F.Solver(fine.params), F.Solver(coarse.params)
    sf.upload(fine.fields)
    sc.upload(coarse.fields)
    ghost_before = sc.state["rho"][0, :NG].clone()
    F.lfc_restrict(sf, sc)
    got = sc.download()
    fa = {k: fine.fields[k][act] for k in ("rho", "vx", "vy")}
    yf = fine.params["ymin"][NG:NG + 65]
    rc, vxc, vyc = L.restrict(fa["rho"], fa["vx"], fa["vy"], yf, ratio=ratio)
    ca = (0, slice(NG, NG + 64 // ratio), slice(None))
    for k, ref in (("rho", rc), ("vx", vxc), ("vy", vyc)):
        assert np.abs(got[k][ca] - ref).max() <= 1e-14 * np.abs(ref).max(), k
    assert sc.state["rho"][0, :NG].equal(ghost_before)


def test_unsupported_meshes_are_rejected():
    from paper_1602_02359_amd import fargo as F
    prob = W.disk2d_planet(nx=96, ny=16)  # nx not a multiple of 64
    s = F.Solver(prob.params)
    s.upload(prob.fields)
    with pytest.raises(F.FargoError):
        F.LFC(s, 1.0, 0.05, 1.45, 1.05, flux_scale=1.0, sigma=1e-3)


def test_training_pipeline_small():
    """Samples along a fine trajectory (256 x 64 restricted onto 64 x 16):
    finite, non-zero targets; training lowers the coarse step's error on the
    samples it saw below the plain step's (relative error < 1) and reports a
    finite held-out error."""
    from paper_1602_02359_amd import learned as LN
    cp, samples = LN.make_samples(12, coarse=dict(nx=64, ny=16), fine=dict(nx=256, ny=64))
    for s in samples:
        t = s["target"]
        assert bool(t.isfinite().all()) and float(t.abs().max()) > 0.0
    sc = LN.scales(cp, samples)
    tr = LN.Trainer(cp, sc)
    train, held = samples[:10], samples[10:]
    losses = tr.train(train, 300, 3e-3, every=100)
    ev, eh = tr.evaluate(train), tr.evaluate(held)
    _say("  pipeline losses", losses, "train", ev, "held", eh)
    assert losses[-1] < losses[0]
    assert ev["relative_error"] < 1.0
    assert np.isfinite(eh["relative_error"])


def test_full_size_forward_and_gradient():
    """The 768 x 256 coarse planet disk of the benchmark: forward pass,
    density change, loss and gradient against the oracle on the same state."""
    c = _setup(nx=768, ny=256, seed=15)
    net, torch = c["net"], c["torch"]
    _say("lfc full size 768 x 256")
    t_dev = torch.from_numpy(c["target"]).cuda()
    net.train_step(t_dev, 1e-3)
    loss, _ = net.result()
    v = net.views()
    grad = net.get_grad()
    fx = c["fields"]
    f = L.features(fx["rho"], fx["vx"], fx["vy"], c["rc"], c["scales"])
    assert np.array_equal(v["f"].float().cpu().numpy().astype(np.float64), f)
    fwd = _forward_layers(v, c["P"])
    bwd = _backward_layers([v], c["P"], grad, [c["target"]], c["sF"], c["invV"], c["sigma"], _wdepth(768, 256, 1))
    d_gpu = v["drho"].cpu().numpy()
    o_gpu = v["o"].double().cpu().numpy()
    d_ref = L.drho(o_gpu, c["sF"], c["invV"])
    assert np.abs(d_gpu - d_ref).max() <= 1e-14 * np.abs(d_ref).max()
    loss_ref = L.loss(d_gpu, c["target"], c["sigma"])
    _say("  loss", loss, loss_ref, "flipped roundings", fwd, bwd)
    assert abs(loss - loss_ref) <= 1e-12 * loss_ref
    Vs = (1.0 / c["invV"])[:, None]
    assert abs(np.sum(d_gpu * Vs)) <= 1e-13 * np.sum(np.abs(d_gpu * Vs))


def test_full_size_train_batch_of_eight():
    """The benchmark's training configuration: the 768 x 256 coarse planet
    disk, eight samples per Adam step (the weight-gradient grid of that batch
    size).  Two samples' layers element by element, and every weight and bias
    gradient, summed over the eight samples, within the FP32 sum bound."""
    c = _setup(nx=768, ny=256, seed=19, max_batch=8)
    net = c["net"]
    smps = _samples(c, 8, 191)
    _say("lfc full size 768 x 256, batch of 8")
    net.train_batch([x[0] for x in smps], 1e-3)
    loss, _ = net.result()
    vb = net.views(8)
    grad = net.get_grad()
    vs = [{k: vb[k][s] for k in vb} for s in range(8)]
    flips = {}
    for s in (0, 7):
        fx = smps[s][1]
        f = L.features(fx["rho"], fx["vx"], fx["vy"], c["rc"], c["scales"])
        assert np.array_equal(_np(vs[s], "f"), f), s
        for k, x in _forward_layers(vs[s], c["P"]).items():
            flips[k] = flips.get(k, 0) + x
    ts = [x[2] for x in smps]
    bwd = _backward_layers(vs, c["P"], grad, ts, c["sF"], c["invV"], c["sigma"], _wdepth(768, 256, 8))
    loss_ref = L.loss_batch([_np(v, "drho") for v in vs], ts, c["sigma"])
    _say("  loss", loss, loss_ref, "flipped roundings", flips, bwd)
    assert abs(loss - loss_ref) <= 1e-12 * loss_ref
