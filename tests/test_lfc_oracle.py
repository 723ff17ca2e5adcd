"""Pins of the learned-flux-correction oracle (oracle/lfc.py) against what
mathematics fixes: an independent correlation routine, adjoint identities,
finite differences of the loss, the telescoping of the flux divergence, the
closed form of Adam's first step, and the conservation and consistency of
the 4 x 4 restriction.  None compares the oracle with itself.
"""
import math

import numpy as np
import pytest
from scipy import signal

from oracle import lfc as L


def _rng(seed=0):
    return np.random.default_rng(seed)


def test_bf16_rounding_known_values():
    """Round to nearest even on the 8-bit significand: ties go to the even
    neighbour, the spacing at 1 is 2^-7."""
    x = [1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -7, math.pi, -0.1, 0.0, 65504.0]
    want = [1.0, 1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7, 3.140625, -0.10009765625, 0.0, 65536.0]
    assert L.bf16(x).tolist() == want


def test_conv_matches_scipy_correlate():
    """Each (out, in) channel pair of `conv` is a 2D cross-correlation with
    wrap-around in i and zero rows beyond j (built from scipy's routine by
    padding one zero row on each side)."""
    rng = _rng(1)
    ny, nx, ci, co = 7, 12, 3, 2
    x = rng.standard_normal((ny, nx, ci))
    w = rng.standard_normal((co, 3, 3, ci))
    b = rng.standard_normal(co)
    got = L.conv(x, w, b)
    want = np.zeros((ny, nx, co))
    for o in range(co):
        want[..., o] = b[o]
        for c in range(ci):
            xp = np.pad(x[..., c], ((1, 1), (0, 0)))
            r = signal.correlate2d(xp, w[o, :, :, c], mode="same", boundary="wrap")
            want[..., o] += r[1:-1]
    assert np.allclose(got, want, rtol=1e-13, atol=1e-13)


def test_conv_transpose_is_adjoint():
    """<conv(x, w), g> = <x, conv_t(g, w)> for zero bias."""
    rng = _rng(2)
    x = rng.standard_normal((5, 8, 4))
    w = rng.standard_normal((3, 3, 3, 4))
    g = rng.standard_normal((5, 8, 3))
    lhs = np.sum(L.conv(x, w, np.zeros(3)) * g)
    rhs = np.sum(x * L.conv_t(g, w))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_conv_weight_gradient_is_directional_derivative():
    """<conv(x, dw), g> = <dw, conv_w(g, x)> (conv is linear in w)."""
    rng = _rng(3)
    x = rng.standard_normal((6, 8, 4))
    g = rng.standard_normal((6, 8, 2))
    dw = rng.standard_normal((2, 3, 3, 4))
    lhs = np.sum(L.conv(x, dw, np.zeros(2)) * g)
    rhs = np.sum(dw * L.conv_w(g, x))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _problem(seed=4, ny=6, nx=8):
    rng = _rng(seed)
    P = {k: v.astype(np.float64) for k, v in L.init_params(rng).items()}
    for k in ("b1", "b2", "b3"):
        P[k] = 0.05 * rng.standard_normal(P[k].shape)
    P["W3"] *= 10.0
    f = rng.standard_normal((ny, nx, L.CIN))
    t = 0.01 * rng.standard_normal((ny, nx))
    invV = 1.0 + rng.random(ny)
    return P, f, t, invV


def test_backward_matches_finite_differences():
    """Unrounded gradients against central differences of the loss in FP64,
    for entries of every weight and bias array."""
    P, f, t, invV = _problem()
    sF, sigma = 0.3, 0.02

    def lossP(Q):
        A = L.forward(f, Q, rounded=False)
        return L.loss(L.drho(A["o"], sF, invV), t, sigma)

    A = L.forward(f, P, rounded=False)
    G = L.backward(A, P, t, sF, invV, sigma, rounded=False)
    rng = _rng(5)
    h = 1e-6
    for k in ("W1", "W2", "W3", "b1", "b2", "b3"):
        for _ in range(4):
            idx = tuple(int(rng.integers(0, s)) for s in P[k].shape)
            Qp = {kk: v.copy() for kk, v in P.items()}
            Qm = {kk: v.copy() for kk, v in P.items()}
            Qp[k][idx] += h
            Qm[k][idx] -= h
            fd = (lossP(Qp) - lossP(Qm)) / (2 * h)
            assert abs(G[k][idx] - fd) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (k, idx, G[k][idx], fd)


def test_batch_gradient_matches_finite_differences():
    """A batch of three samples (different features and targets, one mesh):
    the summed gradients against central differences of the batch loss, the
    mean over every zone of every sample."""
    P, f, t, invV = _problem()
    rng = _rng(8)
    fs = [f, rng.standard_normal(f.shape), rng.standard_normal(f.shape)]
    ts = [t, 0.01 * rng.standard_normal(t.shape), 0.02 * rng.standard_normal(t.shape)]
    sF, sigma = 0.3, 0.02

    def lossP(Q):
        return L.loss_batch([L.drho(L.forward(x, Q, rounded=False)["o"], sF, invV) for x in fs], ts, sigma)

    G = L.backward_batch([L.forward(x, P, rounded=False) for x in fs], P, ts, sF, invV, sigma, rounded=False)
    h = 1e-6
    for k in ("W1", "W2", "W3", "b1", "b2", "b3"):
        for _ in range(3):
            idx = tuple(int(rng.integers(0, s)) for s in P[k].shape)
            Qp = {kk: v.copy() for kk, v in P.items()}
            Qm = {kk: v.copy() for kk, v in P.items()}
            Qp[k][idx] += h
            Qm[k][idx] -= h
            fd = (lossP(Qp) - lossP(Qm)) / (2 * h)
            assert abs(G[k][idx] - fd) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (k, idx, G[k][idx], fd)
    # a batch of one is the single-sample loss and gradient
    A = L.forward(f, P, rounded=False)
    G1 = L.backward_batch([A], P, [t], sF, invV, sigma, rounded=False)
    G0 = L.backward(A, P, t, sF, invV, sigma, rounded=False)
    for k in G0:
        assert np.array_equal(G1[k], G0[k])


def test_flux_divergence_telescopes():
    """The added fluxes only move mass between zones: sum_j V_j sum_i drho = 0
    (periodic in i, no flux through the radial boundary faces), and a uniform
    X flux or a Y flux on the boundary row alone changes nothing."""
    rng = _rng(6)
    ny, nx = 9, 16
    V = 0.5 + rng.random(ny)
    o = rng.standard_normal((ny, nx, 2))
    d = L.drho(o, 0.7, 1.0 / V)
    total = np.sum(d * V[:, None])
    assert abs(total) <= 1e-13 * np.sum(np.abs(d * V[:, None]))
    o2 = np.zeros((ny, nx, 2))
    o2[..., 0] = 3.0
    o2[0, :, 1] = rng.standard_normal(nx)
    assert np.all(L.drho(o2, 1.0, 1.0 / V) == 0.0)


def test_adam_first_step_closed_form():
    """With zero moments, the bias-corrected first Adam step is
    -lr g / (|g| + eps) (Kingma & Ba, Alg. 1)."""
    g = np.array([3.0, -0.5, 1e-3])
    P = {"w": np.array([1.0, 2.0, 3.0])}
    M = {"w": np.zeros(3)}
    V = {"w": np.zeros(3)}
    lr, eps = 0.01, 1e-8
    Pn, Mn, Vn = L.adam(P, {"w": g}, M, V, 1, lr, eps=eps)
    assert np.allclose(Pn["w"], P["w"] - lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)
    assert np.allclose(Mn["w"], 0.1 * g) and np.allclose(Vn["w"], 0.001 * g * g)


def test_adam_minimises_a_quadratic():
    """Repeated Adam steps on 0.5 (w - 2)^2 settle near the minimum."""
    P = {"w": np.array([-1.0])}
    M = {"w": np.zeros(1)}
    V = {"w": np.zeros(1)}
    for n in range(1, 2001):
        P, M, V = L.adam(P, {"w": P["w"] - 2.0}, M, V, n, 0.05)
    assert abs(P["w"][0] - 2.0) < 1e-2


def test_guard_keeps_plain_step():
    rho = np.array([[1.0, 2.0], [0.5, 0.1]])
    d = np.array([[0.01, -0.02], [0.0, -0.2]])
    new, skipped = L.apply(rho, d, 0.5)
    assert skipped and np.array_equal(new, rho)
    new, skipped = L.apply(rho, 0.1 * d, 0.5)
    assert not skipped and np.allclose(new, rho + 0.1 * d)


def _fine_faces(ny, R):
    rin, rout = 0.4, 2.5
    return rin * (rout / rin) ** (np.arange(ny * R + 1) / (ny * R))


def test_restriction_conserves_mass_and_constants():
    """Mass over the coarse zones equals mass over the fine zones; constant
    fields restrict to themselves; a density linear in r restricts to the
    exact mean of r over the zone in the r dr measure."""
    R, ny, nx = 4, 5, 6
    yf = _fine_faces(ny, R)
    rng = _rng(7)
    rho = 1.0 + rng.random((ny * R, nx * R))
    vx = rng.standard_normal((ny * R, nx * R))
    vy = rng.standard_normal((ny * R, nx * R))
    rc, vxc, vyc = L.restrict(rho, vx, vy, yf, R)
    a, b = yf[:-1], yf[1:]
    wf = 0.5 * (b * b - a * a)
    yc = yf[::R]
    wc = 0.5 * (yc[1:] ** 2 - yc[:-1] ** 2)
    mf = np.sum(rho * wf[:, None]) / R      # dphi_fine = dphi_coarse / R
    mc = np.sum(rc * wc[:, None])
    assert abs(mf - mc) <= 1e-13 * mf
    one = np.full((ny * R, nx * R), 2.5)
    r1, v1, w1 = L.restrict(one, one, one, yf, R)
    assert np.allclose(r1, 2.5, rtol=1e-14) and np.allclose(v1, 2.5, rtol=1e-14) and np.allclose(w1, 2.5)
    rf = 0.5 * (a + b)
    lin = np.repeat(rf[:, None], nx * R, axis=1)
    r2, _, _ = L.restrict(lin, one, one, yf, R)
    want = np.array([np.sum(rf[J * R:(J + 1) * R] * wf[J * R:(J + 1) * R]) / np.sum(wf[J * R:(J + 1) * R])
                     for J in range(ny)])
    assert np.allclose(r2[:, 0], want, rtol=1e-14)


def test_restriction_samples_the_coarse_faces():
    """A face velocity that depends only on the face's position restricts to
    its value on the coarse face: v_y on a coarse Y face is the mean of the
    fine Y faces lying on it, v_x on a coarse X face the dr-weighted mean of
    the fine X faces on it."""
    R, ny, nx = 4, 3, 5
    yf = _fine_faces(ny, R)
    phi_f = np.arange(nx * R) * (2 * np.pi / (nx * R))
    vy = np.repeat(np.cos(phi_f)[None, :], ny * R, axis=0)
    vx = np.repeat(np.sin(phi_f)[None, :], ny * R, axis=0)
    rho = np.ones((ny * R, nx * R))
    _, vxc, vyc = L.restrict(rho, vx, vy, yf, R)
    phi_c = np.arange(nx) * (2 * np.pi / nx)
    assert np.allclose(vxc, np.sin(phi_c)[None, :], atol=1e-15)
    want = np.array([np.cos(phi_c + a * 2 * np.pi / (nx * R)) for a in range(R)]).mean(axis=0)
    assert np.allclose(vyc, want[None, :], atol=1e-15)


def test_fp32_sum_bound_and_rounding_interval():
    """The checker the GPU tests use: a sum of bfloat16 products accumulated
    in FP32 in any order stays within sum_bound of the exact sum, and its
    stored rounding within interval(); a conv with its taps mirrored (a
    plausible indexing mistake) lands outside the intervals."""
    rng = np.random.default_rng(7)
    x = L.bf16(rng.standard_normal((6, 16, 32)))
    w = L.bf16(0.1 * rng.standard_normal((32, 3, 3, 32)))
    b = rng.standard_normal(32).astype(np.float32).astype(np.float64)
    z = L.conv(x, w, b)
    za = L.conv(np.abs(x), np.abs(w), np.abs(b))
    d = L.sum_bound(9 * 32 + 1, za)
    # FP32 accumulation, tap by tap and channel by channel, bias last
    acc = np.zeros(z.shape, dtype=np.float32)
    xp = np.zeros((8, 16, 32))
    xp[1:-1] = x
    for ty in range(3):
        for tx in range(3):
            sh = np.roll(xp[ty:ty + 6], -(tx - 1), axis=1).astype(np.float32)
            for ci in range(32):
                acc = acc + sh[..., ci:ci + 1] * w[:, ty, tx, ci].astype(np.float32)
    acc = acc + b.astype(np.float32)
    assert np.all(np.abs(acc.astype(np.float64) - z) <= d)
    lo, mid, hi = L.interval(z, d, relu=True)
    got = L.bf16(np.maximum(acc, np.float32(0.0)))
    assert np.all((got >= lo) & (got <= hi))
    assert np.count_nonzero(got != mid) <= max(8, got.size // 1000)
    # the same layer with mirrored taps
    bad = L.conv(x, w[:, ::-1, ::-1, :], b)
    got_bad = L.bf16(np.maximum(np.float32(bad), np.float32(0.0)))
    outside = np.count_nonzero((got_bad < lo) | (got_bad > hi))
    assert outside > got.size // 2
