"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

Each test names the passage it follows.  None of these compares the oracle
with itself: they use closed forms, invariants stated in the paper, brute
force on tiny inputs, the exact Riemann solution and convergence orders.
"""
import math
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1602_02359_amd import workloads as W
from helpers import active, oracle_run_to, read_golden
import riemann

NG = W.NGH


# ---------------------------------------------------------------------------
# Appendix A: geometric coefficients (Tab. "geom", Eqs. 70-71)
# ---------------------------------------------------------------------------

def _mesh(geometry, ny=12, nz=10, nx=16):
    if geometry == "cart":
        return W.default_params(geometry="cart", nx=nx, ny=ny, nz=nz, xmin=0.0, xmax=1.3,
                                ymin=W.uniform_faces(-0.5, 2.0, ny), zmin=W.uniform_faces(0.1, 0.9, nz))
    if geometry == "cyl":
        return W.default_params(geometry="cyl", nx=nx, ny=ny, nz=nz, xmin=0.0, xmax=2 * math.pi,
                                ymin=W.log_faces(0.4, 2.5, ny), zmin=W.uniform_faces(-0.2, 0.3, nz))
    return W.default_params(geometry="sph", nx=nx, ny=ny, nz=nz, xmin=0.0, xmax=2 * math.pi,
                            ymin=W.log_faces(0.4, 2.5, ny), zmin=W.uniform_faces(1.2, 1.9, nz))


@pytest.mark.parametrize("geometry", ["cart", "cyl", "sph"])
def test_volume_sum_is_analytic_volume(geometry):
    """Eqs. 70-71 give exact volumes: their sum is the analytic box, annulus or
    spherical-shell sector volume (Appendix A asks the reader to check this)."""
    p = _mesh(geometry)
    g = O.geometry(p)
    y0, y1 = p["ymin"][NG], p["ymin"][NG + p["ny"]]
    z0, z1 = p["zmin"][NG], p["zmin"][NG + p["nz"]]
    dphi = p["xmax"] - p["xmin"]
    vol = g["vol"][NG:NG + p["nz"], NG:NG + p["ny"]].sum() * p["nx"]
    if geometry == "cart":
        exact = dphi * (y1 - y0) * (z1 - z0)
    elif geometry == "cyl":
        exact = 0.5 * (y1 ** 2 - y0 ** 2) * dphi * (z1 - z0)
    else:
        exact = (y1 ** 3 - y0 ** 3) / 3.0 * dphi * (math.cos(z0) - math.cos(z1))
    assert abs(vol / exact - 1.0) < 1e-13


@pytest.mark.parametrize("geometry", ["cyl", "sph"])
def test_face_areas_make_exact_divergences(geometry):
    """Face areas of Tab. "geom": the radial fields 1/r (cyl) and 1/r^2 (sph)
    are divergence free, div(r e_r) = 2 (cyl) or 3 (sph), and in spherical
    geometry v_theta = 1/sin(theta) is divergence free."""
    p = _mesh(geometry)
    g = O.geometry(p)
    ymin = p["ymin"]
    zmin = p["zmin"]
    sy, sz, vol = g["sy"], g["sz"], g["vol"]
    power = 1 if geometry == "cyl" else 2
    flux = sy[:, :] / ymin[None, :-1] ** power  # flux of r**-power through face j
    assert np.allclose(flux, flux[:, :1], rtol=1e-14, atol=0)
    # div(r e_r) through cells j = 0..nyg-2
    out = sy[:, 1:] * ymin[None, 1:-1]
    inn = sy[:, :-1] * ymin[None, :-2]
    div = (out - inn) / vol[:, :-1]
    assert np.allclose(div, power + 1, rtol=1e-12, atol=0)
    if geometry == "sph":
        fz = sz / np.sin(zmin[:-1])[:, None]
        assert np.allclose(fz, fz[:1, :], rtol=1e-14, atol=0)


def test_azimuthal_length_cylindrical_is_volume_over_area():
    """With arithmetic cell centres (a reading of Sect. 2.3), V/S_x = r_med dphi
    in cylindrical geometry, the azimuthal length used everywhere in X."""
    p = _mesh("cyl")
    g = O.geometry(p)
    assert np.allclose(g["vol"] / g["sx"], g["dxlen"], rtol=1e-14, atol=0)
    rmed = W.centres(p["ymin"])
    assert np.allclose(g["dxlen"], rmed[None, :] * (2 * math.pi / p["nx"]), rtol=1e-15, atol=0)


def test_cartesian_face_areas():
    p = _mesh("cart")
    g = O.geometry(p)
    dx = (p["xmax"] - p["xmin"]) / p["nx"]
    Ly = np.diff(p["ymin"])[None, :]
    Lz = np.diff(p["zmin"])[:, None]
    assert np.allclose(g["sx"] * dx, g["vol"], rtol=1e-14)
    assert np.allclose(g["sy"] * Ly, g["vol"], rtol=1e-14)
    assert np.allclose(g["sz"] * Lz, g["vol"], rtol=1e-14)


# ---------------------------------------------------------------------------
# Box 3 and the orbital-advection split (Eqs. 29, 32, 37)
# ---------------------------------------------------------------------------

def test_v0_is_midrange_and_minimises_residual_norm():
    """Eq. 37: v0 = (max + min)/2 per ring (brute force); it gives the residual
    velocity with the smallest sup norm (the property the paper asks for)."""
    pr = W.random_problem("cyl", nx=37, ny=5, nz=4, seed=3)
    vx = pr.fields["vx"]
    v0, N, xi = O.ring_split(pr.params, vx, 0.01)
    ring = vx[NG:NG + 4, NG:NG + 5, :]
    assert np.array_equal(v0, 0.5 * (ring.max(axis=2) + ring.min(axis=2)))
    norm = np.abs(ring - v0[..., None]).max(axis=2)
    for eps in (1e-3, -1e-3, 1e-7, -1e-7):
        other = np.abs(ring - (v0 + eps)[..., None]).max(axis=2)
        assert np.all(norm <= other)


def test_split_integer_and_residual():
    """Eq. 29: N = nearest integer of D = v0 dt/dX, residual xi = D - N with
    |xi| <= 1/2; N + xi reproduces D exactly.  Ties: both neighbours are
    valid, the oracle takes the one away from zero."""
    rng = np.random.default_rng(7)
    for _ in range(2000):
        v0 = rng.normal() * 3.0
        dt = rng.random() * 0.05 + 1e-4
        dX = rng.random() * 0.01 + 1e-4
        N, xi = O.split_shift(v0, dt, dX)
        D = (v0 * dt) / dX
        assert abs(xi) <= 0.5
        assert N + xi == D
        assert float(N) == round(N)
    assert O.split_shift(2.5, 1.0, 1.0) == (3, -0.5)
    assert O.split_shift(-2.5, 1.0, 1.0) == (-3, 0.5)
    assert O.split_shift(0.49999999999999994, 1.0, 1.0) == (0, 0.49999999999999994)
    assert O.split_shift(0.0, 1.0, 1.0) == (0, 0.0)


def test_shift_is_circular_permutation():
    """Eq. 32: Q_i <- Q_{i-N}; a pure permutation (np.roll), N then -N is the
    identity, N = nx is the identity."""
    pr = W.random_problem("cart", nx=29, ny=4, nz=3, seed=4)
    p = pr.params
    f = pr.fields["rho"].copy()
    rng = np.random.default_rng(1)
    N = rng.integers(-40, 40, size=(3, 4)).astype(np.int32)
    g = f.copy()
    O.shift(p, g, N)
    for k in range(3):
        for j in range(4):
            ring = f[NG + k, NG + j]
            assert np.array_equal(g[NG + k, NG + j], np.roll(ring, int(N[k, j])))
    # ghosts untouched
    assert np.array_equal(g[:NG], f[:NG]) and np.array_equal(g[:, :NG], f[:, :NG])
    O.shift(p, g, -N)
    assert np.array_equal(g, f)
    O.shift(p, g, np.full((3, 4), 29, np.int32))
    assert np.array_equal(g, f)


# ---------------------------------------------------------------------------
# PPA fractional residual (Eqs. 34-36 and the interface formula)
# ---------------------------------------------------------------------------

def _edges(q):
    """Limited left/right edge values, read back from the interface values
    with a vanishing shift of either sign."""
    QR = np.roll(O.ppa_faces(q, 0.0), -1)   # face f carries QR of zone f-1
    QL = O.ppa_faces(q, -5e-324)             # face f carries QL of zone f
    return QL, QR


def test_ppa_interface_value_is_average_of_parabola():
    """The interface value equals the mean of the zone's reconstructed
    parabola over the fraction |xi| of the zone that crosses the face, for
    either sign of xi; checked by exact polynomial integration."""
    rng = np.random.default_rng(11)
    n = 40
    q = np.cumsum(rng.normal(size=n)) + 3.0 * np.sin(np.arange(n) / 3.0)
    QL, QR = _edges(q)
    for xi in (0.37, -0.37, 0.5, -0.5, 0.05, -0.21, 1.0, -1.0):
        star = O.ppa_faces(q, xi)
        x = abs(xi)
        for f in range(n):
            u = (f - 1) % n if xi >= 0 else f
            dQ = QR[u] - QL[u]
            q6 = 6.0 * (q[u] - 0.5 * (QL[u] + QR[u]))
            par = np.polynomial.Polynomial([QL[u], dQ + q6, -q6])  # QL + x (dQ + q6 (1 - x))
            P = par.integ()
            lo, hi = (1.0 - x, 1.0) if xi >= 0 else (0.0, x)
            avg = (P(hi) - P(lo)) / (hi - lo) if x > 0 else par(hi if xi >= 0 else lo)
            assert abs(star[f] - avg) <= 1e-12 * (1 + abs(avg))
    # the parabola of each zone has the zone's mean
    q6 = 6.0 * (q - 0.5 * (QL + QR))
    assert np.allclose(0.5 * (QL + QR) + q6 / 6.0, q, rtol=0, atol=1e-12)


def test_ppa_edges_monotone_and_flat_at_extrema():
    """Eq. 36: after the fixes each zone's parabola is monotone (|q6| <= |dQ|)
    and zones at local extrema are flat."""
    rng = np.random.default_rng(12)
    q = rng.normal(size=64)
    QL, QR = _edges(q)
    dQ = QR - QL
    q6 = 6.0 * (q - 0.5 * (QL + QR))
    assert np.all(np.abs(q6) <= np.abs(dQ) * (1 + 1e-12) + 1e-13)
    ext = (np.roll(q, -1) - q) * (q - np.roll(q, 1)) <= 0
    assert np.all(QL[ext] == q[ext]) and np.all(QR[ext] == q[ext])


def test_ppa_edge_value_exact_for_cubic():
    """Eq. 35 without limiting is the fourth-order interface value: exact for
    the zone averages of a cubic (on a smooth monotone stretch)."""
    n, h = 64, 0.05
    x = np.arange(n) * h
    cub = np.polynomial.Polynomial([1.0, 1.0, 0.2, 0.1])
    P = cub.integ()
    avg = (P(x + h) - P(x)) / h
    # close the ring smoothly far from the checked stretch
    q = avg.copy()
    QL, QR = _edges(q)
    for i in range(3, n - 4):
        assert abs(QR[i] - cub(x[i] + h)) < 1e-12


def test_ppa_unit_and_zero_shift():
    """|xi| = 1 moves every zone by exactly one (Q* = upwind zone value); xi = 0
    changes nothing; a uniform ring is invariant (bitwise)."""
    rng = np.random.default_rng(13)
    n = 33
    rho = 1.0 + rng.random(n)  # within a factor two: differences are exact
    Q = [rng.normal(size=n)]
    r1 = rho.copy()
    q1 = O.ppa_ring(r1, [Q[0].copy()], 1.0, 1.0, 1.0, 1.0)
    assert np.array_equal(r1, np.roll(rho, 1))
    assert np.allclose(q1[0], np.roll(Q[0], 1), rtol=0, atol=1e-14)
    r2 = rho.copy()
    q2 = O.ppa_ring(r2, [Q[0].copy()], -1.0, 1.0, 1.0, 1.0)
    assert np.array_equal(r2, np.roll(rho, -1))
    assert np.allclose(q2[0], np.roll(Q[0], -1), rtol=0, atol=1e-14)
    r3 = rho.copy()
    q3 = O.ppa_ring(r3, [Q[0].copy()], 0.0, 0.7, 1.3, 2.1)
    assert np.array_equal(r3, rho) and np.array_equal(q3[0], Q[0])
    ru = np.full(n, 1.7)
    qu = O.ppa_ring(ru, [np.full(n, -0.3)], 0.41, 0.7, 1.3, 2.1)
    assert np.all(ru == 1.7) and np.all(qu[0] == -0.3)


def test_ppa_conserves_and_commutes_with_shift():
    """Conservative update (sums preserved to round-off); the residual PPA step
    and the integer shift commute bitwise, since both act identically on
    every zone of a periodic ring."""
    rng = np.random.default_rng(14)
    n = 50
    rho = 0.5 + rng.random(n)
    Q = [rng.normal(size=n), rng.normal(size=n)]
    r = rho.copy()
    out = O.ppa_ring(r, [a.copy() for a in Q], -0.43, 0.9, 1.1, 1.0 / (0.9 * 1.1))
    assert abs(r.sum() - rho.sum()) < 1e-13 * rho.sum()
    for a, b in zip(out, Q):
        assert abs(a.sum() - b.sum()) < 1e-13 * np.abs(b).sum()
    N = 17
    r2 = np.roll(rho, N)
    out2 = O.ppa_ring(r2, [np.roll(a, N) for a in Q], -0.43, 0.9, 1.1, 1.0 / (0.9 * 1.1))
    assert np.array_equal(r2, np.roll(r, N))
    for a, b in zip(out2, out):
        assert np.array_equal(a, np.roll(b, N))


def test_ppa_third_order_on_smooth_profile():
    """PPA advection of zone averages of a smooth periodic profile converges at
    third order away from extrema (order > 2.5 in the L1 norm)."""
    errs = []
    xi = 0.3
    for n in (32, 64, 128, 256):
        h = 1.0 / n
        x = np.arange(n) * h
        F = lambda s: -np.cos(2 * np.pi * s) / (2 * np.pi) + 0.3 * s  # antiderivative of sin + const
        avg = (F(x + h) - F(x)) / h + 2.0
        exact = (F(x + h - xi * h) - F(x - xi * h)) / h + 2.0
        rho = np.ones(n)
        q = O.ppa_ring(rho, [avg.copy()], xi, 1.0, 1.0, 1.0)
        errs.append(np.abs(q[0] - exact).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert orders[-1] > 2.5, orders


# ---------------------------------------------------------------------------
# van Leer upwind sweep (Eqs. flux, 14, 15)
# ---------------------------------------------------------------------------

def _line(faces, w, dt, Qfun, rho=None):
    """Build a line of n zones (2 ghosts each side) on the given faces."""
    n = len(faces) - 5
    xc = 0.5 * (faces[:-1] + faces[1:])  # zones -2..n+1 (n+4 values)
    L = np.diff(faces)
    h = np.diff(xc)                          # centre distances at faces -1..n+1
    Q = Qfun(xc)
    r = np.ones(n + 4) if rho is None else rho
    wf = np.full(n + 1, w)
    S = np.ones(n + 1)
    Vi = 1.0 / L[2:2 + n]
    return n, xc, L, h, Q, r, wf, S, Vi


@pytest.mark.parametrize("w", [0.7, -0.7])
def test_vanleer_advects_linear_profile_exactly_on_stretched_mesh(w):
    """A linear profile is advected exactly: the harmonic-mean slope of a linear
    profile is its slope, and Eq. 15 evaluated with the upwind zone's own width
    (a reading of the garbled v < 0 branch) lands on x_f - w dt/2."""
    faces = np.cumsum(np.r_[0.0, 0.1 * 1.07 ** np.arange(26)])
    dt = 0.05
    n, xc, L, h, Q, r, wf, S, Vi = _line(faces, w, dt, lambda x: 0.3 + 2.0 * x)
    out = O.sweep_line(r.copy(), [Q.copy()], wf, L, h, S, Vi, dt)[0]
    exact = 0.3 + 2.0 * (xc - w * dt)
    assert np.allclose(out[2:2 + n], exact[2:2 + n], rtol=0, atol=1e-13)


def test_vanleer_uniform_state_bitwise_and_tvd():
    """Uniform data are unchanged bitwise (the slope is zero when the one-sided
    differences vanish); random data gain no new extrema at |Courant| <= 1."""
    faces = np.arange(45, dtype=float) * 0.1
    dt = 0.1
    n, xc, L, h, Q, r, wf, S, Vi = _line(faces, 0.8, dt, lambda x: np.full_like(x, 1.25))
    out = O.sweep_line(r.copy(), [Q.copy()], wf, L, h, S, Vi, dt)[0]
    assert np.all(out == 1.25)
    rng = np.random.default_rng(21)
    for w in (0.9, -0.9, 0.3):
        q = rng.random(n + 4)
        out = O.sweep_line(np.ones(n + 4), [q.copy()], np.full(n + 1, w), L, h, S, Vi, dt)[0]
        assert out[2:2 + n].max() <= q.max() + 1e-15
        assert out[2:2 + n].min() >= q.min() - 1e-15


def test_vanleer_closed_line_conserves():
    """Finite-volume form: with no flow through the end faces the volume sums of
    rho and of every other quantity are conserved to round-off."""
    rng = np.random.default_rng(22)
    faces = np.cumsum(np.r_[0.0, 0.05 + 0.1 * rng.random(34)])
    n = len(faces) - 5
    xc = 0.5 * (faces[:-1] + faces[1:])
    L = np.diff(faces)
    h = np.diff(xc)
    w = rng.normal(size=n + 1) * 0.3
    w[0] = w[-1] = 0.0
    rho = 0.5 + rng.random(n + 4)
    Q = rng.normal(size=n + 4)
    Vi = 1.0 / L[2:2 + n]
    r = rho.copy()
    out = O.sweep_line(r, [Q.copy()], w, L, h, np.ones(n + 1), Vi, 0.05)[0]
    V = L[2:2 + n]
    assert abs((r[2:2 + n] * V).sum() - (rho[2:2 + n] * V).sum()) < 1e-14 * (rho[2:2 + n] * V).sum()
    assert abs((out[2:2 + n] * V).sum() - (Q[2:2 + n] * V).sum()) < 1e-14 * np.abs(Q[2:2 + n] * V).sum()


# ---------------------------------------------------------------------------
# Box 6: time step (Eq. cfl2, Eq. 38)
# ---------------------------------------------------------------------------

def test_cfl_static_box_closed_form():
    """At rest only item 1 acts: dt = C min(L_d)/c_s (Eq. cfl2)."""
    p = W.default_params(geometry="cart", nx=8, ny=5, nz=6, xmin=0.0, xmax=0.8,
                         ymin=W.uniform_faces(0.0, 0.35, 5), zmin=W.uniform_faces(0.0, 0.9, 6),
                         eos="iso", bc=("reflect",) * 4)
    pr = W._blank(p)
    pr.fields["cs"][:] = 2.0
    dt = O.cfl_dt(p, pr.copy_fields())
    assert abs(dt / (0.44 * 0.07 / 2.0) - 1.0) < 1e-15


def test_cfl_disk_closed_form_and_orbital_gain():
    """A disk rotating uniformly on each ring with v_r = 0: with orbital
    advection the residual velocity vanishes and dt = C min(dX, dr)/c_s; the
    gain over plain transport is of order 1/h (Sect. 3.5.2)."""
    pr = W.disk2d_cyl(noise=0.0)
    p = pr.params
    dt_f = O.cfl_dt(p, pr.copy_fields())
    r = W.centres(p["ymin"])[NG:NG + p["ny"]]
    dr = np.diff(p["ymin"])[NG:NG + p["ny"]]
    dX = r * 2 * math.pi / p["nx"]
    cs = 0.05 / np.sqrt(r)
    expect = 0.44 * np.min(np.minimum(dX, dr) / cs)
    assert abs(dt_f / expect - 1.0) < 1e-14
    p2 = dict(p, fargo=False)
    dt_p = O.cfl_dt(p2, pr.copy_fields())
    gain = dt_f / dt_p
    assert 0.5 / 0.05 < gain < 2.0 / 0.05


def test_shear_limit_active_only_for_unresolved_scale_height():
    """Eq. 38 only matters when dr > 2H/3 (Sect. 3.5.2)."""
    coarse = W.disk2d_cyl(nx=64, ny=8, rin=0.5, rout=2.0, h=0.02, noise=0.0)
    fine = W.disk2d_cyl(nx=1024, ny=256, rin=0.5, rout=2.0, h=0.02, noise=0.0)
    for pr, active_expected in ((coarse, True), (fine, False)):
        on = O.cfl_dt(pr.params, pr.copy_fields())
        off = O.cfl_dt(dict(pr.params, shear_c0=0.0), pr.copy_fields())
        if active_expected:
            assert on < 0.5 * off
        else:
            assert on == off


def _cart2d(nx=4, ny=5, xlen=4.0, ylo=0.0, yhi=2.5, cs=0.01, **kw):
    """A Cartesian 2D box at rest, isothermal, with FIXED Y sides (ghosts and
    boundary faces as the caller writes them)."""
    kw.setdefault("bc", ("fixed", "fixed", "reflect", "reflect"))
    p = W.default_params(geometry="cart", nx=nx, ny=ny, nz=1, xmin=0.0, xmax=xlen,
                         ymin=W.uniform_faces(ylo, yhi, ny), zmin=np.array([0.0, 1.0]), eos="iso", **kw)
    pr = W._blank(p)
    pr.fields["cs"][:] = cs
    return pr


def test_cfl_item2_takes_both_faces_of_a_cell():
    """Item 2 of Eq. cfl2 with the speed of a cell read on both of its faces
    along j (reading R11).  A 4 x 5 box (dx = 1, dy = 0.5) at rest but for the
    boundary faces: v_y = V on the upper face of the top row (column 2) and
    -2V on the lower face of the bottom row (column 1); the walls are FIXED, so
    box 2 keeps both, and item 3 is off.  The bottom cell of column 1 limits:
    its steps are 0.5/(2V) (item 2) and min(1, 0.5)/c_s (item 1), so
    dt = C / sqrt((2V/0.5)^2 + (c_s/0.5)^2).  Without the -2V face the top
    cell of column 2 limits, with V in place of 2V; a cell read on one face
    only misses one of the two."""
    V, cs = 3.0, 0.01
    for lo, hi in ((-2 * V, V), (0.0, V), (-2 * V, 0.0)):
        pr = _cart2d(cs=cs, cvnr=0.0)
        f = pr.fields
        f["vy"][0, NG, 1] = lo          # lower face of the bottom active row
        f["vy"][0, NG + 5, 2] = hi      # upper face of the top active row
        u = max(abs(lo), abs(hi))
        expect = 0.44 / math.sqrt((u / 0.5) ** 2 + (cs / 0.5) ** 2)
        dt = O.cfl_dt(pr.params, pr.copy_fields())
        assert abs(dt / expect - 1.0) < 1e-15, (lo, hi, dt, expect)


def test_cfl_item3_uniform_compression():
    """Item 3 of Eq. cfl2 (reading R9: L / (4 C_av^2 |dv|) on compressed
    directions) in a uniform compression v_y = -a y on [-2, 2], 8 rows of 0.5,
    with c_s = 0 and FIXED walls.  Every row has dv = -a dy, so item 3 gives
    1/(4 C_av^2 a) = 1/(8a) for C_av = sqrt(2); item 2 is largest in the two
    end rows, where |v_y| = 2a on the wall face: 0.5/(2a).  Hence
    dt = C / (a sqrt(4^2 + 8^2)) = C / (a sqrt(80)), and without the factor 4
    on C_av^2 it would be C / (a sqrt(20))."""
    a = 1.7
    pr = _cart2d(ny=8, ylo=-2.0, yhi=2.0, cs=0.0)
    y = pr.params["ymin"][:-1]
    pr.fields["vy"][0, :, :] = (-a * y)[:, None]
    dt = O.cfl_dt(pr.params, pr.copy_fields())
    assert abs(dt / (0.44 / (a * math.sqrt(80.0))) - 1.0) < 1e-14, dt
    # the same compression along Z in 3D (the third direction of the item)
    p = W.default_params(geometry="cart", nx=3, ny=3, nz=8, xmin=0.0, xmax=3.0,
                         ymin=W.uniform_faces(0.0, 3.0, 3), zmin=W.uniform_faces(-2.0, 2.0, 8), eos="iso",
                         bc=("reflect", "reflect", "fixed", "fixed"))
    pz = W._blank(p)
    pz.fields["cs"][:] = 0.0
    z = p["zmin"][:-1]
    pz.fields["vz"][:] = (-a * z)[:, None, None]
    dt = O.cfl_dt(p, pz.copy_fields())
    assert abs(dt / (0.44 / (a * math.sqrt(80.0))) - 1.0) < 1e-14, dt


def _rings(omegas, nx=16, rin=1.0, rout=2.0, cs=0.01):
    """A cylindrical 2D disk whose ring j turns rigidly at the angular speed
    omegas[j] (ghost rings included), with orbital advection on."""
    ny = len(omegas) - 2 * NG
    p = W.default_params(geometry="cyl", nx=nx, ny=ny, nz=1, xmin=0.0, xmax=2 * math.pi,
                         ymin=W.uniform_faces(rin, rout, ny), zmin=np.array([0.0, 1.0]), eos="iso",
                         fargo=True, bc=("fixed", "fixed", "reflect", "reflect"))
    pr = W._blank(p)
    pr.fields["cs"][:] = cs
    r = W.centres(p["ymin"])
    pr.fields["vx"][0, :, :] = (np.asarray(omegas) * r)[:, None]
    return pr


def test_shear_limit_eq38_compares_angular_speeds():
    """Eq. 38 divides each ring's velocity by its own azimuthal length, so it
    measures the difference of angular speeds.  A rigid rotation (any rate)
    has no shear and the sound speed sets dt = C min(dr, r dphi)/c_s; rings
    turning at 10 j (j the ring index) differ by 10 everywhere, so the shear
    step is C0 dphi / 10 and binds.  With orbital advection the rings' own
    rotation is removed from item 2 (uniform rings: no residual)."""
    ny = 8
    rigid = _rings([50.0] * (ny + 2 * NG))
    dt = O.cfl_dt(rigid.params, rigid.copy_fields())
    dphi = 2 * math.pi / 16
    assert abs(dt / (0.44 * min(1.0 / ny, 1.0 * dphi) / 0.01) - 1.0) < 1e-14, dt
    diff = _rings([10.0 * j for j in range(ny + 2 * NG)])
    dt = O.cfl_dt(diff.params, diff.copy_fields())
    assert abs(dt / (0.44 * dphi / 10.0) - 1.0) < 1e-13, dt


def test_v0_mean_mode_by_brute_force():
    """v0 as the azimuthal mean (Sect. 3.5.1, the alternative to Eq. 37), on
    dyadic values whose sum is exact in any order, so the mean is the brute
    force one to the last bit; then its effect on item 2 of Eq. cfl2: a ring
    reading (0, 0, 0, V) has v0 = V/4 and a largest residual 3V/4 (against
    V/2 for the midrange), so dt = C dx / (3V/4)."""
    rng = np.random.default_rng(17)
    pr = W.random_problem("cyl", nx=64, ny=5, nz=4, seed=3)
    p = dict(pr.params, v0_mode="mean", fargo=True)
    vx = pr.fields["vx"].copy()
    vx[:] = rng.integers(-1024, 1024, size=vx.shape) / 256.0
    v0, N, xi = O.ring_split(p, vx, 0.01)
    ring = vx[NG:NG + 4, NG:NG + 5, :]
    assert np.array_equal(v0, ring.sum(axis=2) / 64.0)
    assert not np.array_equal(v0, 0.5 * (ring.max(axis=2) + ring.min(axis=2)))
    V = 0.8
    for mode, resid in (("mean", 0.75 * V), ("minmax", 0.5 * V)):
        q = _cart2d(nx=4, ny=3, xlen=4.0, cs=0.0, cvnr=0.0, fargo=True, v0_mode=mode)
        q.fields["vx"][0, :, 3] = V
        dt = O.cfl_dt(q.params, q.copy_fields())
        assert abs(dt / (0.44 * 1.0 / resid) - 1.0) < 1e-15, (mode, dt)


# ---------------------------------------------------------------------------
# Whole step: invariants and physics
# ---------------------------------------------------------------------------

def _periodic_box(eos="adi", seed=0, n=(12, 9, 7), fargo=False, uniform=False):
    nx, ny, nz = n
    p = W.default_params(geometry="cart", nx=nx, ny=ny, nz=nz, xmin=0.0, xmax=1.0,
                         ymin=W.uniform_faces(0.0, 0.75, ny), zmin=W.uniform_faces(0.0, 0.6, nz),
                         eos=eos, fargo=fargo, bc=("periodic",) * 4)
    pr = W._blank(p)
    rng = np.random.default_rng(100 + seed)
    f = pr.fields
    if uniform:
        f["vx"][:] = 0.37
        f["vy"][:] = -0.21
        f["vz"][:] = 0.11
        if eos == "adi":
            f["e"][:] = 2.5
        else:
            f["cs"][:] = 1.3
        f["pot"][:] = 0.0
    else:
        f["rho"][:] = 0.5 + rng.random(pr.shape)
        for k in ("vx", "vy", "vz"):
            f[k][:] = 0.3 * (2 * rng.random(pr.shape) - 1)
        if eos == "adi":
            f["e"][:] = 0.5 + rng.random(pr.shape)
        else:
            f["cs"][:] = 0.5 + 0.5 * rng.random(pr.shape)
    return pr


@pytest.mark.parametrize("eos,fargo", [("adi", False), ("iso", True), ("adi", True)])
def test_uniform_state_is_preserved_bitwise(eos, fargo):
    """A uniform state with rho = 1 is a solution; the step keeps it exactly
    (Eq. 18 on the old momenta returns the old velocity, Sect. 3.4.1)."""
    pr = _periodic_box(eos=eos, fargo=fargo, uniform=True)
    f = pr.copy_fields()
    for _ in range(3):
        O.step(pr.params, f)
    for k in ("rho", "vx", "vy", "vz", "e"):
        if f[k] is not None:
            assert np.array_equal(active(pr, f[k]), active(pr, pr.fields[k])), k


@pytest.mark.parametrize("eos", ["adi", "iso"])
def test_mass_and_momenta_conserved_on_periodic_box(eos):
    """Mass and the three momenta sum(rho (v_- + v_+)/2 V) are conserved to
    round-off: the pressure and viscous-pressure sources telescope (Eqs.
    20-25), transport is in flux form and Eq. 18 keeps the sum of left and
    right momenta (Sect. 3.4.1)."""
    pr = _periodic_box(eos=eos, seed=1)
    f = pr.copy_fields()
    O.cfl_dt(pr.params, f)  # box 2: periodic images of the upper faces
    s0, a0 = O.sums(pr.params, f)
    for _ in range(3):
        O.step(pr.params, f)
    s1, a1 = O.sums(pr.params, f)
    for q in range(4):
        assert abs(s1[q] - s0[q]) < 1e-13 * a0[q], (q, s0[q], s1[q])


def test_disk_mass_and_angular_momentum_conserved():
    """Disk with closed radial walls (v_r = 0 on the boundary faces) and an
    axisymmetric potential: mass and angular momentum are conserved to
    round-off, with orbital advection on (Sect. 3.5.1, last paragraphs)."""
    pr = W.disk2d_cyl(nx=96, ny=32, noise=1e-2, omega=0.3)
    f = pr.copy_fields()
    s0, a0 = O.sums(pr.params, f)
    for _ in range(5):
        O.step(pr.params, f)
    s1, a1 = O.sums(pr.params, f)
    assert abs(s1[0] - s0[0]) < 1e-13 * a0[0]
    assert abs(s1[1] - s0[1]) < 1e-13 * a0[1]


@pytest.mark.parametrize("geometry", ["sph", "cyl"])
def test_3d_disk_sector_conserves_mass_and_angular_momentum(geometry):
    """3D random state, reflecting Z walls, fixed radial walls with v_r = 0 on
    the boundary faces, axisymmetric potential, rotating frame, orbital
    advection: mass and angular momentum conserved to round-off."""
    pr = W.random_problem(geometry, nx=24, ny=8, nz=6, eos="adi", seed=5, fargo=True, omega=0.7,
                          bc=("fixed", "fixed", "reflect", "reflect"))
    f = pr.fields
    r = W.centres(pr.params["ymin"])[None, :, None]
    f["pot"][:] = np.broadcast_to(-1.0 / r, f["pot"].shape)
    f["vy"][:, NG, :] = 0.0
    f["vy"][:, NG + pr.params["ny"], :] = 0.0
    g = pr.copy_fields()
    O.cfl_dt(pr.params, g)  # box 2: wall faces and ghosts
    s0, a0 = O.sums(pr.params, g)
    for _ in range(3):
        O.step(pr.params, g)
    s1, a1 = O.sums(pr.params, g)
    assert abs(s1[0] - s0[0]) < 1e-13 * a0[0]
    assert abs(s1[1] - s0[1]) < 1e-13 * a0[1]


def test_sod_shock_tube_against_exact_solution_and_paper():
    """Sect. 5.1.1: 300 zones, t = 2.  Exact Riemann solution; the paper's
    printed shock (8.5) and contact (6.9) positions, shock over 2-3 zones,
    contact over 7-8 zones, and a plateau offset of order 1e-2."""
    gd = read_golden("sod_paper.txt")
    pr = W.sod("y", n=int(gd["cells"]))
    f, nsteps = oracle_run_to(O, pr, gd["t_end"])
    rho = f["rho"][0, NG:NG + 300, 0]
    x = W.centres(pr.params["ymin"])[NG:NG + 300]
    ex = riemann.sample(x, gd["t_end"], gd["interface"], gd["rho_left"], 0.0, gd["p_left"],
                        gd["rho_right"], 0.0, gd["p_right"], gd["gamma"])
    rex = ex[0]
    assert np.abs(rho - rex).mean() < 6e-3
    # shock: the plateau behind it and the undisturbed gas ahead
    post, pre = rex[(x > 7.2) & (x < 8.3)].mean(), gd["rho_right"]
    zone = np.where((x > 7.6) & (rho > pre + 0.1 * (post - pre)) & (rho < pre + 0.9 * (post - pre)))[0]
    assert 1 <= len(zone) <= gd["shock_zones_max"]
    xs = x[np.argmin(np.abs(rho[(x > 7.6)] - 0.5 * (post + pre))) + np.where(x > 7.6)[0][0]]
    assert abs(xs - gd["shock_position"]) < 0.1
    # contact
    left = rex[(x > 5.2) & (x < 6.6)].mean()
    zc = np.where((x > 5.5) & (x < 7.6) & (rho > post + 0.1 * (left - post)) & (rho < post + 0.9 * (left - post)))[0]
    assert 1 <= len(zc) <= gd["contact_zones_max"] + 2
    xc = x[zc].mean()
    assert abs(xc - gd["contact_position"]) < 0.15
    plateau = (x > 7.3) & (x < 8.2)
    off = np.abs(rho[plateau] / rex[plateau] - 1.0).max()
    assert off < 2 * gd["plateau_offset"]


def test_sod_along_y_and_z_identical():
    """The directional sweeps are the same operator on different axes: Sod
    along Y (2D mesh) and along Z (3D mesh, periodic in Y) agree bitwise."""
    py, pz = W.sod("y", n=60), W.sod("z", n=60)
    fy, ny_ = oracle_run_to(O, py, 0.5)
    fz, nz_ = oracle_run_to(O, pz, 0.5)
    assert ny_ == nz_
    for k in ("rho", "e"):
        a = fy[k][0, NG:NG + 60, 0]
        for j in range(NG, NG + 3):
            b = fz[k][NG:NG + 60, j, 0]
            assert np.array_equal(a, b)
    assert np.array_equal(fy["vy"][0, NG:NG + 61, 0], fz["vz"][NG:NG + 61, NG, 0])


def test_sound_wave_second_order_and_isotropic():
    """A linear isothermal sound wave returns after one period with an error
    falling as the square of the zone size, identically along X, Y and Z."""
    res = {}
    for ax in "xyz":
        errs = []
        for n in (32, 64):
            pr = W.sound_wave(ax, n=n, amp=1e-6)
            f, _ = oracle_run_to(O, pr, 1.0)
            d = (active(pr, f["rho"]) - active(pr, pr.fields["rho"])).ravel()
            errs.append(np.abs(d).max() / 1e-6)
        res[ax] = errs
        assert errs[0] / errs[1] > 3.5, (ax, errs)
    assert abs(res["x"][1] - res["y"][1]) < 1e-9 and abs(res["y"][1] - res["z"][1]) < 1e-9


def test_orbital_advection_agrees_with_plain_transport_to_truncation_order():
    """Eq. 27 split into Eqs. fargo1/fargo2 is consistent: the difference
    between runs with and without orbital advection on a smooth disk shrinks
    under refinement (second order here), while orbital advection takes far
    fewer steps."""
    diffs, ratio = [], []
    for ny in (16, 32):
        out = {}
        for fg in (True, False):
            pr = W.disk2d_cyl(nx=3 * ny, ny=ny, rin=0.6, rout=1.6, noise=0.0, fargo=fg,
                              bump=(0.05, 1.0, math.pi, 0.15))
            out[fg] = oracle_run_to(O, pr, 1.0)
        diffs.append(np.abs(out[True][0]["rho"] - out[False][0]["rho"])[0, NG:-NG].mean())
        ratio.append(out[False][1] / out[True][1])
    assert diffs[0] / diffs[1] > 3.0, diffs
    assert min(ratio) > 5.0


def test_compressional_heating_keeps_entropy_on_smooth_flow():
    """Box 7c (work of pressure forces, Eq. 8) keeps the specific entropy
    P/rho^gamma of a smooth compressing/expanding flow uniform up to the
    truncation error; dropping or flipping the term would change it at first
    order in the compression."""
    n = 64
    p = W.default_params(geometry="cart", nx=1, ny=n, nz=1, xmin=0.0, xmax=1.0,
                         ymin=W.uniform_faces(0.0, 1.0, n), zmin=np.array([0.0, 1.0]),
                         eos="adi", gamma=1.4, bc=("periodic",) * 4)
    pr = W._blank(p)
    yf = p["ymin"][:-1][None, :, None]
    pr.fields["vy"][:] = np.broadcast_to(0.05 * np.sin(2 * np.pi * yf), pr.shape)
    f, _ = oracle_run_to(O, pr, 0.5)
    rho = f["rho"][0, NG:NG + n, 0]
    P = 0.4 * f["e"][0, NG:NG + n, 0]
    s = P / rho ** 1.4
    # density changes by several percent, entropy by far less
    assert np.abs(rho - 1.0).max() > 0.02
    assert np.abs(s / s.mean() - 1.0).max() < 2e-4


# ---------------------------------------------------------------------------
# Determinism and error handling
# ---------------------------------------------------------------------------

def test_oracle_result_independent_of_thread_count(tmp_path):
    """OpenMP only splits independent zones: 1 and 4 threads agree bitwise."""
    script = r"""
import sys, numpy as np
sys.path.insert(0, %r)
from oracle import oracle as O
from paper_1602_02359_amd import workloads as W
pr = W.random_problem("sph", nx=20, ny=7, nz=5, eos="adi", seed=9, fargo=True, omega=0.4,
                      bc=("fixed", "outflow", "reflect", "outflow"))
f = pr.copy_fields()
for _ in range(2):
    O.step(pr.params, f)
np.savez(sys.argv[1], **{k: v for k, v in f.items() if v is not None})
""" % os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = []
    for th in (1, 4):
        fn = str(tmp_path / ("o%d.npz" % th))
        env = dict(os.environ, OMP_NUM_THREADS=str(th))
        subprocess.run([sys.executable, "-c", script, fn], check=True, env=env)
        outs.append(np.load(fn))
    for k in outs[0].files:
        assert np.array_equal(outs[0][k], outs[1][k]), k


def test_oracle_reports_invalid_and_nonfinite_input():
    pr = W.random_problem("cart", nx=8, ny=5, nz=4, seed=2)
    f = pr.copy_fields()
    f["rho"][NG + 1, NG + 2, 3] = np.nan
    with pytest.raises(O.OracleError) as e:
        O.step(pr.params, f)
    assert e.value.code == -4
    with pytest.raises(O.OracleError) as e:
        O.cfl_dt(dict(pr.params, ny=2), pr.copy_fields())
    assert e.value.code == -1
    with pytest.raises(O.OracleError) as e:
        O.step(dict(pr.params, geometry="cyl", bc=("periodic",) * 4), pr.copy_fields())
    assert e.value.code == -1


@pytest.mark.parametrize("geometry,eos", [("cart", "adi"), ("cyl", "iso"), ("sph", "adi"), ("cyl", "adi")])
@pytest.mark.parametrize("bc", [("reflect", "outflow", "outflow", "reflect"), ("fixed", "fixed", "reflect", "reflect")])
def test_random_states_stay_finite(geometry, eos, bc):
    pr = W.random_problem(geometry, nx=18, ny=6, nz=5, eos=eos, seed=3, fargo=geometry != "cart", bc=bc)
    f = pr.copy_fields()
    for _ in range(3):
        O.step(pr.params, f)
    for k, v in f.items():
        if v is not None:
            assert np.all(np.isfinite(v)), k


# ---------------------------------------------------------------------------
# Source terms: equilibria and exact steady flows
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["cyl2d", "cyl2d_rotframe", "cyl3d", "sph3d"])
def test_equilibrium_disks_stay_in_equilibrium(case):
    """Disks in rotational (and vertical) equilibrium stay at rest up to the
    truncation error, which falls under refinement: the centrifugal terms
    (Eq. 12 and its generalisation), the potential gradient and, in a
    rotating frame, the frame terms of Tab. "momenta" balance the pressure
    gradient.  A missing or wrong term accelerates the gas at O(1)."""
    res = []
    for n in (12, 24):
        if case.startswith("cyl2d"):
            pr = W.disk2d_cyl(nx=8 * n, ny=4 * n, rin=0.6, rout=1.6, noise=0.0,
                              omega=1.0 if case.endswith("rotframe") else 0.0)
        elif case == "cyl3d":
            pr = W.disk3d_cyl_planet(nx=64, ny=16, nz=n, rin=0.8, rout=1.25, zmax=0.1, q=0.0, noise=0.0)
        else:
            pr = W.disk3d_sph(nx=64, ny=16, nz=n, rin=0.8, rout=1.25, nh=2.0, noise=0.0)
        f = pr.copy_fields()
        t = 0.0
        for _ in range(5):
            t += O.step(pr.params, f)
        v = np.abs(active(pr, f["vy"])).max()
        if f["vz"] is not None:
            v = max(v, np.abs(active(pr, f["vz"])).max())
        res.append(v / t)  # mean spurious acceleration
    assert res[1] < 0.02, res
    assert res[0] / res[1] > 1.8, res


@pytest.mark.parametrize("geometry", ["cyl", "sph"])
def test_uniform_flow_in_curvilinear_coordinates(geometry):
    """A uniform Cartesian flow is force free: its curvilinear components are
    kept steady only if every geometric source term (centrifugal, v_theta^2/r,
    cot(theta) v_phi^2/r) and every transported momentum of Tab. "momenta" is
    right.  The error converges (first order: source/transport splitting) and
    stays well below the O(V^2 t / r) of a missing term."""
    errs = []
    for n in (16, 32):
        pr = W.uniform_flow(geometry, n=n, V=0.1)
        f, _ = oracle_run_to(O, pr, 0.2)
        keys = ("rho", "vx", "vy") + (("vz",) if geometry == "sph" else ())
        errs.append(max(np.abs(active(pr, f[k]) - active(pr, pr.fields[k])).max() for k in keys))
    # a missing term would leave an error of at least V^2 t / r_max = 1e-3
    assert errs[1] < 0.2 * 0.1 ** 2 * 0.2 / 2.0, errs
    assert errs[0] / errs[1] > 1.6, errs


def test_hydrostatic_balance_second_order_isotropic():
    """Isothermal atmosphere in a sinusoidal potential (v = 0): the pressure
    and potential gradients across each face balance to second order, in the
    same way along X, Y and Z."""
    out = {}
    for ax in "xyz":
        vmax = []
        for n in (32, 64):
            pr = W.hydrostatic(ax, n=n)
            f, _ = oracle_run_to(O, pr, 0.5)
            vmax.append(max(np.abs(f[k]).max() for k in ("vx", "vy", "vz") if f[k] is not None))
        out[ax] = vmax
        assert vmax[0] / vmax[1] > 3.5, (ax, vmax)
        assert vmax[1] < 1e-6
    assert abs(out["x"][1] - out["y"][1]) < 1e-15 and abs(out["y"][1] - out["z"][1]) < 1e-15


def test_consistent_transport_keeps_ratio():
    """Consistent transport (Sect. 3.4, end): interpolating Q/rho and using the
    mass flux keeps Q = c rho for a uniform c exactly (to round-off)."""
    rng = np.random.default_rng(31)
    faces = np.cumsum(np.r_[0.0, 0.05 + 0.1 * rng.random(40)])
    n = len(faces) - 5
    xc = 0.5 * (faces[:-1] + faces[1:])
    L = np.diff(faces)
    h = np.diff(xc)
    rho = 0.2 + rng.random(n + 4)
    Q = 3.7 * rho
    w = rng.normal(size=n + 1) * 0.3
    r = rho.copy()
    out = O.sweep_line(r, [Q], w, L, h, np.ones(n + 1), 1.0 / L[2:2 + n], 0.05)[0]
    assert np.allclose(out[2:2 + n], 3.7 * r[2:2 + n], rtol=1e-14, atol=0)
    assert not np.allclose(r, rho)


def test_reflecting_wall_equals_mirror_symmetric_domain():
    """REFLECT (box 2/9 reading): a wall behaves as the mirror plane of a
    symmetric periodic domain twice as large (density, tangential velocities
    even, normal velocity odd)."""
    rng = np.random.default_rng(41)
    nx, ny, nz = 10, 6, 5
    half = W.default_params(geometry="cart", nx=nx, ny=ny, nz=nz, xmin=0.0, xmax=1.0,
                            ymin=W.uniform_faces(0.0, 0.6, ny), zmin=W.uniform_faces(0.0, 0.5, nz),
                            eos="adi", bc=("periodic", "periodic", "reflect", "reflect"))
    full = dict(half, nz=2 * nz, zmin=W.uniform_faces(-0.5, 0.5, 2 * nz), bc=("periodic",) * 4)
    ph, pf = W._blank(half), W._blank(full)
    sh = (nz, ny + 2 * NG, nx)
    rho = 0.5 + rng.random(sh)
    e = 0.5 + rng.random(sh)
    vx, vy = 0.3 * rng.normal(size=sh), 0.3 * rng.normal(size=sh)
    vz = 0.3 * rng.normal(size=(nz + 1, ny + 2 * NG, nx))
    vz[0] = 0.0
    vz[-1] = 0.0
    # half domain: active k = NG..NG+nz-1, faces NG..NG+nz
    for name, a in (("rho", rho), ("e", e), ("vx", vx), ("vy", vy)):
        ph.fields[name][NG:NG + nz] = a
        # full domain: upper half = a, lower half = mirror
        pf.fields[name][NG + nz:NG + 2 * nz] = a
        pf.fields[name][NG:NG + nz] = a[::-1]
    ph.fields["vz"][NG:NG + nz + 1] = vz
    pf.fields["vz"][NG + nz:NG + 2 * nz + 1] = vz
    pf.fields["vz"][NG:NG + nz] = -vz[::-1][:-1]
    fh, ff = ph.copy_fields(), pf.copy_fields()
    dt = 0.3 * O.cfl_dt(half, ph.copy_fields())
    for _ in range(2):
        O.step(half, fh, dt)
        O.step(full, ff, dt)
    for name in ("rho", "e", "vx", "vy", "vz"):
        a = fh[name][NG:NG + nz]
        b = ff[name][NG + nz:NG + 2 * nz]
        assert np.allclose(a, b, rtol=1e-13, atol=1e-15), name


def test_outflow_passes_uniform_flow_unchanged():
    """OUTFLOW (zero-gradient) sides let a uniform flow through unchanged."""
    p = W.default_params(geometry="cart", nx=6, ny=10, nz=8, xmin=0.0, xmax=1.0,
                         ymin=W.uniform_faces(0.0, 1.0, 10), zmin=W.uniform_faces(0.0, 1.0, 8),
                         eos="adi", bc=("outflow",) * 4)
    pr = W._blank(p)
    pr.fields["vx"][:] = 0.25
    pr.fields["vy"][:] = 0.5
    pr.fields["vz"][:] = -0.375
    pr.fields["e"][:] = 1.5
    f = pr.copy_fields()
    for _ in range(3):
        O.step(p, f)
    for k in ("rho", "e", "vx", "vy", "vz"):
        assert np.array_equal(active(pr, f[k]), active(pr, pr.fields[k])), k


# ----------------------------------------------------------------------------
# Box 7d: kinematic viscosity (App. B, Eqs. 73 and 76; cylindrical 2D)
# ----------------------------------------------------------------------------

def _visc_patch(nx, ny, nu, L=1.0, R=1000.0, cs=1e-4, radial="reflect"):
    """A patch of a cylindrical mesh far from the axis (r in [R, R + L], azimuthal
    length L at r = R): the stress reduces to its Cartesian form up to terms of
    order L/R.  Uniform density at rest, no potential."""
    ymin = W.uniform_faces(R, R + L, ny)
    p = W.default_params(geometry="cyl", nx=nx, ny=ny, nz=1, xmin=0.0, xmax=L / R, ymin=ymin,
                         zmin=np.array([0.0, 1.0]), eos="iso", bc=(radial, radial, "reflect", "reflect"),
                         visc=True, cvnr=0.0)
    pr = W._blank(p)
    pr.fields["cs"][:] = cs
    pr.fields["nu"] = np.full(pr.shape, nu)
    return pr


@pytest.mark.parametrize("mode", ["vphi_phi", "vr_r", "vphi_r", "vr_phi"])
def test_viscous_damping_rates(mode):
    """Linear viscous damping of a velocity mode in the Cartesian limit:
    compressive modes decay at (4/3) nu k^2 (the -2/3 div v term of the
    diagonal components), shear modes at nu k^2 (the off-diagonal component),
    each from its own term of Eq. 73."""
    nu, L, R, n = 1e-3, 1.0, 1000.0, 64
    along_phi = mode.endswith("_phi")
    # a mode along phi is uniform in r: zero-gradient radial sides keep it so
    pr = _visc_patch(n if along_phi else 4, 4 if along_phi else n, nu, L, R,
                     radial="outflow" if mode == "vr_phi" else "reflect")
    p, f = pr.params, pr.fields
    A = 1e-6
    if along_phi:   # periodic in X: one wavelength over L
        k = 2.0 * math.pi / L
        x = (np.arange(n) + (0.0 if mode == "vphi_phi" else 0.5)) * (L / n)   # v_phi on X faces, v_r centred in X
        prof = A * np.sin(k * x)[None, None, :]
    else:           # walls in Y: v_r ~ sin (zero on the walls), v_phi ~ cos (zero gradient)
        k = math.pi / L
        faces = p["ymin"][:-1] - R
        centres = W.centres(p["ymin"]) - R
        y = faces if mode == "vr_r" else centres
        prof = A * (np.sin(k * y) if mode == "vr_r" else np.cos(k * y))[None, :, None]
    key = "vx" if mode.startswith("vphi") else "vy"
    f[key][:] = np.broadcast_to(prof, f[key].shape)
    if mode == "vr_r":   # wall faces at rest
        f["vy"][:, NG, :] = 0.0
        f["vy"][:, NG + p["ny"], :] = 0.0
    g, nsteps = oracle_run_to(O, pr, 10.0)
    rate = (4.0 / 3.0 if mode in ("vphi_phi", "vr_r") else 1.0) * nu * k * k
    act = (0, slice(NG + 1, NG + p["ny"] - 1) if mode == "vr_r" else slice(NG, NG + p["ny"]), slice(None))
    a0 = np.abs(np.broadcast_to(prof, f[key].shape)[act]).max()
    a1 = np.abs(g[key][act]).max()
    measured = -math.log(a1 / a0) / 10.0
    assert abs(measured / rate - 1.0) < 0.01, (mode, measured, rate, nsteps)


def test_viscous_cfl_closed_form():
    """Item 4 of Eq. cfl2 at rest: dt = C (dt1^-2 + dt4^-2)^(-1/2) with
    dt1 = Delta/c_s and dt4 = Delta^2 / (4 nu), Delta the smaller zone size."""
    nu, cs = 2e-3, 0.3
    pr = _visc_patch(8, 8, nu, cs=cs)
    p = pr.params
    g = pr.copy_fields()
    dt = O.cfl_dt(p, g)
    dy = (p["ymin"][NG + 1] - p["ymin"][NG])
    rmin = 0.5 * (p["ymin"][NG] + p["ymin"][NG + 1])
    dxl = rmin * (p["xmax"] - p["xmin"]) / p["nx"]
    d = min(dy, dxl)
    want = p["courant"] / math.sqrt((cs / d) ** 2 + (4.0 * nu / d ** 2) ** 2)
    assert abs(dt / want - 1.0) < 1e-12


def test_viscosity_leaves_solid_body_rotation():
    """A rigid rotation v_phi = c r has no shear and no divergence: box 7d
    changes nothing (to round-off), whatever the density field.  The radial
    ghosts carry the same rotation (FIXED sides)."""
    ymin = W.log_faces(0.5, 2.0, 24)
    p = W.default_params(geometry="cyl", nx=32, ny=24, nz=1, xmin=0.0, xmax=2 * math.pi, ymin=ymin,
                         zmin=np.array([0.0, 1.0]), eos="iso", bc=("fixed", "fixed", "reflect", "reflect"))
    pr = W._blank(p)
    rng = np.random.Generator(np.random.PCG64(77))
    f = pr.fields
    f["rho"][:] = 0.5 + rng.random(pr.shape)
    rc = W.centres(ymin)
    f["vx"][:] = 0.7 * rc[None, :, None]
    # no pressure; a potential that balances the centrifugal term of box 7a
    # face by face, so that 7d receives the rigid rotation unchanged
    f["cs"][:] = 0.0
    phi = np.zeros_like(rc)
    for j in range(1, len(rc)):
        vt = 0.35 * (rc[j] + rc[j - 1])
        phi[j] = phi[j - 1] + (rc[j] - rc[j - 1]) * vt * vt / ymin[j]
    f["pot"][:] = phi[None, :, None]
    f["nu"] = 1e-2 * (1.0 + rng.random(pr.shape))
    a = pr.copy_fields()
    b = pr.copy_fields()
    dt = 0.5 * O.cfl_dt(dict(p, visc=True), pr.copy_fields())
    O.step(dict(p, visc=True), a, dt)
    O.step(p, b, dt)
    vmax = np.abs(b["vx"]).max()
    for k in ("rho", "vx", "vy"):
        den = vmax if k.startswith("v") else np.abs(b[k]).max()
        assert np.abs(a[k] - b[k]).max() <= 1e-13 * den, k


def test_viscous_disk_conserves_angular_momentum():
    """Viscous torques are differences of edge fluxes (Eq. 76): with no
    viscosity next to the radial walls, the total angular momentum is conserved
    to round-off over a full step, as mass is."""
    pr = W.disk2d_cyl(nx=64, ny=24, noise=1e-2, omega=0.3)
    p = dict(pr.params, visc=True)
    f = pr.copy_fields()
    r = W.centres(p["ymin"])[None, :, None]
    nu = 1e-4 * np.sqrt(r) * np.ones(pr.shape)
    nu[:, :NG + 1, :] = 0.0
    nu[:, NG + p["ny"] - 1:, :] = 0.0
    f["nu"] = nu
    s0, a0 = O.sums(p, f)
    for _ in range(5):
        O.step(p, f)
    s1, a1 = O.sums(p, f)
    assert abs(s1[0] - s0[0]) < 1e-13 * a0[0]
    assert abs(s1[1] - s0[1]) < 1e-13 * a0[1]


def test_viscous_ring_spreads_as_lynden_bell_pringle():
    """Sect. 5.1, viscous spread of a gaseous ring: nu = 1e-5, 0.1 <= r <= 1.6,
    512 zones evenly spaced, zero-gradient radial boundaries; started from the
    similarity solution at t = 100 and compared with it at t = 200."""
    import lbp
    nu, ny, nx = 1e-5, 512, 4
    ymin = W.uniform_faces(0.1, 1.6, ny)
    p = W.default_params(geometry="cyl", nx=nx, ny=ny, nz=1, xmin=0.0, xmax=2 * math.pi, ymin=ymin,
                         zmin=np.array([0.0, 1.0]), eos="iso", bc=("outflow", "outflow", "reflect", "reflect"),
                         visc=True)
    pr = W._blank(p)
    f = pr.fields
    rc = W.centres(ymin)
    sig = lbp.sigma(rc, nu, 100.0)
    f["rho"][:] = np.maximum(sig, 1e-8 * sig.max())[None, :, None]
    f["vx"][:] = (rc ** -0.5)[None, :, None]
    f["vy"][:] = lbp.v_r(ymin[:-1], nu, 100.0)[None, :, None]
    f["cs"][:] = 1e-4
    f["pot"][:] = (-1.0 / rc)[None, :, None]
    f["nu"] = np.full(pr.shape, nu)
    g, nsteps = oracle_run_to(O, pr, 100.0)
    want = lbp.sigma(rc, nu, 200.0)[NG:NG + ny]
    got = g["rho"][0, NG:NG + ny, 0]
    err = np.abs(got - want).max() / want.max()
    # 1.5e-3 measured; dropping the -v_phi/r term or the r^2 weights gives 0.22 and 0.04
    assert err < 4e-3, err
