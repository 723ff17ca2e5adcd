"""Oracle of the learned flux correction (test infrastructure only).

A plain numpy definition of what the GPU path computes, used by the tests,
the smoke check and the benchmark's CPU leg; it shares no code with the GPU
library.  The method is not in the paper: a small convolutional net on the
coarse 2D (phi, r) state predicts corrections to the mass fluxes through each
zone's lower azimuthal (X) and radial (Y) face.  The corrections enter as a
conservative flux-divergence update of the density, so the mass change sums to
zero over the mesh (the paper's conservation argument, Sect. 3.4, carried over
to the added fluxes).  It is trained to bring one coarse step of the plain
solver (boxes 2-12 of Fig. 1 on the coarse mesh) to the fine solution averaged
4 x 4 conservatively onto the coarse zones.

Definition (all arrays cover active zones only, shape (ny, nx); j = 0 is the
innermost ring; i is periodic):

  features  f = (rho/rho_s - 1, v_y/u_s, v_x/u_s, (r_j - r_mid)/r_span), each
            formed in FP64, rounded to FP32, then to bfloat16;
  layers    z1 = conv(f, W1) + b1, h1 = bf16(relu(z1));
            z2 = conv(h1, W2) + b2, h2 = bf16(relu(z2));
            o  = conv(h2, W3) + b3;
            conv is a 3 x 3 cross-correlation, periodic in i, zero outside the
            active rows in j; operands are bfloat16 (weights rounded from
            their FP32 master values), sums exact here (FP32 on the GPU);
  fluxes    dFx = s_F o[..., 0] on the lower X face of each zone, dFy = s_F
            o[..., 1] on its lower Y face; the radial boundary faces carry no
            correction (dFy of row 0 and the face above the last row are 0);
  update    drho_ij = -(1/V_j) [dFx_{i+1,j} - dFx_ij + dFy_{i,j+1} - dFy_ij];
  loss      L = mean(((drho - t)/sigma)^2) for a target change t; for a
            batch of samples of one mesh, the mean over every zone of every
            sample (one Adam step per batch);
  guard     the corrected density is kept only if rho + drho > 0 and
            |drho| <= g rho in every zone; else the plain step stands.

Backward pass, Adam and the 4 x 4 restriction follow below, each with the
operations the GPU path takes.
"""
from __future__ import annotations

import numpy as np

CIN = 4    # input features
HID = 32   # hidden channels
COUT = 2   # flux corrections (X face, Y face)
LAYERS = ((CIN, HID), (HID, HID), (HID, COUT))


# ---------------------------------------------------------------------------
# bfloat16
# ---------------------------------------------------------------------------

def bf16(x) -> np.ndarray:
    """Round FP32 values to bfloat16, nearest even (values returned as FP64).
    FP64 input is first rounded to FP32, as the GPU path does."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = x.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# the net
# ---------------------------------------------------------------------------

def features(rho, vx, vy, rc, scales, rounded=True) -> np.ndarray:
    """(ny, nx, 4) input features of the active zones (see the module text)."""
    rho_s, u_s, r_mid, r_span = scales
    ny, nx = rho.shape
    f = np.empty((ny, nx, CIN))
    f[..., 0] = rho / rho_s - 1.0
    f[..., 1] = vy / u_s
    f[..., 2] = vx / u_s
    f[..., 3] = ((rc - r_mid) / r_span)[:, None]
    return bf16(f) if rounded else f


def conv(x, w, b) -> np.ndarray:
    """3 x 3 cross-correlation: x (ny, nx, ci), w (co, 3, 3, ci), b (co,)
    -> (ny, nx, co); periodic in i, zero outside the rows in j."""
    ny, nx, _ = x.shape
    co = w.shape[0]
    xp = np.zeros((ny + 2,) + x.shape[1:])
    xp[1:-1] = x
    out = np.broadcast_to(np.asarray(b, dtype=np.float64), (ny, nx, co)).copy()
    for ty in range(3):
        rows = xp[ty:ty + ny]
        for tx in range(3):
            sh = np.roll(rows, -(tx - 1), axis=1)  # sh[:, i] = x[:, i + tx - 1]
            out += sh @ w[:, ty, tx, :].T
    return out


def conv_t(g, w) -> np.ndarray:
    """Adjoint of `conv` in its input: g (ny, nx, co) -> (ny, nx, ci)."""
    ny, nx, _ = g.shape
    ci = w.shape[3]
    out = np.zeros((ny, nx, ci))
    gp = np.zeros((ny + 2,) + g.shape[1:])
    gp[1:-1] = g
    for ty in range(3):
        # output row y took input row y + ty - 1: input row y gets output row y - ty + 1
        rows = gp[2 - ty:2 - ty + ny]
        for tx in range(3):
            sh = np.roll(rows, tx - 1, axis=1)  # sh[:, i] = g[:, i - tx + 1]
            out += sh @ w[:, ty, tx, :]
    return out


def conv_w(g, x) -> np.ndarray:
    """Gradient of sum(g * conv(x, w)) in w: (co, 3, 3, ci)."""
    ny, nx, ci = x.shape
    co = g.shape[2]
    xp = np.zeros((ny + 2, nx, ci))
    xp[1:-1] = x
    dw = np.zeros((co, 3, 3, ci))
    G = g.reshape(-1, co)
    for ty in range(3):
        rows = xp[ty:ty + ny]
        for tx in range(3):
            sh = np.roll(rows, -(tx - 1), axis=1).reshape(-1, ci)
            dw[:, ty, tx, :] = G.T @ sh
    return dw


def init_params(rng: np.random.Generator):
    """FP32 master weights (He-scaled normal draws) and zero biases."""
    P = {}
    for n, (ci, co) in enumerate(LAYERS, 1):
        std = np.sqrt(2.0 / (9 * ci)) * (0.1 if n == len(LAYERS) else 1.0)
        P["W%d" % n] = (rng.standard_normal((co, 3, 3, ci)) * std).astype(np.float32)
        P["b%d" % n] = np.zeros(co, dtype=np.float32)
    return P


def forward(f, P, rounded=True):
    """Activations of the net on features f (BF16-representable)."""
    q = bf16 if rounded else (lambda a: np.asarray(a, dtype=np.float64))
    z1 = conv(f, q(P["W1"]), P["b1"])
    h1 = q(np.maximum(np.float32(z1) if rounded else z1, 0.0))
    z2 = conv(h1, q(P["W2"]), P["b2"])
    h2 = q(np.maximum(np.float32(z2) if rounded else z2, 0.0))
    o = conv(h2, q(P["W3"]), P["b3"])
    return {"f": f, "h1": h1, "h2": h2, "o": o}


# ---------------------------------------------------------------------------
# what an FP32-accumulating implementation may return
# ---------------------------------------------------------------------------

U32 = 2.0 ** -24  # unit roundoff of FP32


def sum_bound(depth: int, abs_sum) -> np.ndarray:
    """Bound on the error of a sum of bfloat16 products (exact in FP32) taken
    in FP32 with at most `depth` additions along any path to the result, at
    up to two units of roundoff each (allowing a matrix unit's accumulation
    to round less tightly than IEEE addition): 2 depth u sum|terms|."""
    return 2.0 * depth * U32 * np.asarray(abs_sum, dtype=np.float64)


def interval(z, delta, relu=False, mask=None):
    """The values a stored bfloat16 result q(x) = bf16(fp32(x)) (after a ReLU,
    or masked to zero where mask is False) can take when x lies within delta
    of the exact z: q is monotone, so [q(z - delta), q(z + delta)], with
    q(z) the oracle's own value."""
    def q(x):
        x = np.float32(x)
        return bf16(np.maximum(x, np.float32(0.0)) if relu else x)
    lo, mid, hi = q(z - delta), q(z), q(z + delta)
    if mask is not None:
        lo, mid, hi = (np.where(mask, a, 0.0) for a in (lo, mid, hi))
    return lo, mid, hi


# ---------------------------------------------------------------------------
# fluxes, update, loss
# ---------------------------------------------------------------------------

def fluxes(o, sF):
    dFx = sF * o[..., 0]
    dFy = sF * o[..., 1]
    dFy[0, :] = 0.0  # inner boundary face
    return dFx, dFy


def divergence(dFx, dFy):
    """dFx_{i+1} - dFx_i + dFy_{j+1} - dFy_j, with no flux through the outer
    boundary face."""
    up = np.zeros_like(dFy)
    up[:-1] = dFy[1:]
    return (np.roll(dFx, -1, axis=1) - dFx) + (up - dFy)


def drho(o, sF, invV):
    dFx, dFy = fluxes(o, sF)
    return -invV[:, None] * divergence(dFx, dFy)


def loss(d, t, sigma) -> float:
    return float(np.mean(((d - t) / sigma) ** 2))


def loss_batch(ds, ts, sigma) -> float:
    """The loss of a batch: the mean over every zone of every sample."""
    return float(sum(np.sum(((d - t) / sigma) ** 2) for d, t in zip(ds, ts)) / sum(d.size for d in ds))


def backward(A, P, t, sF, invV, sigma, rounded=True, count=None):
    """Gradients of the loss in every parameter, from the activations A of
    `forward`.  The layer gradients are rounded to bfloat16 before they enter
    a product, as on the GPU; each bias gradient is the sum of its rounded
    layer gradient.  `count` is the number of zones the loss averages over
    (this sample's, by default; all samples' of a batch)."""
    q = bf16 if rounded else (lambda a: np.asarray(a, dtype=np.float64))
    d = drho(A["o"], sF, invV)
    N = d.size if count is None else count
    g = 2.0 * (d - t) / (N * sigma * sigma)          # dL/d(drho)
    gD = -invV[:, None] * g                           # dL/d(divergence)
    gFx = np.roll(gD, 1, axis=1) - gD                 # Fx_i enters D_{i-1} (+) and D_i (-)
    gFy = np.zeros_like(gD)
    gFy[1:] = gD[:-1] - gD[1:]                        # row 0 face is fixed
    g3 = np.stack([sF * gFx, sF * gFy], axis=-1)
    g3 = q(np.float32(g3) if rounded else g3)
    G = {"W3": conv_w(g3, A["h2"]), "b3": g3.sum(axis=(0, 1))}
    dh2 = conv_t(g3, q(P["W3"]))
    g2 = q(np.where(A["h2"] > 0, np.float32(dh2) if rounded else dh2, 0.0))
    G["W2"] = conv_w(g2, A["h1"])
    G["b2"] = g2.sum(axis=(0, 1))
    dh1 = conv_t(g2, q(P["W2"]))
    g1 = q(np.where(A["h1"] > 0, np.float32(dh1) if rounded else dh1, 0.0))
    G["W1"] = conv_w(g1, A["f"])
    G["b1"] = g1.sum(axis=(0, 1))
    return G


def backward_batch(As, P, ts, sF, invV, sigma, rounded=True):
    """Gradients of the batch loss: each sample's gradient with the loss
    averaged over all zones of the batch, summed over the samples."""
    count = sum(A["o"].shape[0] * A["o"].shape[1] for A in As)
    G = None
    for A, t in zip(As, ts):
        g = backward(A, P, t, sF, invV, sigma, rounded=rounded, count=count)
        G = g if G is None else {k: G[k] + g[k] for k in G}
    return G


# ---------------------------------------------------------------------------
# Adam (Kingma & Ba 2015) on the FP32 master parameters
# ---------------------------------------------------------------------------

def adam(P, G, M, V, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update with bias correction; `step` counts from 1.  Returns
    new (P, M, V) as FP64 arrays."""
    Pn, Mn, Vn = {}, {}, {}
    c1 = 1.0 - beta1 ** step
    c2 = 1.0 - beta2 ** step
    for k in P:
        g = np.asarray(G[k], dtype=np.float64)
        Mn[k] = beta1 * M[k] + (1.0 - beta1) * g
        Vn[k] = beta2 * V[k] + (1.0 - beta2) * g * g
        Pn[k] = P[k] - lr * (Mn[k] / c1) / (np.sqrt(Vn[k] / c2) + eps)
    return Pn, Mn, Vn


# ---------------------------------------------------------------------------
# guard
# ---------------------------------------------------------------------------

def apply(rho, d, guard):
    """(new rho, skipped): the corrected density, or rho unchanged if the
    correction would make a zone non-positive or change it by more than
    guard * rho."""
    new = rho + d
    if np.all(new > 0.0) and np.all(np.abs(d) <= guard * rho):
        return new, False
    return rho.copy(), True


# ---------------------------------------------------------------------------
# 4 x 4 conservative restriction, fine -> coarse (2D cylindrical)
# ---------------------------------------------------------------------------

def restrict(rho_f, vx_f, vy_f, yf_fine, ratio=4):
    """Coarse active fields from fine active fields.

    rho: mass over the coarse zone divided by its volume (zone volumes are
    (r_+^2 - r_-^2)/2 dphi, the fine zones partition the coarse one);
    v_x on a coarse X face: mean of the `ratio` fine X faces on it weighted
    by their areas (radial widths dr);
    v_y on a coarse Y face: mean of the `ratio` fine Y faces on it (equal
    arc lengths)."""
    nyf, nxf = rho_f.shape
    R = ratio
    ny, nx = nyf // R, nxf // R
    a = yf_fine[:-1]
    b = yf_fine[1:]
    w = 0.5 * (b * b - a * a)                        # fine ring volume / dphi
    mass = (rho_f * w[:, None]).reshape(ny, R, nx, R).sum(axis=(1, 3))
    W = w.reshape(ny, R).sum(axis=1) * R
    rho_c = mass / W[:, None]
    dr = (b - a).reshape(ny, R)
    vxr = vx_f[:, ::R].reshape(ny, R, nx)
    vx_c = (vxr * dr[:, :, None]).sum(axis=1) / dr.sum(axis=1)[:, None]
    vy_c = vy_f[::R, :].reshape(ny, nx, R).mean(axis=2)
    return rho_c, vx_c, vy_c
