"""Seeded synthetic inputs for the hydrodynamics step (shared test fixture).

This module builds meshes and initial conditions only: face coordinates,
equilibrium disk profiles, seeded density noise, static potentials and
sound speeds.  It holds none of the numerical method's arithmetic (no
geometric coefficients, no fluxes, no time step), so that both the CPU
oracle and the GPU library can be fed the same arrays without sharing
any code of the method.

Conventions (paper, Sect. 2.2-2.3 and Tab. "corresp"):
  * X = azimuth (periodic, uniform), Y = radius, Z = z (cylindrical) or
    colatitude (spherical).  Cartesian meshes use x, y, z directly.
  * Arrays are float64, C-contiguous, shape (nz_g, ny_g, nx) with
    ny_g = ny + 6 and nz_g = nz + 6 in 3D (nz_g = 1 in 2D): three ghost
    layers in Y and Z, none in X (paper, Sect. 4.1).
  * vx[k, j, i] lives on the lower X face of cell i, vy[k, j, i] on the face
    at ymin[j], vz[k, j, i] on the face at zmin[k]; scalars are cell centred
    (paper, Sect. 2.3, Fig. "cell").
  * Units G = M_star = 1 (potential -1/r in the paper's disk tests).

Inputs stand in for the paper's disk setups; the paper uses no public
benchmark or dataset for this path.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional

import numpy as np

NGH = 3

GEOMETRIES = ("cart", "cyl", "sph")
BC_KINDS = ("periodic", "reflect", "outflow", "fixed")


@dataclasses.dataclass
class Problem:
    """A mesh, its run parameters and the initial state (host arrays)."""

    name: str
    params: Dict
    fields: Dict[str, Optional[np.ndarray]]
    steps: int = 1

    @property
    def shape(self):
        p = self.params
        nzg = p["nz"] + 2 * NGH if p["nz"] > 1 else 1
        return (nzg, p["ny"] + 2 * NGH, p["nx"])

    @property
    def active_cells(self) -> int:
        p = self.params
        return p["nx"] * p["ny"] * p["nz"]

    def copy_fields(self) -> Dict[str, Optional[np.ndarray]]:
        return {k: (None if v is None else v.copy()) for k, v in self.fields.items()}


def default_params(**kw) -> Dict:
    """Run parameters with the paper's defaults (Courant number 0.44, Sect. 3.5)."""
    p = dict(
        geometry="cart", nx=1, ny=3, nz=1, xmin=0.0, xmax=1.0,
        ymin=None, zmin=None,
        eos="iso", gamma=1.4,
        omega=0.0, courant=0.44, cvnr=math.sqrt(2.0), shear_c0=0.44,
        fargo=False, v0_mode="minmax",
        bc=("reflect", "reflect", "reflect", "reflect"),
    )
    p.update(kw)
    return p


# ----------------------------------------------------------------------------
# face coordinates
# ----------------------------------------------------------------------------

def uniform_faces(lo: float, hi: float, n: int, ghosts: bool = True) -> np.ndarray:
    """n cells on [lo, hi] plus NGH ghost cells on each side (n + 2*NGH + 1 faces)."""
    d = (hi - lo) / n
    if not ghosts:
        return np.array([lo, hi], dtype=np.float64)
    idx = np.arange(-NGH, n + NGH + 1, dtype=np.float64)
    f = lo + idx * d
    f[NGH] = lo
    f[NGH + n] = hi
    return f


def log_faces(lo: float, hi: float, n: int) -> np.ndarray:
    """Logarithmic radial faces ymin[j] = lo*(hi/lo)**((j-NGH)/n), ghosts continued."""
    idx = np.arange(-NGH, n + NGH + 1, dtype=np.float64)
    f = lo * (hi / lo) ** (idx / n)
    f[NGH] = lo
    f[NGH + n] = hi
    return f


def centres(faces: np.ndarray) -> np.ndarray:
    return 0.5 * (faces[:-1] + faces[1:])


def _grid(p):
    """Broadcastable coordinate arrays (zc, yc, x_face, x_centre) of shape (nzg,nyg,nx)."""
    nx = p["nx"]
    dx = (p["xmax"] - p["xmin"]) / nx
    xf = p["xmin"] + dx * np.arange(nx, dtype=np.float64)
    xc = xf + 0.5 * dx
    yc = centres(p["ymin"])[None, :, None]
    zc = centres(p["zmin"])[:, None, None]
    return zc, yc, xf[None, None, :], xc[None, None, :]


def _full(shape, a) -> np.ndarray:
    """A new writable C-contiguous float64 array of `shape` holding `a` broadcast."""
    return np.array(np.broadcast_to(a, shape), dtype=np.float64, order="C", copy=True)


def _noise(rng: np.random.Generator, rho: np.ndarray, p: Dict, amp: float):
    """rho <- rho*(1 + amp*(2U-1)) on active cells, drawn in (k, j, i) order."""
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    u = rng.random((nz, ny, nx))
    k0 = NGH if nz > 1 else 0
    sl = (slice(k0, k0 + nz), slice(NGH, NGH + ny), slice(0, nx))
    rho[sl] *= 1.0 + amp * (2.0 * u - 1.0)


# ----------------------------------------------------------------------------
# disk configurations
# ----------------------------------------------------------------------------

def disk2d_cyl(nx=384, ny=128, rin=0.4, rout=2.5, h=0.05, seed=1, noise=1e-3,
               fargo=True, steps=10, omega=0.0, sigma_slope=-0.5, bump=None) -> Problem:
    """2D (phi, r) locally isothermal Keplerian disk, log-spaced radius.

    Sigma = r**sigma_slope, c_s = h r**-0.5, Phi = -1/r, and the azimuthal
    velocity balancing gravity and pressure: v_phi**2 = (1 + (s - 1) h**2)/r
    for Sigma ~ r**s (s = -1/2 gives (1 - 1.5 h**2)/r).  Radial sides keep the
    unperturbed profile in their ghosts (caller-fixed).  `bump` = (amp, r0,
    phi0, width) multiplies the active density by 1 + amp*exp(-d**2/width**2),
    d the distance to (r0, phi0), a smooth non-axisymmetric perturbation.
    """
    p = default_params(
        geometry="cyl", nx=nx, ny=ny, nz=1, xmin=0.0, xmax=2.0 * math.pi,
        ymin=log_faces(rin, rout, ny), zmin=np.array([0.0, 1.0]),
        eos="iso", omega=omega, fargo=fargo,
        bc=("fixed", "fixed", "fixed", "fixed"),
    )
    shape = (1, ny + 2 * NGH, nx)
    zc, r, xf, xc = _grid(p)
    s = sigma_slope
    rho = _full(shape, r ** s)
    cs = _full(shape, h * r ** -0.5)
    pot = _full(shape, -1.0 / r)
    vphi = np.sqrt((1.0 + (s - 1.0) * h * h) / r) - omega * r
    vx = _full(shape, vphi)
    vy = np.zeros(shape)
    if bump is not None:
        amp, r0, phi0, width = bump
        d2 = r * r + r0 * r0 - 2.0 * r * r0 * np.cos(xc - phi0)
        g = 1.0 + amp * np.exp(-d2 / (width * width))
        act = (slice(None), slice(NGH, NGH + ny), slice(None))
        rho[act] = (rho * g)[act]
    rng = np.random.Generator(np.random.PCG64(seed))
    if noise:
        _noise(rng, rho, p, noise)
    return Problem("disk2d_cyl", p, dict(rho=rho, vx=vx, vy=vy, vz=None, e=None, cs=cs, pot=pot), steps)


def disk2d_visc(nx=192, ny=64, rin=0.4, rout=2.5, h=0.05, alpha=1e-3, seed=3, noise=1e-3,
                fargo=True, steps=10) -> Problem:
    """The 2D disk of `disk2d_cyl` with an alpha viscosity: the static field
    nu = alpha c_s H = alpha h**2 r**0.5 (c_s = h r**-0.5, H = h r), box 7d on."""
    pr = disk2d_cyl(nx=nx, ny=ny, rin=rin, rout=rout, h=h, seed=seed, noise=noise, fargo=fargo, steps=steps)
    pr.params["visc"] = True
    zc, r, xf, xc = _grid(pr.params)
    pr.fields["nu"] = _full(pr.shape, alpha * h * h * np.sqrt(r))
    pr.name = "disk2d_visc"
    return pr


def disk_batch(count=256, seed=3, nr_range=(64, 512), h_range=(0.03, 0.10), alpha_exp=(-4.0, -2.0),
               rin=0.4, rout=2.5, noise=1e-3):
    """The parameter sweep of uneven viscous disks: N_r uniform on nr_range,
    N_phi = 3 N_r, aspect ratio h uniform on h_range, alpha = 10**U(alpha_exp),
    each an isothermal `disk2d_visc` with its own noise seed (3000 + d)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for d in range(count):
        nr = int(rng.integers(nr_range[0], nr_range[1] + 1))
        h = float(rng.uniform(*h_range))
        alpha = float(10.0 ** rng.uniform(*alpha_exp))
        pr = disk2d_visc(nx=3 * nr, ny=nr, rin=rin, rout=rout, h=h, alpha=alpha, seed=3000 + d, noise=noise)
        pr.name = "disk%03d" % d
        out.append(pr)
    return out


def disk3d_sph(nx=1536, ny=512, nz=128, rin=0.4, rout=2.5, h=0.05, nh=3.0, gamma=1.4,
               seed=2, noise=1e-3, fargo=True, steps=1) -> Problem:
    """3D (phi, r, theta) adiabatic disk in hydrostatic and rotational equilibrium.

    With R = r sin(theta) and c_iso**2 = h**2/R (so P = c_iso**2 rho),
    rho = R**-1.5 exp((sin(theta) - 1)/h**2)/(sqrt(2 pi) h) and
    v_phi = sqrt((sin(theta) - 2.5 h**2)/R) balance the radial and polar
    equations of motion with Phi = -1/r; e = P/(gamma - 1).  Colatitude spans
    pi/2 +- nh*h.  Radial sides caller-fixed, polar sides reflecting.
    """
    th0 = 0.5 * math.pi - nh * h
    th1 = 0.5 * math.pi + nh * h
    p = default_params(
        geometry="sph", nx=nx, ny=ny, nz=nz, xmin=0.0, xmax=2.0 * math.pi,
        ymin=log_faces(rin, rout, ny), zmin=uniform_faces(th0, th1, nz),
        eos="adi", gamma=gamma, omega=0.0, fargo=fargo,
        bc=("fixed", "fixed", "reflect", "reflect"),
    )
    shape = (nz + 2 * NGH, ny + 2 * NGH, nx)
    th, r, xf, xc = _grid(p)
    st = np.sin(th)
    R = r * st
    rho2 = R ** -1.5 * np.exp((st - 1.0) / (h * h)) / (math.sqrt(2.0 * math.pi) * h)
    rho = _full(shape, rho2)
    rng = np.random.Generator(np.random.PCG64(seed))
    _noise(rng, rho, p, noise)
    ciso2 = _full(shape, h * h / R)
    e = ciso2 * rho / (gamma - 1.0)
    vx = _full(shape, np.sqrt((st - 2.5 * h * h) / R))
    vy = np.zeros(shape)
    vz = np.zeros(shape)
    pot = _full(shape, -1.0 / r)
    return Problem("disk3d_sph", p, dict(rho=rho, vx=vx, vy=vy, vz=vz, e=e, cs=None, pot=pot), steps)


def planet_potential(r, z, phi, q, rp=1.0, phip=0.0, eps=0.03):
    """Star + fixed planet on a circular orbit in the plane z = 0, with the
    indirect term of the star's reflex acceleration: -1/|x| - q/sqrt(d^2+eps^2)
    + q r cos(phi - phip)/rp^2."""
    d2 = r * r + rp * rp - 2.0 * r * rp * np.cos(phi - phip) + z * z
    return (-1.0 / np.sqrt(r * r + z * z) - q / np.sqrt(d2 + eps * eps)
            + q * r * np.cos(phi - phip) / (rp * rp))


def disk3d_cyl_planet(nx=2048, ny=768, nz=96, rin=0.4, rout=2.5, h=0.05, zmax=0.15,
                      q=1e-3, eps_h=0.6, omega=1.0, seed=5, noise=1e-3, fargo=True,
                      steps=100) -> Problem:
    """3D (phi, r, z) locally isothermal disk with a fixed planet (q at r = 1).

    c_s**2 = h**2/r, Sigma = r**-0.5, vertical hydrostatic density
    rho = Sigma/(sqrt(2 pi) h r) exp((1/c_s**2)(1/sqrt(r**2+z**2) - 1/r)) and
    v_phi**2 = (r/sqrt(r**2+z**2) - 2.5 h**2)/r in the inertial frame; the mesh
    co-rotates at omega.  The initial state ignores the planet.  Radial sides
    caller-fixed, vertical sides reflecting.
    """
    p = default_params(
        geometry="cyl", nx=nx, ny=ny, nz=nz, xmin=0.0, xmax=2.0 * math.pi,
        ymin=log_faces(rin, rout, ny), zmin=uniform_faces(-zmax, zmax, nz),
        eos="iso", omega=omega, fargo=fargo,
        bc=("fixed", "fixed", "reflect", "reflect"),
    )
    shape = (nz + 2 * NGH, ny + 2 * NGH, nx)
    z, r, xf, xc = _grid(p)
    c2 = h * h / r
    sph_r = np.sqrt(r * r + z * z)
    rho2 = r ** -0.5 / (math.sqrt(2.0 * math.pi) * h * r) * np.exp((1.0 / c2) * (1.0 / sph_r - 1.0 / r))
    rho = _full(shape, rho2)
    rng = np.random.Generator(np.random.PCG64(seed))
    _noise(rng, rho, p, noise)
    cs = _full(shape, np.sqrt(c2))
    vphi = np.sqrt((r / sph_r - 2.5 * h * h) / r) - omega * r
    vx = _full(shape, vphi)
    vy = np.zeros(shape)
    vz = np.zeros(shape)
    pot = _full(shape, planet_potential(r, z, xc, q, eps=eps_h * h))
    return Problem("disk3d_cyl_planet", p, dict(rho=rho, vx=vx, vy=vy, vz=vz, e=None, cs=cs, pot=pot), steps)


def disk2d_planet(nx=768, ny=256, rin=0.4, rout=2.5, h=0.05, q=1e-3, eps_h=0.6, omega=1.0, seed=4000,
                  noise=1e-3, fargo=True, steps=10) -> Problem:
    """2D (phi, r) locally isothermal disk with a fixed planet (q at r = 1) in
    the frame co-rotating with it: Sigma = r**-0.5, c_s = h r**-0.5, the
    planet potential of the 3D planet disk at z = 0 (softening eps_h h), and
    v_phi**2 = (1 - 1.5 h**2)/r in the inertial frame.  Radial faces are
    log-spaced, so the faces of an (nx, ny) mesh are every 4th face of the
    (4 nx, 4 ny) mesh: the coarse and fine meshes of the learned flux
    correction.  The initial state ignores the planet."""
    p = default_params(
        geometry="cyl", nx=nx, ny=ny, nz=1, xmin=0.0, xmax=2.0 * math.pi,
        ymin=log_faces(rin, rout, ny), zmin=np.array([0.0, 1.0]),
        eos="iso", omega=omega, fargo=fargo,
        bc=("fixed", "fixed", "fixed", "fixed"),
    )
    shape = (1, ny + 2 * NGH, nx)
    zc, r, xf, xc = _grid(p)
    rho = _full(shape, r ** -0.5)
    cs = _full(shape, h * r ** -0.5)
    pot = _full(shape, planet_potential(r, 0.0, xc, q, eps=eps_h * h))
    vx = _full(shape, np.sqrt((1.0 - 1.5 * h * h) / r) - omega * r)
    vy = np.zeros(shape)
    rng = np.random.Generator(np.random.PCG64(seed))
    if noise:
        _noise(rng, rho, p, noise)
    return Problem("disk2d_planet", p, dict(rho=rho, vx=vx, vy=vy, vz=None, e=None, cs=cs, pot=pot), steps)


# ----------------------------------------------------------------------------
# small Cartesian test problems
# ----------------------------------------------------------------------------

def sod(axis="y", n=300, length=10.0, gamma=1.4, courant=0.44) -> Problem:
    """Sod shock tube (paper, Sect. 5.1.1): rho=P=1 left of the midpoint,
    rho=0.125, P=0.1 right of it, v=0, gamma=1.4, reflecting ends.

    axis='y' builds a 2D mesh (nx=1, ny=n); axis='z' a 3D mesh (nx=1, ny=3
    periodic in Y, nz=n)."""
    if axis == "y":
        p = default_params(geometry="cart", nx=1, ny=n, nz=1, xmin=0.0, xmax=1.0,
                           ymin=uniform_faces(0.0, length, n), zmin=np.array([0.0, 1.0]),
                           eos="adi", gamma=gamma, courant=courant,
                           bc=("reflect", "reflect", "reflect", "reflect"))
    elif axis == "z":
        p = default_params(geometry="cart", nx=1, ny=3, nz=n, xmin=0.0, xmax=1.0,
                           ymin=uniform_faces(0.0, 3.0, 3), zmin=uniform_faces(0.0, length, n),
                           eos="adi", gamma=gamma, courant=courant,
                           bc=("periodic", "periodic", "reflect", "reflect"))
    else:
        raise ValueError(axis)
    prob = _blank(p)
    zc, yc, xf, xc = _grid(p)
    s = yc if axis == "y" else zc
    left = s < 0.5 * length
    shape = prob.shape
    rho = _full(shape, np.where(left, 1.0, 0.125))
    P = _full(shape, np.where(left, 1.0, 0.1))
    prob.fields.update(rho=rho, e=P / (gamma - 1.0))
    prob.name = "sod_" + axis
    return prob


def _blank(p: Dict) -> Problem:
    nzg = p["nz"] + 2 * NGH if p["nz"] > 1 else 1
    shape = (nzg, p["ny"] + 2 * NGH, p["nx"])
    f = dict(rho=np.ones(shape), vx=np.zeros(shape), vy=np.zeros(shape),
             vz=np.zeros(shape) if p["nz"] > 1 else None,
             e=np.ones(shape) if p["eos"] == "adi" else None,
             cs=np.ones(shape) if p["eos"] == "iso" else None,
             pot=np.zeros(shape))
    return Problem("blank", p, f, 1)


def sound_wave(axis="y", n=64, amp=1e-6, cs=1.0, length=1.0) -> Problem:
    """Linear isothermal sound wave travelling towards +axis on a periodic
    Cartesian mesh: rho = 1 + amp sin(kx), v = amp cs sin(kx) (at faces)."""
    kwave = 2.0 * math.pi / length
    if axis == "x":
        p = default_params(geometry="cart", nx=n, ny=3, nz=1, xmin=0.0, xmax=length,
                           ymin=uniform_faces(0.0, 3.0, 3), zmin=np.array([0.0, 1.0]),
                           eos="iso", bc=("periodic",) * 4)
    elif axis == "y":
        p = default_params(geometry="cart", nx=1, ny=n, nz=1, xmin=0.0, xmax=1.0,
                           ymin=uniform_faces(0.0, length, n), zmin=np.array([0.0, 1.0]),
                           eos="iso", bc=("periodic",) * 4)
    else:
        p = default_params(geometry="cart", nx=1, ny=3, nz=n, xmin=0.0, xmax=1.0,
                           ymin=uniform_faces(0.0, 3.0, 3), zmin=uniform_faces(0.0, length, n),
                           eos="iso", bc=("periodic",) * 4)
    prob = _blank(p)
    shape = prob.shape
    zc, yc, xf, xc = _grid(p)
    if axis == "x":
        sc, sf = xc, xf
    elif axis == "y":
        sc, sf = yc, p["ymin"][:-1][None, :, None]
    else:
        sc, sf = zc, p["zmin"][:-1][:, None, None]
    prob.fields["rho"] = _full(shape, 1.0 + amp * np.sin(kwave * sc))
    prob.fields["cs"] = _full(shape, cs)
    v = _full(shape, amp * cs * np.sin(kwave * sf))
    prob.fields["v" + axis] = v
    prob.name = "sound_" + axis
    return prob


def random_problem(geometry="cart", nx=40, ny=9, nz=7, eos="adi", seed=0,
                   bc=("reflect", "reflect", "reflect", "reflect"), fargo=False,
                   omega=0.0, vamp=0.3) -> Problem:
    """Strongly perturbed random state on a small mesh: exercises every branch
    (upwind sign, slope limiting, artificial viscosity, PPA extremum fixes)."""
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    if geometry == "cart":
        ymin = uniform_faces(0.0, 1.0, ny)
        zmin = uniform_faces(0.0, 1.0, nz) if nz > 1 else np.array([0.0, 1.0])
        xmax = 1.0
    elif geometry == "cyl":
        ymin = log_faces(0.5, 1.5, ny)
        zmin = uniform_faces(-0.2, 0.2, nz) if nz > 1 else np.array([0.0, 1.0])
        xmax = 2.0 * math.pi
    else:
        ymin = log_faces(0.5, 1.5, ny)
        zmin = uniform_faces(0.5 * math.pi - 0.3, 0.5 * math.pi + 0.3, nz)
        xmax = 2.0 * math.pi
    p = default_params(geometry=geometry, nx=nx, ny=ny, nz=nz, xmin=0.0, xmax=xmax,
                       ymin=ymin, zmin=zmin, eos=eos, fargo=fargo, omega=omega, bc=tuple(bc))
    prob = _blank(p)
    shape = prob.shape
    f = prob.fields
    f["rho"] = 0.5 + rng.random(shape)
    zc, yc, xf, xc = _grid(p)
    if geometry == "cart":
        base = np.zeros((1, 1, 1))
    else:
        base = _full(shape, (1.0 / np.sqrt(yc)) - omega * yc)
    f["vx"] = base + vamp * (2.0 * rng.random(shape) - 1.0)
    f["vy"] = vamp * (2.0 * rng.random(shape) - 1.0)
    if nz > 1:
        f["vz"] = vamp * (2.0 * rng.random(shape) - 1.0)
    if eos == "adi":
        f["e"] = 0.5 + rng.random(shape)
    else:
        f["cs"] = 0.3 + 0.2 * rng.random(shape)
    f["pot"] = 0.1 * (2.0 * rng.random(shape) - 1.0)
    if geometry != "cart":
        f["pot"] = f["pot"] - 1.0 / _full(shape, yc)
    prob.name = "random_%s_%s" % (geometry, eos)
    return prob



def uniform_flow(geometry="cyl", n=16, V=0.1, cs=1.0, fargo=False) -> Problem:
    """A uniform Cartesian flow V e_x written in curvilinear components (an
    exact steady solution of the Euler equations without forces), on a
    sector with caller-fixed ghosts holding the exact solution.

    cylindrical (2D): v_r = V cos(phi), v_phi = -V sin(phi) on r in [1, 2];
    spherical (3D):   v_r = V sin(th) cos(phi), v_th = V cos(th) cos(phi),
                      v_phi = -V sin(phi) on r in [1, 2], th in pi/2 +- 0.4.
    Each component is evaluated at the centre of its own face."""
    if geometry == "cyl":
        p = default_params(geometry="cyl", nx=4 * n, ny=n, nz=1, xmin=0.0, xmax=2 * math.pi,
                           ymin=uniform_faces(1.0, 2.0, n), zmin=np.array([0.0, 1.0]),
                           eos="iso", fargo=fargo, bc=("fixed",) * 4)
    else:
        p = default_params(geometry="sph", nx=4 * n, ny=n, nz=n, xmin=0.0, xmax=2 * math.pi,
                           ymin=uniform_faces(1.0, 2.0, n),
                           zmin=uniform_faces(0.5 * math.pi - 0.4, 0.5 * math.pi + 0.4, n),
                           eos="iso", fargo=fargo, bc=("fixed",) * 4)
    pr = _blank(p)
    shape = pr.shape
    zc, yc, xf, xc = _grid(p)
    yf = p["ymin"][:-1][None, :, None]
    pr.fields["cs"][:] = cs
    if geometry == "cyl":
        pr.fields["vy"] = _full(shape, V * np.cos(xc) + 0.0 * yf)
        pr.fields["vx"] = _full(shape, -V * np.sin(xf) + 0.0 * yc)
    else:
        zf = p["zmin"][:-1][:, None, None]
        pr.fields["vy"] = _full(shape, V * np.sin(zc) * np.cos(xc) + 0.0 * yf)
        pr.fields["vz"] = _full(shape, V * np.cos(zf) * np.cos(xc) + 0.0 * yc)
        pr.fields["vx"] = _full(shape, -V * np.sin(xf) + 0.0 * yc + 0.0 * zc)
    pr.name = "uniform_flow_" + geometry
    return pr


def hydrostatic(axis="y", n=32, amp=0.3, cs=1.0) -> Problem:
    """Isothermal atmosphere in a periodic sinusoidal potential on a Cartesian
    mesh: Phi = amp sin(2 pi s), rho = exp(-Phi/cs**2), v = 0 (exact static
    solution)."""
    if axis == "x":
        p = default_params(geometry="cart", nx=n, ny=3, nz=1, xmin=0.0, xmax=1.0,
                           ymin=uniform_faces(0.0, 3.0, 3), zmin=np.array([0.0, 1.0]),
                           eos="iso", bc=("periodic",) * 4)
    elif axis == "y":
        p = default_params(geometry="cart", nx=1, ny=n, nz=1, xmin=0.0, xmax=1.0,
                           ymin=uniform_faces(0.0, 1.0, n), zmin=np.array([0.0, 1.0]),
                           eos="iso", bc=("periodic",) * 4)
    else:
        p = default_params(geometry="cart", nx=1, ny=3, nz=n, xmin=0.0, xmax=1.0,
                           ymin=uniform_faces(0.0, 3.0, 3), zmin=uniform_faces(0.0, 1.0, n),
                           eos="iso", bc=("periodic",) * 4)
    pr = _blank(p)
    shape = pr.shape
    zc, yc, xf, xc = _grid(p)
    s = {"x": xc, "y": yc, "z": zc}[axis]
    phi = _full(shape, amp * np.sin(2 * math.pi * s))
    pr.fields["pot"] = phi
    pr.fields["rho"] = np.exp(-phi / (cs * cs))
    pr.fields["cs"][:] = cs
    pr.name = "hydrostatic_" + axis
    return pr

CONFIGS = {
    # 2D polar isothermal Keplerian disk, 128 x 384, 10 steps, FARGO on
    "disk2d": lambda **kw: disk2d_cyl(**kw),
    # 3D spherical adiabatic disk, 1536 x 512 x 128
    "sph3d": lambda **kw: disk3d_sph(**kw),
    # 3D cylindrical isothermal disk with planet, 2048 x 768 x 96, 100 steps
    "cyl3d_planet": lambda **kw: disk3d_cyl_planet(**kw),
    # learned flux correction: coarse 768 x 256 and fine 3072 x 1024 planet disks
    "lfc_coarse": lambda **kw: disk2d_planet(**kw),
    "lfc_fine": lambda **kw: disk2d_planet(**dict(dict(nx=3072, ny=1024), **kw)),
}


def make(name: str, **kw) -> Problem:
    return CONFIGS[name](**kw)
