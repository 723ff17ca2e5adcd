"""Spreading of a narrow viscous ring (constant kinematic viscosity): the
similarity solution of Lynden-Bell & Pringle (1974) quoted in Sect. 5.1
("Viscous spread of a gaseous ring").  The printed formulas leave the order
of the Bessel function out; for constant viscosity it is 1/4, which is also
what the radial velocity formula of that section needs (the ratio
I_{-3/4}/I_{1/4}).  Units: ring radius R0 = 1 and mass M = 1 by default.

Sigma(r, t) = M / (pi R0^2 tau) u^(-1/4) I_{1/4}(2u/tau) exp(-(1 + u^2)/tau)
v_r(r, t)   = (6 nu / (tau R0)) [u - I_{-3/4}(2u/tau) / I_{1/4}(2u/tau)]
with u = r / R0 and tau = 12 nu t / R0^2.  Exponentially scaled Bessel
functions keep both finite for narrow rings."""
import numpy as np
from scipy.special import ive


def tau_of(nu, t, r0=1.0):
    return 12.0 * nu * t / r0 ** 2


def sigma(r, nu, t, mass=1.0, r0=1.0):
    tau = tau_of(nu, t, r0)
    u = np.asarray(r, dtype=np.float64) / r0
    x = 2.0 * u / tau
    # I_{1/4}(x) exp(-(1 + u^2)/tau) = ive(1/4, x) exp(x - (1 + u^2)/tau) = ive exp(-(1 - u)^2 / tau)
    return mass / (np.pi * r0 ** 2 * tau) * u ** -0.25 * ive(0.25, x) * np.exp(-(1.0 - u) ** 2 / tau)


def v_r(r, nu, t, r0=1.0):
    tau = tau_of(nu, t, r0)
    u = np.asarray(r, dtype=np.float64) / r0
    x = 2.0 * u / tau
    return 6.0 * nu / (tau * r0) * (u - ive(-0.75, x) / ive(0.25, x))
