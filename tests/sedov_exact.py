"""Self-similar solution of the point blast (Sedov-Taylor) in a gamma-law gas.

Test-only; shares nothing with the oracle or the GPU library.  A blast of
energy E released at a point in gas of density rho0 at negligible pressure
drives a spherical shock of radius R(t) = (E t^2 / (alpha rho0))^(1/5)
(dimensional analysis fixes the exponent; alpha depends on gamma only).

Behind the shock, with xi = r / R, u = R' f(xi), rho = rho0 g(xi) and
p = rho0 R'^2 h(xi), the Euler equations (mass, momentum, and entropy
conserved along particle paths, with R'' = -3 R'^2 / (2 R)) reduce to three
ordinary differential equations in xi:
    (f - xi) g' + g f'          = -2 g f / xi
    (f - xi) f' + h' / g        = 3 f / 2
    (f - xi) (h'/h - gamma g'/g) = 3
started at xi = 1 from the strong-shock jump conditions f = h = 2/(gamma+1),
g = (gamma+1)/(gamma-1) and integrated inward.  The energy inside the shock,
E = 4 pi rho0 R'^2 R^3 int_0^1 (g f^2/2 + h/(gamma-1)) xi^2 dxi with
R' = 2R/(5t), gives alpha = (16 pi / 25) int_0^1 (...) xi^2 dxi.
"""
import math

import numpy as np
from scipy.integrate import solve_ivp


def _rhs(xi, y, gamma):
    f, g, h = y
    a = f - xi
    A = np.array([[g, a, 0.0],
                  [a, 0.0, 1.0 / g],
                  [0.0, -gamma * a / g, a / h]])
    b = np.array([-2.0 * g * f / xi, 1.5 * f, 3.0])
    return np.linalg.solve(A, b)


def profile(gamma=1.4, xi_min=1e-3, n=4000):
    """(xi, (f, g, h)) on [xi_min, 1], increasing xi."""
    y0 = [2.0 / (gamma + 1.0), (gamma + 1.0) / (gamma - 1.0), 2.0 / (gamma + 1.0)]
    xs = np.linspace(1.0, xi_min, n)
    sol = solve_ivp(_rhs, (1.0, xi_min), y0, t_eval=xs, args=(gamma,), rtol=1e-11,
                    atol=1e-13, method="DOP853")
    return sol.t[::-1], sol.y[:, ::-1]


def alpha(gamma=1.4):
    """E = alpha rho0 R^5 / t^2."""
    xi, (f, g, h) = profile(gamma)
    integrand = (0.5 * g * f * f + h / (gamma - 1.0)) * xi * xi
    return 16.0 * math.pi / 25.0 * np.trapezoid(integrand, xi)


def shock_radius(t, e_blast=1.0, rho0=1.0, gamma=1.4):
    return (e_blast * t * t / (alpha(gamma) * rho0)) ** 0.2


def measured_radius(rho, r, nbins, rmax):
    """Shock radius of a blast from cell densities ``rho`` at cell-centre
    radii ``r``: the shell-averaged density profile's outer half-maximum
    point (where the smeared front has risen halfway from the ambient density
    1 to the profile's peak), linearly interpolated between shells."""
    rho, r = np.ravel(rho), np.ravel(r)
    edges = np.linspace(0.0, rmax, nbins + 1)
    idx = np.clip(np.digitize(r, edges) - 1, 0, nbins - 1)
    keep = r < rmax
    cnt = np.bincount(idx[keep], minlength=nbins)
    prof = np.bincount(idx[keep], weights=rho[keep], minlength=nbins) / np.maximum(cnt, 1)
    k = int(np.argmax(prof))
    half = 1.0 + 0.5 * (prof[k] - 1.0)
    j = k
    while j + 1 < nbins and prof[j + 1] > half:
        j += 1
    c = 0.5 * (edges[:-1] + edges[1:])
    return c[j] + (prof[j] - half) / (prof[j] - prof[j + 1]) * (c[j + 1] - c[j])
