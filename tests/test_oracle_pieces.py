"""Pins of the oracle's building blocks against closed forms, identities and
hand-checkable special cases (no GPU)."""
import math

import numpy as np
import pytest

G = 1.4


def test_prim_cons_round_trip(orc):
    rng = np.random.default_rng(0)
    for _ in range(2000):
        q = np.array([rng.uniform(0.1, 10), *rng.uniform(-3, 3, 3), rng.uniform(0.01, 10)])
        U = orc.cons_of_prim(q, G)
        U2 = orc.cons_of_prim(orc.prim_of_cons(U, G), G)
        ulp = np.spacing(np.abs(U))
        assert np.all(np.abs(U2 - U) <= 4 * ulp + 1e-300), (q, U, U2)


def test_cons_of_prim_closed_form(orc):
    # E = p/(gamma-1) + rho |u|^2 / 2, momenta rho*u
    U = orc.cons_of_prim([2.0, 1.0, -2.0, 0.5, 0.8], G)
    assert U[0] == 2.0 and U[1] == 2.0 and U[2] == -4.0 and U[3] == 1.0
    assert U[4] == pytest.approx(0.8 / 0.4 + 0.5 * 2.0 * (1 + 4 + 0.25), rel=1e-15)


# ----------------------------------------------------------------- PPM

def _cubic_avgs(coef, x0, h):
    """exact cell averages of a cubic over cells [x0+m h, x0+(m+1) h], m=0..4"""
    a, b, c, d = coef
    F = lambda x: a * x + b * x**2 / 2 + c * x**3 / 3 + d * x**4 / 4
    return np.array([(F(x0 + (m + 1) * h) - F(x0 + m * h)) / h for m in range(5)])


def test_ppm_interfaces_exact_on_cubic(orc):
    # monotone, gently curved cubic: the slopes are unlimited (central) and the
    # parabola limiter is inactive, so the interface values are the 4th-order
    # ones, which are exact for cubic cell averages
    coef = (1.0, 0.3, 0.05, 0.01)
    f = lambda x: coef[0] + coef[1] * x + coef[2] * x**2 + coef[3] * x**3
    h = 0.1
    x0 = 0.2
    a = _cubic_avgs(coef, x0, h)
    aL, aR = orc.ppm_parabola(a)
    xl = x0 + 2 * h
    xr = x0 + 3 * h
    assert abs(aL - f(xl)) <= 1e-14 * abs(f(xl))
    assert abs(aR - f(xr)) <= 1e-14 * abs(f(xr))


def test_ppm_constant_data_exact(orc):
    for c in (0.0, 1.0, -3.25, 1e-300, 7.5e10):
        a = np.full(5, c)
        assert orc.ppm_parabola(a) == (c, c)
        for lam in (-2.0, -0.5, 0.0, 0.5, 2.0):
            assert orc.ppm_integrals(a, lam, 0.3) == (c, c)


def test_ppm_local_extremum_flattened(orc):
    # a cell that is a local maximum gets a flat (constant) profile
    for a in ([0.0, 1.0, 3.0, 1.5, 0.2], [5.0, 4.0, 1.0, 2.0, 2.5], [0, 0, 0, 1, 1]):
        aL, aR = orc.ppm_parabola(np.array(a, dtype=float))
        assert aL == a[2] and aR == a[2]


def _parabola(aL, aR, a, xi):
    dA = aR - aL
    a6 = 6.0 * (a - 0.5 * (aL + aR))
    return aL + xi * (dA + a6 * (1.0 - xi))


def test_ppm_limited_parabola_monotone_and_conservative(orc):
    # whatever the data, the limited parabola averages to the cell value and
    # is monotone on the cell (no new extrema)
    rng = np.random.default_rng(1)
    xi = np.linspace(0, 1, 201)
    for _ in range(3000):
        a = rng.normal(size=5) * rng.choice([1e-3, 1.0, 1e3])
        aL, aR = orc.ppm_parabola(a)
        if aL == aR:
            assert aL == a[2]
            continue
        assert min(aL, aR) <= a[2] <= max(aL, aR)
        prof = _parabola(aL, aR, a[2], xi)
        scale = np.max(np.abs(a)) * 1e-12
        dif = np.diff(prof)
        assert np.all(dif >= -scale) or np.all(dif <= scale)
        # mean of the parabola over the cell (Simpson is exact for quadratics)
        mean = (prof[0] + 4 * prof[100] + prof[200]) / 6.0
        assert abs(mean - a[2]) <= scale * 10


def test_ppm_integral_over_whole_cell_is_average(orc):
    # s = |lam| dt/dx = 1: the swept region is the whole cell
    rng = np.random.default_rng(2)
    for _ in range(500):
        a = rng.normal(size=5)
        ip, _ = orc.ppm_integrals(a, 2.0, 0.5)
        _, im = orc.ppm_integrals(a, -2.0, 0.5)
        assert abs(ip - a[2]) <= 1e-14 * max(1.0, np.max(np.abs(a)))
        assert abs(im - a[2]) <= 1e-14 * max(1.0, np.max(np.abs(a)))


def test_ppm_integral_matches_quadrature(orc):
    # Ip = average of the parabola over [1-s, 1], Im over [0, s]
    rng = np.random.default_rng(3)
    for _ in range(300):
        a = rng.normal(size=5)
        aL, aR = orc.ppm_parabola(a)
        s = rng.uniform(0.05, 0.95)
        ip, _ = orc.ppm_integrals(a, s, 1.0)
        _, im = orc.ppm_integrals(a, -s, 1.0)
        xs = np.linspace(1 - s, 1, 4001)
        ref_p = np.trapezoid(_parabola(aL, aR, a[2], xs), xs) / s
        xs = np.linspace(0, s, 4001)
        ref_m = np.trapezoid(_parabola(aL, aR, a[2], xs), xs) / s
        assert abs(ip - ref_p) < 1e-7 and abs(im - ref_m) < 1e-7
        # waves moving away from a face leave the face value
        ip0, im0 = orc.ppm_integrals(a, 0.0, 1.0)
        assert ip0 == aR and im0 == aL


# ----------------------------------------------------------------- tracing

def test_trace_uniform_is_exact(orc):
    q = np.array([[1.3, 0.4, -0.2, 0.7, 2.1]] * 5)
    for d in range(3):
        hi, lo = orc.trace(q, d, G, 0.4)
        assert np.array_equal(hi, q[2]) and np.array_equal(lo, q[2])


@pytest.mark.parametrize("un", [0.7, -0.7])
def test_trace_entropy_wave_is_upwind_average(orc, un):
    # pressure and velocity uniform, density varying: only the entropy wave
    # (speed un) carries a jump; the traced density is the average of the
    # density parabola over the region that wave sweeps into the face
    rho = np.array([1.0, 1.1, 1.25, 1.3, 1.32])
    q = np.zeros((5, 5))
    q[:, 0] = rho
    q[:, 1] = un
    q[:, 4] = 1.0
    dtdx = 0.35
    hi, lo = orc.trace(q, 0, G, dtdx)
    ip, im = orc.ppm_integrals(rho, un, dtdx)
    if un > 0:
        assert hi[0] == pytest.approx(ip, rel=2e-16, abs=0)
        aL, _ = orc.ppm_parabola(rho)
        # the low face sees no entropy wave: its density is the - wave's, which
        # at un - c < 0 is the integral near the low face
        _, im_minus = orc.ppm_integrals(rho, un - math.sqrt(G / 1.25), dtdx)
        assert lo[0] == pytest.approx(im_minus, rel=2e-16)
    else:
        assert lo[0] == pytest.approx(im, rel=2e-16, abs=0)
    for f in (hi, lo):
        assert f[1] == un and f[4] == 1.0 and f[2] == 0.0 and f[3] == 0.0


def test_trace_axis_relabelling(orc):
    # tracing along y with (u, v) swapped equals tracing along x
    rng = np.random.default_rng(4)
    q = np.column_stack([rng.uniform(0.5, 2, 5), rng.normal(size=5) * 0.3,
                         rng.normal(size=5) * 0.3, rng.normal(size=5) * 0.3,
                         rng.uniform(0.5, 2, 5)])
    hx, lx = orc.trace(q, 0, G, 0.3)
    qy = q[:, [0, 2, 1, 3, 4]]
    hy, ly = orc.trace(qy, 1, G, 0.3)
    assert np.array_equal(hx, hy[[0, 2, 1, 3, 4]])
    assert np.array_equal(lx, ly[[0, 2, 1, 3, 4]])


# ----------------------------------------------------------------- HLLC

def _phys_flux(q, d, g=G):
    rho, p = q[0], q[4]
    u = q[1 + d]
    E = p / (g - 1) + 0.5 * rho * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2)
    F = np.array([rho * u, rho * u * q[1], rho * u * q[2], rho * u * q[3], (E + p) * u])
    F[1 + d] += p
    return F


def test_hllc_consistency(orc):
    rng = np.random.default_rng(5)
    for _ in range(500):
        q = np.array([rng.uniform(0.1, 5), *rng.normal(size=3), rng.uniform(0.1, 5)])
        for d in range(3):
            F = orc.hllc(q, q, d, G)
            ref = _phys_flux(q, d)
            assert np.allclose(F, ref, rtol=1e-14, atol=1e-14 * np.max(np.abs(ref)))


def test_hllc_stationary_contact(orc):
    qL = np.array([1.0, 0.0, 0.3, -0.2, 0.7])
    qR = np.array([0.2, 0.0, -0.5, 0.1, 0.7])
    F = orc.hllc(qL, qR, 0, G)
    assert F[0] == 0.0 and F[2] == 0.0 and F[3] == 0.0 and F[4] == 0.0
    assert F[1] == 0.7


def test_hllc_moving_contact_is_upwind(orc):
    # an isolated contact moving at speed u0 is resolved exactly: the flux is
    # the physical flux of the upwind state
    for u0 in (0.4, -0.4):
        qL = np.array([1.0, u0, 0.0, 0.0, 1.0])
        qR = np.array([0.3, u0, 0.0, 0.0, 1.0])
        F = orc.hllc(qL, qR, 0, G)
        ref = _phys_flux(qL if u0 > 0 else qR, 0)
        assert np.allclose(F, ref, rtol=1e-13, atol=1e-14)


def test_hllc_supersonic_upwind(orc):
    qL = np.array([1.0, 3.0, 0.1, 0.2, 1.0])
    qR = np.array([0.5, 2.5, -0.1, 0.0, 0.5])
    assert np.array_equal(orc.hllc(qL, qR, 0, G), _phys_flux(qL, 0)) or \
        np.allclose(orc.hllc(qL, qR, 0, G), _phys_flux(qL, 0), rtol=1e-15)
    qL2 = qL.copy(); qL2[1] = -3.0
    qR2 = qR.copy(); qR2[1] = -2.5
    assert np.allclose(orc.hllc(qL2, qR2, 0, G), _phys_flux(qR2, 0), rtol=1e-15)


def test_hllc_mirror_symmetry(orc):
    # x -> -x swaps the states and flips the normal velocity; the mass, energy
    # and transverse-momentum fluxes change sign, the normal-momentum flux not
    rng = np.random.default_rng(6)
    for _ in range(300):
        qL = np.array([rng.uniform(0.1, 3), *rng.normal(size=3), rng.uniform(0.1, 3)])
        qR = np.array([rng.uniform(0.1, 3), *rng.normal(size=3), rng.uniform(0.1, 3)])
        F = orc.hllc(qL, qR, 0, G)
        mL = qR.copy(); mL[1] = -mL[1]
        mR = qL.copy(); mR[1] = -mR[1]
        Fm = orc.hllc(mL, mR, 0, G)
        expect = np.array([-F[0], F[1], -F[2], -F[3], -F[4]])
        sc = np.max(np.abs(F)) + 1.0
        assert np.allclose(Fm, expect, rtol=1e-15, atol=1e-15 * sc)


def test_hllc_star_flux_rankine_hugoniot(orc):
    # across the contact, F*_R - F*_L = S* (U*_R - U*_L); equivalently the flux
    # is continuous as S* crosses 0.  Check continuity by sliding both states'
    # velocities so that S* passes through zero.
    qL = np.array([1.0, 0.0, 0.2, 0.1, 1.0])
    qR = np.array([0.5, 0.0, -0.1, 0.3, 0.6])
    base = orc.hllc(qL, qR, 0, G)
    # find the shift that puts S* at zero by bisection on the mass flux sign
    lo, hi = -1.0, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        a, b = qL.copy(), qR.copy()
        a[1] += mid; b[1] += mid
        if orc.hllc(a, b, 0, G)[0] > 0:
            hi = mid
        else:
            lo = mid
    a1, b1 = qL.copy(), qR.copy(); a1[1] += lo; b1[1] += lo
    a2, b2 = qL.copy(), qR.copy(); a2[1] += hi; b2[1] += hi
    assert np.allclose(orc.hllc(a1, b1, 0, G), orc.hllc(a2, b2, 0, G), atol=1e-12)
    assert np.all(np.isfinite(base))
