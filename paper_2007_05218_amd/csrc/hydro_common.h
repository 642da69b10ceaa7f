// hydro_common.h -- device-side building blocks of the CTU-PPM-HLLC step.
//
// Scheme: the paper's Castro hydro (bibliography entry CastroI; Sec. III
// describes its slope stencil and polynomial reconstruction): PPM parabolae
// with the monotonised-central slope and the Colella-Woodward (1984)
// parabola limiter (optionally after their shock flattening), characteristic
// tracing to the faces, an HLLC Riemann
// solver (Toro, Spruce & Speares 1994) with Davis (1988) wave-speed bounds,
// and the 3-D corner transport upwind coupling (Colella 1990, Saltzman 1994).
//
// Arithmetic contract: every expression below is evaluated in the
// parenthesisation written, in binary64, without FMA contraction (the
// library is built with -ffp-contract=off); division and sqrt are the
// correctly rounded IEEE operations; min/max are explicit compares.  This
// makes results independent of tiling and batch composition.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hydro {

constexpr double kC6 = 1.0 / 6.0;
constexpr double kC23 = 2.0 / 3.0;

__device__ __forceinline__ double dmin(double a, double b) { return a < b ? a : b; }
__device__ __forceinline__ double dmax(double a, double b) { return a > b ? a : b; }

// ---------------------------------------------------------------- EOS

// (rho, u, v, w, p) of a conserved state, and 1/rho.  The reciprocal of the
// density is formed once per state and multiplies (likewise 1/(gamma-1) and
// 1/c^2): FP64 division is a ten-instruction sequence on gfx950.
struct Prim {
    double r, u, v, w, p, ri;
};

__device__ __forceinline__ Prim prim_of(double U0, double U1, double U2, double U3,
                                        double U4, double gm1)
{
    Prim q;
    q.r = U0;
    q.ri = 1.0 / U0;
    q.u = U1 * q.ri;
    q.v = U2 * q.ri;
    q.w = U3 * q.ri;
    double ke = (0.5 * q.r) * ((q.u * q.u + q.v * q.v) + q.w * q.w);
    q.p = gm1 * (U4 - ke);
    return q;
}

// sound speed of a cell state (its 1/rho known)
__device__ __forceinline__ double sound_ri(double gamma, double p, double ri)
{
    return sqrt((gamma * p) * ri);
}

// total energy density of a primitive state; igm1 = 1/(gamma-1)
__device__ __forceinline__ double energy(double r, double u, double v, double w,
                                         double p, double igm1)
{
    return p * igm1 + (0.5 * r) * ((u * u + v * v) + w * w);
}

// velocity component a (0,1,2) of a primitive state
__device__ __forceinline__ double vel(const Prim &q, int a)
{
    return a == 0 ? q.u : (a == 1 ? q.v : q.w);
}

// ---------------------------------------------------------------- PPM

__device__ __forceinline__ double mc_slope(double am, double a0, double ap)
{
    double dl = a0 - am;
    double dr = ap - a0;
    double dc = 0.5 * (ap - am);
    if (dl * dr > 0.0)
        return copysign(dmin(dmin(fabs(dc), 2.0 * fabs(dl)), 2.0 * fabs(dr)), dc);
    return 0.0;
}

// Limited parabola of the middle cell of a[0..4]; returns its low/high face
// values, the jump dA = aR - aL and the curvature term a6.
struct Parab {
    double aL, aR, dA, a6;
};

// unlimited interface value between cells with averages al, ar and slopes
// sl, sr (the fourth-order interpolant with the limited slopes)
__device__ __forceinline__ double ppm_iface(double al, double ar, double sl, double sr)
{
    return 0.5 * (al + ar) - (sr - sl) * kC6;
}

// the parabola limiter applied to cell average a2 with unlimited interface
// values aL (low face) and aR (high face)
__device__ __forceinline__ Parab ppm_limit(double a2, double aL, double aR);

// Shock flattening (Colella & Woodward 1984, Sec. 4): with the cell's
// coefficient f < 1 the unlimited interface values move toward the cell
// average before the limiter (f = 1: untouched, so an unflattened cell
// computes exactly what it computes without flattening)
__device__ __forceinline__ Parab ppm_limit_flat(double a2, double aL, double aR, double f)
{
    if (f < 1.0) {
        aL = f * aL + (1.0 - f) * a2;
        aR = f * aR + (1.0 - f) * a2;
    }
    return ppm_limit(a2, aL, aR);
}

__device__ __forceinline__ Parab ppm(double a0, double a1, double a2, double a3, double a4,
                                     double f = 1.0)
{
    double sm = mc_slope(a0, a1, a2);
    double s0 = mc_slope(a1, a2, a3);
    double sp = mc_slope(a2, a3, a4);
    return ppm_limit_flat(a2, ppm_iface(a1, a2, sm, s0), ppm_iface(a2, a3, s0, sp), f);
}

__device__ __forceinline__ Parab ppm_limit(double a2, double aL, double aR)
{
    if ((aR - a2) * (a2 - aL) <= 0.0) {
        aL = a2;
        aR = a2;
    } else {
        double dA = aR - aL;
        double m = a2 - 0.5 * (aL + aR);
        double t1 = dA * m;
        double t2 = (dA * dA) * kC6;
        if (t1 > t2)
            aL = 3.0 * a2 - 2.0 * aR;
        else if (-t2 > t1)
            aR = 3.0 * a2 - 2.0 * aL;
    }
    Parab P;
    P.aL = aL;
    P.aR = aR;
    P.dA = aR - aL;
    P.a6 = 6.0 * (a2 - 0.5 * (aL + aR));
    return P;
}

// average over the part of the cell next to the high face swept in dt by a
// wave of speed lam (the face value when lam <= 0)
__device__ __forceinline__ double int_hi(const Parab &P, double lam, double dtdx)
{
    double s = (lam > 0.0 ? lam : 0.0) * dtdx;
    return P.aR - (0.5 * s) * (P.dA - (1.0 - kC23 * s) * P.a6);
}

// the same next to the low face, for lam < 0
__device__ __forceinline__ double int_lo(const Parab &P, double lam, double dtdx)
{
    double s = (lam < 0.0 ? -lam : 0.0) * dtdx;
    return P.aL + (0.5 * s) * (P.dA + (1.0 - kC23 * s) * P.a6);
}

// ---------------------------------------------------------------- tracing

// Traced face states of one cell along axis d.  Inputs: the five primitive
// stencils along d (index 2 = the cell), its sound speed c.  Variables in
// trace order: rho, un (normal velocity), ut1, ut2 (transverse, lab order),
// p.  Output states are in lab order (rho, u, v, w, p).
//
// Waves - / 0 / + with speeds un-c, un, un+c at the cell centre.  The high
// face takes the + wave's integral as reference and subtracts, for each
// other wave moving toward it (lam > 0), its amplitude times the right
// eigenvector; the low face mirrors this with the - wave and lam < 0.
struct Face {
    double r, u, v, w, p;
    double ri;  // 1/r, where a consumer needs it (HLLC inputs)
};

__device__ __forceinline__ void set_lab(Face &f, int d, double r, double un, double ut1,
                                        double ut2, double p)
{
    f.r = r;
    f.p = p;
    if (d == 0) {
        f.u = un; f.v = ut1; f.w = ut2;
    } else if (d == 1) {
        f.u = ut1; f.v = un; f.w = ut2;
    } else {
        f.u = ut1; f.v = ut2; f.w = un;
    }
}

// the tracing proper, from the five limited parabolae of the cell
__device__ __forceinline__ void trace_parab(const Parab &Pr, const Parab &Pu, const Parab &P1,
                                            const Parab &P2, const Parab &Pp, double rho,
                                            double un, double c, double ri, int d, double dtdx,
                                            Face &hi, Face &lo)
{
    const double lm = un - c, l0 = un, lp = un + c;
    const double rc = rho * c;
    const double cs2 = c * c;
    const double ics2 = 1.0 / cs2;
    const double cor = c * ri;

    {  // high face, reference = + wave
        double r_r = int_hi(Pr, lp, dtdx);
        double r_u = int_hi(Pu, lp, dtdx);
        double r_p = int_hi(Pp, lp, dtdx);
        double dum = r_u - int_hi(Pu, lm, dtdx);
        double dpm = r_p - int_hi(Pp, lm, dtdx);
        double drz = r_r - int_hi(Pr, l0, dtdx);
        double dpz = r_p - int_hi(Pp, l0, dtdx);
        double am = lm > 0.0 ? (0.5 * (dpm - rc * dum)) * ics2 : 0.0;
        double az = l0 > 0.0 ? drz - dpz * ics2 : 0.0;
        double t1 = l0 > 0.0 ? int_hi(P1, l0, dtdx) : int_hi(P1, lp, dtdx);
        double t2 = l0 > 0.0 ? int_hi(P2, l0, dtdx) : int_hi(P2, lp, dtdx);
        set_lab(hi, d, r_r - (am + az), r_u + cor * am, t1, t2, r_p - cs2 * am);
    }
    {  // low face, reference = - wave
        double r_r = int_lo(Pr, lm, dtdx);
        double r_u = int_lo(Pu, lm, dtdx);
        double r_p = int_lo(Pp, lm, dtdx);
        double dup = r_u - int_lo(Pu, lp, dtdx);
        double dpp = r_p - int_lo(Pp, lp, dtdx);
        double drz = r_r - int_lo(Pr, l0, dtdx);
        double dpz = r_p - int_lo(Pp, l0, dtdx);
        double ap = lp < 0.0 ? (0.5 * (dpp + rc * dup)) * ics2 : 0.0;
        double az = l0 < 0.0 ? drz - dpz * ics2 : 0.0;
        double t1 = l0 < 0.0 ? int_lo(P1, l0, dtdx) : int_lo(P1, lm, dtdx);
        double t2 = l0 < 0.0 ? int_lo(P2, l0, dtdx) : int_lo(P2, lm, dtdx);
        set_lab(lo, d, r_r - (az + ap), r_u - cor * ap, t1, t2, r_p - cs2 * ap);
    }
}

__device__ __forceinline__ void trace_cell(const double (&rs)[5], const double (&uns)[5],
                                           const double (&t1s)[5], const double (&t2s)[5],
                                           const double (&ps)[5], double c, double ri, int d,
                                           double dtdx, Face &hi, Face &lo, double f = 1.0)
{
    trace_parab(ppm(rs[0], rs[1], rs[2], rs[3], rs[4], f),
                ppm(uns[0], uns[1], uns[2], uns[3], uns[4], f),
                ppm(t1s[0], t1s[1], t1s[2], t1s[3], t1s[4], f),
                ppm(t2s[0], t2s[1], t2s[2], t2s[3], t2s[4], f),
                ppm(ps[0], ps[1], ps[2], ps[3], ps[4], f), rs[2], uns[2], c, ri, d, dtdx, hi,
                lo);
}

// PPM along a column marched cell by cell (the z-direction of the marching
// kernels): the slope and the high interface value a cell computes are its
// upper neighbour's low slope and low interface value, so each step forms
// one new slope and one interface value.  State at cell k: a = a(k),
// an = a(k+1), s = slope(k), iL = unlimited interface value at k-1/2.
struct PPMColumn {
    double a, an, s, iL;
    // start at cell k from a(k-2) .. a(k+1)
    __device__ __forceinline__ void init(double am2, double am1, double a0, double ap1)
    {
        const double sm = mc_slope(am2, am1, a0);
        a = a0;
        an = ap1;
        s = mc_slope(am1, a0, ap1);
        iL = ppm_iface(am1, a0, sm, s);
    }
    // the limited parabola of the current cell (flattening coefficient f),
    // given a(k+2); then move to k+1
    __device__ __forceinline__ Parab step(double ap2, double f = 1.0)
    {
        const double sp = mc_slope(a, an, ap2);
        const double iR = ppm_iface(a, an, s, sp);
        const Parab P = ppm_limit_flat(a, iL, iR, f);
        a = an;
        an = ap2;
        s = sp;
        iL = iR;
        return P;
    }
};

// ---------------------------------------------------------------- HLLC

struct Flux {
    double m, mu, mv, mw, e;  // mass, x/y/z momentum, energy
};

__device__ __forceinline__ double fvel(const Face &q, int d)
{
    return d == 0 ? q.u : (d == 1 ? q.v : q.w);
}

// physical flux of state q (total energy E) through a d-face
__device__ __forceinline__ Flux phys_flux(const Face &q, double E, int d)
{
    double un = fvel(q, d);
    double m = q.r * un;
    Flux F;
    F.m = m;
    F.mu = m * q.u;
    F.mv = m * q.v;
    F.mw = m * q.w;
    if (d == 0) F.mu = m * un + q.p;
    else if (d == 1) F.mv = m * un + q.p;
    else F.mw = m * un + q.p;
    F.e = (E + q.p) * un;
    return F;
}

// HLLC flux through a d-face (input states carry 1/rho in .ri).  The four cases (left state, left star, right
// star, right state) are decided first; then only the chosen side's energy,
// physical flux and (if needed) star correction F_K + S_K (U*_K - U_K) are
// evaluated, each with exactly the arithmetic of its case.
__device__ __forceinline__ Flux hllc(const Face &L, const Face &R, int d, double gamma,
                                     double igm1)
{
    const double rL = L.r, uL = fvel(L, d), pL = L.p;
    const double rR = R.r, uR = fvel(R, d), pR = R.p;
    const double cL = sound_ri(gamma, pL, L.ri);
    const double cR = sound_ri(gamma, pR, R.ri);
    const double SL = dmin(uL - cL, uR - cR);
    const double SR = dmax(uL + cL, uR + cR);
    const double num = ((pR - pL) + (rL * uL) * (SL - uL)) - (rR * uR) * (SR - uR);
    const double den = rL * (SL - uL) - rR * (SR - uR);
    const double Ss = num / den;
    const bool sL = 0.0 <= SL, sS = 0.0 <= Ss, sR = 0.0 < SR;
    const bool left = sL || sS;
    const bool star = !sL && (sS || sR);
    Face K;
    K.r = left ? L.r : R.r;
    K.u = left ? L.u : R.u;
    K.v = left ? L.v : R.v;
    K.w = left ? L.w : R.w;
    K.p = left ? L.p : R.p;
    const double SK = left ? SL : SR;
    const double E = energy(K.r, K.u, K.v, K.w, K.p, igm1);
    Flux F = phys_flux(K, E, d);
    if (star) {
        const double r = K.r, uK = fvel(K, d), pK = K.p;
        double chi = (SK - uK) / (SK - Ss);
        double s0 = chi * r;
        double su = chi * (r * K.u);
        double sv = chi * (r * K.v);
        double sw = chi * (r * K.w);
        if (d == 0) su = chi * (r * Ss);
        else if (d == 1) sv = chi * (r * Ss);
        else sw = chi * (r * Ss);
        double se = chi * (E + (r * (Ss - uK)) * (Ss + pK / (r * (SK - uK))));
        F.m = F.m + SK * (s0 - r);
        F.mu = F.mu + SK * (su - r * K.u);
        F.mv = F.mv + SK * (sv - r * K.v);
        F.mw = F.mw + SK * (sw - r * K.w);
        F.e = F.e + SK * (se - E);
    }
    return F;
}

// ---------------------------------------------------------------- corrections

// Corrected state prim(U(q) - ...).  V = corrected conserved state; when its
// density or pressure is not positive, q is kept and bit 8 is raised.  The
// result carries 1/rho.
__device__ __forceinline__ Face accept(const Face &q, double V0, double V1, double V2,
                                       double V3, double V4, double gm1, int &err)
{
    Prim c = prim_of(V0, V1, V2, V3, V4, gm1);
    Face f;
    if (c.r <= 0.0 || c.p <= 0.0) {
        err |= 8;
        f = q;
        f.ri = 1.0 / q.r;
        return f;
    }
    f.r = c.r;
    f.u = c.u;
    f.v = c.v;
    f.w = c.w;
    f.p = c.p;
    f.ri = c.ri;
    return f;
}

}  // namespace hydro
