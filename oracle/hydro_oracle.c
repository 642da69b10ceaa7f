/*
 * hydro_oracle.c -- FP64 CPU oracle of one unsplit CTU-PPM + HLLC step.
 *
 * TEST INFRASTRUCTURE ONLY (see hydro_oracle.h): used by the tests, the smoke
 * check and the CPU-baseline leg of the benchmark, never by the product path.
 *
 * The code is deliberately plain: every stage of the step is computed over
 * its whole index region into its own array, in the order the method takes
 * them, and the only parallelism is an OpenMP loop over the outer index of
 * each stage.  Nothing is fused, tiled or reordered.
 *
 * Method (the paper's Castro hydro, bibliography entry CastroI; the paper's
 * Sec. III describes its slope stencil and polynomial reconstruction):
 *   A0 ghost fill, A1 primitive variables, A2 CFL timestep,
 *   A3 PPM parabolae with the monotonised-central slope and the
 *      Colella-Woodward (1984) parabola limiter,
 *   A4 characteristic tracing of the parabolae to the cell faces over dt,
 *   A5 HLLC fluxes of the traced states (round 1),
 *   A6 corner coupling: each traced state corrected by dt/3 of one
 *      transverse flux difference, then HLLC (round 2, 6 flux families),
 *   A7 final states: each traced state corrected by dt/2 of the two
 *      round-2 transverse flux differences, then HLLC (round 3),
 *   A8 conservative update plus a time-centred constant-gravity source,
 *   A9 (optional) passively advected species, carried by the mass fluxes of
 *      the three rounds.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no -ffast-math).
 */
#include "hydro_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* hook for the operation-counting build (oracle/opcount.cpp): marks the end
 * of stage k of orc_advance_region; a no-op here */
#ifndef ORC_STAGE_MARK
#define ORC_STAGE_MARK(k) ((void)0)
#endif

#define C6 (1.0 / 6.0)
#define C23 (2.0 / 3.0)

static inline double mn(double a, double b) { return a < b ? a : b; }
static inline double mx(double a, double b) { return a > b ? a : b; }

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* box geometry                                                        */
/* ------------------------------------------------------------------ */

static void extents(const orc_box *b, long long s[3])
{
    for (int d = 0; d < 3; ++d) s[d] = (long long)b->n[d] + 2LL * b->ng;
}

long long orc_state_elems(const orc_box *b)
{
    long long s[3];
    extents(b, s);
    return 5LL * s[0] * s[1] * s[2];
}

static int box_ok(const orc_box *b)
{
    if (!b || b->ng < 3) return 0;
    for (int d = 0; d < 3; ++d) {
        if (b->n[d] < 1 || !(b->dx[d] > 0.0)) return 0;
        for (int side = 0; side < 2; ++side) {
            int bc = side ? b->bc_hi[d] : b->bc_lo[d];
            if (bc < ORC_BC_PERIODIC || bc > ORC_BC_REFLECT) return 0;
            if (bc != ORC_BC_OUTFLOW && b->n[d] < b->ng) return 0;
        }
        if ((b->bc_lo[d] == ORC_BC_PERIODIC) != (b->bc_hi[d] == ORC_BC_PERIODIC))
            return 0;
    }
    return 1;
}

/* linear offset of cell (i,j,k) within one component */
static inline long long cidx(const long long s[3], int ng, int i, int j, int k)
{
    return ((long long)(k + ng) * s[1] + (j + ng)) * s[0] + (i + ng);
}

/* ------------------------------------------------------------------ */
/* A0: ghost fill                                                      */
/* ------------------------------------------------------------------ */

/* Source index along one axis for ghost index g (g < 0 or g >= n) and the
 * sign applied to the normal momentum.  Periodic wraps, outflow copies the
 * nearest valid cell, reflect mirrors about the face. */
static int ghost_src(int g, int n, int bc_lo, int bc_hi, int *flip)
{
    *flip = 0;
    if (g < 0) {
        int m = -1 - g; /* g = -1-m */
        if (bc_lo == ORC_BC_PERIODIC) return n - 1 - m;
        if (bc_lo == ORC_BC_OUTFLOW) return 0;
        *flip = 1;
        return m;
    } else {
        int m = g - n; /* g = n+m */
        if (bc_hi == ORC_BC_PERIODIC) return m;
        if (bc_hi == ORC_BC_OUTFLOW) return n - 1;
        *flip = 1;
        return n - 1 - m;
    }
}

/* fill the ghosts of nc components; hydro: component 1+d is the
 * d-momentum, whose sign a reflecting face flips */
static void fill_comps(double *U, const orc_box *b, int nc, int hydro)
{
    long long s[3];
    extents(b, s);
    const long long cs = s[0] * s[1] * s[2];
    const int ng = b->ng;
    /* axis d is filled over the full range of the axes already filled
     * (those < d) and over the valid range of the axes not yet filled */
    for (int d = 0; d < 3; ++d) {
        int lo[3], hi[3];
        for (int e = 0; e < 3; ++e) {
            lo[e] = e < d ? -ng : 0;
            hi[e] = e < d ? b->n[e] + ng : b->n[e];
        }
        for (int side = 0; side < 2; ++side) {
            lo[d] = side ? b->n[d] : -ng;
            hi[d] = side ? b->n[d] + ng : 0;
            for (int k = lo[2]; k < hi[2]; ++k)
                for (int j = lo[1]; j < hi[1]; ++j)
                    for (int i = lo[0]; i < hi[0]; ++i) {
                        int p[3] = {i, j, k}, q[3] = {i, j, k}, flip;
                        q[d] = ghost_src(p[d], b->n[d], b->bc_lo[d],
                                         b->bc_hi[d], &flip);
                        long long dst = cidx(s, ng, p[0], p[1], p[2]);
                        long long src = cidx(s, ng, q[0], q[1], q[2]);
                        for (int c = 0; c < nc; ++c) {
                            double v = U[c * cs + src];
                            U[c * cs + dst] = (hydro && flip && c == 1 + d) ? -v : v;
                        }
                    }
        }
    }
}

int orc_fill_ghosts(double *U, const orc_box *b)
{
    if (!U || !box_ok(b)) return -1;
    fill_comps(U, b, 5, 1);
    return 0;
}

int orc_fill_ghosts_species(double *S, int nspec, const orc_box *b)
{
    if (!S || nspec < 1 || nspec > ORC_MAX_SPECIES || !box_ok(b)) return -1;
    fill_comps(S, b, nspec, 0);
    return 0;
}

/* ------------------------------------------------------------------ */
/* A1: equation of state and variable changes                          */
/* ------------------------------------------------------------------ */

/* (rho,u,v,w,p) and the sound speed c from conserved variables.  The
 * reciprocal of the density is formed once and multiplies, as do 1/(gamma-1)
 * and 1/c^2 below: one division per state instead of one per use. */
static void prim_c(const double U[5], double gamma, double gm1, double q[6])
{
    double rho = U[0];
    double rinv = 1.0 / rho;
    double u = U[1] * rinv;
    double v = U[2] * rinv;
    double w = U[3] * rinv;
    double ke = (0.5 * rho) * ((u * u + v * v) + w * w);
    double p = gm1 * (U[4] - ke);
    q[0] = rho;
    q[1] = u;
    q[2] = v;
    q[3] = w;
    q[4] = p;
    q[5] = sqrt((gamma * p) * rinv);
}

void orc_prim_of_cons(const double U[5], double gamma, double q[5])
{
    double t[6];
    prim_c(U, gamma, gamma - 1.0, t);
    for (int v = 0; v < 5; ++v) q[v] = t[v];
}

/* conserved variables of a primitive state; igm1 = 1/(gamma-1) */
static void cons_of(const double q[5], double igm1, double U[5])
{
    double rho = q[0], u = q[1], v = q[2], w = q[3], p = q[4];
    U[0] = rho;
    U[1] = rho * u;
    U[2] = rho * v;
    U[3] = rho * w;
    U[4] = p * igm1 + (0.5 * rho) * ((u * u + v * v) + w * w);
}

void orc_cons_of_prim(const double q[5], double gamma, double U[5])
{
    cons_of(q, 1.0 / (gamma - 1.0), U);
}

/* ------------------------------------------------------------------ */
/* A2: CFL timestep                                                    */
/* ------------------------------------------------------------------ */

int orc_estimate_dt(const double *U, const orc_box *b, const orc_params *pr,
                    double *dt)
{
    if (!U || !dt || !pr || !box_ok(b)) return -1;
    long long s[3];
    extents(b, s);
    const long long cs = s[0] * s[1] * s[2];
    const double gamma = pr->gamma, gm1 = gamma - 1.0;
    double smax[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < b->n[2]; ++k)
        for (int j = 0; j < b->n[1]; ++j)
            for (int i = 0; i < b->n[0]; ++i) {
                long long o = cidx(s, b->ng, i, j, k);
                double Uc[5], q[6];
                for (int c = 0; c < 5; ++c) Uc[c] = U[c * cs + o];
                prim_c(Uc, gamma, gm1, q);
                for (int d = 0; d < 3; ++d)
                    smax[d] = mx(smax[d], fabs(q[1 + d]) + q[5]);
            }
    *dt = pr->cfl * mn(mn(b->dx[0] / smax[0], b->dx[1] / smax[1]),
                       b->dx[2] / smax[2]);
    return 0;
}

/* ------------------------------------------------------------------ */
/* A3: PPM reconstruction                                              */
/* ------------------------------------------------------------------ */

/* monotonised-central limited slope of the middle value */
static double mc_slope(double am, double a0, double ap)
{
    double dl = a0 - am;
    double dr = ap - a0;
    double dc = 0.5 * (ap - am);
    if (dl * dr > 0.0)
        return copysign(mn(mn(fabs(dc), 2.0 * fabs(dl)), 2.0 * fabs(dr)), dc);
    return 0.0;
}

/* limited face values (aL at i-1/2, aR at i+1/2) of cell i from a[i-2..i+2];
 * f is the cell's shock-flattening coefficient (1: none) */
static void ppm_faces(const double a[5], double f, double *aLo, double *aRo)
{
    double dm = mc_slope(a[0], a[1], a[2]); /* slope of cell i-1 */
    double d0 = mc_slope(a[1], a[2], a[3]); /* slope of cell i   */
    double dp = mc_slope(a[2], a[3], a[4]); /* slope of cell i+1 */
    /* fourth-order interface values */
    double aL = 0.5 * (a[1] + a[2]) - (d0 - dm) * C6;
    double aR = 0.5 * (a[2] + a[3]) - (dp - d0) * C6;
    double ac = a[2];
    /* shock flattening (Colella & Woodward 1984, Sec. 4): near a strong
     * shock the interface values move toward the cell average, by the
     * coefficient f, before the limiter */
    if (f < 1.0) {
        aL = f * aL + (1.0 - f) * ac;
        aR = f * aR + (1.0 - f) * ac;
    }
    /* Colella-Woodward parabola limiter */
    if ((aR - ac) * (ac - aL) <= 0.0) {
        aL = ac;
        aR = ac;
    } else {
        double dA = aR - aL;
        double m = ac - 0.5 * (aL + aR);
        double t1 = dA * m;
        double t2 = (dA * dA) * C6;
        if (t1 > t2)
            aL = 3.0 * ac - 2.0 * aR;
        else if (-t2 > t1)
            aR = 3.0 * ac - 2.0 * aL;
    }
    *aLo = aL;
    *aRo = aR;
}

void orc_ppm_parabola(const double a5[5], double out[2])
{
    ppm_faces(a5, 1.0, &out[0], &out[1]);
}

void orc_ppm_parabola_flat(const double a5[5], double f, double out[2])
{
    ppm_faces(a5, f, &out[0], &out[1]);
}

/* ------------------------------------------------------------------ */
/* shock flattening (Colella & Woodward 1984, Sec. 4)                  */
/* ------------------------------------------------------------------ */

/* Along one axis, cell i is in a shock when the flow converges there
 * (u[i-1] - u[i+1] > 0) and the pressure jumps across it by more than
 * FL_EPS of the smaller neighbouring pressure; its steepness measure
 * z = |p[i+1]-p[i-1]| / |p[i+2]-p[i-2]| (near 1/2 in a smooth profile, near
 * 1 in a shock spread over two cells) gives chi = clamp(FL_W2 (z - FL_W1),
 * 0, 1) there, 0 elsewhere.  The cell's coefficient along the axis is
 * 1 - max(chi[i], chi[i+s]), where s points to the lower-pressure side
 * (s = -1 when p[i+1] > p[i-1], else +1): a cell next to a shock on its
 * high-pressure side -- the gas the shock has just passed -- is flattened
 * with it. */
#define FL_W1 0.75
#define FL_W2 10.0
#define FL_EPS 0.33
#define FL_TINY 1e-300

/* chi of the centre of p5[0..4], u3[0..2] (cells i-2..i+2 and i-1..i+1) */
static double flat_chi(const double p5[5], const double u3[3])
{
    double dp = p5[3] - p5[1];
    double dp2 = p5[4] - p5[0];
    double z = fabs(dp) / mx(fabs(dp2), FL_TINY);
    double chi = mn(1.0, mx(0.0, FL_W2 * (z - FL_W1)));
    int shock = (u3[0] - u3[2] > 0.0) && (fabs(dp) > FL_EPS * mn(p5[3], p5[1]));
    return shock ? chi : 0.0;
}

double orc_flatten_1d(const double p7[7], const double un7[7])
{
    /* chi of cells i-1, i, i+1 */
    double chi[3];
    for (int m = 0; m < 3; ++m) chi[m] = flat_chi(&p7[m], &un7[m + 1]);
    int s = p7[4] > p7[2] ? -1 : 1;
    return 1.0 - mx(chi[1], chi[1 + s]);
}

/* average of the parabola over the part of the cell swept by a wave of speed
 * lam in time dt (s = |lam| dt/dx), next to the high face (lam > 0) or next
 * to the low face (lam < 0); a wave moving away leaves the face value */
static double edge_hi(double ac, double aL, double aR, double lam, double dtdx)
{
    double dA = aR - aL;
    double a6 = 6.0 * (ac - 0.5 * (aL + aR));
    double s = (lam > 0.0 ? lam : 0.0) * dtdx;
    return aR - (0.5 * s) * (dA - (1.0 - C23 * s) * a6);
}

static double edge_lo(double ac, double aL, double aR, double lam, double dtdx)
{
    double dA = aR - aL;
    double a6 = 6.0 * (ac - 0.5 * (aL + aR));
    double s = (lam < 0.0 ? -lam : 0.0) * dtdx;
    return aL + (0.5 * s) * (dA + (1.0 - C23 * s) * a6);
}

void orc_ppm_integrals(const double a5[5], double lam, double dtdx, double *Ip,
                       double *Im)
{
    double aL, aR;
    ppm_faces(a5, 1.0, &aL, &aR);
    *Ip = edge_hi(a5[2], aL, aR, lam, dtdx);
    *Im = edge_lo(a5[2], aL, aR, lam, dtdx);
}

/* ------------------------------------------------------------------ */
/* A4: characteristic tracing                                          */
/* ------------------------------------------------------------------ */

/* the other two axes of d, in lab order */
static void transverse(int d, int *t1, int *t2)
{
    *t1 = d == 0 ? 1 : 0;
    *t2 = d == 2 ? 1 : 2;
}

/* Face states of the cell at the centre of the stencil q[m] (cells i-2..i+2
 * along d; q[m] = rho,u,v,w,p), sound speed c of the centre cell.
 *
 * Waves nu = -, 0, + with speeds lam = un-c, un, un+c at the cell centre.
 * At the high face the reference state is the + wave's integral; a wave
 * reaches the face when lam > 0 and then enters through its amplitude
 * alpha = l_nu . (ref - I_nu), l_nu the left eigenvector of the primitive
 * system; the face state is ref - sum_nu alpha_nu r_nu.  The low face is the
 * mirror image with the - wave as reference and lam < 0. */
static void trace_cell(const double q[5][5], double c, int d, double dtdx, double flat,
                       double qhi[5], double qlo[5])
{
    int t1, t2;
    transverse(d, &t1, &t2);
    const int var[5] = {0, 1 + d, 1 + t1, 1 + t2, 4}; /* rho,un,ut1,ut2,p */
    const double rho = q[2][0];
    const double un = q[2][1 + d];
    const double lam[3] = {un - c, un, un + c};

    /* limited parabola of each variable (trace order) */
    double ac[5], aL[5], aR[5];
    for (int v = 0; v < 5; ++v) {
        double a[5];
        for (int m = 0; m < 5; ++m) a[m] = q[m][var[v]];
        ppm_faces(a, flat, &aL[v], &aR[v]);
        ac[v] = a[2];
    }
#define IP(v, nu) edge_hi(ac[v], aL[v], aR[v], lam[nu], dtdx)
#define IM(v, nu) edge_lo(ac[v], aL[v], aR[v], lam[nu], dtdx)

    const double rc = rho * c;
    const double cs2 = c * c;
    const double ics2 = 1.0 / cs2;
    const double cor = c * (1.0 / rho);
    double f[5];

    /* high face: reference = + wave */
    {
        double r_rho = IP(0, 2), r_un = IP(1, 2), r_p = IP(4, 2);
        double dum = r_un - IP(1, 0);
        double dpm = r_p - IP(4, 0);
        double drz = r_rho - IP(0, 1);
        double dpz = r_p - IP(4, 1);
        double am = lam[0] > 0.0 ? (0.5 * (dpm - rc * dum)) * ics2 : 0.0;
        double az = lam[1] > 0.0 ? drz - dpz * ics2 : 0.0;
        f[0] = r_rho - (am + az);
        f[1] = r_un + cor * am;
        f[2] = lam[1] > 0.0 ? IP(2, 1) : IP(2, 2);
        f[3] = lam[1] > 0.0 ? IP(3, 1) : IP(3, 2);
        f[4] = r_p - cs2 * am;
        for (int v = 0; v < 5; ++v) qhi[var[v]] = f[v];
    }
    /* low face: reference = - wave */
    {
        double r_rho = IM(0, 0), r_un = IM(1, 0), r_p = IM(4, 0);
        double dup = r_un - IM(1, 2);
        double dpp = r_p - IM(4, 2);
        double drz = r_rho - IM(0, 1);
        double dpz = r_p - IM(4, 1);
        double ap = lam[2] < 0.0 ? (0.5 * (dpp + rc * dup)) * ics2 : 0.0;
        double az = lam[1] < 0.0 ? drz - dpz * ics2 : 0.0;
        f[0] = r_rho - (az + ap);
        f[1] = r_un - cor * ap;
        f[2] = lam[1] < 0.0 ? IM(2, 1) : IM(2, 0);
        f[3] = lam[1] < 0.0 ? IM(3, 1) : IM(3, 0);
        f[4] = r_p - cs2 * ap;
        for (int v = 0; v < 5; ++v) qlo[var[v]] = f[v];
    }
#undef IP
#undef IM
}

void orc_trace(const double q5[5][5], int d, double gamma, double dtdx,
               double qhi[5], double qlo[5])
{
    double c = sqrt((gamma * q5[2][4]) * (1.0 / q5[2][0]));
    trace_cell(q5, c, d, dtdx, 1.0, qhi, qlo);
}

/* ------------------------------------------------------------------ */
/* A5-A7: HLLC Riemann solver                                          */
/* ------------------------------------------------------------------ */

/* flux of one state through a face normal to d; E is its total energy */
static void phys_flux(const double q[5], double E, int d, double F[5])
{
    double un = q[1 + d];
    double m = q[0] * un;
    F[0] = m;
    for (int e = 0; e < 3; ++e) F[1 + e] = m * q[1 + e];
    F[1 + d] = m * un + q[4];
    F[4] = (E + q[4]) * un;
}

/* HLLC star-region flux on side K with wave speed SK (Toro, Spruce &
 * Speares 1994): F*_K = F_K + S_K (U*_K - U_K) */
static void star_flux(const double q[5], double E, int d, double SK, double Ss,
                      double F[5])
{
    double rho = q[0], uK = q[1 + d], pK = q[4];
    double FK[5], UK[5], Us[5];
    phys_flux(q, E, d, FK);
    UK[0] = rho;
    UK[1] = rho * q[1];
    UK[2] = rho * q[2];
    UK[3] = rho * q[3];
    UK[4] = E;
    double chi = (SK - uK) / (SK - Ss);
    Us[0] = chi * rho;
    for (int e = 0; e < 3; ++e) Us[1 + e] = chi * (rho * q[1 + e]);
    Us[1 + d] = chi * (rho * Ss);
    Us[4] = chi * (E + (rho * (Ss - uK)) * (Ss + pK / (rho * (SK - uK))));
    for (int v = 0; v < 5; ++v) F[v] = FK[v] + SK * (Us[v] - UK[v]);
}

static double total_energy(const double q[5], double igm1)
{
    return q[4] * igm1 + (0.5 * q[0]) * ((q[1] * q[1] + q[2] * q[2]) + q[3] * q[3]);
}

/* igm1 = 1/(gamma-1) */
static void hllc(const double qL[5], const double qR[5], int d, double gamma,
                 double igm1, double F[5])
{
    double rL = qL[0], uL = qL[1 + d], pL = qL[4];
    double rR = qR[0], uR = qR[1 + d], pR = qR[4];
    double EL = total_energy(qL, igm1);
    double ER = total_energy(qR, igm1);
    double cL = sqrt((gamma * pL) * (1.0 / rL));
    double cR = sqrt((gamma * pR) * (1.0 / rR));
    /* Davis (1988) wave-speed bounds */
    double SL = mn(uL - cL, uR - cR);
    double SR = mx(uL + cL, uR + cR);
    double num = ((pR - pL) + (rL * uL) * (SL - uL)) - (rR * uR) * (SR - uR);
    double den = rL * (SL - uL) - rR * (SR - uR);
    double Ss = num / den;
    if (0.0 <= SL)
        phys_flux(qL, EL, d, F);
    else if (0.0 <= Ss)
        star_flux(qL, EL, d, SL, Ss, F);
    else if (0.0 < SR)
        star_flux(qR, ER, d, SR, Ss, F);
    else
        phys_flux(qR, ER, d, F);
}

void orc_hllc(const double qL[5], const double qR[5], int d, double gamma,
              double F[5])
{
    hllc(qL, qR, d, gamma, 1.0 / (gamma - 1.0), F);
}

/* ------------------------------------------------------------------ */
/* region arrays                                                       */
/* ------------------------------------------------------------------ */

typedef struct {
    int lo[3], hi[3]; /* index range (cells, or faces named by the cell above) */
    int nc;
    double *v;
} fld;

static int fld_make(fld *f, const int lo[3], const int hi[3], int nc)
{
    long long len = nc;
    for (int d = 0; d < 3; ++d) {
        f->lo[d] = lo[d];
        f->hi[d] = hi[d];
        len *= (long long)(hi[d] - lo[d]);
    }
    f->nc = nc;
    f->v = (double *)malloc((size_t)len * sizeof(double));
    return f->v != NULL;
}

static inline double *fat(const fld *f, const int p[3])
{
    long long e0 = f->hi[0] - f->lo[0], e1 = f->hi[1] - f->lo[1];
    long long o = ((long long)(p[2] - f->lo[2]) * e1 + (p[1] - f->lo[1])) * e0 +
                  (p[0] - f->lo[0]);
    return f->v + o * f->nc; /* the components of one point are contiguous */
}

/* iterate p over [lo,hi) with the outer two loops shared among threads */
#define FOR_REGION(lo, hi, p, ...)                                           \
    _Pragma("omp parallel for collapse(2) schedule(static) reduction(|:err)") \
    for (int k_ = (lo)[2]; k_ < (hi)[2]; ++k_)                               \
        for (int j_ = (lo)[1]; j_ < (hi)[1]; ++j_)                           \
            for (int i_ = (lo)[0]; i_ < (hi)[0]; ++i_) {                      \
                int p[3] = {i_, j_, k_};                                      \
                __VA_ARGS__                                                   \
            }

/* Primitive form of a corrected conserved state V; when its density or
 * pressure is not positive the uncorrected state q is kept instead and the
 * fallback error bit is returned. */
static int accept_state(const double V[5], const double q[5], double gm1,
                        double out[5])
{
    double rho = V[0];
    double rinv = 1.0 / rho;
    double u = V[1] * rinv;
    double v = V[2] * rinv;
    double w = V[3] * rinv;
    double ke = (0.5 * rho) * ((u * u + v * v) + w * w);
    double p = gm1 * (V[4] - ke);
    if (rho <= 0.0 || p <= 0.0) {
        for (int m = 0; m < 5; ++m) out[m] = q[m];
        return ORC_ERR_FALLBACK;
    }
    out[0] = rho;
    out[1] = u;
    out[2] = v;
    out[3] = w;
    out[4] = p;
    return 0;
}

int orc_accept_state(const double V[5], const double q[5], double gamma, double out[5])
{
    return accept_state(V, q, gamma - 1.0, out);
}

/* ------------------------------------------------------------------ */
/* one step on an output region                                        */
/* ------------------------------------------------------------------ */

/* One step of the hydro state U and, when nspec > 0, of the nspec partial
 * densities S (rho X_s, same layout, ghosts filled) into Snew. */
static int advance(const double *U, double *Unew, const double *S, double *Snew,
                   int nspec, const orc_box *b, const orc_params *pr, double dt,
                   const int lo[3], const int hi[3], int *errp)
{
    if (!U || !Unew || !pr || !errp || !box_ok(b)) return -1;
    if (nspec < 0 || nspec > ORC_MAX_SPECIES || (nspec > 0 && (!S || !Snew))) return -1;
    for (int d = 0; d < 3; ++d)
        if (lo[d] < 0 || hi[d] > b->n[d] || lo[d] >= hi[d]) return -1;

    long long s[3];
    extents(b, s);
    const long long cs = s[0] * s[1] * s[2];
    const int ng = b->ng;
    const double gamma = pr->gamma, gm1 = gamma - 1.0, igm1 = 1.0 / gm1;
    int err = 0;
    int rc = 0;

    /* shock flattening reads pressures four cells out */
    const int flat = pr->flatten;
    if (flat < 0 || flat > 2 || (flat == 1 && ng < 4)) return -1;
    const int pw = flat == 1 ? 4 : 3;
    int g3lo[3], g3hi[3], g1lo[3], g1hi[3];
    for (int d = 0; d < 3; ++d) {
        g3lo[d] = lo[d] - pw;
        g3hi[d] = hi[d] + pw;
        g1lo[d] = lo[d] - 1;
        g1hi[d] = hi[d] + 1;
    }

    fld prim, fl, qhi[3], qlo[3], F1[3], F2[3][3], F3[3];
    fld X, Xhi[3], Xlo[3], G1[3], G2[3][3], G3[3]; /* species (A9) */
    memset(&X, 0, sizeof X);
    memset(Xhi, 0, sizeof Xhi);
    memset(Xlo, 0, sizeof Xlo);
    memset(G1, 0, sizeof G1);
    memset(G2, 0, sizeof G2);
    memset(G3, 0, sizeof G3);
    memset(&prim, 0, sizeof prim);
    memset(&fl, 0, sizeof fl);
    memset(qhi, 0, sizeof qhi);
    memset(qlo, 0, sizeof qlo);
    memset(F1, 0, sizeof F1);
    memset(F2, 0, sizeof F2);
    memset(F3, 0, sizeof F3);

    /* A1: primitives (and c) on every cell the stencil reaches */
    if (!fld_make(&prim, g3lo, g3hi, 6)) { rc = -2; goto done; }
    FOR_REGION(g3lo, g3hi, p, {
        long long o = cidx(s, ng, p[0], p[1], p[2]);
        double Uc[5];
        for (int c = 0; c < 5; ++c) Uc[c] = U[c * cs + o];
        prim_c(Uc, gamma, gm1, fat(&prim, p));
    })
    ORC_STAGE_MARK(1);

    /* shock-flattening coefficient of every traced cell: the smallest of
     * its three axes' coefficients */
    if (flat) {
        if (!fld_make(&fl, g1lo, g1hi, 1)) { rc = -2; goto done; }
        FOR_REGION(g1lo, g1hi, p, {
            double f = 1.0;
            if (flat == 2) {
                f = 0.0;
            } else {
                for (int d = 0; d < 3; ++d) {
                    double p7[7], un7[7];
                    for (int m = 0; m < 7; ++m) {
                        int r[3] = {p[0], p[1], p[2]};
                        r[d] += m - 3;
                        p7[m] = fat(&prim, r)[4];
                        un7[m] = fat(&prim, r)[1 + d];
                    }
                    f = mn(f, orc_flatten_1d(p7, un7));
                }
            }
            fat(&fl, p)[0] = f;
        })
    }

    /* A3 + A4: traced states at both faces of every cell, each direction,
     * on the cells one beyond the output region; then the half-step
     * gravity kick on the velocity of every face state */
    for (int d = 0; d < 3; ++d) {
        if (!fld_make(&qhi[d], g1lo, g1hi, 5) || !fld_make(&qlo[d], g1lo, g1hi, 5)) {
            rc = -2;
            goto done;
        }
        const double dtdx = dt / b->dx[d];
        FOR_REGION(g1lo, g1hi, p, {
            double q5[5][5];
            for (int m = 0; m < 5; ++m) {
                int r[3] = {p[0], p[1], p[2]};
                r[d] += m - 2;
                const double *qq = fat(&prim, r);
                for (int v = 0; v < 5; ++v) q5[m][v] = qq[v];
            }
            double c = fat(&prim, p)[5];
            double *hiq = fat(&qhi[d], p), *loq = fat(&qlo[d], p);
            trace_cell(q5, c, d, dtdx, flat ? fat(&fl, p)[0] : 1.0, hiq, loq);
            for (int e = 0; e < 3; ++e)
                if (pr->grav[e] != 0.0) {
                    hiq[1 + e] = hiq[1 + e] + (0.5 * dt) * pr->grav[e];
                    loq[1 + e] = loq[1 + e] + (0.5 * dt) * pr->grav[e];
                }
        })
    }

    ORC_STAGE_MARK(4);

    /* A5: round-1 fluxes at d-faces; face f lies between cells f-1 and f */
    for (int d = 0; d < 3; ++d) {
        int flo[3], fhi[3];
        for (int e = 0; e < 3; ++e) {
            flo[e] = e == d ? lo[e] : lo[e] - 1;
            fhi[e] = e == d ? hi[e] + 1 : hi[e] + 1;
        }
        if (!fld_make(&F1[d], flo, fhi, 5)) { rc = -2; goto done; }
        FOR_REGION(flo, fhi, p, {
            int l[3] = {p[0], p[1], p[2]};
            l[d] -= 1;
            hllc(fat(&qhi[d], l), fat(&qlo[d], p), d, gamma, igm1, fat(&F1[d], p));
        })
    }

    ORC_STAGE_MARK(5);

    /* A6: corner coupling.  F2[t][s] is the flux through t-faces of the
     * states traced along t and corrected by dt/3 of the round-1 s-flux
     * difference across the cell they came from. */
    for (int t = 0; t < 3; ++t)
        for (int sd = 0; sd < 3; ++sd) {
            if (sd == t) continue;
            const int d = 3 - t - sd; /* the third axis */
            int flo[3], fhi[3];
            flo[t] = lo[t];
            fhi[t] = hi[t] + 1;
            flo[sd] = lo[sd];
            fhi[sd] = hi[sd];
            flo[d] = lo[d] - 1;
            fhi[d] = hi[d] + 1;
            if (!fld_make(&F2[t][sd], flo, fhi, 5)) { rc = -2; goto done; }
            const double fac = dt / (3.0 * b->dx[sd]);
            FOR_REGION(flo, fhi, p, {
                int cl[3] = {p[0], p[1], p[2]}, cr[3] = {p[0], p[1], p[2]};
                cl[t] -= 1;
                double qc[2][5];
                for (int side = 0; side < 2; ++side) {
                    const int *c = side ? cr : cl;
                    int cu[3] = {c[0], c[1], c[2]};
                    cu[sd] += 1;
                    const double *Flo = fat(&F1[sd], c), *Fhi = fat(&F1[sd], cu);
                    const double *q = side ? fat(&qlo[t], c) : fat(&qhi[t], c);
                    double Uq[5], V[5];
                    cons_of(q, igm1, Uq);
                    for (int v = 0; v < 5; ++v)
                        V[v] = Uq[v] - fac * (Fhi[v] - Flo[v]);
                    err |= accept_state(V, q, gm1, qc[side]);
                }
                hllc(qc[0], qc[1], t, gamma, igm1, fat(&F2[t][sd], p));
            })
        }

    ORC_STAGE_MARK(6);

    /* A7: final states, corrected by dt/2 of both round-2 transverse flux
     * differences, and the round-3 fluxes at d-faces of the output region */
    for (int d = 0; d < 3; ++d) {
        int t1, t2;
        transverse(d, &t1, &t2);
        int flo[3], fhi[3];
        for (int e = 0; e < 3; ++e) {
            flo[e] = lo[e];
            fhi[e] = e == d ? hi[e] + 1 : hi[e];
        }
        if (!fld_make(&F3[d], flo, fhi, 5)) { rc = -2; goto done; }
        const double f1 = dt / (2.0 * b->dx[t1]);
        const double f2 = dt / (2.0 * b->dx[t2]);
        FOR_REGION(flo, fhi, p, {
            int cl[3] = {p[0], p[1], p[2]}, cr[3] = {p[0], p[1], p[2]};
            cl[d] -= 1;
            double qf[2][5];
            for (int side = 0; side < 2; ++side) {
                const int *c = side ? cr : cl;
                int c1[3] = {c[0], c[1], c[2]}, c2[3] = {c[0], c[1], c[2]};
                c1[t1] += 1;
                c2[t2] += 1;
                const double *A0 = fat(&F2[t1][t2], c), *A1 = fat(&F2[t1][t2], c1);
                const double *B0 = fat(&F2[t2][t1], c), *B1 = fat(&F2[t2][t1], c2);
                const double *q = side ? fat(&qlo[d], c) : fat(&qhi[d], c);
                double Uq[5], V[5];
                cons_of(q, igm1, Uq);
                for (int v = 0; v < 5; ++v)
                    V[v] = (Uq[v] - f1 * (A1[v] - A0[v])) - f2 * (B1[v] - B0[v]);
                err |= accept_state(V, q, gm1, qf[side]);
            }
            hllc(qf[0], qf[1], d, gamma, igm1, fat(&F3[d], p));
        })
    }

    ORC_STAGE_MARK(7);

    /* A8: conservative update and time-centred gravity source */
    {
        const double dtdx[3] = {dt / b->dx[0], dt / b->dx[1], dt / b->dx[2]};
        FOR_REGION(lo, hi, p, {
            long long o = cidx(s, ng, p[0], p[1], p[2]);
            double Un[5], Us[5];
            for (int v = 0; v < 5; ++v) {
                int px[3] = {p[0] + 1, p[1], p[2]};
                int py[3] = {p[0], p[1] + 1, p[2]};
                int pz[3] = {p[0], p[1], p[2] + 1};
                double du = dtdx[0] * (fat(&F3[0], px)[v] - fat(&F3[0], p)[v]);
                du = du + dtdx[1] * (fat(&F3[1], py)[v] - fat(&F3[1], p)[v]);
                du = du + dtdx[2] * (fat(&F3[2], pz)[v] - fat(&F3[2], p)[v]);
                Un[v] = U[v * cs + o];
                Us[v] = Un[v] - du;
            }
            for (int e = 0; e < 3; ++e)
                if (pr->grav[e] != 0.0) {
                    double hg = (0.5 * dt) * pr->grav[e];
                    double mnew = Us[1 + e] + hg * (Un[0] + Us[0]);
                    Us[4] = Us[4] + hg * (Un[1 + e] + mnew);
                    Us[1 + e] = mnew;
                }
            double qn[6];
            prim_c(Us, gamma, gm1, qn);
            for (int v = 0; v < 5; ++v) {
                if (!isfinite(Us[v])) err |= ORC_ERR_NONFINITE;
                Unew[v * cs + o] = Us[v];
            }
            if (Us[0] <= 0.0) err |= ORC_ERR_RHO;
            if (qn[4] <= 0.0) err |= ORC_ERR_P;
        })
    }

    ORC_STAGE_MARK(8);

    /* A9: passively advected species.  A species is carried by the gas: its
     * flux through a face is the mass flux there times the mass fraction X
     * of the cell the mass comes from (the face state on the side the mass
     * flux leaves, the low side when it is zero).  Its face values are traced
     * like a transverse velocity -- it changes only across the contact wave
     * -- and corrected like the density: X of a corrected state is the
     * corrected partial density over the corrected density, each formed from
     * the same flux differences, the traced X kept where that density is not
     * positive. */
    if (nspec > 0) {
        const int ns = nspec;
        if (!fld_make(&X, g3lo, g3hi, ns)) { rc = -2; goto done; }
        FOR_REGION(g3lo, g3hi, p, {
            long long o = cidx(s, ng, p[0], p[1], p[2]);
            const double rho = fat(&prim, p)[0];
            for (int c = 0; c < ns; ++c) fat(&X, p)[c] = S[c * cs + o] / rho;
        })
        for (int d = 0; d < 3; ++d) {
            if (!fld_make(&Xhi[d], g1lo, g1hi, ns) || !fld_make(&Xlo[d], g1lo, g1hi, ns)) {
                rc = -2;
                goto done;
            }
            const double dtdx = dt / b->dx[d];
            FOR_REGION(g1lo, g1hi, p, {
                const double un = fat(&prim, p)[1 + d], c = fat(&prim, p)[5];
                const double f = flat ? fat(&fl, p)[0] : 1.0;
                for (int sp = 0; sp < ns; ++sp) {
                    double a[5], aL, aR;
                    for (int m = 0; m < 5; ++m) {
                        int r[3] = {p[0], p[1], p[2]};
                        r[d] += m - 2;
                        a[m] = fat(&X, r)[sp];
                    }
                    ppm_faces(a, f, &aL, &aR);
                    fat(&Xhi[d], p)[sp] = edge_hi(a[2], aL, aR, un > 0.0 ? un : un + c, dtdx);
                    fat(&Xlo[d], p)[sp] = edge_lo(a[2], aL, aR, un < 0.0 ? un : un - c, dtdx);
                }
            })
        }
        /* round 1 */
        for (int d = 0; d < 3; ++d) {
            if (!fld_make(&G1[d], F1[d].lo, F1[d].hi, ns)) { rc = -2; goto done; }
            FOR_REGION(F1[d].lo, F1[d].hi, p, {
                int l[3] = {p[0], p[1], p[2]};
                l[d] -= 1;
                const double F = fat(&F1[d], p)[0];
                for (int sp = 0; sp < ns; ++sp)
                    fat(&G1[d], p)[sp] = F * (F >= 0.0 ? fat(&Xhi[d], l)[sp] : fat(&Xlo[d], p)[sp]);
            })
        }
        /* round 2: corner-coupled states (dt/3 of one transverse difference) */
        for (int t = 0; t < 3; ++t)
            for (int sd = 0; sd < 3; ++sd) {
                if (sd == t) continue;
                const fld *Fm = &F2[t][sd];
                if (!fld_make(&G2[t][sd], Fm->lo, Fm->hi, ns)) { rc = -2; goto done; }
                const double fac = dt / (3.0 * b->dx[sd]);
                FOR_REGION(Fm->lo, Fm->hi, p, {
                    int cl[3] = {p[0], p[1], p[2]}, cr[3] = {p[0], p[1], p[2]};
                    cl[t] -= 1;
                    double xc[2][ORC_MAX_SPECIES];
                    for (int side = 0; side < 2; ++side) {
                        const int *c = side ? cr : cl;
                        int cu[3] = {c[0], c[1], c[2]};
                        cu[sd] += 1;
                        const double rq = side ? fat(&qlo[t], c)[0] : fat(&qhi[t], c)[0];
                        const double *xq = side ? fat(&Xlo[t], c) : fat(&Xhi[t], c);
                        const double den = rq - fac * (fat(&F1[sd], cu)[0] - fat(&F1[sd], c)[0]);
                        for (int sp = 0; sp < ns; ++sp) {
                            const double num =
                                rq * xq[sp] - fac * (fat(&G1[sd], cu)[sp] - fat(&G1[sd], c)[sp]);
                            xc[side][sp] = den > 0.0 ? num / den : xq[sp];
                        }
                    }
                    const double F = fat(Fm, p)[0];
                    for (int sp = 0; sp < ns; ++sp)
                        fat(&G2[t][sd], p)[sp] = F * (F >= 0.0 ? xc[0][sp] : xc[1][sp]);
                })
            }
        /* round 3: final states (dt/2 of both round-2 transverse differences) */
        for (int d = 0; d < 3; ++d) {
            int t1, t2;
            transverse(d, &t1, &t2);
            if (!fld_make(&G3[d], F3[d].lo, F3[d].hi, ns)) { rc = -2; goto done; }
            const double f1 = dt / (2.0 * b->dx[t1]);
            const double f2 = dt / (2.0 * b->dx[t2]);
            FOR_REGION(F3[d].lo, F3[d].hi, p, {
                int cl[3] = {p[0], p[1], p[2]}, cr[3] = {p[0], p[1], p[2]};
                cl[d] -= 1;
                double xf[2][ORC_MAX_SPECIES];
                for (int side = 0; side < 2; ++side) {
                    const int *c = side ? cr : cl;
                    int c1[3] = {c[0], c[1], c[2]}, c2[3] = {c[0], c[1], c[2]};
                    c1[t1] += 1;
                    c2[t2] += 1;
                    const double rq = side ? fat(&qlo[d], c)[0] : fat(&qhi[d], c)[0];
                    const double *xq = side ? fat(&Xlo[d], c) : fat(&Xhi[d], c);
                    const double den = (rq - f1 * (fat(&F2[t1][t2], c1)[0] - fat(&F2[t1][t2], c)[0])) -
                                       f2 * (fat(&F2[t2][t1], c2)[0] - fat(&F2[t2][t1], c)[0]);
                    for (int sp = 0; sp < ns; ++sp) {
                        const double num =
                            (rq * xq[sp] - f1 * (fat(&G2[t1][t2], c1)[sp] - fat(&G2[t1][t2], c)[sp])) -
                            f2 * (fat(&G2[t2][t1], c2)[sp] - fat(&G2[t2][t1], c)[sp]);
                        xf[side][sp] = den > 0.0 ? num / den : xq[sp];
                    }
                }
                const double F = fat(&F3[d], p)[0];
                for (int sp = 0; sp < ns; ++sp)
                    fat(&G3[d], p)[sp] = F * (F >= 0.0 ? xf[0][sp] : xf[1][sp]);
            })
        }
        /* conservative update of the partial densities */
        {
            const double dtdx[3] = {dt / b->dx[0], dt / b->dx[1], dt / b->dx[2]};
            FOR_REGION(lo, hi, p, {
                long long o = cidx(s, ng, p[0], p[1], p[2]);
                int px[3] = {p[0] + 1, p[1], p[2]};
                int py[3] = {p[0], p[1] + 1, p[2]};
                int pz[3] = {p[0], p[1], p[2] + 1};
                for (int sp = 0; sp < ns; ++sp) {
                    double du = dtdx[0] * (fat(&G3[0], px)[sp] - fat(&G3[0], p)[sp]);
                    du = du + dtdx[1] * (fat(&G3[1], py)[sp] - fat(&G3[1], p)[sp]);
                    du = du + dtdx[2] * (fat(&G3[2], pz)[sp] - fat(&G3[2], p)[sp]);
                    const double v = S[sp * cs + o] - du;
                    if (!isfinite(v)) err |= ORC_ERR_NONFINITE;
                    Snew[sp * cs + o] = v;
                }
            })
        }
    }

done:
    free(prim.v);
    free(fl.v);
    free(X.v);
    for (int d = 0; d < 3; ++d) {
        free(qhi[d].v);
        free(qlo[d].v);
        free(F1[d].v);
        free(F3[d].v);
        free(Xhi[d].v);
        free(Xlo[d].v);
        free(G1[d].v);
        free(G3[d].v);
        for (int e = 0; e < 3; ++e) {
            free(F2[d][e].v);
            free(G2[d][e].v);
        }
    }
    *errp |= err;
    return rc;
}

int orc_advance_region(const double *U, double *Unew, const orc_box *b,
                       const orc_params *pr, double dt, const int lo[3],
                       const int hi[3], int *errp)
{
    return advance(U, Unew, NULL, NULL, 0, b, pr, dt, lo, hi, errp);
}

int orc_advance_region_species(const double *U, double *Unew, const double *S,
                               double *Snew, int nspec, const orc_box *b,
                               const orc_params *pr, double dt, const int lo[3],
                               const int hi[3], int *errp)
{
    if (nspec < 1) return -1;
    return advance(U, Unew, S, Snew, nspec, b, pr, dt, lo, hi, errp);
}

int orc_advance_box(const double *U, double *Unew, const orc_box *b,
                    const orc_params *p, double dt, int *err)
{
    if (!b) return -1;
    int lo[3] = {0, 0, 0};
    return orc_advance_region(U, Unew, b, p, dt, lo, b->n, err);
}
