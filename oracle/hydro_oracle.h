/*
 * hydro_oracle.h -- FP64 CPU oracle for the unsplit CTU-PPM + HLLC advance of
 * a gamma-law gas on one box with ghost cells.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the benchmark's CPU-baseline leg can check the GPU library
 * against a plain, slow, obviously correct implementation.  No product code
 * may link, load or call it.
 *
 * What is computed.  The paper (Katz et al. 2020, "Preparing Nuclear
 * Astrophysics for Exascale") describes the hydro only in outline: a slope
 * stencil over neighbouring zones that reconstructs a polynomial (Sec. III),
 * a hydro + EOS coupling exercised by the Sedov test (Sec. IV-A), throughput
 * in zones per microsecond (Sec. IV) and a timestep proportional to the zone
 * width (Sec. V).  The scheme itself is the one of the paper's Castro
 * reference (bibliography entry CastroI): Colella & Woodward 1984 PPM with
 * characteristic tracing, the 3-D corner transport upwind (CTU) coupling of
 * Colella 1990 / Saltzman 1994, and an HLLC Riemann solver (Toro, Spruce &
 * Speares 1994) with Davis 1988 wave speeds.  Every point the paper leaves
 * open is fixed by one written reading; the readings are listed in the
 * design notes of this repository.
 *
 * Data layout (shared convention with the GPU library, but no shared code):
 *   a box has n[3] valid cells and ng ghost layers; one component occupies
 *   s0*s1*s2 doubles with s_d = n_d + 2*ng, x fastest, then y, then z;
 *   the five components (rho, rho*u, rho*v, rho*w, E) follow one another
 *   (structure of arrays, the Fab order of Sec. II).  Cell (i,j,k) with
 *   -ng <= i < n0+ng etc. lives at ((k+ng)*s1 + (j+ng))*s0 + (i+ng).
 *
 * Arithmetic contract: IEEE binary64, no contraction of a*b+c into an FMA,
 * correctly rounded division and square root, expressions evaluated in the
 * parenthesisation written in the source.  Build with -ffp-contract=off and
 * without -ffast-math.
 */
#ifndef HYDRO_ORACLE_H
#define HYDRO_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BC_PERIODIC = 0, ORC_BC_OUTFLOW = 1, ORC_BC_REFLECT = 2 };

/* error bits (sticky OR) */
enum {
    ORC_ERR_NONFINITE = 1, /* an updated value is NaN or Inf            */
    ORC_ERR_RHO = 2,       /* updated density <= 0                      */
    ORC_ERR_P = 4,         /* updated pressure <= 0                     */
    ORC_ERR_FALLBACK = 8   /* a corrected transverse state was rejected */
};

typedef struct {
    int n[3];      /* valid cells per axis, >= 1 (>= ng on periodic/reflect axes) */
    int ng;        /* ghost layers, >= 3 */
    double dx[3];  /* cell widths */
    int bc_lo[3];  /* ORC_BC_* at the low face of each axis */
    int bc_hi[3];  /* ORC_BC_* at the high face of each axis */
} orc_box;

typedef struct {
    double gamma;   /* ratio of specific heats, > 1 */
    double cfl;     /* Courant number, 0 < cfl <= 1 */
    double grav[3]; /* constant gravitational acceleration */
    int flatten;    /* shock flattening: 0 off, 1 on (needs ng >= 4), 2 full
                       flattening of every cell (coefficient 0; a test mode) */
} orc_params;

#define ORC_MAX_SPECIES 8

/* Number of doubles of one state array (all five components, with ghosts). */
long long orc_state_elems(const orc_box *b);

/* Fill every ghost cell of U from its valid cells and the boundary kinds:
 * x ghosts over the valid (j,k) first, then y ghosts over all i, then z
 * ghosts over all (i,j), so edges and corners are defined.  Returns 0, or -1
 * for an invalid box. */
int orc_fill_ghosts(double *U, const orc_box *b);

/* CFL timestep of the valid cells of U (ghosts are not read):
 * dt = cfl * min_d (dx_d / max_cells(|u_d| + c)).  Returns 0 or -1. */
int orc_estimate_dt(const double *U, const orc_box *b, const orc_params *p,
                    double *dt);

/* One CTU step of length dt.  U must have its ghosts filled.  The new state
 * is written to Unew on the output region lo <= (i,j,k) < hi (valid-cell
 * coordinates, 0 <= lo < hi <= n); nothing else of Unew is touched.  The
 * result on a cell does not depend on the region it was computed in.  Error
 * bits are OR-ed into *err.  Returns 0, -1 for invalid arguments, -2 when
 * out of memory. */
int orc_advance_region(const double *U, double *Unew, const orc_box *b,
                       const orc_params *p, double dt, const int lo[3],
                       const int hi[3], int *err);

/* orc_advance_region with nspec passively advected species as well
 * (1 <= nspec <= ORC_MAX_SPECIES): S holds their partial densities rho X_s
 * in the state layout (nspec components, ghosts filled); Snew receives them
 * on the output region.  U and Unew are as in orc_advance_region, whose
 * results this function reproduces bit for bit. */
int orc_advance_region_species(const double *U, double *Unew, const double *S,
                               double *Snew, int nspec, const orc_box *b,
                               const orc_params *p, double dt, const int lo[3],
                               const int hi[3], int *err);

/* Ghost fill of nspec species components, by the rules of orc_fill_ghosts
 * without any sign flip.  Returns 0 or -1. */
int orc_fill_ghosts_species(double *S, int nspec, const orc_box *b);

/* orc_advance_region over the whole valid box. */
int orc_advance_box(const double *U, double *Unew, const orc_box *b,
                    const orc_params *p, double dt, int *err);

/* ---- the scheme's pieces, exported so tests can pin each of them ---- */

/* Limited PPM parabola of cell i from a[i-2..i+2] (a5[0..4]):
 * out[0] = a_L (value at the low face), out[1] = a_R (high face). */
void orc_ppm_parabola(const double a5[5], double out[2]);

/* The same with the shock-flattening coefficient f of the cell (1: none). */
void orc_ppm_parabola_flat(const double a5[5], double f, double out[2]);

/* Shock-flattening coefficient of the centre cell of a 7-cell pencil along
 * one axis: p7[m], un7[m] = pressure and velocity along the axis of cell
 * i+m-3.  1 means no flattening. */
double orc_flatten_1d(const double p7[7], const double un7[7]);

/* Averages of the cell's parabola over the domain of dependence of a wave of
 * speed lam over dtdx = dt/dx: *Ip toward the high face, *Im toward the low
 * face. */
void orc_ppm_integrals(const double a5[5], double lam, double dtdx, double *Ip,
                       double *Im);

/* Traced face states of one cell along axis d from the primitive stencil
 * q5[m][v] = primitive v (rho,u,v,w,p) of cell i+m-2 along d, m = 0..4.
 * qhi = state at the high face, qlo = state at the low face, both
 * (rho,u,v,w,p), without gravity. */
void orc_trace(const double q5[5][5], int d, double gamma, double dtdx,
               double qhi[5], double qlo[5]);

/* HLLC flux through a face normal to axis d between primitive states qL,qR
 * (rho,u,v,w,p); F = (mass, x-, y-, z-momentum, energy). */
void orc_hllc(const double qL[5], const double qR[5], int d, double gamma,
              double F[5]);

/* Primitive (rho,u,v,w,p) <-> conserved (rho,rho u,rho v,rho w,E). */
void orc_prim_of_cons(const double U[5], double gamma, double q[5]);
void orc_cons_of_prim(const double q[5], double gamma, double U[5]);

/* The rule that accepts or rejects a transverse-corrected state: out = the
 * primitive form (rho,u,v,w,p) of the corrected conserved state V when its
 * density and pressure are both positive, else out = q (the uncorrected
 * primitive state) and the return value is ORC_ERR_FALLBACK (0 otherwise).
 * The corner (dt/3) and final (dt/2) stages of the step apply exactly this
 * function to every corrected face state. */
int orc_accept_state(const double V[5], const double q[5], double gamma, double out[5]);

/* Number of OpenMP threads the oracle runs on (1 when built without it). */
int orc_num_threads(void);

/* Threads of the oracle's later calls made from the calling host thread
 * (several host threads may each advance their own boxes at once). */
void orc_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
