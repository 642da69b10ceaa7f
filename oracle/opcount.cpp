// opcount.cpp -- operation-counting build of the oracle (test infrastructure).
//
// The oracle's C source is compiled as C++ with every `double` replaced by a
// scalar type whose arithmetic operators count themselves.  The count of one
// cell-update is the difference between advancing an N x N x N output region
// and an (N+1) x N x N one, divided by N*N: every stage's region grows by
// exactly one slab of cells, so the halo work cancels.  Counted: + and -
// (add), * (mul), / (div), sqrt, and comparisons (cmp, not flops); unary
// minus, fabs and copysign are sign operations and are not counted.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

struct OpCounts {
    long long add, mul, div, sqrt_, cmp;
};
static OpCounts g_ops;
static OpCounts g_mark[9];  // counts at the end of each marked stage

static void stage_mark(int k) { g_mark[k] = g_ops; }
#define ORC_STAGE_MARK(k) stage_mark(k)

struct D {
    double v;
    D() : v(0.0) {}
    D(double x) : v(x) {}
};
static inline D operator+(D a, D b) { g_ops.add++; return D(a.v + b.v); }
static inline D operator-(D a, D b) { g_ops.add++; return D(a.v - b.v); }
static inline D operator*(D a, D b) { g_ops.mul++; return D(a.v * b.v); }
static inline D operator/(D a, D b) { g_ops.div++; return D(a.v / b.v); }
static inline D operator-(D a) { return D(-a.v); }
static inline bool operator<(D a, D b) { g_ops.cmp++; return a.v < b.v; }
static inline bool operator>(D a, D b) { g_ops.cmp++; return a.v > b.v; }
static inline bool operator<=(D a, D b) { g_ops.cmp++; return a.v <= b.v; }
static inline bool operator>=(D a, D b) { g_ops.cmp++; return a.v >= b.v; }
static inline bool operator!=(D a, D b) { return a.v != b.v; }
static inline bool operator==(D a, D b) { return a.v == b.v; }
static inline D sqrt(D a) { g_ops.sqrt_++; return D(::sqrt(a.v)); }
static inline D fabs(D a) { return D(::fabs(a.v)); }
static inline D copysign(D a, D b) { return D(::copysign(a.v, b.v)); }
static inline bool isfinite(D a) { return std::isfinite(a.v); }
static inline bool operator!(D a) { return !a.v; }

#undef _OPENMP
#define double D
#include "hydro_oracle.c"
#undef double

extern "C" {

/* Operation counts of one orc_advance_region call on the output region
 * [0,N)^3 of the box (U with ghosts filled): ops[k] = (add, mul, div, sqrt,
 * cmp) spent in the stages that end at mark k (1: primitives, 4: PPM +
 * tracing, 5: round-1 fluxes, 6: corner coupling + round 2, 7: final states
 * + round 3, 8: update); rows 0, 2, 3 are unused. */
int orc_opcount_region(const double *U, const orc_box *b, const orc_params *p, double dt,
                       int N, double ops[9][5])
{
    double *Un = (double *)malloc(sizeof(double) * orc_state_elems(b));
    if (!Un) return -2;
    int err = 0;
    int lo[3] = {0, 0, 0};
    int hi[3] = {N, N, N};
    memset(&g_ops, 0, sizeof g_ops);
    memset(g_mark, 0, sizeof g_mark);
    int rc = orc_advance_region((const D *)U, (D *)Un, b, p, D(dt), lo, hi, &err);
    free(Un);
    OpCounts prev = {0, 0, 0, 0, 0};
    for (int k = 0; k < 9; ++k) {
        for (int v = 0; v < 5; ++v) ops[k][v] = 0.0;
        if (k != 1 && k < 4) continue;
        const OpCounts &m = g_mark[k];
        ops[k][0] = (double)(m.add - prev.add);
        ops[k][1] = (double)(m.mul - prev.mul);
        ops[k][2] = (double)(m.div - prev.div);
        ops[k][3] = (double)(m.sqrt_ - prev.sqrt_);
        ops[k][4] = (double)(m.cmp - prev.cmp);
        prev = m;
    }
    return rc;
}
}
