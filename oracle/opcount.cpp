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

/* ops[5] = add, mul, div, sqrt, cmp of one cell-update, interior cells of a
 * box with uniform-ish data from U (ghosts filled), region sizes N and N+1. */
int orc_opcount_cell(const double *U, const orc_box *b, const orc_params *p,
                     double dt, int N, double ops[5])
{
    double *Un = (double *)malloc(sizeof(double) * orc_state_elems(b));
    if (!Un) return -2;
    int err = 0;
    int lo[3] = {0, 0, 0};
    int hiA[3] = {N, N, N}, hiB[3] = {N + 1, N, N};
    OpCounts a, c;
    memset(&g_ops, 0, sizeof g_ops);
    int rc = orc_advance_region((const D *)U, (D *)Un, b, p, D(dt), lo, hiA, &err);
    a = g_ops;
    memset(&g_ops, 0, sizeof g_ops);
    rc |= orc_advance_region((const D *)U, (D *)Un, b, p, D(dt), lo, hiB, &err);
    c = g_ops;
    free(Un);
    double nn = (double)N * N;
    ops[0] = (c.add - a.add) / nn;
    ops[1] = (c.mul - a.mul) / nn;
    ops[2] = (c.div - a.div) / nn;
    ops[3] = (c.sqrt_ - a.sqrt_) / nn;
    ops[4] = (c.cmp - a.cmp) / nn;
    return rc;
}
}
