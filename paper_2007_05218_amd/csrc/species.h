// species.h -- passively advected species: ns mass fractions X_s carried by
// the gas, stored as partial densities rho X_s (their own array, the state
// layout, ns components).
//
// A species moves with the gas: through every face its flux is the mass
// flux of the same Riemann solve times the mass fraction of the side the
// mass comes from (the face state on the side the flux leaves; the low side
// when the flux is zero).  So the species pass needs, from the hydro step,
// the traced densities (the trace kernel's workspace) and the mass fluxes
// of all twelve solve families (exported by the flux kernel), and repeats
// the three rounds of the unsplit step for X alone: one fused, z-marching
// kernel per box tile and species (species_fused.h).  This file holds the
// pass's arguments (one box or a batch) and the species ghost fill.
#pragma once

namespace {

constexpr int kMaxSpecies = 8;

// Species workspace of a box: the 12 mass-flux fields of the gas step
// (doubles, each field mf_stride long, faces named by the cell above over
// the index box [-1, n] per axis), in the order F1 x, y, z; F2 (x|y), (x|z),
// (y|x), (y|z), (z|x), (z|y); F3 x, y, z.
struct SpArgs {
    Geo g;
    const double *U;    // gas state (ghosts filled)
    const double *S;    // partial densities (ghosts filled)
    double *Sn;         // new partial densities (valid cells written)
    const char *ws;     // the hydro workspace (traced states, flattening)
    const double *mf;   // mass-flux export
    const double *dt;
    int ns;
    int flat;           // flattening coefficients present in the workspace
    long long E;        // field stride (doubles)
    double gamma;
};

// A batch of boxes (nb >= 1; nb == 0: the single box of SpArgs).  Each
// species stage's blocks (the fused pass: tiles) are dealt to the boxes by
// the plan's prefix sums; box b's mass fluxes start 12 * epre[b] doubles
// into the species workspace (epre: the prefix of the boxes' field
// strides).
struct SpBatch {
    int nb;
    const unsigned *pre;  // this stage's block prefix, nb+1 entries
    const Geo *geos;
    const double *const *Us;
    const double *const *Ss;
    double *const *Sns;
    const char *ws;
    const long long *wsoff;  // doubles from the workspace base
    double *sws;
    const long long *epre;
    const double *dts;
    int dt_stride;
};

// this block's box (A rewritten for it) and block index within the box
__device__ __forceinline__ long long sp_box(SpArgs &A, const SpBatch &B)
{
    if (B.nb == 0) return blockIdx.x;
    int lo = 0, hi = B.nb;
    const unsigned x = blockIdx.x;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (B.pre[mid] <= x) lo = mid;
        else hi = mid;
    }
    const int b = lo;
    A.g = B.geos[b];
    A.U = B.Us ? B.Us[b] : nullptr;
    A.S = B.Ss ? B.Ss[b] : nullptr;
    A.Sn = B.Sns ? B.Sns[b] : nullptr;
    A.ws = B.ws ? B.ws + B.wsoff[b] * (long long)sizeof(double) : nullptr;
    A.E = mf_stride(A.g.n[0], A.g.n[1], A.g.n[2]);
    if (B.sws) A.mf = B.sws + 12 * B.epre[b];
    A.dt = B.dts ? B.dts + (long long)b * B.dt_stride : nullptr;
    return (long long)(x - B.pre[b]);
}

// ghost cells of the species array: the gas's boundary rules without any
// sign flip (each ghost cell copies the cell its per-axis mapping names)
__global__ void __launch_bounds__(kBlock) k_sp_fill(SpArgs A, SpBatch B)
{
    long long t = sp_box(A, B) * kBlock + threadIdx.x;
    const Geo &g = A.g;
    double *S = const_cast<double *>(A.S);
    const int ns = A.ns;
    if (t >= g.cs) return;
    const int i = (int)(t % g.s[0]) - g.ng;
    const long long r = t / g.s[0];
    const int j = (int)(r % g.s[1]) - g.ng;
    const int k = (int)(r / g.s[1]) - g.ng;
    const bool gi = i < 0 || i >= g.n[0], gj = j < 0 || j >= g.n[1], gk = k < 0 || k >= g.n[2];
    if (!gi && !gj && !gk) return;
    int flip;
    const int si = gi ? ghost_src(i, g.n[0], g.bc_lo[0], g.bc_hi[0], flip) : i;
    const int sj = gj ? ghost_src(j, g.n[1], g.bc_lo[1], g.bc_hi[1], flip) : j;
    const int sk = gk ? ghost_src(k, g.n[2], g.bc_lo[2], g.bc_hi[2], flip) : k;
    const long long src = cell(g, si, sj, sk);
    for (int s = 0; s < ns; ++s) S[s * g.cs + t] = S[s * g.cs + src];
}

}  // namespace
