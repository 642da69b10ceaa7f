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
// the three rounds of the unsplit step for X alone:
//   k_sp_trace   X = rho X / rho; each cell's limited parabola of X along
//                each axis (flattened like the gas), averaged toward each
//                face like a transverse velocity: over the contact wave when
//                it moves toward the face, else over the outermost wave;
//   k_sp_corner  corner-coupled X of each traced state: the corrected
//                partial density over the corrected density, both
//                corrected by dt/3 of the round-1 flux difference across the
//                cell along one transverse axis (the traced X where that
//                density is not positive); the round-2 species fluxes;
//   k_sp_final   final X (dt/2 of both round-2 transverse differences);
//                the round-3 species fluxes;
//   k_sp_update  the conservative update of rho X.
// One thread per cell or face of the index box [-1, n] per axis (faces
// named by the cell above); every stage reads its inputs from HBM.
#pragma once

namespace {

constexpr int kMaxSpecies = 8;
// parts per cell or face of the trace, corner and final stages (all axes,
// one traced axis with its two flux families, one axis)
constexpr int kSpTraceParts = 1, kSpCornerParts = 3, kSpFinalParts = 3;

// Species-pass arrays (doubles, each field mf_stride long, in order):
// 12 mass-flux fields | traced X: 6 ns (axis, high/low, species) |
// round-2 species fluxes: 6 ns (family, species) | round-3: 3 ns
struct SpArgs {
    Geo g;
    const double *U;    // gas state (ghosts filled)
    const double *S;    // partial densities (ghosts filled)
    double *Sn;         // new partial densities (valid cells written)
    const char *ws;     // the hydro workspace (traced states, flattening)
    const double *mf;   // mass-flux export
    double *Xt, *G2, *G3;
    const double *dt;
    int ns;
    int flat;           // flattening coefficients present in the workspace
    long long E;        // field stride (doubles)
    double gamma;
};

// A batch of boxes (nb >= 1; nb == 0: the single box of SpArgs).  Each
// species stage's blocks are dealt to the boxes by the plan's prefix sums;
// box b's species arrays start (12 + 15 ns) * epre[b] doubles into the
// species workspace (epre: the prefix of the boxes' field strides).
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
    if (B.sws) {
        A.mf = B.sws + (12 + 15 * (long long)A.ns) * B.epre[b];
        A.Xt = const_cast<double *>(A.mf) + 12 * A.E;
        A.G2 = A.Xt + 6 * A.ns * A.E;
        A.G3 = A.G2 + 6 * A.ns * A.E;
    }
    A.dt = B.dts ? B.dts + (long long)b * B.dt_stride : nullptr;
    return (long long)(x - B.pre[b]);
}

// component a (0, 1, 2) of a 3-vector by selects, not by indexing (a
// runtime index into the box's geometry would put it in scratch memory)
template <typename T>
__device__ __forceinline__ T sel3(const T (&v)[3], int a)
{
    return a == 0 ? v[0] : (a == 1 ? v[1] : v[2]);
}

__device__ __forceinline__ bool sp_decode(const SpArgs &A, long long t, int &x, int &y, int &z)
{
    const int e0 = A.g.n[0] + 2, e1 = A.g.n[1] + 2, e2 = A.g.n[2] + 2;
    if (t >= (long long)e0 * e1 * e2) return false;
    x = (int)(t % e0) - 1;
    t /= e0;
    y = (int)(t % e1) - 1;
    z = (int)(t / e1) - 1;
    return true;
}

__device__ __forceinline__ long long sp_idx(const SpArgs &A, int x, int y, int z)
{
    return mf_index(A.g.n[0], A.g.n[1], x, y, z);
}

// traced density of cell (x, y, z) along axis d: high face (side 0) or low
// face (side 1), from the hydro workspace
__device__ __forceinline__ double sp_rho_traced(const SpArgs &A, int d, int side, int x, int y,
                                                int z)
{
    WS w;
    w.base = const_cast<char *>(A.ws);
    w.pitch = ws_pitch(A.g.n[0], A.g.n[1]);
    w.nxb = ws_xblocks(A.g.n[0]);
    return ws_ld(w.plane(z), w.off(x, y), side ? QLO(d, 0) : QHI(d, 0));
}

// Block b (within its box) of a stage with nf parts per face (flux families
// or axes): part (b / 8) % nf of cell block ((b / 8) / nf) * 8 + b % 8.  Blocks are dealt to
// the 8 XCDs round-robin (b % 8), so the nf parts of one cell block run on
// one XCD, close in time, and share what they read in its L2.
__device__ __forceinline__ long long sp_part(long long b, int nf, int &part)
{
    const long long r = b / 8;
    part = (int)(r % nf);
    return ((r / nf) * 8 + b % 8) * kBlock + threadIdx.x;
}
__host__ inline unsigned sp_part_blocks(long long items, int nf)
{
    const long long nb = (items + kBlock - 1) / kBlock;
    return (unsigned)((nb + 7) / 8 * 8 * nf);
}

// the (t|s) family index: (x|y) (x|z) (y|x) (y|z) (z|x) (z|y)
__host__ __device__ constexpr int sp_fam(int t, int s) { return 2 * t + (s > t ? s - 1 : s); }

// Trace stage: one thread per cell, all three axes.
__global__ void __launch_bounds__(kBlock) k_sp_trace(SpArgs A, SpBatch B)
{
    int x, y, z, part;
    const long long t = sp_part(sp_box(A, B), kSpTraceParts, part);
    if (!sp_decode(A, t, x, y, z)) return;
    const Geo &g = A.g;
    const double gm1 = A.gamma - 1.0;
    const long long c = cell(g, x, y, z);
    const Prim q = prim_of(A.U[c], A.U[g.cs + c], A.U[2 * g.cs + c], A.U[3 * g.cs + c],
                           A.U[4 * g.cs + c], gm1);
    const double cs = sound_ri(A.gamma, q.p, q.ri);
    double f = 1.0;
    if (A.flat)
        f = ((const double *)(A.ws + ws_flat_off(g.n[0], g.n[1], g.n[2])))[t];
    const double dt = *A.dt;
    const long long stride[3] = {1, (long long)g.s[0], (long long)g.s[0] * g.s[1]};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double un = d == 0 ? q.u : (d == 1 ? q.v : q.w);
        const double dtdx = dt / g.dx[d];
        for (int s = 0; s < A.ns; ++s) {
            double a[5];
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                const long long cm = c + (m - 2) * stride[d];
                a[m] = A.S[s * g.cs + cm] / A.U[cm];
            }
            const Parab P = ppm(a[0], a[1], a[2], a[3], a[4], f);
            A.Xt[((d * 2 + 0) * A.ns + s) * A.E + t] = int_hi(P, un > 0.0 ? un : un + cs, dtdx);
            A.Xt[((d * 2 + 1) * A.ns + s) * A.E + t] = int_lo(P, un < 0.0 ? un : un - cs, dtdx);
        }
    }
}

// Corner stage: one part per traced axis td; a thread takes the face of
// both (td|sd) families (sd the other two axes), which share the traced
// densities and X of the face's two cells.  For each: both sides' traced X
// corrected by dt/3 of the round-1 species flux difference across their cell
// along sd (the round-1 species flux through an sd-face is its mass flux
// times the traced X of the side the mass leaves), then the round-2 species
// flux through the face.
__global__ void __launch_bounds__(kBlock) k_sp_corner(SpArgs A, SpBatch B)
{
    int p[3], td;
    const long long t = sp_part(sp_box(A, B), kSpCornerParts, td);
    if (!sp_decode(A, t, p[0], p[1], p[2])) return;
    if (sel3(p, td) < 0) return;  // faces of the family: td in [0, n]
    long long ic[2];
    double rq[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        int c[3] = {p[0], p[1], p[2]};
        if (!side) c[td] -= 1;
        ic[side] = sp_idx(A, c[0], c[1], c[2]);
        rq[side] = sp_rho_traced(A, td, side, c[0], c[1], c[2]);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int sd = td == 0 ? 1 + k : (td == 1 ? 2 * k : k);
        // sd in [0, n), the third axis in [-1, n]
        const int psd = sel3(p, sd);
        if (psd < 0 || psd >= sel3(A.g.n, sd)) continue;
        const double fac = *A.dt / (3.0 * sel3(A.g.dx, sd));
        const double *F1 = A.mf + sd * A.E;
        long long iu[2], il[2];  // each side's sd-neighbours above and below
        double Fl[2], Fh[2], den[2];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            int c[3] = {p[0], p[1], p[2]};
            if (!side) c[td] -= 1;
            c[sd] += 1;
            iu[side] = sp_idx(A, c[0], c[1], c[2]);
            c[sd] -= 2;
            il[side] = sp_idx(A, c[0], c[1], c[2]);
            Fl[side] = F1[ic[side]];
            Fh[side] = F1[iu[side]];
            den[side] = rq[side] - fac * (Fh[side] - Fl[side]);
        }
        const int fam = sp_fam(td, sd);
        const double F = A.mf[(3 + fam) * A.E + t];
        for (int s = 0; s < A.ns; ++s) {
            const double *Xq0 = A.Xt + ((td * 2 + 0) * A.ns + s) * A.E;
            const double *Xq1 = A.Xt + ((td * 2 + 1) * A.ns + s) * A.E;
            const double *Xh = A.Xt + ((sd * 2 + 0) * A.ns + s) * A.E;
            const double *Xl = A.Xt + ((sd * 2 + 1) * A.ns + s) * A.E;
            double xs[2];
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const double xq = (side ? Xq1 : Xq0)[ic[side]];
                const double gh = Fh[side] * (Fh[side] >= 0.0 ? Xh[ic[side]] : Xl[iu[side]]);
                const double gl = Fl[side] * (Fl[side] >= 0.0 ? Xh[il[side]] : Xl[ic[side]]);
                const double num = rq[side] * xq - fac * (gh - gl);
                xs[side] = den[side] > 0.0 ? num / den[side] : xq;
            }
            A.G2[(fam * A.ns + s) * A.E + t] = F * (F >= 0.0 ? xs[0] : xs[1]);
        }
    }
}

// Final stage: one part per axis d.  Each thread takes one d-face: both
// sides' traced X corrected by dt/2 of the two round-2 transverse species
// flux differences, then the round-3 species flux through the face.
__global__ void __launch_bounds__(kBlock) k_sp_final(SpArgs A, SpBatch B)
{
    int p[3], d;
    const long long t = sp_part(sp_box(A, B), kSpFinalParts, d);
    if (!sp_decode(A, t, p[0], p[1], p[2])) return;
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    // faces: d in [0, n], the transverse axes in [0, n)
    const int pd = sel3(p, d), p1 = sel3(p, t1), p2 = sel3(p, t2);
    if (pd < 0 || p1 < 0 || p1 >= sel3(A.g.n, t1) || p2 < 0 || p2 >= sel3(A.g.n, t2)) return;
    const double dt = *A.dt;
    const double f1 = dt / (2.0 * sel3(A.g.dx, t1));
    const double f2 = dt / (2.0 * sel3(A.g.dx, t2));
    const int fa = sp_fam(t1, t2), fb = sp_fam(t2, t1);
    long long ic[2], i1[2], i2[2];
    double rq[2], den[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        int c[3] = {p[0], p[1], p[2]};
        if (!side) c[d] -= 1;
        int c1[3] = {c[0], c[1], c[2]}, c2[3] = {c[0], c[1], c[2]};
        c1[t1] += 1;
        c2[t2] += 1;
        ic[side] = sp_idx(A, c[0], c[1], c[2]);
        i1[side] = sp_idx(A, c1[0], c1[1], c1[2]);
        i2[side] = sp_idx(A, c2[0], c2[1], c2[2]);
        rq[side] = sp_rho_traced(A, d, side, c[0], c[1], c[2]);
        const double *MA = A.mf + (3 + fa) * A.E, *MB = A.mf + (3 + fb) * A.E;
        den[side] = (rq[side] - f1 * (MA[i1[side]] - MA[ic[side]])) -
                    f2 * (MB[i2[side]] - MB[ic[side]]);
    }
    const double F = A.mf[(9 + d) * A.E + t];
    for (int s = 0; s < A.ns; ++s) {
        const double *GA = A.G2 + (fa * A.ns + s) * A.E;
        const double *GB = A.G2 + (fb * A.ns + s) * A.E;
        double xs[2];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const double xq = A.Xt[((d * 2 + side) * A.ns + s) * A.E + ic[side]];
            const double num = (rq[side] * xq - f1 * (GA[i1[side]] - GA[ic[side]])) -
                               f2 * (GB[i2[side]] - GB[ic[side]]);
            xs[side] = den[side] > 0.0 ? num / den[side] : xq;
        }
        A.G3[(d * A.ns + s) * A.E + t] = F * (F >= 0.0 ? xs[0] : xs[1]);
    }
}

__global__ void __launch_bounds__(kBlock) k_sp_update(SpArgs A, SpBatch B, int *err_dev)
{
    long long t = sp_box(A, B) * kBlock + threadIdx.x;
    const Geo &g = A.g;
    const long long nv = (long long)g.n[0] * g.n[1] * g.n[2];
    if (t >= nv) return;
    const int x = (int)(t % g.n[0]);
    t /= g.n[0];
    const int y = (int)(t % g.n[1]);
    const int z = (int)(t / g.n[1]);
    const double dt = *A.dt;
    const double ax = dt / g.dx[0], ay = dt / g.dx[1], az = dt / g.dx[2];
    const long long i0 = sp_idx(A, x, y, z);
    const long long ix = sp_idx(A, x + 1, y, z), iy = sp_idx(A, x, y + 1, z),
                    iz = sp_idx(A, x, y, z + 1);
    const long long c = cell(g, x, y, z);
    int err = 0;
    for (int s = 0; s < A.ns; ++s) {
        const double *Gx = A.G3 + (0 * A.ns + s) * A.E;
        const double *Gy = A.G3 + (1 * A.ns + s) * A.E;
        const double *Gz = A.G3 + (2 * A.ns + s) * A.E;
        double du = ax * (Gx[ix] - Gx[i0]);
        du = du + ay * (Gy[iy] - Gy[i0]);
        du = du + az * (Gz[iz] - Gz[i0]);
        const double v = A.S[s * g.cs + c] - du;
        if (!isfinite(v)) err |= HYDRO_ERR_NONFINITE;
        A.Sn[s * g.cs + c] = v;
    }
    if (err) atomicOr(err_dev, err);
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
