// species_fused.h -- the species pass in one kernel: trace, corner coupling,
// final states and the conservative update of one species' partial density
// rho X, for one box tile, marching along z.
//
// Every value is formed with the species step's own arithmetic, operation
// for operation: X = rho X / rho; each cell's limited parabola of
// X along each axis (flattened like the gas) averaged toward each face over
// the contact wave when it moves toward the face, else over the outermost
// wave; round-1 species flux = mass flux x X of the side the mass leaves
// (the low side for a zero flux); corner X = corrected partial density over
// corrected density (dt/3 of one transverse round-1 difference), the traced
// X where that density is not positive; round-2 species fluxes; final X
// (dt/2 of both transverse round-2 differences); round-3 species fluxes;
// update.  Nothing but the new partial densities goes back to HBM.
//
// Tile: a 256-thread block covers 16 x 16 columns, the inner 14 x 14 the
// output columns (the one-column ring supplies the transverse neighbours a
// flux difference needs), one species, and marches over the planes
// z0-1 .. z1 of its z-segment [z0, z1).  Iteration q traces plane q across
// (x and y, from an LDS plane of X with a two-cell halo) and plane q+1 along
// z (from the lane's own column of X, planes q-1 .. q+3, in registers),
// forms the round-1 and corner values of plane q, the round-2 species flux
// through the z-face between q-1 and q, and finishes plane p = q-1: its
// final states, round-3 fluxes and update.  x-neighbour values come from
// DPP lane shifts inside the wavefront, y-neighbour values through LDS (one
// barrier per exchange; the next plane's X enters the LDS plane with the
// last exchange, so an iteration has three), z-neighbour values are carried
// in registers.  The gas's mass fluxes (all twelve families, exported by the
// flux kernel), its traced densities (the trace kernel's workspace) and
// flattening coefficients are read at the lane's own column only.
#pragma once

namespace {

constexpr int kSB = 16;            // tile side (columns), output 14 x 14
constexpr int kSOut = kSB - 2;
constexpr int kSZ = 32;            // z-segment length
constexpr int kSRW = kSB + 4;      // LDS plane side (two-cell halo)

// blocks of one box in the fused species stage, per species
__host__ __device__ inline long long sp_fused_tiles(const Geo &g)
{
    return (long long)((g.n[0] + kSOut - 1) / kSOut) * ((g.n[1] + kSOut - 1) / kSOut) *
           ((g.n[2] + kSZ - 1) / kSZ);
}

// corrected X of a traced state: partial density over density, both
// corrected by the same flux difference; the traced X where the density is
// not positive
__device__ __forceinline__ double sp_corr1(double rq, double xq, double dF, double dG,
                                           double fac)
{
    const double den = rq - fac * dF;
    const double num = rq * xq - fac * dG;
    return den > 0.0 ? num / den : xq;
}
__device__ __forceinline__ double sp_corr2(double rq, double xq, double dFa, double dGa,
                                           double dFb, double dGb, double f1, double f2)
{
    const double den = (rq - f1 * dFa) - f2 * dFb;
    const double num = (rq * xq - f1 * dGa) - f2 * dGb;
    return den > 0.0 ? num / den : xq;
}
// species flux through a face: mass flux times X of the side it leaves
__device__ __forceinline__ double sp_flux(double F, double xlow, double xhigh)
{
    return F * (F >= 0.0 ? xlow : xhigh);
}

// (value of lane t-1, value of lane t+1) of the wavefront: DPP shifts, as
// the gas flux kernel exchanges x-neighbours
__device__ __forceinline__ double sp_prev(double v) { return dpp_prev(v); }
__device__ __forceinline__ double sp_next(double v) { return dpp_next(v); }

struct SpZ {      // z-traced X of one plane of the lane's column
    double h, l;  // high face, low face
};

__global__ void __launch_bounds__(256) k_sp_fused(SpArgs A, SpBatch B, int *err_dev)
{
    __shared__ double xp[kSRW * kSRW];  // X of the tile's plane q, two-cell halo
    __shared__ double eb[3][256];       // y-exchange: traced X (high, low), F1y
    __shared__ double ec[6][256];       // y-exchange: corner X, F2 (y|x), (y|z)
    __shared__ double ed[3][256];       // y-exchange: final X (high, low), F3y

    // block -> (tile, species): blocks are dealt to the 8 XCDs round-robin,
    // so each XCD gets a contiguous run of tiles and the species of one tile
    // run on one XCD, close in time, sharing the gas data they read
    const long long nblk = (long long)gridDim.x;
    long long L;
    {
        const long long per = nblk / 8, rem = nblk % 8;
        const long long xx = blockIdx.x % 8, ii = blockIdx.x / 8;
        L = xx * per + (xx < rem ? xx : rem) + ii;
    }
    const int ns = A.ns;
    const int s = (int)(L % ns);
    long long tile = L / ns;
    if (B.nb) {  // the box of this tile: largest b with pre[b] <= tile
        int lo = 0, hi = B.nb;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (B.pre[mid] <= tile) lo = mid;
            else hi = mid;
        }
        const int b = lo;
        tile -= B.pre[b];
        A.g = B.geos[b];
        A.U = B.Us[b];
        A.S = B.Ss[b];
        A.Sn = B.Sns[b];
        A.ws = B.ws + B.wsoff[b] * (long long)sizeof(double);
        A.E = mf_stride(A.g.n[0], A.g.n[1], A.g.n[2]);
        A.mf = B.sws + 12 * B.epre[b];
        A.dt = B.dts + (long long)b * B.dt_stride;
    }
    const Geo &g = A.g;
    const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2], ng = g.ng;
    const int ntx = (n0 + kSOut - 1) / kSOut, nty = (n1 + kSOut - 1) / kSOut;
    const int ix = (int)(tile % ntx);
    tile /= ntx;
    const int iy = (int)(tile % nty);
    const int iz = (int)(tile / nty);
    const int x0 = ix * kSOut, y0 = iy * kSOut;
    const int z0 = iz * kSZ, z1 = min(n2, z0 + kSZ);

    const int t = threadIdx.x;
    const int tx = t % kSB, ty = t / kSB;
    const int x = x0 - 1 + tx, y = y0 - 1 + ty;
    const int tD = ty >= 1 ? t - kSB : t, tU = ty + 1 < kSB ? t + kSB : t;
    const bool outc = tx >= 1 && tx <= kSOut && ty >= 1 && ty <= kSOut && x < n0 && y < n1;
    // loads of the lane's own column: clamped into the index box [-1, n]
    // (columns beyond it belong to unused lanes)
    const int xc = min(x, n0), yc = min(y, n1);

    const double gamma = A.gamma, gm1 = gamma - 1.0;
    const double dt = *A.dt;
    const double dtdx = dt / g.dx[0], dtdy = dt / g.dx[1], dtdz = dt / g.dx[2];
    const double fx3 = dt / (3.0 * g.dx[0]), fy3 = dt / (3.0 * g.dx[1]),
                 fz3 = dt / (3.0 * g.dx[2]);
    const double fx2 = dt / (2.0 * g.dx[0]), fy2 = dt / (2.0 * g.dx[1]),
                 fz2 = dt / (2.0 * g.dx[2]);
    const double ax = dtdx, ay = dtdy, az = dtdz;

    const double *Sg = A.S + (long long)s * g.cs;
    const double *rho = A.U;
    const long long E = A.E;
    const double *mf = A.mf;
    const double *flat =
        A.flat ? (const double *)(A.ws + ws_flat_off(n0, n1, n2)) : nullptr;
    WS w;
    w.base = const_cast<char *>(A.ws);
    w.pitch = ws_pitch(n0, n1);
    w.nxb = ws_xblocks(n0);
    const unsigned wo = w.off(xc, yc);

    // (every access below is a uniform base plus the lane's 32-bit byte
    // offset: one component of a box and one field of the index box stay
    // below 2 GiB)
    auto zcl = [&](int z) { return min(max(z, -ng), n2 + ng - 1); };
    auto mfz = [&](int z) { return min(max(z, -1), n2); };  // plane clamp of the index box
    auto mfo = [&](int z) { return (unsigned)mf_index(n0, n1, xc, yc, mfz(z)) * 8u; };
    auto cbo = [&](int cx, int cy, int z) { return (unsigned)cell(g, cx, cy, z) * 8u; };
    // X of the lane's own column at plane z
    auto xown = [&](int z) {
        const unsigned bo = cbo(xc, yc, zcl(z));
        return ldb(Sg, bo) / ldb(rho, bo);
    };
    // primitives of the own cell at plane z: the velocities across the
    // axes and the sound speed
    struct Lam {
        double u, v, w, c, f;
    };
    auto lam_of = [&](int z) {
        const unsigned bo = cbo(xc, yc, zcl(z));
        const Prim q = prim_of(ldb(A.U, bo), ldb(A.U + g.cs, bo), ldb(A.U + 2 * g.cs, bo),
                               ldb(A.U + 3 * g.cs, bo), ldb(A.U + 4 * g.cs, bo), gm1);
        Lam l;
        l.u = q.u;
        l.v = q.v;
        l.w = q.w;
        l.c = sound_ri(gamma, q.p, q.ri);
        l.f = flat ? ldb(flat, mfo(z)) : 1.0;
        return l;
    };
    // traced X at both faces along an axis, from the 5-cell pencil a[]
    auto trace = [&](const double *a, double un, double cs, double f, double dtd) {
        const Parab P = ppm(a[0], a[1], a[2], a[3], a[4], f);
        SpZ r;
        r.h = int_hi(P, un > 0.0 ? un : un + cs, dtd);
        r.l = int_lo(P, un < 0.0 ? un : un - cs, dtd);
        return r;
    };

    // ---- prologue: the column's X window and the z-traces of planes
    // z0-2 and z0-1 (the first iteration's "previous" planes)
    double wz[5];
    for (int m = 0; m < 5; ++m) wz[m] = xown(z0 - 3 + m);  // planes z0-3 .. z0+1
    SpZ zt_prev, zt_cur;
    {
        double a0[5] = {xown(z0 - 4), wz[0], wz[1], wz[2], wz[3]};  // around z0-2
        const Lam l0 = lam_of(z0 - 2);
        zt_prev = trace(a0, l0.w, l0.c, l0.f, dtdz);
        const Lam l1 = lam_of(z0 - 1);
        zt_cur = trace(wz, l1.w, l1.c, l1.f, dtdz);
    }
    Lam lam_q = lam_of(z0 - 1);  // the own cell of plane q

    // carries from plane to plane (values of the previous plane; zero until
    // the first iteration has run: what they feed in the first iteration is
    // never used)
    double cz_xh_zx = 0.0, cz_xh_zy = 0.0;   // corner X (z|x), (z|y), high face
    double cz_G2zx = 0.0, cz_G2zy = 0.0;     // G2 (z|x), (z|y) through the low z-face
    double cz_F2zx = 0.0, cz_F2zy = 0.0;     // F2 of the same faces
    double cz_xfh = 0.0;                     // final z X, high face
    double cz_G3z = 0.0;                     // G3 z through the low z-face
    double cp_dF2yz = 0.0, cp_dG2yz = 0.0;   // in-plane differences (y|z), (x|z)
    double cp_dF2xz = 0.0, cp_dG2xz = 0.0;
    double cp_xh = 0.0, cp_xl = 0.0, cp_yh = 0.0, cp_yl = 0.0;  // traced X x, y
    double cp_rxh = 0.0, cp_rxl = 0.0, cp_ryh = 0.0, cp_ryl = 0.0;  // traced rho x, y
    int err = 0;

    // X of the tile's plane z with its two-cell halo, for the LDS plane:
    // this thread's cells t and t + 256 (of 400)
    auto xplane = [&](int z, double &v0, double &v1) {
        const int zq = zcl(z);
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const int r = t + 256 * m;
            double v = 0.0;
            if (r < kSRW * kSRW) {
                const int rx = r % kSRW, ry = r / kSRW;
                const int cx = min(max(x0 - 3 + rx, -ng), n0 + ng - 1);
                const int cy = min(max(y0 - 3 + ry, -ng), n1 + ng - 1);
                const unsigned bo = cbo(cx, cy, zq);
                v = ldb(Sg, bo) / ldb(rho, bo);
            }
            (m ? v1 : v0) = v;
        }
    };
    // the same in two parts inside the z-march: the partial densities and
    // densities fetched with the iteration's other loads (by every lane, the
    // second cell's index clamped into the plane: lanes past its 400 cells
    // fetch a cell they do not store), the division where the plane is
    // stored -- a division right after its loads (in a branch, as above)
    // would make the iteration's later loads wait for them
    auto xplane_ld = [&](int z, double (&sr)[4]) {
        const int zq = zcl(z);
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const int r = min(t + 256 * m, kSRW * kSRW - 1);
            const int rx = r % kSRW, ry = r / kSRW;
            const int cx = min(max(x0 - 3 + rx, -ng), n0 + ng - 1);
            const int cy = min(max(y0 - 3 + ry, -ng), n1 + ng - 1);
            const unsigned bo = cbo(cx, cy, zq);
            sr[2 * m] = ldb(Sg, bo);
            sr[2 * m + 1] = ldb(rho, bo);
        }
    };
    auto xplane_put = [&](double v0, double v1) {
        xp[t] = v0;
        if (t + 256 < kSRW * kSRW) xp[t + 256] = v1;
    };
    {
        double v0, v1;
        xplane(z0 - 1, v0, v1);
        xplane_put(v0, v1);
    }
    __syncthreads();

    for (int q = z0 - 1; q <= z1; ++q) {
        const int p = q - 1;
        // (the LDS plane holds X of plane q: written before the previous
        // iteration's last barrier)
        // the next plane's X for the LDS plane, stored after this
        // iteration's second barrier (when every wave has traced plane q)
        double xsr[4];
        xplane_ld(q + 1, xsr);
        // the old partial density of the cell updated at the end of the
        // z-step (plane p), fetched with the other loads (every lane, at its
        // clamped column: the updating lanes' own cell)
        const double s_old = ldb(Sg, cbo(xc, yc, zcl(p)));
        // own column: plane q+3 of the X window, the cell of plane q+1
        const double xnew = xown(q + 3);
        const Lam lam_n = lam_of(q + 1);
        // mass fluxes through the own cell's faces (index box position)
        const unsigned iq = mfo(q);
        auto mfl = [&](int f, unsigned o) { return ldb(mf + f * E, o); };
        const double F1x = mfl(0, iq), F1y = mfl(1, iq), F1z = mfl(2, iq);
        const double F1zn = mfl(2, mfo(q + 1));
        const double F2xy = mfl(3, iq), F2xz = mfl(4, iq), F2yx = mfl(5, iq),
                     F2yz = mfl(6, iq), F2zx = mfl(7, iq), F2zy = mfl(8, iq);
        const double F3z = mfl(11, iq);
        const unsigned ip = mfo(p);
        const double F3x = mfl(9, ip), F3y = mfl(10, ip);
        // traced densities of plane q
        const char *pq = w.plane(min(max(q, -2), n2 + 1));
        const double rxh = ws_ld(pq, wo, QHI(0, 0)), rxl = ws_ld(pq, wo, QLO(0, 0));
        const double ryh = ws_ld(pq, wo, QHI(1, 0)), ryl = ws_ld(pq, wo, QLO(1, 0));
        const double rzh = ws_ld(pq, wo, QHI(2, 0)), rzl = ws_ld(pq, wo, QLO(2, 0));

        // ------------------------------------------------ traces
        const int rc = (ty + 2) * kSRW + (tx + 2);
        double a[5];
        for (int m = 0; m < 5; ++m) a[m] = xp[rc + (m - 2)];
        const SpZ tx_ = trace(a, lam_q.u, lam_q.c, lam_q.f, dtdx);
        for (int m = 0; m < 5; ++m) a[m] = xp[rc + (m - 2) * kSRW];
        const SpZ ty_ = trace(a, lam_q.v, lam_q.c, lam_q.f, dtdy);
        // z: plane q+1 from the window q-1 .. q+3
        for (int m = 0; m < 4; ++m) wz[m] = wz[m + 1];
        wz[4] = xnew;
        const SpZ zt_next = trace(wz, lam_n.w, lam_n.c, lam_n.f, dtdz);

        // ------------------------------------------------ round 1
        // y: the neighbours' traced X and the upper face's mass flux
        eb[0][t] = ty_.h;
        eb[1][t] = ty_.l;
        eb[2][t] = F1y;
        // x: within the wavefront
        const double F1xn = sp_next(F1x);
        const double dF1x = F1xn - F1x;
        const double dG1x = sp_flux(F1xn, tx_.h, sp_next(tx_.l)) - sp_flux(F1x, sp_prev(tx_.h), tx_.l);
        // z: the own column
        const double dF1z = F1zn - F1z;
        const double dG1z = sp_flux(F1zn, zt_cur.h, zt_next.l) - sp_flux(F1z, zt_prev.h, zt_cur.l);
        __syncthreads();
        const double F1yn = eb[2][tU];
        const double dF1y = F1yn - F1y;
        const double dG1y = sp_flux(F1yn, ty_.h, eb[1][tU]) - sp_flux(F1y, eb[0][tD], ty_.l);

        // ------------------------------------------------ corner X of plane q
        const double c_xy_h = sp_corr1(rxh, tx_.h, dF1y, dG1y, fy3);
        const double c_xy_l = sp_corr1(rxl, tx_.l, dF1y, dG1y, fy3);
        const double c_xz_h = sp_corr1(rxh, tx_.h, dF1z, dG1z, fz3);
        const double c_xz_l = sp_corr1(rxl, tx_.l, dF1z, dG1z, fz3);
        const double c_yx_h = sp_corr1(ryh, ty_.h, dF1x, dG1x, fx3);
        const double c_yx_l = sp_corr1(ryl, ty_.l, dF1x, dG1x, fx3);
        const double c_yz_h = sp_corr1(ryh, ty_.h, dF1z, dG1z, fz3);
        const double c_yz_l = sp_corr1(ryl, ty_.l, dF1z, dG1z, fz3);
        const double c_zx_h = sp_corr1(rzh, zt_cur.h, dF1x, dG1x, fx3);
        const double c_zx_l = sp_corr1(rzl, zt_cur.l, dF1x, dG1x, fx3);
        const double c_zy_h = sp_corr1(rzh, zt_cur.h, dF1y, dG1y, fy3);
        const double c_zy_l = sp_corr1(rzl, zt_cur.l, dF1y, dG1y, fy3);

        // ------------------------------------------------ round 2
        ec[0][t] = c_yx_h;
        ec[1][t] = c_yx_l;
        ec[2][t] = c_yz_h;
        ec[3][t] = c_yz_l;
        ec[4][t] = F2yx;
        ec[5][t] = F2yz;
        // x-families: both x-faces of the cell
        const double F2xyn = sp_next(F2xy), F2xzn = sp_next(F2xz);
        const double dF2xy = F2xyn - F2xy, dF2xz = F2xzn - F2xz;
        const double dG2xy = sp_flux(F2xyn, c_xy_h, sp_next(c_xy_l)) -
                             sp_flux(F2xy, sp_prev(c_xy_h), c_xy_l);
        const double dG2xz = sp_flux(F2xzn, c_xz_h, sp_next(c_xz_l)) -
                             sp_flux(F2xz, sp_prev(c_xz_h), c_xz_l);
        // z-families: through the z-face between q-1 and q; their
        // z-differences over plane p
        const double G2zx = sp_flux(F2zx, cz_xh_zx, c_zx_l);
        const double G2zy = sp_flux(F2zy, cz_xh_zy, c_zy_l);
        const double dF2zx_p = F2zx - cz_F2zx, dG2zx_p = G2zx - cz_G2zx;
        const double dF2zy_p = F2zy - cz_F2zy, dG2zy_p = G2zy - cz_G2zy;
        __syncthreads();
        const double F2yxn = ec[4][tU], F2yzn = ec[5][tU];
        const double dF2yx = F2yxn - F2yx, dF2yz = F2yzn - F2yz;
        const double dG2yx = sp_flux(F2yxn, c_yx_h, ec[1][tU]) - sp_flux(F2yx, ec[0][tD], c_yx_l);
        const double dG2yz = sp_flux(F2yzn, c_yz_h, ec[3][tU]) - sp_flux(F2yz, ec[2][tD], c_yz_l);

        // ------------------------------------------------ final states
        // z of plane q (t1 = x, t2 = y)
        const double fz_h = sp_corr2(rzh, zt_cur.h, dF2xy, dG2xy, dF2yx, dG2yx, fx2, fy2);
        const double fz_l = sp_corr2(rzl, zt_cur.l, dF2xy, dG2xy, dF2yx, dG2yx, fx2, fy2);
        const double G3zq = sp_flux(F3z, cz_xfh, fz_l);
        // x of plane p (t1 = y, t2 = z), y of plane p (t1 = x, t2 = z)
        const double fx_h = sp_corr2(cp_rxh, cp_xh, cp_dF2yz, cp_dG2yz, dF2zy_p, dG2zy_p, fy2, fz2);
        const double fx_l = sp_corr2(cp_rxl, cp_xl, cp_dF2yz, cp_dG2yz, dF2zy_p, dG2zy_p, fy2, fz2);
        const double fy_h = sp_corr2(cp_ryh, cp_yh, cp_dF2xz, cp_dG2xz, dF2zx_p, dG2zx_p, fx2, fz2);
        const double fy_l = sp_corr2(cp_ryl, cp_yl, cp_dF2xz, cp_dG2xz, dF2zx_p, dG2zx_p, fx2, fz2);

        // ------------------------------------------------ round 3, plane p
        ed[0][t] = fy_h;
        ed[1][t] = fy_l;
        ed[2][t] = F3y;
        // ... and divided where they are stored
        xplane_put(xsr[0] / xsr[1], xsr[2] / xsr[3]);
        const double F3xn = sp_next(F3x);
        const double dG3x = sp_flux(F3xn, fx_h, sp_next(fx_l)) - sp_flux(F3x, sp_prev(fx_h), fx_l);
        __syncthreads();
        const double F3yn = ed[2][tU];
        const double dG3y = sp_flux(F3yn, fy_h, ed[1][tU]) - sp_flux(F3y, ed[0][tD], fy_l);

        // ------------------------------------------------ update plane p
        if (outc && p >= z0) {
            double du = ax * dG3x;
            du = du + ay * dG3y;
            du = du + az * (G3zq - cz_G3z);
            const unsigned bo = cbo(x, y, p);
            const double v = s_old - du;
            if (!isfinite(v)) err |= HYDRO_ERR_NONFINITE;
            stb64(A.Sn + (long long)s * g.cs, bo, v);
        }

        // ------------------------------------------------ carries
        zt_prev = zt_cur;
        zt_cur = zt_next;
        lam_q = lam_n;
        cz_xh_zx = c_zx_h;
        cz_xh_zy = c_zy_h;
        cz_G2zx = G2zx;
        cz_G2zy = G2zy;
        cz_F2zx = F2zx;
        cz_F2zy = F2zy;
        cz_xfh = fz_h;
        cz_G3z = G3zq;
        cp_dF2yz = dF2yz;
        cp_dG2yz = dG2yz;
        cp_dF2xz = dF2xz;
        cp_dG2xz = dG2xz;
        cp_xh = tx_.h;
        cp_xl = tx_.l;
        cp_yh = ty_.h;
        cp_yl = ty_.l;
        cp_rxh = rxh;
        cp_rxl = rxl;
        cp_ryh = ryh;
        cp_ryl = ryl;
    }
    if (err) atomicOr(err_dev, err);
}

}  // namespace
