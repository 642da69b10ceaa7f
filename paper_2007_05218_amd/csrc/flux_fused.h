// flux_fused.h -- the second half of the CTU step in one kernel:
// round-1 HLLC, corner coupling + round-2 HLLC, final states + round-3 HLLC,
// conservative update, for one box tile, marching along z.
//
// Input (HBM workspace, written by the trace kernel): the traced face states
// of every cell in all three directions; the round-1 fluxes are solved here
// from them.  Output: the new state of the tile's cells (and, optionally,
// the CFL timestep of the new state).  Nothing else goes back to HBM:
// x-neighbour exchanges stay inside the wavefront (DPP lane shifts),
// y-neighbour exchanges go through LDS, and the z-direction couplings
// (fluxes through z-faces and the z-differences of the (z|s) fluxes) are
// carried from plane to plane in registers or, for
// values a lane alone needs a plane later, in its own LDS slots (which keeps
// the kernel within its register budget: spilled registers would go to
// scratch memory and cost HBM traffic).
//
// Tile: a 256-thread block covers BX x BY columns (BX*BY = 256) of which the
// inner (BX-2) x (BY-2) are output columns; the one-column ring supplies the
// transverse neighbours every flux difference needs.  A block marches over
// planes z0-1 .. z1 of its z-segment [z0, z1); iteration q computes the
// in-plane round-2 fluxes of plane q, the z-face fluxes between q-1 and q,
// and finishes plane q-1 (its final x/y states need the (z|s) fluxes on both
// of its z-faces).
//
// Error bits: a transverse-corrected state raises the fallback bit only
// where the whole-box step computes it (the flux it feeds lies in that
// flux's region of the box) and where this tile computes it from valid data
// (every neighbour exchange it depends on had the neighbour in the tile, and
// every z-carry it uses was computed in this segment); overlapping tiles may
// raise the same bit twice, which OR absorbs.
#pragma once

namespace {

constexpr int kFT = 256;  // threads of a fused-flux block

struct XBuf {
    double v[10][kFT];
};

__device__ __forceinline__ void put5(double (*b)[kFT], int k0, int t, double a0, double a1,
                                     double a2, double a3, double a4)
{
    b[k0 + 0][t] = a0;
    b[k0 + 1][t] = a1;
    b[k0 + 2][t] = a2;
    b[k0 + 3][t] = a3;
    b[k0 + 4][t] = a4;
}
// states are exchanged without their 1/rho (5 slots from k0); the reader
// forms it, as the writer did, as 1/rho
__device__ __forceinline__ void putF(double (*b)[kFT], int k0, int t, const Face &f)
{
    put5(b, k0, t, f.r, f.u, f.v, f.w, f.p);
}
__device__ __forceinline__ void putX(double (*b)[kFT], int k0, int t, const Flux &f)
{
    put5(b, k0, t, f.m, f.mu, f.mv, f.mw, f.e);
}
__device__ __forceinline__ Face getF(double (*b)[kFT], int k0, int t)
{
    Face f;
    f.r = b[k0 + 0][t];
    f.u = b[k0 + 1][t];
    f.v = b[k0 + 2][t];
    f.w = b[k0 + 3][t];
    f.p = b[k0 + 4][t];
    f.ri = 1.0 / f.r;
    return f;
}
// the same without forming 1/rho
__device__ __forceinline__ Face getF_raw(double (*b)[kFT], int k0, int t)
{
    Face f;
    f.r = b[k0 + 0][t];
    f.u = b[k0 + 1][t];
    f.v = b[k0 + 2][t];
    f.w = b[k0 + 3][t];
    f.p = b[k0 + 4][t];
    f.ri = 0.0;
    return f;
}
__device__ __forceinline__ Flux getX(double (*b)[kFT], int k0, int t)
{
    Flux f;
    f.m = b[k0 + 0][t];
    f.mu = b[k0 + 1][t];
    f.mv = b[k0 + 2][t];
    f.mw = b[k0 + 3][t];
    f.e = b[k0 + 4][t];
    return f;
}

// hi - lo, component-wise
__device__ __forceinline__ Flux fdiff(const Flux &hi, const Flux &lo)
{
    Flux d;
    d.m = hi.m - lo.m;
    d.mu = hi.mu - lo.mu;
    d.mv = hi.mv - lo.mv;
    d.mw = hi.mw - lo.mw;
    d.e = hi.e - lo.e;
    return d;
}

// Loads and stores at a 32-bit byte offset from a uniform field base (one
// component of a box is below 2 GiB), so the address is a scalar base plus
// one VGPR.  The pointers are marked as global memory: through a generic
// pointer the access would be a flat one, which the hardware counts with the
// LDS accesses as well, so every wait for an LDS read would also wait for the
// loads in flight (the prefetch of the next plane among them).
typedef __attribute__((address_space(1))) double gdouble;
__device__ __forceinline__ double ldb(const double *f, unsigned bo)
{
    return *(const gdouble *)((const __attribute__((address_space(1))) char *)f + bo);
}
__device__ __forceinline__ void stb64(double *f, unsigned bo, double v)
{
    *(gdouble *)((__attribute__((address_space(1))) char *)f + bo) = v;
}

// A plane pointer kept opaque to the compiler (an empty statement that may
// change it): loads then address as the plane's scalar base plus the lane's
// 32-bit column offset, instead of a 64-bit per-lane sum hoisted out of the
// z-loop (two more vector registers held for the whole loop).
typedef const __attribute__((address_space(1))) char gchar;
__device__ __forceinline__ gchar *opaque_plane(const char *p)
{
    asm volatile("" : "+s"(p));
    return (gchar *)p;
}
__device__ __forceinline__ Face load_face_b(gchar *pp, unsigned lo, int f0)
{
    auto ld = [&](int f) {
        return *(const __attribute__((address_space(1))) double *)(pp + lo + ws_foff(f));
    };
    Face f;
    f.r = ld(f0 + 0);
    f.u = ld(f0 + 1);
    f.v = ld(f0 + 2);
    f.w = ld(f0 + 3);
    f.p = ld(f0 + 4);
    f.ri = 0.0;
    return f;
}

// a traced state from fields f0 .. f0+4 of the column at offset lo of plane pp
__device__ __forceinline__ Face load_face_b(const char *pp, unsigned lo, int f0)
{
    Face f;
    f.r = ws_ld(pp, lo, f0 + 0);
    f.u = ws_ld(pp, lo, f0 + 1);
    f.v = ws_ld(pp, lo, f0 + 2);
    f.w = ws_ld(pp, lo, f0 + 3);
    f.p = ws_ld(pp, lo, f0 + 4);
    f.ri = 0.0;
    return f;
}

// a traced state with its 1/rho, as a Riemann problem takes it
__device__ __forceinline__ Face with_ri(Face f)
{
    f.ri = 1.0 / f.r;
    return f;
}

// corner state: prim(U(q) - fac * dF), with the rejection rule
__device__ __forceinline__ Face corner_state(const Face &q, const Flux &dF, double fac,
                                             double gm1, double igm1, int &fb)
{
    const double E = energy(q.r, q.u, q.v, q.w, q.p, igm1);
    double V0 = q.r - fac * dF.m;
    double V1 = (q.r * q.u) - fac * dF.mu;
    double V2 = (q.r * q.v) - fac * dF.mv;
    double V3 = (q.r * q.w) - fac * dF.mw;
    double V4 = E - fac * dF.e;
    fb = 0;
    return accept(q, V0, V1, V2, V3, V4, gm1, fb);
}

// final state: prim((U(q) - f1 * dA) - f2 * dB), with the rejection rule
__device__ __forceinline__ Face final_state2(const Face &q, const Flux &dA, const Flux &dB,
                                             double f1, double f2, double gm1, double igm1,
                                             int &fb)
{
    const double E = energy(q.r, q.u, q.v, q.w, q.p, igm1);
    double V0 = (q.r - f1 * dA.m) - f2 * dB.m;
    double V1 = ((q.r * q.u) - f1 * dA.mu) - f2 * dB.mu;
    double V2 = ((q.r * q.v) - f1 * dA.mv) - f2 * dB.mv;
    double V3 = ((q.r * q.w) - f1 * dA.mw) - f2 * dB.mw;
    double V4 = (E - f1 * dA.e) - f2 * dB.e;
    fb = 0;
    return accept(q, V0, V1, V2, V3, V4, gm1, fb);
}

__device__ __forceinline__ bool inr(int v, int lo, int hi) { return v >= lo && v <= hi; }

// tile decomposition of one box for the fused kernels
struct Tile {
    int BX, BY, TX, TY;
    int x0, y0, z0, z1;
};

__device__ __forceinline__ Tile tile_of(const Geo &g, long long blk, long long nblk)
{
    Tile T;
    T.BX = g.tbx2;
    T.BY = flux_rows(g.tbx2);
    T.TX = T.BX - 2;
    T.TY = T.BY - 2;
    const int ntx = (g.n[0] + T.TX - 1) / T.TX;
    const int nty = (g.n[1] + T.TY - 1) / T.TY;
    // spread neighbouring tiles over one XCD: blocks are dealt round-robin to
    // the 8 XCDs, so give each XCD a contiguous run of tiles (shared halo
    // rows then meet in that XCD's L2)
    long long per = nblk / 8, rem = nblk % 8;
    long long x = blk % 8, i = blk / 8;
    long long t = x * per + (x < rem ? x : rem) + i;
    if (t >= nblk) t = blk;  // (cannot happen; keeps the mapping total)
    const int ix = (int)(t % ntx);
    t /= ntx;
    const int iy = (int)(t % nty);
    const int iz = (int)(t / nty);
    T.x0 = ix * T.TX;
    T.y0 = iy * T.TY;
    const int zs = seg_len(g.n[2], g.tzs2);
    T.z0 = iz * zs;
    T.z1 = min(g.n[2], T.z0 + zs);
    return T;
}

// x-neighbour exchange inside the wavefront: tile rows are runs of BX lanes,
// whole rows in each wavefront, so a lane's low and high x-neighbours are
// lanes t-1 and t+1 of its own wavefront, and a DPP shift of the whole
// wavefront by one lane delivers their values with no LDS traffic and no
// barrier.  (A lane at
// a row end receives another row's value or its own; nothing it computes
// from it is used.)
// (bound_ctrl: the lane at the wavefront's end, which has no source lane,
// reads zero instead of keeping an old value, so each 32-bit half is one
// DPP move with no copy of the old value first)
__device__ __forceinline__ double dpp_prev(double v)  // lane t-1's v
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x138, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double dpp_next(double v)  // lane t+1's v
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x130, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
// the low x-neighbour's state; its 1/rho is the neighbour's (formed there,
// as 1/rho, by the state's primitive conversion or by with_ri)
__device__ __forceinline__ Face prevF(const Face &f)
{
    Face g;
    g.r = dpp_prev(f.r);
    g.u = dpp_prev(f.u);
    g.v = dpp_prev(f.v);
    g.w = dpp_prev(f.w);
    g.p = dpp_prev(f.p);
    g.ri = dpp_prev(f.ri);
    return g;
}
// the high x-neighbour's flux minus this lane's
__device__ __forceinline__ Flux next_minus(const Flux &f)
{
    Flux d;
    d.m = dpp_next(f.m) - f.m;
    d.mu = dpp_next(f.mu) - f.mu;
    d.mv = dpp_next(f.mv) - f.mv;
    d.mw = dpp_next(f.mw) - f.mw;
    d.e = dpp_next(f.e) - f.e;
    return d;
}

#ifndef HYDRO_FUSED_WAVES
#define HYDRO_FUSED_WAVES 2
#endif
// EX: also export the mass flux of every Riemann solve the box step makes
// (twelve fields, one per flux family, over faces named by the cell above,
// coordinates -1 .. n per axis) for the species pass.  A tile stores a flux
// only where it computed it from valid data; tiles that overlap store the
// same value.
template <bool EX>
__global__ void __launch_bounds__(kFT) __attribute__((amdgpu_waves_per_eu(HYDRO_FUSED_WAVES)))
k_flux_fused(Launch L, double gamma, double cfl, double gx, double gy, double gz, int *err_dev,
             double *mflux, const long long *mf_pre, int mf_mul)
{
    // y-neighbour exchanges alternate between two buffers, so each needs one
    // barrier (its readers of two exchanges back are past the barrier of the
    // exchange between); x-neighbour exchanges stay in the wavefront (DPP)
    __shared__ XBuf ya, yb;
    // own-lane carries: dF2xz, dF2yz of the previous plane, F3z through its
    // low face, F1z through the current plane's low face
    __shared__ double cz[20][kFT];
    Box1 o = resolve(L);
    const Geo &g = o.g;
    const WS &ws = o.ws;
    const Tile T = tile_of(g, o.blk, o.nblk);
    const int t = threadIdx.x;
    // lane -> column: each wavefront holds 64 / BX whole rows of BX lanes
    // (the x-exchanges are shifts of the whole wavefront, so a row must not
    // straddle two); lanes past the last whole row (BX = 18: lanes 54-63)
    // are idle: they repeat the last row's last column, exchange with no
    // neighbour and write nothing
    const int rpw = 64 / T.BX, lw = t & 63;
    const bool act = lw < rpw * T.BX;
    const int tx = act ? lw % T.BX : T.BX - 1;
    const int ty = (t >> 6) * rpw + (act ? lw / T.BX : rpw - 1);
    auto lane_of = [&](int yy) { return (yy / rpw) * 64 + (yy % rpw) * T.BX + tx; };
    const int x = T.x0 - 1 + tx, y = T.y0 - 1 + ty;
    const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
    // loads come from the clamped column (inside the traced region); results
    // of columns outside it are never used
    const int xc = min(x, n0), yc = min(y, n1);
    const int tD = act && ty >= 1 ? lane_of(ty - 1) : t;
    const int tU = act && ty + 1 < T.BY ? lane_of(ty + 1) : t;
    // neighbour lanes present in the tile: a value that depends on an
    // exchange with a missing neighbour is never used and raises no error bit
    const bool hL = act && tx >= 1, hR = act && tx + 1 < T.BX, hD = act && ty >= 1,
               hU = act && ty + 1 < T.BY;
    const bool outc =
        act && tx >= 1 && tx <= T.TX && ty >= 1 && ty <= T.TY && x < n0 && y < n1;

    // region tests of the whole-box step (where it computes each quantity)
    const bool rx_f = inr(x, 0, n0), rx_fh = inr(x + 1, 0, n0), rx_c = inr(x, 0, n0 - 1),
               rx_w = inr(x, -1, n0);
    const bool ry_f = inr(y, 0, n1), ry_fh = inr(y + 1, 0, n1), ry_c = inr(y, 0, n1 - 1),
               ry_w = inr(y, -1, n1);

    const double gm1 = gamma - 1.0;
    const double igm1 = 1.0 / gm1;
    const double dt = *o.dt;
    const double fx3 = dt / (3.0 * g.dx[0]), fy3 = dt / (3.0 * g.dx[1]),
                 fz3 = dt / (3.0 * g.dx[2]);
    const double fx2 = dt / (2.0 * g.dx[0]), fy2 = dt / (2.0 * g.dx[1]),
                 fz2 = dt / (2.0 * g.dx[2]);
    const double ax = dt / g.dx[0], ay = dt / g.dx[1], az = dt / g.dx[2];
    const unsigned wo = ws.off(xc, yc);  // own column in the workspace
    // mass-flux export: field f of face (x, y, z).  Bit f of exm: the lane
    // computes field f from valid data and its face lies in the field's
    // region (the plane's conditions are checked where the flux is formed).
    // (a batch: box b's export starts mf_mul * mf_pre[b] doubles in)
    if (EX && mf_pre) mflux += mf_mul * mf_pre[o.b];
    const long long mfE = EX ? mf_stride(n0, n1, n2) : 0;
    const long long mfP = (long long)(n0 + 2) * (n1 + 2);
    // (a uniform plane base plus the lane's 32-bit byte offset, as for the
    // workspace: (n0+2)(n1+2) doubles fit 32-bit offsets for every valid box.
    // The base is formed at each store and kept opaque: otherwise the
    // compiler hoists the twelve per-lane 64-bit field addresses out of the
    // z-loop, and they spill)
    const unsigned mfo = (unsigned)((y + 1) * (n0 + 2) + (x + 1)) * 8u;
    auto mf_put = [&](int f, int z, double v) {
        const char *fb = (const char *)(mflux + f * mfE + (long long)(z + 1) * mfP);
        asm volatile("" : "+s"(fb));
        stb64((double *)fb, mfo, v);
    };
    unsigned exm = 0;
    if (EX && act) {
        const bool ex_x = inr(x, -1, n0), ex_y = inr(y, -1, n1);
        const bool fx = hL && rx_f, fy = hD && ry_f, cx = hL && hR && rx_c, cy = hD && hU && ry_c;
        exm = (unsigned)(fx && ex_y) << 0 | (unsigned)(fy && ex_x) << 1 |
              (unsigned)(ex_x && ex_y) << 2 | (unsigned)(fx && cy) << 3 |
              (unsigned)(fx && ex_y) << 4 | (unsigned)(fy && cx) << 5 |
              (unsigned)(fy && ex_x) << 6 | (unsigned)(cx && ex_y) << 7 |
              (unsigned)(cy && ex_x) << 8 | (unsigned)(fx && cy) << 9 |
              (unsigned)(fy && cx) << 10 | (unsigned)(cx && cy) << 11;
    }
    auto exb = [&](int f) { return EX && ((exm >> f) & 1u); };

    // plane-to-plane carries (values of the previous plane)
    // (zero until the first plane has been processed; the values derived from
    // them in the first two planes of a segment are never used)
    // (the three states are carried without their 1/rho, which the solve
    // re-forms from the carried density as 1/rho: six fewer registers held
    // through the z-march, fewer spilled)
    Face c_zx_hi = {}, c_zy_hi = {}, fz_hi = {};  // corner (z|x), (z|y), final z: high face
    Flux F2zx = {}, F2zy = {};    // (z|x), (z|y) fluxes through the plane's low z-face
    int err = 0;
    // CFL bound of the lane's new cells, for the next step's timestep
    double dtn = __longlong_as_double((long long)kInfBits);

    for (int q = T.z0 - 1; q <= T.z1; ++q) {
        gchar *pq = opaque_plane(ws.plane(q));
        // (the (s|z) corner states of the warm-up plane use the round-1 z-flux
        // below it, which this segment does not have: the previous segment
        // covers them)
        const bool rz_c = inr(q, 0, n2 - 1) && q >= T.z0, rz_w = inr(q, -1, n2);
        // ---------------------------------------------------- loads
        // (all issued before the first wait: the next plane's low z-state,
        // which no other load's wait then holds back, and the high y-state,
        // whose exchange opens the z-step; the other loads complete while
        // the block meets at the barrier)
        const Face qz_lo_n = load_face_b(opaque_plane(ws.plane(q + 1)), wo, QLO(2, 0));  // next plane
        const Face qy_hi = load_face_b(pq, wo, QHI(1, 0));
        putF(ya.v, 0, t, qy_hi);
        const Face qx_lo = load_face_b(pq, wo, QLO(0, 0)), qx_hi = load_face_b(pq, wo, QHI(0, 0));
        const Face qy_lo = load_face_b(pq, wo, QLO(1, 0));
        const Face qz_lo = load_face_b(pq, wo, QLO(2, 0)), qz_hi = load_face_b(pq, wo, QHI(2, 0));
        __syncthreads();
        // ---------------------------------------------------- round-1 fluxes
        // through each lane's low x/y faces (the low neighbour's high state
        // from the neighbour lane: x in the wavefront, y through LDS) and
        // through the plane's high z-face; their differences over the cell
        // (solved in the order their loads complete: y, x, then z)
        {
            const Flux F1y = hllc(getF(ya.v, 0, tD), with_ri(qy_lo), 1, gamma, igm1);
            putX(yb.v, 0, t, F1y);
            if (exb(1) && rz_w) mf_put(1, q, F1y.m);
        }
        const Flux F1x = hllc(prevF(with_ri(qx_hi)), with_ri(qx_lo), 0, gamma, igm1);
        if (exb(0) && rz_w) mf_put(0, q, F1x.m);
        const Flux dF1x = next_minus(F1x);
        const Flux F1zn = hllc(with_ri(qz_hi), with_ri(qz_lo_n), 2, gamma, igm1);
        if (exb(2) && inr(q + 1, 0, n2)) mf_put(2, q + 1, F1zn.m);
        // (the round-1 z-flux carried from the plane below is never used
        // before the first plane's)
        const Flux dF1z = fdiff(F1zn, getX(cz, 15, t));
        putX(cz, 15, t, F1zn);
        __syncthreads();
        const Flux dF1y = fdiff(getX(yb.v, 0, tU), getX(yb.v, 0, t));

        // ---------------------------------------------------- corner states, round-2 fluxes
        int fb;
        {  // high (y|x), (y|z) states to the upper neighbour
            Face h = corner_state(qy_hi, dF1x, fx3, gm1, igm1, fb);  // (y|x)
            if (fb && hL && hR && ry_fh && rx_c && rz_w) err |= fb;
            putF(ya.v, 0, t, h);
            h = corner_state(qy_hi, dF1z, fz3, gm1, igm1, fb);  // (y|z)
            if (fb && ry_fh && rz_c && rx_w) err |= fb;
            putF(ya.v, 5, t, h);
        }
        // x-families: the low neighbour's high state from the neighbour lane;
        // the x-differences of the fluxes right away
        Flux dxy, dxz;
        {
            Face h = corner_state(qx_hi, dF1y, fy3, gm1, igm1, fb);  // (x|y)
            if (fb && hD && hU && rx_fh && ry_c && rz_w) err |= fb;
            Face l = corner_state(qx_lo, dF1y, fy3, gm1, igm1, fb);
            if (fb && hD && hU && rx_f && ry_c && rz_w) err |= fb;
            const Flux Fxy = hllc(prevF(h), l, 0, gamma, igm1);
            dxy = next_minus(Fxy);
            if (exb(3) && rz_w) mf_put(3, q, Fxy.m);
            h = corner_state(qx_hi, dF1z, fz3, gm1, igm1, fb);  // (x|z)
            if (fb && rx_fh && rz_c && ry_w) err |= fb;
            l = corner_state(qx_lo, dF1z, fz3, gm1, igm1, fb);
            if (fb && rx_f && rz_c && ry_w) err |= fb;
            const Flux Fxz = hllc(prevF(h), l, 0, gamma, igm1);
            dxz = next_minus(Fxz);
            if (exb(4) && rz_c) mf_put(4, q, Fxz.m);
        }
        __syncthreads();
        {  // y-families
            Face l = corner_state(qy_lo, dF1x, fx3, gm1, igm1, fb);  // (y|x)
            if (fb && hL && hR && ry_f && rx_c && rz_w) err |= fb;
            const Flux Fyx = hllc(getF(ya.v, 0, tD), l, 1, gamma, igm1);
            putX(yb.v, 0, t, Fyx);
            if (exb(5) && rz_w) mf_put(5, q, Fyx.m);
            l = corner_state(qy_lo, dF1z, fz3, gm1, igm1, fb);  // (y|z)
            if (fb && ry_f && rz_c && rx_w) err |= fb;
            const Flux Fyz = hllc(getF(ya.v, 5, tD), l, 1, gamma, igm1);
            putX(yb.v, 5, t, Fyz);
            if (exb(6) && rz_c) mf_put(6, q, Fyz.m);
        }
        // z-families: the flux through the z-face between q-1 and q
        const bool rz_f = inr(q, 0, n2), rz_fh = inr(q + 1, 0, n2);
        Flux dzx, dzy;
        {
            Face l = corner_state(qz_lo, dF1x, fx3, gm1, igm1, fb);  // (z|x)
            if (fb && hL && hR && rz_f && rx_c && ry_w) err |= fb;
            Flux Fzx = hllc(with_ri(c_zx_hi), l, 2, gamma, igm1);
            if (exb(7) && q >= T.z0 && rz_f) mf_put(7, q, Fzx.m);
            Face h = corner_state(qz_hi, dF1x, fx3, gm1, igm1, fb);
            if (fb && hL && hR && rz_fh && rx_c && ry_w) err |= fb;
            c_zx_hi = h;
            c_zx_hi.ri = 0.0;
            l = corner_state(qz_lo, dF1y, fy3, gm1, igm1, fb);  // (z|y)
            if (fb && hD && hU && rz_f && ry_c && rx_w) err |= fb;
            Flux Fzy = hllc(with_ri(c_zy_hi), l, 2, gamma, igm1);
            if (exb(8) && q >= T.z0 && rz_f) mf_put(8, q, Fzy.m);
            h = corner_state(qz_hi, dF1y, fy3, gm1, igm1, fb);
            if (fb && hD && hU && rz_fh && ry_c && rx_w) err |= fb;
            c_zy_hi = h;
            c_zy_hi.ri = 0.0;
            // z-differences of the (z|s) fluxes of plane q-1
            dzx = fdiff(Fzx, F2zx);
            dzy = fdiff(Fzy, F2zy);
            F2zx = Fzx;
            F2zy = Fzy;
        }
        __syncthreads();
        // ---------------------------------------------------- final states
        // the traced x/y states of plane q-1 for its final states, fetched
        // before the final z state of plane q is formed so that their
        // latency hides behind it (lanes whose final x or y states are never
        // used skip them: the ring rows for x, the ring columns for y, and
        // every lane in a segment's warm-up plane)
        const int p = q - 1;
        const bool pv = p >= T.z0;  // plane p is finished in this segment
        const bool rp_c = inr(p, 0, n2 - 1);
        Face pxl = {}, pxh = {}, pyl = {}, pyh = {};
        {
            gchar *pp = opaque_plane(ws.plane(p));
            if (pv && hD && hU) {
                pxl = load_face_b(pp, wo, QLO(0, 0));
                pxh = load_face_b(pp, wo, QHI(0, 0));
            }
            if (pv && hL && hR) {
                pyl = load_face_b(pp, wo, QLO(1, 0));
                pyh = load_face_b(pp, wo, QHI(1, 0));
            }
        }
        // final z state of plane q
        const Flux dyx = fdiff(getX(yb.v, 0, tU), getX(yb.v, 0, t));
        const bool zin = hL && hR && hD && hU && rx_c && ry_c;
        Face zl = final_state2(qz_lo, dxy, dyx, fx2, fy2, gm1, igm1, fb);
        if (fb && zin && rz_f) err |= fb;
        Face zh = final_state2(qz_hi, dxy, dyx, fx2, fy2, gm1, igm1, fb);
        if (fb && zin && rz_fh) err |= fb;
        const Flux F3zq = hllc(with_ri(fz_hi), zl, 2, gamma, igm1);
        if (exb(11) && q >= T.z0 && rz_f) mf_put(11, q, F3zq.m);
        fz_hi = zh;
        fz_hi.ri = 0.0;
        // y-difference of the (y|z) fluxes of plane q (used next plane)
        const Flux dyz = fdiff(getX(yb.v, 5, tU), getX(yb.v, 5, t));
        // final x and y states of plane q-1
        Face xl, xh, yl, yh;
        {
            const Face a = pxl, b = pxh;
            const Flux dF2yz = getX(cz, 5, t);
            xl = final_state2(a, dF2yz, dzy, fy2, fz2, gm1, igm1, fb);
            if (fb && pv && hD && hU && rx_f && ry_c && rp_c) err |= fb;
            xh = final_state2(b, dF2yz, dzy, fy2, fz2, gm1, igm1, fb);
            if (fb && pv && hD && hU && rx_fh && ry_c && rp_c) err |= fb;
        }
        {
            const Face a = pyl, b = pyh;
            const Flux dF2xz = getX(cz, 0, t);
            yl = final_state2(a, dF2xz, dzx, fx2, fz2, gm1, igm1, fb);
            if (fb && pv && hL && hR && ry_f && rx_c && rp_c) err |= fb;
            yh = final_state2(b, dF2xz, dzx, fx2, fz2, gm1, igm1, fb);
            if (fb && pv && hL && hR && ry_fh && rx_c && rp_c) err |= fb;
        }
        putX(cz, 0, t, dxz);
        putX(cz, 5, t, dyz);
        // ---------------------------------------------------- round-3 in-plane fluxes
        putF(ya.v, 0, t, yh);
        ya.v[5][t] = yh.ri;  // the upper neighbour takes yh with its 1/rho
        // x: the low neighbour's high state from the neighbour lane; the
        // flux difference over the cell, times dt/dx, right away
        Flux dux;
        {
            const Flux F3x = hllc(prevF(xh), xl, 0, gamma, igm1);
            if (exb(9) && pv && rp_c) mf_put(9, p, F3x.m);
            const Flux d = next_minus(F3x);
            dux.m = ax * d.m;
            dux.mu = ax * d.mu;
            dux.mv = ax * d.mv;
            dux.mw = ax * d.mw;
            dux.e = ax * d.e;
        }
        __syncthreads();
        {
            Face yd = getF_raw(ya.v, 0, tD);
            yd.ri = ya.v[5][tD];
            const Flux F3y = hllc(yd, yl, 1, gamma, igm1);
            putX(yb.v, 0, t, F3y);
            if (exb(10) && pv && rp_c) mf_put(10, p, F3y.m);
        }
        __syncthreads();
        // ---------------------------------------------------- update plane p
        if (outc && pv) {
            const Flux dy = fdiff(getX(yb.v, 0, tU), getX(yb.v, 0, t));
            const Flux F3z = getX(cz, 10, t);
            const double dxv[5] = {dux.m, dux.mu, dux.mv, dux.mw, dux.e};
            const double dyv[5] = {dy.m, dy.mu, dy.mv, dy.mw, dy.e};
            const double Fz[5][2] = {{F3z.m, F3zq.m}, {F3z.mu, F3zq.mu}, {F3z.mv, F3zq.mv},
                                     {F3z.mw, F3zq.mw}, {F3z.e, F3zq.e}};
            const unsigned bo = (unsigned)cell(g, x, y, p) * 8u;
            double Uo[5], Us[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                double du = dxv[v];
                du = du + ay * dyv[v];
                du = du + az * (Fz[v][1] - Fz[v][0]);
                Uo[v] = ldb(o.U + v * g.cs, bo);
                Us[v] = Uo[v] - du;
            }
            const double h = 0.5 * dt;
            const double gg[3] = {gx, gy, gz};
#pragma unroll
            for (int e = 0; e < 3; ++e)
                if (gg[e] != 0.0) {
                    double hg = h * gg[e];
                    double mnew = Us[1 + e] + hg * (Uo[0] + Us[0]);
                    Us[4] = Us[4] + hg * (Uo[1 + e] + mnew);
                    Us[1 + e] = mnew;
                }
            Prim qn = prim_of(Us[0], Us[1], Us[2], Us[3], Us[4], gm1);
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                if (!isfinite(Us[v])) err |= HYDRO_ERR_NONFINITE;
                stb64(o.Un + v * g.cs, bo, Us[v]);
            }
            if (Us[0] <= 0.0) err |= HYDRO_ERR_RHO;
            if (qn.p <= 0.0) err |= HYDRO_ERR_P;
            if (o.dtn) dtn = dmin(dtn, cfl_cell(qn, gamma, g.dx));
        }
        putX(cz, 10, t, F3zq);
    }
    if (err && act) atomicOr(err_dev, err);
    // (every lane has passed the z-march's last barrier, and the last reads
    // of ya happened before it: ya is free)
    if (o.dtn) block_dt_min(dtn, cfl, o.dtn, L.dtn_min, ya.v[0]);
}

}  // namespace
