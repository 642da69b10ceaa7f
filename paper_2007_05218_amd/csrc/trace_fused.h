// trace_fused.h -- the first half of the CTU step in one kernel: primitive
// variables, PPM reconstruction and characteristic tracing in all three
// directions (with the half-step gravity kick), for one box tile, marching
// along z.
//
// Output (HBM workspace): the traced face states of every cell one beyond
// the valid region -- the input of the fused flux kernel, which also solves
// the round-1 Riemann problems from them (a round-1 flux costs less to
// compute there than its five doubles cost to store here and read back
// there).  Each cell's primitives are computed once per block: a plane of
// the tile plus a two-cell ring enters an LDS ring of three planes (the x/y
// stencils read the centre plane from it) and each column marches its own
// z-direction PPM, one new slope and interface value per plane.  This is the
// one-zone-per-thread stencil of the paper's Sec. III with the neighbouring
// primitives staged on chip instead of re-read and re-converted from global
// memory.
//
// Tile: a 256-thread block covers BX x BY output columns
// [x0, x0+BX) x [y0, y0+BY) of the traced region and marches over its
// planes [z0, z1).
#pragma once

namespace {

constexpr int kTT = 256;      // threads of a fused-trace block
constexpr int kTPlane = 432;  // LDS cells of one plane: (BX+4)(BY+4) <= 432 for BX in {8,16,18,32}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// a traced state into fields f0 .. f0+4 of the column at offset lo of plane pp
__device__ __forceinline__ void stb(const char *pp, unsigned lo, int f0, const Face &f)
{
    ws_st(pp, lo, f0 + 0, f.r);
    ws_st(pp, lo, f0 + 1, f.u);
    ws_st(pp, lo, f0 + 2, f.v);
    ws_st(pp, lo, f0 + 3, f.w);
    ws_st(pp, lo, f0 + 4, f.p);
}

// FLAT: apply each traced cell's shock-flattening coefficient (computed by
// k_flatten into the workspace) to its fifteen parabolae
template <bool FLAT>
__global__ void __launch_bounds__(kTT) __attribute__((amdgpu_waves_per_eu(3)))
k_trace_fused(Launch L, double gamma, double gx, double gy, double gz)
{
    __shared__ double pl[3][5][kTPlane];  // primitive planes (rho, u, v, w, p), ring of 3
    Box1 o = resolve(L);
    const Geo &g = o.g;
    const WS &ws = o.ws;
    if (o.blk == 0 && threadIdx.x == 0) {
        // the next step's timestep, which the flux kernel (launched after
        // this one) reduces into, starts at +inf
        if (o.dtn) *o.dtn = kInfBits;
        if (L.dtn_min && o.b == 0) *L.dtn_min = kInfBits;
    }
    const int BX = g.tbx1, BY = kTT / g.tbx1;
    const int RW = BX + 4, RH = BY + 4;
    const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2], ng = g.ng;
    // tiles cover the traced region [-1, n+1) of each axis
    const int ntx = (n0 + 2 + BX - 1) / BX, nty = (n1 + 2 + BY - 1) / BY;
    long long tt;
    {
        long long per = o.nblk / 8, rem = o.nblk % 8;
        long long xx = o.blk % 8, ii = o.blk / 8;
        tt = xx * per + (xx < rem ? xx : rem) + ii;
    }
    const int ix = (int)(tt % ntx);
    tt /= ntx;
    const int iy = (int)(tt % nty);
    const int iz = (int)(tt / nty);
    const int x0 = -1 + ix * BX, y0 = -1 + iy * BY;
    const int zs = seg_len(n2 + 2, g.tzs1);
    const int z0 = -1 + iz * zs, z1 = min(n2 + 1, z0 + zs);

    const int t = threadIdx.x;
    const int tx = t % BX, ty = t / BX;
    const int x = x0 + tx, y = y0 + ty;  // this thread's column
    // (with BX = 18 the tile has 14 rows, 252 of the 256 threads; the other
    // four only keep the block's barriers)
    const bool inner = x <= n0 && y <= n1 && t < BX * BY;
    const int rc = (ty + 2) * RW + (tx + 2);  // own column in the plane buffer
    const unsigned wo = ws.off(inner ? x : n0, inner ? y : n1);  // own column in the workspace

    const double dt = *o.dt;
    const double dtdx = dt / g.dx[0], dtdy = dt / g.dx[1], dtdz = dt / g.dx[2];
    const double h = 0.5 * dt;
    const double gm1 = gamma - 1.0;

    // Region plane of prims: cells (x0-2 .. x0+BX+1) x (y0-2 .. y0+BY+1) of
    // plane z, indices clamped into the ghosted box (clamped cells feed only
    // unused lanes).  Each thread owns region cells t and t+256; their
    // conserved values are fetched one plane ahead into registers so the
    // global-memory latency overlaps the tracing of the current plane.
    const int nreg = RW * RH;
    double pf[2][5];
    auto fetch = [&](int z) {
        const int zc = clampi(z, -ng, n2 + ng - 1);
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const int r = t + m * kTT;
            if (r < nreg) {
                const int rx = r % RW, ry = r / RW;
                const int cx = clampi(x0 - 2 + rx, -ng, n0 + ng - 1);
                const int cy = clampi(y0 - 2 + ry, -ng, n1 + ng - 1);
                const unsigned bo = (unsigned)cell(g, cx, cy, zc) * 8u;
#pragma unroll
                for (int v = 0; v < 5; ++v) pf[m][v] = ldb(o.U + v * g.cs, bo);
            }
        }
    };
    auto commit = [&](int z) {
        const int slot = (z + 6) % 3;
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const int r = t + m * kTT;
            if (r < nreg) {
                Prim q = prim_of(pf[m][0], pf[m][1], pf[m][2], pf[m][3], pf[m][4], gm1);
                pl[slot][0][r] = q.r;
                pl[slot][1][r] = q.u;
                pl[slot][2][r] = q.v;
                pl[slot][3][r] = q.w;
                pl[slot][4][r] = q.p;
            }
        }
    };

    // z-direction PPM of the own column (rho, u, v, w, p), marched with the
    // planes; started from planes z0-2 .. z0+1
    PPMColumn zr, zu, zv, zw, zp;
    {
        double c0[4][5];
        for (int z = z0 - 2; z <= z0 + 1; ++z) {
            fetch(z);
            commit(z);
            __syncthreads();
            const int slot = (z + 6) % 3;
#pragma unroll
            for (int v = 0; v < 5; ++v) c0[z - (z0 - 2)][v] = pl[slot][v][rc];
            __syncthreads();
        }
        zr.init(c0[0][0], c0[1][0], c0[2][0], c0[3][0]);
        zu.init(c0[0][1], c0[1][1], c0[2][1], c0[3][1]);
        zv.init(c0[0][2], c0[1][2], c0[2][2], c0[3][2]);
        zw.init(c0[0][3], c0[1][3], c0[2][3], c0[3][3]);
        zp.init(c0[0][4], c0[1][4], c0[2][4], c0[3][4]);
    }
    fetch(z0 + 2);

    for (int p = z0; p < z1; ++p) {
        commit(p + 2);
        if (p + 1 < z1) fetch(p + 3);
        __syncthreads();
        // the cell's own primitives, and its z-parabolae given plane p+2
        const double rho = zr.a, wz = zw.a;
        const double ri = 1.0 / rho;  // as the cell's primitive conversion forms it
        const double c = sound_ri(gamma, zp.a, ri);
        double fl = 1.0;
        if (FLAT && inner)
            fl = o.flat[((long long)(p + 1) * (n1 + 2) + (y + 1)) * (n0 + 2) + (x + 1)];
        Parab Pr, Pu, Pv, Pw, Pp;
        {
            const int slot = (p + 2 + 6) % 3;
            Pr = zr.step(pl[slot][0][rc], fl);
            Pu = zu.step(pl[slot][1][rc], fl);
            Pv = zv.step(pl[slot][2][rc], fl);
            Pw = zw.step(pl[slot][3][rc], fl);
            Pp = zp.step(pl[slot][4][rc], fl);
        }
        const int slot = (p + 6) % 3;
        Face hi, lo;
        const char *pp = ws.plane(p);
        // ------------------------------------------------ z trace
        trace_parab(Pr, Pw, Pu, Pv, Pp, rho, wz, c, ri, 2, dtdz, hi, lo);
        if (gx != 0.0) { hi.u = hi.u + h * gx; lo.u = lo.u + h * gx; }
        if (gy != 0.0) { hi.v = hi.v + h * gy; lo.v = lo.v + h * gy; }
        if (gz != 0.0) { hi.w = hi.w + h * gz; lo.w = lo.w + h * gz; }
        if (inner) {
            stb(pp, wo, QHI(2, 0), hi);
            stb(pp, wo, QLO(2, 0), lo);
        }
        // ------------------------------------------------ x and y traces of plane p
        {
            double rs[5], a1[5], a2[5], a3[5], ps[5];
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                const int r = rc + (m - 2);
                rs[m] = pl[slot][0][r];
                a1[m] = pl[slot][1][r];
                a2[m] = pl[slot][2][r];
                a3[m] = pl[slot][3][r];
                ps[m] = pl[slot][4][r];
            }
            trace_cell(rs, a1, a2, a3, ps, c, ri, 0, dtdx, hi, lo, fl);
        }
        if (gx != 0.0) { hi.u = hi.u + h * gx; lo.u = lo.u + h * gx; }
        if (gy != 0.0) { hi.v = hi.v + h * gy; lo.v = lo.v + h * gy; }
        if (gz != 0.0) { hi.w = hi.w + h * gz; lo.w = lo.w + h * gz; }
        if (inner) {
            stb(pp, wo, QHI(0, 0), hi);
            stb(pp, wo, QLO(0, 0), lo);
        }
        {
            double rs[5], a1[5], a2[5], a3[5], ps[5];
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                const int r = rc + (m - 2) * RW;
                rs[m] = pl[slot][0][r];
                a1[m] = pl[slot][2][r];
                a2[m] = pl[slot][1][r];
                a3[m] = pl[slot][3][r];
                ps[m] = pl[slot][4][r];
            }
            trace_cell(rs, a1, a2, a3, ps, c, ri, 1, dtdy, hi, lo, fl);
        }
        if (gx != 0.0) { hi.u = hi.u + h * gx; lo.u = lo.u + h * gx; }
        if (gy != 0.0) { hi.v = hi.v + h * gy; lo.v = lo.v + h * gy; }
        if (gz != 0.0) { hi.w = hi.w + h * gz; lo.w = lo.w + h * gz; }
        if (inner) {
            stb(pp, wo, QHI(1, 0), hi);
            stb(pp, wo, QLO(1, 0), lo);
        }
        __syncthreads();
    }
}

}  // namespace
