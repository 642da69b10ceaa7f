// flatten.h -- shock-flattening coefficients (Colella & Woodward 1984,
// Sec. 4) of the traced cells of a box, read by the trace kernel when
// flattening is on.
//
// Along one axis, a cell lies in a shock when the flow converges across it
// (u[i-1] - u[i+1] > 0) and the pressure jumps across it by more than
// kFlEps of the smaller neighbouring pressure; the steepness
// z = |p[i+1]-p[i-1]| / |p[i+2]-p[i-2]| (about 1/2 in a smooth profile, near 1
// in a shock two cells wide) then gives chi = clamp(kFlW2 (z - kFlW1), 0, 1),
// else chi = 0.  The axis coefficient is 1 - max(chi[i], chi[i+s]) with s
// toward the lower-pressure neighbour (the cell just behind a shock is
// flattened with it), and the cell's coefficient is the smallest of its three
// axes' (x, then y, then z).  Computed for every traced cell (x in [-1,n0],
// y in [-1,n1], z in [-1,n2]); the 7-cell pencils reach four cells out, into
// the fourth ghost layer.
#pragma once

namespace {

constexpr double kFlW1 = 0.75, kFlW2 = 10.0, kFlEps = 0.33, kFlTiny = 1e-300;

// the coefficient of the centre of a 7-cell pencil (cells i-3 .. i+3) of
// pressures p and velocities u along the pencil's axis
__device__ __forceinline__ double flat_axis(const double (&p)[7], const double (&u)[7])
{
    double chi[3];  // cells i-1, i, i+1
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const double dp = p[m + 3] - p[m + 1];
        const double dp2 = p[m + 4] - p[m];
        const double z = fabs(dp) / dmax(fabs(dp2), kFlTiny);
        const double c = dmin(1.0, dmax(0.0, kFlW2 * (z - kFlW1)));
        const bool shock = u[m + 1] - u[m + 3] > 0.0 && fabs(dp) > kFlEps * dmin(p[m + 3], p[m + 1]);
        chi[m] = shock ? c : 0.0;
    }
    const double nb = p[4] > p[2] ? chi[0] : chi[2];
    return 1.0 - dmax(chi[1], nb);
}

// Tiles: a 256-thread block covers kFlB x kFlB columns of the traced region
// and marches over a z-segment of at most kFlZ planes.  Each plane's
// pressures and in-plane velocities, on the tile plus a three-cell ring, are
// converted from U once into LDS (the x and y pencils read them there); each
// column carries its own z-pencil (pressure and normal velocity of the
// planes z-3 .. z+3) in registers.  The conserved values of the next plane
// (the thread's ring cells and its column's cell three planes ahead) are
// fetched one z-step ahead, so their latency overlaps the current plane.
constexpr int kFlW = kFlB + 6;

__global__ void __launch_bounds__(kBlock) k_flatten(Launch L, double gamma)
{
    __shared__ double sp[kFlW * kFlW], su[kFlW * kFlW], sv[kFlW * kFlW];
    Box1 o = resolve(L);
    const Geo &g = o.g;
    const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2], ng = g.ng;
    const int ntx = (n0 + 2 + kFlB - 1) / kFlB, nty = (n1 + 2 + kFlB - 1) / kFlB;
    // blocks are dealt to the 8 XCDs round-robin: give each XCD a contiguous
    // run of tiles, so neighbouring tiles, which read each other's ring
    // cells, share that XCD's L2
    long long tt;
    {
        const long long per = o.nblk / 8, rem = o.nblk % 8;
        const long long xx = o.blk % 8, ii = o.blk / 8;
        tt = xx * per + (xx < rem ? xx : rem) + ii;
    }
    const int ix = (int)(tt % ntx);
    tt /= ntx;
    const int iy = (int)(tt % nty);
    const int iz = (int)(tt / nty);
    const int x0 = -1 + ix * kFlB, y0 = -1 + iy * kFlB;
    // the traced planes [-1, n2+1) in equal z-segments (as many as planes of
    // kFlZ need), each marched by one block
    const int nseg = (n2 + 2 + kFlZ - 1) / kFlZ, seg = (n2 + 2 + nseg - 1) / nseg;
    const int z0 = -1 + iz * seg, z1 = min(n2 + 1, z0 + seg);
    const int t = threadIdx.x, tx = t % kFlB, ty = t / kFlB;
    const int x = x0 + tx, y = y0 + ty;
    const bool inner = x <= n0 && y <= n1;
    const double gm1 = gamma - 1.0;
    // byte offset of a cell, its coordinates clamped into the ghosted box
    // (clamped cells only feed lanes whose results are not stored; one
    // component of a box is below 2 GiB)
    auto off_at = [&](int i, int j, int k) {
        i = min(max(i, -ng), n0 + ng - 1);
        j = min(max(j, -ng), n1 + ng - 1);
        k = min(max(k, -ng), n2 + ng - 1);
        return (unsigned)cell(g, i, j, k) * 8u;
    };
    auto load5 = [&](unsigned bo, double (&c)[5]) {
#pragma unroll
        for (int v = 0; v < 5; ++v) c[v] = ldb(o.U + v * g.cs, bo);
    };
    auto prim5 = [&](const double (&c)[5]) { return prim_of(c[0], c[1], c[2], c[3], c[4], gm1); };
    // the ring cells of a plane this thread converts: t and t + 256 (of 484)
    constexpr int kRing = kFlW * kFlW;
    static_assert(kRing <= 2 * kBlock, "two ring cells per thread");
    const int r1 = t + kBlock;
    const bool has1 = r1 < kRing;
    const int rx0 = x0 - 3 + t % kFlW, ry0 = y0 - 3 + t / kFlW;
    const int rx1 = x0 - 3 + r1 % kFlW, ry1 = y0 - 3 + r1 / kFlW;
    double c0[5], c1[5], cz[5];  // next plane: ring cells, own column's cell
    auto fetch = [&](int z) {
        load5(off_at(rx0, ry0, z), c0);
        if (has1) load5(off_at(rx1, ry1, z), c1);
        load5(off_at(x, y, z + 3), cz);
    };
    // own column's z-pencil: pressure and z-velocity of planes z-3 .. z+3
    double zp[7], zw[7];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        double c[5];
        load5(off_at(x, y, z0 - 3 + m), c);
        const Prim q = prim5(c);
        zp[m] = q.p;
        zw[m] = q.w;
    }
    fetch(z0);
    for (int z = z0; z < z1; ++z) {
        {
            Prim q = prim5(c0);
            sp[t] = q.p;
            su[t] = q.u;
            sv[t] = q.v;
            if (has1) {
                q = prim5(c1);
                sp[r1] = q.p;
                su[r1] = q.u;
                sv[r1] = q.v;
            }
            q = prim5(cz);
            zp[6] = q.p;
            zw[6] = q.w;
        }
        if (z + 1 < z1) fetch(z + 1);
        __syncthreads();
        const int rc = (ty + 3) * kFlW + (tx + 3);
        double px[7], ux[7], py[7], vy[7];
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            px[m] = sp[rc + (m - 3)];
            ux[m] = su[rc + (m - 3)];
            py[m] = sp[rc + (m - 3) * kFlW];
            vy[m] = sv[rc + (m - 3) * kFlW];
        }
        double f = 1.0;
        f = dmin(f, flat_axis(px, ux));
        f = dmin(f, flat_axis(py, vy));
        f = dmin(f, flat_axis(zp, zw));
        if (inner)
            o.flat[((long long)(z + 1) * (n1 + 2) + (y + 1)) * (n0 + 2) + (x + 1)] = f;
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            zp[m] = zp[m + 1];
            zw[m] = zw[m + 1];
        }
        __syncthreads();
    }
}

}  // namespace
