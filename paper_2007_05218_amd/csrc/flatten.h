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
// axes'.  One thread per traced cell (x in [-1,n0], y in [-1,n1],
// z in [-1,n2]); the 7-cell pencils reach four cells out, into the fourth
// ghost layer.
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

__global__ void __launch_bounds__(kBlock) k_flatten(Launch L, double gamma)
{
    Box1 o = resolve(L);
    const Geo &g = o.g;
    const long long ex0 = g.n[0] + 2, ex1 = g.n[1] + 2, ex2 = g.n[2] + 2;
    const long long t = o.blk * kBlock + threadIdx.x;
    if (t >= ex0 * ex1 * ex2) return;
    const int x = (int)(t % ex0) - 1;
    const int y = (int)((t / ex0) % ex1) - 1;
    const int z = (int)(t / (ex0 * ex1)) - 1;
    const double gm1 = gamma - 1.0;
    const double *U = o.U;
    const long long c0 = cell(g, x, y, z);
    double f = 1.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const long long st = stride(g, d);
        double p[7], u[7];
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            const long long c = c0 + (m - 3) * st;
            const Prim q = prim_of(U[c], U[g.cs + c], U[2 * g.cs + c], U[3 * g.cs + c],
                                   U[4 * g.cs + c], gm1);
            p[m] = q.p;
            u[m] = d == 0 ? q.u : (d == 1 ? q.v : q.w);
        }
        f = dmin(f, flat_axis(p, u));
    }
    o.flat[t] = f;
}

}  // namespace
