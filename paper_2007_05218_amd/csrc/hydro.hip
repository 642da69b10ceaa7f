// hydro.hip -- gfx950 kernels and the C ABI (include/hydro.h) of one
// CTU-PPM-HLLC hydro step on boxes with ghost cells.
//
// The step's stages (the method's A0-A8) run in a few fused launches, each
// covering one box or a whole batch of boxes:
//   k_fill         ghost cells of U from the boundary kinds (one pass: each
//                  axis maps independently, so edges and corners need no
//                  ordering)
//   k_dt           per-cell min_d dx_d/(|u_d|+c), wave64 shuffle -> LDS -> one
//                  64-bit atomicMin per block on the bit pattern (positive
//                  doubles order like unsigned integers), scaled by cfl; only
//                  for a state no advance produced
//   k_flatten      shock-flattening coefficients (flatten.h; only with
//                  flattening on)
//   k_trace_fused  primitives, PPM and characteristic tracing, both faces,
//                  each direction, on the cells one beyond the valid region,
//                  + half-step gravity kick (trace_fused.h); the traced
//                  states go to the caller's HBM workspace
//   k_flux_fused   round-1 HLLC, corner coupling (dt/3 transverse
//                  corrections) + round-2 HLLC, final states (dt/2) +
//                  round-3 HLLC, conservative update + time-centred gravity
//                  source + error bits, and the new state's CFL timestep
//                  (flux_fused.h); with species, also the mass flux of every
//                  Riemann solve
//   k_sp_fused     the species pass: the three rounds of the step for the
//                  mass fractions of passively advected species, carried by
//                  those mass fluxes, and the update of their partial
//                  densities, in one z-march (species_fused.h); k_sp_fill
//                  fills the species' ghosts (species.h)
//
// Batching: a plan lists, for every stage, a work list of the boxes and the
// prefix sum of their block counts; a block finds its box by binary search,
// so one launch per stage serves hundreds of uneven boxes (the per-box
// launches of the paper's Sec. IV-A replaced by one launch over the whole
// list).
#include "hydro_common.h"
#include "../../include/hydro.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <algorithm>
#include <mutex>
#include <vector>

using namespace hydro;

namespace {

constexpr int kBlock = 256;
constexpr unsigned long long kInfBits = 0x7FF0000000000000ULL;  // +inf as a bit pattern

struct Geo {
    int n[3];
    int ng;
    int s[3];
    long long cs;  // doubles per component (s0*s1*s2)
    double dx[3];
    int bc_lo[3], bc_hi[3];
    // tiles of the fused kernels (block = 256 threads = tbx x 256/tbx columns,
    // marching over z-segments of tzs planes): trace kernel, flux kernel
    int tbx1, tzs1, tbx2, tzs2;
};

// rows of a flux-kernel tile of width bx: 64 / bx whole rows per wavefront,
// four wavefronts (bx = 18: three rows of 18 lanes each, twelve rows)
__host__ __device__ constexpr int flux_rows(int bx) { return 4 * (64 / bx); }

// z-segments of a kernel over N planes with at most zs planes each, made
// equal: ceil(N / zs) segments of ceil(N / segments) planes (the last may be
// shorter; none is empty)
__host__ __device__ constexpr int seg_len(int N, int zs)
{
    return (N + (N + zs - 1) / zs - 1) / ((N + zs - 1) / zs);
}

// workspace fields: traced face states (direction d, high/low face,
// component v)
__host__ __device__ constexpr int QHI(int d, int v) { return d * 10 + v; }
__host__ __device__ constexpr int QLO(int d, int v) { return d * 10 + 5 + v; }
constexpr int kFields = 30;
constexpr int kXB = 16;  // cells of an x-block of the workspace
// byte offset of field f within a cell's slot of an x-block run (the cell's
// own offset is 16 bytes per cell): pair (axis, component), then face
__host__ __device__ constexpr int ws_foff(int f)
{
    return ((f / 10) * 5 + f % 5) * (kXB * 16) + ((f % 10) / 5) * 8;
}

// stages (block-count prefix arrays are kept per stage)
enum { ST_FILL = 0, ST_DT = 1, ST_TRACE = 2, ST_FLUX = 3, ST_FLAT = 4, ST_COUNT = 5 };
constexpr int kDtCellsPerThread = 4;
constexpr long long kDtMaxBlocks = 4096;


__device__ __forceinline__ long long cell(const Geo &g, int i, int j, int k)
{
    return ((long long)(k + g.ng) * g.s[1] + (j + g.ng)) * g.s[0] + (i + g.ng);
}

__device__ __forceinline__ long long stride(const Geo &g, int d)
{
    return d == 0 ? 1LL : (d == 1 ? (long long)g.s[0] : (long long)g.s[0] * g.s[1]);
}

// Workspace of one box: the traced face states of the cells x in [-1, n0],
// y in [-1, n1], z in [-2, n2+1] (the traced region plus one plane on each
// side that the flux kernel's first and last z-steps read and never use).
// Plane by plane, row by row, each run of 16 cells of a row (x-block) keeps
// its 30 fields together, as 15 pairs: the high- and low-face states of one
// component along one axis.  Pair k of the run is 16 cells x 16 bytes (two
// 128-byte lines) at k*256 bytes from the run's start, a cell's high-face
// value first, its low-face value beside it.  A lane's 30 fields are then one
// per-lane offset plus constant offsets from a per-plane base (no address
// register per field); the streams a kernel writes or reads at once are
// neighbouring lines instead of 30 arrays a large power of two apart, which
// land on the same memory channels; and the two states of a pair, which the
// kernels store and load together, move as one 16-byte access (half the
// memory instructions of one field per access).
__host__ __device__ __forceinline__ int ws_xblocks(int n0) { return (n0 + 2 + kXB - 1) / kXB; }
__host__ __device__ __forceinline__ long long ws_pitch(int n0, int n1)  // bytes per plane
{
    return (long long)(n1 + 2) * ws_xblocks(n0) * (kFields * kXB * 8);
}
// After the traced states, the workspace holds the shock-flattening
// coefficient of every traced cell (x in [-1, n0], y in [-1, n1],
// z in [-1, n2], x fastest), used only when flattening is on.
__host__ __device__ __forceinline__ long long ws_flat_off(int n0, int n1, int n2)  // bytes
{
    return (ws_pitch(n0, n1) * (n2 + 4) + 255) / 256 * 256;
}
struct WS {
    char *base;        // plane z = -2
    long long pitch;   // bytes per plane
    int nxb;           // x-blocks per row
    __device__ __forceinline__ const char *plane(int z) const
    {
        return base + (long long)(z + 2) * pitch;
    }
    // byte offset of column (x, y) within a plane
    __device__ __forceinline__ unsigned off(int x, int y) const
    {
        const unsigned X = (unsigned)(x + 1);
        return ((unsigned)(y + 1) * (unsigned)nxb + (X / kXB)) * (unsigned)(kFields * kXB * 8) +
               (X % kXB) * 16u;
    }
};
// field f of the column at byte offset lo of plane pointer pp
__device__ __forceinline__ double ws_ld(const char *pp, unsigned lo, int f)
{
    return *(const double *)((pp + (size_t)lo) + ws_foff(f));
}
__device__ __forceinline__ void ws_st(const char *pp, unsigned lo, int f, double v)
{
    // (streamed past the caches: the workspace is far larger than them and
    // is read back by the next kernel, not this one)
    __builtin_nontemporal_store(
        v, (__attribute__((address_space(1))) double *)((const_cast<char *>(pp) + (size_t)lo) +
                                                        ws_foff(f)));
}

struct Reg {
    int lo[3];
    int ext[3];
};

__host__ __device__ inline long long reg_count(const Reg &r)
{
    return (long long)r.ext[0] * r.ext[1] * r.ext[2];
}

__device__ __forceinline__ bool reg_cell(const Reg &r, long long t, int &i, int &j, int &k)
{
    if (t < 0 || t >= reg_count(r)) return false;
    i = r.lo[0] + (int)(t % r.ext[0]);
    t /= r.ext[0];
    j = r.lo[1] + (int)(t % r.ext[1]);
    k = r.lo[2] + (int)(t / r.ext[1]);
    return true;
}

// tiles of the flattening kernel (flatten.h): kFlB x kFlB columns of the
// traced region, z-segments of kFlZ planes
constexpr int kFlB = 16, kFlZ = 32;

// blocks of one box in a stage
__host__ inline long long stage_blocks(const Geo &g, int st)
{
    if (st == ST_TRACE) {  // tiles of tbx x 256/tbx columns over [-1, n+1)
        const long long TX = g.tbx1, TY = 256 / g.tbx1;
        return ((g.n[0] + 2 + TX - 1) / TX) * ((g.n[1] + 2 + TY - 1) / TY) *
               ((g.n[2] + 2 + g.tzs1 - 1) / g.tzs1);
    }
    if (st == ST_FLUX) {  // tiles of (tbx-2) x (rows-2) columns over [0, n)
        const long long TX = g.tbx2 - 2, TY = flux_rows(g.tbx2) - 2;
        return ((g.n[0] + TX - 1) / TX) * ((g.n[1] + TY - 1) / TY) *
               ((g.n[2] + g.tzs2 - 1) / g.tzs2);
    }
    const long long nv = (long long)g.n[0] * g.n[1] * g.n[2];
    if (st == ST_FLAT)
        return (long long)((g.n[0] + 2 + kFlB - 1) / kFlB) * ((g.n[1] + 2 + kFlB - 1) / kFlB) *
               ((g.n[2] + 2 + kFlZ - 1) / kFlZ);
    long long items = st == ST_FILL ? g.cs - nv : nv;
    if (st == ST_DT) {
        long long b = (items + (long long)kBlock * kDtCellsPerThread - 1) /
                      ((long long)kBlock * kDtCellsPerThread);
        return b < 1 ? 1 : (b > kDtMaxBlocks ? kDtMaxBlocks : b);
    }
    return (items + kBlock - 1) / kBlock;
}

// ---------------------------------------------------------------- launch args

// One launch covers either a single box (nb == 0; everything by value) or a
// batch (nb >= 1; per-box data in device arrays of a plan).
struct Launch {
    // single box
    Geo g;
    const double *U;
    double *Un;
    double *ws;
    const double *dt;
    // batch
    int nb;
    const Geo *geos;
    const unsigned *pre;  // this stage's block prefix, nb+1 entries
    const double *const *Us;
    double *const *Uns;
    const long long *wsoff;  // doubles from the workspace base
    const double *dts;
    int dt_stride;
    const int *order;  // box of each work-list position (null: the identity)
    // optional: the CFL timestep of the new state, reduced by the flux kernel
    // (per box, as 64-bit patterns for atomicMin) and the minimum over boxes
    unsigned long long *dtn;
    unsigned long long *dtn_min;
};

// Faces and cells of the index box [-1, n0] x [-1, n1] x [-1, n2] (faces
// named by the cell above them): the layout of the mass-flux export, each
// field padded to 256 bytes.
__host__ __device__ inline long long mf_stride(int n0, int n1, int n2)
{
    return ((long long)(n0 + 2) * (n1 + 2) * (n2 + 2) + 31) / 32 * 32;
}
__host__ __device__ inline long long mf_index(int n0, int n1, int x, int y, int z)
{
    return ((long long)(z + 1) * (n1 + 2) + (y + 1)) * (n0 + 2) + (x + 1);
}

struct Box1 {
    Geo g;
    const double *U;
    double *Un;
    WS ws;
    const double *dt;
    int b;            // box index within the batch (0 for a single box)
    long long blk;    // block index within the box
    long long nblk;   // blocks of this box in this stage
    unsigned long long *dtn;  // this box's next-step timestep (bit pattern), or null
    double *flat;             // this box's flattening coefficients (workspace), or null
};

__device__ __forceinline__ Box1 resolve(const Launch &L)
{
    Box1 o;
    if (L.nb == 0) {
        o.g = L.g;
        o.U = L.U;
        o.Un = L.Un;
        o.ws.base = (char *)L.ws;
        o.dt = L.dt;
        o.b = 0;
        o.blk = blockIdx.x;
        o.nblk = gridDim.x;
    } else {
        // largest b with pre[b] <= blockIdx.x
        int lo = 0, hi = L.nb;
        const unsigned x = blockIdx.x;
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (L.pre[mid] <= x) lo = mid;
            else hi = mid;
        }
        const int b = L.order ? L.order[lo] : lo;
        o.b = b;
        o.g = L.geos[b];
        o.U = L.Us ? L.Us[b] : nullptr;
        o.Un = L.Uns ? L.Uns[b] : nullptr;
        o.ws.base = L.ws ? (char *)(L.ws + L.wsoff[b]) : nullptr;
        o.dt = L.dts ? L.dts + (long long)b * L.dt_stride : nullptr;
        o.blk = x - L.pre[lo];
        o.nblk = L.pre[lo + 1] - L.pre[lo];
    }
    o.dtn = L.dtn ? L.dtn + o.b : nullptr;
    o.ws.pitch = ws_pitch(o.g.n[0], o.g.n[1]);
    o.ws.nxb = ws_xblocks(o.g.n[0]);
    o.flat = o.ws.base ? (double *)(o.ws.base + ws_flat_off(o.g.n[0], o.g.n[1], o.g.n[2]))
                       : nullptr;
    return o;
}

// ---------------------------------------------------------------- ghost fill

__device__ __forceinline__ int ghost_src(int g, int n, int bl, int bh, int &flip)
{
    if (g < 0) {
        int m = -1 - g;
        if (bl == HYDRO_BC_PERIODIC) return n - 1 - m;
        if (bl == HYDRO_BC_OUTFLOW) return 0;
        flip = 1;
        return m;
    }
    if (g >= n) {
        int m = g - n;
        if (bh == HYDRO_BC_PERIODIC) return m;
        if (bh == HYDRO_BC_OUTFLOW) return n - 1;
        flip = 1;
        return n - 1 - m;
    }
    return g;
}

// dt_bits (per box, may be null) and dtmin_bits (may be null) are reset to
// +inf here so the following dt launch can min-reduce into them
__global__ void __launch_bounds__(kBlock) k_fill(Launch L, unsigned long long *dt_bits,
                                                 unsigned long long *dtmin_bits)
{
    Box1 o = resolve(L);
    const Geo &g = o.g;
    double *U = const_cast<double *>(o.U);
    long long t = o.blk * kBlock + threadIdx.x;
    if (t == 0) {
        if (dt_bits) dt_bits[o.b] = kInfBits;
        if (dtmin_bits && o.b == 0) *dtmin_bits = kInfBits;
    }
    const long long s0 = g.s[0], s1 = g.s[1];
    const long long ng2 = 2LL * g.ng;
    const long long cz = ng2 * s1 * s0;
    const long long cy = (long long)g.n[2] * ng2 * s0;
    const long long cx = (long long)g.n[2] * g.n[1] * ng2;
    if (t >= cz + cy + cx) return;
    int i, j, k;
    if (t < cz) {
        i = (int)(t % s0) - g.ng;
        t /= s0;
        j = (int)(t % s1) - g.ng;
        int kk = (int)(t / s1);
        k = kk < g.ng ? kk - g.ng : g.n[2] + (kk - g.ng);
    } else if (t < cz + cy) {
        t -= cz;
        i = (int)(t % s0) - g.ng;
        t /= s0;
        int jj = (int)(t % ng2);
        j = jj < g.ng ? jj - g.ng : g.n[1] + (jj - g.ng);
        k = (int)(t / ng2);
    } else {
        t -= cz + cy;
        int ii = (int)(t % ng2);
        i = ii < g.ng ? ii - g.ng : g.n[0] + (ii - g.ng);
        t /= ng2;
        j = (int)(t % g.n[1]);
        k = (int)(t / g.n[1]);
    }
    int fx = 0, fy = 0, fz = 0;
    int si = ghost_src(i, g.n[0], g.bc_lo[0], g.bc_hi[0], fx);
    int sj = ghost_src(j, g.n[1], g.bc_lo[1], g.bc_hi[1], fy);
    int sk = ghost_src(k, g.n[2], g.bc_lo[2], g.bc_hi[2], fz);
    const long long dst = cell(g, i, j, k), src = cell(g, si, sj, sk);
    U[dst] = U[src];
    double mu = U[g.cs + src], mv = U[2 * g.cs + src], mw = U[3 * g.cs + src];
    U[g.cs + dst] = fx ? -mu : mu;
    U[2 * g.cs + dst] = fy ? -mv : mv;
    U[3 * g.cs + dst] = fz ? -mw : mw;
    U[4 * g.cs + dst] = U[4 * g.cs + src];
}

// ---------------------------------------------------------------- dt

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = dmin(v, __shfl_xor(v, o, 64));
    return v;
}

// the CFL bound of one cell: min_d dx_d / (|u_d| + c)
__device__ __forceinline__ double cfl_cell(const Prim &q, double gamma, const double (&dx)[3])
{
    double c = sound_ri(gamma, q.p, q.ri);
    double a = dx[0] / (fabs(q.u) + c);
    double b = dx[1] / (fabs(q.v) + c);
    double e = dx[2] / (fabs(q.w) + c);
    return dmin(dmin(a, b), e);
}

// cfl times the minimum of m over a 256-thread block, atomically min-ed into
// *box_bits and (if not null) *min_bits as 64-bit patterns (positive doubles
// order like their bit patterns).  fl(cfl*x) is monotone in x, so the min of
// the scaled block minima is the scaled global minimum, bit for bit, in any
// order.  Every thread of the block must call it; part is LDS scratch for
// kBlock/64 doubles that no thread uses meanwhile.
__device__ __forceinline__ void block_dt_min(double m, double cfl, unsigned long long *box_bits,
                                             unsigned long long *min_bits, double *part)
{
    m = wave_min(m);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) part[wid] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = part[0];
        for (int w = 1; w < kBlock / 64; ++w) b = dmin(b, part[w]);
        unsigned long long v = (unsigned long long)__double_as_longlong(cfl * b);
        atomicMin(box_bits, v);
        if (min_bits) atomicMin(min_bits, v);
    }
}

__global__ void __launch_bounds__(kBlock) k_dt(Launch L, double gamma, double cfl,
                                               unsigned long long *dt_bits,
                                               unsigned long long *dtmin_bits)
{
    Box1 o = resolve(L);
    const Geo &g = o.g;
    const double *U = o.U;
    const double gm1 = gamma - 1.0;
    const long long nvalid = (long long)g.n[0] * g.n[1] * g.n[2];
    double m = __longlong_as_double((long long)kInfBits);
    for (long long t = o.blk * kBlock + threadIdx.x; t < nvalid; t += o.nblk * kBlock) {
        int i = (int)(t % g.n[0]);
        long long r = t / g.n[0];
        int j = (int)(r % g.n[1]);
        int k = (int)(r / g.n[1]);
        long long c0 = cell(g, i, j, k);
        Prim q = prim_of(U[c0], U[g.cs + c0], U[2 * g.cs + c0], U[3 * g.cs + c0],
                         U[4 * g.cs + c0], gm1);
        m = dmin(m, cfl_cell(q, gamma, g.dx));
    }
    __shared__ double part[kBlock / 64];
    block_dt_min(m, cfl, dt_bits + o.b, dtmin_bits, part);
}

#include "flux_fused.h"
#include "flatten.h"
#include "trace_fused.h"
#include "species.h"
#include "species_fused.h"

// ---------------------------------------------------------------- host side

bool box_valid(const hydro_box *b)
{
    if (!b || b->ng < 3 || b->ng > 8) return false;
    for (int d = 0; d < 3; ++d) {
        if (b->n[d] < 1 || b->n[d] > (1 << 20) || !(b->dx[d] > 0.0) || !isfinite(b->dx[d]))
            return false;
        for (int side = 0; side < 2; ++side) {
            int bc = side ? b->bc_hi[d] : b->bc_lo[d];
            if (bc < HYDRO_BC_PERIODIC || bc > HYDRO_BC_REFLECT) return false;
            if (bc != HYDRO_BC_OUTFLOW && b->n[d] < b->ng) return false;
        }
        if ((b->bc_lo[d] == HYDRO_BC_PERIODIC) != (b->bc_hi[d] == HYDRO_BC_PERIODIC))
            return false;
    }
    long long cs = 1;
    for (int d = 0; d < 3; ++d) cs *= (long long)b->n[d] + 2 * b->ng;
    // the fused kernels address one state component, and one workspace
    // plane, with 32-bit byte offsets
    return cs < (1LL << 28) && ws_pitch(b->n[0], b->n[1]) < (1LL << 31);
}

bool params_valid(const hydro_params *p)
{
    return p && p->gamma > 1.0 && isfinite(p->gamma) && p->cfl > 0.0 && p->cfl <= 1.0 &&
           isfinite(p->grav[0]) && isfinite(p->grav[1]) && isfinite(p->grav[2]) &&
           (p->flatten == 0 || p->flatten == 1);
}

// flattening reads pressures four cells out: every box needs four ghost layers
bool flatten_ok(const hydro_params *p, const hydro_box *boxes, int nb)
{
    if (!p->flatten) return true;
    for (int b = 0; b < nb; ++b)
        if (boxes[b].ng < 4) return false;
    return true;
}

// Built-in tile choice for the fused kernels when no tuned table applies
// (from a sweep on the 512^3 box): both kernels prefer square tiles
// (16 x 16 columns; the flux kernel rows of 18 where they cover a small box
// with fewer tiles); the trace kernel z-segments of 16-32 planes (more
// blocks, planes in flight kept in cache), the flux kernel up to 64 planes
// (a segment costs it two warm-up planes).  Either kernel splits a box's
// planes into segments of equal length no longer than the chosen one (a box
// 16 planes tall traces its 18 planes as 9 + 9, not 16 + 2).
int default_zs(long long tiles, int nz, int zmax)
{
    long long nzs = (8192 + tiles - 1) / tiles;  // aim at >= 8192 blocks (32 per CU)
    int zs = (int)((nz + nzs - 1) / nzs);
    if (zs < 16) zs = 16;
    if (zs > zmax) zs = zmax;
    return zs;
}

// flux-kernel tiles covering an n0 x n1 cross-section with rows of bx lanes
long long flux_tiles(int bx, int n0, int n1)
{
    const long long tx = bx - 2, ty = flux_rows(bx) - 2;
    return ((n0 + tx - 1) / tx) * ((n1 + ty - 1) / ty);
}

void set_default_tiles(Geo &g)
{
    // the trace kernel: 16 x 16 columns; for a box 15 to 30 cells wide, its
    // 17 to 32 traced columns in one tile row: 18 x 14 (15 or 16 cells, the
    // autotuner's choice for such boxes) or 32 x 8
    g.tbx1 = g.n[0] >= 15 && g.n[0] <= 16 ? 18 : (g.n[0] >= 17 && g.n[0] <= 30 ? 32 : 16);
    const int by1 = 256 / g.tbx1;
    g.tzs1 = default_zs((long long)((g.n[0] + 2 + g.tbx1 - 1) / g.tbx1) *
                            ((g.n[1] + 2 + by1 - 1) / by1),
                        g.n[2] + 2, 32);
    // the flux kernel: rows of 16 lanes, or of 18 where they cover the cross
    // section with fewer tiles (every tile costs the same 256 lanes), as for
    // boxes 16 or 32 cells wide; other widths are left to a tuned table
    g.tbx2 = 16;
    long long tiles = flux_tiles(16, g.n[0], g.n[1]);
    if (flux_tiles(18, g.n[0], g.n[1]) < tiles) {
        g.tbx2 = 18;
        tiles = flux_tiles(18, g.n[0], g.n[1]);
    }
    g.tzs2 = default_zs(tiles, g.n[2], 64);
}

// tile widths: the trace kernel's tiles are tbx x (256/tbx) columns (18: 18 x
// 14, four threads idle); the flux kernel's
// rows of tbx lanes fill each wavefront with 64/tbx whole rows (18: three
// rows and ten idle lanes, for boxes 16 or 32 cells wide)
bool tile_valid(int tbx, int tzs)
{
    return (tbx == 8 || tbx == 16 || tbx == 18 || tbx == 32) && tzs >= 1;
}

Geo make_geo(const hydro_box *b)
{
    Geo g;
    for (int d = 0; d < 3; ++d) {
        g.n[d] = b->n[d];
        g.s[d] = b->n[d] + 2 * b->ng;
        g.dx[d] = b->dx[d];
        g.bc_lo[d] = b->bc_lo[d];
        g.bc_hi[d] = b->bc_hi[d];
    }
    g.ng = b->ng;
    g.cs = (long long)g.s[0] * g.s[1] * g.s[2];
    set_default_tiles(g);
    return g;
}

size_t box_ws_bytes(const Geo &g)
{
    const size_t flat = (size_t)(g.n[0] + 2) * (g.n[1] + 2) * (g.n[2] + 2) * sizeof(double);
    return (size_t)ws_flat_off(g.n[0], g.n[1], g.n[2]) + (flat + 255) / 256 * 256;
}

Launch single(const Geo &g, const double *U, double *Un, void *ws, const double *dt)
{
    Launch L;
    memset(&L, 0, sizeof L);
    L.g = g;
    L.U = U;
    L.Un = Un;
    L.ws = (double *)ws;
    L.dt = dt;
    L.nb = 0;
    return L;
}

// ---------------------------------------------------------------- profiling hook

enum { PG_FILL, PG_DT, PG_TRACE, PG_FUSED, PG_SPECIES, PG_COUNT };
const char *const kPgNames[PG_COUNT] = {"fill", "dt", "trace", "flux_update", "species"};
hipEvent_t g_ev[2 * PG_COUNT];
bool g_ev_on = false;

inline void prof(int group, int end, hipStream_t st)
{
    if (g_ev_on) (void)hipEventRecord(g_ev[2 * group + end], st);
}

hydro_status launch_status()
{
    return hipGetLastError() == hipSuccess ? HYDRO_OK : HYDRO_EHIP;
}

// the whole advance, given a launch template and per-stage grid sizes
// (mflux: the mass-flux export for the species pass, or null; for a batch,
// box b's part starts mf_mul * mf_pre[b] doubles in)
hydro_status enqueue_advance(Launch L, const long long *grid, const unsigned *const *pre,
                             const int *const *order, const hydro_params *prm, int32_t *err32,
                             hipStream_t st, double *mflux = nullptr,
                             const long long *mf_pre = nullptr, int mf_mul = 0)
{
    int *err_dev = (int *)err32;
    const double gamma = prm->gamma;
    auto set = [&](int stage) {
        if (L.nb) {
            L.pre = pre[stage];
            L.order = order[stage];
        }
        return dim3((unsigned)grid[stage]);
    };
    prof(PG_TRACE, 0, st);
    if (prm->flatten) {
        hipLaunchKernelGGL(k_flatten, set(ST_FLAT), dim3(kBlock), 0, st, L, gamma);
        hipLaunchKernelGGL(k_trace_fused<true>, set(ST_TRACE), dim3(kTT), 0, st, L, gamma,
                           prm->grav[0], prm->grav[1], prm->grav[2]);
    } else {
        hipLaunchKernelGGL(k_trace_fused<false>, set(ST_TRACE), dim3(kTT), 0, st, L, gamma,
                           prm->grav[0], prm->grav[1], prm->grav[2]);
    }
    prof(PG_TRACE, 1, st);
    prof(PG_FUSED, 0, st);
    if (mflux)
        hipLaunchKernelGGL(k_flux_fused<true>, set(ST_FLUX), dim3(kFT), 0, st, L, gamma,
                           prm->cfl, prm->grav[0], prm->grav[1], prm->grav[2], err_dev, mflux,
                           mf_pre, mf_mul);
    else
        hipLaunchKernelGGL(k_flux_fused<false>, set(ST_FLUX), dim3(kFT), 0, st, L, gamma,
                           prm->cfl, prm->grav[0], prm->grav[1], prm->grav[2], err_dev,
                           (double *)nullptr, (const long long *)nullptr, 0);
    prof(PG_FUSED, 1, st);
    return launch_status();
}

// ---------------------------------------------------------------- tile table

// A tuned tile table: a flat JSON object mapping a box shape "NXxNYxNZ" to
// [tbx, tzs] (tile width in columns, z-segment length; both kernels) or
// [tbx1, tzs1, tbx2, tzs2] (trace kernel, flux kernel), where a pair 0, 0
// keeps that kernel's built-in tile, e.g.
//   {"16x32x64": [16, 32], "64x64x64": [32, 64, 0, 0]}
// as written by the package's autotuner.  Shapes not listed keep the
// built-in choice.  Returns false on a syntax error or an invalid tile.
struct TileRule {
    int n[3];
    int t[4];  // tbx1, tzs1, tbx2, tzs2
};

bool parse_tiles(const char *js, std::vector<TileRule> &out)
{
    const char *c = js;
    auto ws = [&]() { while (*c == ' ' || *c == '\n' || *c == '\t' || *c == '\r') ++c; };
    auto num = [&](int &v) {
        ws();
        if (*c < '0' || *c > '9') return false;
        long long a = 0;
        while (*c >= '0' && *c <= '9') {
            a = a * 10 + (*c - '0');
            if (a > (1 << 30)) return false;
            ++c;
        }
        v = (int)a;
        return true;
    };
    ws();
    if (*c++ != '{') return false;
    ws();
    if (*c == '}') return true;
    for (;;) {
        TileRule r;
        ws();
        if (*c++ != '"') return false;
        if (!num(r.n[0]) || *c++ != 'x' || !num(r.n[1]) || *c++ != 'x' || !num(r.n[2]))
            return false;
        if (*c++ != '"') return false;
        ws();
        if (*c++ != ':') return false;
        ws();
        if (*c++ != '[') return false;
        int k = 0;
        for (;;) {
            if (k == 4 || !num(r.t[k])) return false;
            ++k;
            ws();
            if (*c == ',') {
                ++c;
                continue;
            }
            if (*c++ != ']') return false;
            break;
        }
        if (k == 2) {  // one tile for both kernels
            r.t[2] = r.t[0];
            r.t[3] = r.t[1];
        } else if (k != 4) {
            return false;
        }
        for (int kk = 0; kk < 4; kk += 2)
            if (!(r.t[kk] == 0 && r.t[kk + 1] == 0) && !tile_valid(r.t[kk], r.t[kk + 1]))
                return false;
        out.push_back(r);
        ws();
        if (*c == ',') {
            ++c;
            continue;
        }
        if (*c++ != '}') return false;
        ws();
        return *c == 0;
    }
}

// ---------------------------------------------------------------- plans

// species stages of a batch (blocks per box: ghost cells of the state
// layout; tiles of the fused pass, whose launch has one block per tile and
// species)
enum { SPS_FILL, SPS_FUSED, SPS_COUNT };

__host__ inline long long species_stage_blocks(const Geo &g, int st)
{
    if (st == SPS_FILL) return (g.cs + kBlock - 1) / kBlock;
    return sp_fused_tiles(g);
}

// A plan: the per-stage work lists of a list of boxes, in one device
// buffer.  The buffer is laid out for `cap` boxes (fixed offsets), so a plan
// made with a capacity can be refilled for any list of up to cap boxes by
// one asynchronous copy from a pinned staging buffer, ordered on the stream
// with the launches that use it.
constexpr int kMaxPlanBoxes = 1 << 20;
constexpr int kPlanStaging = 4;  // pinned staging buffers of a capacity plan

struct Plan {
    int nb = 0;   // boxes in the current list
    int cap = 0;  // boxes the device buffer is laid out for
    std::vector<TileRule> rules;
    std::vector<hydro_box> boxes;
    std::vector<Geo> geos;
    size_t ws_bytes = 0;
    long long grid[ST_COUNT] = {};  // total blocks per stage
    long long sp_grid[SPS_COUNT] = {};
    long long etot = 0;  // sum of the boxes' field strides (species arrays)
    // device buffer, for cap boxes: [Geo cap][long long wsoff cap]
    // [int order ST_COUNT x cap][unsigned pre ST_COUNT x (cap+1)]
    // [unsigned species pre SPS_COUNT x (cap+1)][long long epre cap+1]
    std::vector<char> image;  // its host image for the current list
    size_t off_w = 0, off_o = 0, off_p = 0, off_s = 0, off_e = 0, bytes = 0;
    void *dev = nullptr;
    const Geo *geos_dev = nullptr;
    const long long *wsoff_dev = nullptr;
    const int *order_dev[ST_COUNT] = {};
    const unsigned *pre_dev[ST_COUNT] = {};
    const unsigned *sp_pre_dev[SPS_COUNT] = {};
    const long long *epre_dev = nullptr;
    // capacity plans: pinned staging buffers and the event of each one's last copy
    int nstage = 0, next_stage = 0;
    void *stage[kPlanStaging] = {};
    hipEvent_t stage_ev[kPlanStaging] = {};
    int stage_used[kPlanStaging] = {};
};

inline size_t round256(size_t v) { return (v + 255) / 256 * 256; }

// capacity, tile table and buffer layout
hydro_status plan_init(Plan *P, int cap, const char *autotune_json)
{
    if (autotune_json && !parse_tiles(autotune_json, P->rules)) return HYDRO_EINVAL;
    P->cap = cap;
    const size_t C = (size_t)cap;
    P->off_w = round256(sizeof(Geo) * C);
    P->off_o = P->off_w + round256(sizeof(long long) * C);
    P->off_p = P->off_o + round256(sizeof(int) * ST_COUNT * C);
    P->off_s = P->off_p + round256(sizeof(unsigned) * ST_COUNT * (C + 1));
    P->off_e = P->off_s + round256(sizeof(unsigned) * SPS_COUNT * (C + 1));
    P->bytes = P->off_e + sizeof(long long) * (C + 1);
    return HYDRO_OK;
}

// validate the boxes and build the work lists and the buffer's host image
hydro_status plan_build(Plan *P, const hydro_box *boxes, int nb)
{
    if (nb < 1 || nb > P->cap) return HYDRO_EINVAL;
    if (P->bytes == 0) plan_init(P, P->cap, nullptr);
    const size_t C = (size_t)P->cap;
    P->nb = nb;
    P->boxes.assign(boxes, boxes + nb);
    P->geos.clear();
    P->ws_bytes = 0;
    P->image.assign(P->bytes, 0);
    char *img = P->image.data();
    long long *wsoff = (long long *)(img + P->off_w);
    for (int b = 0; b < nb; ++b) {
        if (!box_valid(&boxes[b])) return HYDRO_EINVAL;
        Geo g = make_geo(&boxes[b]);
        for (const TileRule &r : P->rules)
            if (r.n[0] == g.n[0] && r.n[1] == g.n[1] && r.n[2] == g.n[2]) {
                if (r.t[0] != 0) {
                    g.tbx1 = r.t[0];
                    g.tzs1 = r.t[1];
                }
                if (r.t[2] != 0) {
                    g.tbx2 = r.t[2];
                    g.tzs2 = r.t[3];
                }
            }
        P->geos.push_back(g);
        wsoff[b] = (long long)(P->ws_bytes / sizeof(double));
        P->ws_bytes += box_ws_bytes(g);
    }
    memcpy(img, P->geos.data(), sizeof(Geo) * nb);
    // Work lists: for the marching kernels, boxes in order of decreasing
    // block length (the z-planes one block marches over), so the longest
    // blocks start first and short ones fill the end of the launch; the
    // other stages take the boxes in the given order.
    int *order = (int *)(img + P->off_o);
    unsigned *pre = (unsigned *)(img + P->off_p);
    for (int s = 0; s < ST_COUNT; ++s) {
        int *o = order + (size_t)s * C;
        for (int b = 0; b < nb; ++b) o[b] = b;
        auto zlen = [&](int b) {
            const Geo &g = P->geos[b];
            if (s == ST_FLUX) return seg_len(g.n[2], g.tzs2);
            if (s == ST_TRACE) return seg_len(g.n[2] + 2, g.tzs1);
            return 0;
        };
        std::stable_sort(o, o + nb, [&](int a, int b) { return zlen(a) > zlen(b); });
        unsigned *ps = pre + (size_t)s * (C + 1);
        unsigned long long acc = 0;
        for (int i = 0; i < nb; ++i) {
            ps[i] = (unsigned)acc;
            acc += (unsigned long long)stage_blocks(P->geos[o[i]], s);
        }
        if (acc >= (1ULL << 31)) return HYDRO_EINVAL;
        ps[nb] = (unsigned)acc;
        P->grid[s] = (long long)acc;
    }
    // the species stages take the boxes in the given order
    unsigned *spre = (unsigned *)(img + P->off_s);
    for (int s = 0; s < SPS_COUNT; ++s) {
        unsigned *ps = spre + (size_t)s * (C + 1);
        unsigned long long acc = 0;
        for (int b = 0; b < nb; ++b) {
            ps[b] = (unsigned)acc;
            acc += (unsigned long long)species_stage_blocks(P->geos[b], s);
        }
        if (acc >= (1ULL << 31)) return HYDRO_EINVAL;
        ps[nb] = (unsigned)acc;
        P->sp_grid[s] = (long long)acc;
    }
    long long *epre = (long long *)(img + P->off_e);
    epre[0] = 0;
    for (int b = 0; b < nb; ++b)
        epre[b + 1] = epre[b] + mf_stride(P->geos[b].n[0], P->geos[b].n[1], P->geos[b].n[2]);
    P->etot = epre[nb];
    return HYDRO_OK;
}

// the device buffer (and, for a capacity plan, nstage pinned staging buffers)
hydro_status plan_alloc(Plan *P, int nstage)
{
    if (hipMalloc(&P->dev, P->bytes) != hipSuccess) {
        P->dev = nullptr;
        return HYDRO_EHIP;
    }
    char *base = (char *)P->dev;
    const size_t C = (size_t)P->cap;
    P->geos_dev = (const Geo *)base;
    P->wsoff_dev = (const long long *)(base + P->off_w);
    for (int s = 0; s < ST_COUNT; ++s) {
        P->order_dev[s] = (const int *)(base + P->off_o) + (size_t)s * C;
        P->pre_dev[s] = (const unsigned *)(base + P->off_p) + (size_t)s * (C + 1);
    }
    for (int s = 0; s < SPS_COUNT; ++s)
        P->sp_pre_dev[s] = (const unsigned *)(base + P->off_s) + (size_t)s * (C + 1);
    P->epre_dev = (const long long *)(base + P->off_e);
    for (int k = 0; k < nstage; ++k) {
        if (hipHostMalloc(&P->stage[k], P->bytes, hipHostMallocDefault) != hipSuccess) {
            P->stage[k] = nullptr;
            return HYDRO_EHIP;
        }
        if (hipEventCreateWithFlags(&P->stage_ev[k], hipEventDisableTiming) != hipSuccess) {
            P->stage_ev[k] = nullptr;
            return HYDRO_EHIP;
        }
        P->nstage = k + 1;
    }
    return HYDRO_OK;
}

// release everything a plan holds (waits for its pending copies first)
void plan_free(Plan *P)
{
    for (int k = 0; k < kPlanStaging; ++k) {
        if (P->stage_ev[k]) {
            if (P->stage_used[k]) (void)hipEventSynchronize(P->stage_ev[k]);
            (void)hipEventDestroy(P->stage_ev[k]);
        }
        if (P->stage[k]) (void)hipHostFree(P->stage[k]);
    }
    if (P->dev) (void)hipFree(P->dev);
    delete P;
}

// the species pass of one box (B.nb == 0) or a batch (B with the plan's
// tile prefix sums): one fused launch, a block per tile and species
void enqueue_species(const SpArgs &A, SpBatch B, const long long *grid,
                     const unsigned *const *pre, int32_t *err_dev, hipStream_t st)
{
    if (B.nb) B.pre = pre[SPS_FUSED];
    prof(PG_SPECIES, 0, st);
    hipLaunchKernelGGL(k_sp_fused, dim3((unsigned)(grid[SPS_FUSED] * A.ns)), dim3(256), 0, st,
                       A, B, (int *)err_dev);
    prof(PG_SPECIES, 1, st);
}

}  // namespace

extern "C" {

size_t hydro_state_elems(const hydro_box *box)
{
    if (!box_valid(box)) return 0;
    return (size_t)(5 * make_geo(box).cs);
}

size_t hydro_workspace_bytes(const hydro_box *boxes, int nboxes)
{
    if (!boxes || nboxes < 1) return 0;
    size_t tot = 0;
    for (int b = 0; b < nboxes; ++b) {
        if (!box_valid(&boxes[b])) return 0;
        tot += box_ws_bytes(make_geo(&boxes[b]));
    }
    return tot;
}

hydro_status hydro_fill_ghosts(double *U_dev, const hydro_box *box, void *stream)
{
    if (!U_dev || !box_valid(box)) return HYDRO_EINVAL;
    Geo g = make_geo(box);
    hipStream_t st = (hipStream_t)stream;
    Launch L = single(g, U_dev, nullptr, nullptr, nullptr);
    prof(PG_FILL, 0, st);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)stage_blocks(g, ST_FILL)), dim3(kBlock), 0, st,
                       L, (unsigned long long *)nullptr, (unsigned long long *)nullptr);
    prof(PG_FILL, 1, st);
    return launch_status();
}

hydro_status estimate_dt(double *U_dev, const hydro_box *box, const hydro_params *prm,
                         double *dt_dev, void *stream)
{
    if (!U_dev || !dt_dev || !box_valid(box) || !params_valid(prm)) return HYDRO_EINVAL;
    Geo g = make_geo(box);
    hipStream_t st = (hipStream_t)stream;
    Launch L = single(g, U_dev, nullptr, nullptr, nullptr);
    prof(PG_FILL, 0, st);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)stage_blocks(g, ST_FILL)), dim3(kBlock), 0, st,
                       L, (unsigned long long *)dt_dev, (unsigned long long *)nullptr);
    prof(PG_FILL, 1, st);
    prof(PG_DT, 0, st);
    hipLaunchKernelGGL(k_dt, dim3((unsigned)stage_blocks(g, ST_DT)), dim3(kBlock), 0, st, L,
                       prm->gamma, prm->cfl, (unsigned long long *)dt_dev,
                       (unsigned long long *)nullptr);
    prof(PG_DT, 1, st);
    return launch_status();
}

// byte ranges [a, a+na) and [b, b+nb) overlap
static bool overlaps(const void *a, size_t na, const void *b, size_t nb)
{
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

// argument checks of advance_box that do not involve the workspace
static hydro_status advance_box_args(const double *U_dev, double *U_new_dev,
                                     const hydro_box *box, const hydro_params *prm,
                                     const double *dt_dev, double *dt_next_dev, int32_t *err_dev)
{
    if (!U_dev || !U_new_dev || !dt_dev || !err_dev || !box_valid(box) || !params_valid(prm) ||
        !flatten_ok(prm, box, 1))
        return HYDRO_EINVAL;
    if (dt_next_dev && overlaps(dt_next_dev, sizeof(double), dt_dev, sizeof(double)))
        return HYDRO_EINVAL;
    const size_t ub = 5 * (size_t)make_geo(box).cs * sizeof(double);
    if (overlaps(U_dev, ub, U_new_dev, ub)) return HYDRO_EINVAL;  // the new state vs the old
    return HYDRO_OK;
}

hydro_status advance_box(const double *U_dev, double *U_new_dev, const hydro_box *box,
                         const hydro_params *prm, const double *dt_dev, double *dt_next_dev,
                         void *ws_dev, size_t ws_bytes, int32_t *err_dev, void *stream)
{
    hydro_status rc = advance_box_args(U_dev, U_new_dev, box, prm, dt_dev, dt_next_dev, err_dev);
    if (rc != HYDRO_OK) return rc;
    if (!ws_dev || (((uintptr_t)ws_dev) & 255)) return HYDRO_EINVAL;
    Geo g = make_geo(box);
    const size_t ub = 5 * (size_t)g.cs * sizeof(double);
    // the workspace must not overlap the states it is read and written with
    if (overlaps(ws_dev, ws_bytes, U_dev, ub) || overlaps(ws_dev, ws_bytes, U_new_dev, ub))
        return HYDRO_EINVAL;
    if (ws_bytes < box_ws_bytes(g)) return HYDRO_ENOWS;
    long long grid[ST_COUNT];
    for (int s = 0; s < ST_COUNT; ++s) grid[s] = stage_blocks(g, s);
    Launch L = single(g, U_dev, U_new_dev, ws_dev, dt_dev);
    L.dtn = (unsigned long long *)dt_next_dev;
    return enqueue_advance(L, grid, nullptr, nullptr, prm, err_dev, (hipStream_t)stream);
}

// ---------------------------------------------------------------- no-allocation variant

}  // extern "C"

namespace {

// advance_box_noalloc's workspace: one static device array per GPU, held
// until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol); the device
// address each GPU holds it at is looked up once per device.
constexpr size_t kNoAllocBytes = HYDRO_NOALLOC_WS_BYTES;
static __device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// device address of `scratch` on the device `stream` runs on
hydro_status scratch_address(hipStream_t stream, void **out)
{
    int cur = -1, dev = -1;
    if (hipGetDevice(&cur) != hipSuccess) return HYDRO_EHIP;
    dev = cur;
    if (stream && hipStreamGetDevice(stream, &dev) != hipSuccess) return HYDRO_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return HYDRO_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        if (dev != cur && hipSetDevice(dev) != hipSuccess) return HYDRO_EHIP;
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (dev != cur) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) return HYDRO_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HYDRO_OK;
}

}  // namespace

extern "C" {

hydro_status advance_box_noalloc(const double *U_dev, double *U_new_dev, const hydro_box *box,
                                 const hydro_params *prm, const double *dt_dev,
                                 double *dt_next_dev, int32_t *err_dev, void *stream)
{
    hydro_status rc = advance_box_args(U_dev, U_new_dev, box, prm, dt_dev, dt_next_dev, err_dev);
    if (rc != HYDRO_OK) return rc;
    const Geo g = make_geo(box);
    const size_t need = box_ws_bytes(g);
    if (need > kNoAllocBytes) return HYDRO_ENOWS;
    void *ws = nullptr;
    const hipStream_t st = (hipStream_t)stream;
    if ((rc = scratch_address(st, &ws)) != HYDRO_OK) return rc;
    const size_t ub = 5 * (size_t)g.cs * sizeof(double);
    if (overlaps(ws, need, U_dev, ub) || overlaps(ws, need, U_new_dev, ub)) return HYDRO_EINVAL;
    long long grid[ST_COUNT];
    for (int s = 0; s < ST_COUNT; ++s) grid[s] = stage_blocks(g, s);
    Launch L = single(g, U_dev, U_new_dev, ws, dt_dev);
    L.dtn = (unsigned long long *)dt_next_dev;
    return enqueue_advance(L, grid, nullptr, nullptr, prm, err_dev, st);
}

size_t hydro_species_workspace_bytes(const hydro_box *box, int nspec)
{
    if (!box_valid(box) || nspec < 1 || nspec > kMaxSpecies) return 0;
    const Geo g = make_geo(box);
    return (size_t)12 * (size_t)mf_stride(g.n[0], g.n[1], g.n[2]) * sizeof(double);
}

hydro_status hydro_fill_ghosts_species(double *S_dev, int nspec, const hydro_box *box,
                                       void *stream)
{
    if (!S_dev || nspec < 1 || nspec > kMaxSpecies || !box_valid(box)) return HYDRO_EINVAL;
    SpArgs A;
    memset(&A, 0, sizeof A);
    A.g = make_geo(box);
    A.S = S_dev;
    A.ns = nspec;
    SpBatch B;
    memset(&B, 0, sizeof B);
    hipLaunchKernelGGL(k_sp_fill, dim3((unsigned)species_stage_blocks(A.g, SPS_FILL)),
                       dim3(kBlock), 0, (hipStream_t)stream, A, B);
    return launch_status();
}

hydro_status advance_box_species(const double *U_dev, double *U_new_dev, const double *S_dev,
                                 double *S_new_dev, int nspec, const hydro_box *box,
                                 const hydro_params *prm, const double *dt_dev,
                                 double *dt_next_dev, void *ws_dev, size_t ws_bytes,
                                 void *sws_dev, size_t sws_bytes, int32_t *err_dev, void *stream)
{
    // argument errors first, then the workspace sizes
    if (!U_dev || !U_new_dev || !S_dev || !S_new_dev || !dt_dev || !ws_dev || !sws_dev ||
        !err_dev || nspec < 1 || nspec > kMaxSpecies || !box_valid(box) || !params_valid(prm) ||
        !flatten_ok(prm, box, 1) || ((uintptr_t)ws_dev & 255) || ((uintptr_t)sws_dev & 255))
        return HYDRO_EINVAL;
    if (dt_next_dev && overlaps(dt_next_dev, sizeof(double), dt_dev, sizeof(double)))
        return HYDRO_EINVAL;
    const Geo g = make_geo(box);
    const size_t sbytes = (size_t)nspec * g.cs * sizeof(double);
    const size_t ubytes = (size_t)5 * g.cs * sizeof(double);
    // no array written (U_new, S_new, both workspaces) may overlap another
    // array
    if (overlaps(U_dev, ubytes, U_new_dev, ubytes) || overlaps(S_dev, sbytes, S_new_dev, sbytes) ||
        overlaps(S_new_dev, sbytes, U_dev, ubytes) || overlaps(S_new_dev, sbytes, U_new_dev, ubytes) ||
        overlaps(S_new_dev, sbytes, ws_dev, ws_bytes) || overlaps(S_dev, sbytes, U_new_dev, ubytes) ||
        overlaps(ws_dev, ws_bytes, S_dev, sbytes) || overlaps(ws_dev, ws_bytes, U_dev, ubytes) ||
        overlaps(ws_dev, ws_bytes, U_new_dev, ubytes) ||
        overlaps(sws_dev, sws_bytes, S_dev, sbytes) || overlaps(sws_dev, sws_bytes, S_new_dev, sbytes) ||
        overlaps(sws_dev, sws_bytes, U_dev, ubytes) || overlaps(sws_dev, sws_bytes, U_new_dev, ubytes) ||
        overlaps(sws_dev, sws_bytes, ws_dev, ws_bytes))
        return HYDRO_EINVAL;
    if (ws_bytes < box_ws_bytes(g) || sws_bytes < hydro_species_workspace_bytes(box, nspec))
        return HYDRO_ENOWS;
    const hipStream_t st = (hipStream_t)stream;
    long long grid[ST_COUNT];
    for (int s = 0; s < ST_COUNT; ++s) grid[s] = stage_blocks(g, s);
    Launch L = single(g, U_dev, U_new_dev, ws_dev, dt_dev);
    L.dtn = (unsigned long long *)dt_next_dev;
    double *mf = (double *)sws_dev;
    hydro_status rc = enqueue_advance(L, grid, nullptr, nullptr, prm, err_dev, st, mf);
    if (rc != HYDRO_OK) return rc;
    // the species pass
    SpArgs A;
    memset(&A, 0, sizeof A);
    A.g = g;
    A.U = U_dev;
    A.S = S_dev;
    A.Sn = S_new_dev;
    A.ws = (const char *)ws_dev;
    A.E = mf_stride(g.n[0], g.n[1], g.n[2]);
    A.mf = mf;
    A.dt = dt_dev;
    A.ns = nspec;
    A.flat = prm->flatten;
    A.gamma = prm->gamma;
    long long grid_sp[SPS_COUNT];
    for (int s = 0; s < SPS_COUNT; ++s) grid_sp[s] = species_stage_blocks(g, s);
    SpBatch B;
    memset(&B, 0, sizeof B);
    enqueue_species(A, B, grid_sp, nullptr, err_dev, st);
    return launch_status();
}

hydro_status hydro_plan_create(const hydro_box *boxes, int nb, const char *autotune_json,
                               void **plan_out)
{
    if (!boxes || nb < 1 || !plan_out) return HYDRO_EINVAL;
    *plan_out = nullptr;
    Plan *P = new (std::nothrow) Plan();
    if (!P) return HYDRO_EINVAL;
    hydro_status rc = plan_init(P, nb, autotune_json);
    if (rc == HYDRO_OK) rc = plan_build(P, boxes, nb);
    if (rc == HYDRO_OK) rc = plan_alloc(P, 0);
    // a fixed plan is set up once: a synchronous upload
    if (rc == HYDRO_OK && hipMemcpy(P->dev, P->image.data(), P->image.size(),
                                    hipMemcpyHostToDevice) != hipSuccess)
        rc = HYDRO_EHIP;
    if (rc != HYDRO_OK) {
        plan_free(P);
        return rc;
    }
    *plan_out = P;
    return HYDRO_OK;
}

hydro_status hydro_plan_create_capacity(int capacity, const char *autotune_json, void **plan_out)
{
    if (capacity < 1 || capacity > kMaxPlanBoxes || !plan_out) return HYDRO_EINVAL;
    *plan_out = nullptr;
    Plan *P = new (std::nothrow) Plan();
    if (!P) return HYDRO_EINVAL;
    hydro_status rc = plan_init(P, capacity, autotune_json);
    if (rc == HYDRO_OK) rc = plan_alloc(P, kPlanStaging);
    if (rc != HYDRO_OK) {
        plan_free(P);
        return rc;
    }
    P->nb = 0;
    *plan_out = P;
    return HYDRO_OK;
}

hydro_status hydro_plan_update(void *plan, const hydro_box *boxes, int nb, void *stream)
{
    Plan *P = (Plan *)plan;
    if (!P || P->nstage == 0 || !boxes || nb < 1 || nb > P->cap) return HYDRO_EINVAL;
    // validate into a copy first, so a rejected update leaves the plan as it was
    Plan Q;
    Q.cap = P->cap;
    Q.rules = P->rules;
    hydro_status rc = plan_build(&Q, boxes, nb);
    if (rc != HYDRO_OK) return rc;
    // the next pinned staging buffer; wait only for the copy that last used it
    const int k = P->next_stage;
    if (P->stage_used[k] && hipEventSynchronize(P->stage_ev[k]) != hipSuccess) return HYDRO_EHIP;
    memcpy(P->stage[k], Q.image.data(), Q.image.size());
    const hipStream_t st = (hipStream_t)stream;
    if (hipMemcpyAsync(P->dev, P->stage[k], Q.image.size(), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipEventRecord(P->stage_ev[k], st) != hipSuccess)
        return HYDRO_EHIP;
    P->stage_used[k] = 1;
    P->next_stage = (k + 1) % P->nstage;
    // host-side fields: every launch enqueued from here on uses the new lists
    P->nb = Q.nb;
    P->boxes.swap(Q.boxes);
    P->geos.swap(Q.geos);
    P->ws_bytes = Q.ws_bytes;
    memcpy(P->grid, Q.grid, sizeof P->grid);
    memcpy(P->sp_grid, Q.sp_grid, sizeof P->sp_grid);
    P->etot = Q.etot;
    return HYDRO_OK;
}

int hydro_plan_boxes(const void *plan)
{
    const Plan *P = (const Plan *)plan;
    return P ? P->nb : -1;
}

size_t hydro_plan_workspace_bytes(const void *plan)
{
    const Plan *P = (const Plan *)plan;
    return P ? P->ws_bytes : 0;
}

void hydro_plan_destroy(void *plan)
{
    Plan *P = (Plan *)plan;
    if (!P) return;
    plan_free(P);
}

static Launch batch_launch(const Plan *P, double *const *Us, double *const *Uns, void *ws,
                           const double *dts, int dt_stride)
{
    Launch L;
    memset(&L, 0, sizeof L);
    L.nb = P->nb;
    L.geos = P->geos_dev;
    L.Us = Us;
    L.Uns = Uns;
    L.ws = (double *)ws;
    L.wsoff = P->wsoff_dev;
    L.dts = dts;
    L.dt_stride = dt_stride;
    return L;
}

hydro_status estimate_dt_boxes(int nb, double *const *U_ptrs_dev, const void *plan,
                               const hydro_params *prm, double *dt_dev, double *dt_min_dev,
                               void *stream)
{
    const Plan *P = (const Plan *)plan;
    if (!P || nb < 1 || nb != P->nb || !U_ptrs_dev || !dt_dev || !params_valid(prm))
        return HYDRO_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Launch L = batch_launch(P, U_ptrs_dev, nullptr, nullptr, nullptr, 0);
    L.pre = P->pre_dev[ST_FILL];
    L.order = P->order_dev[ST_FILL];
    prof(PG_FILL, 0, st);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)P->grid[ST_FILL]), dim3(kBlock), 0, st, L,
                       (unsigned long long *)dt_dev, (unsigned long long *)dt_min_dev);
    prof(PG_FILL, 1, st);
    L.pre = P->pre_dev[ST_DT];
    L.order = P->order_dev[ST_DT];
    prof(PG_DT, 0, st);
    hipLaunchKernelGGL(k_dt, dim3((unsigned)P->grid[ST_DT]), dim3(kBlock), 0, st, L,
                       prm->gamma, prm->cfl, (unsigned long long *)dt_dev,
                       (unsigned long long *)dt_min_dev);
    prof(PG_DT, 1, st);
    return launch_status();
}

hydro_status advance_boxes(int nb, const double *const *U_ptrs_dev,
                           double *const *U_new_ptrs_dev, const void *plan,
                           const hydro_params *prm, const double *dt_dev, int dt_stride,
                           double *dt_next_dev, double *dt_next_min_dev, void *ws_dev,
                           size_t ws_bytes, int32_t *err_dev, void *stream)
{
    const Plan *P = (const Plan *)plan;
    if (!P || nb < 1 || nb != P->nb || !U_ptrs_dev || !U_new_ptrs_dev || !dt_dev || !ws_dev ||
        !err_dev || !params_valid(prm) || (dt_stride != 0 && dt_stride != 1) ||
        (dt_next_min_dev && !dt_next_dev) || !flatten_ok(prm, P->boxes.data(), P->nb))
        return HYDRO_EINVAL;
    {  // the next-step timesteps must not overlap the ones in use or each other
        const size_t ndt = (dt_stride ? (size_t)nb : 1) * sizeof(double);
        const size_t nn = (size_t)nb * sizeof(double);
        if (dt_next_dev && overlaps(dt_next_dev, nn, dt_dev, ndt)) return HYDRO_EINVAL;
        if (dt_next_min_dev && (overlaps(dt_next_min_dev, sizeof(double), dt_dev, ndt) ||
                                overlaps(dt_next_min_dev, sizeof(double), dt_next_dev, nn)))
            return HYDRO_EINVAL;
    }
    if (((uintptr_t)ws_dev) & 255) return HYDRO_EINVAL;
    if (ws_bytes < P->ws_bytes) return HYDRO_ENOWS;
    Launch L = batch_launch(P, (double *const *)U_ptrs_dev, U_new_ptrs_dev, ws_dev, dt_dev,
                            dt_stride);
    L.dtn = (unsigned long long *)dt_next_dev;
    L.dtn_min = (unsigned long long *)dt_next_min_dev;
    return enqueue_advance(L, P->grid, P->pre_dev, P->order_dev, prm, err_dev,
                           (hipStream_t)stream);
}

size_t hydro_species_workspace_bytes_boxes(const hydro_box *boxes, int nb, int nspec)
{
    if (!boxes || nb < 1) return 0;
    size_t tot = 0;
    for (int b = 0; b < nb; ++b) {
        const size_t n = hydro_species_workspace_bytes(&boxes[b], nspec);
        if (!n) return 0;
        tot += n;
    }
    return tot;
}

hydro_status hydro_fill_ghosts_boxes_species(int nb, double *const *S_ptrs_dev, int nspec,
                                             const void *plan, void *stream)
{
    const Plan *P = (const Plan *)plan;
    if (!P || nb < 1 || nb != P->nb || !S_ptrs_dev || nspec < 1 || nspec > kMaxSpecies)
        return HYDRO_EINVAL;
    SpArgs A;
    memset(&A, 0, sizeof A);
    A.ns = nspec;
    SpBatch B;
    memset(&B, 0, sizeof B);
    B.nb = nb;
    B.pre = P->sp_pre_dev[SPS_FILL];
    B.geos = P->geos_dev;
    B.Ss = (const double *const *)S_ptrs_dev;
    hipLaunchKernelGGL(k_sp_fill, dim3((unsigned)P->sp_grid[SPS_FILL]), dim3(kBlock), 0,
                       (hipStream_t)stream, A, B);
    return launch_status();
}

hydro_status advance_boxes_species(int nb, const double *const *U_ptrs_dev,
                                   double *const *U_new_ptrs_dev,
                                   const double *const *S_ptrs_dev,
                                   double *const *S_new_ptrs_dev, int nspec, const void *plan,
                                   const hydro_params *prm, const double *dt_dev, int dt_stride,
                                   double *dt_next_dev, double *dt_next_min_dev, void *ws_dev,
                                   size_t ws_bytes, void *sws_dev, size_t sws_bytes,
                                   int32_t *err_dev, void *stream)
{
    const Plan *P = (const Plan *)plan;
    if (!P || nb < 1 || nb != P->nb || !S_ptrs_dev || !S_new_ptrs_dev || !sws_dev || nspec < 1 ||
        nspec > kMaxSpecies || ((uintptr_t)sws_dev & 255) ||
        (ws_dev && overlaps(sws_dev, sws_bytes, ws_dev, ws_bytes)))
        return HYDRO_EINVAL;
    if (sws_bytes < (size_t)12 * (size_t)P->etot * sizeof(double))
        return HYDRO_ENOWS;
    if (!U_ptrs_dev || !U_new_ptrs_dev || !dt_dev || !ws_dev || !err_dev ||
        !params_valid(prm) || (dt_stride != 0 && dt_stride != 1) ||
        (dt_next_min_dev && !dt_next_dev) || !flatten_ok(prm, P->boxes.data(), P->nb))
        return HYDRO_EINVAL;
    {
        const size_t ndt = (dt_stride ? (size_t)nb : 1) * sizeof(double);
        const size_t nn = (size_t)nb * sizeof(double);
        if (dt_next_dev && overlaps(dt_next_dev, nn, dt_dev, ndt)) return HYDRO_EINVAL;
        if (dt_next_min_dev && (overlaps(dt_next_min_dev, sizeof(double), dt_dev, ndt) ||
                                overlaps(dt_next_min_dev, sizeof(double), dt_next_dev, nn)))
            return HYDRO_EINVAL;
    }
    if (((uintptr_t)ws_dev) & 255) return HYDRO_EINVAL;
    if (ws_bytes < P->ws_bytes) return HYDRO_ENOWS;
    const hipStream_t st = (hipStream_t)stream;
    Launch L = batch_launch(P, (double *const *)U_ptrs_dev, U_new_ptrs_dev, ws_dev, dt_dev,
                            dt_stride);
    L.dtn = (unsigned long long *)dt_next_dev;
    L.dtn_min = (unsigned long long *)dt_next_min_dev;
    hydro_status rc = enqueue_advance(L, P->grid, P->pre_dev, P->order_dev, prm, err_dev, st,
                                      (double *)sws_dev, P->epre_dev, 12);
    if (rc != HYDRO_OK) return rc;
    SpArgs A;
    memset(&A, 0, sizeof A);
    A.ns = nspec;
    A.flat = prm->flatten;
    A.gamma = prm->gamma;
    SpBatch B;
    memset(&B, 0, sizeof B);
    B.nb = nb;
    B.geos = P->geos_dev;
    B.Us = U_ptrs_dev;
    B.Ss = S_ptrs_dev;
    B.Sns = S_new_ptrs_dev;
    B.ws = (const char *)ws_dev;
    B.wsoff = P->wsoff_dev;
    B.sws = (double *)sws_dev;
    B.epre = P->epre_dev;
    B.dts = dt_dev;
    B.dt_stride = dt_stride;
    enqueue_species(A, B, P->sp_grid, P->sp_pre_dev, err_dev, st);
    return launch_status();
}

hydro_status hydro_fill_ghosts_boxes(int nb, double *const *U_ptrs_dev, const void *plan,
                                     void *stream)
{
    const Plan *P = (const Plan *)plan;
    if (!P || nb < 1 || nb != P->nb || !U_ptrs_dev) return HYDRO_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Launch L = batch_launch(P, U_ptrs_dev, nullptr, nullptr, nullptr, 0);
    L.pre = P->pre_dev[ST_FILL];
    L.order = P->order_dev[ST_FILL];
    prof(PG_FILL, 0, st);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)P->grid[ST_FILL]), dim3(kBlock), 0, st, L,
                       (unsigned long long *)nullptr, (unsigned long long *)nullptr);
    prof(PG_FILL, 1, st);
    return launch_status();
}

int hydro_stage_count(void) { return PG_COUNT; }

const char *hydro_stage_name(int s) { return (s >= 0 && s < PG_COUNT) ? kPgNames[s] : ""; }

hydro_status hydro_set_stage_events(void *const *events)
{
    if (!events) {
        g_ev_on = false;
        return HYDRO_OK;
    }
    for (int i = 0; i < 2 * PG_COUNT; ++i)
        if (!events[i]) return HYDRO_EINVAL;
    for (int i = 0; i < 2 * PG_COUNT; ++i) g_ev[i] = (hipEvent_t)events[i];
    g_ev_on = true;
    return HYDRO_OK;
}

const char *hydro_status_string(hydro_status s)
{
    switch (s) {
    case HYDRO_OK: return "HYDRO_OK";
    case HYDRO_EINVAL: return "HYDRO_EINVAL: invalid argument";
    case HYDRO_EHIP: return "HYDRO_EHIP: HIP runtime or launch failure";
    case HYDRO_ENOWS: return "HYDRO_ENOWS: workspace too small";
    }
    return "unknown hydro_status";
}

}  // extern "C"
