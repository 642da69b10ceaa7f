// level.hip -- ghost exchange between the boxes of one level (Sec. II: a
// level's data is a list of boxes that together cover the problem domain, and
// the neighbour data a box's stencil needs comes from the boxes next to it).
//
// The boxes of a level tile a domain of D0 x D1 x D2 cells exactly.  Every
// ghost cell of every box is filled with the value that the whole domain,
// held as one box and ghost-filled under the domain's boundary kinds, has at
// the same place: a ghost cell at domain index g maps axis by axis to a valid
// domain cell s (inside: itself; periodic: wrapped; outflow: nearest domain
// cell; reflect: mirror image, normal momentum negated), and takes the value
// of s from whichever box owns it.  The box that owns s is found in an owner
// map over the domain at the granularity of the largest cell count dividing
// every box corner and side, built once when the level is created.
//
// One launch fills every box: each thread copies one ghost cell (five
// components), blocks walk each box's ghost region as z-slabs, then y-slabs,
// then x-slabs, x fastest, so reads and writes stream along x.  Ghost cells
// are only written and valid cells only read, so no ordering between boxes is
// needed.
#include "../../include/hydro.h"

#include <hip/hip_runtime.h>

#include <new>
#include <numeric>
#include <vector>

namespace {

constexpr int kLBlock = 256;
constexpr long long kMaxOwnerCells = 1LL << 24;

struct LBox {
    int n[3];
    int ng;
    int lo[3];  // domain index of valid cell (0, 0, 0)
    int s0, s1;
    long long cs;  // doubles per component
};

struct LevelArgs {
    const LBox *bx;
    const unsigned *pre;  // prefix sum of blocks per box (nb + 1)
    const int *owner;     // owner map, (D2/G) x (D1/G) x (D0/G), x fastest
    int nb;
    int dom[3], bc_lo[3], bc_hi[3];
    int G, om0, om1;
};

// source index along one axis of the domain for index g (|g| within one
// domain width of the domain), and whether the normal momentum flips sign
__device__ __forceinline__ int dom_src(int g, int D, int bl, int bh, int &flip)
{
    if (g < 0) {
        if (bl == HYDRO_BC_PERIODIC) return g + D;
        if (bl == HYDRO_BC_OUTFLOW) return 0;
        flip = 1;
        return -1 - g;
    }
    if (g >= D) {
        if (bh == HYDRO_BC_PERIODIC) return g - D;
        if (bh == HYDRO_BC_OUTFLOW) return D - 1;
        flip = 1;
        return 2 * D - 1 - g;
    }
    return g;
}

__device__ __forceinline__ long long lcell(const LBox &B, int i, int j, int k)
{
    return ((long long)(k + B.ng) * B.s1 + (j + B.ng)) * B.s0 + (i + B.ng);
}

// The ghost cell this thread fills: box b (block prefix search), the cell
// (i, j, k) in box coordinates, its source box o and source cell, and the
// reflections (fx, fy, fz) on the way.  False for threads past the box's
// ghost cells.
struct LGhost {
    int b, o;
    long long dst, src;
    int fx, fy, fz;
};

__device__ __forceinline__ bool level_ghost(const LevelArgs &L, LGhost &G)
{
    int b = 0, hi = L.nb;
    const unsigned x = blockIdx.x;
    while (hi - b > 1) {
        const int mid = (b + hi) >> 1;
        if (L.pre[mid] <= x) b = mid;
        else hi = mid;
    }
    const LBox B = L.bx[b];
    long long t = (long long)(x - L.pre[b]) * kLBlock + threadIdx.x;
    const long long s0 = B.s0, s1 = B.s1, ng2 = 2LL * B.ng;
    const long long cz = ng2 * s1 * s0;
    const long long cy = (long long)B.n[2] * ng2 * s0;
    const long long cx = (long long)B.n[2] * B.n[1] * ng2;
    if (t >= cz + cy + cx) return false;
    int i, j, k;
    if (t < cz) {
        i = (int)(t % s0) - B.ng;
        t /= s0;
        j = (int)(t % s1) - B.ng;
        const int kk = (int)(t / s1);
        k = kk < B.ng ? kk - B.ng : B.n[2] + (kk - B.ng);
    } else if (t < cz + cy) {
        t -= cz;
        i = (int)(t % s0) - B.ng;
        t /= s0;
        const int jj = (int)(t % ng2);
        j = jj < B.ng ? jj - B.ng : B.n[1] + (jj - B.ng);
        k = (int)(t / ng2);
    } else {
        t -= cz + cy;
        const int ii = (int)(t % ng2);
        i = ii < B.ng ? ii - B.ng : B.n[0] + (ii - B.ng);
        t /= ng2;
        j = (int)(t % B.n[1]);
        k = (int)(t / B.n[1]);
    }
    G.fx = G.fy = G.fz = 0;
    const int sx = dom_src(B.lo[0] + i, L.dom[0], L.bc_lo[0], L.bc_hi[0], G.fx);
    const int sy = dom_src(B.lo[1] + j, L.dom[1], L.bc_lo[1], L.bc_hi[1], G.fy);
    const int sz = dom_src(B.lo[2] + k, L.dom[2], L.bc_lo[2], L.bc_hi[2], G.fz);
    const int o = L.owner[((long long)(sz / L.G) * L.om1 + sy / L.G) * L.om0 + sx / L.G];
    const LBox S = L.bx[o];
    G.b = b;
    G.o = o;
    G.src = lcell(S, sx - S.lo[0], sy - S.lo[1], sz - S.lo[2]);
    G.dst = lcell(B, i, j, k);
    return true;
}

__global__ void __launch_bounds__(kLBlock) k_fill_level(LevelArgs L, double *const *Us)
{
    LGhost G;
    if (!level_ghost(L, G)) return;
    const long long scs = L.bx[G.o].cs, dcs = L.bx[G.b].cs;
    const double *U = Us[G.o];
    double *V = Us[G.b];
    const long long src = G.src, dst = G.dst;
    const double r = U[src], mu = U[scs + src], mv = U[2 * scs + src],
                 mw = U[3 * scs + src], e = U[4 * scs + src];
    V[dst] = r;
    V[dcs + dst] = G.fx ? -mu : mu;
    V[2 * dcs + dst] = G.fy ? -mv : mv;
    V[3 * dcs + dst] = G.fz ? -mw : mw;
    V[4 * dcs + dst] = e;
}

// the same for ns species components (no sign flip)
__global__ void __launch_bounds__(kLBlock) k_fill_level_species(LevelArgs L, double *const *Ss,
                                                                  int ns)
{
    LGhost G;
    if (!level_ghost(L, G)) return;
    const long long scs = L.bx[G.o].cs, dcs = L.bx[G.b].cs;
    const double *S = Ss[G.o];
    double *V = Ss[G.b];
    for (int c = 0; c < ns; ++c) V[c * dcs + G.dst] = S[c * scs + G.src];
}

struct LevelPlan {
    int nb;
    long long blocks;
    LevelArgs args;
    void *dev;  // [LBox nb][unsigned pre nb+1][int owner]
};

bool bc_ok(int bc) { return bc >= HYDRO_BC_PERIODIC && bc <= HYDRO_BC_REFLECT; }

}  // namespace

extern "C" {

hydro_status hydro_level_create(const hydro_box *boxes, const int32_t *lo, int nb,
                                const int32_t *dom, const int32_t *bc_lo,
                                const int32_t *bc_hi, void **level)
{
    if (!level) return HYDRO_EINVAL;
    *level = nullptr;
    if (!boxes || !lo || nb < 1 || !dom || !bc_lo || !bc_hi) return HYDRO_EINVAL;
    long long dvol = 1;
    for (int d = 0; d < 3; ++d) {
        if (dom[d] < 1 || dom[d] > (1 << 20) || !bc_ok(bc_lo[d]) || !bc_ok(bc_hi[d]))
            return HYDRO_EINVAL;
        if ((bc_lo[d] == HYDRO_BC_PERIODIC) != (bc_hi[d] == HYDRO_BC_PERIODIC))
            return HYDRO_EINVAL;
        dvol *= dom[d];
    }
    std::vector<LBox> bx(nb);
    std::vector<unsigned> pre(nb + 1, 0);
    long long vol = 0, blocks = 0;
    int G = 0;
    for (int b = 0; b < nb; ++b) {
        const hydro_box &h = boxes[b];
        if (hydro_state_elems(&h) == 0) return HYDRO_EINVAL;
        LBox &B = bx[b];
        long long cells = 1, grown = 1;
        for (int d = 0; d < 3; ++d) {
            const long long l = lo[3 * b + d];
            if (l < 0 || l + h.n[d] > dom[d] || h.ng > dom[d]) return HYDRO_EINVAL;
            B.n[d] = h.n[d];
            B.lo[d] = (int)l;
            G = std::gcd(G, std::gcd((int)l, h.n[d]));
            cells *= h.n[d];
            grown *= (long long)h.n[d] + 2 * h.ng;
        }
        B.ng = h.ng;
        B.s0 = h.n[0] + 2 * h.ng;
        B.s1 = h.n[1] + 2 * h.ng;
        B.cs = grown;
        vol += cells;
        pre[b] = (unsigned)blocks;
        blocks += (grown - cells + kLBlock - 1) / kLBlock;
        if (blocks >= (1LL << 31)) return HYDRO_EINVAL;
    }
    pre[nb] = (unsigned)blocks;
    if (vol != dvol) return HYDRO_EINVAL;
    for (int d = 0; d < 3; ++d) G = std::gcd(G, (int)dom[d]);
    const int om0 = dom[0] / G, om1 = dom[1] / G, om2 = dom[2] / G;
    if ((long long)om0 * om1 * om2 > kMaxOwnerCells) return HYDRO_EINVAL;
    // owner map: the boxes' volumes add up to the domain's, so no overlap
    // means they cover it
    std::vector<int> owner((size_t)om0 * om1 * om2, -1);
    for (int b = 0; b < nb; ++b) {
        const LBox &B = bx[b];
        for (int k = B.lo[2] / G; k < (B.lo[2] + B.n[2]) / G; ++k)
            for (int j = B.lo[1] / G; j < (B.lo[1] + B.n[1]) / G; ++j)
                for (int i = B.lo[0] / G; i < (B.lo[0] + B.n[0]) / G; ++i) {
                    int &w = owner[((size_t)k * om1 + j) * om0 + i];
                    if (w >= 0) return HYDRO_EINVAL;
                    w = b;
                }
    }
    const size_t nbx = sizeof(LBox) * nb, npre = sizeof(unsigned) * (nb + 1),
                 nown = sizeof(int) * owner.size();
    const size_t opre = (nbx + 255) & ~(size_t)255, oown = (opre + npre + 255) & ~(size_t)255;
    LevelPlan *P = new (std::nothrow) LevelPlan();
    if (!P) return HYDRO_EINVAL;
    if (hipMalloc(&P->dev, oown + nown) != hipSuccess) {
        delete P;
        return HYDRO_EHIP;
    }
    char *base = (char *)P->dev;
    if (hipMemcpy(base, bx.data(), nbx, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(base + opre, pre.data(), npre, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(base + oown, owner.data(), nown, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(P->dev);
        delete P;
        return HYDRO_EHIP;
    }
    P->nb = nb;
    P->blocks = blocks;
    LevelArgs &A = P->args;
    A.bx = (const LBox *)base;
    A.pre = (const unsigned *)(base + opre);
    A.owner = (const int *)(base + oown);
    A.nb = nb;
    for (int d = 0; d < 3; ++d) {
        A.dom[d] = dom[d];
        A.bc_lo[d] = bc_lo[d];
        A.bc_hi[d] = bc_hi[d];
    }
    A.G = G;
    A.om0 = om0;
    A.om1 = om1;
    *level = P;
    return HYDRO_OK;
}

void hydro_level_destroy(void *level)
{
    LevelPlan *P = (LevelPlan *)level;
    if (!P) return;
    (void)hipFree(P->dev);
    delete P;
}

hydro_status hydro_fill_ghosts_level(int nb, double *const *U_ptrs_dev, const void *level,
                                     void *stream)
{
    const LevelPlan *P = (const LevelPlan *)level;
    if (!P || nb != P->nb || !U_ptrs_dev) return HYDRO_EINVAL;
    if (P->blocks == 0) return HYDRO_OK;
    hipLaunchKernelGGL(k_fill_level, dim3((unsigned)P->blocks), dim3(kLBlock), 0,
                       (hipStream_t)stream, P->args, U_ptrs_dev);
    return hipGetLastError() == hipSuccess ? HYDRO_OK : HYDRO_EHIP;
}

hydro_status hydro_fill_ghosts_level_species(int nb, double *const *S_ptrs_dev, int nspec,
                                             const void *level, void *stream)
{
    const LevelPlan *P = (const LevelPlan *)level;
    if (!P || nb != P->nb || !S_ptrs_dev || nspec < 1 || nspec > 8) return HYDRO_EINVAL;
    if (P->blocks == 0) return HYDRO_OK;
    hipLaunchKernelGGL(k_fill_level_species, dim3((unsigned)P->blocks), dim3(kLBlock), 0,
                       (hipStream_t)stream, P->args, S_ptrs_dev, nspec);
    return hipGetLastError() == hipSuccess ? HYDRO_OK : HYDRO_EHIP;
}

}  // extern "C"
