/*
 * hydro.h -- C ABI of the MI355X (gfx950) FP64 hydrodynamics library.
 *
 * One time step of the unsplit corner-transport-upwind (CTU) PPM scheme with
 * an HLLC Riemann solver for a gamma-law gas, on boxes of cells with ghost
 * layers.  The paper (Katz et al. 2020) describes this hydro only in outline
 * -- a slope stencil over neighbouring zones reconstructing a polynomial
 * (Sec. III), boxes of multi-component fluid data distributed as a list
 * (Sec. II, Fig. 1), small boxes batched over streams (Sec. IV-A), a timestep
 * proportional to the zone width (Sec. V) -- and takes the scheme from its
 * Castro reference (bibliography entry CastroI).
 *
 * Conventions for every entry point:
 *  - Pointers named *_dev are device pointers; box/params descriptors are
 *    host pointers unless named *_dev.  The caller owns every buffer; the
 *    library never allocates or frees device memory in these calls (plans
 *    own one device buffer, allocated in hydro_plan_create).
 *  - All work is enqueued on `stream` (a hipStream_t; NULL = the null
 *    stream) and is asynchronous: no call synchronises the host.
 *  - Argument errors are reported synchronously (HYDRO_EINVAL, nothing is
 *    enqueued); launch failures return HYDRO_EHIP.  Numerical problems are
 *    OR-ed into the caller's device int32 *err_dev (HYDRO_ERR_* bits), which
 *    the caller reads after synchronising.  No call throws or aborts.
 *  - The timestep is passed by device pointer so a whole step can be
 *    captured in a HIP graph.
 *  - Calls on different streams with disjoint buffers do not interact.
 *
 * State layout (a "Fab", Sec. II): a box has n[3] valid cells and ng ghost
 * layers per side.  One component is a dense array of s0*s1*s2 doubles,
 * s_d = n_d + 2 ng, x fastest; the five components rho, rho*u, rho*v, rho*w,
 * E (total energy density) follow one another (structure of arrays).  Cell
 * (i,j,k), -ng <= i < n0+ng, lives at ((k+ng)*s1 + (j+ng))*s0 + (i+ng).
 * hydro_state_elems() gives the total number of doubles (5 s0 s1 s2).
 *
 * Arithmetic: IEEE binary64 throughout, no fused multiply-add contraction,
 * correctly rounded division and square root; results do not depend on the
 * launch configuration, on the batch a box is advanced in, or on the
 * stream.
 */
#ifndef HYDRO_H
#define HYDRO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HYDRO_OK = 0,
    HYDRO_EINVAL = 1, /* invalid argument; nothing enqueued            */
    HYDRO_EHIP = 2,   /* a HIP runtime call or kernel launch failed     */
    HYDRO_ENOWS = 3   /* the workspace passed is smaller than required  */
} hydro_status;

typedef enum {
    HYDRO_BC_PERIODIC = 0, /* ghost = valid cell one period away               */
    HYDRO_BC_OUTFLOW = 1,  /* ghost = nearest valid cell (zero gradient)       */
    HYDRO_BC_REFLECT = 2   /* ghost = mirror image, normal momentum negated     */
} hydro_bc;

/* error bits OR-ed into *err_dev */
enum {
    HYDRO_ERR_NONFINITE = 1, /* an updated value is NaN or Inf                       */
    HYDRO_ERR_RHO = 2,       /* an updated density is <= 0                           */
    HYDRO_ERR_P = 4,         /* an updated pressure is <= 0                          */
    HYDRO_ERR_FALLBACK = 8   /* a transverse-corrected face state had rho<=0 or p<=0 and
                                the uncorrected state was used (informational)       */
};

/* A box (Sec. II "Box"/"Fab"): 64 bytes, 8-byte aligned.  One component
 * (with ghosts) must stay below 2^28 doubles (2 GiB), e.g. up to 636^3 valid
 * cells with 4 ghost layers; larger domains are split into boxes. */
typedef struct hydro_box {
    int32_t n[3];     /* valid cells per axis, >= 1; >= ng on periodic/reflect axes */
    int32_t ng;       /* ghost layers per side, 3 <= ng <= 8 (the stencil reads 3)  */
    double dx[3];     /* cell widths, > 0                                           */
    int32_t bc_lo[3]; /* hydro_bc at the low face of each axis                      */
    int32_t bc_hi[3]; /* hydro_bc at the high face; periodic must be paired         */
} hydro_box;

/* Physical and numerical parameters. */
typedef struct hydro_params {
    double gamma;    /* ratio of specific heats, > 1                    */
    double cfl;      /* Courant number, 0 < cfl <= 1                    */
    double grav[3];  /* constant gravitational acceleration (lab axes)  */
    int32_t flatten; /* shock flattening of the PPM parabolae (Colella &
                        Woodward 1984, Sec. 4; the paper's Castro hydro
                        uses it for its Sedov runs): 0 off, 1 on.  On needs
                        ng >= 4 in every box advanced (HYDRO_EINVAL
                        otherwise); where no cell meets the shock test the
                        results are bitwise those with it off            */
} hydro_params;

/* Doubles in one state array of `box` (all five components, with ghosts);
 * 0 for an invalid box. */
size_t hydro_state_elems(const hydro_box *box);

/* Device workspace, in bytes, that advance_box (nboxes = 1) or advance_boxes
 * needs for these boxes; 0 for invalid boxes. */
size_t hydro_workspace_bytes(const hydro_box *boxes, int nboxes);

/* Ghost fill (the neighbour data of Sec. II/IV-A): every ghost cell of U_dev
 * takes the value of the valid cell it maps to under the box's boundary
 * kinds, mapped axis by axis, so edges and corners are defined; reflected
 * axes negate their momentum component.  In place. */
hydro_status hydro_fill_ghosts(double *U_dev, const hydro_box *box, void *stream);

/* CFL timestep (Sec. V: dt proportional to the zone width): fills the
 * ghosts of U_dev (as hydro_fill_ghosts), then writes to *dt_dev
 *     dt = cfl * min over axes d of dx_d / max over valid cells (|u_d| + c),
 * c = sqrt(gamma p / rho).  The result is exact (min/max are exact) and
 * independent of the launch.  *dt_dev is used as the reduction's accumulator;
 * no other scratch is needed.  For a state with rho <= 0 or p <= 0 or
 * non-finite values somewhere (what advance_box flags with error bits 1, 2,
 * 4) the value is unspecified. */
hydro_status estimate_dt(double *U_dev, const hydro_box *box, const hydro_params *prm,
                         double *dt_dev, void *stream);

/* One CTU-PPM-HLLC step of length *dt_dev (Sec. III's reconstruction
 * stencil; the scheme of the paper's CastroI reference): writes the valid
 * cells of U_new_dev from U_dev, whose ghosts must be filled (estimate_dt
 * does it).  Ghost cells of U_new_dev are not written.  U_new_dev must not
 * overlap U_dev.  ws_dev must hold hydro_workspace_bytes(box, 1) bytes
 * (HYDRO_ENOWS otherwise), aligned to 256 bytes, overlapping neither state
 * (HYDRO_EINVAL); its contents on entry do not matter.  Error bits go to *err_dev (not cleared by the call).
 * If dt_next_dev is not NULL it receives the CFL timestep of the new state,
 * bitwise what estimate_dt gives for U_new_dev (its valid cells decide it),
 * reduced in the update's epilogue instead of a separate pass over U_new:
 * a stepping loop then needs only hydro_fill_ghosts before the next
 * advance_box.  It must not overlap *dt_dev (HYDRO_EINVAL).  When the
 * new state raises error bit 1, 2 or 4 the value is unspecified. */
hydro_status advance_box(const double *U_dev, double *U_new_dev, const hydro_box *box,
                         const hydro_params *prm, const double *dt_dev, double *dt_next_dev,
                         void *ws_dev, size_t ws_bytes, int32_t *err_dev, void *stream);

/* advance_box for callers that cannot allocate device memory (code under
 * HIP graph capture that must not call hipMalloc, tight serving loops,
 * harnesses that forbid allocation): the same step, bitwise the same results
 * and the same argument rules, without a workspace argument.  The traced
 * states live instead in a static device array of HYDRO_NOALLOC_WS_BYTES
 * (128 MiB) that the library holds on every GPU it runs on until the process
 * ends; the call allocates nothing.  Boxes whose workspace
 * (hydro_workspace_bytes(box, 1)) exceeds it -- a 78^3 box fits, a 79^3
 * box does not -- return HYDRO_ENOWS with nothing enqueued.  All calls on one GPU
 * share that array: calls whose work overlaps in time on one GPU (different
 * streams, or host threads without ordering between them) race and give
 * wrong results; calls ordered on one stream are safe.  Its contents on entry
 * do not matter (the call writes every value it reads).  The first call on a
 * device looks up the array's address there (HYDRO_EHIP if that fails). */
#define HYDRO_NOALLOC_WS_BYTES ((size_t)128 << 20)
hydro_status advance_box_noalloc(const double *U_dev, double *U_new_dev, const hydro_box *box,
                                 const hydro_params *prm, const double *dt_dev,
                                 double *dt_next_dev, int32_t *err_dev, void *stream);

/* Passively advected species (the multi-component fluid state of Sec. II's
 * Fabs; the isotopes a reaction network follows, Sec. IV-B): nspec mass
 * fractions X_s (1 <= nspec <= 8) carried by the gas, held as partial
 * densities rho X_s in their own array: nspec components in the state
 * layout (component s at offset s * s0 s1 s2 doubles).
 *
 * Species workspace, in bytes, that advance_box_species needs for this box
 * and species count: the mass fluxes of every Riemann solve of the gas step
 * (twelve face fields), which the species pass reads; the species' own face
 * values never leave the chip, so the size does not grow with nspec.  0 for
 * invalid arguments. */
size_t hydro_species_workspace_bytes(const hydro_box *box, int nspec);

/* Ghost fill of the species array S_dev by the rules of hydro_fill_ghosts,
 * with no sign flip at reflecting faces.  In place. */
hydro_status hydro_fill_ghosts_species(double *S_dev, int nspec, const hydro_box *box,
                                       void *stream);

/* advance_box, plus the same step for the species: S_new_dev receives the
 * valid cells of rho X_s after the step, from S_dev (ghosts filled).  The gas
 * arguments and results are exactly those of advance_box (its new state is
 * identical bit for bit).  Through every face the species flux is the mass
 * flux of the same Riemann solve times the mass fraction of the side the
 * mass leaves (the low side for a zero flux); face values of X are traced
 * like a transverse velocity (they change across the contact wave only), and
 * corrected like the density: each transverse-corrected X is the corrected
 * partial density over the corrected density, formed from the same flux
 * differences, the traced X kept where that density is not positive.
 * sws_dev (sws_bytes >= hydro_species_workspace_bytes(box, nspec), else
 * HYDRO_ENOWS; 256-byte aligned) is scratch whose contents on entry do not
 * matter.  No array written (U_new_dev, S_new_dev, ws_dev, sws_dev) may
 * overlap another of the arrays passed (HYDRO_EINVAL).  A
 * non-finite new partial density raises error bit 1. */
hydro_status advance_box_species(const double *U_dev, double *U_new_dev, const double *S_dev,
                                 double *S_new_dev, int nspec, const hydro_box *box,
                                 const hydro_params *prm, const double *dt_dev,
                                 double *dt_next_dev, void *ws_dev, size_t ws_bytes,
                                 void *sws_dev, size_t sws_bytes, int32_t *err_dev, void *stream);

/* Species of a batch of boxes (the plan's boxes, in its order): the species
 * workspace that advance_boxes_species needs for them (the sum of
 * hydro_species_workspace_bytes over the boxes); 0 for invalid arguments. */
size_t hydro_species_workspace_bytes_boxes(const hydro_box *boxes, int nb, int nspec);

/* hydro_fill_ghosts_species for every box of a plan, each by its own
 * boundary kinds, in one launch; S_ptrs_dev: device array of nb species
 * pointers.  For boxes that tile one domain use
 * hydro_fill_ghosts_level_species. */
hydro_status hydro_fill_ghosts_boxes_species(int nb, double *const *S_ptrs_dev, int nspec,
                                             const void *plan, void *stream);

/* advance_boxes plus the species of every box (as advance_box_species does
 * for one box): S_ptrs_dev / S_new_ptrs_dev are device arrays of nb species
 * pointers (ghosts of the S arrays filled); the gas arguments and results
 * are exactly those of advance_boxes.  sws_dev: at least
 * hydro_species_workspace_bytes_boxes(boxes, nb, nspec) bytes (HYDRO_ENOWS
 * otherwise), 256-byte aligned, not overlapping ws_dev (HYDRO_EINVAL); box
 * b's part lies at the sum of the earlier boxes' sizes.  The S arrays of
 * different boxes must not overlap, nor any S_new array any other array. */
hydro_status advance_boxes_species(int nb, const double *const *U_ptrs_dev,
                                   double *const *U_new_ptrs_dev,
                                   const double *const *S_ptrs_dev,
                                   double *const *S_new_ptrs_dev, int nspec, const void *plan,
                                   const hydro_params *prm, const double *dt_dev, int dt_stride,
                                   double *dt_next_dev, double *dt_next_min_dev, void *ws_dev,
                                   size_t ws_bytes, void *sws_dev, size_t sws_bytes,
                                   int32_t *err_dev, void *stream);

/* Batched timestep over a list of boxes (a level of Sec. II's MultiFab):
 * fills the ghosts of every box, writes each box's dt to dt_dev[b] and, if
 * dt_min_dev is not NULL, the minimum over boxes to *dt_min_dev.
 * U_ptrs_dev[b] (device array of nb device pointers) is box b's state;
 * `boxes` is the host array of nb boxes given to hydro_plan_create for
 * `plan`.  Each dt_dev[b] is bitwise the value estimate_dt gives for box b. */
hydro_status estimate_dt_boxes(int nb, double *const *U_ptrs_dev, const void *plan,
                               const hydro_params *prm, double *dt_dev,
                               double *dt_min_dev, void *stream);

/* Batched step (Sec. IV-A: many boxes per GPU instead of one stream per
 * box): advances every box of `plan` by its own timestep dt_dev[b]
 * (dt_stride = 1) or by one shared timestep dt_dev[0] (dt_stride = 0), with
 * one launch per stage for all boxes together.  Every box's result is
 * bitwise the one advance_box gives it.  ws_dev must hold
 * hydro_workspace_bytes(boxes, nb) bytes.  If dt_next_dev is not NULL,
 * dt_next_dev[b] receives box b's next timestep as advance_box's dt_next_dev
 * does, and, if dt_next_min_dev is not NULL too, *dt_next_min_dev the
 * minimum over boxes (bitwise what estimate_dt_boxes gives for the new
 * states); neither may overlap the timesteps in use or each other. */
hydro_status advance_boxes(int nb, const double *const *U_ptrs_dev,
                           double *const *U_new_ptrs_dev, const void *plan,
                           const hydro_params *prm, const double *dt_dev, int dt_stride,
                           double *dt_next_dev, double *dt_next_min_dev, void *ws_dev,
                           size_t ws_bytes, int32_t *err_dev, void *stream);

/* Ghost fill of every box of `plan` (hydro_fill_ghosts per box, one launch):
 * with the timesteps advance_boxes reduced, a batched stepping loop is
 * hydro_fill_ghosts_boxes + advance_boxes. */
hydro_status hydro_fill_ghosts_boxes(int nb, double *const *U_ptrs_dev, const void *plan,
                                     void *stream);

/* A level whose boxes tile one problem domain (Sec. II: a level's boxes
 * cover the domain, and a box's stencil reads neighbour data from the boxes
 * next to it).  boxes[b] (valid cells n, ghost depth ng) has its valid cell
 * (0,0,0) at domain index lo[3b .. 3b+2]; the boxes must cover the
 * dom[0] x dom[1] x dom[2] domain exactly, without overlap, and every ng
 * must be <= each dom[d].  bc_lo/bc_hi are the domain's boundary kinds
 * (periodic paired); the boxes' own bc fields are not used by the level.
 * The owner map the level keeps has (D0/G)(D1/G)(D2/G) entries, G the
 * greatest common divisor of all box corners, sides and domain sizes; more
 * than 2^24 entries is HYDRO_EINVAL.  *level receives an opaque handle that
 * owns one device buffer; HYDRO_EINVAL for an invalid or non-tiling layout,
 * HYDRO_EHIP if the device buffer cannot be set up. */
hydro_status hydro_level_create(const hydro_box *boxes, const int32_t *lo, int nb,
                                const int32_t *dom, const int32_t *bc_lo,
                                const int32_t *bc_hi, void **level);
void hydro_level_destroy(void *level);

/* Ghost exchange of a level (a FillBoundary analogue), one launch: every
 * ghost cell of every box takes the value that the whole domain, held as one
 * box with the level's boundary kinds and filled by hydro_fill_ghosts, has at
 * the same domain index -- from the neighbouring box that owns it, across a
 * periodic face, or by the outflow/reflect rule at a domain face.  Bitwise
 * copies (reflection only negates).  U_ptrs_dev: device array of nb state
 * pointers in the level's box order; states must not overlap.  With the
 * timesteps that advance_boxes reduces, a stepping loop over a tiled domain
 * is hydro_fill_ghosts_level + advance_boxes with the shared timestep, and
 * every box's new valid cells equal the whole domain's advanced as one box. */
hydro_status hydro_fill_ghosts_level(int nb, double *const *U_ptrs_dev, const void *level,
                                     void *stream);

/* The ghost exchange of hydro_fill_ghosts_level for the species arrays of
 * the level's boxes (nspec components each, no sign flip at reflecting
 * faces).  S_ptrs_dev: device array of nb species pointers. */
hydro_status hydro_fill_ghosts_level_species(int nb, double *const *S_ptrs_dev, int nspec,
                                             const void *level, void *stream);

/* Plan for a fixed list of boxes: validates them, chooses the tile shapes
 * (autotune_json: NULL for the built-in choice, else a JSON object mapping
 * box shapes "NXxNYxNZ" to [tbx, tzs] for both fused kernels or
 * [tbx1, tzs1, tbx2, tzs2] for the trace and flux kernels: tile width
 * tbx in {8,16,18,32} (trace kernel: tiles of tbx1 x 256/tbx1 columns;
 * flux kernel: rows of tbx2 lanes, 64/tbx2 whole rows per wavefront, four
 * wavefronts, the outer ring of columns supplying neighbours), z-segment
 * length tzs >= 1 (at most: a box's planes are split into equal segments no
 * longer than tzs); a pair 0, 0 keeps that kernel's built-in tile; as written by
 * the package's autotuner) and builds the device work list.  *plan receives
 * an opaque handle.  HYDRO_EINVAL for an invalid box or table. */
hydro_status hydro_plan_create(const hydro_box *boxes, int nb, const char *autotune_json,
                               void **plan);

/* A plan whose list of boxes changes while it is in use (the serving loop
 * of Sec. III's device-resident data: runs join and leave a batch while
 * their states stay on the GPU).  hydro_plan_create_capacity makes an empty
 * plan for lists of up to `capacity` boxes (1 <= capacity <= 2^20), with
 * the tile table as in hydro_plan_create; it allocates the plan's device
 * buffer and a few pinned host staging buffers once.  Until its first
 * update the plan has no boxes and every batched call on it is
 * HYDRO_EINVAL.  HYDRO_EHIP if an allocation fails. */
hydro_status hydro_plan_create_capacity(int capacity, const char *autotune_json, void **plan);

/* Replace the plan's list by boxes[0..nb) (1 <= nb <= capacity; the host
 * array is read during the call only).  The new work lists are written to a
 * pinned staging buffer and copied to the plan's device buffer with an
 * asynchronous copy on `stream`, so batched calls enqueued afterwards on
 * that stream use the new list and calls enqueued before it the old one:
 * every call using the plan must be on that one stream.  The host blocks
 * only when all staging buffers still wait for earlier copies (the copy
 * enqueued four updates back).  No device memory is allocated.  Box b of the
 * new list is the b-th pointer of the pointer arrays the batched calls take;
 * the workspace they need becomes hydro_plan_workspace_bytes(plan).
 * HYDRO_EINVAL (plan unchanged) for an invalid box, nb out of range, or a
 * plan made by hydro_plan_create. */
hydro_status hydro_plan_update(void *plan, const hydro_box *boxes, int nb, void *stream);

/* Boxes in the plan's current list (0 for an empty capacity plan, -1 for
 * NULL), and the workspace in bytes that the batched calls need for it. */
int hydro_plan_boxes(const void *plan);
size_t hydro_plan_workspace_bytes(const void *plan);

/* Release a plan (waiting for its pending staging copies). */
void hydro_plan_destroy(void *plan);

/* Profiling aid.  The library's kernels form hydro_stage_count() stage
 * groups (hydro_stage_name(s): "fill", "dt", ... in launch order).  After
 * hydro_set_stage_events(ev) with ev an array of 2*hydro_stage_count() HIP
 * events (hipEvent_t, created by the caller), every call records ev[2s] on
 * its stream before the first launch of stage group s and ev[2s+1] after the
 * last, so the caller can read each group's device time with
 * hipEventElapsedTime after synchronising.  NULL switches recording off.
 * Process-wide setting; not meant for concurrent calls. */
int hydro_stage_count(void);
const char *hydro_stage_name(int s);
hydro_status hydro_set_stage_events(void *const *events);

/* Human-readable name of a status code (static string). */
const char *hydro_status_string(hydro_status st);

#ifdef __cplusplus
}
#endif
#endif /* HYDRO_H */
