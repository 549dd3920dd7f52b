/*
 * af.h -- C ABI of the MI355X Active Flux patch-step library (libaf.so).
 *
 * The library advances the Cartesian-grid Active Flux (AF) method of
 * Calhoun, Chudzik & Helzel (arXiv 2205.07572) on a quadtree of equal-size
 * patches on one AMD Instinct MI355X (gfx950) GPU.
 *
 * Method (Sec. 2): each cell carries its average and the point values at its
 * corners and edge midpoints; cell (i,j) owns the average Q_ij, the left-edge
 * midpoint Q_{i-1/2,j}, the bottom-left corner Q_{i-1/2,j-1/2} and the
 * bottom-edge midpoint Q_{i,j-1/2}.  A step reconstructs the continuous
 * biquadratic in every cell, evolves the point values to t+dt/2 and t+dt
 * with the exact operators of linear advection (Sec. 2.1), of advection in
 * the solid-body rotation field (Sec. 4.2, exact characteristic circles) or
 * of acoustics (Sec. 2.3, Eymann-Roe formula), forms Simpson space-time fluxes
 * (eq. Simpson-2d) and updates the averages conservatively (eq. 2dfv).
 * Patches exchange data through two ghost layers (Sec. 3.1, 3.2), finer
 * levels subcycle (Sec. 3.2) and the coarse-fine flux mismatch is repaired
 * by the Berger-Colella fix (Sec. 3.2, global conservation).
 *
 * Conventions common to every call
 *  - All state, flux-register, tag and value buffers are caller-owned DEVICE
 *    memory; the library never frees them.  Library-owned objects (af_ctx,
 *    af_hier) hold only small tables.
 *  - Every launching call takes a hipStream_t (0 = the null stream) and is
 *    asynchronous.  Arguments are validated on the host before anything is
 *    launched; on error nothing is launched.
 *  - Every call returns af_status (AF_OK = 0, negative on error);
 *    af_last_error() returns a thread-local message for the last failure.
 *  - Periodic boundaries on the rectangle [x0,x0+lx] x [y0,y0+ly].
 *
 * State layout (af_state)
 *  Four arrays dof[k], k = AF_AVG, AF_CORNER, AF_XEDGE, AF_YEDGE, each of
 *  shape [ncomp][npatch][m+5][pitch] of the problem precision (double for
 *  AF_FP64, float for AF_FP32), ncomp = 1 (advection and rotation, q) or 3
 *  (acoustics, p,u,v).  Row r, column c of a patch plane hold the DOF of local index
 *  (i,j) = (c-2, r-2): cells of the interior are i,j in [0,m), the two ghost
 *  layers extend to [-2, m+2).  Valid entries: avg i,j in [-2,m+2); corner
 *  i,j in [-2,m+2]; xedge (point (x_{i-1/2}, y_j)) i in [-2,m+2], j in
 *  [-2,m+2); yedge (point (x_i, y_{j-1/2})) i in [-2,m+2), j in [-2,m+2].
 *  Other entries are padding.  pitch >= m+5.
 */
#ifndef AF_H
#define AF_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AF_OK = 0,
  AF_ERR_ARG = -1,      /* bad argument value or combination */
  AF_ERR_CFL = -2,      /* time step violates eq. cfl-adv (with the largest speed) or eq. cfl-acoustics */
  AF_ERR_LAYOUT = -3,   /* bad pitch / patch count / alignment */
  AF_ERR_BALANCE = -4,  /* leaf set is not a 2:1 corner-balanced cover */
  AF_ERR_DEVICE = -5,   /* HIP runtime error */
  AF_ERR_STATE = -6     /* call not valid in the object's current state */
} af_status;

/* AF_ROTATION: q_t + (a q)_x + (b q)_y = 0 with a = -omega (y - yc),
 * b = omega (x - xc) (Sec. 4.2, eq. solidbody).  The field is not periodic;
 * the data are, so results are those of the paper's test as long as the
 * data vanish near the domain boundary.
 * AF_SWIRL: the same equation with the time-dependent field of Sec. 4.3,
 * a = -(Psi(x, y + dy/2, t) - Psi(x, y - dy/2, t))/dy, b = (Psi(x + dx/2, y,
 * t) - Psi(x - dx/2, y, t))/dx, Psi = sin^2(pi x) sin^2(pi y) cos(pi t)/pi
 * (eq. swirlODE, dx, dy of the level), feet by one classical Runge-Kutta
 * step backwards in time, fluxes with the face-midpoint velocity at each
 * Simpson time (eq. swirlF, swirlG).  |a|, |b| <= 1.
 * AF_BURGERS: q_t + (q^2/2)_x + (q^2/2)_y = 0 (Sec. 2.2, eq. burgers2d),
 * unlimited.  Each point value is found from q = q^n(P - q tau (1, 1))
 * (eq. burgers-sol) by two fixed-point iterations (eq. Burgers-iterativ)
 * started from the mean of the cell averages around the node; fluxes are
 * the Simpson rule of q^2/2.  qmax bounds |q| for the CFL check; the source
 * cell of a foot is kept within the one-cell stencil, so a step whose
 * iterates exceed qmax reads no memory outside the patch block. */
typedef enum { AF_ADVECTION = 0, AF_ACOUSTICS = 1, AF_ROTATION = 2, AF_SWIRL = 3, AF_BURGERS = 4 } af_equation;
typedef enum { AF_FP64 = 0, AF_FP32 = 1 } af_precision;
enum { AF_AVG = 0, AF_CORNER = 1, AF_XEDGE = 2, AF_YEDGE = 3 };
enum { AF_SIDE_W = 0, AF_SIDE_E = 1, AF_SIDE_S = 2, AF_SIDE_N = 3 };
/* step regions (Sec. 3.2: "the first layer of ghost cells is updated along
 * with all interior cells") */
enum { AF_REGION_INTERIOR = 0, AF_REGION_LAYER1 = 1 };
/* tagging criteria (Sec. 4.1: q_max - q_min per patch; Sec. 4.4: centred
 * gradient) */
enum { AF_TAG_GRADIENT = 0, AF_TAG_MAXMIN = 1 };

typedef struct {
  int32_t eq;          /* af_equation */
  int32_t prec;        /* af_precision: AF_FP32 = FP32 state and arithmetic,
                          FP64 flux registers and sums */
  int32_t m;           /* interior cells per patch side: even, 4..128 */
  int32_t n0x, n0y;    /* level-0 patches per side */
  int32_t lmax;        /* finest level a hierarchy may hold (<= 12) */
  double x0, y0, lx, ly; /* periodic domain */
  double a, b;         /* advection velocity (eq. advection2d) */
  double c;            /* speed of sound (eq. acoustics) */
  double omega;        /* AF_ROTATION: angular velocity (pi in Sec. 4.2) */
  double xc, yc;       /* AF_ROTATION: centre of rotation */
  double qmax;         /* AF_BURGERS: bound on |q| over the run (CFL check), > 0 */
} af_problem;

typedef struct {
  void* dof[4];        /* device pointers, see "State layout" */
  int32_t npatch;      /* patches the arrays hold (>= leaves addressed) */
  int32_t pitch;       /* row pitch in elements, >= m+5 */
} af_state;

typedef struct af_ctx af_ctx;
typedef struct af_hier af_hier;

const char* af_last_error(void);

/* Context: validates the problem and keeps its constants.  Owns nothing on
 * the device except a small reduction workspace. */
af_status af_ctx_create(const af_problem* prob, af_ctx** out);
af_status af_ctx_destroy(af_ctx* ctx);
/* Patch-step tile height (cell rows of one patch per 256-thread block);
 * supported: m=8: 8; m=16: 8,16; m=32: 4,8; m=64: 2,4; m=128: 2.  The
 * autotuner picks it; results do not depend on it. */
af_status af_ctx_set_tile(af_ctx* ctx, int32_t ty);
int32_t af_ctx_get_tile(const af_ctx* ctx);
/* Fused pairs of finest-level substeps in the batched coarse step of
 * af_amr_coarse_step (on = 1, the default; off = 0): with m = 8 or 16 and a
 * finest level F >= 2, one block takes both substeps of a pair of level F
 * (Sec. 3.2) from one staging of its halo, the first (layer-1 region) into
 * on-chip memory, the second from there, and the launches of the odd time
 * points go away.  Results are bit-identical with it off; only which of the
 * two buffers holds level F in the middle of a coarse step differs.
 * AF_ERR_ARG for a null ctx or on not 0 or 1. */
af_status af_ctx_set_fused_pairs(af_ctx* ctx, int32_t on);
int32_t af_ctx_get_fused_pairs(const af_ctx* ctx); /* -1 for a null ctx */

/* ---------------------------------------------------------------------
 * Hierarchy (Sec. 3): a leaf set of the quadtree.  Leaf k is patch k of
 * every af_state used with it.  Leaves must be sorted by level (patches of
 * one level are a contiguous range); af_hier_regrid returns them sorted by
 * (level, iy, ix).  Creation checks that the leaves tile the domain exactly
 * and are 2:1 balanced across edges AND corners (periodic), else
 * AF_ERR_BALANCE.  The object holds host and device tables (per-level
 * patch lookup, side relations, coarse-fine face list); it is immutable.
 * --------------------------------------------------------------------- */
af_status af_hier_create(af_ctx* ctx, int32_t nleaves, const int32_t* level,
                         const int32_t* ix, const int32_t* iy, af_hier** out);
af_status af_hier_destroy(af_hier* h);
int32_t af_hier_num_leaves(const af_hier* h);
/* host arrays of length af_hier_num_leaves() */
af_status af_hier_get_leaves(const af_hier* h, int32_t* level, int32_t* ix, int32_t* iy);
/* leaves of `level` are [*first, *first + *count) */
af_status af_hier_level_range(const af_hier* h, int32_t level, int32_t* first, int32_t* count);
int32_t af_hier_finest_level(const af_hier* h);
/* side relation of each leaf, host int8 [n][4] (W,E,S,N): 0 same level,
 * -1 coarser neighbour, +1 finer neighbours */
af_status af_hier_side_relations(const af_hier* h, int8_t* rel);

/* ---------------------------------------------------------------------
 * af_patch_step -- one AF time step of `count` patches of one level
 * (Sec. 2: eq. poly, eq. advection-update / eq. ERFormula,
 * eq. Simpson-2d, eq. 2dfv).
 *   in, out    states (distinct buffers of equal layout); the patches
 *              [first, first+count) are read from `in` (interior and ghost
 *              layers must be current) and written to `out`.
 *   level      the patches' level; dx = lx/(n0x m 2^level), likewise dy.
 *   dt         time step; AF_ERR_CFL if max(|a| dt/dx, |b| dt/dy) > 1
 *              (advection, eq. cfl-adv; for AF_ROTATION with the largest
 *              |a| and |b| on the domain, for AF_SWIRL with |a|, |b| = 1)
 *              or c dt / min(dx,dy) > 1/2 (acoustics, eq. cfl-acoustics).
 *   t          time at the start of the step (used by AF_SWIRL only).
 *   region     AF_REGION_INTERIOR: averages of cells [0,m)^2 and all nodes
 *              of the closed square [0,m]^2 are written;
 *              AF_REGION_LAYER1: cells [-1,m+1)^2 and nodes [-1,m+1]^2.
 *              Other entries of `out` are left untouched.
 *   flux_reg   NULL, or FP64 registers [npatch][4][m][ncomp] (side-major
 *              W,E,S,N; index along the side); for every patch side whose
 *              bit is set in side_mask[patch] the step ADDS F*dy*dt (x-faces)
 *              or G*dx*dt (y-faces) of the m boundary faces of the interior.
 *   side_mask  device uint8 [npatch]; NULL = no recording.
 *   leaf_xy    device int32 [npatch][2]: (ix, iy) of each patch at its
 *              level (af_hier_leaf_xy), which places the patch at
 *              (x0 + ix m dx, y0 + iy m dy).  Required for AF_ROTATION and
 *              AF_SWIRL (AF_ERR_ARG if NULL), ignored otherwise.
 * --------------------------------------------------------------------- */
af_status af_patch_step(af_ctx* ctx, const af_state* in, af_state* out, int32_t first,
                        int32_t count, int32_t level, double dt, double t, int32_t region,
                        double* flux_reg, const uint8_t* side_mask, const int32_t* leaf_xy,
                        hipStream_t stream);

/* ---------------------------------------------------------------------
 * af_ghost_fill -- ghost data exchange between patches (Sec. 3.1 and
 * Sec. 3.2).  Each level's data lives in bufs[(level_buf_mask >> level) & 1]
 * (pass the same state twice and mask 0 for a single buffer).  For every
 * leaf of level >= tmin, every DOF outside its interior cells and strictly
 * inside-nodes is set from the leaves of level >= smin:
 *   averages: same level copy; finer: mean of the four fine averages
 *   (fine->coarse transfer); coarser: Simpson 3x3 of the coarse
 *   reconstruction over the fine cell (coarse->fine transfer);
 *   nodes: the finest leaf whose closed square contains the node
 *   (fine values win on coarse-fine lines); same/finer: copy the vertex,
 *   coarser: evaluate the coarse reconstruction.  Candidates of one level
 *   are tried in the order (hi,hi),(lo,hi),(hi,lo),(lo,lo).
 * DOFs without an admissible source keep their values (at non-synchronised
 * times the patch's own layer-1 values serve over coarser neighbours).
 * Two launches: same-level/fine->coarse, then coarse->fine.
 * --------------------------------------------------------------------- */
af_status af_ghost_fill(af_ctx* ctx, const af_hier* h, af_state* bufs, uint32_t level_buf_mask,
                        int32_t tmin, int32_t smin, hipStream_t stream);

/* ---------------------------------------------------------------------
 * af_flux_correct -- Berger-Colella conservative fix (Sec. 3.2) for all
 * coarse cells of `level` adjacent to leaves of level+1:
 *   Q_c += s (R_c - sum R_f) / (dx_c dy_c),  s = +1 (E,N sides), -1 (W,S),
 * with R_c the coarse register entry of the face and R_f the two fine
 * entries facing it (accumulated over the two fine substeps).  The
 * registers used are then zeroed.  flux_reg as in af_patch_step.
 * --------------------------------------------------------------------- */
af_status af_flux_correct(af_ctx* ctx, const af_hier* h, af_state* bufs,
                          uint32_t level_buf_mask, int32_t level, double* flux_reg,
                          hipStream_t stream);

/* ---------------------------------------------------------------------
 * af_regrid_tag -- per-patch refinement flag (Sec. 3; criteria of Sec. 4.1
 * and 4.4).  mode AF_TAG_GRADIENT: value = max over interior cells of
 * max(|Q_{i+1,j}-Q_{i-1,j}|/(2dx), |Q_{i,j+1}-Q_{i,j-1}|/(2dy)) of component
 * `comp` (uses ghost layer 1); AF_TAG_MAXMIN: max - min of interior
 * averages.  tag = +1 if value >= theta_r and level < lmax; -1 if value <
 * theta_c and level > 0; else 0.  tags: device int8 [nleaves]; values:
 * device double [nleaves] or NULL.
 * --------------------------------------------------------------------- */
af_status af_regrid_tag(af_ctx* ctx, const af_hier* h, const af_state* bufs,
                        uint32_t level_buf_mask, int32_t mode, int32_t comp, double theta_r,
                        double theta_c, int8_t* tags, double* values, hipStream_t stream);

/* af_hier_regrid -- host only: the leaf set after applying tags (host int8
 * [nleaves]): (a) refine leaves tagged +1 below lmax; (b) refine any leaf
 * touching (edge or corner, periodic) a leaf two or more levels finer,
 * until none does; (c) a family of four sibling leaves all tagged -1
 * coarsens if its parent would touch no leaf finer than the siblings (all
 * families judged on the set after (b)); sorted by (level, iy, ix). */
af_status af_hier_regrid(af_ctx* ctx, const af_hier* old, const int8_t* tags, af_hier** out);

/* af_regrid_apply -- device DOF transfer from `old` to `new_h` (Sec. 3.1):
 * unchanged leaves copy their interior and closed-square nodes; refined
 * leaves interpolate from the parent (reconstruction at fine nodes, Simpson
 * for fine averages); coarsened leaves average four children and copy fine
 * vertices.  Writes every leaf of new_h into `dst` (ghosts are not filled:
 * call af_ghost_fill(tmin=0, smin=0) after), and resolves new_h's ghost-fill
 * plans, so that its first coarse step does not.  Synchronises the stream. */
af_status af_regrid_apply(af_ctx* ctx, const af_hier* old, const af_state* old_bufs,
                          uint32_t old_mask, const af_hier* new_h, af_state* dst,
                          hipStream_t stream);

/* af_reduce_sum -- FP64 sum over leaves of interior averages times cell
 * area, per component (global conservation, Sec. 3.2).  out: device double
 * [ncomp]. */
af_status af_reduce_sum(af_ctx* ctx, const af_hier* h, const af_state* bufs,
                        uint32_t level_buf_mask, double* out, hipStream_t stream);

/* af_reduce_sum_noalloc -- af_reduce_sum for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Same result, bit for bit, from the same kernels; the
 * per-leaf partial sums live in a statically allocated device array of
 * 196608 doubles (1.5 MiB, nleaves * ncomp <= 196608, else AF_ERR_ARG), one
 * per GPU, held until the process ends.  Calls no hipMalloc, hipFree or
 * allocating library routine.  The hierarchy's device tables must already
 * exist (any earlier launching call with it, or af_hier_leaf_xy, uploads
 * them), else AF_ERR_STATE.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (concurrent streams or threads) race; calls
 * ordered on one stream do not (every partial sum is written before it is
 * read, so nothing needs clearing between calls). */
af_status af_reduce_sum_noalloc(af_ctx* ctx, const af_hier* h, const af_state* bufs,
                                uint32_t level_buf_mask, double* out, hipStream_t stream);

/* ---------------------------------------------------------------------
 * af_level_advance -- nsteps AF steps (Sec. 2) of all leaves of `level`, for
 * a level whose every leaf has same-level leaves as its eight neighbours
 * (e.g. a uniform level; else AF_ERR_STATE).  Each launch takes K steps
 * (temporal blocking): a block gathers its patch and a K-cell halo straight
 * from the neighbours' interiors (the values a same-level ghost fill would
 * copy), advances K steps in LDS and writes the interior averages and the
 * closed-square nodes to the other buffer.  Equal to nsteps x (af_ghost_fill
 * + af_patch_step) up to rounding order: for advection with the upwind source
 * pattern (a, b > 0, both directional Courant numbers below 1/2) each step is
 * one pass in which a cell's new average is a fixed combination of the 25 old
 * DOFs of its source cells, composed on the host from eq. 2dfv and eq.
 * Simpson-2d.  AF_ADVECTION and AF_ACOUSTICS only (AF_ERR_ARG for the other
 * equations, which step with af_patch_step).  The level's data moves between
 * bufs[0] and bufs[1] (*level_buf_mask bit `level` updated after every
 * launch); ghost layers of the result are NOT filled.
 * --------------------------------------------------------------------- */
af_status af_level_advance(af_ctx* ctx, af_hier* h, af_state* bufs, uint32_t* level_buf_mask,
                           int32_t level, double dt, int32_t nsteps, hipStream_t stream);
/* level-advance kernel shapes (steps per launch K, block size) available for
 * the context's problem; af_ctx_set_advance_shape picks one (autotuner).  For
 * advection the list includes shapes that only the upwind one-pass kernel
 * runs (both Courant numbers positive and below 1/2, so that every node
 * traces back, as in Sec. 2.1, into the upwind neighbour cell).  With other
 * weights af_level_advance replaces such a shape by the default one. */
int32_t af_ctx_advance_shapes(const af_ctx* ctx, int32_t* ks, int32_t* nts, int32_t cap);
/* the shapes of that list that only the upwind one-pass kernel runs (the
 * ones af_level_advance replaces by the default shape for other weights);
 * same conventions: returns their count (-1 for a null ctx), writes at most
 * cap of them to the optional arrays */
int32_t af_ctx_advance_shapes_upwind(const af_ctx* ctx, int32_t* ks, int32_t* nts, int32_t cap);
af_status af_ctx_set_advance_shape(af_ctx* ctx, int32_t k, int32_t nt);
/* the shape af_level_advance will use (the tuned one, else the default: the
 * largest K, then the smallest block), for advection with both velocity
 * components positive assuming time steps small enough for the upwind
 * pattern */
af_status af_ctx_get_advance_shape(const af_ctx* ctx, int32_t* k, int32_t* nt);

/* af_autotune -- picks, by timing `reps` launches of each candidate with HIP
 * events on `stream`, the fastest patch-step tile height and (if the level's
 * leaves all have same-level neighbours) the fastest level-advance shape for
 * this context; best times per step (microseconds) are returned through the
 * optional pointers (-1 if the level advance does not apply).  It steps the
 * data in bufs (use scratch data).  Synchronises the stream. */
af_status af_autotune(af_ctx* ctx, af_hier* h, af_state* bufs, int32_t level, double dt, int32_t reps,
                      double* best_step_us, double* best_advance_us, hipStream_t stream);

/* ---------------------------------------------------------------------
 * af_amr_coarse_step -- one coarse time step dt0 of the whole hierarchy
 * from time t0 with subcycling (Sec. 3.2): full fill; then advance(0): step
 * level l with dt0/2^l (layer-1 region for the first of each pair of fine
 * substeps), recursively advance level l+1 twice with a same-or-finer fill
 * between, then the conservative fix of level l.  Levels ping-pong between
 * bufs[0] and bufs[1]; *level_buf_mask is updated.  flux_reg: FP64
 * [npatch][4][m][ncomp], zero on entry (left zero on exit).
 * flags: AF_STEP_GRAPH replays a hipGraph captured on first use for this
 * (hierarchy, mask, dt0, and t0 for AF_SWIRL; at most 64 graphs are kept per
 * hierarchy, the stream is drained and the cache emptied when it is full, so
 * AF_SWIRL graphs are reused only at repeated t0); AF_STEP_GLOBAL takes one
 * step of dt0 on every level at once, without subcycling (global time
 * stepping, the corollary of Sec. 4.3; dt0 must satisfy the finest level's
 * CFL): full fill, every level steps its interior, then the conservative
 * fix of every level.
 * A hierarchy that is one complete level steps without the fill: its patch
 * steps read the cells outside a patch from the neighbours' interiors (the
 * values the fill would copy).  Otherwise, for AF_ADVECTION and AF_ACOUSTICS
 * the subcycled step is batched by start time: with F the finest level and
 * tau = 0 .. 2^F - 1 in finest steps, one launch steps every patch of every
 * level that starts a step at tau, reading each ghost DOF from the source
 * the fill of that time resolves it to (same-level copy, mean of four finer
 * averages, coarser reconstruction) without writing the fill to memory; a
 * launch before it makes the conservative fix of the levels that have just
 * completed a pair of substeps and copies finer or same-level vertices onto
 * the closed-square boundary nodes of leaves with a neighbour of another
 * level (the part of the fill a coarser reconstruction reads).  2^F + 2^(F-1)
 * + 1 launches per coarse step, 2^(F-1) + 2^(F-1) + 1 with fused pairs (see
 * af_ctx_set_fused_pairs); results equal the recursion above.  In
 * every case the ghost layers of the result are not filled; call
 * af_ghost_fill before reading them.
 * --------------------------------------------------------------------- */
enum { AF_STEP_GRAPH = 1, AF_STEP_GLOBAL = 2 };
af_status af_amr_coarse_step(af_ctx* ctx, af_hier* h, af_state* bufs, uint32_t* level_buf_mask,
                             double t0, double dt0, double* flux_reg, int32_t flags,
                             hipStream_t stream);

/* ---------------------------------------------------------------------
 * af_amr_coarse_steps -- nsteps > 0 coarse steps of dt0 from t0 (step k
 * from t0 + k dt0), each as af_amr_coarse_step with the same flags
 * (AF_STEP_GLOBAL allowed, AF_STEP_GRAPH not), in one call: the state
 * between two of them is not returned, so on the batched path the last
 * launch of a step (the conservative fix of levels 0..F-1, cell averages
 * only) joins the first launch of the next (vertex copies, nodes only), one
 * launch fewer per step.  The result is bit for bit that of nsteps calls of
 * af_amr_coarse_step.  Arguments and errors as for af_amr_coarse_step, and
 * AF_ERR_ARG for nsteps <= 0 or other flags.
 * --------------------------------------------------------------------- */
af_status af_amr_coarse_steps(af_ctx* ctx, af_hier* h, af_state* bufs, uint32_t* level_buf_mask,
                              double t0, double dt0, int32_t nsteps, double* flux_reg, int32_t flags,
                              hipStream_t stream);

/* device uint8 [nleaves]: bit s set when side s borders another level */
const uint8_t* af_hier_side_mask(const af_hier* h);
/* Device int32 [nleaves][2] of the leaves' (ix, iy), the leaf_xy argument of
 * af_patch_step; owned by the hierarchy, uploaded on first use (NULL on a
 * device error). */
const int32_t* af_hier_leaf_xy(const af_hier* h);

/* =====================================================================
 * Learned regrid tagger (a project addition; not part of the paper's
 * method).  A CNN of three 3x3 convolutions (nin -> 32 -> 32 -> 32, zero
 * padding, ReLU) on 16x16 patch fields, global average pooling and a linear
 * head to 3 classes (coarsen, keep, refine), trained with softmax
 * cross-entropy.  Convolutions run as BF16 implicit GEMMs on the matrix
 * cores with FP32 accumulation; parameters, bias, ReLU, head, loss and the
 * optimizer are FP32.  Parameters are packed W1[32][nin][3][3], b1, W2, b2,
 * W3, b3, Wh[3][32], bh (host float arrays of af_cnn_num_params()).
 * The object owns its parameters, optimizer state and workspace.
 * ===================================================================== */
typedef struct af_cnn af_cnn;
const char* af_cnn_last_error(void);
af_status af_cnn_create(int32_t nin, af_cnn** out);
af_status af_cnn_destroy(af_cnn* cnn);
int32_t af_cnn_num_params(const af_cnn* cnn);
af_status af_cnn_set_params(af_cnn* cnn, const float* host_params); /* also resets the optimizer */
af_status af_cnn_get_params(const af_cnn* cnn, float* host_params);
/* per-channel standardisation of the features, host arrays [nin] */
af_status af_cnn_set_normalization(af_cnn* cnn, const float* mean, const float* inv_std);
/* x: device FP32 [B][nin][16][16]; logits: device FP32 [B][3]; acts: NULL or
 * device FP32 [3][B*256][32] receiving the three layers' pre-activations
 * (pixel-major, channel-minor). */
af_status af_cnn_forward(af_cnn* cnn, const float* x, int32_t B, float* logits, float* acts,
                         hipStream_t stream);
/* mean cross-entropy over the batch (device float [1]) and its gradient
 * (device float [num_params], or NULL for the internal buffer used by
 * af_cnn_adam_step).  labels: device int32 [B], 0 coarsen, 1 keep, 2 refine.
 * dacts: NULL or device FP32 [3][B*256][32] receiving, for each layer, the
 * gradient of the loss with respect to its post-ReLU output (pixel-major,
 * channel-minor), the upstream gradient its backward pass consumes.  Every
 * reduction (weight gradients over pixels, bias gradients, batch sums of the
 * head) adds its terms in a fixed order, so the result is deterministic. */
af_status af_cnn_loss_grad(af_cnn* cnn, const float* x, const int32_t* labels, int32_t B, float* loss,
                           float* grad, float* dacts, hipStream_t stream);
/* Adam (beta1 0.9, beta2 0.999, eps 1e-8) step t >= 1 with learning rate lr;
 * grad NULL = the internal gradient of the last af_cnn_loss_grad. */
af_status af_cnn_adam_step(af_cnn* cnn, const float* grad, float lr, int32_t t, hipStream_t stream);
/* features of every leaf (m = 16 only): 12 channels (p,u,v) x (avg, corner,
 * xedge, yedge) of the cells' owned DOFs, then the leaf level, standardised;
 * x: device FP32 [nleaves][nin][16][16]. */
af_status af_cnn_features(af_ctx* ctx, af_cnn* cnn, const af_hier* h, const af_state* bufs,
                          uint32_t level_buf_mask, float* x, hipStream_t stream);
/* learned tags with the plain criterion as fallback: refine if the network
 * or the plain tag (device int8 [nleaves], from af_regrid_tag) says refine,
 * coarsen only if both say coarsen, the plain tag if the network output is
 * not finite; level limits as af_regrid_tag.  tags: device int8 [nleaves];
 * learned: NULL or device int8 [nleaves] receiving the network's own tag
 * (2 where it fell back). */
af_status af_cnn_tag(af_ctx* ctx, af_cnn* cnn, const af_hier* h, const af_state* bufs,
                     uint32_t level_buf_mask, const int8_t* plain, int8_t* tags, int8_t* learned,
                     hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* AF_H */
