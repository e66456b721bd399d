/*
 * mgrav -- gravity interaction lists on one AMD MI355X (gfx950).
 *
 * C ABI of the data-parallel core of the PKDGRAV3 gravity solver
 * (Potter, Stadel & Teyssier, arXiv:1609.08621): evaluation of per-bucket
 * interaction lists -- softened particle-particle (PP) and particle-cell
 * (PC) multipole interactions with moments to 4th order -- plus the Ewald
 * correction of the periodic box, for the particles of the active sink
 * buckets.  The paper describes the problem and method in Sec. 3.1 (tree,
 * opening radius, interaction lists, multipole order, precision, Ewald),
 * Sec. 3.2 (active particles of individual time steps) and Sec. 3.3 (the
 * split of work between tree walk and interaction evaluation).
 *
 * Conventions used by every call:
 *   - Units: G = 1.  Potential of a softened point mass m at distance r is
 *     -m / sqrt(r^2 + eps^2) (Plummer softening).
 *   - Particles are in tree order: every cell owns the contiguous range
 *     [cell_first[c], cell_first[c] + cell_count[c]).
 *   - Periodic images: id 0 is the box itself, ids 1..26 the replicas
 *     shifted by (ix, iy, iz) * L with (ix, iy, iz) in {-1,0,1}^3 \ {0},
 *     enumerated in lexicographic order (ix slowest).
 *   - Packed moments of a cell (32 doubles, about the cell's centre of
 *     mass, raw i.e. not trace-free): [0] mass; [1..6] order 2
 *     (xx xy xz yy yz zz); [7..16] order 3 (xxx xxy xxz xyy xyz xzz yyy
 *     yyz yzz zzz); [17..31] order 4 (xxxx xxxy xxxz xxyy xxyz xxzz xyyy
 *     xyyz xyzz xzzz yyyy yyyz yyzz yzzz zzzz), each component being
 *     sum_j m_j prod_a (x_j - X)_a.  The dipole vanishes about the centre
 *     of mass and is not stored.
 *   - Every call returns an mgrav_status; nothing else crosses the ABI (no
 *     exceptions, no abort).  After a failure mgrav_last_error() holds a
 *     message until the next call on the same context.
 *   - "device" pointers are HIP device (HBM) addresses on the context's
 *     GPU, "host" pointers are ordinary CPU memory.  Memory passed in is
 *     borrowed: the library never frees it, and never allocates device
 *     memory itself (the caller provides a workspace, or binds to the
 *     library's static one with mgrav_bind_static).
 */
#ifndef MGRAV_H
#define MGRAV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MGRAV_VERSION_MAJOR 0
#define MGRAV_VERSION_MINOR 3

/* Largest bucket (leaf) the device kernels accept; the paper's optimum
 * bucket size is about 16 (Sec. 3.1). */
#define MGRAV_MAX_BUCKET 16
/* Largest particle count: PP list entries pack a particle index in 27 bits. */
#define MGRAV_MAX_PARTICLES (1LL << 27)

typedef enum {
    MGRAV_OK = 0,
    MGRAV_ERR_INVALID_ARG = 1, /* bad scalar argument or null pointer      */
    MGRAV_ERR_BAD_TREE = 2,    /* tree inconsistent (found on the device)  */
    MGRAV_ERR_BAD_LIST = 3,    /* list entry out of range / not a leaf     */
    MGRAV_ERR_DEVICE = 4,      /* a HIP runtime call failed                */
    MGRAV_ERR_NO_MEMORY = 5,   /* workspace smaller than required          */
    MGRAV_ERR_TIMEOUT = 6,     /* mgrav_wait deadline passed               */
    MGRAV_ERR_STATE = 7,       /* call out of order (e.g. compute before bind) */
    MGRAV_ERR_NOT_TRAINED = 8  /* surrogate Ewald requested without weights */
} mgrav_status;

typedef struct mgrav_ctx mgrav_ctx;

/* Version as major * 1000 + minor. */
int mgrav_version(void);

/* Static text for a status code. */
const char *mgrav_status_string(mgrav_status s);

/* Message of the last failed call on ctx ("" if none).  Valid until the
 * next call on ctx.  ctx may be NULL (then the message of the last failed
 * mgrav_create or host-side call of this thread). */
const char *mgrav_last_error(const mgrav_ctx *ctx);

/* Create a context on HIP device `device`; all work is enqueued on
 * `hip_stream` (a hipStream_t, NULL = the default stream).  A context is
 * not thread-safe; use one per stream. */
mgrav_status mgrav_create(int device, void *hip_stream, mgrav_ctx **out);

/* Release the context (host resources only; waits for its stream). */
void mgrav_destroy(mgrav_ctx *ctx);

/* ------------------------------------------------------------------ */
/* Host-side input preparation: tree build and checklist walk.         */
/* These run on the CPU (OpenMP), on host pointers, and produce the    */
/* tree and interaction lists that the device calls consume.           */
/* ------------------------------------------------------------------ */

/* Binary tree of Sec. 3.1: cells bisect the longest side of their
 * geometric box at its midpoint (two equal-volume children; lowest axis
 * index on ties; coordinates >= midpoint go to the upper child; an empty
 * half shrinks the box and bisection repeats; after 64 halvings on a path
 * cells split by index halves).  The root is [0, L)^3 when L > 0 and the
 * particles' bounding box when L == 0.  Leaves (buckets) hold at most
 * `bucket` particles.  Cells are numbered node-left-right; within a cell
 * particles keep their input order.  Per cell: centre of mass, tight
 * bounding box, b_max = largest distance of a particle from the centre of
 * mass, packed moments.
 *   pos  [n][3], mass [n]: input order (host).
 *   Outputs (host, caller-allocated with room for `cap` cells; 2n cells
 *   always suffice): perm[n] (input index of the k-th particle in tree
 *   order), cell_first[cap], cell_count[cap], child[cap][2] (-1 = leaf),
 *   com[cap][3], bmax[cap], bbox[cap][6] (lo xyz, hi xyz), mom[cap][32],
 *   bucket_cell[cap] (cell of the b-th leaf in order).
 *   *n_cell and *n_bucket receive the counts.
 * Errors: INVALID_ARG for n < 1, bucket outside 1..MGRAV_MAX_BUCKET,
 * non-finite input, L > 0 with a coordinate outside [0, L), non-positive
 * mass, or cap too small. */
mgrav_status mgrav_tree_build_host(int64_t n, const double *pos, const double *mass, double L,
                                   int bucket, int64_t cap, int64_t *perm, int64_t *cell_first,
                                   int32_t *cell_count, int32_t *child, double *com,
                                   double *bmax, double *bbox, double *mom,
                                   int32_t *bucket_cell, int64_t *n_cell, int64_t *n_bucket);

/* Bucket-sink checklist walk (Sec. 3.1).  For every bucket S the
 * checklist starts with the root cell seen through images 0..n_images-1;
 * entries are taken from the front and a source cell C seen through
 * image n becomes
 *   PC  if |X_C + n L - X_S| > b_max,C / theta + b_max,S and the
 *       bounding boxes (C shifted by n L) are at least 2 eps apart,
 *   PP  otherwise if C is a leaf,
 *   and is otherwise opened: its two children are appended to the end.
 * Pass 1 (mgrav_lists_count_host) writes CSR offsets pp_off[n_bucket+1]
 * and pc_off[n_bucket+1]; pass 2 (mgrav_lists_fill_host) fills
 * pp_src/pc_src (source cell index) and pp_img/pc_img (image id) in
 * checklist order.  All arrays are host memory; tree arrays as produced
 * by mgrav_tree_build_host.  n_images is 1 (open, L = 0) or 27.
 * Errors: INVALID_ARG for theta <= 0, eps < 0, n_images not 1 or 27, or
 * n_images 27 with L <= 0. */
mgrav_status mgrav_lists_count_host(int64_t n_bucket, const int32_t *bucket_cell,
                                    const int32_t *child, const double *com, const double *bmax,
                                    const double *bbox, double theta, double eps, double L,
                                    int n_images, int64_t *pp_off, int64_t *pc_off);
mgrav_status mgrav_lists_fill_host(int64_t n_bucket, const int32_t *bucket_cell,
                                   const int32_t *child, const double *com, const double *bmax,
                                   const double *bbox, double theta, double eps, double L,
                                   int n_images, const int64_t *pp_off, const int64_t *pc_off,
                                   int32_t *pp_src, uint8_t *pp_img, int32_t *pc_src,
                                   uint8_t *pc_img);

/* ------------------------------------------------------------------ */
/* Device-side input preparation: the same tree and checklist walk on  */
/* the GPU (device pointers), and the two trees of Sec. 3.2.           */
/* ------------------------------------------------------------------ */

/* Outputs of mgrav_tree_build, device memory owned by the caller, with
 * room for `cap` cells: the arrays of mgrav_tree_build_host (perm as
 * int64), plus the particles in tree order (pos [n][3], mass [n]), which
 * mgrav_bind takes as they are. */
typedef struct {
    int64_t *perm;
    double *pos;
    double *mass;
    int64_t *cell_first;
    int32_t *cell_count;
    int32_t *child;
    double *com;
    double *bmax;
    double *bbox;
    double *mom;
    int32_t *bucket_cell;
} mgrav_tree_dev;

/* Device workspace of mgrav_tree_build for n particles, leaves of at most
 * `bucket` and room for `cap` cells (about 100 bytes per particle plus
 * 80 per cell).  INVALID_ARG for n outside 1 .. MGRAV_MAX_PARTICLES,
 * bucket outside 1 .. MGRAV_MAX_BUCKET, cap outside 1 .. 2n + 2. */
mgrav_status mgrav_tree_workspace_size(int64_t n, int bucket, int64_t cap, size_t *bytes);

/* The tree of mgrav_tree_build_host, built on the device from pos [n][3]
 * and mass [n] (device, input order): the same cells in the same
 * node-left-right order, particles in the same tree order, identical
 * bounding boxes, and for buckets identical centres of mass, b_max and
 * moments.  A parent's mass, first moments and box come from its
 * children (its centre of mass may differ from the host builder's
 * particle-order sum in the last bits), its order-2..4 moments are its
 * children's shifted to its centre of mass (the parallel-axis expansion,
 * exact up to rounding), and its b_max is taken over its particles.
 * With `group` (device [n] uint8, nullable) particles with group 0 and
 * group != 0 get a tree each -- the fixed and the very active tree of
 * Sec. 3.2 -- over the same root box (that of all particles), so that
 * both bisect space along the same planes; they are stored as one
 * forest: the first tree's particles (in tree order), then the second's;
 * the first tree's cells (root 0), then the second's (root
 * *n_cell_first), buckets likewise.  Both groups must be non-empty.
 * Blocking (the host reads one count per level).  *n_cell_first (nullable)
 * receives the first tree's cell count (= n_cell for one tree).  Errors:
 * INVALID_ARG for bad sizes, non-finite input, non-positive mass, a
 * periodic coordinate outside [0, L), an empty group, or "capacity" in
 * the message when the tree needs more than cap cells (build again with
 * a larger cap); NO_MEMORY for a workspace below
 * mgrav_tree_workspace_size. */
mgrav_status mgrav_tree_build(mgrav_ctx *ctx, int64_t n, const double *pos, const double *mass,
                              const uint8_t *group, double L, int bucket, void *workspace,
                              size_t bytes, int64_t cap, const mgrav_tree_dev *out,
                              int64_t *n_cell, int64_t *n_bucket, int64_t *n_cell_first);

/* Sec. 3.2 keeps the fixed tree and rebuilds only the very active one.
 * mgrav_tree_offset turns a tree that mgrav_tree_build built alone, from
 * the particles ids[0 .. n_particles-1] of a forest's input (device int64,
 * in input order), into one tree of that forest, in place: cell_first +=
 * particle_offset, child (where >= 0) and bucket_cell += cell_offset,
 * perm[i] = ids[perm[i]] (ids NULL: the subset is the input range from
 * particle_offset, perm[i] += particle_offset).  The arrays of `t` are device memory, sized
 * n_cell (cell_first, child), n_bucket (bucket_cell) and n_particles
 * (perm).  Built this way into consecutive ranges of one set of arrays
 * (the group-0 particles with offsets 0, then the others with offsets
 * the first tree's cell and particle counts), two trees equal, array for
 * array, the forest one mgrav_tree_build call with the group array
 * writes, when the box is periodic (an open forest takes the root box of
 * all particles, a tree built alone that of its own).  Blocking.
 * INVALID_ARG for null pointers, sizes out of range, fewer ids than
 * particles or a perm entry outside [0, n_ids). */
mgrav_status mgrav_tree_offset(mgrav_ctx *ctx, const mgrav_tree_dev *t, int64_t n_cell,
                               int64_t n_bucket, int64_t n_particles, int64_t cell_offset,
                               int64_t particle_offset, const int64_t *ids, int64_t n_ids);

/* The checklist walk of mgrav_lists_count_host / _fill_host on the
 * device, for the sink buckets sink_cell[n_sink] (cells, device memory;
 * for one tree its bucket_cell, for a forest the second tree's buckets),
 * the checklist seeded with every root (roots[0 .. n_roots-1], host
 * values, in that order) seen through images 0 .. n_images-1.  Tree
 * arrays (child, com, bmax, bbox; device) as mgrav_tree_build writes
 * them. */
typedef struct {
    int64_t n_cell;
    const int32_t *child;
    const double *com;
    const double *bmax;
    const double *bbox;
    int n_roots;          /* 1 or 2 */
    int32_t roots[2];
    double theta, eps, L; /* theta > 0, eps >= 0, L = 0 (open) or the box */
    int n_images;         /* 1 or 27 (L > 0) */
    int64_t n_sink;
    const int32_t *sink_cell;
} mgrav_walk;

/* Device workspace of the walk (96 bytes per cell, 24 per sink, and the
 * overflow pass's rings: 64 x 8 x (2^14 .. 2^20) bytes). */
mgrav_status mgrav_lists_workspace_size(int64_t n_cell, int64_t n_sink, size_t *bytes);

/* Pass 1: pp_off[n_sink + 1] and pc_off[n_sink + 1] (device) receive the
 * CSR offsets of the lists; *n_pp and *n_pc (host, nullable) their
 * totals.  Pass 2 fills pp_src, pp_img, pc_src, pc_img (device) in
 * checklist order, with the offsets of pass 1 and the same workspace
 * contents or a new one.  Each sink's checklist runs in an LDS ring of
 * 1024 entries; sinks whose checklist outgrows it (sparse buckets of a
 * very active tree among dense fixed cells) are walked again by a second
 * pass with a ring of up to 2^20 entries in the workspace (NO_MEMORY if
 * one outgrows that too).  BAD_TREE for a cell index outside the tree,
 * INVALID_ARG for bad scalars.  Blocking. */
mgrav_status mgrav_lists_count(mgrav_ctx *ctx, const mgrav_walk *walk, void *workspace,
                               size_t bytes, int64_t *pp_off, int64_t *pc_off, int64_t *n_pp,
                               int64_t *n_pc);
mgrav_status mgrav_lists_fill(mgrav_ctx *ctx, const mgrav_walk *walk, void *workspace,
                              size_t bytes, const int64_t *pp_off, const int64_t *pc_off,
                              int32_t *pp_src, uint8_t *pp_img, int32_t *pc_src,
                              uint8_t *pc_img);

/* ------------------------------------------------------------------ */
/* The persistent particle store of Sec. 3.4 and the steps of the      */
/* hierarchical kick-drift-kick integrator of Sec. 3.2 (device).       */
/* ------------------------------------------------------------------ */

/* 28 bytes per particle: a position as three unsigned 32-bit integers,
 * x = origin + q * scale per axis (periodic box: origin 0 and scale
 * L / 2^32, so the integers wrap as the box does; open: a grid slightly
 * larger than the particles' extent), the velocity as three floats, and
 * one word with the rung (bits 0..7) and a group id (bits 8..31).  The
 * arrays are device memory owned by the caller. */
typedef struct {
    uint32_t *q;      /* [n][3] */
    float *vel;       /* [n][3] */
    uint32_t *aux;    /* [n]    */
    double origin[3];
    double scale;     /* length of one integer step (> 0) */
} mgrav_store;

/* q = nearest grid point (ties to even) of pos [n][3] (device, double),
 * modulo 2^32 when `periodic`, else INVALID_ARG if a point lies off the
 * grid; vel [n][3] (device, nullable: zero) copied; aux cleared.  All the
 * store calls are blocking and return INVALID_ARG for null pointers, n
 * outside 1 .. 2^27, a non-finite origin or scale <= 0. */
mgrav_status mgrav_store_encode(mgrav_ctx *ctx, int64_t n, const double *pos, const float *vel,
                                int periodic, const mgrav_store *st);
/* pos = origin + q * scale (device [n][3], double, one fused multiply-add
 * per coordinate, as the evaluation reads pos_q; exact when the values fit
 * 53 bits), vel copied when non-NULL. */
mgrav_status mgrav_store_decode(mgrav_ctx *ctx, int64_t n, const mgrav_store *st, double *pos,
                                float *vel);
/* out[k] = in[perm[k]] for every array of the store (the tree order of
 * mgrav_tree_build's perm); separate output arrays. */
mgrav_status mgrav_store_permute(mgrav_ctx *ctx, int64_t n, const mgrav_store *in,
                                 const int64_t *perm, const mgrav_store *out);
/* Drift every particle by dt: q += nearest integer of v dt / scale (exact
 * integer arithmetic, wrapping when periodic; INVALID_ARG if an open-box
 * coordinate leaves the grid). */
mgrav_status mgrav_store_drift(mgrav_ctx *ctx, int64_t n, const mgrav_store *st, double dt,
                               int periodic);
/* The same drift for the particles on rungs rung_lo <= rung < rung_hi
 * only (Sec. 3.2: the fixed particles drift to the middle of the fixed
 * rung's step and from there to its end, the very active ones substep by
 * substep).  INVALID_ARG also for a range outside 0 .. 256. */
mgrav_status mgrav_store_drift_rungs(mgrav_ctx *ctx, int64_t n, const mgrav_store *st, double dt,
                                     int periodic, int rung_lo, int rung_hi);
/* Half kick of the particles on rungs >= rung_lo: v += a dt_base / 2^(rung+1),
 * acc [3][n] float SoA (device, as mgrav_compute writes it), in double and
 * rounded to float once. */
mgrav_status mgrav_store_kick(mgrav_ctx *ctx, int64_t n, const mgrav_store *st, const float *acc,
                              double dt_base, int rung_lo);
/* New rungs of the particles on rungs >= rung_lo (those at the end of
 * their step): the time-step criterion of Sec. 3.2, dt_i = eta
 * sqrt(eps / |a_i|) (eta = 0.2 in the paper), gives the smallest rung l
 * with dt_base / 2^l <= dt_i, clamped to [rung_floor, rung_max]
 * (rung_floor: the shallowest rung whose step boundary is now). */
mgrav_status mgrav_store_rungs(mgrav_ctx *ctx, int64_t n, const mgrav_store *st, const float *acc,
                               double eps, double eta, double dt_base, int rung_lo,
                               int rung_floor, int rung_max);
/* active[i] = 1 if rung >= rung_lo else 0 (device uint8 [n]; the mask of
 * mgrav_set_active). */
mgrav_status mgrav_store_active(mgrav_ctx *ctx, int64_t n, const mgrav_store *st, int rung_lo,
                                uint8_t *active);

/* ------------------------------------------------------------------ */
/* Fast multipole form (Sec. 3.1): cell-cell (CC) and cell-particle    */
/* (CP) interactions into local expansions of each sink cell.          */
/* ------------------------------------------------------------------ */

/* The walk over sink cells, in node-left-right order from the root
 * (checklist: the root through every image), each with the checklist its
 * parent kept.  A source -- a cell, or a particle of an opened leaf
 * (opening radius 0, a point box) -- seen through image n is, for sink S:
 *   CC (cell) / CP (particle) if |X_C + nL - X_S| > 1.5 RO_S + RO_C and
 *     the boxes are at least 2 eps apart (RO = b_max / theta; the factor
 *     1.5 on the sink is the paper's);
 *   at a bucket S: PP of the particle for a particle source; PC if
 *     |X_C + nL - X_S| > RO_C + b_max,S with the boxes 2 eps apart (the
 *     bucket walk's rule); PP of the whole leaf if C is a leaf; else
 *     opened (children appended to the checklist);
 *   at a larger S: a particle, or a cell smaller than S (b_max,C <
 *     b_max,S), stays on the checklist of S's children; a cell at least as
 *     large is opened (a leaf into its particles, in tree order).
 * Outputs (host, like mgrav_lists_*_host): per bucket pp_off / pc_off
 * [n_bucket + 1] and entries pp_src, pp_img, pp_sub (0: the whole leaf,
 * k + 1: its k-th particle), pc_src, pc_img; per cell cc_off [n_cell + 1]
 * and entries cc_src (source cell, or ~p for tree-order particle p),
 * cc_img.  pos: tree-order positions [n][3] (host). */
mgrav_status mgrav_fmm_lists_count_host(int64_t n_cell, const int64_t *cell_first,
                                        const int32_t *cell_count, const int32_t *child,
                                        const double *com, const double *bmax,
                                        const double *bbox, const double *pos, double theta,
                                        double eps, double L, int n_images, int64_t *pp_off,
                                        int64_t *pc_off, int64_t *cc_off);
mgrav_status mgrav_fmm_lists_fill_host(int64_t n_cell, const int64_t *cell_first,
                                       const int32_t *cell_count, const int32_t *child,
                                       const double *com, const double *bmax, const double *bbox,
                                       const double *pos, double theta, double eps, double L,
                                       int n_images, const int64_t *pp_off, const int64_t *pc_off,
                                       const int64_t *cc_off, int32_t *pp_src, uint8_t *pp_img,
                                       uint8_t *pp_sub, int32_t *pc_src, uint8_t *pc_img,
                                       int32_t *cc_src, uint8_t *cc_img);

/* The CC / CP part of the forces, on the device (all pointers device
 * memory; particles and cells as for mgrav_bind). */
typedef struct {
    int64_t n, n_cell, n_bucket;
    const int32_t *child;
    const double *com;
    const double *mom;
    const int64_t *cell_first;
    const int32_t *cell_count;
    const int32_t *bucket_cell;
    const double *pos;        /* [n][3] tree order */
    const double *mass;       /* [n], or NULL: mass_uniform */
    double mass_uniform;
    double eps, box_L;
    const int64_t *cc_off;    /* [n_cell + 1] */
    const int32_t *cc_src;
    const uint8_t *cc_img;
    const uint8_t *active;    /* [n] or NULL: every particle */
} mgrav_fmm;

/* Device workspace of mgrav_fmm_apply (56 doubles and 4 bytes per cell). */
mgrav_status mgrav_fmm_workspace_size(int64_t n_cell, size_t *bytes);

/* Every cell's own local expansion L_a = d^a phi(X_S), |a| <= 5 (56
 * values, about its centre of mass), from its CC entries,
 *   L_a = sum_{k in {0,2,3,4}, k + |a| <= 5} (-1)^k/k! M_k . d^(k+a) G(R),
 * and CP entries, L_a = m d^a G(R) (R = X_S - source - nL, G = -(R^2 +
 * eps^2)^(-1/2), total order kept to 5); each bucket's expansion is its
 * ancestors' shifted down one level at a time (L'_a = sum_{b >= a} L_b
 * d^(b-a)/(b-a)!) plus its own, and is evaluated at its active particles:
 * acc -= grad phi, pot += phi (phi = sum_a L_a h^a/a!), added in double
 * and rounded once.  Call after mgrav_compute on the same stream (acc, pot
 * as it writes them).  Double precision.  local_out (nullable, device
 * [n_bucket][56]) receives the buckets' expansions.  Blocking.  BAD_LIST
 * for an entry out of range; INVALID_ARG / NO_MEMORY as usual. */
mgrav_status mgrav_fmm_apply(mgrav_ctx *ctx, const mgrav_fmm *f, void *workspace, size_t bytes,
                             float *acc, float *pot, double *local_out);

/* ------------------------------------------------------------------ */
/* Device-side evaluation.                                             */
/* ------------------------------------------------------------------ */

/* The problem: particles in tree order, the tree and the per-bucket
 * interaction lists, all in DEVICE memory (borrowed until the next
 * mgrav_bind or mgrav_destroy).  Scalars are host values. */
typedef struct {
    int64_t n;               /* particles (1 .. MGRAV_MAX_PARTICLES)          */
    const double *pos;       /* [n][3] positions, tree order (or pos_q below) */
    const double *mass;      /* [n] masses (> 0), or NULL (mass_uniform)      */
    double eps;              /* Plummer softening (> 0)                       */
    double theta;            /* opening angle the lists were built with (> 0) */
    double box_L;            /* periodic box side; 0 = open boundaries         */
    int n_images;            /* 1 (open) or 27 (periodic: box + 26 replicas)  */
    int64_t n_cell;          /* cells of the tree                             */
    int64_t n_bucket;        /* leaves (buckets)                              */
    const int64_t *cell_first; /* [n_cell]                                    */
    const int32_t *cell_count; /* [n_cell]                                    */
    const int32_t *child;      /* [n_cell][2], -1 for leaves                  */
    const double *com;         /* [n_cell][3] centres of mass                 */
    const double *bbox;        /* [n_cell][6] bounding boxes (lo xyz, hi xyz) */
    const double *mom;         /* [n_cell][32] packed moments (see above)     */
    const int32_t *bucket_cell;/* [n_bucket] cell of each bucket              */
    const int64_t *pp_off;     /* [n_bucket+1] CSR offsets of the PP lists    */
    const int32_t *pp_src;     /* [n_pp] source leaf cell                     */
    const uint8_t *pp_img;     /* [n_pp] image id                             */
    const int64_t *pc_off;     /* [n_bucket+1] CSR offsets of the PC lists    */
    const int32_t *pc_src;     /* [n_pc] source cell                          */
    const uint8_t *pc_img;     /* [n_pc] image id                             */
    int64_t n_pp;              /* = pp_off[n_bucket] (host copy)              */
    int64_t n_pc;              /* = pc_off[n_bucket] (host copy)              */
    /* Positions from the integer coordinates of a particle store (Sec. 3.4)
     * instead of `pos` (exactly one of the two is non-NULL):
     * x = q_origin + pos_q * q_scale per axis, [n][3] in tree order. */
    const uint32_t *pos_q;
    double q_origin[3];
    double q_scale;
    /* With mass == NULL every particle has this mass (> 0). */
    double mass_uniform;
    /* PP entries naming one particle of their source leaf (nullable: whole
     * leaves): pp_sub[e] = 0 for the whole leaf pp_src[e], k + 1 for its
     * k-th particle in tree order (the walk of mgrav_fmm_lists_*_host). */
    const uint8_t *pp_sub;
} mgrav_problem;

/* Device workspace the caller must provide to mgrav_bind for `p`:
 * 16 bytes per particle (staged offsets and masses) + 4 (active list)
 * + 32 (Ewald correction buffered beside the PP + PC kernel),
 * 176 + 32 + 2 bytes per cell (PC records, cell centres and ranges, two
 * flags of the masked staging), 16 per PP entry, 53 per bucket (work
 * descriptor, queue, cost bin) and about 1.6 MB of fixed tables, each
 * segment aligned to 256 bytes. */
mgrav_status mgrav_workspace_size(const mgrav_problem *p, size_t *bytes);

/* Bind a problem: checks the scalar arguments on the host and arranges
 * for the staging kernels to run first in the next mgrav_compute (a
 * mgrav_wait that comes first runs them itself).  The staging kernels
 *   (1) store every particle as float offsets from its bucket's centre
 *       (the centre itself stays in double precision) and its mass,
 *   (2) convert each cell's moments into the float coefficients of the
 *       order-4 PC expansion,
 *   (3) turn every PP entry into a float offset between the source
 *       bucket's centre plus the image shift and the sink bucket's centre,
 *       computed in double.
 * PC entries are read as given by the PP + PC kernel, which forms the
 * offset of the cell's centre of mass (plus image shift) from the sink
 * bucket's centre in double.
 * Indices in the tree and lists are checked on the device; a bad entry is
 * neutralised (never dereferenced) and reported by the next mgrav_wait as
 * BAD_TREE or BAD_LIST.  `workspace` is a device buffer of at least
 * mgrav_workspace_size() bytes, 256-byte aligned, owned by the caller and
 * borrowed until the next bind or destroy.  The device reads the positions
 * and lists when the staging runs, so binding once per step with moved
 * positions (same buffers) re-stages them.  When the compute that stages
 * has a mask (mgrav_set_active), only what its active buckets read is
 * staged (their particles, PP entries and work, the particles of their PP
 * source leaves, the records of their PC source cells; every bucket's work
 * descriptor) and the staging stays pending: the next compute stages again
 * for its own mask, or everything without one.  Results do not depend on
 * which staging ran.  Re-binding is allowed at any time after the previous
 * work on the stream. */
mgrav_status mgrav_bind(mgrav_ctx *ctx, const mgrav_problem *p, void *workspace, size_t bytes);

/* Size of the library's static workspace (64 MiB; one copy per GPU). */
#define MGRAV_STATIC_WORKSPACE_BYTES (64LL << 20)

/* For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * mgrav_bind, with the library's own static workspace in place of a
 * caller buffer -- MGRAV_STATIC_WORKSPACE_BYTES of device memory per GPU,
 * reserved when the library is loaded and held until the process ends.
 * The call allocates nothing (no hipMalloc, no hipFree); with
 * MGRAV_LAUNCH_DIRECT the computes that follow only enqueue kernels (the
 * graph launch mode builds a HIP graph at its first compute).  Problems
 * whose mgrav_workspace_size exceeds the static size fail NO_MEMORY with
 * the two sizes in mgrav_last_error (about 5 * 10^5 particles of the
 * configurations here fit).  Every context bound this way on one GPU
 * shares that GPU's workspace and finds the contents the last compute on
 * it left: re-bind before computing if another context has computed there
 * since, and never let computes of two such contexts overlap in time (they
 * would overwrite each other's staged data).  Other errors as mgrav_bind. */
mgrav_status mgrav_bind_static(mgrav_ctx *ctx, const mgrav_problem *p);

/* Ewald correction of the periodic box (Sec. 3.1): a multipole expansion
 * of the root cell's field in the Ewald kernel psi, evaluated in double
 * precision at every active particle.  psi is the periodic potential of a
 * unit mass (neutralising background, zero mean) minus the 27 nearest
 * images' Newtonian potentials:
 *   psi(r) = sum_{|n|_inf<=1} erf(a|r-nL|)/|r-nL|
 *          - sum_{1<|n|_inf<=real_layers} erfc(a|r-nL|)/|r-nL|
 *          - 1/(pi L^3) sum_{0<|h|^2<=h2max} exp(-pi^2 h^2/(a L)^2) ... (with
 *            a = alpha / L and wave vectors 2 pi h / L)
 *          + pi / (alpha^2 L).
 * The correction at particle x from root moments M_k about X is
 *   phi = sum_k (-1)^k / k!  M_k . d^k psi(x - X),  acc = -grad phi,
 * with k in {0} (order 0), {0, 2} (order 2) or {0, 2, 3, 4} (order 4;
 * the paper's "5th order": kernel derivatives through order 5 in the
 * force).  mode NONE switches the correction off (open boundaries need
 * nothing); EXACT uses the sums above.  SURROGATE evaluates the trained
 * network of mgrav_mlp_* instead: the field of the monopoles of the
 * `top_cells` (1 = root, 8 or 64) tree cells at depth log2(top_cells)
 * (a leaf met earlier stands for its branch), psi from the network at
 * every (particle, cell) pair, added in double.  SURROGATE without weights
 * fails NOT_TRAINED; another top_cells value fails INVALID_ARG.
 *
 * SURROGATE_FALLBACK keeps the exact sums as the judge of the network and
 * its fallback, decided on the device at every compute: the exact
 * correction and the surrogate are evaluated at the sample of particles
 * j * sample_stride (j = 0, 1, ...; active ones only), and
 *   err = sqrt( mean |a_surrogate - a_exact|^2 / |a_base + a_exact|^2 )
 * over that sample (the rms relative force error the surrogate adds),
 * a_base being the PP + PC acceleration already in acc (zero when the
 * compute leaves out PP and PC, so err is then relative to the correction
 * itself).  If err <= fallback_tol the surrogate is applied
 * to every active particle, else the exact correction (alpha, real_layers,
 * h2max, order as for EXACT); an empty sample also takes the exact path.
 * mgrav_stats reports err, the sample size and which path ran.  The
 * sample holds at most 16384 particles: sample_stride 0 picks
 * ceil(n / 8192), and a smaller stride than ceil(n / 16384) is raised to
 * it.  Needs weights (NOT_TRAINED) and valid parameters for both modes. */
typedef enum {
    MGRAV_EWALD_NONE = 0,
    MGRAV_EWALD_EXACT = 1,
    MGRAV_EWALD_SURROGATE = 2,
    MGRAV_EWALD_SURROGATE_FALLBACK = 3
} mgrav_ewald_mode;

typedef struct {
    int mode;          /* mgrav_ewald_mode                                 */
    double alpha;      /* Gaussian split in units of 1/L (e.g. 2.6)        */
    int real_layers;   /* |n|_inf <= real_layers in real space (>= 1)      */
    int h2max;         /* k-space terms with 0 < |h|^2 <= h2max (0..64)    */
    int order;         /* 0, 2 or 4 (moments of the root used)             */
    int top_cells;     /* surrogate: 1 = root monopole, 8 or 64 cells      */
    double fallback_tol; /* SURROGATE_FALLBACK: largest accepted err (>= 0) */
    int64_t sample_stride; /* SURROGATE_FALLBACK: 0 = default (see above)  */
} mgrav_ewald;

/* Defaults after every bind: EXACT with alpha 2.6, real_layers 1,
 * h2max 10, order 4 (top_cells 1, fallback_tol 1e-4, sample_stride 0) when
 * box_L > 0; NONE when open.  Call it again after each bind to keep
 * another setting. */
mgrav_status mgrav_set_ewald(mgrav_ctx *ctx, const mgrav_ewald *cfg);

/* Active particles of an individual-time-step substep (Sec. 3.2): only
 * buckets holding at least one active particle are evaluated, and only
 * active particles' outputs are written (inactive entries keep their
 * values).  active: device [n] uint8 (non-zero = active), read at every
 * mgrav_compute (the caller may change its contents between calls), or
 * NULL = all particles active. */
mgrav_status mgrav_set_active(mgrav_ctx *ctx, const uint8_t *active_dev);

/* Parts of the evaluation, for mgrav_compute_parts. */
#define MGRAV_PART_PP 1
#define MGRAV_PART_PC 2
#define MGRAV_PART_EWALD 4
#define MGRAV_PART_ALL 7

/* Evaluate the bound lists: acc[3][n] (SoA: all x, then all y, then all
 * z) and pot[n], float, tree order, device memory.  The PP and PC sums
 * are computed in float with float accumulation; the Ewald correction in
 * double, added to the float sums in double and rounded once.  The self
 * pair (i, image 0) is excluded; a particle's own replicas are included.
 * Asynchronous: returns after enqueueing; use mgrav_wait.  In the graph
 * launch mode (mgrav_set_launch_mode) the first call with a given set of
 * arguments builds a HIP graph of the launch sequence and later calls
 * replay it; in the direct mode the kernels are enqueued one by one. */
mgrav_status mgrav_compute(mgrav_ctx *ctx, float *acc, float *pot);

/* As mgrav_compute, restricted to the parts in `parts` (MGRAV_PART_*). */
mgrav_status mgrav_compute_parts(mgrav_ctx *ctx, int parts, float *acc, float *pot);

/* Counters and timings of the last compute. */
typedef struct {
    int64_t n_pp_interactions;   /* sink particle x source particle x image  */
    int64_t n_pc_interactions;   /* sink particle x source cell x image      */
    int64_t n_active_buckets;
    int64_t n_active_particles;
    double ms_total;             /* stream time of the last compute          */
    double ms_interact;          /* PP + PC kernel of the last compute: its  */
                                 /* span on the device wall clock, from its  */
                                 /* first queue claim to its last wave's exit */
    double ms_ewald;             /* Ewald kernels of the last compute (with  */
                                 /* direct launches and exact Ewald they run */
                                 /* beside the PP + PC kernel)               */
    int graph_replay;            /* 1: launched from captured HIP graphs     */
    int interact_variant;        /* PP + PC kernel variant of the last compute */
    int graph_error;             /* 0, or the HIP error code that made this  */
                                 /* context fall back to direct launches     */
    int ewald_fallback;          /* SURROGATE_FALLBACK: 1 = the exact path   */
                                 /* ran, 0 = the surrogate was accepted      */
    int64_t ewald_samples;       /* SURROGATE_FALLBACK: active sample size   */
    double ewald_sample_err;     /* SURROGATE_FALLBACK: err of the sample    */
    int queue_local;             /* 1: the work queue was laid out for       */
                                 /* locality (mgrav_set_queue_order)         */
    int queue_pad;
} mgrav_stats;

/* Wait for the context's work with a watchdog (mgrav_watchdog_poll on an
 * event recorded after the enqueued work): when `timeout_s` (<= 0: wait
 * forever) passes first it returns TIMEOUT and marks the context failed (it
 * must be re-bound); the event is released on every path.  Reports
 * device-side validation failures from the last bind (BAD_TREE / BAD_LIST).
 * stats may be NULL. */
mgrav_status mgrav_wait(mgrav_ctx *ctx, double timeout_s, mgrav_stats *stats);

/* The watchdog policy of mgrav_wait, on any completion query: calls
 * query(user) until it returns 0 (done) or a negative value (failed), spinning
 * for the first 2 ms and then sleeping 50 us (to 50 ms) or 500 us between
 * calls; returns OK, DEVICE for a failed query, or TIMEOUT once `timeout_s`
 * (> 0; <= 0 waits forever) has passed without completion.  The paper met
 * GPUs that accepted work and never finished it (Appendix A); this bounds
 * every wait.  Host only: touches no device, so it can be driven by a fake
 * query (INVALID_ARG for a NULL query). */
mgrav_status mgrav_watchdog_poll(int (*query)(void *user), void *user, double timeout_s);

/* ------------------------------------------------------------------ */
/* Learned Ewald correction (not in the paper; replaces the exact sums  */
/* of mgrav_set_ewald's EXACT mode when mode SURROGATE is selected).    */
/* ------------------------------------------------------------------ */

/* psi and grad psi of a unit mass in the unit box (the kernel described
 * at mgrav_set_ewald, double precision, the same sums as EXACT mode) at
 * n points r[n][3] (device); out[n][4] (device) = psi, d psi/dx, d psi/dy,
 * d psi/dz.  Used to produce training data and as the exact reference.
 * Errors: INVALID_ARG for alpha outside (0.5, 10), real_layers outside
 * 1..4, h2max outside 0..64. */
mgrav_status mgrav_ewald_psi(mgrav_ctx *ctx, const double *r, int64_t n, double alpha,
                             int real_layers, int h2max, double *out);

/* The surrogate is a network u -> (psi(u) - psi(0) + (2 pi/3)|u|^2,
 * grad psi(u) + (4 pi/3) u) on the fundamental octant u in [0, 1)^3 of
 * the unit box (psi is even in every coordinate), 3 -> 128 -> 128 -> 128
 * -> 4 with SiLU, weights rounded to bfloat16, float accumulation.  Its
 * parameters are one float vector of 34052 values in the order W1[128][3],
 * b1[128], W2[128][128], b2[128], W3[128][128], b3[128], W4[4][128], b4[4]
 * (row-major, output x input).  The network needs a device workspace of
 * mgrav_mlp_workspace_size(max_batch) bytes (max_batch: largest training
 * batch, a multiple of 1024), attached to a context; it is borrowed until
 * the next attach or destroy. */
mgrav_status mgrav_mlp_workspace_size(int64_t max_batch, size_t *bytes);
mgrav_status mgrav_mlp_attach(mgrav_ctx *ctx, void *workspace, size_t bytes, int64_t max_batch);

/* Load parameters (host, 34052 floats) and psi(0) of the Ewald parameters
 * the network was trained for; resets the optimiser state.  Blocking. */
mgrav_status mgrav_mlp_set_weights(mgrav_ctx *ctx, const float *params, int64_t count,
                                   double psi0);
/* Copy the current parameters to the host.  Blocking. */
mgrav_status mgrav_mlp_get_weights(mgrav_ctx *ctx, float *params, int64_t count);

/* y[n][4] = network(x[n][3]) (device, float).  Asynchronous. */
mgrav_status mgrav_mlp_forward(mgrav_ctx *ctx, const float *x, int64_t n, float *y);

/* grad[34052] (device) = d(sum_ij dy[i][j] y[i][j]) / d params for
 * y = network(x), x[n][3], dy[n][4] (device); n a multiple of 1024 and at
 * most max_batch.  Asynchronous. */
mgrav_status mgrav_mlp_backward(mgrav_ctx *ctx, const float *x, const float *dy, int64_t n,
                                float *grad);

typedef struct {
    int epochs;          /* passes over the samples (1..4096)              */
    int batch;           /* samples per step, multiple of 1024             */
    float lr, lr_min;    /* cosine schedule from lr to lr_min              */
    float beta1, beta2, adam_eps;  /* Adam                                 */
    float loss_weight[4];          /* weights of the four squared errors   */
    double psi0;         /* psi(0) for the Ewald parameters of the data     */
} mgrav_train_cfg;

/* Train on n samples: points u[n][3] in [0,1)^3 and psi[n][4] = (psi,
 * grad psi) at them (device, double; e.g. from mgrav_ewald_psi).  Each
 * step takes `batch` samples in an order fixed per epoch (an affine
 * bijection of the sample index), runs forward, backward and one Adam
 * update on the device; loss_host (nullable, host) receives the mean
 * weighted squared error of every epoch.  Starts from the weights set by
 * mgrav_mlp_set_weights.  Blocking. */
mgrav_status mgrav_mlp_train(mgrav_ctx *ctx, const double *u, const double *psi, int64_t n,
                             const mgrav_train_cfg *cfg, double *loss_host);

/* ---- Autotuning of the PP + PC kernel (persistent launch, Sec. 3.3) ----
 * The PP + PC kernel is compiled in a few variants: PP source entries
 * expanded into LDS per fill (`pp_chunk`, 16 particles x 16 B each), the
 * occupancy the register allocation aims at (`waves_per_simd`) and whether
 * the next PC chunk's cell records are loaded while the current one is
 * evaluated (`pc_prefetch`, 2-wave variants only).  Which is
 * fastest depends on the lists (lengths, PP/PC mix) and on the device.
 *
 * mgrav_interact_variants: number of variants (> 0).
 * mgrav_interact_variant_info: the parameters of one; INVALID_ARG out of
 *   range.  Any output may be NULL.
 * mgrav_set_interact_variant: use `variant` from the next compute on
 *   (default 0).  INVALID_ARG out of range.
 * mgrav_autotune: on the bound problem, runs the PP + PC parts with every
 *   variant (the first run of each untimed, then at least two timed runs,
 *   more while `budget_ms` of wall time lasts) and ranks them by median
 *   kernel time.  Then it times back-to-back computes of every part (3 to
 *   12, about a quarter of `budget_ms` each) from a graph and from direct
 *   launches, for the fastest variant and, when that one is not a 2-wave
 *   variant, for the fastest 2-wave one too (only those leave room for the
 *   exact Ewald correction beside the kernel), and keeps the fastest
 *   variant and launch mode for later computes (mgrav_set_interact_variant,
 *   mgrav_set_launch_mode); the variant is stored in `*chosen` (nullable).
 *   `acc`/`pot` (device, as for
 *   mgrav_compute) are overwritten by the trial runs.  `ms_per_variant`
 *   (host, nullable, mgrav_interact_variants() entries) receives each
 *   median, or -1 when not timed.  `cache_path` (nullable) names a text file
 *   of lines "mgrav-autotune <key> <variant> <launch mode>", the key being
 *   device, CU count and the list shape (n, buckets, PP and PC entries,
 *   images): a matching line is used without timing; otherwise the result is
 *   appended.  If the file cannot be appended to, the choices still apply
 *   and the call returns INVALID_ARG.  STATE before bind; errors of the trial
 *   computes are returned as they are.  Blocking. */
mgrav_status mgrav_interact_variants(int *count);
mgrav_status mgrav_interact_variant_info(int variant, int *pp_chunk, int *waves_per_simd,
                                         int *pc_prefetch);
mgrav_status mgrav_set_interact_variant(mgrav_ctx *ctx, int variant);
mgrav_status mgrav_autotune(mgrav_ctx *ctx, float *acc, float *pot, const char *cache_path,
                            double budget_ms, int *chosen, double *ms_per_variant);

/* How a compute is launched: MGRAV_LAUNCH_GRAPH (default) replays one HIP
 * graph per compute (captured at the first compute with a given set of
 * arguments); MGRAV_LAUNCH_DIRECT enqueues the kernels one by one.  In both
 * the exact Ewald correction runs beside the PP + PC kernel when both are
 * computed (a parallel branch of the graph, or a second stream of the
 * context), into a buffer that is added afterwards with the same
 * arithmetic.  Results are identical; which is faster depends on the
 * runtime (mgrav_stats graph_replay tells which one the last compute
 * used).  INVALID_ARG for another value. */
enum { MGRAV_LAUNCH_GRAPH = 0, MGRAV_LAUNCH_DIRECT = 1 };
mgrav_status mgrav_set_launch_mode(mgrav_ctx *ctx, int mode);

/* Order of the PP + PC kernel's work queue (Sec. 3.3: the persistent
 * kernel pulls sink buckets from one queue).  MGRAV_QUEUE_LPT: the active
 * buckets by estimated cost, most expensive first (in factors of 2), so the
 * kernel ends on short items.  MGRAV_QUEUE_LOCAL: only the buckets within a
 * factor 8 of the most expensive stay in front, in that order; the rest
 * follow in bucket (tree) order, cut into one segment per die of the chip,
 * each drained first by the wavefronts of its own die (then by the others),
 * so that the buckets one L2 serves at the same time share their source
 * cells.  MGRAV_QUEUE_AUTO (default): LOCAL when no mask is set and the
 * problem has 131072 buckets or more, else LPT.  Results are identical under every order (mgrav_stats
 * queue_local tells which layout the last compute used); INVALID_ARG for
 * another value.  Applies from the next compute. */
enum { MGRAV_QUEUE_AUTO = 0, MGRAV_QUEUE_LPT = 1, MGRAV_QUEUE_LOCAL = 2 };
mgrav_status mgrav_set_queue_order(mgrav_ctx *ctx, int order);

#ifdef __cplusplus
}
#endif

#endif /* MGRAV_H */
