/*
 * FP64 CPU oracle for the gravity hot path of PKDGRAV3
 * (Potter, Stadel & Teyssier, arXiv:1609.08621).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously
 * correct reference that the GPU library is checked against.  Only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code with the GPU library and includes none of
 * its headers.
 *
 * Everything is double precision.  Tensors are handled in full Cartesian
 * form (3^k components for order k) and contracted by brute-force sums over
 * index tuples, so that each formula can be checked against the paper's
 * description by eye.  Units: G = 1.
 *
 * What is computed, and where the paper states it:
 *   - binary tree, longest-axis equal-volume bisection, bucket leaves,
 *     particles in contiguous hierarchically sorted ranges    (Sec. 3.1)
 *   - per cell: centre of mass (expansion centre), bounding box, b_max,
 *     opening radius RO = b_max / theta                        (Sec. 3.1)
 *   - multipole moments about the centre of mass to 4th order
 *     (hexadecapole)                                            (Sec. 3.1)
 *   - bucket-sink checklist walk seeded with the root and its 26 periodic
 *     replicas; a source is accepted as a particle-cell (PC) interaction
 *     when it is beyond its opening radius plus the sink's extent and the
 *     bounding boxes are at least two softening lengths apart; opened leaf
 *     cells become particle-particle (PP) interactions       (Sec. 3.1)
 *   - PP and PC interactions (softened, order-4 moments)     (Sec. 3.1)
 *   - Ewald correction of the periodic box as a multipole expansion of the
 *     root cell, derivatives of the Ewald kernel through 5th order
 *                                                             (Sec. 3.1)
 *   - direct summation (open and periodic) as the plain definition
 *
 * Readings of points the paper leaves open (softening form, PC acceptance
 * rule for bucket sinks, tie-breaks, Ewald parameters) are listed in the
 * design notes and repeated next to the code that applies them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_SQRT_PI 1.7724538509055160273
#define ORC_PI 3.14159265358979323846

/* Threads the OpenMP loops below use. */
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Periodic images: id 0 is the box itself, ids 1..26 the neighbouring  */
/* replicas in lexicographic (ix, iy, iz) order, each in {-1, 0, 1}.    */
/* ------------------------------------------------------------------ */
void orc_image_shift(int id, double L, double out[3]) {
    if (id == 0) {
        out[0] = out[1] = out[2] = 0.0;
        return;
    }
    int k = 0;
    for (int ix = -1; ix <= 1; ++ix)
        for (int iy = -1; iy <= 1; ++iy)
            for (int iz = -1; iz <= 1; ++iz) {
                if (ix == 0 && iy == 0 && iz == 0) continue;
                ++k;
                if (k == id) {
                    out[0] = ix * L;
                    out[1] = iy * L;
                    out[2] = iz * L;
                    return;
                }
            }
    out[0] = out[1] = out[2] = NAN;
}

/* ------------------------------------------------------------------ */
/* Packed symmetric moments: index tuples with non-decreasing axes, in */
/* lexicographic order.  mom[0]=M, [1..6]=order 2, [7..16]=order 3,    */
/* [17..31]=order 4.  Order 1 vanishes about the centre of mass.       */
/* ------------------------------------------------------------------ */
static int packed_base(int k) {
    switch (k) {
    case 0: return 0;
    case 2: return 1;
    case 3: return 7;
    case 4: return 17;
    default: return -1;
    }
}

/* position of a sorted tuple within its order's packed block */
static int packed_index(int k, const int *sorted) {
    int idx = 0;
    /* enumerate non-decreasing tuples in lexicographic order and count */
    int t[4] = {0, 0, 0, 0};
    for (;;) {
        int same = 1;
        for (int i = 0; i < k; ++i)
            if (t[i] != sorted[i]) same = 0;
        if (same) return idx;
        ++idx;
        /* next non-decreasing tuple */
        int i = k - 1;
        while (i >= 0 && t[i] == 2) --i;
        if (i < 0) return -1;
        t[i]++;
        for (int j = i + 1; j < k; ++j) t[j] = t[i];
    }
}

static void digits(int k, int flat, int *a) {
    for (int i = k - 1; i >= 0; --i) {
        a[i] = flat % 3;
        flat /= 3;
    }
}

static void sort_small(int k, int *a) {
    for (int i = 1; i < k; ++i)
        for (int j = i; j > 0 && a[j - 1] > a[j]; --j) {
            int t = a[j];
            a[j] = a[j - 1];
            a[j - 1] = t;
        }
}

static const int POW3[8] = {1, 3, 9, 27, 81, 243, 729, 2187};

/* Expand packed moments of one cell into full tensors M2[9], M3[27], M4[81]. */
static void unpack_moments(const double *mom, double *M2, double *M3, double *M4) {
    double *full[5] = {0, 0, M2, M3, M4};
    for (int k = 2; k <= 4; ++k) {
        for (int f = 0; f < POW3[k]; ++f) {
            int a[4];
            digits(k, f, a);
            sort_small(k, a);
            full[k][f] = mom[packed_base(k) + packed_index(k, a)];
        }
    }
}

/* ------------------------------------------------------------------ */
/* Derivative tensors of a radial function.                            */
/*                                                                     */
/* For f(|R|) with radial derivatives a_n = ((1/r) d/dr)^n f, the k-th */
/* Cartesian derivative is a sum over all ways of grouping the k index */
/* positions into m disjoint pairs and k-2m singles:                   */
/*   d^k f / dR_{i1}..dR_{ik} = sum_pairings a_{k-m} prod(delta) prod(R) */
/* (each derivative either lands on a_n, raising n and adding a single  */
/* R factor, or on an existing R factor, turning it into a delta).      */
/* The table below lists, for every full index tuple, the surviving     */
/* pairings as (n, powers of Rx, Ry, Rz, multiplicity).                 */
/* ------------------------------------------------------------------ */
#define ORC_KMAX 5
typedef struct {
    int n, ex, ey, ez, mult;
} DTerm;
typedef struct {
    int nterm;
    DTerm term[32];
} DEntry;
static DEntry dtab_store[364];
static DEntry *dtab[ORC_KMAX + 1];
static int dtab_ready = 0;

static void add_term(DEntry *e, int n, int ex, int ey, int ez) {
    for (int i = 0; i < e->nterm; ++i) {
        DTerm *t = &e->term[i];
        if (t->n == n && t->ex == ex && t->ey == ey && t->ez == ez) {
            t->mult++;
            return;
        }
    }
    DTerm *t = &e->term[e->nterm++];
    t->n = n;
    t->ex = ex;
    t->ey = ey;
    t->ez = ez;
    t->mult = 1;
}

/* Recursively enumerate pairings of positions; used[] marks consumed. */
static void enum_pairings(int k, const int *axis, int *used, int npair, int *cnt, DEntry *e) {
    int first = -1;
    for (int i = 0; i < k; ++i)
        if (!used[i]) {
            first = i;
            break;
        }
    if (first < 0) {
        add_term(e, k - npair, cnt[0], cnt[1], cnt[2]);
        return;
    }
    /* option 1: position `first` is a single R factor */
    used[first] = 1;
    cnt[axis[first]]++;
    enum_pairings(k, axis, used, npair, cnt, e);
    cnt[axis[first]]--;
    /* option 2: pair `first` with a later unused position (delta) */
    for (int j = first + 1; j < k; ++j) {
        if (used[j] || axis[j] != axis[first]) continue; /* delta vanishes */
        used[j] = 1;
        enum_pairings(k, axis, used, npair + 1, cnt, e);
        used[j] = 0;
    }
    used[first] = 0;
}

void orc_init(void) {
    if (dtab_ready) return;
    int off = 0;
    for (int k = 0; k <= ORC_KMAX; ++k) {
        dtab[k] = &dtab_store[off];
        for (int f = 0; f < POW3[k]; ++f) {
            int axis[ORC_KMAX], used[ORC_KMAX] = {0}, cnt[3] = {0, 0, 0};
            digits(k, f, axis);
            DEntry *e = &dtab[k][f];
            e->nterm = 0;
            enum_pairings(k, axis, used, 0, cnt, e);
        }
        off += POW3[k];
    }
    dtab_ready = 1;
}

/* Fill T[k][flat] for k = 0..kmax from the radial derivatives a[0..kmax]. */
static void radial_tensors(const double R[3], const double *a, int kmax, double *T[]) {
    double p[3][ORC_KMAX + 1];
    for (int d = 0; d < 3; ++d) {
        p[d][0] = 1.0;
        for (int e = 1; e <= ORC_KMAX; ++e) p[d][e] = p[d][e - 1] * R[d];
    }
    for (int k = 0; k <= kmax; ++k)
        for (int f = 0; f < POW3[k]; ++f) {
            const DEntry *e = &dtab[k][f];
            double s = 0.0;
            for (int i = 0; i < e->nterm; ++i) {
                const DTerm *t = &e->term[i];
                s += t->mult * a[t->n] * p[0][t->ex] * p[1][t->ey] * p[2][t->ez];
            }
            T[k][f] = s;
        }
}

/* ------------------------------------------------------------------ */
/* Tree (Sec. 3.1).                                                    */
/* Reading of the tie-breaks: longest axis of the cell's geometric box  */
/* (lowest axis index on ties); split at the midpoint, particles with   */
/* x >= mid go to the upper (right) child; if one half is empty the     */
/* geometric box shrinks to the occupied half and bisection repeats;    */
/* after 64 halvings along a path (coincident points) a cell is split   */
/* by index halves.  Cells are numbered in node-left-right order.       */
/* Partitioning is stable, so particles keep their input order inside   */
/* every cell.                                                         */
/* ------------------------------------------------------------------ */
typedef struct {
    const double *pos;
    int64_t *idx, *tmp;
    int bucket;
    int64_t ncell, cap;
    int overflow;
    int64_t *cell_first;
    int32_t *cell_count, *child;
} TreeBuild;

static int64_t tb_cell(TreeBuild *t, int64_t first, int64_t count, const double lo[3],
                       const double hi[3], int depth) {
    int64_t c = t->ncell++;
    if (c >= t->cap) {
        t->overflow = 1;
        return c;
    }
    t->cell_first[c] = first;
    t->cell_count[c] = (int32_t)count;
    t->child[2 * c] = -1;
    t->child[2 * c + 1] = -1;
    if (count <= t->bucket) return c;

    double blo[3] = {lo[0], lo[1], lo[2]}, bhi[3] = {hi[0], hi[1], hi[2]};
    double llo[3], lhi[3], rlo[3], rhi[3];
    int64_t nl;
    for (;;) {
        if (depth >= 64) { /* coincident points: split by index halves */
            nl = (count + 1) / 2;
            memcpy(llo, blo, sizeof blo);
            memcpy(lhi, bhi, sizeof bhi);
            memcpy(rlo, blo, sizeof blo);
            memcpy(rhi, bhi, sizeof bhi);
            break;
        }
        int ax = 0;
        for (int d = 1; d < 3; ++d)
            if (bhi[d] - blo[d] > bhi[ax] - blo[ax]) ax = d;
        double mid = 0.5 * (blo[ax] + bhi[ax]);
        /* stable partition: lower half first, then upper half */
        int64_t nlow = 0, nup = 0;
        for (int64_t i = 0; i < count; ++i) {
            int64_t p = t->idx[first + i];
            if (t->pos[3 * p + ax] < mid) t->idx[first + nlow++] = p;
            else t->tmp[nup++] = p;
        }
        for (int64_t i = 0; i < nup; ++i) t->idx[first + nlow + i] = t->tmp[i];
        nl = nlow;
        depth++;
        if (nl == 0) {
            blo[ax] = mid;
            continue;
        }
        if (nl == count) {
            bhi[ax] = mid;
            continue;
        }
        memcpy(llo, blo, sizeof blo);
        memcpy(lhi, bhi, sizeof bhi);
        memcpy(rlo, blo, sizeof blo);
        memcpy(rhi, bhi, sizeof bhi);
        lhi[ax] = mid;
        rlo[ax] = mid;
        break;
    }
    int64_t l = tb_cell(t, first, nl, llo, lhi, depth);
    int64_t r = tb_cell(t, first + nl, count - nl, rlo, rhi, depth);
    if (!t->overflow) {
        t->child[2 * c] = (int32_t)l;
        t->child[2 * c + 1] = (int32_t)r;
    }
    return c;
}

/* Per-cell centre of mass, tight bounding box, b_max and packed moments,
 * all computed directly from the cell's particles (no shifting of child
 * moments), summing in tree order. */
static void cell_properties(int64_t c, const double *pos, const double *mass, const int64_t *perm,
                            const int64_t *cell_first, const int32_t *cell_count, double *com,
                            double *bmax, double *bbox, double *mom) {
    int64_t f = cell_first[c], n = cell_count[c];
    double M = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = f; i < f + n; ++i) {
        int64_t p = perm[i];
        double m = mass[p];
        M += m;
        mx += m * pos[3 * p + 0];
        my += m * pos[3 * p + 1];
        mz += m * pos[3 * p + 2];
        for (int d = 0; d < 3; ++d) {
            if (pos[3 * p + d] < lo[d]) lo[d] = pos[3 * p + d];
            if (pos[3 * p + d] > hi[d]) hi[d] = pos[3 * p + d];
        }
    }
    double X[3] = {mx / M, my / M, mz / M};
    double b2 = 0.0;
    double M2[9] = {0}, M3[27] = {0}, M4[81] = {0};
    for (int64_t i = f; i < f + n; ++i) {
        int64_t p = perm[i];
        double m = mass[p];
        double s[3] = {pos[3 * p] - X[0], pos[3 * p + 1] - X[1], pos[3 * p + 2] - X[2]};
        double r2 = s[0] * s[0] + s[1] * s[1] + s[2] * s[2];
        if (r2 > b2) b2 = r2;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                M2[3 * a + b] += m * s[a] * s[b];
                for (int cc = 0; cc < 3; ++cc) {
                    M3[9 * a + 3 * b + cc] += m * s[a] * s[b] * s[cc];
                    for (int d = 0; d < 3; ++d)
                        M4[27 * a + 9 * b + 3 * cc + d] += m * s[a] * s[b] * s[cc] * s[d];
                }
            }
    }
    for (int d = 0; d < 3; ++d) {
        com[3 * c + d] = X[d];
        bbox[6 * c + d] = lo[d];
        bbox[6 * c + 3 + d] = hi[d];
    }
    bmax[c] = sqrt(b2);
    double *pm = mom + 32 * c;
    pm[0] = M;
    double *full[5] = {0, 0, M2, M3, M4};
    for (int k = 2; k <= 4; ++k)
        for (int fl = 0; fl < POW3[k]; ++fl) {
            int a[4];
            digits(k, fl, a);
            int sorted = 1;
            for (int i = 1; i < k; ++i)
                if (a[i] < a[i - 1]) sorted = 0;
            if (!sorted) continue;
            pm[packed_base(k) + packed_index(k, a)] = full[k][fl];
        }
}

/* Build the tree.  pos: input order, AoS [n][3].  Returns the number of
 * cells, or -1 if `cap` cells are not enough (2n always suffices). */
/* Build the tree with the root's geometric box given (root_box: lo xyz,
 * hi xyz), or the default root (root_box NULL).  Sec. 3.2 builds the tree
 * of the very active particles over the geometric structure of the fixed
 * tree: with the same root box both trees bisect space along the same
 * planes, so their cells coincide wherever both are refined. */
int64_t orc_tree_build_box(int64_t n, const double *pos, const double *mass, double L,
                           int bucket, const double *root_box, int64_t cap, int64_t *perm,
                           int64_t *cell_first, int32_t *cell_count, int32_t *child, double *com,
                           double *bmax, double *bbox, double *mom, int32_t *bucket_cell,
                           int64_t *n_bucket);

int64_t orc_tree_build(int64_t n, const double *pos, const double *mass, double L, int bucket,
                       int64_t cap, int64_t *perm, int64_t *cell_first, int32_t *cell_count,
                       int32_t *child, double *com, double *bmax, double *bbox, double *mom,
                       int32_t *bucket_cell, int64_t *n_bucket) {
    return orc_tree_build_box(n, pos, mass, L, bucket, NULL, cap, perm, cell_first, cell_count,
                              child, com, bmax, bbox, mom, bucket_cell, n_bucket);
}

int64_t orc_tree_build_box(int64_t n, const double *pos, const double *mass, double L,
                           int bucket, const double *root_box, int64_t cap, int64_t *perm,
                           int64_t *cell_first, int32_t *cell_count, int32_t *child, double *com,
                           double *bmax, double *bbox, double *mom, int32_t *bucket_cell,
                           int64_t *n_bucket) {
    orc_init();
    if (n <= 0 || bucket < 1) return -1;
    TreeBuild t;
    t.pos = pos;
    t.idx = perm;
    t.tmp = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    t.bucket = bucket;
    t.ncell = 0;
    t.cap = cap;
    t.overflow = 0;
    t.cell_first = cell_first;
    t.cell_count = cell_count;
    t.child = child;
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    double lo[3], hi[3];
    if (root_box) { /* the root's box is given */
        for (int d = 0; d < 3; ++d) {
            lo[d] = root_box[d];
            hi[d] = root_box[3 + d];
        }
    } else if (L > 0.0) { /* periodic: the root is the box [0, L)^3 */
        for (int d = 0; d < 3; ++d) {
            lo[d] = 0.0;
            hi[d] = L;
        }
    } else { /* open: the root is the tight bounding box */
        for (int d = 0; d < 3; ++d) {
            lo[d] = INFINITY;
            hi[d] = -INFINITY;
        }
        for (int64_t i = 0; i < n; ++i)
            for (int d = 0; d < 3; ++d) {
                if (pos[3 * i + d] < lo[d]) lo[d] = pos[3 * i + d];
                if (pos[3 * i + d] > hi[d]) hi[d] = pos[3 * i + d];
            }
    }
    tb_cell(&t, 0, n, lo, hi, 0);
    free(t.tmp);
    if (t.overflow) return -1;
    /* cells are independent: each is computed from its own particles */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < t.ncell; ++c)
        cell_properties(c, pos, mass, perm, cell_first, cell_count, com, bmax, bbox, mom);
    int64_t nb = 0;
    for (int64_t c = 0; c < t.ncell; ++c)
        if (child[2 * c] < 0) bucket_cell[nb++] = (int32_t)c;
    *n_bucket = nb;
    return t.ncell;
}

/* ------------------------------------------------------------------ */
/* Interaction lists: bucket-sink checklist walk (Sec. 3.1).           */
/* The checklist starts with the root and its replicas (image ids in   */
/* increasing order); entries are taken from the front, and an opened  */
/* cell's children are appended at the end.  A source cell C seen      */
/* through image n is                                                  */
/*   PC  if |X_C + n L - X_S| > b_max,C / theta + b_max,S              */
/*       and the bounding boxes are at least 2 eps apart,              */
/*   PP  otherwise, if C is a leaf (its particles, RO = 0),            */
/*   opened otherwise.                                                 */
/* (The sink-side factor 1.5 of the paper belongs to cell-cell         */
/* interactions, which this path does not form.)                       */
/* ------------------------------------------------------------------ */
static int accept_pc(int64_t c, int img, int64_t s, const double *com, const double *bmax,
                     const double *bbox, double theta, double eps, double L) {
    double sh[3];
    orc_image_shift(img, L, sh);
    double dx = com[3 * c + 0] + sh[0] - com[3 * s + 0];
    double dy = com[3 * c + 1] + sh[1] - com[3 * s + 1];
    double dz = com[3 * c + 2] + sh[2] - com[3 * s + 2];
    double d = sqrt(dx * dx + dy * dy + dz * dz);
    if (!(d > bmax[c] / theta + bmax[s])) return 0;
    double g2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double clo = bbox[6 * c + a] + sh[a], chi = bbox[6 * c + 3 + a] + sh[a];
        double slo = bbox[6 * s + a], shi = bbox[6 * s + 3 + a];
        double g = 0.0;
        if (clo - shi > g) g = clo - shi;
        if (slo - chi > g) g = slo - chi;
        g2 += g * g;
    }
    return sqrt(g2) >= 2.0 * eps;
}

/* Walk one sink bucket.  If the output arrays are NULL only counts. */
/* The checklist starts with every root (in the given order), each seen
 * through images 0 .. n_img-1.  One root (cell 0) for a single tree; two
 * for the fixed and the very active tree of Sec. 3.2, walked together. */
static void walk_bucket(int64_t s, const int32_t *child, const double *com, const double *bmax,
                        const double *bbox, double theta, double eps, double L, int n_img,
                        int n_roots, const int32_t *roots, int64_t *npp, int64_t *npc,
                        int32_t *pp_src, uint8_t *pp_img, int32_t *pc_src, uint8_t *pc_img) {
    int64_t cap = 1024, head = 0, tail = 0;
    while (cap < 2 * (int64_t)n_roots * n_img) cap *= 2;
    int64_t *qc = (int64_t *)malloc(sizeof(int64_t) * cap);
    int *qi = (int *)malloc(sizeof(int) * cap);
    for (int r = 0; r < n_roots; ++r)
        for (int i = 0; i < n_img; ++i) {
            qc[tail] = roots[r];
            qi[tail] = i;
            ++tail;
        }
    int64_t kpp = 0, kpc = 0;
    while (head < tail) {
        int64_t c = qc[head];
        int img = qi[head];
        ++head;
        if (accept_pc(c, img, s, com, bmax, bbox, theta, eps, L)) {
            if (pc_src) {
                pc_src[kpc] = (int32_t)c;
                pc_img[kpc] = (uint8_t)img;
            }
            ++kpc;
        } else if (child[2 * c] < 0) {
            if (pp_src) {
                pp_src[kpp] = (int32_t)c;
                pp_img[kpp] = (uint8_t)img;
            }
            ++kpp;
        } else {
            if (tail + 2 > cap) {
                cap *= 2;
                qc = (int64_t *)realloc(qc, sizeof(int64_t) * cap);
                qi = (int *)realloc(qi, sizeof(int) * cap);
            }
            qc[tail] = child[2 * c];
            qi[tail] = img;
            ++tail;
            qc[tail] = child[2 * c + 1];
            qi[tail] = img;
            ++tail;
        }
    }
    free(qc);
    free(qi);
    *npp = kpp;
    *npc = kpc;
}

/* Pass 1: per-bucket list lengths as CSR offsets (pp_off, pc_off:
 * n_bucket+1), for a checklist seeded with the n_roots cells `roots`. */
void orc_lists_count_roots(int64_t n_bucket, const int32_t *bucket_cell, const int32_t *child,
                           const double *com, const double *bmax, const double *bbox,
                           double theta, double eps, double L, int n_img, int n_roots,
                           const int32_t *roots, int64_t *pp_off, int64_t *pc_off) {
    pp_off[0] = 0;
    pc_off[0] = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < n_bucket; ++b) {
        int64_t a, c;
        walk_bucket(bucket_cell[b], child, com, bmax, bbox, theta, eps, L, n_img, n_roots, roots,
                    &a, &c, NULL, NULL, NULL, NULL);
        pp_off[b + 1] = a;
        pc_off[b + 1] = c;
    }
    for (int64_t b = 0; b < n_bucket; ++b) {
        pp_off[b + 1] += pp_off[b];
        pc_off[b + 1] += pc_off[b];
    }
}

/* Pass 2: fill the lists in checklist order. */
void orc_lists_fill_roots(int64_t n_bucket, const int32_t *bucket_cell, const int32_t *child,
                          const double *com, const double *bmax, const double *bbox, double theta,
                          double eps, double L, int n_img, int n_roots, const int32_t *roots,
                          const int64_t *pp_off, const int64_t *pc_off, int32_t *pp_src,
                          uint8_t *pp_img, int32_t *pc_src, uint8_t *pc_img) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < n_bucket; ++b) {
        int64_t a, c;
        walk_bucket(bucket_cell[b], child, com, bmax, bbox, theta, eps, L, n_img, n_roots, roots,
                    &a, &c, pp_src + pp_off[b], pp_img + pp_off[b], pc_src + pc_off[b],
                    pc_img + pc_off[b]);
    }
}

/* The single tree: the checklist starts with its root, cell 0. */
static const int32_t ORC_ROOT0[1] = {0};

void orc_lists_count(int64_t n_bucket, const int32_t *bucket_cell, const int32_t *child,
                     const double *com, const double *bmax, const double *bbox, double theta,
                     double eps, double L, int n_img, int64_t *pp_off, int64_t *pc_off) {
    orc_lists_count_roots(n_bucket, bucket_cell, child, com, bmax, bbox, theta, eps, L, n_img, 1,
                          ORC_ROOT0, pp_off, pc_off);
}

void orc_lists_fill(int64_t n_bucket, const int32_t *bucket_cell, const int32_t *child,
                    const double *com, const double *bmax, const double *bbox, double theta,
                    double eps, double L, int n_img, const int64_t *pp_off, const int64_t *pc_off,
                    int32_t *pp_src, uint8_t *pp_img, int32_t *pc_src, uint8_t *pc_img) {
    orc_lists_fill_roots(n_bucket, bucket_cell, child, com, bmax, bbox, theta, eps, L, n_img, 1,
                         ORC_ROOT0, pp_off, pc_off, pp_src, pp_img, pc_src, pc_img);
}

/* ------------------------------------------------------------------ */
/* Softened Green's function.  Reading of the softening: Plummer,       */
/* G(r) = -1/sqrt(r^2 + eps^2), used for PP and, as the function whose  */
/* Taylor expansion the multipoles represent, for PC as well.           */
/* Radial derivatives of g = (r^2+eps^2)^(-1/2):                        */
/*   a_n = ((1/r) d/dr)^n g = (-1)^n (2n-1)!! (r^2+eps^2)^(-(2n+1)/2).  */
/* ------------------------------------------------------------------ */
static void plummer_radial(double r2, double eps2, int nmax, double *a) {
    double D = r2 + eps2;
    double base = 1.0 / sqrt(D);
    double df = 1.0; /* (2n-1)!! */
    for (int n = 0; n <= nmax; ++n) {
        if (n > 0) df *= (2 * n - 1);
        a[n] = ((n & 1) ? -1.0 : 1.0) * df * base * pow(D, -(double)n);
    }
}

/* Potential and acceleration at x from a cell with packed moments about
 * its centre of mass X (already shifted by the image):
 *   phi  = sum_{k=0,2,3,4} (-1)^k/k!  M_k . d^k G(R)
 *   acc  = -grad phi,  R = x - X,  G = -g.
 * This is the Taylor expansion of sum_j m_j G(x - x_j) about X.        */
static void pc_eval(const double *mom, const double X[3], const double x[3], double eps2,
                    double out[4]) {
    static const double fact[6] = {1, 1, 2, 6, 24, 120};
    double R[3] = {x[0] - X[0], x[1] - X[1], x[2] - X[2]};
    double a[6];
    plummer_radial(R[0] * R[0] + R[1] * R[1] + R[2] * R[2], eps2, 5, a);
    double T0[1], T1[3], T2[9], T3[27], T4[81], T5[243];
    double *T[6] = {T0, T1, T2, T3, T4, T5};
    radial_tensors(R, a, 5, T);
    double M2[9], M3[27], M4[81];
    unpack_moments(mom, M2, M3, M4);
    double M0[1] = {mom[0]};
    const double *Mk[5] = {M0, NULL, M2, M3, M4};
    double phi = 0.0, acc[3] = {0, 0, 0};
    for (int k = 0; k <= 4; ++k) {
        if (k == 1) continue; /* dipole vanishes about the centre of mass */
        double c = ((k & 1) ? -1.0 : 1.0) / fact[k];
        double sp = 0.0;
        for (int f = 0; f < POW3[k]; ++f) sp += Mk[k][f] * T[k][f];
        phi += -c * sp; /* G = -g */
        for (int b = 0; b < 3; ++b) {
            double sa = 0.0;
            for (int f = 0; f < POW3[k]; ++f) sa += Mk[k][f] * T[k + 1][3 * f + b];
            acc[b] += c * sa; /* -grad(-g term) */
        }
    }
    out[0] = acc[0];
    out[1] = acc[1];
    out[2] = acc[2];
    out[3] = phi;
}

/* Exported for the pins: one PC interaction at a point. */
void orc_pc_point(const double *mom32, const double X[3], const double x[3], double eps,
                  double out[4]) {
    orc_init();
    pc_eval(mom32, X, x, eps * eps, out);
}

/* Exported for the pins: centre of mass and packed moments of a point set. */
void orc_moments(int64_t n, const double *pos, const double *mass, double com[3],
                 double mom32[32]) {
    orc_init();
    int64_t *perm = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    int64_t first = 0;
    int32_t cnt = (int32_t)n;
    double bmax, bbox[6];
    cell_properties(0, pos, mass, perm, &first, &cnt, com, &bmax, bbox, mom32);
    free(perm);
}

/* ------------------------------------------------------------------ */
/* Ewald kernel (Sec. 3.1, periodic boundaries).                       */
/* In a unit box, for a unit mass at the origin with a neutralising     */
/* background, the periodic potential is phi_per; psi is what the      */
/* periodic field adds to the 27 nearest images (box + 26 replicas):   */
/*   psi(r) = phi_per(r) + sum_{n in N1} 1/|r - n|                     */
/*          = sum_{n in N1} erf(a|r-n|)/|r-n|                          */
/*            - sum_{n not in N1, |n|_inf <= R} erfc(a|r-n|)/|r-n|     */
/*            - (1/pi) sum_{0<|h|^2<=H} exp(-pi^2 h^2/a^2)/h^2 cos(2 pi h.r) */
/*            + pi/a^2.                                                */
/* Radial derivatives are taken from integral representations,         */
/*   erf(a r)/r  = (2/sqrt(pi)) int_0^a exp(-t^2 r^2) dt,              */
/*   erfc(a r)/r = (2/sqrt(pi)) int_a^inf exp(-t^2 r^2) dt,            */
/* so ((1/r) d/dr)^n brings down (-2 t^2)^n under the integral, which   */
/* is evaluated by Gauss-Legendre quadrature (no cancellation at r=0). */
/* A box of side L scales as psi_L(r) = psi(r/L)/L.                     */
/* ------------------------------------------------------------------ */
#define ORC_GL_MAX 256
static double gl_x[ORC_GL_MAX], gl_w[ORC_GL_MAX];
static int gl_n = 0;

/* Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on the
 * Legendre polynomial P_n (three-term recurrence). */
void orc_set_quadrature(int n) {
    if (n > ORC_GL_MAX) n = ORC_GL_MAX;
    for (int i = 0; i < n; ++i) {
        double z = cos(ORC_PI * (i + 0.75) / (n + 0.5)), pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            double z1 = z;
            z = z1 - p1 / pp;
            if (fabs(z - z1) < 1e-16) break;
        }
        {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
        }
        gl_x[i] = z;
        gl_w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
    gl_n = n;
}

/* a_n for erf(alpha r)/r (lower = 1, t in [0, alpha]) or erfc(alpha r)/r
 * (lower = 0, t in [alpha, alpha + 12/r]). */
static void ewald_radial(double r, double alpha, int is_erf, int nmax, double *a) {
    if (gl_n == 0) orc_set_quadrature(128);
    double t0, t1;
    if (is_erf) {
        t0 = 0.0;
        t1 = alpha;
    } else {
        t0 = alpha;
        t1 = alpha + 12.0 / r;
    }
    double half = 0.5 * (t1 - t0), mid = 0.5 * (t1 + t0);
    for (int n = 0; n <= nmax; ++n) a[n] = 0.0;
    for (int q = 0; q < gl_n; ++q) {
        double t = mid + half * gl_x[q];
        double w = half * gl_w[q] * exp(-t * t * r * r);
        double p = 1.0;
        for (int n = 0; n <= nmax; ++n) {
            a[n] += w * p;
            p *= -2.0 * t * t;
        }
    }
    for (int n = 0; n <= nmax; ++n) a[n] *= 2.0 / ORC_SQRT_PI;
}

/* Derivative tensors D_k of psi (unit box) at r, k = 0..kmax, written
 * consecutively into out (1 + 3 + 9 + ... values).  rmax: outer real-space
 * shell |n|_inf <= rmax (1 = only the 27 near images); h2max: k-space
 * cut-off on |h|^2. */
void orc_ewald_derivs(const double r[3], double alpha, int rmax, int h2max, int kmax,
                      double *out) {
    orc_init();
    double *D[ORC_KMAX + 1];
    int off = 0;
    for (int k = 0; k <= kmax; ++k) {
        D[k] = out + off;
        for (int f = 0; f < POW3[k]; ++f) D[k][f] = 0.0;
        off += POW3[k];
    }
    double T0[1], T1[3], T2[9], T3[27], T4[81], T5[243];
    double *T[6] = {T0, T1, T2, T3, T4, T5};
    double a[ORC_KMAX + 1];
    /* real space */
    for (int ix = -rmax; ix <= rmax; ++ix)
        for (int iy = -rmax; iy <= rmax; ++iy)
            for (int iz = -rmax; iz <= rmax; ++iz) {
                int near = abs(ix) <= 1 && abs(iy) <= 1 && abs(iz) <= 1;
                double v[3] = {r[0] - ix, r[1] - iy, r[2] - iz};
                double rho = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                ewald_radial(rho, alpha, near, kmax, a);
                radial_tensors(v, a, kmax, T);
                double sgn = near ? 1.0 : -1.0;
                for (int k = 0; k <= kmax; ++k)
                    for (int f = 0; f < POW3[k]; ++f) D[k][f] += sgn * T[k][f];
            }
    /* reciprocal space: d^k cos(2 pi h.r) = (2 pi)^k h^(x)k cos(2 pi h.r + k pi/2) */
    int hm = (int)ceil(sqrt((double)h2max));
    for (int hx = -hm; hx <= hm; ++hx)
        for (int hy = -hm; hy <= hm; ++hy)
            for (int hz = -hm; hz <= hm; ++hz) {
                int h2 = hx * hx + hy * hy + hz * hz;
                if (h2 == 0 || h2 > h2max) continue;
                double h[3] = {hx, hy, hz};
                double c = exp(-ORC_PI * ORC_PI * h2 / (alpha * alpha)) / h2 / ORC_PI;
                double th = 2.0 * ORC_PI * (hx * r[0] + hy * r[1] + hz * r[2]);
                for (int k = 0; k <= kmax; ++k) {
                    double ck = -c * pow(2.0 * ORC_PI, k) * cos(th + k * 0.5 * ORC_PI);
                    for (int f = 0; f < POW3[k]; ++f) {
                        int ax[ORC_KMAX];
                        digits(k, f, ax);
                        double prod = 1.0;
                        for (int i = 0; i < k; ++i) prod *= h[ax[i]];
                        D[k][f] += ck * prod;
                    }
                }
            }
    D[0][0] += ORC_PI / (alpha * alpha);
}

/* Ewald correction at a particle from the root moments:
 *   phi_corr = sum_{k=0,2,3,4} (-1)^k/k! M_k . d^k psi_L(R),
 *   acc_corr = -grad phi_corr,  R = x - X_root.                       */
static void ewald_root_eval(const double *mom, const double X[3], const double x[3], double L,
                            double alpha, int rmax, int h2max, double out[4]) {
    static const double fact[6] = {1, 1, 2, 6, 24, 120};
    double r[3] = {(x[0] - X[0]) / L, (x[1] - X[1]) / L, (x[2] - X[2]) / L};
    double buf[364];
    orc_ewald_derivs(r, alpha, rmax, h2max, 5, buf);
    double *D[6];
    int off = 0;
    for (int k = 0; k <= 5; ++k) {
        D[k] = buf + off;
        off += POW3[k];
    }
    double M2[9], M3[27], M4[81];
    unpack_moments(mom, M2, M3, M4);
    double M0[1] = {mom[0]};
    const double *Mk[5] = {M0, NULL, M2, M3, M4};
    double phi = 0.0, acc[3] = {0, 0, 0};
    for (int k = 0; k <= 4; ++k) {
        if (k == 1) continue;
        double c = ((k & 1) ? -1.0 : 1.0) / fact[k];
        double sp = 0.0;
        for (int f = 0; f < POW3[k]; ++f) sp += Mk[k][f] * D[k][f];
        phi += c * sp * pow(L, -1.0 - k);
        for (int b = 0; b < 3; ++b) {
            double sa = 0.0;
            for (int f = 0; f < POW3[k]; ++f) sa += Mk[k][f] * D[k + 1][3 * f + b];
            acc[b] -= c * sa * pow(L, -2.0 - k);
        }
    }
    out[0] = acc[0];
    out[1] = acc[1];
    out[2] = acc[2];
    out[3] = phi;
}

void orc_ewald_root_point(const double *mom32, const double X[3], const double x[3], double L,
                          double alpha, int rmax, int h2max, double out[4]) {
    orc_init();
    ewald_root_eval(mom32, X, x, L, alpha, rmax, h2max, out);
}

/* ------------------------------------------------------------------ */
/* Evaluation of the lists (and the Ewald correction) for every         */
/* particle of the selected sink buckets.  Particles are in tree order. */
/* parts: bit 0 = PP, bit 1 = PC, bit 2 = Ewald.  Self term (i, image 0) */
/* is excluded from PP; the particle's own replicas are included.       */
/* ------------------------------------------------------------------ */
void orc_eval_sub(int64_t n, const double *pos, const double *mass, double eps, double L,
                  const int64_t *cell_first, const int32_t *cell_count, const double *com,
                  const double *mom, int64_t n_bucket, const int32_t *bucket_cell,
                  const int64_t *pp_off, const int32_t *pp_src, const uint8_t *pp_img,
                  const uint8_t *pp_sub, const int64_t *pc_off, const int32_t *pc_src,
                  const uint8_t *pc_img, int64_t n_sel, const int32_t *sel, int parts,
                  double ew_alpha, int ew_rmax, int ew_h2max, double *acc, double *pot);

void orc_eval(int64_t n, const double *pos, const double *mass, double eps, double L,
              const int64_t *cell_first, const int32_t *cell_count, const double *com,
              const double *mom, int64_t n_bucket, const int32_t *bucket_cell,
              const int64_t *pp_off, const int32_t *pp_src, const uint8_t *pp_img,
              const int64_t *pc_off, const int32_t *pc_src, const uint8_t *pc_img,
              int64_t n_sel, const int32_t *sel, int parts, double ew_alpha, int ew_rmax,
              int ew_h2max, double *acc, double *pot) {
    orc_eval_sub(n, pos, mass, eps, L, cell_first, cell_count, com, mom, n_bucket, bucket_cell,
                 pp_off, pp_src, pp_img, NULL, pc_off, pc_src, pc_img, n_sel, sel, parts,
                 ew_alpha, ew_rmax, ew_h2max, acc, pot);
}

/* As orc_eval, with PP entries that may name a single particle of their
 * source leaf: pp_sub[e] = 0 for the whole leaf, k + 1 for its k-th
 * particle (pp_sub NULL: whole leaves). */
void orc_eval_sub(int64_t n, const double *pos, const double *mass, double eps, double L,
                  const int64_t *cell_first, const int32_t *cell_count, const double *com,
                  const double *mom, int64_t n_bucket, const int32_t *bucket_cell,
                  const int64_t *pp_off, const int32_t *pp_src, const uint8_t *pp_img,
                  const uint8_t *pp_sub, const int64_t *pc_off, const int32_t *pc_src,
                  const uint8_t *pc_img, int64_t n_sel, const int32_t *sel, int parts,
                  double ew_alpha, int ew_rmax, int ew_h2max, double *acc, double *pot) {
    orc_init();
    if (gl_n == 0) orc_set_quadrature(128);
    (void)n;
    double eps2 = eps * eps;
    int64_t nb = sel ? n_sel : n_bucket;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < nb; ++q) {
        int64_t b = sel ? sel[q] : q;
        int64_t sc = bucket_cell[b];
        for (int64_t i = cell_first[sc]; i < cell_first[sc] + cell_count[sc]; ++i) {
            const double *x = pos + 3 * i;
            double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
            if (parts & 1) {
                for (int64_t e = pp_off[b]; e < pp_off[b + 1]; ++e) {
                    int64_t c = pp_src[e];
                    double sh[3];
                    orc_image_shift(pp_img[e], L, sh);
                    int64_t j0 = cell_first[c], j1 = cell_first[c] + cell_count[c];
                    if (pp_sub && pp_sub[e] > 0) {
                        j0 = cell_first[c] + pp_sub[e] - 1;
                        j1 = j0 + 1;
                    }
                    for (int64_t j = j0; j < j1; ++j) {
                        if (j == i && pp_img[e] == 0) continue;
                        double rx = x[0] - (pos[3 * j] + sh[0]);
                        double ry = x[1] - (pos[3 * j + 1] + sh[1]);
                        double rz = x[2] - (pos[3 * j + 2] + sh[2]);
                        double D = rx * rx + ry * ry + rz * rz + eps2;
                        double w = 1.0 / sqrt(D);
                        double w3 = w * w * w;
                        ax -= mass[j] * w3 * rx;
                        ay -= mass[j] * w3 * ry;
                        az -= mass[j] * w3 * rz;
                        ph -= mass[j] * w;
                    }
                }
            }
            if (parts & 2) {
                for (int64_t e = pc_off[b]; e < pc_off[b + 1]; ++e) {
                    int64_t c = pc_src[e];
                    double sh[3], X[3], o[4];
                    orc_image_shift(pc_img[e], L, sh);
                    for (int d = 0; d < 3; ++d) X[d] = com[3 * c + d] + sh[d];
                    pc_eval(mom + 32 * c, X, x, eps2, o);
                    ax += o[0];
                    ay += o[1];
                    az += o[2];
                    ph += o[3];
                }
            }
            if ((parts & 4) && L > 0.0) {
                double o[4];
                ewald_root_eval(mom, com, x, L, ew_alpha, ew_rmax, ew_h2max, o);
                ax += o[0];
                ay += o[1];
                az += o[2];
                ph += o[3];
            }
            acc[3 * i] = ax;
            acc[3 * i + 1] = ay;
            acc[3 * i + 2] = az;
            pot[i] = ph;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Direct summation: the plain definitions the tree approximates.      */
/* ------------------------------------------------------------------ */
void orc_direct_open(int64_t n, const double *pos, const double *mass, double eps, double *acc,
                     double *pot) {
    double eps2 = eps * eps;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double ax = 0, ay = 0, az = 0, ph = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double rx = pos[3 * i] - pos[3 * j], ry = pos[3 * i + 1] - pos[3 * j + 1],
                   rz = pos[3 * i + 2] - pos[3 * j + 2];
            double D = rx * rx + ry * ry + rz * rz + eps2;
            double w = 1.0 / sqrt(D);
            ax -= mass[j] * w * w * w * rx;
            ay -= mass[j] * w * w * w * ry;
            az -= mass[j] * w * w * w * rz;
            ph -= mass[j] * w;
        }
        acc[3 * i] = ax;
        acc[3 * i + 1] = ay;
        acc[3 * i + 2] = az;
        pot[i] = ph;
    }
}

/* Periodic: softened 27 nearest images (self term excluded) plus the
 * Ewald kernel psi of every pair, including the particle's own psi(0).  */
void orc_direct_periodic(int64_t n, const double *pos, const double *mass, double eps, double L,
                         double alpha, int rmax, int h2max, double *acc, double *pot) {
    orc_init();
    if (gl_n == 0) orc_set_quadrature(128);
    double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i) {
        double ax = 0, ay = 0, az = 0, ph = 0;
        for (int64_t j = 0; j < n; ++j) {
            for (int img = 0; img < 27; ++img) {
                if (j == i && img == 0) continue;
                double sh[3];
                orc_image_shift(img, L, sh);
                double rx = pos[3 * i] - pos[3 * j] - sh[0];
                double ry = pos[3 * i + 1] - pos[3 * j + 1] - sh[1];
                double rz = pos[3 * i + 2] - pos[3 * j + 2] - sh[2];
                double D = rx * rx + ry * ry + rz * rz + eps2;
                double w = 1.0 / sqrt(D);
                ax -= mass[j] * w * w * w * rx;
                ay -= mass[j] * w * w * w * ry;
                az -= mass[j] * w * w * w * rz;
                ph -= mass[j] * w;
            }
            double r[3] = {(pos[3 * i] - pos[3 * j]) / L, (pos[3 * i + 1] - pos[3 * j + 1]) / L,
                           (pos[3 * i + 2] - pos[3 * j + 2]) / L};
            double d[4];
            orc_ewald_derivs(r, alpha, rmax, h2max, 1, d);
            ph += mass[j] * d[0] / L;
            ax -= mass[j] * d[1] / (L * L);
            ay -= mass[j] * d[2] / (L * L);
            az -= mass[j] * d[3] / (L * L);
        }
        acc[3 * i] = ax;
        acc[3 * i + 1] = ay;
        acc[3 * i + 2] = az;
        pot[i] = ph;
    }
}

/* ------------------------------------------------------------------ */
/* Fast multipole form of the walk (Sec. 3.1): cell-cell (CC) and      */
/* cell-particle (CP) interactions into a local expansion of the       */
/* potential about each sink cell's centre of mass, to 5th order.      */
/*                                                                    */
/* Sink cells are visited in node-left-right order from the root, the  */
/* root's checklist holding the root seen through every image.  A sink */
/* S takes its checklist from the front (opened cells append their     */
/* children at the end).  A source C (a cell, or a particle of an      */
/* opened leaf: RO = 0, b_max = 0, a point box) seen through image n   */
/* is                                                                  */
/*   CC (cell) or CP (particle) if |X_C + nL - X_S| > 1.5 RO_S + RO_C    */
/*       and the boxes are at least 2 eps apart (the sink's opening     */
/*       radius enlarged by the paper's factor 1.5),                    */
/*   at a leaf S (a bucket: the group is the bucket):                   */
/*     PP of the single particle for a particle source,                */
/*     PC if |X_C + nL - X_S| > RO_C + b_max,S and the boxes are at     */
/*         least 2 eps apart (the rule of the bucket walk),             */
/*     PP of the whole bucket C if C is a leaf, else opened;            */
/*   at a larger S: a particle source is kept for the sink's children; */
/*     a cell source at least as large as the sink (b_max,C >= b_max,S) */
/*     is opened (a leaf into its particles, in order), a smaller one   */
/*     kept.                                                            */
/* Children of S start from the kept entries, in order.                */
/*                                                                    */
/* The local expansion of S holds L_a = d^a phi(X_S) for |a| <= 5:      */
/*   CC: L_a = sum_{k in {0,2,3,4}, k + |a| <= 5} (-1)^k/k! M_k .       */
/*             d^(k+a) G(R),  R = X_S - X_C - nL                        */
/*   CP: L_a = m d^a G(R),  R = X_S - x_p - nL                          */
/* (terms of total order above 5 are dropped); a child's expansion is   */
/* its own plus its parent's shifted to it,                            */
/*   L'_a = sum_{b >= a} L_b d^(b-a)/(b-a)!,  d = X_child - X_parent,   */
/* and a particle at x in a bucket S gets                              */
/*   phi = sum_a L_a h^a/a!,  acc = -grad phi,  h = x - X_S.            */
/* All tensors are full Cartesian tensors (3^n components of order n).  */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t idx;  /* cell, or tree-order particle */
    int img;
    int part;     /* 1: a particle (of leaf `leaf`, index `sub` in it) */
    int64_t leaf;
    int sub;
} FEnt;

typedef struct {
    FEnt *e;
    int64_t n, cap;
} FList;

static void fl_push(FList *l, FEnt x) {
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 256;
        l->e = (FEnt *)realloc(l->e, sizeof(FEnt) * (size_t)l->cap);
    }
    l->e[l->n++] = x;
}

typedef struct {
    const int64_t *cell_first;
    const int32_t *cell_count;
    const int32_t *child;
    const double *com, *bmax, *bbox, *pos;
    double theta, eps, L;
    int fill;
    /* bucket lists (per leaf, in leaf order) and cell lists */
    int64_t bucket, *pp_off, *pc_off, *cc_off;
    int32_t *pp_src, *pc_src, *cc_src;
    uint8_t *pp_img, *pp_sub, *pc_img, *cc_img;
    int64_t npp, npc, ncc;
} FWalk;

static void fmm_source(const FWalk *w, const FEnt *e, double X[3], double lo[3], double hi[3],
                       double *ro, double *bm) {
    double sh[3];
    orc_image_shift(e->img, w->L, sh);
    if (e->part) {
        for (int d = 0; d < 3; ++d) {
            X[d] = w->pos[3 * e->idx + d] + sh[d];
            lo[d] = hi[d] = X[d];
        }
        *ro = 0.0;
        *bm = 0.0;
    } else {
        for (int d = 0; d < 3; ++d) {
            X[d] = w->com[3 * e->idx + d] + sh[d];
            lo[d] = w->bbox[6 * e->idx + d] + sh[d];
            hi[d] = w->bbox[6 * e->idx + 3 + d] + sh[d];
        }
        *ro = w->bmax[e->idx] / w->theta;
        *bm = w->bmax[e->idx];
    }
}

static double box_gap(const double lo[3], const double hi[3], const double *sb) {
    double g2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double g = 0.0;
        if (lo[a] - sb[3 + a] > g) g = lo[a] - sb[3 + a];
        if (sb[a] - hi[a] > g) g = sb[a] - hi[a];
        g2 += g * g;
    }
    return sqrt(g2);
}

static void fmm_sink(FWalk *w, int64_t S, const FList *in) {
    FList q = {0, 0, 0}, keep = {0, 0, 0};
    for (int64_t i = 0; i < in->n; ++i) fl_push(&q, in->e[i]);
    const int leaf = w->child[2 * S] < 0;
    const double *XS = w->com + 3 * S, *sb = w->bbox + 6 * S;
    const double ro_s = w->bmax[S] / w->theta;
    int64_t b = -1;
    if (leaf) {
        b = w->bucket++;
        if (!w->fill) {
            w->pp_off[b + 1] = 0;
            w->pc_off[b + 1] = 0;
        }
    }
    int64_t kpp = 0, kpc = 0, kcc = 0;
    for (int64_t i = 0; i < q.n; ++i) {
        FEnt e = q.e[i];
        double X[3], lo[3], hi[3], ro, bm;
        fmm_source(w, &e, X, lo, hi, &ro, &bm);
        double dx = X[0] - XS[0], dy = X[1] - XS[1], dz = X[2] - XS[2];
        double d = sqrt(dx * dx + dy * dy + dz * dz);
        double gap = box_gap(lo, hi, sb);
        if (d > 1.5 * ro_s + ro && gap >= 2.0 * w->eps) {
            if (w->fill) {
                int64_t k = w->cc_off[S] + kcc;
                w->cc_src[k] = e.part ? (int32_t)~e.idx : (int32_t)e.idx;
                w->cc_img[k] = (uint8_t)e.img;
            }
            ++kcc;
        } else if (leaf) {
            if (e.part) {
                if (w->fill) {
                    int64_t k = w->pp_off[b] + kpp;
                    w->pp_src[k] = (int32_t)e.leaf;
                    w->pp_img[k] = (uint8_t)e.img;
                    w->pp_sub[k] = (uint8_t)(e.sub + 1);
                }
                ++kpp;
            } else if (d > ro + w->bmax[S] && gap >= 2.0 * w->eps) {
                if (w->fill) {
                    int64_t k = w->pc_off[b] + kpc;
                    w->pc_src[k] = (int32_t)e.idx;
                    w->pc_img[k] = (uint8_t)e.img;
                }
                ++kpc;
            } else if (w->child[2 * e.idx] < 0) {
                if (w->fill) {
                    int64_t k = w->pp_off[b] + kpp;
                    w->pp_src[k] = (int32_t)e.idx;
                    w->pp_img[k] = (uint8_t)e.img;
                    w->pp_sub[k] = 0;
                }
                ++kpp;
            } else {
                for (int s = 0; s < 2; ++s) {
                    FEnt c = {w->child[2 * e.idx + s], e.img, 0, -1, 0};
                    fl_push(&q, c);
                }
            }
        } else if (e.part) {
            fl_push(&keep, e);
        } else if (bm >= w->bmax[S]) {
            if (w->child[2 * e.idx] < 0) {
                for (int s = 0; s < w->cell_count[e.idx]; ++s) {
                    FEnt p = {w->cell_first[e.idx] + s, e.img, 1, e.idx, s};
                    fl_push(&q, p);
                }
            } else {
                for (int s = 0; s < 2; ++s) {
                    FEnt c = {w->child[2 * e.idx + s], e.img, 0, -1, 0};
                    fl_push(&q, c);
                }
            }
        } else {
            fl_push(&keep, e);
        }
    }
    free(q.e);
    if (!w->fill) {
        w->cc_off[S + 1] = kcc;
        if (leaf) {
            w->pp_off[b + 1] = kpp;
            w->pc_off[b + 1] = kpc;
        }
    }
    if (!leaf) {
        fmm_sink(w, w->child[2 * S], &keep);
        fmm_sink(w, w->child[2 * S + 1], &keep);
    }
    free(keep.e);
}

/* Two passes, as the bucket walk: fill = 0 writes per-bucket PP / PC
 * lengths into pp_off[1..], pc_off[1..] and per-cell CC/CP lengths into
 * cc_off[1..], then turns them into offsets; fill = 1 writes the entries
 * (PP: source leaf, image, sub = 0 for the whole leaf or k + 1 for its
 * k-th particle; CC/CP: source cell, or ~p for tree-order particle p). */
void orc_fmm_walk(int64_t n_cell, const int64_t *cell_first, const int32_t *cell_count,
                  const int32_t *child, const double *com, const double *bmax, const double *bbox,
                  const double *pos, double theta, double eps, double L, int n_img, int fill,
                  int64_t *pp_off, int32_t *pp_src, uint8_t *pp_img, uint8_t *pp_sub,
                  int64_t *pc_off, int32_t *pc_src, uint8_t *pc_img, int64_t *cc_off,
                  int32_t *cc_src, uint8_t *cc_img) {
    FWalk w = {cell_first, cell_count, child, com, bmax, bbox, pos, theta, eps, L, fill, 0,
               pp_off, pc_off, cc_off, pp_src, pc_src, cc_src, pp_img, pp_sub, pc_img, cc_img,
               0, 0, 0};
    FList root = {0, 0, 0};
    for (int i = 0; i < n_img; ++i) {
        FEnt e = {0, i, 0, -1, 0};
        fl_push(&root, e);
    }
    if (!fill) {
        pp_off[0] = pc_off[0] = cc_off[0] = 0;
    }
    fmm_sink(&w, 0, &root);
    free(root.e);
    if (!fill) {
        for (int64_t b = 0; b < w.bucket; ++b) {
            pp_off[b + 1] += pp_off[b];
            pc_off[b + 1] += pc_off[b];
        }
        for (int64_t c = 0; c < n_cell; ++c) cc_off[c + 1] += cc_off[c];
    }
}

#define FMM_P 5
/* offsets of the order-n blocks in a 364-value full local expansion */
static const int LOFF[FMM_P + 2] = {0, 1, 4, 13, 40, 121, 364};

/* Derivative tensors of G = -g through order 5 at R. */
static void green_tensors(const double R[3], double eps2, double *T[]) {
    double a[ORC_KMAX + 1];
    plummer_radial(R[0] * R[0] + R[1] * R[1] + R[2] * R[2], eps2, FMM_P, a);
    radial_tensors(R, a, FMM_P, T);
    for (int n = 0; n <= FMM_P; ++n)
        for (int f = 0; f < POW3[n]; ++f) T[n][f] = -T[n][f];
}

/* Add the CC or CP contribution of one entry to the expansion Lc (364). */
static void fmm_m2l(const double *mom, double mass, int part, const double XS[3],
                    const double XC[3], double eps2, double *Lc) {
    static const double fact[6] = {1, 1, 2, 6, 24, 120};
    double R[3] = {XS[0] - XC[0], XS[1] - XC[1], XS[2] - XC[2]};
    double T0[1], T1[3], T2[9], T3[27], T4[81], T5[243];
    double *T[6] = {T0, T1, T2, T3, T4, T5};
    green_tensors(R, eps2, T);
    if (part) {
        for (int n = 0; n <= FMM_P; ++n)
            for (int f = 0; f < POW3[n]; ++f) Lc[LOFF[n] + f] += mass * T[n][f];
        return;
    }
    double M2[9], M3[27], M4[81];
    unpack_moments(mom, M2, M3, M4);
    double M0[1] = {mom[0]};
    const double *Mk[5] = {M0, NULL, M2, M3, M4};
    for (int n = 0; n <= FMM_P; ++n)
        for (int k = 0; k <= 4 && k + n <= FMM_P; ++k) {
            if (k == 1) continue;
            double c = ((k & 1) ? -1.0 : 1.0) / fact[k];
            for (int f = 0; f < POW3[n]; ++f) {
                double s = 0.0;
                for (int j = 0; j < POW3[k]; ++j) s += Mk[k][j] * T[k + n][j * POW3[n] + f];
                Lc[LOFF[n] + f] += c * s;
            }
        }
}

/* L' = L shifted from its centre by d (both 364 values). */
static void fmm_l2l(const double *L, const double d[3], double *out) {
    static const double fact[6] = {1, 1, 2, 6, 24, 120};
    for (int n = 0; n <= FMM_P; ++n)
        for (int f = 0; f < POW3[n]; ++f) {
            double s = 0.0;
            for (int m = n; m <= FMM_P; ++m) {
                int k = m - n;
                for (int j = 0; j < POW3[k]; ++j) {
                    int ax[ORC_KMAX];
                    digits(k, j, ax);
                    double dp = 1.0;
                    for (int q = 0; q < k; ++q) dp *= d[ax[q]];
                    s += L[LOFF[m] + f * POW3[k] + j] * dp / fact[k];
                }
            }
            out[LOFF[n] + f] = s;
        }
}

/* Potential and acceleration at offset h from the expansion's centre. */
static void fmm_l2p(const double *L, const double h[3], double out[4]) {
    static const double fact[6] = {1, 1, 2, 6, 24, 120};
    double phi = 0.0, g[3] = {0, 0, 0};
    for (int n = 0; n <= FMM_P; ++n)
        for (int f = 0; f < POW3[n]; ++f) {
            int ax[ORC_KMAX];
            digits(n, f, ax);
            double hp = 1.0;
            for (int q = 0; q < n; ++q) hp *= h[ax[q]];
            phi += L[LOFF[n] + f] * hp / fact[n];
            if (n >= 1) {
                /* d/dh_a of the order-n term: the first index is a, the
                 * rest contracted with h (symmetric tensor) */
                double hq = 1.0;
                for (int q = 1; q < n; ++q) hq *= h[ax[q]];
                g[ax[0]] += L[LOFF[n] + f] * hq / fact[n - 1];
            }
        }
    out[0] = -g[0];
    out[1] = -g[1];
    out[2] = -g[2];
    out[3] = phi;
}

/* Local expansions of every cell (364 values each, about its centre of
 * mass): own CC/CP contributions, then shifted down from the root in
 * node-left-right order (parents come before their children). */
void orc_fmm_local(int64_t n_cell, const int32_t *child, const double *com, const double *mom,
                   const double *pos, const double *mass, double eps, double L,
                   const int64_t *cc_off, const int32_t *cc_src, const uint8_t *cc_img,
                   double *local) {
    orc_init();
    double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < n_cell; ++c) {
        double *Lc = local + 364 * c;
        for (int f = 0; f < 364; ++f) Lc[f] = 0.0;
        for (int64_t e = cc_off[c]; e < cc_off[c + 1]; ++e) {
            double sh[3], X[3];
            orc_image_shift(cc_img[e], L, sh);
            int32_t s = cc_src[e];
            if (s < 0) {
                int64_t p = ~(int64_t)s;
                for (int d = 0; d < 3; ++d) X[d] = pos[3 * p + d] + sh[d];
                fmm_m2l(NULL, mass[p], 1, com + 3 * c, X, eps2, Lc);
            } else {
                for (int d = 0; d < 3; ++d) X[d] = com[3 * s + d] + sh[d];
                fmm_m2l(mom + 32 * s, 0.0, 0, com + 3 * c, X, eps2, Lc);
            }
        }
    }
    double *tmp = (double *)malloc(sizeof(double) * 364);
    for (int64_t p = 0; p < n_cell; ++p) {
        if (child[2 * p] < 0) continue;
        for (int s = 0; s < 2; ++s) {
            int64_t c = child[2 * p + s];
            double d[3] = {com[3 * c] - com[3 * p], com[3 * c + 1] - com[3 * p + 1],
                           com[3 * c + 2] - com[3 * p + 2]};
            fmm_l2l(local + 364 * p, d, tmp);
            for (int f = 0; f < 364; ++f) local[364 * c + f] += tmp[f];
        }
    }
    free(tmp);
}

/* The local expansion of each particle's bucket evaluated at it (L2P),
 * written to acc / pot of the particles of the selected buckets. */
void orc_fmm_l2p(int64_t n_bucket, const int32_t *bucket_cell, const int64_t *cell_first,
                 const int32_t *cell_count, const double *com, const double *pos,
                 const double *local, double *acc, double *pot) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t b = 0; b < n_bucket; ++b) {
        int64_t c = bucket_cell[b];
        for (int64_t i = cell_first[c]; i < cell_first[c] + cell_count[c]; ++i) {
            double h[3] = {pos[3 * i] - com[3 * c], pos[3 * i + 1] - com[3 * c + 1],
                           pos[3 * i + 2] - com[3 * c + 2]};
            double o[4];
            fmm_l2p(local + 364 * c, h, o);
            acc[3 * i] = o[0];
            acc[3 * i + 1] = o[1];
            acc[3 * i + 2] = o[2];
            pot[i] = o[3];
        }
    }
}

/* The exposed parts of the expansion machinery, for the pins: the
 * expansion of one source (cell moments or a particle) about X_S, its
 * shift, and its evaluation. */
void orc_fmm_m2l_point(const double *mom32, double mass, int part, const double XS[3],
                       const double XC[3], double eps, double *L364) {
    orc_init();
    for (int f = 0; f < 364; ++f) L364[f] = 0.0;
    fmm_m2l(mom32, mass, part, XS, XC, eps * eps, L364);
}

void orc_fmm_l2l_point(const double *L364, const double d[3], double *out364) {
    orc_init();
    fmm_l2l(L364, d, out364);
}

void orc_fmm_l2p_point(const double *L364, const double h[3], double out[4]) {
    orc_init();
    fmm_l2p(L364, h, out);
}
