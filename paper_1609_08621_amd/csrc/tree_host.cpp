// Host-side input preparation for the mgrav device path: the binary tree
// and the bucket-sink checklist walk of arXiv:1609.08621, Sec. 3.1.
//
// The paper keeps tree building and walking on the CPU and sends the
// resulting PP/PC interaction lists to the GPU (Sec. 3.3); this file is
// that CPU side.  The produced arrays are the tree/list inputs that
// mgrav_bind() consumes (see include/mgrav.h for their layout).
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mgrav.h"
#include "internal.h"

namespace {

// Symmetric tensor components of order 2, 3, 4 in the packed order of the
// ABI (non-decreasing axis tuples, lexicographic).
struct Packed {
    int k;
    int ax[4];
};

const Packed kPacked[31] = {
    {2, {0, 0}}, {2, {0, 1}}, {2, {0, 2}}, {2, {1, 1}}, {2, {1, 2}}, {2, {2, 2}},
    {3, {0, 0, 0}}, {3, {0, 0, 1}}, {3, {0, 0, 2}}, {3, {0, 1, 1}}, {3, {0, 1, 2}},
    {3, {0, 2, 2}}, {3, {1, 1, 1}}, {3, {1, 1, 2}}, {3, {1, 2, 2}}, {3, {2, 2, 2}},
    {4, {0, 0, 0, 0}}, {4, {0, 0, 0, 1}}, {4, {0, 0, 0, 2}}, {4, {0, 0, 1, 1}},
    {4, {0, 0, 1, 2}}, {4, {0, 0, 2, 2}}, {4, {0, 1, 1, 1}}, {4, {0, 1, 1, 2}},
    {4, {0, 1, 2, 2}}, {4, {0, 2, 2, 2}}, {4, {1, 1, 1, 1}}, {4, {1, 1, 1, 2}},
    {4, {1, 1, 2, 2}}, {4, {1, 2, 2, 2}}, {4, {2, 2, 2, 2}},
};

struct Box {
    double lo[3], hi[3];
};

struct Pending {
    int64_t parent;  // -1 for the root
    int side;        // 0 = lower child, 1 = upper child
    int64_t first, count;
    Box box;         // geometric box
    int depth;       // halvings along the path from the root
};

// Stable split of idx[first, first+count) by coordinate `axis` < mid.
int64_t stable_split(const double* pos, int64_t* idx, int64_t* scratch, int64_t first,
                     int64_t count, int axis, double mid) {
    int64_t lo = 0, hi = 0;
    int64_t* seg = idx + first;
    for (int64_t i = 0; i < count; ++i) {
        const int64_t p = seg[i];
        if (pos[3 * p + axis] < mid)
            seg[lo++] = p;
        else
            scratch[hi++] = p;
    }
    std::memcpy(seg + lo, scratch, sizeof(int64_t) * hi);
    return lo;
}

}  // namespace

extern "C" mgrav_status mgrav_tree_build_host(int64_t n, const double* pos, const double* mass,
                                              double L, int bucket, int64_t cap, int64_t* perm,
                                              int64_t* cell_first, int32_t* cell_count,
                                              int32_t* child, double* com, double* bmax,
                                              double* bbox, double* mom, int32_t* bucket_cell,
                                              int64_t* n_cell_out, int64_t* n_bucket_out) {
    using mgrav_internal::set_host_error;
    if (n < 1 || !pos || !mass || !perm || !cell_first || !cell_count || !child || !com ||
        !bmax || !bbox || !mom || !bucket_cell || !n_cell_out || !n_bucket_out)
        return set_host_error(MGRAV_ERR_INVALID_ARG, "tree_build: null pointer or n < 1");
    if (bucket < 1 || bucket > MGRAV_MAX_BUCKET)
        return set_host_error(MGRAV_ERR_INVALID_ARG, "tree_build: bucket outside 1..16");
    if (!(L >= 0.0) || !std::isfinite(L))
        return set_host_error(MGRAV_ERR_INVALID_ARG, "tree_build: bad box size");
    for (int64_t i = 0; i < n; ++i) {
        if (!(mass[i] > 0.0) || !std::isfinite(mass[i]))
            return set_host_error(MGRAV_ERR_INVALID_ARG, "tree_build: mass must be > 0");
        for (int d = 0; d < 3; ++d) {
            const double x = pos[3 * i + d];
            if (!std::isfinite(x))
                return set_host_error(MGRAV_ERR_INVALID_ARG, "tree_build: non-finite position");
            if (L > 0.0 && (x < 0.0 || x >= L))
                return set_host_error(MGRAV_ERR_INVALID_ARG,
                                      "tree_build: periodic position outside [0, L)");
        }
    }

    Box root;
    if (L > 0.0) {
        for (int d = 0; d < 3; ++d) {
            root.lo[d] = 0.0;
            root.hi[d] = L;
        }
    } else {
        for (int d = 0; d < 3; ++d) {
            root.lo[d] = pos[d];
            root.hi[d] = pos[d];
        }
        for (int64_t i = 1; i < n; ++i)
            for (int d = 0; d < 3; ++d) {
                root.lo[d] = std::min(root.lo[d], pos[3 * i + d]);
                root.hi[d] = std::max(root.hi[d], pos[3 * i + d]);
            }
    }

    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    std::vector<int64_t> scratch(n);

    // Depth-first construction with an explicit stack.  A cell gets its
    // id when it is popped and the lower child is pushed last, so ids come
    // out in node-left-right order.
    int64_t ncell = 0;
    std::vector<Pending> stack;
    stack.push_back({-1, 0, 0, n, root, 0});
    while (!stack.empty()) {
        const Pending c = stack.back();
        stack.pop_back();
        const int64_t id = ncell++;
        if (id >= cap)
            return set_host_error(MGRAV_ERR_INVALID_ARG, "tree_build: cell capacity too small");
        if (c.parent >= 0) child[2 * c.parent + c.side] = static_cast<int32_t>(id);
        cell_first[id] = c.first;
        cell_count[id] = static_cast<int32_t>(c.count);
        child[2 * id] = -1;
        child[2 * id + 1] = -1;
        if (c.count <= bucket) continue;

        Box b = c.box;
        int depth = c.depth;
        int64_t nlow = 0;
        Box lower = b, upper = b;
        for (;;) {
            if (depth >= 64) {  // coincident points: halve by index
                nlow = (c.count + 1) / 2;
                lower = b;
                upper = b;
                break;
            }
            int axis = 0;
            for (int d = 1; d < 3; ++d)
                if (b.hi[d] - b.lo[d] > b.hi[axis] - b.lo[axis]) axis = d;
            const double mid = 0.5 * (b.lo[axis] + b.hi[axis]);
            nlow = stable_split(pos, perm, scratch.data(), c.first, c.count, axis, mid);
            ++depth;
            if (nlow == 0) {
                b.lo[axis] = mid;  // empty lower half: shrink and bisect again
            } else if (nlow == c.count) {
                b.hi[axis] = mid;  // empty upper half
            } else {
                lower = b;
                upper = b;
                lower.hi[axis] = mid;
                upper.lo[axis] = mid;
                break;
            }
        }
        stack.push_back({id, 1, c.first + nlow, c.count - nlow, upper, depth});
        stack.push_back({id, 0, c.first, nlow, lower, depth});
    }
    const int64_t n_cell = ncell;

    // Per-cell centre of mass, bounding box, b_max and packed moments,
    // each from the cell's own particles in tree order.
    std::vector<int32_t> leaf_flag(n_cell);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < n_cell; ++c) {
        const int64_t f = cell_first[c], k = cell_count[c];
        double M = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t i = f; i < f + k; ++i) {
            const int64_t p = perm[i];
            const double m = mass[p];
            const double* x = pos + 3 * p;
            M += m;
            mx += m * x[0];
            my += m * x[1];
            mz += m * x[2];
            for (int d = 0; d < 3; ++d) {
                lo[d] = x[d] < lo[d] ? x[d] : lo[d];
                hi[d] = x[d] > hi[d] ? x[d] : hi[d];
            }
        }
        const double X[3] = {mx / M, my / M, mz / M};
        double r2max = 0.0;
        double acc[31] = {0};
        for (int64_t i = f; i < f + k; ++i) {
            const int64_t p = perm[i];
            const double m = mass[p];
            const double s[3] = {pos[3 * p] - X[0], pos[3 * p + 1] - X[1], pos[3 * p + 2] - X[2]};
            const double r2 = s[0] * s[0] + s[1] * s[1] + s[2] * s[2];
            r2max = r2 > r2max ? r2 : r2max;
            for (int q = 0; q < 31; ++q) {
                double t = m;
                for (int j = 0; j < kPacked[q].k; ++j) t *= s[kPacked[q].ax[j]];
                acc[q] += t;
            }
        }
        for (int d = 0; d < 3; ++d) {
            com[3 * c + d] = X[d];
            bbox[6 * c + d] = lo[d];
            bbox[6 * c + 3 + d] = hi[d];
        }
        bmax[c] = std::sqrt(r2max);
        mom[32 * c] = M;
        for (int q = 0; q < 31; ++q) mom[32 * c + 1 + q] = acc[q];
        leaf_flag[c] = child[2 * c] < 0;
    }
    int64_t nb = 0;
    for (int64_t c = 0; c < n_cell; ++c)
        if (leaf_flag[c]) bucket_cell[nb++] = static_cast<int32_t>(c);
    *n_cell_out = n_cell;
    *n_bucket_out = nb;
    return MGRAV_OK;
}

namespace {

struct WalkArgs {
    const int32_t* child;
    const double* com;
    const double* bmax;
    const double* bbox;
    double theta, eps, L;
    int n_images;
};

void image_offset(int id, double L, double out[3]) {
    static const int8_t kShift[27][3] = {
        {0, 0, 0},    {-1, -1, -1}, {-1, -1, 0}, {-1, -1, 1}, {-1, 0, -1}, {-1, 0, 0},
        {-1, 0, 1},   {-1, 1, -1},  {-1, 1, 0},  {-1, 1, 1},  {0, -1, -1}, {0, -1, 0},
        {0, -1, 1},   {0, 0, -1},   {0, 0, 1},   {0, 1, -1},  {0, 1, 0},   {0, 1, 1},
        {1, -1, -1},  {1, -1, 0},   {1, -1, 1},  {1, 0, -1},  {1, 0, 0},   {1, 0, 1},
        {1, 1, -1},   {1, 1, 0},    {1, 1, 1}};
    for (int d = 0; d < 3; ++d) out[d] = kShift[id][d] * L;
}

// The acceptance test of a source cell for the whole sink bucket: beyond
// the source's opening radius plus the sink's own extent, and bounding
// boxes at least two softening lengths apart.
bool accepted(const WalkArgs& w, int64_t src, int img, int64_t sink) {
    double sh[3];
    image_offset(img, w.L, sh);
    const double dx = w.com[3 * src + 0] + sh[0] - w.com[3 * sink + 0];
    const double dy = w.com[3 * src + 1] + sh[1] - w.com[3 * sink + 1];
    const double dz = w.com[3 * src + 2] + sh[2] - w.com[3 * sink + 2];
    const double dist = std::sqrt(dx * dx + dy * dy + dz * dz);
    if (!(dist > w.bmax[src] / w.theta + w.bmax[sink])) return false;
    double gap2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double src_lo = w.bbox[6 * src + a] + sh[a];
        const double src_hi = w.bbox[6 * src + 3 + a] + sh[a];
        double g = 0.0;
        g = std::max(g, src_lo - w.bbox[6 * sink + 3 + a]);
        g = std::max(g, w.bbox[6 * sink + a] - src_hi);
        gap2 += g * g;
    }
    return std::sqrt(gap2) >= 2.0 * w.eps;
}

// Ring-buffer checklist; returns list lengths and optionally fills them.
struct Checklist {
    std::vector<int32_t> cell;
    std::vector<uint8_t> img;
    size_t head = 0, tail = 0, mask = 0;
    void reset(size_t cap) {
        size_t c = 64;
        while (c < cap) c <<= 1;
        cell.assign(c, 0);
        img.assign(c, 0);
        mask = c - 1;
        head = tail = 0;
    }
    bool empty() const { return head == tail; }
    void push(int32_t c, uint8_t i) {
        if (tail - head == cell.size()) grow();
        cell[tail & mask] = c;
        img[tail & mask] = i;
        ++tail;
    }
    void grow() {
        std::vector<int32_t> nc(cell.size() * 2);
        std::vector<uint8_t> ni(cell.size() * 2);
        size_t k = 0;
        for (size_t i = head; i < tail; ++i, ++k) {
            nc[k] = cell[i & mask];
            ni[k] = img[i & mask];
        }
        cell.swap(nc);
        img.swap(ni);
        mask = cell.size() - 1;
        head = 0;
        tail = k;
    }
};

void walk(const WalkArgs& w, int64_t sink, Checklist& q, int64_t* npp, int64_t* npc,
          int32_t* pp_src, uint8_t* pp_img, int32_t* pc_src, uint8_t* pc_img) {
    q.head = q.tail = 0;
    for (int i = 0; i < w.n_images; ++i) q.push(0, static_cast<uint8_t>(i));
    int64_t kpp = 0, kpc = 0;
    while (!q.empty()) {
        const int32_t c = q.cell[q.head & q.mask];
        const uint8_t im = q.img[q.head & q.mask];
        ++q.head;
        if (accepted(w, c, im, sink)) {
            if (pc_src) {
                pc_src[kpc] = c;
                pc_img[kpc] = im;
            }
            ++kpc;
        } else if (w.child[2 * c] < 0) {
            if (pp_src) {
                pp_src[kpp] = c;
                pp_img[kpp] = im;
            }
            ++kpp;
        } else {
            q.push(w.child[2 * c], im);
            q.push(w.child[2 * c + 1], im);
        }
    }
    *npp = kpp;
    *npc = kpc;
}

mgrav_status check_walk_args(double theta, double eps, double L, int n_images) {
    using mgrav_internal::set_host_error;
    if (!(theta > 0.0)) return set_host_error(MGRAV_ERR_INVALID_ARG, "lists: theta must be > 0");
    if (!(eps >= 0.0)) return set_host_error(MGRAV_ERR_INVALID_ARG, "lists: eps must be >= 0");
    if (n_images != 1 && n_images != 27)
        return set_host_error(MGRAV_ERR_INVALID_ARG, "lists: n_images must be 1 or 27");
    if (n_images == 27 && !(L > 0.0))
        return set_host_error(MGRAV_ERR_INVALID_ARG, "lists: 27 images need box_L > 0");
    return MGRAV_OK;
}

}  // namespace

extern "C" mgrav_status mgrav_lists_count_host(int64_t n_bucket, const int32_t* bucket_cell,
                                               const int32_t* child, const double* com,
                                               const double* bmax, const double* bbox,
                                               double theta, double eps, double L,
                                               int n_images, int64_t* pp_off, int64_t* pc_off) {
    mgrav_status st = check_walk_args(theta, eps, L, n_images);
    if (st != MGRAV_OK) return st;
    if (n_bucket < 1 || !bucket_cell || !child || !com || !bmax || !bbox || !pp_off || !pc_off)
        return mgrav_internal::set_host_error(MGRAV_ERR_INVALID_ARG, "lists: null pointer");
    const WalkArgs w{child, com, bmax, bbox, theta, eps, L, n_images};
    pp_off[0] = 0;
    pc_off[0] = 0;
#pragma omp parallel
    {
        Checklist q;
        q.reset(1024);
#pragma omp for schedule(dynamic, 32)
        for (int64_t b = 0; b < n_bucket; ++b) {
            int64_t a = 0, c = 0;
            walk(w, bucket_cell[b], q, &a, &c, nullptr, nullptr, nullptr, nullptr);
            pp_off[b + 1] = a;
            pc_off[b + 1] = c;
        }
    }
    for (int64_t b = 0; b < n_bucket; ++b) {
        pp_off[b + 1] += pp_off[b];
        pc_off[b + 1] += pc_off[b];
    }
    return MGRAV_OK;
}

extern "C" mgrav_status mgrav_lists_fill_host(int64_t n_bucket, const int32_t* bucket_cell,
                                              const int32_t* child, const double* com,
                                              const double* bmax, const double* bbox,
                                              double theta, double eps, double L, int n_images,
                                              const int64_t* pp_off, const int64_t* pc_off,
                                              int32_t* pp_src, uint8_t* pp_img, int32_t* pc_src,
                                              uint8_t* pc_img) {
    mgrav_status st = check_walk_args(theta, eps, L, n_images);
    if (st != MGRAV_OK) return st;
    if (n_bucket < 1 || !bucket_cell || !child || !com || !bmax || !bbox || !pp_off || !pc_off ||
        (!pp_src && pp_off[n_bucket] > 0) || (!pc_src && pc_off[n_bucket] > 0))
        return mgrav_internal::set_host_error(MGRAV_ERR_INVALID_ARG, "lists: null pointer");
    const WalkArgs w{child, com, bmax, bbox, theta, eps, L, n_images};
#pragma omp parallel
    {
        Checklist q;
        q.reset(1024);
#pragma omp for schedule(dynamic, 32)
        for (int64_t b = 0; b < n_bucket; ++b) {
            int64_t a = 0, c = 0;
            walk(w, bucket_cell[b], q, &a, &c, pp_src + pp_off[b], pp_img + pp_off[b],
                 pc_src + pc_off[b], pc_img + pc_off[b]);
        }
    }
    return MGRAV_OK;
}

// ---------------------------------------------------------------------
// Fast-multipole walk (Sec. 3.1): sink cells from the root in
// node-left-right order, each with the checklist its parent kept.  A
// source (a cell, or a particle of an opened leaf: opening radius 0, a
// point box) seen through an image is a CC / CP interaction of the sink
// when it lies beyond 1.5 RO_sink + RO_source with the boxes at least
// 2 eps apart; at a bucket sink the rest becomes PP (a particle, or a
// whole leaf) or PC (the bucket walk's rule) or is opened; at a larger sink
// a particle or a source smaller than the sink stays for the children,
// a source at least as large is opened (a leaf into its particles).
// ---------------------------------------------------------------------
namespace {

struct FEntry {
    int32_t idx;   // cell, or tree-order particle
    uint8_t img;
    uint8_t part;  // 1: particle `idx`, particle `sub` of leaf `leaf`
    uint8_t sub;
    int32_t leaf;
};

struct FmmArgs {
    const int64_t* cell_first;
    const int32_t* cell_count;
    const int32_t* child;
    const double *com, *bmax, *bbox, *pos;
    double theta, eps, L;
    const int64_t* leaf_no;  // bucket number of each leaf (-1 otherwise)
    bool fill;
    int64_t *pp_off, *pc_off, *cc_off;
    int32_t *pp_src, *pc_src, *cc_src;
    uint8_t *pp_img, *pp_sub, *pc_img, *cc_img;
};

// The sink S with checklist `in`; the children's checklist goes to `keep`.
void fmm_visit(const FmmArgs& w, int64_t S, const std::vector<FEntry>& in,
               std::vector<FEntry>& keep) {
    std::vector<FEntry> q(in);
    keep.clear();
    const bool leaf = w.child[2 * S] < 0;
    const double* XS = w.com + 3 * S;
    const double* sb = w.bbox + 6 * S;
    const double ro_s = w.bmax[S] / w.theta;
    const int64_t b = leaf ? w.leaf_no[S] : -1;
    int64_t kpp = 0, kpc = 0, kcc = 0;
    for (size_t i = 0; i < q.size(); ++i) {
        const FEntry e = q[i];
        double sh[3];
        image_offset(e.img, w.L, sh);
        double X[3], lo[3], hi[3], ro, bm;
        if (e.part) {
            for (int d = 0; d < 3; ++d) {
                X[d] = w.pos[3 * int64_t(e.idx) + d] + sh[d];
                lo[d] = hi[d] = X[d];
            }
            ro = bm = 0.0;
        } else {
            for (int d = 0; d < 3; ++d) {
                X[d] = w.com[3 * int64_t(e.idx) + d] + sh[d];
                lo[d] = w.bbox[6 * int64_t(e.idx) + d] + sh[d];
                hi[d] = w.bbox[6 * int64_t(e.idx) + 3 + d] + sh[d];
            }
            bm = w.bmax[e.idx];
            ro = bm / w.theta;
        }
        const double dx = X[0] - XS[0], dy = X[1] - XS[1], dz = X[2] - XS[2];
        const double dist = std::sqrt(dx * dx + dy * dy + dz * dz);
        double g2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double g = 0.0;
            if (lo[a] - sb[3 + a] > g) g = lo[a] - sb[3 + a];
            if (sb[a] - hi[a] > g) g = sb[a] - hi[a];
            g2 += g * g;
        }
        const bool apart = std::sqrt(g2) >= 2.0 * w.eps;
        if (dist > 1.5 * ro_s + ro && apart) {
            if (w.fill) {
                const int64_t k = w.cc_off[S] + kcc;
                w.cc_src[k] = e.part ? ~e.idx : e.idx;
                w.cc_img[k] = e.img;
            }
            ++kcc;
        } else if (leaf) {
            if (e.part || (!(dist > ro + w.bmax[S] && apart) && w.child[2 * e.idx] < 0)) {
                if (w.fill) {
                    const int64_t k = w.pp_off[b] + kpp;
                    w.pp_src[k] = e.part ? e.leaf : e.idx;
                    w.pp_img[k] = e.img;
                    w.pp_sub[k] = e.part ? uint8_t(e.sub + 1) : uint8_t(0);
                }
                ++kpp;
            } else if (dist > ro + w.bmax[S] && apart) {
                if (w.fill) {
                    const int64_t k = w.pc_off[b] + kpc;
                    w.pc_src[k] = e.idx;
                    w.pc_img[k] = e.img;
                }
                ++kpc;
            } else {
                q.push_back(FEntry{w.child[2 * e.idx], e.img, 0, 0, -1});
                q.push_back(FEntry{w.child[2 * e.idx + 1], e.img, 0, 0, -1});
            }
        } else if (!e.part && bm >= w.bmax[S]) {
            if (w.child[2 * e.idx] < 0) {
                const int32_t f = int32_t(w.cell_first[e.idx]);
                for (int s = 0; s < w.cell_count[e.idx]; ++s)
                    q.push_back(FEntry{f + s, e.img, 1, uint8_t(s), e.idx});
            } else {
                q.push_back(FEntry{w.child[2 * e.idx], e.img, 0, 0, -1});
                q.push_back(FEntry{w.child[2 * e.idx + 1], e.img, 0, 0, -1});
            }
        } else {
            keep.push_back(e);
        }
    }
    if (!w.fill) {
        w.cc_off[S + 1] = kcc;
        if (leaf) {
            w.pp_off[b + 1] = kpp;
            w.pc_off[b + 1] = kpc;
        }
    }
}

// Depth-first over the sinks with an explicit stack; subtrees of more than
// `task_cells` cells become OpenMP tasks (each writes only its own cells'
// and buckets' entries).
void fmm_subtree(const FmmArgs& w, int64_t root, std::vector<FEntry> list) {
    struct Frame {
        int64_t S;
        std::vector<FEntry> list;
    };
    std::vector<Frame> stack;
    stack.push_back(Frame{root, std::move(list)});
    std::vector<FEntry> keep;
    while (!stack.empty()) {
        Frame f = std::move(stack.back());
        stack.pop_back();
        fmm_visit(w, f.S, f.list, keep);
        if (w.child[2 * f.S] < 0) continue;
        const int64_t c0 = w.child[2 * f.S], c1 = w.child[2 * f.S + 1];
        if (w.cell_count[f.S] > 65536) {
#pragma omp task firstprivate(c1, keep) shared(w)
            fmm_subtree(w, c1, keep);
#pragma omp task firstprivate(c0, keep) shared(w)
            fmm_subtree(w, c0, keep);
        } else {
            stack.push_back(Frame{c1, keep});
            stack.push_back(Frame{c0, keep});
        }
    }
}

mgrav_status fmm_run(FmmArgs& w, int64_t n_cell, int n_images) {
    std::vector<int64_t> leaf_no(n_cell, -1);
    int64_t nb = 0;
    for (int64_t c = 0; c < n_cell; ++c)
        if (w.child[2 * c] < 0) leaf_no[c] = nb++;
    w.leaf_no = leaf_no.data();
    std::vector<FEntry> root;
    for (int i = 0; i < n_images; ++i) root.push_back(FEntry{0, uint8_t(i), 0, 0, -1});
    if (!w.fill) {
        w.pp_off[0] = w.pc_off[0] = w.cc_off[0] = 0;
    }
#pragma omp parallel
#pragma omp single
    fmm_subtree(w, 0, root);
    if (!w.fill) {
        for (int64_t b = 0; b < nb; ++b) {
            w.pp_off[b + 1] += w.pp_off[b];
            w.pc_off[b + 1] += w.pc_off[b];
        }
        for (int64_t c = 0; c < n_cell; ++c) w.cc_off[c + 1] += w.cc_off[c];
    }
    return MGRAV_OK;
}

}  // namespace

extern "C" mgrav_status mgrav_fmm_lists_count_host(
    int64_t n_cell, const int64_t* cell_first, const int32_t* cell_count, const int32_t* child,
    const double* com, const double* bmax, const double* bbox, const double* pos, double theta,
    double eps, double L, int n_images, int64_t* pp_off, int64_t* pc_off, int64_t* cc_off) {
    mgrav_status st = check_walk_args(theta, eps, L, n_images);
    if (st != MGRAV_OK) return st;
    if (n_cell < 1 || !cell_first || !cell_count || !child || !com || !bmax || !bbox || !pos ||
        !pp_off || !pc_off || !cc_off)
        return mgrav_internal::set_host_error(MGRAV_ERR_INVALID_ARG, "fmm lists: null pointer");
    FmmArgs w{cell_first, cell_count, child, com, bmax, bbox, pos, theta, eps, L, nullptr, false,
              pp_off, pc_off, cc_off, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
              nullptr};
    return fmm_run(w, n_cell, n_images);
}

extern "C" mgrav_status mgrav_fmm_lists_fill_host(
    int64_t n_cell, const int64_t* cell_first, const int32_t* cell_count, const int32_t* child,
    const double* com, const double* bmax, const double* bbox, const double* pos, double theta,
    double eps, double L, int n_images, const int64_t* pp_off, const int64_t* pc_off,
    const int64_t* cc_off, int32_t* pp_src, uint8_t* pp_img, uint8_t* pp_sub, int32_t* pc_src,
    uint8_t* pc_img, int32_t* cc_src, uint8_t* cc_img) {
    mgrav_status st = check_walk_args(theta, eps, L, n_images);
    if (st != MGRAV_OK) return st;
    if (n_cell < 1 || !cell_first || !cell_count || !child || !com || !bmax || !bbox || !pos ||
        !pp_off || !pc_off || !cc_off || !pp_src || !pp_img || !pp_sub || !pc_src || !pc_img ||
        !cc_src || !cc_img)
        return mgrav_internal::set_host_error(MGRAV_ERR_INVALID_ARG, "fmm lists: null pointer");
    FmmArgs w{cell_first, cell_count, child, com, bmax, bbox, pos, theta, eps, L, nullptr, true,
              const_cast<int64_t*>(pp_off), const_cast<int64_t*>(pc_off),
              const_cast<int64_t*>(cc_off), pp_src, pc_src, cc_src, pp_img, pp_sub, pc_img, cc_img};
    return fmm_run(w, n_cell, n_images);
}
