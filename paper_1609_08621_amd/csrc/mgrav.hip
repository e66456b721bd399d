// mgrav: device evaluation of PKDGRAV3 interaction lists on MI355X (gfx950).
//
// Paper: Potter, Stadel & Teyssier, arXiv:1609.08621.  Sec. 3.1 defines
// the tree, the PP and PC interaction lists, the multipole order (moments
// to 4th order), single-precision interactions and the Ewald correction;
// Sec. 3.3 assigns PP, PC and Ewald work to the GPU; Sec. 3.2 restricts
// work to the active particles of a substep.
//
// Launch sequence of one mgrav_compute (one HIP graph, or direct launches):
//   k_select       active buckets -> cost bins, interaction counts, the
//                  list of active particles; its last block orders the bins
//   k_order_scatter  work queue, most expensive bins first
//   k_interact     persistent: PP + PC for every queued sink bucket
//   k_ewald_setup  root coefficients and k-space table (periodic only)
//   k_ewald        FP64 Ewald correction per active particle, added to
//                  the float tree sums in double and rounded once (or the
//                  learned correction, or both with the judge)
//   k_copy_control counters to the host, then cleared for the next compute
// The first compute after mgrav_bind starts with the staging kernels
// k_stage_cells (cell records, centres, bucket ranges) and k_stage_bucket
// (particles, PP entries, work descriptors).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/mgrav.h"
#include "internal.h"

// Digest of the kernel sources this library was built from (the build
// script passes it; part of the autotuning cache key).
#ifndef MGRAV_SOURCE_DIGEST
#define MGRAV_SOURCE_DIGEST "unversioned"
#endif

// Workspace of mgrav_bind_static: a fixed device array, one copy per GPU
// the library runs on, held until the process ends.  Host code never uses
// its name as an address: the device address of each GPU's copy is looked
// up once per device (scratch_address) and passed to the kernels.
static __device__ __align__(256) unsigned char scratch[MGRAV_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int kWave = 64;
constexpr int kBucket = MGRAV_MAX_BUCKET;  // 16 sinks per work item
constexpr int kRec = 44;                   // floats per staged cell record
// Variants of the PP + PC kernel that the autotuner chooses from: PP
// entries expanded into LDS per fill (LDS = 16 x 16 B per entry) and the
// occupancy target (waves per SIMD) the register allocation aims at.
// The 2-wave variants can also prefetch the next PC chunk's records.
constexpr int kNumVariants = 6;
constexpr int kVariantChunk[kNumVariants] = {48, 32, 64, 32, 32, 64};
constexpr int kVariantWaves[kNumVariants] = {3, 3, 2, 2, 2, 2};
constexpr bool kVariantPrefetch[kNumVariants] = {false, false, false, false, true, true};
constexpr int kMaxH2 = 64;                 // largest k-space cut-off |h|^2
constexpr int kMaxHalfK = 1054;            // half-space wave vectors with |h|^2 <= 64
constexpr int kEwCoefSlots = 128;          // Ewald radial constants after the k-space rows
constexpr int kErrTree = 1, kErrList = 2, kErrParticle = 4;

// Control block at the start of the workspace.
constexpr int kCostBins = 64;
constexpr int kXcd = 8;  // accelerator dies of the chip, each with its own L2

// Queue layouts (RunArgs::queue_order; MGRAV_QUEUE_* of the header):
// longest processing time first over the whole queue, or locality first:
// the few most expensive buckets (within a factor 8 of the costliest) in
// that order, then the rest in bucket (tree) order cut into kXcd
// segments, one per die, so that the buckets one L2 serves at a time are
// neighbours in space and share most of their source cells.  Automatic:
// locality when every particle is active and there are kLocalityMinItems
// buckets or more (the buckets of a substep's mask are scattered through
// the tree and share less; there cost order measured as fast or faster).
constexpr int kQueueAuto = 0, kQueueLpt = 1, kQueueLocal = 2;
constexpr int kLocalityMinItems = 1 << 17;
constexpr int kTopBins = 3;  // cost bins (factors of 2) that stay in front

struct Control {
    int err;
    int n_items;
    int head;
    int pad;
    unsigned long long n_pp_int;
    unsigned long long n_pc_int;
    unsigned long long n_active_p;
    unsigned long long n_active_b;
    int bin_count[kCostBins];   // active buckets per cost bin
    int bin_cursor[kCostBins];  // next queue slot of each bin
    double ew_err;                  // surrogate judge: error of the sample
    unsigned long long ew_samples;  // surrogate judge: active particles sampled
    int ew_fallback;                // surrogate judge: 1 = exact path taken
    int ew_pad;
    unsigned long long n_list;      // active particles listed by k_select (mask set)
    int sel_done;                   // k_select blocks finished (the last one orders the bins)
    int waves_done;                 // k_interact waves finished (the last one stamps t_k1)
    unsigned long long t_k0, t_k1;  // k_interact's first claim and last exit, device wall clock
    int order_local;                // queue laid out for locality (set by k_select)
    int n_top;                      // queue slots before the per-die segments (all if LPT)
    int front_lo;                   // cost bins >= this one are in LPT order in front
    int seg_head[kXcd];             // next slot of each per-die segment
};

// Per-compute fields back to zero: at the end of every compute (after the
// copy to the host) and at staging, so each compute starts from zero
// without a kernel of its own.  One block; every thread may call it.
__device__ void reset_compute_counters(Control* ctl) {
    if (threadIdx.x == 0) {
        ctl->n_items = 0;
        ctl->head = 0;
        ctl->n_pp_int = ctl->n_pc_int = ctl->n_active_p = ctl->n_active_b = 0;
        ctl->ew_err = 0.0;
        ctl->ew_samples = 0;
        ctl->ew_fallback = 0;
        ctl->n_list = 0;
        ctl->sel_done = 0;
        ctl->waves_done = 0;
        ctl->t_k0 = ctl->t_k1 = 0;
        ctl->order_local = 0;
        ctl->n_top = 0;
        ctl->front_lo = 0;
    }
    for (int q = threadIdx.x; q < kCostBins; q += blockDim.x) ctl->bin_count[q] = 0;
    for (int q = threadIdx.x; q < kXcd; q += blockDim.x) ctl->seg_head[q] = 0;
}

// Image shifts in units of L: id 0 the box, 1..26 lexicographic {-1,0,1}^3.
__constant__ signed char c_shift[27][3] = {
    {0, 0, 0},   {-1, -1, -1}, {-1, -1, 0}, {-1, -1, 1}, {-1, 0, -1}, {-1, 0, 0}, {-1, 0, 1},
    {-1, 1, -1}, {-1, 1, 0},   {-1, 1, 1},  {0, -1, -1}, {0, -1, 0},  {0, -1, 1}, {0, 0, -1},
    {0, 0, 1},   {0, 1, -1},   {0, 1, 0},   {0, 1, 1},   {1, -1, -1}, {1, -1, 0}, {1, -1, 1},
    {1, 0, -1},  {1, 0, 0},    {1, 0, 1},   {1, 1, -1},  {1, 1, 0},   {1, 1, 1}};

// Per-bucket work descriptor written by the staging kernels; every range
// in it has been checked against the array it indexes.
struct BucketWork {
    int first;           // first sink particle
    int nsink;           // sink particles (0 = bucket skipped)
    int self;            // own bucket is on the PP list at image 0
    int nsrc;            // source particles over the PP list
    long long pp0, pp1;  // PP entries [pp0, pp1)
    long long pc0, pc1;  // PC entries [pc0, pc1)
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace segments (byte offsets from the workspace base).
struct Layout {
    size_t ctl, pdat, work, items, bins, cellrec, ppent, ewald, ewsample, cinfo, plist, ewbuf,
        need, total;
};

// Per cell, written first by the staging: the bounding-box centre and, for
// a cell that is a valid bucket (a leaf with 1..16 particles inside [0, n)),
// its particle range (count 0 otherwise).  The particle and PP staging
// then read one record per cell instead of four arrays.
struct CellInfo {
    double cx, cy, cz;
    int first, count;
};

// Sample of the surrogate judge: at most kMaxEwaldSamples particles, one
// record of kSampleRec doubles each (exact acceleration, valid flag, the
// PP + PC acceleration before the correction, the surrogate's acceleration).
constexpr int64_t kMaxEwaldSamples = 16384;
constexpr int64_t kDefaultEwaldSamples = 8192;
constexpr int kSampleRec = 12;

Layout make_layout(int64_t n, int64_t n_cell, int64_t n_bucket, int64_t n_pp, int64_t n_pc) {
    Layout l{};
    size_t o = 0;
    l.ctl = o;
    o += align256(sizeof(Control));
    l.pdat = o;
    o += align256(sizeof(float4) * n);
    l.work = o;
    o += align256(sizeof(BucketWork) * n_bucket);
    l.items = o;
    o += align256(sizeof(int) * n_bucket);
    l.bins = o;
    o += align256(sizeof(signed char) * n_bucket);
    l.cellrec = o;
    o += align256(sizeof(float) * kRec * n_cell);
    l.ppent = o;
    o += align256(sizeof(float4) * (n_pp > 0 ? n_pp : 1));
    l.ewald = o;
    o += align256(sizeof(double) * (64 + 8 * kMaxHalfK + kEwCoefSlots));
    l.ewsample = o;
    o += align256(sizeof(double) * kSampleRec * kMaxEwaldSamples);
    l.cinfo = o;
    o += align256(sizeof(CellInfo) * n_cell);
    l.plist = o;
    o += align256(sizeof(int) * n);
    l.ewbuf = o;
    o += align256(sizeof(double) * 4 * n);
    l.need = o;  // two flags per cell for the staging of a masked compute
    o += align256(2 * size_t(n_cell));
    l.total = o;
    return l;
}

// ---------------------------------------------------------------------
// Staging (mgrav_bind)
// ---------------------------------------------------------------------
// Where particle positions come from: double coordinates, or the integer
// coordinates of the particle store (x = origin + q * scale per axis).
struct PosIn {
    const double* pos;  // [n][3], or NULL
    const uint32_t* q;  // [n][3] when pos is NULL
    double ox, oy, oz, scale;
};

__device__ __forceinline__ void load_pos(const PosIn& in, int64_t i, double& x, double& y,
                                         double& z) {
    if (in.pos) {
        x = in.pos[3 * i];
        y = in.pos[3 * i + 1];
        z = in.pos[3 * i + 2];
    } else {
        // one fused multiply-add, as the store's decode: the tree built from
        // decoded positions and the staging see the same values
        x = fma(double(in.q[3 * i]), in.scale, in.ox);
        y = fma(double(in.q[3 * i + 1]), in.scale, in.oy);
        z = fma(double(in.q[3 * i + 2]), in.scale, in.oz);
    }
}

PosIn pos_in(const mgrav_problem& p) {
    return PosIn{p.pos, p.pos_q, p.q_origin[0], p.q_origin[1], p.q_origin[2], p.q_scale};
}

struct StageArgs {
    int64_t n, n_cell, n_bucket, n_pp, n_pc;
    int n_images;
    double L, eps;
    PosIn pin;
    const double* __restrict__ mass;  // or NULL: every mass is mass_uniform
    double mass_uniform;
    const int64_t* __restrict__ cell_first;
    const int32_t* __restrict__ cell_count;
    const int32_t* __restrict__ child;
    const double* __restrict__ com;
    const double* __restrict__ bbox;
    const double* __restrict__ mom;
    const int32_t* __restrict__ bucket_cell;
    const int64_t* __restrict__ pp_off;
    const int32_t* __restrict__ pp_src;
    const uint8_t* __restrict__ pp_img;
    const uint8_t* __restrict__ pp_sub;  // nullable: 0 whole leaf, k + 1 its k-th particle
    const int64_t* __restrict__ pc_off;
    const int32_t* __restrict__ pc_src;
    Control* ctl;
    float4* pdat;
    BucketWork* work;
    float* cellrec;
    float4* ppent;
    CellInfo* cinfo;
    // Staging for a masked compute (active set): only what the active
    // buckets read.  need_rec[c]: cell c is a PC source of an active bucket
    // (its record); need_src[c]: leaf c is a PP source or the sink of an
    // active bucket (its particles and CellInfo).  NULL: stage everything.
    const uint8_t* __restrict__ active;
    uint8_t* need_rec;
    uint8_t* need_src;
};

// The bounding-box centre and, for a valid bucket (a leaf with 1..16
// particles inside [0, n)), the particle range of cell c (count 0 otherwise).
__device__ __forceinline__ CellInfo cell_info(const StageArgs& a, int64_t c) {
    const double* bb = a.bbox + 6 * c;
    CellInfo ci;
    ci.cx = 0.5 * (bb[0] + bb[3]);
    ci.cy = 0.5 * (bb[1] + bb[4]);
    ci.cz = 0.5 * (bb[2] + bb[5]);
    const int64_t f = a.cell_first[c];
    const int k = a.cell_count[c];
    const bool ok = a.child[2 * c] < 0 && k >= 1 && k <= kBucket && f >= 0 && f + k <= a.n;
    ci.first = ok ? int(f) : 0;
    ci.count = ok ? k : 0;
    return ci;
}

// The control block (counters, error bits) into pinned host memory: the
// last kernel of a compute; the host reads it after the completion event.
__global__ void k_copy_control(Control* ctl, Control* host) {
    const int* src = reinterpret_cast<const int*>(ctl);
    int* dst = reinterpret_cast<int*>(host);
    for (int i = threadIdx.x; i < int(sizeof(Control) / sizeof(int)); i += blockDim.x)
        dst[i] = src[i];
    __syncthreads();
    reset_compute_counters(ctl);
}

// Inverse of the length unit in which a cell's PC interactions are
// evaluated: 2^-e with 2^e the smallest power of two above both the
// softening length and the distance from the centre of mass to the
// farthest corner of the bounding box.  In this unit the radial
// derivatives of order up to 5 stay O(1) for every accepted cell (they
// would overflow float for small cells a few softening lengths away), and
// since the unit is a power of two the rescaling itself rounds nothing.
__device__ float cell_inv_unit(const StageArgs& a, int64_t c) {
    const double* bb = a.bbox + 6 * c;
    const double* x = a.com + 3 * c;
    double r2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double d = fmax(x[k] - bb[k], bb[3 + k] - x[k]);
        r2 += d * d;
    }
    const double b = fmax(sqrt(r2), a.eps);
    int e = 0;
    (void)frexp(b, &e);                 // b < 2^e
    e = e < -100 ? -100 : (e > 100 ? 100 : e);  // NaN or absurd boxes stay finite
    return float(ldexp(1.0, -e));
}

// (2) cells: float coefficients of the order-4 expansion (multipole_terms,
// pc_one), the order-k ones in units of the cell's length unit (times t^k),
// and t = 1 / unit in the last word.  (Staging moments and records through
// LDS for contiguous access, or four lanes per cell each storing a quarter,
// measured slower.)
//
// Also, per cell, the bounding-box centre and, for a valid bucket (a leaf
// with 1..16 particles inside [0, n)), its particle range (CellInfo), and
// block 0 clears the control block (error bits and counters): this is the
// first staging kernel.
__global__ void k_stage_cells(StageArgs a) {
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) a.ctl->err = 0;
        reset_compute_counters(a.ctl);
    }
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= a.n_cell) return;
    if (!a.active || a.need_src[c]) a.cinfo[c] = cell_info(a, c);
    if (a.active && !a.need_rec[c]) return;
    const double* m = a.mom + 32 * c;
    double r[kRec];
    r[0] = m[0];
    r[1] = 0.5 * (m[1] + m[4] + m[6]);
    for (int i = 0; i < 6; ++i) r[2 + i] = 0.5 * m[1 + i];
    r[8] = -0.5 * (m[7] + m[10] + m[12]);
    r[9] = -0.5 * (m[8] + m[13] + m[15]);
    r[10] = -0.5 * (m[9] + m[14] + m[16]);
    r[11] = 0.125 * (m[17] + m[27] + m[31] + 2.0 * (m[20] + m[22] + m[29]));
    for (int i = 0; i < 10; ++i) r[12 + i] = -m[7 + i] / 6.0;
    r[22] = 0.25 * (m[17] + m[20] + m[22]);
    r[23] = 0.25 * (m[18] + m[23] + m[25]);
    r[24] = 0.25 * (m[19] + m[24] + m[26]);
    r[25] = 0.25 * (m[20] + m[27] + m[29]);
    r[26] = 0.25 * (m[21] + m[28] + m[30]);
    r[27] = 0.25 * (m[22] + m[29] + m[31]);
    for (int i = 0; i < 15; ++i) r[28 + i] = m[17 + i] / 24.0;
    // the group of each radial derivative a_n carries its (2n - 1)!! (see pc_one)
    for (int i = 2; i < 12; ++i) r[i] *= 3.0;
    for (int i = 12; i < 28; ++i) r[i] *= 15.0;
    for (int i = 28; i < 43; ++i) r[i] *= 105.0;
    const double t = cell_inv_unit(a, c), t2 = t * t, t3 = t2 * t, t4 = t3 * t;
    for (int i = 1; i < 8; ++i) r[i] *= t2;
    for (int i = 8; i < 11; ++i) r[i] *= t3;
    r[11] *= t4;
    for (int i = 12; i < 22; ++i) r[i] *= t3;
    for (int i = 22; i < kRec - 1; ++i) r[i] *= t4;
    r[43] = t;
    float4* out = reinterpret_cast<float4*>(a.cellrec + kRec * c);
    for (int i = 0; i < kRec / 4; ++i)
        out[i] = make_float4(float(r[4 * i]), float(r[4 * i + 1]), float(r[4 * i + 2]),
                             float(r[4 * i + 3]));
}

// (3) per sink bucket, 16 lanes: its particles (float offsets from the
// bucket's bounding-box centre, kept in double, and masses; lane k takes
// particle k), its PP entries (offset between the source bucket's centre
// plus the image shift and the sink bucket's centre, in double, rounded to
// float; the source's first particle and count packed into the fourth
// word; each lane keeps kStageRound entries in flight), the check of its
// PC range, and its work descriptor.  The PC entries themselves are read,
// checked and turned into offsets by the interact kernel.
constexpr int kStageLanes = 16;
constexpr int kStageRound = 4;
__device__ inline int group_or(int v) {
    for (int o = kStageLanes / 2; o > 0; o >>= 1) v |= __shfl_xor(v, o);
    return v;
}
__device__ inline int group_sum(int v) {
    for (int o = kStageLanes / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
// Staging for a masked compute: clear the two flag arrays (a fill kernel,
// so that the staging can be captured in a graph), then mark what the
// active buckets read: their own leaves and PP source leaves (particles,
// CellInfo) and their PC source cells (records).  Plain stores of 1: every
// writer stores the same value.  Entries outside their arrays are skipped
// here and reported by the staging.
__global__ void __launch_bounds__(256) k_need_clear(StageArgs a) {
    uint32_t* w = reinterpret_cast<uint32_t*>(a.need_rec);  // need_src follows need_rec
    const int64_t words = (2 * a.n_cell + 3) / 4;           // within the padded segment
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < words;
         i += int64_t(gridDim.x) * blockDim.x)
        w[i] = 0u;
}

// One lane per bucket finds whether any of its particles is active (a
// masked compute touches a few per cent of the buckets: for most of them
// the test is all the work); then the active buckets of the wave's 64 have
// their lists marked by groups of 16 lanes, four buckets at a time, each
// lane with kStageRound entries in flight.
template <typename Mark>
__device__ __forceinline__ void mark_range(const int32_t* src, int64_t e0, int64_t e1,
                                           int64_t n_cell, int sl, Mark&& mark) {
    for (int64_t eb = e0 + sl; eb < e1; eb += kStageRound * kStageLanes) {
        int32_t v[kStageRound];
#pragma unroll
        for (int u = 0; u < kStageRound; ++u) {
            const int64_t e = eb + u * kStageLanes;
            v[u] = e < e1 ? src[e] : -1;
        }
#pragma unroll
        for (int u = 0; u < kStageRound; ++u)
            if (v[u] >= 0 && v[u] < n_cell) mark(v[u]);
    }
}

__global__ void __launch_bounds__(256) k_need_mark(StageArgs a) {
    const int lane = int(threadIdx.x & (kWave - 1));
    const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int s = -1;
    bool act = false;
    if (b < a.n_bucket) {
        const int64_t c = a.bucket_cell[b];
        if (c >= 0 && c < a.n_cell) {
            s = int(c);
            const CellInfo ci = cell_info(a, c);
            for (int k = 0; k < ci.count; ++k) act |= a.active[ci.first + k] != 0;
        }
    }
    const int64_t b0 = b - lane;
    const int g = lane / kStageLanes, sl = lane % kStageLanes;
    for (uint64_t todo = __ballot(act); todo;) {
        uint64_t m = todo;  // this group's bucket: the g-th remaining one
        for (int t = 0; t < kWave / kStageLanes - 1; ++t)
            if (t < g) m &= m - 1;
        for (int t = 0; t < kWave / kStageLanes; ++t) todo &= todo - 1;  // (wave-uniform)
        const int l = m ? __builtin_ctzll(m) : 0;
        const int sc = __shfl(s, l);
        if (!m) continue;
        const int64_t bb = b0 + l;
        if (sl == 0) a.need_src[sc] = 1;
        const int64_t e0 = a.pp_off[bb], e1 = a.pp_off[bb + 1];
        if (e0 >= 0 && e0 <= e1 && e1 <= a.n_pp)
            mark_range(a.pp_src, e0, e1, a.n_cell, sl, [&](int32_t c) { a.need_src[c] = 1; });
        const int64_t g0 = a.pc_off[bb], g1 = a.pc_off[bb + 1];
        if (g0 >= 0 && g0 <= g1 && g1 <= a.n_pc)
            mark_range(a.pc_src, g0, g1, a.n_cell, sl, [&](int32_t c) { a.need_rec[c] = 1; });
    }
}

// The staging of bucket b by a group of 16 lanes (lane sl of the group):
// its sink particles when stage_sinks, its PP entries and the check of its
// PC range when act, and, when write_work, its work descriptor and error
// bits.  A group with nothing to do passes act, stage_sinks and write_work
// false and only takes part in the group reductions.
__device__ __forceinline__ void stage_bucket_group(const StageArgs& a, int64_t b, int sl,
                                                   int64_t s, bool sink_ok, const CellInfo& ci,
                                                   bool act, bool stage_sinks, bool write_work) {
    // the sink particles
    if (ci.count == 0) {
        if (sl == 0 && write_work) atomicOr(&a.ctl->err, kErrTree);
    } else if (sl < ci.count && stage_sinks) {
        const int64_t p = ci.first + sl;
        double x, y, z;
        load_pos(a.pin, p, x, y, z);
        const double m = a.mass ? a.mass[p] : a.mass_uniform;
        if (!(isfinite(x) && isfinite(y) && isfinite(z) && m > 0.0 && isfinite(m)))
            atomicOr(&a.ctl->err, kErrParticle);
        a.pdat[p] = make_float4(float(x - ci.cx), float(y - ci.cy), float(z - ci.cz), float(m));
    }
    // the PP entries (of an active bucket only, with a mask)
    const int64_t e0 = act ? a.pp_off[b] : 0, e1 = act ? a.pp_off[b + 1] : 0;
    const bool range_ok = e0 >= 0 && e0 <= e1 && e1 <= a.n_pp;
    int nsrc = 0, self = 0, bad = 0;
    if (!range_ok || !sink_ok) bad = 1;
    if (range_ok) {
        for (int64_t eb = e0 + sl; eb < e1; eb += kStageRound * kStageLanes) {
            int64_t src[kStageRound];
            int img[kStageRound], sub[kStageRound];
#pragma unroll
            for (int u = 0; u < kStageRound; ++u) {
                const int64_t e = eb + u * kStageLanes;
                src[u] = e < e1 ? int64_t(a.pp_src[e]) : -1;
                img[u] = e < e1 ? int(a.pp_img[e]) : 0;
                sub[u] = e < e1 && a.pp_sub ? int(a.pp_sub[e]) : 0;
            }
            CellInfo si[kStageRound];
#pragma unroll
            for (int u = 0; u < kStageRound; ++u)
                si[u] = src[u] >= 0 && src[u] < a.n_cell ? a.cinfo[src[u]]
                                                         : CellInfo{0.0, 0.0, 0.0, 0, 0};
#pragma unroll
            for (int u = 0; u < kStageRound; ++u) {
                const int64_t e = eb + u * kStageLanes;
                if (e >= e1) continue;
                float4 out = make_float4(0.f, 0.f, 0.f, __int_as_float(0));
                if (sink_ok && img[u] < a.n_images && si[u].count > 0 && sub[u] <= si[u].count) {
                    // a whole source leaf, or one particle of it (same centre)
                    const int first = sub[u] ? si[u].first + sub[u] - 1 : si[u].first;
                    const int count = sub[u] ? 1 : si[u].count;
                    out.x = float(si[u].cx + c_shift[img[u]][0] * a.L - ci.cx);
                    out.y = float(si[u].cy + c_shift[img[u]][1] * a.L - ci.cy);
                    out.z = float(si[u].cz + c_shift[img[u]][2] * a.L - ci.cz);
                    out.w = __uint_as_float(uint32_t(first) | (uint32_t(count) << 27));
                    nsrc += count;
                    if (src[u] == s && img[u] == 0) self = 1;
                } else {
                    bad = 1;
                }
                a.ppent[e] = out;
            }
        }
    }
    const int64_t g0 = act ? a.pc_off[b] : 0, g1 = act ? a.pc_off[b + 1] : 0;
    const bool pc_ok = g0 >= 0 && g0 <= g1 && g1 <= a.n_pc;
    if (!pc_ok) bad = 1;
    bad = group_or(bad);
    self = group_or(self);
    nsrc = group_sum(nsrc);
    if (sl == 0 && write_work) {
        if (bad) atomicOr(&a.ctl->err, kErrList);
        BucketWork w;
        w.first = ci.count ? ci.first : 0;
        w.nsink = ci.count;
        w.self = self;
        w.nsrc = nsrc;
        w.pp0 = range_ok ? e0 : 0;
        w.pp1 = range_ok ? e1 : 0;
        w.pc0 = pc_ok && sink_ok ? g0 : 0;
        w.pc1 = pc_ok && sink_ok ? g1 : 0;
        a.work[b] = w;
    }
}

// Without a mask: every bucket, 16 lanes each.
__global__ void __launch_bounds__(256) k_stage_bucket(StageArgs a) {
    const int64_t b = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kStageLanes;
    const int sl = int(threadIdx.x % kStageLanes);
    if (b >= a.n_bucket) return;  // whole groups: the first n_bucket groups are in range
    const int64_t s = a.bucket_cell[b];
    const bool sink_ok = s >= 0 && s < a.n_cell;
    const CellInfo ci = sink_ok ? a.cinfo[s] : CellInfo{0.0, 0.0, 0.0, 0, 0};
    stage_bucket_group(a, b, sl, s, sink_ok, ci, true, true, true);
}

// With a mask: one lane per bucket finds whether it is active and whether
// its particles are read (as PP sources of active buckets), and writes
// the descriptor of an inactive bucket (no lists); the buckets with
// anything to stage then go through the 16-lane staging, four at a time.
__global__ void __launch_bounds__(256) k_stage_bucket_masked(StageArgs a) {
    const int lane = int(threadIdx.x & (kWave - 1));
    const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t b0 = b - lane;
    int s = -1;
    CellInfo ci{0.0, 0.0, 0.0, 0, 0};
    bool act = false, stage = false;
    if (b < a.n_bucket) {
        const int64_t c = a.bucket_cell[b];
        const bool sink_ok = c >= 0 && c < a.n_cell;
        if (sink_ok) {
            s = int(c);
            ci = cell_info(a, c);
            for (int k = 0; k < ci.count; ++k) act |= a.active[ci.first + k] != 0;
            stage = a.need_src[c] != 0;
        }
        if (!act) {
            if (ci.count == 0) atomicOr(&a.ctl->err, kErrTree);
            if (!sink_ok) atomicOr(&a.ctl->err, kErrList);
            BucketWork w;
            w.first = ci.count ? ci.first : 0;
            w.nsink = ci.count;
            w.self = 0;
            w.nsrc = 0;
            w.pp0 = w.pp1 = w.pc0 = w.pc1 = 0;
            a.work[b] = w;
        }
    }
    const int g = lane / kStageLanes, sl = lane % kStageLanes;
    for (uint64_t todo = __ballot(act || stage); todo;) {
        uint64_t m = todo;  // this group's bucket: the g-th remaining one
        for (int t = 0; t < kWave / kStageLanes - 1; ++t)
            if (t < g) m &= m - 1;
        for (int t = 0; t < kWave / kStageLanes; ++t) todo &= todo - 1;  // (wave-uniform)
        const bool valid = m != 0;
        const int l = valid ? __builtin_ctzll(m) : 0;
        CellInfo cb;
        cb.cx = __shfl(ci.cx, l);
        cb.cy = __shfl(ci.cy, l);
        cb.cz = __shfl(ci.cz, l);
        cb.first = __shfl(ci.first, l);
        cb.count = __shfl(ci.count, l);
        const int sb = __shfl(s, l);
        const bool ab = __shfl(act ? 1 : 0, l) != 0 && valid;
        const bool stb = __shfl(stage ? 1 : 0, l) != 0 && valid;
        stage_bucket_group(a, b0 + l, sl, sb, true, valid ? cb : CellInfo{0.0, 0.0, 0.0, 0, 0},
                           ab, stb, ab);
    }
}

// ---------------------------------------------------------------------
// Per-compute kernels
// ---------------------------------------------------------------------
struct RunArgs {
    int64_t n, n_bucket;
    const uint8_t* __restrict__ active;
    Control* ctl;
    const float4* __restrict__ pdat;
    const BucketWork* __restrict__ work;
    int* items;
    signed char* bins;  // cost bin of each active bucket, -1 if inactive
    const float* __restrict__ cellrec;
    const float4* __restrict__ ppent;
    const int32_t* __restrict__ pc_src;       // [n_pc] source cell
    const uint8_t* __restrict__ pc_img;       // [n_pc] image id
    const double* __restrict__ com;           // [n_cell][3]
    const double* __restrict__ bbox;          // [n_cell][6]
    const int32_t* __restrict__ bucket_cell;  // [n_bucket]
    int64_t n_cell;
    double L;
    int n_images;
    float* __restrict__ acc;  // [3][n]
    float* __restrict__ pot;  // [n]
    float eps2;
    int parts;
    int* plist;  // with a mask: the active particles, for the Ewald kernels
    int queue_order;  // kQueueAuto, kQueueLpt or kQueueLocal
};

__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
    for (int o = 1; o < kWave; o <<= 1) {
        const int t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

// Active buckets into the work queue (in bucket order when all particles
// are active) and the interaction counts of the active sinks.  With a mask,
// also the list of active particles (block-aggregated appends; the order
// of blocks in it is not fixed, and nothing depends on it).
constexpr int kSelectThreads = 256;
__global__ void __launch_bounds__(kSelectThreads) k_select(RunArgs a) {
    __shared__ int hist[kCostBins];
    __shared__ int wsum[kSelectThreads / kWave];
    __shared__ unsigned long long lbase;
    if (threadIdx.x < kCostBins) hist[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    unsigned long long npp = 0, npc = 0, nact = 0, nb = 0;
    // grid-stride over the buckets (the same trip count for the whole
    // block): a bounded grid keeps the same-address atomics few
    for (int64_t b0 = int64_t(blockIdx.x) * blockDim.x; b0 < a.n_bucket;
         b0 += int64_t(gridDim.x) * blockDim.x) {
        const int64_t b = b0 + threadIdx.x;
        BucketWork wk{};
        int na = 0;
        if (b < a.n_bucket) {
            wk = a.work[b];
            na = wk.nsink;
            if (a.active) {
                na = 0;
                for (int k = 0; k < wk.nsink; ++k) na += a.active[wk.first + k] != 0;
            }
            int bin = -1;
            if (na > 0) {
                // work of the bucket in FLOP, binned by its base-2 logarithm
                const unsigned long long cost =
                    (unsigned long long)wk.nsink *
                    ((unsigned long long)wk.nsrc * 20ull +
                     (unsigned long long)(wk.pc1 - wk.pc0) * 242ull);
                bin = 63 - __clzll(cost | 1ull);
                atomicAdd(&hist[bin], 1);
            }
            a.bins[b] = (signed char)bin;
            if (na > 0) {
                nact += na;
                nb += 1;
                npp += (unsigned long long)na * (unsigned long long)wk.nsrc;
                npc += (unsigned long long)na * (unsigned long long)(wk.pc1 - wk.pc0);
            }
        }
        if (a.plist) {  // append this block's active particles
            const int incl = wave_incl_scan(na, lane);
            if (lane == kWave - 1) wsum[w] = incl;
            __syncthreads();
            int before = 0, total = 0;
            for (int q = 0; q < kSelectThreads / kWave; ++q) {
                before += q < w ? wsum[q] : 0;
                total += wsum[q];
            }
            if (threadIdx.x == 0) lbase = atomicAdd(&a.ctl->n_list, (unsigned long long)total);
            __syncthreads();
            int64_t slot = int64_t(lbase) + before + incl - na;
            for (int k = 0; k < wk.nsink && na > 0; ++k)
                if (a.active[wk.first + k]) a.plist[slot++] = wk.first + k;
            __syncthreads();  // wsum and lbase are rewritten by the next round
        }
    }
    // block reduction, one atomic per block
    __shared__ unsigned long long red[4][kSelectThreads / kWave];
    for (int o = kWave / 2; o > 0; o >>= 1) {
        npp += __shfl_xor(npp, o);
        npc += __shfl_xor(npc, o);
        nact += __shfl_xor(nact, o);
        nb += __shfl_xor(nb, o);
    }
    if (lane == 0) {
        red[0][w] = npp;
        red[1][w] = npc;
        red[2][w] = nact;
        red[3][w] = nb;
    }
    __syncthreads();
    if (threadIdx.x < kCostBins && hist[threadIdx.x])
        atomicAdd(&a.ctl->bin_count[threadIdx.x], hist[threadIdx.x]);
    __shared__ int last;
    if (threadIdx.x == 0) {
        unsigned long long s[4] = {0, 0, 0, 0};
        for (int i = 0; i < kSelectThreads / kWave; ++i)
            for (int q = 0; q < 4; ++q) s[q] += red[q][i];
        if (s[2]) {
            atomicAdd(&a.ctl->n_pp_int, s[0]);
            atomicAdd(&a.ctl->n_pc_int, s[1]);
            atomicAdd(&a.ctl->n_active_p, s[2]);
            atomicAdd(&a.ctl->n_active_b, s[3]);
        }
    }
    // the last block to finish lays out the queue: most expensive cost bins
    // first (longest processing time first, to within a factor 2), so the
    // persistent kernel ends on short items; or, for locality, only the top
    // kTopBins bins so, and the rest in bucket order behind them
    __syncthreads();  // this block's bin counts are added
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(&a.ctl->sel_done, 1) == int(gridDim.x) - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    if (threadIdx.x < kCostBins)  // every block's counts, read at device scope
        hist[threadIdx.x] = __atomic_load_n(&a.ctl->bin_count[threadIdx.x], __ATOMIC_RELAXED);
    __syncthreads();
    if (threadIdx.x == 0) {
        int total = 0, top = -1;
        for (int q = kCostBins - 1; q >= 0; --q) {
            total += hist[q];
            if (top < 0 && hist[q] > 0) top = q;
        }
        const bool local = a.queue_order == kQueueLocal ||
                           (a.queue_order == kQueueAuto && a.active == nullptr &&
                            total >= kLocalityMinItems);
        const int lo = local && top >= kTopBins ? top - kTopBins + 1 : 0;  // LPT: bins >= lo
        int off = 0;
        for (int q = kCostBins - 1; q >= 0 && q >= lo; --q) {
            a.ctl->bin_cursor[q] = off;
            off += hist[q];
        }
        a.ctl->bin_cursor[0] = lo > 0 ? off : a.ctl->bin_cursor[0];  // the shared range
        a.ctl->front_lo = lo;
        a.ctl->n_top = local ? off : total;
        a.ctl->order_local = local ? 1 : 0;
        a.ctl->n_items = total;
    }
}

// Block-aggregated scatter: one global atomic per (block, bin) reserves a
// range of queue slots; ranks inside the block come from LDS atomics.  In
// the locality layout the bins below the top ones share one range, and
// the block's buckets keep their order in it (ranks from a block scan).
constexpr int kScatterThreads = 1024;
__global__ void __launch_bounds__(kScatterThreads) k_order_scatter(RunArgs a) {
    __shared__ int cnt[kCostBins];
    __shared__ int base[kCostBins];
    __shared__ int wtot[kScatterThreads / kWave];
    __shared__ int run_base;
    if (threadIdx.x < kCostBins) cnt[threadIdx.x] = 0;
    const int front_lo = a.ctl->front_lo;  // set by k_select (0: every bin in front)
    __syncthreads();
    const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int bin = -1, rank = 0;
    if (b < a.n_bucket) bin = a.bins[b];
    const bool front = bin >= 0 && bin >= front_lo;
    if (front) rank = atomicAdd(&cnt[bin], 1);
    // ranks of the shared range, in bucket order
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int in_run = bin >= 0 && !front ? 1 : 0;
    const int incl = wave_incl_scan(in_run, lane);
    if (lane == kWave - 1) wtot[w] = incl;
    __syncthreads();
    if (threadIdx.x < kCostBins && cnt[threadIdx.x] > 0)
        base[threadIdx.x] = atomicAdd(&a.ctl->bin_cursor[threadIdx.x], cnt[threadIdx.x]);
    int before = 0, total = 0;
    for (int q = 0; q < kScatterThreads / kWave; ++q) {
        before += q < w ? wtot[q] : 0;
        total += wtot[q];
    }
    if (threadIdx.x == 0 && total > 0) run_base = atomicAdd(&a.ctl->bin_cursor[0], total);
    __syncthreads();
    if (front) a.items[base[bin] + rank] = int(b);
    if (in_run) a.items[run_base + before + incl - 1] = int(b);
}

// Order-4 PC expansion of one cell at one point, float.
//   R = x - X (sink minus expansion centre), D = R.R + eps^2,
//   a_n = ((1/r) d/dr)^n D^(-1/2) = (-1)^n (2n-1)!! D^(-(2n+1)/2),
//   phi = -sum_n a_n P_n(R),  acc = sum_n (a_{n+1} P_n R + a_n grad P_n),
// with P_0 = M, P_1 = tr(M2)/2, P_2 = R.M2.R/2 - tr(M3).R/2 + tr tr(M4)/8,
// P_3 = -M3[RRR]/6 + R.tr(M4).R/4, P_4 = M4[RRRR]/24: the Taylor series of
// the softened potential about the centre of mass, grouped by radial
// derivative.  The coefficients are the moment combinations
// r[0]=M, r[1]=trM2/2, r[2..7]=M2/2, r[8..10]=-trM3/2, r[11]=ttrM4/8,
// r[12..21]=-M3/6, r[22..27]=trM4/4, r[28..42]=M4/24 (the float records
// of the PC kernel hold groups 2, 3, 4 times 3, 15, 105; the Ewald table
// holds them as they are).
template <typename T, typename Rec>
__device__ __forceinline__ void multipole_terms(const Rec& r, T x, T y, T z, T& P2, T& P3,
                                                T& P4, T& g2x, T& g2y, T& g2z, T& g3x, T& g3y,
                                                T& g3z, T& v4x, T& v4y, T& v4z) {
    const T xx = x * x, yy = y * y, zz = z * z;
    const T x2 = x + x, y2 = y + y;
    const T qxy = x2 * y, qxz = x2 * z, qyz = y2 * z;
    // order 2 (with the traced parts of orders 3 and 4): h2 = M2/2 R + r8..10,
    // each chain started from its constant so that it is all FMAs
    const T h2x = r[2] * x + (r[3] * y + (r[4] * z + r[8]));
    const T h2y = r[3] * x + (r[5] * y + (r[6] * z + r[9]));
    const T h2z = r[4] * x + (r[6] * y + (r[7] * z + r[10]));
    P2 = x * h2x + y * h2y + z * h2z + r[11];
    g2x = T(2) * h2x - r[8];  // 2 (M2/2 R) + r8
    g2y = T(2) * h2y - r[9];
    g2z = T(2) * h2z - r[10];
    // order 3 (with the once-traced part of order 4): h3 = v3 + w4, the v3
    // chain started from w4
    const T w4x = r[22] * x + r[23] * y + r[24] * z;
    const T w4y = r[23] * x + r[25] * y + r[26] * z;
    const T w4z = r[24] * x + r[26] * y + r[27] * z;
    const T h3x = r[12] * xx + (r[15] * yy + (r[17] * zz + (r[13] * qxy + (r[14] * qxz +
                  (r[16] * qyz + w4x)))));
    const T h3y = r[13] * xx + (r[18] * yy + (r[20] * zz + (r[15] * qxy + (r[16] * qxz +
                  (r[19] * qyz + w4y)))));
    const T h3z = r[14] * xx + (r[19] * yy + (r[21] * zz + (r[16] * qxy + (r[17] * qxz +
                  (r[20] * qyz + w4z)))));
    P3 = x * h3x + y * h3y + z * h3z;
    g3x = T(3) * h3x - w4x;  // 3 v3 + 2 w4
    g3y = T(3) * h3y - w4y;
    g3z = T(3) * h3z - w4z;
    // order 4: cubic monomials with their multiplicities folded in
    const T x3 = T(3) * x, y3 = T(3) * y, z3 = T(3) * z;
    const T cxxx = xx * x, cxxy = xx * y3, cxxz = xx * z3, cxyy = yy * x3, cxyz = qxy * z3;
    const T cxzz = zz * x3, cyyy = yy * y, cyyz = yy * z3, cyzz = zz * y3, czzz = zz * z;
    v4x = r[28] * cxxx + r[29] * cxxy + r[30] * cxxz + r[31] * cxyy + r[32] * cxyz +
          r[33] * cxzz + r[34] * cyyy + r[35] * cyyz + r[36] * cyzz + r[37] * czzz;
    v4y = r[29] * cxxx + r[31] * cxxy + r[32] * cxxz + r[34] * cxyy + r[35] * cxyz +
          r[36] * cxzz + r[38] * cyyy + r[39] * cyyz + r[40] * cyzz + r[41] * czzz;
    v4z = r[30] * cxxx + r[32] * cxxy + r[33] * cxxz + r[35] * cxyy + r[36] * cxyz +
          r[37] * cxzz + r[39] * cyyy + r[40] * cyyz + r[41] * cyzz + r[42] * czzz;
    P4 = x * v4x + y * v4y + z * v4z;
}

struct Acc4 {
    float x, y, z, p;
};

__device__ __forceinline__ void pp_one(float sx, float sy, float sz, float m, float px, float py,
                                       float pz, float eps2, Acc4& A) {
    // source minus sink: the force on the sink points along +d
    const float dx = sx - px, dy = sy - py, dz = sz - pz;
    const float D = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
    const float w = __builtin_amdgcn_rsqf(D);
    const float mw = m * w;
    const float w2 = w * w;
    const float mw3 = mw * w2;
    A.p -= mw;
    A.x = fmaf(mw3, dx, A.x);
    A.y = fmaf(mw3, dy, A.y);
    A.z = fmaf(mw3, dz, A.z);
}

// In the cell's length unit 1/t: R' = t R (the centre offset c arrives
// scaled), eps2t = t^2 eps^2, moments of order k times t^k.  Then
// phi = t phi'(R') and acc = t^2 acc'(R'): one factor t is folded into a_n,
// the other into the acceleration's coefficients.
//
// With a_n = a0 u^n (2n-1)!!, u = -1/D, and the staged groups already
// carrying (2n-1)!! (so the multipole_terms outputs are Q_n = (2n-1)!! P_n
// and their gradients), the radial sums are polynomials in u:
//   sum_n a_n P_n     = a0 f(u),             f(u) = sum_n u^n Q_n,
//   sum_n a_{n+1} P_n = a0 u (f + 2u f'(u)), since (2n+1)!! = (2n+1)(2n-1)!!,
//   sum_n a_n grad P_n = sum_n a0 u^n grad Q_n,
// with f and f' from one Horner pass.
__device__ __forceinline__ void pc_one(const float (&r)[kRec], float t, float cx, float cy,
                                       float cz, float px, float py, float pz, float eps2t,
                                       Acc4& A) {
    const float x = fmaf(px, t, -cx), y = fmaf(py, t, -cy), z = fmaf(pz, t, -cz);
    const float D = fmaf(x, x, fmaf(y, y, fmaf(z, z, eps2t)));
    const float w = __builtin_amdgcn_rsqf(D);
    const float a0 = w * t;
    const float u = -(w * w);
    float Q2, Q3, Q4, g2x, g2y, g2z, g3x, g3y, g3z, v4x, v4y, v4z;
    multipole_terms<float>(r, x, y, z, Q2, Q3, Q4, g2x, g2y, g2z, g3x, g3y, g3z, v4x, v4y, v4z);
    const float f3 = fmaf(u, Q4, Q3);
    const float f2 = fmaf(u, f3, Q2);
    const float d2 = fmaf(u, Q4, f3);
    const float f1 = fmaf(u, f2, r[1]);
    const float d1 = fmaf(u, d2, f2);
    const float f0 = fmaf(u, f1, r[0]);
    const float d0 = fmaf(u, d1, f1);
    A.p = fmaf(-a0, f0, A.p);
    // the second factor t rides on a1, so each acceleration component is
    // four FMAs into its sum
    const float a1 = (a0 * t) * u;
    const float S = a1 * fmaf(u + u, d0, f0);
    const float b2 = a1 * u, b3 = b2 * u, b4x4 = b3 * (4.f * u);  // grad Q4 = 4 v4
    A.x = fmaf(b4x4, v4x, fmaf(b3, g3x, fmaf(b2, g2x, fmaf(S, x, A.x))));
    A.y = fmaf(b4x4, v4y, fmaf(b3, g3y, fmaf(b2, g2y, fmaf(S, y, A.y))));
    A.z = fmaf(b4x4, v4z, fmaf(b3, g3z, fmaf(b2, g2z, fmaf(S, z, A.z))));
}

// Load of a wave-uniform element of memory that no kernel running at the
// same time writes: through the constant address space the compiler emits a
// scalar load into scalar registers.  (The host compilation pass only needs
// the function to exist.)
template <typename T>
__device__ __forceinline__ T load_uniform(const T* p, int64_t i) {
#if defined(__HIP_DEVICE_COMPILE__)
    return ((const __attribute__((address_space(4))) T*)p)[i];
#else
    return p[i];
#endif
}

// PC entry f of a list ending at f1, for a sink bucket centred at C
// (double): the cell's record and the offset of its centre of mass (plus
// the image shift) from C, formed in double and scaled by the cell's
// length unit before rounding to float.  Every lane loads a valid record,
// so the loads need neither a branch nor a zero fill: an entry at or past
// f1 reads the list's last entry (the caller guarantees f1 > the chunk's
// first entry, so that entry exists), and an entry with a cell index or image id
// out of range is reported (BAD_LIST) and reads cell 0.  Such lanes then get
// t = 0 and the offset (-1, 0, 0): R' = (1, 0, 0), D' = 1 and a_0 = 0, so
// every term is finite and adds zero.
__device__ __forceinline__ void load_pc(const RunArgs& a, int64_t f, int64_t f1, double Cx,
                                        double Cy, double Cz, float (&r)[kRec], float& cx,
                                        float& cy, float& cz) {
    const bool in = f < f1;
    const int64_t fc = in ? f : f1 - 1;
    const int src = a.pc_src[fc];
    const int im = a.pc_img[fc];
    const bool ok = src >= 0 && src < a.n_cell && im < a.n_images;
    if (in && !ok) atomicOr(&a.ctl->err, kErrList);
    const bool use = in && ok;
    const int cell = ok ? src : 0;
    const int img = ok ? im : 0;
    const float4* rec = reinterpret_cast<const float4*>(a.cellrec + kRec * int64_t(cell));
#pragma unroll
    for (int i = 0; i < kRec / 4; ++i) {
        const float4 q = rec[i];
        r[4 * i] = q.x;
        r[4 * i + 1] = q.y;
        r[4 * i + 2] = q.z;
        r[4 * i + 3] = q.w;
    }
    // image id 0 is the box, 1..26 the other points of {-1,0,1}^3 in
    // lexicographic order: k is the position in the full 27-point order
    const int k = img == 0 ? 13 : (img <= 13 ? img - 1 : img);
    const double t = double(r[kRec - 1]);
    const double* X = a.com + 3 * int64_t(cell);
    const float ox = float((X[0] + double(k / 9 - 1) * a.L - Cx) * t);
    const float oy = float((X[1] + double(k / 3 % 3 - 1) * a.L - Cy) * t);
    const float oz = float((X[2] + double(k % 3 - 1) * a.L - Cz) * t);
    cx = use ? ox : -1.f;
    cy = use ? oy : 0.f;
    cz = use ? oz : 0.f;
    r[kRec - 1] = use ? r[kRec - 1] : 0.f;
}

// The sink count as a value the compiler must read again where it is used:
// the per-sink tests then stay scalar compares inside each chunk instead of
// sixteen 64-bit lane masks hoisted out of the chunk loops, which would
// take scalar registers that the kernel's arguments need.
__device__ __forceinline__ int sink_count(int n) {
    asm volatile("; sink count %0" : "+s"(n));
    return n;
}

// A wavefront's place in the work queue: the front (one head for all), then
// its die's segment, then the other dies' segments in turn, each until it
// runs dry.  Only lane 0's copy is used.
struct QueueCursor {
    int phase;  // 0: front; 1: segments
    int seg;    // segment being drained
    int tries;  // segments found empty
};

// Claims a queue slot of the cursor's current range (its result is read
// later, by queue_resolve, so the atomic's latency hides behind an item).
__device__ __forceinline__ int queue_issue(Control* ctl, const QueueCursor& q) {
    return atomicAdd(q.phase == 0 ? &ctl->head : &ctl->seg_head[q.seg], 1);
}

// The item of a claim, moving on to the next range while the current one
// is empty; n_items when every range is.
__device__ int queue_resolve(Control* ctl, QueueCursor& q, int raw, int n_top, int n_items,
                             bool local) {
    for (;;) {
        if (q.phase == 0) {
            if (raw < n_top) return raw;
            if (!local) return n_items;
            q.phase = 1;
        } else {
            const int64_t span = int64_t(n_items) - n_top;
            const int lo = n_top + int(span * q.seg / kXcd);
            const int hi = n_top + int(span * (q.seg + 1) / kXcd);
            if (raw < hi - lo) return lo + raw;
            if (++q.tries == kXcd) return n_items;
            q.seg = (q.seg + 1) % kXcd;
        }
        raw = atomicAdd(&ctl->seg_head[q.seg], 1);
    }
}

// Register slots of a work item's sinks: the active sinks of even index
// fill slots 0..7 in order and those of odd index slots 8..15, so that the
// sinks of a bucket split evenly between the two halves of the slot range
// (the split last PC chunk below gives each half of the wavefront one
// half), only active sinks are evaluated, and a sink's half (its index's
// parity) is the same with or without a mask: its sums then see the same
// operations in the same lanes, so a masked compute gives the bits of the
// full one.  mask: bit k = sink k is active (bit 0 of each pair even).
__device__ __forceinline__ int slot_rank_bit(uint32_t m, int r) {
    // index of the r-th (from 0) set bit of m, 16 if there is none
    for (int t = 0; t < kBucket / 2 - 1; ++t)
        if (t < r) m &= m - 1u;
    return m ? __builtin_ctz(m) : kBucket;
}

// Persistent PP + PC kernel.  One wavefront per work item (a sink bucket
// of up to 16 particles).  The sink particles are wave-uniform (scalar
// registers); lanes own sources: PP source particles expanded into LDS,
// PC cells' coefficient records in vector registers.  Each lane keeps
// 16 x 4 partial sums; a transposing butterfly reduction leaves lane l
// with component l&3 of the sink in slot l>>2.
template <int kChunk, int kWaves, bool kPrefetch>
__global__ void __launch_bounds__(kWave)
    __attribute__((amdgpu_waves_per_eu(kWaves, 8))) k_interact(RunArgs a) {
    static_assert(kChunk >= 1 && kChunk <= kWave, "a PP fill uses one entry per lane");
    constexpr int kLdsSrc = kChunk * kBucket;  // source particles per fill
    __shared__ float4 lds[kLdsSrc];
    __shared__ int4 etab[kChunk];    // per PP entry of a fill: LDS base, count, first
    __shared__ float4 edel[kChunk];  // per PP entry of a fill: source-sink offset
    const int lane = threadIdx.x;
    // fixed by earlier kernels
    const int n_items = __builtin_amdgcn_readfirstlane(
        __atomic_load_n(&a.ctl->n_items, __ATOMIC_RELAXED));
    const int n_top =
        __builtin_amdgcn_readfirstlane(__atomic_load_n(&a.ctl->n_top, __ATOMIC_RELAXED));
    const bool local =
        __builtin_amdgcn_readfirstlane(__atomic_load_n(&a.ctl->order_local, __ATOMIC_RELAXED));
    // single-wave blocks go to the dies in turn: block b runs on die b mod 8
    QueueCursor qc{0, int(blockIdx.x % kXcd), 0};
    int item = 0;
    if (lane == 0) item = queue_resolve(a.ctl, qc, queue_issue(a.ctl, qc), n_top, n_items, local);
    item = __builtin_amdgcn_readfirstlane(__shfl(item, 0));
    // the kernel's span on the device wall clock: from the first claim to the
    // exit of the last wave (every wave exits right after its last item)
    if (item == 0 && lane == 0) a.ctl->t_k0 = (unsigned long long)wall_clock64();
    for (;;) {
        if (item >= n_items) break;
        // claim the next queue slot now; its latency hides behind this item
        int next = 0;
        if (lane == 0) next = queue_issue(a.ctl, qc);
        const int b = load_uniform(a.items, item);
        const BucketWork wk = load_uniform(a.work, b);
        const int first = wk.first;
        const int nsink = wk.nsink;
        if (nsink <= 0) {
            if (lane == 0) next = queue_resolve(a.ctl, qc, next, n_top, n_items, local);
            item = __builtin_amdgcn_readfirstlane(__shfl(next, 0));
            continue;
        }
        // the sink bucket's centre (double; its cell was checked when staged)
        const int64_t sc = load_uniform(a.bucket_cell, b);
        const double Cx = 0.5 * (load_uniform(a.bbox, 6 * sc) + load_uniform(a.bbox, 6 * sc + 3));
        const double Cy =
            0.5 * (load_uniform(a.bbox, 6 * sc + 1) + load_uniform(a.bbox, 6 * sc + 4));
        const double Cz =
            0.5 * (load_uniform(a.bbox, 6 * sc + 2) + load_uniform(a.bbox, 6 * sc + 5));

        // The bucket's sink particles are wave-uniform.  A 2-wave variant
        // without the PC prefetch has vector registers to spare (the sinks
        // take 48 of them, 223 in all): a vector load keeps them there and
        // leaves the scalar registers to the kernel's arguments, which
        // otherwise spill into vector lanes and are read back in every chunk.
        // The other variants (168 vector registers at most with 3 waves, the
        // prefetch's 44 more with 2) read them through the constant address
        // space as scalar loads into scalar registers.
        constexpr bool kSinksInVgprs = kWaves == 2 && !kPrefetch;
        constexpr int kHalf = kBucket / 2;
        uint32_t me, mo;  // active sinks of even and of odd index
        {
            const bool on = lane < nsink && (a.active == nullptr || a.active[first + lane]);
            const uint32_t m = uint32_t(__ballot(on)) & 0xFFFFu;
            me = __builtin_amdgcn_readfirstlane(m & 0x5555u);
            mo = __builtin_amdgcn_readfirstlane(m & 0xAAAAu);
        }
        const int n_even = __builtin_popcount(me), n_odd = __builtin_popcount(mo);
        const int k_any = __builtin_ctz(me | mo | 0x10000u);  // a sink for the empty slots
        float sx[kBucket], sy[kBucket], sz[kBucket];
        {
            uint32_t re = me, ro = mo;
#pragma unroll
            for (int i = 0; i < kBucket; ++i) {
                uint32_t& r = i < kHalf ? re : ro;
                const int k = r ? __builtin_ctz(r) : k_any;
                r &= r - 1u;
                const int p = first + (k < nsink ? k : 0);
                const float4 q = kSinksInVgprs ? a.pdat[p] : load_uniform(a.pdat, p);
                sx[i] = q.x;
                sy[i] = q.y;
                sz[i] = q.z;
            }
        }
        Acc4 acc[kBucket];
#pragma unroll
        for (int i = 0; i < kBucket; ++i) acc[i] = Acc4{0.f, 0.f, 0.f, 0.f};

        if (a.parts & MGRAV_PART_PP) {
            const int64_t e0 = wk.pp0, e1 = wk.pp1;
            for (int64_t c0 = e0; c0 < e1; c0 += kChunk) {
                const int64_t e = c0 + lane;
                int cnt = 0, sfirst = 0;
                float4 ent = make_float4(0.f, 0.f, 0.f, 0.f);
                // lanes beyond the chunk stay empty: at most kChunk * 16
                // source particles go to LDS per fill
                if (lane < kChunk && e < e1) {
                    ent = a.ppent[e];
                    const uint32_t bits = __float_as_uint(ent.w);
                    sfirst = int(bits & 0x07FFFFFFu);
                    cnt = int(bits >> 27);
                }
                const int incl = wave_incl_scan(cnt, lane);
                const int total = __builtin_amdgcn_readfirstlane(__shfl(incl, kWave - 1));
                const int base = incl - cnt;
                // Cooperative copy of the chunk's source particles into LDS:
                // the entry table goes to LDS, then each step moves 4 entries
                // (16 lanes each, one particle per lane; an entry's particles
                // are contiguous).  Four steps are unrolled with unconditional
                // loads (inactive lanes read particle 0) so that four loads per
                // lane are in flight at once.
                if (lane < kChunk) {
                    etab[lane] = make_int4(base, cnt, sfirst, 0);
                    edel[lane] = ent;
                }
                __syncthreads();
                const int nent = int(e1 - c0 < kChunk ? e1 - c0 : kChunk);
                const int eg = lane >> 4, ek = lane & 15;
                for (int j0 = 0; j0 < nent; j0 += 16) {
                    float4 q[4];
                    int4 tb[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int e = j0 + 4 * u + eg;
                        tb[u] = e < nent ? etab[e] : make_int4(0, 0, 0, 0);
                        const int src = ek < tb[u].y ? tb[u].z + ek : 0;
                        q[u] = a.pdat[src];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int e = j0 + 4 * u + eg;
                        if (ek < tb[u].y) {
                            const float4 d = edel[e];
                            lds[tb[u].x + ek] =
                                make_float4(q[u].x + d.x, q[u].y + d.y, q[u].z + d.z, q[u].w);
                        }
                    }
                }
                __syncthreads();
                // two sources per lane while two full rows remain (a sink's
                // scalar operands then serve two interactions), then one
                int t0 = 0;
                for (; t0 + 2 * kWave <= total; t0 += 2 * kWave) {
                    const float4 s = lds[t0 + lane];
                    const float4 s2 = lds[t0 + kWave + lane];
                    const int ne = sink_count(n_even), no = sink_count(n_odd);
#pragma unroll
                    for (int i = 0; i < kBucket; ++i)
                        if (i < kHalf ? i < ne : i - kHalf < no) {
                            pp_one(s.x, s.y, s.z, s.w, sx[i], sy[i], sz[i], a.eps2, acc[i]);
                            pp_one(s2.x, s2.y, s2.z, s2.w, sx[i], sy[i], sz[i], a.eps2, acc[i]);
                        }
                }
                for (; t0 < total; t0 += kWave) {
                    const int t = t0 + lane;
                    // padding lanes: a massless source at the bucket centre (finite, adds 0)
                    const float4 s = t < total ? lds[t] : make_float4(0.f, 0.f, 0.f, 0.f);
                    const int ne = sink_count(n_even), no = sink_count(n_odd);
#pragma unroll
                    for (int i = 0; i < kBucket; ++i)
                        if (i < kHalf ? i < ne : i - kHalf < no)
                            pp_one(s.x, s.y, s.z, s.w, sx[i], sy[i], sz[i], a.eps2, acc[i]);
                }
                __syncthreads();
            }
        }
        if (a.parts & MGRAV_PART_PC) {
            const int64_t f0 = wk.pc0, f1 = wk.pc1;
            if constexpr (kPrefetch) {
                // the next chunk's records load while this one computes
                // (44 more registers: the 2-wave variants have them)
                // (load_pc reads entry f1 - 1 for lanes past the end, so it
                // is called only for a non-empty list)
                float rn[kRec], nx = 0.f, ny = 0.f, nz = 0.f;
                if (f0 < f1) load_pc(a, f0 + lane, f1, Cx, Cy, Cz, rn, nx, ny, nz);
                for (int64_t c0 = f0; c0 < f1; c0 += kWave) {
                    float r[kRec];
#pragma unroll
                    for (int i = 0; i < kRec; ++i) r[i] = rn[i];
                    const float cx = nx, cy = ny, cz = nz;
                    if (c0 + kWave < f1)
                        load_pc(a, c0 + kWave + lane, f1, Cx, Cy, Cz, rn, nx, ny, nz);
                    const float t = r[kRec - 1];
                    const float eps2t = a.eps2 * t * t;
                    const int ne = sink_count(n_even), no = sink_count(n_odd);
#pragma unroll
                    for (int i = 0; i < kBucket; ++i)
                        if (i < kHalf ? i < ne : i - kHalf < no)
                            pc_one(r, t, cx, cy, cz, sx[i], sy[i], sz[i], eps2t, acc[i]);
                }
            } else {
                // In the 3-wave variants a last chunk of at most 32 entries is
                // split: both halves of the wavefront take all its entries, the
                // lower half for the sinks in slots 0..7 and the upper half for
                // those in 8..15, which halves its passes over the sinks.  (In
                // the 2-wave variants the split code measured 4-6 % slower.)
                constexpr bool kSplitTail = kWaves == 3;
                const int rem = int((f1 - f0) & (kWave - 1));
                const bool split = kSplitTail && rem > 0 && rem <= kWave / 2 && nsink >= 2;
                const int64_t fend = split ? f1 - rem : f1;
                for (int64_t c0 = f0; c0 < fend; c0 += kWave) {
                    float r[kRec], cx, cy, cz;
                    load_pc(a, c0 + lane, f1, Cx, Cy, Cz, r, cx, cy, cz);
                    const float t = r[kRec - 1];
                    const float eps2t = a.eps2 * t * t;
                    const int ne = sink_count(n_even), no = sink_count(n_odd);
#pragma unroll
                    for (int i = 0; i < kBucket; ++i)
                        if (i < kHalf ? i < ne : i - kHalf < no)
                            pc_one(r, t, cx, cy, cz, sx[i], sy[i], sz[i], eps2t, acc[i]);
                }
                if constexpr (kSplitTail) if (split) {
                    const bool upper = lane >= kWave / 2;
                    float r[kRec], cx, cy, cz;
                    // entries at or past f1 (lanes beyond rem in each half) add zero
                    load_pc(a, fend + (lane & (kWave / 2 - 1)), f1, Cx, Cy, Cz, r, cx, cy, cz);
                    const float t = r[kRec - 1];
                    const float eps2t = a.eps2 * t * t;
                    const int ne = sink_count(n_even), no = sink_count(n_odd);
#pragma unroll
                    for (int j = 0; j < kHalf; ++j)
                        if (j < ne || j < no) {  // either slot j or j + 8 may be empty
                            const bool lo = j < ne, hi = j < no;
                            const float px = upper ? sx[j + kHalf] : sx[j];
                            const float py = upper ? sy[j + kHalf] : sy[j];
                            const float pz = upper ? sz[j + kHalf] : sz[j];
                            Acc4 A = upper ? acc[j + kHalf] : acc[j];
                            pc_one(r, t, cx, cy, cz, px, py, pz, eps2t, A);
                            if (!upper) {
                                if (lo) acc[j] = A;
                            } else if (hi) {
                                acc[j + kHalf] = A;
                            }
                        }
                }
            }
        }

        // transposing butterfly: v[4*i + c] (slot i) summed over lanes -> lane 4*i + c
        float v[4 * kBucket];
#pragma unroll
        for (int i = 0; i < kBucket; ++i) {
            v[4 * i] = acc[i].x;
            v[4 * i + 1] = acc[i].y;
            v[4 * i + 2] = acc[i].z;
            v[4 * i + 3] = acc[i].p;
        }
#pragma unroll
        for (int o = kWave / 2; o >= 1; o >>= 1) {
            const bool up = (lane & o) != 0;
#pragma unroll
            for (int k = 0; k < o; ++k) {
                const float keep = up ? v[k + o] : v[k];
                const float send = up ? v[k] : v[k + o];
                v[k] = keep + __shfl_xor(send, o);
            }
        }
        const int slot = lane >> 2, comp = lane & 3;
        const int i = slot_rank_bit(slot < kHalf ? me : mo, slot & (kHalf - 1));
        if (i < nsink) {  // an active sink (16: an empty slot)
            const int p = first + i;
            {
                float val = v[0];
                if (comp == 3 && (a.parts & MGRAV_PART_PP) && wk.self) {
                    // remove the self pair, which entered as -m_i / eps
                    const float4 q = a.pdat[p];
                    const float D = fmaf(0.f, 0.f, fmaf(0.f, 0.f, fmaf(0.f, 0.f, a.eps2)));
                    val += q.w * __builtin_amdgcn_rsqf(D);
                }
                float* out = comp == 3 ? a.pot : a.acc + int64_t(comp) * a.n;
                out[p] = val;
            }
        }
        if (lane == 0) next = queue_resolve(a.ctl, qc, next, n_top, n_items, local);
        item = __builtin_amdgcn_readfirstlane(__shfl(next, 0));
    }
    if (lane == 0 && atomicAdd(&a.ctl->waves_done, 1) == int(gridDim.x) - 1)
        a.ctl->t_k1 = (unsigned long long)wall_clock64();
}

// The compiled variants of the PP + PC kernel, by index.
#define MGRAV_VARIANT(V) k_interact<kVariantChunk[V], kVariantWaves[V], kVariantPrefetch[V]>

const void* interact_kernel(int v) {
    switch (v) {
        case 1: return reinterpret_cast<const void*>(&MGRAV_VARIANT(1));
        case 2: return reinterpret_cast<const void*>(&MGRAV_VARIANT(2));
        case 3: return reinterpret_cast<const void*>(&MGRAV_VARIANT(3));
        case 4: return reinterpret_cast<const void*>(&MGRAV_VARIANT(4));
        case 5: return reinterpret_cast<const void*>(&MGRAV_VARIANT(5));
        default: return reinterpret_cast<const void*>(&MGRAV_VARIANT(0));
    }
}

void launch_interact(int v, dim3 grid, hipStream_t stream, const RunArgs& r) {
    switch (v) {
        case 1: hipLaunchKernelGGL((MGRAV_VARIANT(1)), grid, dim3(kWave), 0, stream, r); break;
        case 2: hipLaunchKernelGGL((MGRAV_VARIANT(2)), grid, dim3(kWave), 0, stream, r); break;
        case 3: hipLaunchKernelGGL((MGRAV_VARIANT(3)), grid, dim3(kWave), 0, stream, r); break;
        case 4: hipLaunchKernelGGL((MGRAV_VARIANT(4)), grid, dim3(kWave), 0, stream, r); break;
        case 5: hipLaunchKernelGGL((MGRAV_VARIANT(5)), grid, dim3(kWave), 0, stream, r); break;
        default: hipLaunchKernelGGL((MGRAV_VARIANT(0)), grid, dim3(kWave), 0, stream, r); break;
    }
}
#undef MGRAV_VARIANT
static_assert(kNumVariants == 6, "interact_kernel and launch_interact list every variant");
static_assert(kQueueAuto == MGRAV_QUEUE_AUTO && kQueueLpt == MGRAV_QUEUE_LPT &&
                  kQueueLocal == MGRAV_QUEUE_LOCAL,
              "queue orders match the header");

// ---------------------------------------------------------------------
// Ewald correction (FP64)
// ---------------------------------------------------------------------
struct EwaldArgs {
    int64_t n;
    PosIn pin;
    const double* __restrict__ mom;   // root = cell 0
    const double* __restrict__ com;   // root = cell 0
    const uint8_t* __restrict__ active;
    double* table;                    // workspace: [0..43] coefficients, [64..] k-table
    float* __restrict__ acc;
    float* __restrict__ pot;
    double L, alpha;
    int real_layers, h2max, hmax, order, accumulate;
    // Judge of the surrogate.  With `sample` set, index j < n_sample stands
    // for particle j * stride, and its exact acceleration, a valid flag and
    // the PP + PC acceleration before the correction go to
    // sample[kSampleRec * j + 0..7] instead of acc and pot.  With `gate`
    // set, the kernel does nothing unless the judge chose the exact path.
    int64_t stride, n_sample;
    double* sample;
    const Control* gate;
    // With `list` set (a mask is in use): the particles are list[j] for
    // j < ctl->n_list, taken by a grid-stride loop over a bounded grid.
    const int* list;
    const Control* ctl;
    // With `ewbuf` set (the correction overlaps the PP + PC kernel): the
    // correction goes to ewbuf[4 i + 0..3] (acceleration, potential) in
    // double, and k_ewald_add adds it once the PP + PC sums are written.
    double* ewbuf;
};

// Packed symmetric components of orders 2, 3, 4: multiplicity (number of
// index orderings) and axes.
__constant__ int c_m2[6] = {1, 2, 2, 1, 2, 1};
__constant__ int c_ax2[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
__constant__ int c_m3[10] = {1, 3, 3, 3, 6, 3, 1, 3, 3, 1};
__constant__ int c_ax3[10][3] = {{0, 0, 0}, {0, 0, 1}, {0, 0, 2}, {0, 1, 1}, {0, 1, 2},
                                 {0, 2, 2}, {1, 1, 1}, {1, 1, 2}, {1, 2, 2}, {2, 2, 2}};
__constant__ int c_m4[15] = {1, 4, 4, 6, 12, 6, 4, 12, 12, 4, 1, 4, 6, 4, 1};
__constant__ int c_ax4[15][4] = {{0, 0, 0, 0}, {0, 0, 0, 1}, {0, 0, 0, 2}, {0, 0, 1, 1},
                                 {0, 0, 1, 2}, {0, 0, 2, 2}, {0, 1, 1, 1}, {0, 1, 1, 2},
                                 {0, 1, 2, 2}, {0, 2, 2, 2}, {1, 1, 1, 1}, {1, 1, 1, 2},
                                 {1, 1, 2, 2}, {1, 2, 2, 2}, {2, 2, 2, 2}};

#include "erfcx_poly.inc"

// The power series of the near images' g_5 in Horner form: coefficient j
// is (-1)^j / (j! (2j + 11)) (the factorial an exact integer literal, one
// rounding each); 26 terms reach double precision for x <= 2.  And
// 1/(2n + 1) for the downward recurrence: constants, so the loops below
// divide nothing.
constexpr int kEwSeriesTerms = 26;
__constant__ double c_ew_series[kEwSeriesTerms] = {
    1.0 / (1.0 * 11), -1.0 / (1.0 * 13),
    1.0 / (2.0 * 15), -1.0 / (6.0 * 17),
    1.0 / (24.0 * 19), -1.0 / (120.0 * 21),
    1.0 / (720.0 * 23), -1.0 / (5040.0 * 25),
    1.0 / (40320.0 * 27), -1.0 / (362880.0 * 29),
    1.0 / (3628800.0 * 31), -1.0 / (39916800.0 * 33),
    1.0 / (479001600.0 * 35), -1.0 / (6227020800.0 * 37),
    1.0 / (87178291200.0 * 39), -1.0 / (1307674368000.0 * 41),
    1.0 / (20922789888000.0 * 43), -1.0 / (355687428096000.0 * 45),
    1.0 / (6402373705728000.0 * 47), -1.0 / (121645100408832000.0 * 49),
    1.0 / (2432902008176640000.0 * 51), -1.0 / (51090942171709440000.0 * 53),
    1.0 / (1124000727777607680000.0 * 55), -1.0 / (25852016738884976640000.0 * 57),
    1.0 / (620448401733239439360000.0 * 59), -1.0 / (15511210043330985984000000.0 * 61)};
__constant__ double c_ew_inv_2n1[6] = {1.0 / 1, 1.0 / 3, 1.0 / 5, 1.0 / 7, 1.0 / 9, 1.0 / 11};

// Constants of the radial functions, written by k_ewald_setup after the
// k-space rows and read per image through scalar loads (kept in memory so
// that they do not occupy vector registers across the image loop).
constexpr int kEwCoef = 64 + 8 * kMaxHalfK;
constexpr int kEwSeries = 0;                     // the series coefficients
constexpr int kEwInv2n1 = kEwSeries + kEwSeriesTerms;  // 1 / (2n + 1), n < 6
constexpr int kEwErfcx = kEwInv2n1 + 6;          // erfcx polynomial, kErfcxDeg + 1 values
constexpr int kEwK = kEwErfcx + 19;              // k_m = (-2 alpha^2)^m / (alpha sqrt(pi)), m < 6
constexpr int kEwG5 = kEwK + 6;   // 2 alpha / sqrt(pi) (-32 alpha^10)
constexpr int kEwAl2 = kEwG5 + 1; // alpha^2
constexpr int kEwTs = kEwAl2 + 1; // (2 / alpha) kErfcxScale
constexpr int kEwCoefCount = kEwTs + 1;
static_assert(kErfcxDeg + 1 == 19, "erfcx block size");
static_assert(kEwCoefCount <= kEwCoefSlots, "radial constants overflow their block");

// Root coefficients in unit-box scaling (order k scaled by L^-k), masked
// by the requested order, and the k-space table for the half space of
// wave vectors (each row stands for h and -h).  One block: the candidate
// vectors h (hx >= 0, |hy|, |hz| <= hmax, in lexicographic order) are
// taken 256 at a time, one per thread, and compacted by a block prefix
// sum, so the table order does not depend on the thread count.
constexpr int kSetupThreads = 256;
__global__ void __launch_bounds__(kSetupThreads) k_ewald_setup(EwaldArgs a) {
    const double* m = a.mom;
    // unit-box scaling by multiplication (one thread runs this part: no
    // divisions in its chain)
    const double iL = 1.0 / a.L, iL2 = iL * iL, iL3 = iL2 * iL, iL4 = iL3 * iL;
    if (threadIdx.x == 0) {
        double r[kRec];
        r[0] = m[0];
        r[1] = 0.5 * (m[1] + m[4] + m[6]) * iL2;
        for (int i = 0; i < 6; ++i) r[2 + i] = 0.5 * m[1 + i] * iL2;
        r[8] = -0.5 * (m[7] + m[10] + m[12]) * iL3;
        r[9] = -0.5 * (m[8] + m[13] + m[15]) * iL3;
        r[10] = -0.5 * (m[9] + m[14] + m[16]) * iL3;
        r[11] = 0.125 * (m[17] + m[27] + m[31] + 2.0 * (m[20] + m[22] + m[29])) * iL4;
        for (int i = 0; i < 10; ++i) r[12 + i] = -m[7 + i] * (1.0 / 6.0) * iL3;
        r[22] = 0.25 * (m[17] + m[20] + m[22]) * iL4;
        r[23] = 0.25 * (m[18] + m[23] + m[25]) * iL4;
        r[24] = 0.25 * (m[19] + m[24] + m[26]) * iL4;
        r[25] = 0.25 * (m[20] + m[27] + m[29]) * iL4;
        r[26] = 0.25 * (m[21] + m[28] + m[30]) * iL4;
        r[27] = 0.25 * (m[22] + m[29] + m[31]) * iL4;
        for (int i = 0; i < 15; ++i) r[28 + i] = m[17 + i] * (1.0 / 24.0) * iL4;
        r[43] = 0.0;
        if (a.order < 4) {  // drop orders 3 and 4 (and their traces)
            for (int i = 8; i < 11; ++i) r[i] = 0.0;
            r[11] = 0.0;
            for (int i = 12; i < kRec; ++i) r[i] = 0.0;
        }
        if (a.order < 2) {
            for (int i = 1; i < kRec; ++i) r[i] = 0.0;
        }
        for (int i = 0; i < kRec; ++i) a.table[i] = r[i];
        a.table[45] = m[0] * 3.14159265358979323846 / (a.alpha * a.alpha);  // background
    }

    // k-space: phi += -(1/pi) sum_h c_h (A_h cos th + B_h sin th), th = 2 pi h.r,
    // c_h = exp(-pi^2 h^2 / alpha^2) / h^2, A_h = M - 2 pi^2 Q2 + 2 pi^4/3 Q4,
    // B_h = -4 pi^3/3 Q3, Q_k = M_k[h..h] (unit-box moments).
    const double PI = 3.14159265358979323846;
    const int hm = a.hmax, side = 2 * hm + 1;
    const int n_cand = (hm + 1) * side * side;
    __shared__ int wave_total[kSetupThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    double* tab = a.table + 64;
    int nk = 0;
    for (int c0 = 0; c0 < n_cand; c0 += kSetupThreads) {
        const int cidx = c0 + int(threadIdx.x);
        int hx = 0, hy = 0, hz = 0;
        bool keep = false;
        if (cidx < n_cand) {
            hx = cidx / (side * side);
            hy = (cidx / side) % side - hm;
            hz = cidx % side - hm;
            const int h2 = hx * hx + hy * hy + hz * hz;
            keep = h2 != 0 && h2 <= a.h2max && !(hx == 0 && (hy < 0 || (hy == 0 && hz < 0)));
        }
        const unsigned long long mask = __ballot(keep);
        const int in_wave = __popcll(mask & ((1ull << lane) - 1ull));
        if (lane == 0) wave_total[w] = __popcll(mask);
        __syncthreads();
        int before = nk;
        for (int q = 0; q < w; ++q) before += wave_total[q];
        int chunk = 0;
        for (int q = 0; q < kSetupThreads / kWave; ++q) chunk += wave_total[q];
        __syncthreads();  // wave_total is rewritten by the next chunk
        const int slot = before + in_wave;
        if (keep && slot < kMaxHalfK) {
            const int h2 = hx * hx + hy * hy + hz * hz;
            const double h[3] = {double(hx), double(hy), double(hz)};
            double Q2 = 0, Q3 = 0, Q4 = 0;
            for (int q = 0; q < 6; ++q)
                Q2 += c_m2[q] * m[1 + q] * iL2 * h[c_ax2[q][0]] * h[c_ax2[q][1]];
            for (int q = 0; q < 10; ++q)
                Q3 += c_m3[q] * m[7 + q] * iL3 * h[c_ax3[q][0]] * h[c_ax3[q][1]] * h[c_ax3[q][2]];
            for (int q = 0; q < 15; ++q)
                Q4 += c_m4[q] * m[17 + q] * iL4 * h[c_ax4[q][0]] * h[c_ax4[q][1]] *
                      h[c_ax4[q][2]] * h[c_ax4[q][3]];
            if (a.order < 4) Q3 = Q4 = 0.0;
            if (a.order < 2) Q2 = 0.0;
            const double A = m[0] - 2.0 * PI * PI * Q2 + 2.0 * PI * PI * PI * PI / 3.0 * Q4;
            const double B = -4.0 * PI * PI * PI / 3.0 * Q3;
            const double cc = exp(-PI * PI * h2 / (a.alpha * a.alpha)) / h2;
            double* row = tab + 8 * slot;
            row[0] = h[0];
            row[1] = h[1];
            row[2] = h[2];
            row[3] = -(2.0 / PI) * cc * A;  // cos coefficient of phi (pair doubled)
            row[4] = -(2.0 / PI) * cc * B;  // sin coefficient of phi
            row[5] = -4.0 * cc * A;         // sin coefficient of acc / h
            row[6] = 4.0 * cc * B;          // cos coefficient of acc / h
            // the axis indices for the phase tables of k_ewald
            reinterpret_cast<int64_t*>(row)[7] =
                int64_t(hx) | (int64_t(hy + hm) << 8) | (int64_t(hz + hm) << 16);
        }
        nk += chunk;
    }
    if (threadIdx.x == 0) a.table[44] = double(nk < kMaxHalfK ? nk : kMaxHalfK);
    // constants of the radial functions
    double* cf = a.table + kEwCoef;
    const int t = threadIdx.x;
    if (t < kEwSeriesTerms) cf[kEwSeries + t] = c_ew_series[t];
    if (t < 6) cf[kEwInv2n1 + t] = c_ew_inv_2n1[t];
    if (t <= kErfcxDeg) cf[kEwErfcx + t] = c_erfcx[t];
    if (t == 0) {
        const double SQRT_PI = 1.77245385090551602729;
        const double al = a.alpha, al2 = al * al;
        double k = 1.0 / (al * SQRT_PI);
        cf[kEwK] = k;
        for (int m = 1; m < 6; ++m) {
            k = k * (-2.0 * al2);
            cf[kEwK + m] = k;
        }
        cf[kEwG5] = 2.0 * al / SQRT_PI * (-32.0 * al2 * al2 * al2 * al2 * al2);
        cf[kEwAl2] = al2;
        cf[kEwTs] = (2.0 / al) * kErfcxScale;
    }
}


struct TableRec {
    const double* t;
    __device__ double operator[](int i) const { return load_uniform(t, i); }
};


// Radial derivatives g_n = ((1/r) d/dr)^n of erf(alpha r)/r, n = 0..5, for
// the near images (|n_a| <= 1), unit box.  With alpha r < sqrt(2): g_5 from
// its power series
//   g_5 = (2 alpha/sqrt(pi)) (-2 alpha^2)^5 sum_j (-x)^j / (j! (2j + 11)),
//   x = alpha^2 r^2,
// the rest by the downward recurrence g_n = -(r^2 g_{n+1} + k_{n+1} e^{-x})
// / (2n+1) with k_m = (-2 alpha^2)^m / (alpha sqrt(pi)); otherwise upward
// from the closed form (the same recurrence solved for g_{n+1}), with
// erf(z) = 1 - e^{-z^2} erfcx(z), erfcx from its polynomial in 2/z.
// E = exp(-alpha^2 r^2) is passed in (built from per-axis factors).
template <typename C>
__device__ __forceinline__ void ewald_radial_near(const C& c, double r2, double E, double g[6]) {
    const double x = c[kEwAl2] * r2;
    if (x < 2.0) {
        double sum = c[kEwSeries + kEwSeriesTerms - 1];
#pragma unroll
        for (int j = kEwSeriesTerms - 2; j >= 0; --j) sum = fma(sum, x, c[kEwSeries + j]);
        g[5] = c[kEwG5] * sum;
#pragma unroll
        for (int n = 4; n >= 0; --n)
            g[n] = -(r2 * g[n + 1] + c[kEwK + n + 1] * E) * c[kEwInv2n1 + n];
        return;
    }
    // 1/r from the hardware reciprocal square root refined by two Newton
    // steps y <- y (3 - r2 y^2) / 2 (each squares the relative error)
    double inv_r = __builtin_amdgcn_rsq(r2);
    inv_r = inv_r * fma(-0.5 * r2, inv_r * inv_r, 1.5);
    inv_r = inv_r * fma(-0.5 * r2, inv_r * inv_r, 1.5);
    const double inv_r2 = inv_r * inv_r;
    // beyond z = 6.5, e^{-z^2} erfcx(z) < 1e-19 and erf(z) = 1 in double
    double er = 1.0;
    if (x < 42.25) {  // z < 6.5
        const double t = fma(c[kEwTs], inv_r, kErfcxShift);
        double h = c[kEwErfcx + kErfcxDeg];
#pragma unroll
        for (int k = kErfcxDeg - 1; k >= 0; --k) h = fma(h, t, c[kEwErfcx + k]);
        er = fma(-E, h, 1.0);
    }
    g[0] = er * inv_r;
#pragma unroll
    for (int n = 0; n < 5; ++n)
        g[n + 1] = -(double(2 * n + 1) * g[n] + c[kEwK + n + 1] * E) * inv_r2;
}

// The same for the outer real-space shells, of -erfc(alpha r)/r.
template <typename C>
__device__ void ewald_radial_far(const C& c, double r2, double alpha, double g[6]) {
    const double E = exp(-c[kEwAl2] * r2);
    double inv_r = __builtin_amdgcn_rsq(r2);
    inv_r = inv_r * fma(-0.5 * r2, inv_r * inv_r, 1.5);
    inv_r = inv_r * fma(-0.5 * r2, inv_r * inv_r, 1.5);
    const double inv_r2 = inv_r * inv_r;
    double e = erfc(alpha * r2 * inv_r) * inv_r;
    g[0] = -e;
#pragma unroll
    for (int n = 0; n < 5; ++n) {
        e = (c[kEwK + n + 1] * E - double(2 * n + 1) * e) * inv_r2;
        g[n + 1] = -e;
    }
}

// The same constants computed in registers, for kernels without the table
// (the training-data kernel).
struct RadialConstsLocal {
    double kk[6], g5, al2, ts;
    __device__ explicit RadialConstsLocal(double al) {
        const double SQRT_PI = 1.77245385090551602729;
        al2 = al * al;
        kk[0] = 1.0 / (al * SQRT_PI);
        for (int m = 1; m < 6; ++m) kk[m] = kk[m - 1] * (-2.0 * al2);
        g5 = 2.0 * al / SQRT_PI * (-32.0 * al2 * al2 * al2 * al2 * al2);
        ts = (2.0 / al) * kErfcxScale;
    }
    __device__ double operator[](int i) const {
        if (i < kEwInv2n1) return c_ew_series[i - kEwSeries];
        if (i < kEwErfcx) return c_ew_inv_2n1[i - kEwInv2n1];
        if (i < kEwK) return c_erfcx[i - kEwErfcx];
        if (i < kEwG5) return kk[i - kEwK];
        if (i == kEwG5) return g5;
        if (i == kEwAl2) return al2;
        return ts;
    }
};

__device__ void ewald_radial(double r2, double alpha, bool near, double g[6]) {
    const RadialConstsLocal c(alpha);
    if (near)
        ewald_radial_near(c, r2, exp(-c[kEwAl2] * r2), g);
    else
        ewald_radial_far(c, r2, alpha, g);
}

// Dynamic LDS of k_ewald: per thread, 2 (hmax + 1) complex phase factors.
// Blocks of 128 threads up to hmax = 5 (24 KB; 16 KB at hmax = 3), 64 above
// (at most 18 KB at hmax = 8).
constexpr int kEwaldThreads = 128;
inline int ewald_threads(int hmax) { return hmax <= 5 ? kEwaldThreads : kEwaldThreads / 2; }
inline size_t ewald_lds_bytes(int hmax) {
    return sizeof(double2) * size_t(2 * (hmax + 1)) * size_t(ewald_threads(hmax));
}

// One image's terms, order by order into the sums: phi += sum_n g_n P_n,
// acc -= sum_n (g_{n+1} P_n R + g_n grad P_n), with the same grouping of
// the moments as multipole_terms (each order's intermediates die before
// the next order starts).
__device__ __forceinline__ void ewald_real_terms(const TableRec& r, double x, double y, double z,
                                                 const double (&g)[6], double& phi, double& ax,
                                                 double& ay, double& az) {
    double S = fma(g[2], r[1], g[1] * r[0]);
    phi = fma(g[1], r[1], fma(g[0], r[0], phi));
    const double xx = x * x, yy = y * y, zz = z * z;
    {
        const double h2x = r[2] * x + (r[3] * y + (r[4] * z + r[8]));
        const double h2y = r[3] * x + (r[5] * y + (r[6] * z + r[9]));
        const double h2z = r[4] * x + (r[6] * y + (r[7] * z + r[10]));
        const double P2 = x * h2x + y * h2y + z * h2z + r[11];
        phi = fma(g[2], P2, phi);
        S = fma(g[3], P2, S);
        ax -= g[2] * (2.0 * h2x - r[8]);
        ay -= g[2] * (2.0 * h2y - r[9]);
        az -= g[2] * (2.0 * h2z - r[10]);
    }
    {
        const double qxy = 2.0 * x * y, qxz = 2.0 * x * z, qyz = 2.0 * y * z;
        const double w4x = r[22] * x + r[23] * y + r[24] * z;
        const double w4y = r[23] * x + r[25] * y + r[26] * z;
        const double w4z = r[24] * x + r[26] * y + r[27] * z;
        const double h3x = r[12] * xx + (r[15] * yy + (r[17] * zz + (r[13] * qxy + (r[14] * qxz +
                           (r[16] * qyz + w4x)))));
        const double h3y = r[13] * xx + (r[18] * yy + (r[20] * zz + (r[15] * qxy + (r[16] * qxz +
                           (r[19] * qyz + w4y)))));
        const double h3z = r[14] * xx + (r[19] * yy + (r[21] * zz + (r[16] * qxy + (r[17] * qxz +
                           (r[20] * qyz + w4z)))));
        const double P3 = x * h3x + y * h3y + z * h3z;
        phi = fma(g[3], P3, phi);
        S = fma(g[4], P3, S);
        ax -= g[3] * (3.0 * h3x - w4x);
        ay -= g[3] * (3.0 * h3y - w4y);
        az -= g[3] * (3.0 * h3z - w4z);
    }
    {
        const double x3 = 3.0 * x, y3 = 3.0 * y, z3 = 3.0 * z;
        const double cxxx = xx * x, cxxy = xx * y3, cxxz = xx * z3, cxyy = yy * x3;
        const double cxyz = 2.0 * x * y * z3;
        const double cxzz = zz * x3, cyyy = yy * y, cyyz = yy * z3, cyzz = zz * y3, czzz = zz * z;
        const double v4x = r[28] * cxxx + r[29] * cxxy + r[30] * cxxz + r[31] * cxyy +
                           r[32] * cxyz + r[33] * cxzz + r[34] * cyyy + r[35] * cyyz +
                           r[36] * cyzz + r[37] * czzz;
        const double v4y = r[29] * cxxx + r[31] * cxxy + r[32] * cxxz + r[34] * cxyy +
                           r[35] * cxyz + r[36] * cxzz + r[38] * cyyy + r[39] * cyyz +
                           r[40] * cyzz + r[41] * czzz;
        const double v4z = r[30] * cxxx + r[32] * cxxy + r[33] * cxxz + r[35] * cxyy +
                           r[36] * cxyz + r[37] * cxzz + r[39] * cyyy + r[40] * cyyz +
                           r[41] * cyzz + r[42] * czzz;
        const double P4 = x * v4x + y * v4y + z * v4z;
        phi = fma(g[4], P4, phi);
        S = fma(g[5], P4, S);
        const double g44 = 4.0 * g[4];
        ax -= g44 * v4x;
        ay -= g44 * v4y;
        az -= g44 * v4z;
    }
    ax -= S * x;
    ay -= S * y;
    az -= S * z;
}

// The correction at particle i into acc and pot, or into the judge's
// sample record `out`.
__device__ __forceinline__ void ewald_particle(const EwaldArgs& a, int64_t i, double* out,
                                               double2* ew_lds) {
    const TableRec rec{a.table};
    const TableRec coef{a.table + kEwCoef};
    const double invL = 1.0 / a.L;
    double xi0, xi1, xi2;
    load_pos(a.pin, i, xi0, xi1, xi2);
    const double rx = (xi0 - a.com[0]) * invL;
    const double ry = (xi1 - a.com[1]) * invL;
    const double rz = (xi2 - a.com[2]) * invL;
    double phi = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
    const int R = a.real_layers;
    // exp(-alpha^2 |r - n|^2) of the 27 near images as products of per-axis
    // factors exp(-alpha^2 (r_a - n_a)^2), n_a in {-1, 0, 1}: 9 exponentials
    const double al2 = a.alpha * a.alpha;
    double fxa[3], fya[3], fza[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double dx = rx - (k - 1), dy = ry - (k - 1), dz = rz - (k - 1);
        fxa[k] = exp(-al2 * dx * dx);
        fya[k] = exp(-al2 * dy * dy);
        fza[k] = exp(-al2 * dz * dz);
    }
    const int Rn = R < 1 ? R : 1;
    for (int ix = -Rn; ix <= Rn; ++ix)
        for (int iy = -Rn; iy <= Rn; ++iy)
            for (int iz = -Rn; iz <= Rn; ++iz) {
                // reload the table values per image (scalar loads, cheap)
                // rather than keeping them live across the loop
                asm volatile("" ::: "memory");
                const double x = rx - ix, y = ry - iy, z = rz - iz;
                const double r2 = x * x + y * y + z * z;
                // wave-uniform selects, no indexed registers
                const double fx = ix < 0 ? fxa[0] : (ix == 0 ? fxa[1] : fxa[2]);
                const double fy = iy < 0 ? fya[0] : (iy == 0 ? fya[1] : fya[2]);
                const double fz = iz < 0 ? fza[0] : (iz == 0 ? fza[1] : fza[2]);
                double g[6];
                ewald_radial_near(coef, r2, fx * fy * fz, g);
                ewald_real_terms(rec, x, y, z, g, phi, ax, ay, az);
            }
    // outer shells (max |n_a| >= 2)
    for (int ix = -R; ix <= R; ++ix)
        for (int iy = -R; iy <= R; ++iy)
            for (int iz = -R; iz <= R; ++iz) {
                if (ix >= -1 && ix <= 1 && iy >= -1 && iy <= 1 && iz >= -1 && iz <= 1) continue;
                asm volatile("" ::: "memory");
                const double x = rx - ix, y = ry - iy, z = rz - iz;
                const double r2 = x * x + y * y + z * z;
                double g[6];
                ewald_radial_far(coef, r2, a.alpha, g);
                ewald_real_terms(rec, x, y, z, g, phi, ax, ay, az);
            }
    // k space over the table rows, which come in order of hx (then hy, hz).
    // The factor e^{i 2 pi hx x} advances in registers as hx grows; each
    // thread keeps e^{i 2 pi k r_a} for k = 0..hmax (y, z) in LDS (its own
    // column, built by repeated rotation), negative k by conjugation.
    const int hm = a.hmax, T = blockDim.x, tid = threadIdx.x;
    double2* ey = ew_lds;             // [hm + 1][T]
    double2* ez = ey + (hm + 1) * T;  // [hm + 1][T]
    double s1x, c1x;
    sincospi(2.0 * rx, &s1x, &c1x);
    {
        double s1, c1;
        sincospi(2.0 * ry, &s1, &c1);
        double c = 1.0, s = 0.0;
        ey[tid] = make_double2(1.0, 0.0);
        for (int k = 1; k <= hm; ++k) {
            const double t = c * c1 - s * s1;
            s = s * c1 + c * s1;
            c = t;
            ey[k * T + tid] = make_double2(c, s);
        }
        sincospi(2.0 * rz, &s1, &c1);
        c = 1.0;
        s = 0.0;
        ez[tid] = make_double2(1.0, 0.0);
        for (int k = 1; k <= hm; ++k) {
            const double t = c * c1 - s * s1;
            s = s * c1 + c * s1;
            c = t;
            ez[k * T + tid] = make_double2(c, s);
        }
    }
    const double* tab = a.table + 64;
    const int64_t* key = reinterpret_cast<const int64_t*>(tab);
    const int nk = int(load_uniform(a.table, 44));
    double cx = 1.0, sx = 0.0;
    int hx_at = 0;
    for (int q = 0; q < nk; ++q) {
        const int row = 8 * q;
        const int64_t kk = load_uniform(key, row + 7);  // hx | (hy + hm) << 8 | (hz + hm) << 16
        const int hx = int(kk & 0xff);
        for (; hx_at < hx; ++hx_at) {  // wave-uniform
            const double t = cx * c1x - sx * s1x;
            sx = sx * c1x + cx * s1x;
            cx = t;
        }
        const int jy = int((kk >> 8) & 0xff) - hm, jz = int((kk >> 16) & 0xff) - hm;
        double2 py = ey[(jy < 0 ? -jy : jy) * T + tid];
        double2 pz = ez[(jz < 0 ? -jz : jz) * T + tid];
        if (jy < 0) py.y = -py.y;
        if (jz < 0) pz.y = -pz.y;
        const double cxy = cx * py.x - sx * py.y, sxy = sx * py.x + cx * py.y;
        const double c = cxy * pz.x - sxy * pz.y, s = sxy * pz.x + cxy * pz.y;
        phi += load_uniform(tab, row + 3) * c + load_uniform(tab, row + 4) * s;
        const double f = load_uniform(tab, row + 5) * s + load_uniform(tab, row + 6) * c;
        ax += f * load_uniform(tab, row);
        ay += f * load_uniform(tab, row + 1);
        az += f * load_uniform(tab, row + 2);
    }
    phi += load_uniform(a.table, 45);
    // physical units: potential / L, acceleration / L^2
    phi *= invL;
    const double invL2 = invL * invL;
    ax *= invL2;
    ay *= invL2;
    az *= invL2;
    float* px = a.acc + i;
    float* py = a.acc + a.n + i;
    float* pz = a.acc + 2 * a.n + i;
    if (out) {
        out[0] = ax;
        out[1] = ay;
        out[2] = az;
        out[3] = 1.0;
        out[4] = a.accumulate ? double(*px) : 0.0;
        out[5] = a.accumulate ? double(*py) : 0.0;
        out[6] = a.accumulate ? double(*pz) : 0.0;
        out[7] = 0.0;
    } else if (a.ewbuf) {
        double* e = a.ewbuf + 4 * i;
        e[0] = ax;
        e[1] = ay;
        e[2] = az;
        e[3] = phi;
    } else if (a.accumulate) {
        *px = float(double(*px) + ax);
        *py = float(double(*py) + ay);
        *pz = float(double(*pz) + az);
        a.pot[i] = float(double(a.pot[i]) + phi);
    } else {
        *px = float(ax);
        *py = float(ay);
        *pz = float(az);
        a.pot[i] = float(phi);
    }
}

// One thread per particle (or per sampled particle of the judge).
__global__ void __launch_bounds__(kEwaldThreads) k_ewald(EwaldArgs a) {
    extern __shared__ double2 ew_lds[];
    if (a.gate && a.gate->ew_fallback == 0) return;
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= (a.sample ? a.n_sample : a.n)) return;
    const int64_t i = a.sample ? j * a.stride : j;
    double* out = a.sample ? a.sample + kSampleRec * j : nullptr;
    if (i >= a.n || (a.active && !a.active[i])) {
        if (out)
            for (int k = 0; k < kSampleRec; ++k) out[k] = 0.0;
        return;
    }
    ewald_particle(a, i, out, ew_lds);
}

// Every particle (no mask), over a grid of one wave per SIMD, for the
// correction that runs beside the PP + PC kernel: its waves take one slot
// per SIMD from the start, so the two kernels share every SIMD instead of
// the correction waiting for the PP + PC kernel's tail.
constexpr int kEwaldBesideBlocksPerCU = 2;  // 2 waves each: one per SIMD
__global__ void __launch_bounds__(kEwaldThreads) k_ewald_beside(EwaldArgs a) {
    extern __shared__ double2 ew_lds[];
    for (int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < a.n;
         j += int64_t(gridDim.x) * blockDim.x) {
        asm volatile("" ::: "memory");  // table reads stay inside the loop
        ewald_particle(a, j, nullptr, ew_lds);
    }
}

// The listed active particles (a mask is in use), over a bounded grid: a
// grid covering every particle would spend most of its time starting
// blocks that exit, each holding its LDS tables while it does.
__global__ void __launch_bounds__(kEwaldThreads) __attribute__((amdgpu_waves_per_eu(3)))
k_ewald_list(EwaldArgs a) {
    extern __shared__ double2 ew_lds[];
    if (a.gate && a.gate->ew_fallback == 0) return;
    const int64_t count = int64_t(a.ctl->n_list);
    for (int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < count;
         j += int64_t(gridDim.x) * blockDim.x) {
        asm volatile("" ::: "memory");  // table reads stay inside the loop
        ewald_particle(a, a.list[j], nullptr, ew_lds);
    }
}

// The buffered correction added to the PP + PC sums, in double and rounded
// once (the same arithmetic as the accumulating epilogue above).
__global__ void __launch_bounds__(256) k_ewald_add(EwaldArgs a) {
    const int64_t count = a.list ? int64_t(a.ctl->n_list) : a.n;
    for (int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < count;
         j += int64_t(gridDim.x) * blockDim.x) {
        const int64_t i = a.list ? int64_t(a.list[j]) : j;
        if (!a.list && a.active && !a.active[i]) continue;
        const double* e = a.ewbuf + 4 * i;
        float* px = a.acc + i;
        float* py = a.acc + a.n + i;
        float* pz = a.acc + 2 * a.n + i;
        *px = float(double(*px) + e[0]);
        *py = float(double(*py) + e[1]);
        *pz = float(double(*pz) + e[2]);
        a.pot[i] = float(double(a.pot[i]) + e[3]);
    }
}

// The surrogate's verdict from the sample (one block, fixed summation
// order): err = sqrt(mean over the valid records of |a_s - a_e|^2 /
// |a_base + a_e|^2), the rms relative force error the surrogate adds; the
// exact path is chosen when err > tol, err is not a number, or no sampled
// particle was active.  A record with zero total force and a non-zero
// deviation counts as infinitely wrong.
constexpr int kJudgeThreads = 256;
__global__ void __launch_bounds__(kJudgeThreads) k_ewald_judge(Control* ctl,
                                                               const double* sample,
                                                               int64_t n_sample, double tol) {
    __shared__ double s_sum[kJudgeThreads], s_cnt[kJudgeThreads];
    double sum = 0.0, cnt = 0.0;
    for (int64_t j = threadIdx.x; j < n_sample; j += kJudgeThreads) {
        const double* r = sample + kSampleRec * j;
        if (r[3] == 0.0) continue;
        const double dx = r[8] - r[0], dy = r[9] - r[1], dz = r[10] - r[2];
        const double tx = r[4] + r[0], ty = r[5] + r[1], tz = r[6] + r[2];
        const double num = dx * dx + dy * dy + dz * dz;
        const double den = tx * tx + ty * ty + tz * tz;
        sum += den > 0.0 ? num / den : (num > 0.0 ? INFINITY : 0.0);
        cnt += 1.0;
    }
    s_sum[threadIdx.x] = sum;
    s_cnt[threadIdx.x] = cnt;
    __syncthreads();
    for (int h = kJudgeThreads / 2; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h) {
            s_sum[threadIdx.x] += s_sum[threadIdx.x + h];
            s_cnt[threadIdx.x] += s_cnt[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double n = s_cnt[0];
        const double err = n > 0.0 ? sqrt(s_sum[0] / n) : 0.0;
        ctl->ew_err = err;
        ctl->ew_samples = (unsigned long long)(n);
        ctl->ew_fallback = (n == 0.0 || !(err <= tol)) ? 1 : 0;
    }
}

#include "mlp_kernels.inc"

constexpr int kMlpMaxEpochs = 4096;

struct MlpLayoutT {
    size_t theta, m, v, grad, eff, w2f, w3f, w2b, w3b, xb, tb, dy, z1, z2, z3, a1, a2, h3, dz1,
        dz2, dz3, tile_loss, wpart, ctl, cells, total;
};

// The surrogate network attached to a context: a caller-provided device
// workspace holding parameters, optimiser state and training buffers.
struct MlpState {
    char* ws = nullptr;
    int64_t max_batch = 0;
    MlpLayoutT lay{};
    bool has_weights = false;
    double psi0 = 0.0;
};

}  // namespace

// ---------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------
namespace mgrav_internal {
thread_local std::string g_host_error;
mgrav_status set_host_error(mgrav_status s, const std::string& msg) {
    g_host_error = msg;
    return s;
}
}  // namespace mgrav_internal

struct mgrav_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;  // direct launches: exact Ewald beside the PP + PC kernel
    int n_cu = 0;
    int wall_khz = 0;  // device wall clock rate (wall_clock64 ticks per ms)
    std::string arch;  // gcnArchName, part of the autotuning cache key
    int interact_blocks[kNumVariants] = {};  // persistent grid per variant
    int occupancy_status = 0;
    int variant = 0;  // PP + PC kernel variant in use (mgrav_autotune)
    int queue_order = MGRAV_QUEUE_AUTO;  // work-queue layout (mgrav_set_queue_order)
    std::string err;
    bool bound = false;
    bool failed = false;
    mgrav_problem prob{};
    char* ws = nullptr;
    Layout lay{};
    mgrav_ewald ewald{};
    const uint8_t* active = nullptr;
    hipEvent_t ev_start = nullptr, ev_end = nullptr;
    hipEvent_t ev_k0 = nullptr, ev_k1 = nullptr, ev_e1 = nullptr;  // around k_interact / k_ewald
    hipEvent_t ev_e0 = nullptr;       // start of the Ewald work when it overlaps k_interact
    bool last_overlap = false;        // the last compute ran the Ewald on the side stream
    bool have_run = false;
    // graph cache: the captured launch sequence and the arguments it holds,
    // one set for computes that start with the staging of a fresh bind and
    // one for those that do not (so alternating use never recaptures)
    struct GraphSet {
        hipGraphExec_t gexec[3] = {nullptr, nullptr, nullptr};
        hipGraph_t graph[3] = {nullptr, nullptr, nullptr};
        struct LaunchSet* set = nullptr;
    } gs[2];
    int last_set = -1;            // graph set of the last compute
    bool stage_pending = false;   // bound, staging kernels not yet enqueued
    bool stage_partial = false;   // the last staging covered a mask's needs only
    bool no_graph = false;        // capture failed once: launch directly
    int graph_error = 0;          // the HIP error that made it fail
    bool direct = false;          // MGRAV_LAUNCH_DIRECT chosen: no graphs
    Control* host_ctl = nullptr;  // pinned
    int* store_err = nullptr;     // pinned: error words of the particle-store kernels
    MlpState mlp;
};

// Everything a compute launches, compared byte-wise to decide whether the
// captured graph can be replayed.
struct LaunchSet {
    int stage;     // 1: the staging kernels of a fresh bind run first
    StageArgs s;   // their arguments (stage = 1)
    Control* host_ctl;
    RunArgs r;
    EwaldArgs e;
    SurrogateArgs sg;
    const int32_t* child;
    const double* mom;
    const double* com;
    int64_t n, n_bucket, n_cell;
    int use_mask, tree, ewald, variant, interact_blocks, surrogate_blocks;
    // exact Ewald beside the PP + PC kernel: the correction goes to the
    // workspace's double buffer on a branch of its own (a second stream, or
    // a parallel branch of the graph) and is added once both are done;
    // `early`: the branch starts with the compute rather than after phase 0
    int overlap, early;
    // SURROGATE_FALLBACK: the judge's sample
    double* sample;
    int64_t sample_stride, n_sample;
    double judge_tol;
    int sample_ewald_blocks, sample_surrogate_blocks;
};

namespace {

mgrav_status fail(mgrav_ctx* c, mgrav_status s, const std::string& msg) {
    if (c) c->err = msg;
    mgrav_internal::g_host_error = msg;
    return s;
}

mgrav_status hip_fail(mgrav_ctx* c, hipError_t e, const char* what) {
    return fail(c, MGRAV_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Device address of each GPU's copy of `scratch`, looked up by
// mgrav_create with that device current, once per device.
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
bool g_scratch_done[kMaxScratchDevices] = {};
void* g_scratch_ptr[kMaxScratchDevices] = {};
hipError_t g_scratch_err[kMaxScratchDevices] = {};

void scratch_lookup(int device) {
    if (device < 0 || device >= kMaxScratchDevices) return;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_done[device]) return;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) (void)hipGetLastError();
    g_scratch_err[device] = e;
    g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
    g_scratch_done[device] = true;
}

#define HIP_TRY(ctx, expr)                                   \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
    } while (0)

void drop_set(mgrav_ctx* c, int k) {
    mgrav_ctx::GraphSet& g = c->gs[k];
    for (int i = 0; i < 3; ++i) {
        if (g.gexec[i]) (void)hipGraphExecDestroy(g.gexec[i]);
        if (g.graph[i]) (void)hipGraphDestroy(g.graph[i]);
        g.gexec[i] = nullptr;
        g.graph[i] = nullptr;
    }
    delete g.set;
    g.set = nullptr;
}

void drop_graph(mgrav_ctx* c) {
    drop_set(c, 0);
    drop_set(c, 1);
    c->last_set = -1;
}

StageArgs stage_args(mgrav_ctx* c) {
    const mgrav_problem& p = c->prob;
    StageArgs a{};
    a.n = p.n;
    a.n_cell = p.n_cell;
    a.n_bucket = p.n_bucket;
    a.n_pp = p.n_pp;
    a.n_pc = p.n_pc;
    a.n_images = p.n_images;
    a.L = p.box_L;
    a.eps = p.eps;
    a.pin = pos_in(p);
    a.mass = p.mass;
    a.mass_uniform = p.mass_uniform;
    a.cell_first = p.cell_first;
    a.cell_count = p.cell_count;
    a.child = p.child;
    a.com = p.com;
    a.bbox = p.bbox;
    a.mom = p.mom;
    a.bucket_cell = p.bucket_cell;
    a.pp_off = p.pp_off;
    a.pp_src = p.pp_src;
    a.pp_img = p.pp_img;
    a.pp_sub = p.pp_sub;
    a.pc_off = p.pc_off;
    a.pc_src = p.pc_src;
    char* w = c->ws;
    a.ctl = reinterpret_cast<Control*>(w + c->lay.ctl);
    a.pdat = reinterpret_cast<float4*>(w + c->lay.pdat);
    a.work = reinterpret_cast<BucketWork*>(w + c->lay.work);
    a.cellrec = reinterpret_cast<float*>(w + c->lay.cellrec);
    a.ppent = reinterpret_cast<float4*>(w + c->lay.ppent);
    a.cinfo = reinterpret_cast<CellInfo*>(w + c->lay.cinfo);
    a.active = nullptr;  // everything; make_launch sets the mask for a masked compute
    a.need_rec = reinterpret_cast<uint8_t*>(w + c->lay.need);
    a.need_src = a.need_rec + p.n_cell;
    return a;
}

mgrav_status check_problem(mgrav_ctx* c, const mgrav_problem* p) {
    if (!p) return fail(c, MGRAV_ERR_INVALID_ARG, "problem is NULL");
    if (p->n < 1 || p->n > MGRAV_MAX_PARTICLES)
        return fail(c, MGRAV_ERR_INVALID_ARG, "n must be in 1 .. 2^27");
    if (p->n_cell < 1 || p->n_bucket < 1 || p->n_bucket > p->n || p->n_cell > 2 * p->n)
        return fail(c, MGRAV_ERR_INVALID_ARG, "bad n_cell / n_bucket");
    if (!(p->eps > 0.0) || !std::isfinite(p->eps))
        return fail(c, MGRAV_ERR_INVALID_ARG, "eps must be finite and > 0");
    if (!(p->theta > 0.0)) return fail(c, MGRAV_ERR_INVALID_ARG, "theta must be > 0");
    if (p->n_images != 1 && p->n_images != 27)
        return fail(c, MGRAV_ERR_INVALID_ARG, "n_images must be 1 or 27");
    if (p->n_images == 27 && !(p->box_L > 0.0))
        return fail(c, MGRAV_ERR_INVALID_ARG, "27 images need box_L > 0");
    if (p->box_L < 0.0 || !std::isfinite(p->box_L))
        return fail(c, MGRAV_ERR_INVALID_ARG, "bad box_L");
    if (p->n_pp < 0 || p->n_pc < 0) return fail(c, MGRAV_ERR_INVALID_ARG, "negative list size");
    if (!p->pos == !p->pos_q)
        return fail(c, MGRAV_ERR_INVALID_ARG, "give exactly one of pos and pos_q");
    if (p->pos_q && (!(p->q_scale > 0.0) || !std::isfinite(p->q_scale) ||
                     !std::isfinite(p->q_origin[0]) || !std::isfinite(p->q_origin[1]) ||
                     !std::isfinite(p->q_origin[2])))
        return fail(c, MGRAV_ERR_INVALID_ARG, "pos_q needs a finite origin and scale > 0");
    if (!p->mass && (!(p->mass_uniform > 0.0) || !std::isfinite(p->mass_uniform)))
        return fail(c, MGRAV_ERR_INVALID_ARG, "mass NULL needs mass_uniform > 0");
    if (!p->cell_first || !p->cell_count || !p->child || !p->com || !p->bbox || !p->mom ||
        !p->bucket_cell || !p->pp_off || !p->pc_off)
        return fail(c, MGRAV_ERR_INVALID_ARG, "null device pointer in problem");
    if ((p->n_pp > 0 && (!p->pp_src || !p->pp_img)) || (p->n_pc > 0 && (!p->pc_src || !p->pc_img)))
        return fail(c, MGRAV_ERR_INVALID_ARG, "null list pointer");
    return MGRAV_OK;
}

}  // namespace

extern "C" {

int mgrav_version(void) { return MGRAV_VERSION_MAJOR * 1000 + MGRAV_VERSION_MINOR; }

const char* mgrav_status_string(mgrav_status s) {
    switch (s) {
    case MGRAV_OK: return "ok";
    case MGRAV_ERR_INVALID_ARG: return "invalid argument";
    case MGRAV_ERR_BAD_TREE: return "bad tree";
    case MGRAV_ERR_BAD_LIST: return "bad interaction list";
    case MGRAV_ERR_DEVICE: return "device error";
    case MGRAV_ERR_NO_MEMORY: return "workspace too small";
    case MGRAV_ERR_TIMEOUT: return "timeout";
    case MGRAV_ERR_STATE: return "call out of order";
    case MGRAV_ERR_NOT_TRAINED: return "surrogate not trained";
    }
    return "unknown status";
}

const char* mgrav_last_error(const mgrav_ctx* ctx) {
    return ctx ? ctx->err.c_str() : mgrav_internal::g_host_error.c_str();
}

mgrav_status mgrav_create(int device, void* hip_stream, mgrav_ctx** out) {
    if (!out) return fail(nullptr, MGRAV_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(nullptr, MGRAV_ERR_INVALID_ARG, "no such device");
    mgrav_ctx* c = new mgrav_ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    e = hipSetDevice(device);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(nullptr, e, "hipSetDevice");
    }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(nullptr, e, "hipGetDeviceProperties");
    }
    c->n_cu = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
    scratch_lookup(device);  // the device is current
    if (hipDeviceGetAttribute(&c->wall_khz, hipDeviceAttributeWallClockRate, device) !=
        hipSuccess) {
        (void)hipGetLastError();  // tolerated: kernel spans then come from events
        c->wall_khz = 0;
    }
    for (int v = 0; v < kNumVariants; ++v) {
        int per_cu = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, interact_kernel(v), kWave, 0);
        if (e != hipSuccess || per_cu < 1) {
            (void)hipGetLastError();  // tolerated: fall back to a fixed occupancy
            per_cu = 8;
            c->occupancy_status = int(e);
        }
        c->interact_blocks[v] = per_cu * c->n_cu;
    }
    if (hipEventCreate(&c->ev_start) != hipSuccess || hipEventCreate(&c->ev_end) != hipSuccess ||
        hipEventCreate(&c->ev_k0) != hipSuccess || hipEventCreate(&c->ev_k1) != hipSuccess ||
        hipEventCreate(&c->ev_e1) != hipSuccess || hipEventCreate(&c->ev_e0) != hipSuccess ||
        hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->host_ctl), sizeof(Control)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->store_err), 64) != hipSuccess) {
        mgrav_destroy(c);
        return fail(nullptr, MGRAV_ERR_DEVICE, "event / pinned allocation failed");
    }
    *out = c;
    return MGRAV_OK;
}

void mgrav_destroy(mgrav_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->side) (void)hipStreamSynchronize(c->side);
    drop_graph(c);
    if (c->ev_start) (void)hipEventDestroy(c->ev_start);
    if (c->ev_end) (void)hipEventDestroy(c->ev_end);
    if (c->ev_k0) (void)hipEventDestroy(c->ev_k0);
    if (c->ev_k1) (void)hipEventDestroy(c->ev_k1);
    if (c->ev_e1) (void)hipEventDestroy(c->ev_e1);
    if (c->ev_e0) (void)hipEventDestroy(c->ev_e0);
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->host_ctl) (void)hipHostFree(c->host_ctl);
    if (c->store_err) (void)hipHostFree(c->store_err);
    delete c;
}

mgrav_status mgrav_workspace_size(const mgrav_problem* p, size_t* bytes) {
    if (!bytes) return fail(nullptr, MGRAV_ERR_INVALID_ARG, "bytes is NULL");
    mgrav_status s = check_problem(nullptr, p);
    if (s != MGRAV_OK) return s;
    *bytes = make_layout(p->n, p->n_cell, p->n_bucket, p->n_pp, p->n_pc).total;
    return MGRAV_OK;
}

mgrav_status mgrav_bind(mgrav_ctx* c, const mgrav_problem* p, void* workspace, size_t bytes) {
    if (!c) return fail(nullptr, MGRAV_ERR_INVALID_ARG, "ctx is NULL");
    c->err.clear();
    mgrav_status s = check_problem(c, p);
    if (s != MGRAV_OK) return s;
    const Layout lay = make_layout(p->n, p->n_cell, p->n_bucket, p->n_pp, p->n_pc);
    if (!workspace) return fail(c, MGRAV_ERR_INVALID_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(c, MGRAV_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (bytes < lay.total) return fail(c, MGRAV_ERR_NO_MEMORY, "workspace too small");
    HIP_TRY(c, hipSetDevice(c->device));
    c->prob = *p;
    c->ws = static_cast<char*>(workspace);
    c->lay = lay;
    c->bound = false;
    c->failed = false;
    c->have_run = false;
    c->active = nullptr;
    if (p->box_L > 0.0 && p->n_images == 27)
        c->ewald = mgrav_ewald{MGRAV_EWALD_EXACT, 2.6, 1, 10, 4, 1, 1e-4, 0};
    else
        c->ewald = mgrav_ewald{MGRAV_EWALD_NONE, 2.6, 1, 10, 4, 1, 1e-4, 0};

    // the staging kernels run at the start of the next compute (inside its
    // first graph) or, if a wait comes first, at that wait
    c->stage_pending = true;
    c->stage_partial = false;
    c->bound = true;
    return MGRAV_OK;
}

mgrav_status mgrav_bind_static(mgrav_ctx* c, const mgrav_problem* p) {
    if (!c) return fail(nullptr, MGRAV_ERR_INVALID_ARG, "ctx is NULL");
    c->err.clear();
    mgrav_status s = check_problem(c, p);
    if (s != MGRAV_OK) return s;
    const size_t need = make_layout(p->n, p->n_cell, p->n_bucket, p->n_pp, p->n_pc).total;
    if (need > size_t(MGRAV_STATIC_WORKSPACE_BYTES))
        return fail(c, MGRAV_ERR_NO_MEMORY,
                    "problem needs " + std::to_string(need) +
                        " bytes of workspace; the static scratch holds " +
                        std::to_string(size_t(MGRAV_STATIC_WORKSPACE_BYTES)) +
                        " (bind it with mgrav_bind and a workspace)");
    if (c->device >= kMaxScratchDevices)
        return fail(c, MGRAV_ERR_INVALID_ARG, "static scratch serves devices 0..63 only");
    void* ptr = nullptr;
    hipError_t e = hipSuccess;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        ptr = g_scratch_ptr[c->device];
        e = g_scratch_err[c->device];
    }
    if (!ptr)
        return hip_fail(c, e != hipSuccess ? e : hipErrorInvalidSymbol,
                        "hipGetSymbolAddress(scratch)");
    return mgrav_bind(c, p, ptr, size_t(MGRAV_STATIC_WORKSPACE_BYTES));
}

mgrav_status mgrav_set_ewald(mgrav_ctx* c, const mgrav_ewald* cfg) {
    if (!c) return fail(nullptr, MGRAV_ERR_INVALID_ARG, "ctx is NULL");
    c->err.clear();
    if (!c->bound) return fail(c, MGRAV_ERR_STATE, "set_ewald before bind");
    if (!cfg) return fail(c, MGRAV_ERR_INVALID_ARG, "cfg is NULL");
    if (cfg->mode == MGRAV_EWALD_NONE) {
        c->ewald = *cfg;
        return MGRAV_OK;
    }
    if (cfg->mode != MGRAV_EWALD_EXACT && cfg->mode != MGRAV_EWALD_SURROGATE &&
        cfg->mode != MGRAV_EWALD_SURROGATE_FALLBACK)
        return fail(c, MGRAV_ERR_INVALID_ARG, "unknown mode");
    if (!(c->prob.box_L > 0.0) || c->prob.n_images != 27)
        return fail(c, MGRAV_ERR_INVALID_ARG, "Ewald needs a periodic problem");
    if (cfg->mode != MGRAV_EWALD_EXACT) {
        if (!c->mlp.ws || !c->mlp.has_weights)
            return fail(c, MGRAV_ERR_NOT_TRAINED, "no surrogate weights loaded");
        if (cfg->top_cells != 1 && cfg->top_cells != 8 && cfg->top_cells != 64)
            return fail(c, MGRAV_ERR_INVALID_ARG, "top_cells must be 1, 8 or 64");
        if (cfg->mode == MGRAV_EWALD_SURROGATE) {
            c->ewald = *cfg;
            return MGRAV_OK;
        }
        if (!(cfg->fallback_tol >= 0.0))
            return fail(c, MGRAV_ERR_INVALID_ARG, "fallback_tol must be >= 0");
        if (cfg->sample_stride < 0)
            return fail(c, MGRAV_ERR_INVALID_ARG, "sample_stride must be >= 0");
    }
    if (!(cfg->alpha > 0.5 && cfg->alpha < 10.0))
        return fail(c, MGRAV_ERR_INVALID_ARG, "alpha outside (0.5, 10)");
    if (cfg->real_layers < 1 || cfg->real_layers > 4)
        return fail(c, MGRAV_ERR_INVALID_ARG, "real_layers outside 1..4");
    if (cfg->h2max < 0 || cfg->h2max > kMaxH2)
        return fail(c, MGRAV_ERR_INVALID_ARG, "h2max outside 0..64");
    if (cfg->order != 0 && cfg->order != 2 && cfg->order != 4)
        return fail(c, MGRAV_ERR_INVALID_ARG, "order must be 0, 2 or 4");
    c->ewald = *cfg;
    return MGRAV_OK;
}

mgrav_status mgrav_set_active(mgrav_ctx* c, const uint8_t* active_dev) {
    if (!c) return fail(nullptr, MGRAV_ERR_INVALID_ARG, "ctx is NULL");
    c->err.clear();
    if (!c->bound) return fail(c, MGRAV_ERR_STATE, "set_active before bind");
    c->active = active_dev;
    return MGRAV_OK;
}

static void make_launch(mgrav_ctx* c, int parts, float* acc, float* pot, LaunchSet* L) {
    std::memset(L, 0, sizeof(*L));  // padding too: the struct is compared byte-wise
    const mgrav_problem& p = c->prob;
    L->stage = c->stage_pending ? 1 : 0;
    if (L->stage) {
        L->s = stage_args(c);
        // with a mask, stage only what the active buckets read; the staging
        // then stays pending for the next compute
        L->s.active = c->active;
    }
    L->host_ctl = c->host_ctl;
    char* w = c->ws;
    RunArgs& r = L->r;
    r.n = p.n;
    r.n_bucket = p.n_bucket;
    r.active = c->active;
    r.ctl = reinterpret_cast<Control*>(w + c->lay.ctl);
    r.pdat = reinterpret_cast<const float4*>(w + c->lay.pdat);
    r.work = reinterpret_cast<const BucketWork*>(w + c->lay.work);
    r.items = reinterpret_cast<int*>(w + c->lay.items);
    r.bins = reinterpret_cast<signed char*>(w + c->lay.bins);
    r.cellrec = reinterpret_cast<const float*>(w + c->lay.cellrec);
    r.ppent = reinterpret_cast<const float4*>(w + c->lay.ppent);
    r.pc_src = p.pc_src;
    r.pc_img = p.pc_img;
    r.com = p.com;
    r.bbox = p.bbox;
    r.bucket_cell = p.bucket_cell;
    r.n_cell = p.n_cell;
    r.L = p.box_L;
    r.n_images = p.n_images;
    r.acc = acc;
    r.pot = pot;
    r.eps2 = float(p.eps * p.eps);
    r.parts = parts;
    int* plist = c->active ? reinterpret_cast<int*>(w + c->lay.plist) : nullptr;
    r.plist = plist;
    r.queue_order = c->queue_order;
    L->n = p.n;
    L->n_bucket = p.n_bucket;
    L->use_mask = c->active ? 1 : 0;
    L->tree = (parts & (MGRAV_PART_PP | MGRAV_PART_PC)) != 0;
    L->ewald = (parts & MGRAV_PART_EWALD) ? c->ewald.mode : MGRAV_EWALD_NONE;
    const bool judge = L->ewald == MGRAV_EWALD_SURROGATE_FALLBACK;
    L->variant = c->variant;
    L->interact_blocks = int(p.n_bucket < c->interact_blocks[c->variant]
                                 ? p.n_bucket
                                 : c->interact_blocks[c->variant]);
    if (L->ewald == MGRAV_EWALD_SURROGATE || judge) {
        SurrogateArgs& g = L->sg;
        const MlpLayoutT& ml = c->mlp.lay;
        g.n = p.n;
        g.pin = pos_in(p);
        g.active = c->active;
        g.cells = reinterpret_cast<const double*>(c->mlp.ws + ml.cells);
        g.ncell = c->ewald.top_cells;
        g.L = p.box_L;
        g.psi0 = c->mlp.psi0;
        g.eff = reinterpret_cast<const float*>(c->mlp.ws + ml.eff);
        g.w2f = reinterpret_cast<const bf16x8*>(c->mlp.ws + ml.w2f);
        g.w3f = reinterpret_cast<const bf16x8*>(c->mlp.ws + ml.w3f);
        g.acc = acc;
        g.pot = pot;
        g.accumulate = L->tree;
        g.list = plist;
        g.ctl = r.ctl;
        L->child = p.child;
        L->mom = p.mom;
        L->com = p.com;
        L->n_cell = p.n_cell;
        const int per_group = 16 / (g.ncell < 16 ? g.ncell : 16);
        const int64_t groups = (p.n + per_group - 1) / per_group;
        const int64_t wpb = kSurrogateThreads / kWave;
        const int64_t blocks = (groups + wpb - 1) / wpb;
        L->surrogate_blocks = int(blocks < 8 * c->n_cu ? blocks : 8 * c->n_cu);
    }
    if (L->ewald == MGRAV_EWALD_EXACT || judge) {
        EwaldArgs& e = L->e;
        e.n = p.n;
        e.pin = pos_in(p);
        e.mom = p.mom;
        e.com = p.com;
        e.active = c->active;
        e.table = reinterpret_cast<double*>(w + c->lay.ewald);
        e.acc = acc;
        e.pot = pot;
        e.L = p.box_L;
        e.alpha = c->ewald.alpha;
        e.real_layers = c->ewald.real_layers;
        e.h2max = c->ewald.h2max;
        e.hmax = int(std::floor(std::sqrt(double(e.h2max)) + 1e-9));
        e.order = c->ewald.order;
        e.accumulate = L->tree;
        e.list = plist;
        e.ctl = r.ctl;
        if (L->tree && L->ewald == MGRAV_EWALD_EXACT) {
            // Beside the PP + PC kernel.  Without a mask and next to a 2-wave
            // PP + PC variant the branch starts with the compute (the
            // correction reads only the caller's positions and root moments)
            // and takes one wave per SIMD before the PP + PC kernel fills the
            // GPU.  Next to a 3-wave variant, or with a mask (the list of
            // active particles comes from phase 0), it starts after phase 0
            // and fills the PP + PC kernel's tail: a correction wave beside
            // two waves of a 3-wave variant (room enough for its registers)
            // made the 512^3 clustered step 24 % slower than the tail.
            L->overlap = 1;
            L->early = (!e.list && kVariantWaves[L->variant] == 2) ? 1 : 0;
            e.ewbuf = reinterpret_cast<double*>(w + c->lay.ewbuf);
        }
    }
    if (judge) {
        // every stride-th particle, at most kMaxEwaldSamples of them
        const int64_t min_stride = (p.n + kMaxEwaldSamples - 1) / kMaxEwaldSamples;
        int64_t stride = c->ewald.sample_stride > 0
                             ? c->ewald.sample_stride
                             : (p.n + kDefaultEwaldSamples - 1) / kDefaultEwaldSamples;
        if (stride < min_stride) stride = min_stride;
        if (stride < 1) stride = 1;
        L->sample = reinterpret_cast<double*>(w + c->lay.ewsample);
        L->sample_stride = stride;
        L->n_sample = (p.n + stride - 1) / stride;
        L->judge_tol = c->ewald.fallback_tol;
        const int64_t et = ewald_threads(L->e.hmax);
        L->sample_ewald_blocks = int((L->n_sample + et - 1) / et);
        const int per_group = 16 / (L->sg.ncell < 16 ? L->sg.ncell : 16);
        const int64_t groups = (L->n_sample + per_group - 1) / per_group;
        const int64_t wpb = kSurrogateThreads / kWave;
        const int64_t sb = (groups + wpb - 1) / wpb;
        L->sample_surrogate_blocks = int(sb < 8 * c->n_cu ? sb : 8 * c->n_cu);
    }
}

// The staging kernels of mgrav_bind (positions, cells, PP and PC entries).
static void enqueue_stage(hipStream_t st, const StageArgs& a) {
    const unsigned per_bucket = unsigned((a.n_bucket + 255) / 256);  // one thread per bucket
    if (a.active) {
        const int64_t words = (2 * a.n_cell + 3) / 4;
        const int64_t gb = (words + 255) / 256;
        hipLaunchKernelGGL(k_need_clear, dim3(unsigned(gb < 1024 ? gb : 1024)), dim3(256), 0, st,
                           a);
        hipLaunchKernelGGL(k_need_mark, dim3(per_bucket), dim3(256), 0, st, a);
    }
    hipLaunchKernelGGL(k_stage_cells, dim3(unsigned((a.n_cell + 255) / 256)), dim3(256), 0, st,
                       a);
    if (a.active) {
        hipLaunchKernelGGL(k_stage_bucket_masked, dim3(per_bucket), dim3(256), 0, st, a);
    } else {
        const int64_t nb = a.n_bucket * kStageLanes;
        hipLaunchKernelGGL(k_stage_bucket, dim3(unsigned((nb + 255) / 256)), dim3(256), 0, st, a);
    }
}

// Exact correction of every active particle: one thread per particle, or,
// with a mask, a bounded grid over the list of active particles.
static void launch_ewald_all(mgrav_ctx* c, const LaunchSet& L, const EwaldArgs& e,
                             hipStream_t st) {
    const int et = ewald_threads(e.hmax);
    const size_t lds = ewald_lds_bytes(e.hmax);
    const int64_t nb = (L.n + et - 1) / et;
    if (e.list) {
        const int64_t cap = 16 * int64_t(c->n_cu);
        hipLaunchKernelGGL(k_ewald_list, dim3(unsigned(nb < cap ? nb : cap)), dim3(et), lds, st,
                           e);
    } else {
        hipLaunchKernelGGL(k_ewald, dim3(unsigned(nb)), dim3(et), lds, st, e);
    }
}

// The launch sequence in three phases: 0 = queue set-up, 1 = PP + PC,
// 2 = Ewald (or, with the overlap, the Ewald branch and the join).  Each
// is captured as its own graph so that timing events can be recorded
// between them.
static void enqueue_phase(mgrav_ctx* c, const LaunchSet& L, int phase) {
    if (phase == 0) {
        if (L.stage) enqueue_stage(c->stream, L.s);
        const int64_t sel = (L.n_bucket + 255) / 256;
        hipLaunchKernelGGL(k_select, dim3(unsigned(sel < 4 * c->n_cu ? sel : 4 * c->n_cu)),
                           dim3(256), 0, c->stream, L.r);
        hipLaunchKernelGGL(k_order_scatter,
                           dim3(unsigned((L.n_bucket + kScatterThreads - 1) / kScatterThreads)),
                           dim3(kScatterThreads), 0, c->stream, L.r);
    } else if (phase == 1 && L.tree) {
        launch_interact(L.variant, dim3(unsigned(L.interact_blocks)), c->stream, L.r);
    } else if (phase == 2 && L.ewald == MGRAV_EWALD_EXACT) {
        hipLaunchKernelGGL(k_ewald_setup, dim3(1), dim3(kSetupThreads), 0, c->stream, L.e);
        launch_ewald_all(c, L, L.e, c->stream);
    } else if (phase == 2 && L.ewald == MGRAV_EWALD_SURROGATE) {
        hipLaunchKernelGGL(k_surrogate_cells, dim3(1), dim3(kWave), 0, c->stream, L.child, L.com,
                           L.mom, L.n_cell, L.sg.ncell, const_cast<double*>(L.sg.cells));
        hipLaunchKernelGGL(k_ewald_surrogate, dim3(unsigned(L.surrogate_blocks)),
                           dim3(kSurrogateThreads), 0,
                           c->stream, L.sg);
    } else if (phase == 2 && L.ewald == MGRAV_EWALD_SURROGATE_FALLBACK) {
        // both corrections on the sample, the verdict, then the chosen one
        // everywhere (the other launch exits at once)
        const int et = ewald_threads(L.e.hmax);
        const size_t lds = ewald_lds_bytes(L.e.hmax);
        hipLaunchKernelGGL(k_ewald_setup, dim3(1), dim3(kSetupThreads), 0, c->stream, L.e);
        hipLaunchKernelGGL(k_surrogate_cells, dim3(1), dim3(kWave), 0, c->stream, L.child, L.com,
                           L.mom, L.n_cell, L.sg.ncell, const_cast<double*>(L.sg.cells));
        EwaldArgs es = L.e;
        es.sample = L.sample;
        es.stride = L.sample_stride;
        es.n_sample = L.n_sample;
        es.list = nullptr;
        hipLaunchKernelGGL(k_ewald, dim3(unsigned(L.sample_ewald_blocks)), dim3(et), lds,
                           c->stream, es);
        SurrogateArgs ss = L.sg;
        ss.sample = L.sample;
        ss.stride = L.sample_stride;
        ss.n_sample = L.n_sample;
        ss.list = nullptr;
        hipLaunchKernelGGL(k_ewald_surrogate, dim3(unsigned(L.sample_surrogate_blocks)),
                           dim3(kSurrogateThreads), 0, c->stream, ss);
        hipLaunchKernelGGL(k_ewald_judge, dim3(1), dim3(kJudgeThreads), 0, c->stream, L.r.ctl,
                           L.sample, L.n_sample, L.judge_tol);
        SurrogateArgs sg = L.sg;
        sg.gate = L.r.ctl;
        hipLaunchKernelGGL(k_ewald_surrogate, dim3(unsigned(L.surrogate_blocks)),
                           dim3(kSurrogateThreads), 0, c->stream, sg);
        EwaldArgs eg = L.e;
        eg.gate = L.r.ctl;
        launch_ewald_all(c, L, eg, c->stream);
    }
    if (phase == 2)
        hipLaunchKernelGGL(k_copy_control, dim3(1), dim3(kWave), 0, c->stream, L.r.ctl,
                           L.host_ctl);
}

// The exact correction into the double buffer (the branch beside the
// PP + PC kernel) and, once both are done, its addition to the PP + PC sums
// followed by the copy of the control block (the join).
static void enqueue_ewald_branch(mgrav_ctx* c, const LaunchSet& L, hipStream_t st) {
    hipLaunchKernelGGL(k_ewald_setup, dim3(1), dim3(kSetupThreads), 0, st, L.e);
    if (L.early)
        hipLaunchKernelGGL(k_ewald_beside, dim3(unsigned(kEwaldBesideBlocksPerCU * c->n_cu)),
                           dim3(ewald_threads(L.e.hmax)), ewald_lds_bytes(L.e.hmax), st, L.e);
    else
        launch_ewald_all(c, L, L.e, st);
}

static void enqueue_ewald_join(mgrav_ctx* c, const LaunchSet& L, hipStream_t st) {
    const int64_t nb = (L.n + 255) / 256;
    hipLaunchKernelGGL(k_ewald_add, dim3(unsigned(nb < 8 * c->n_cu ? nb : 8 * c->n_cu)),
                       dim3(256), 0, st, L.e);
    hipLaunchKernelGGL(k_copy_control, dim3(1), dim3(kWave), 0, st, L.r.ctl, L.host_ctl);
}

// One graph per compute: each phase is captured into a graph of its own,
// and a parent graph holds them as child-graph nodes with the context's
// timing events as event-record nodes in between (ev_start, phase 0, ev_k0,
// phase 1, ev_k1, phase 2, ev_e1, ev_end).  With exact Ewald beside the
// PP + PC kernel, the correction is a parallel branch (ev_e0, correction,
// ev_e1) that starts after ev_start or after phase 0, and a join piece
// (addition to the PP + PC sums, control copy) waits for both branches.
// The parent is built explicitly because the HIP runtime PyTorch ships
// rejects event records inside a stream capture.  On any failure the
// context falls back to direct launches, and graph_error = 1000 * step +
// HIP error records why (steps 1-4: capture of the pieces, 5: parent, 6:
// its nodes, 7: instantiation).
static void capture_graphs(mgrav_ctx* c, const LaunchSet& L) {
    hipStreamCaptureStatus cs;
    if (c->no_graph) return;
    if (c->stream == nullptr) {  // the legacy default stream cannot be captured
        c->no_graph = true;
        c->graph_error = int(hipErrorInvalidValue);
        return;
    }
    hipError_t q = hipStreamIsCapturing(c->stream, &cs);
    if (q != hipSuccess || cs != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        c->no_graph = true;
        c->graph_error = q != hipSuccess ? int(q) : int(hipErrorStreamCaptureUnsupported);
        return;
    }
    mgrav_ctx::GraphSet& g = c->gs[L.stage];
    int step = 0;
    hipError_t e = hipSuccess;
    // captured pieces: phase 0, 1, 2 or, with the overlap, phase 0, 1, the
    // Ewald branch (slot 2) and the join (slot 3)
    hipGraph_t piece[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int k = 0; k < 4 && e == hipSuccess; ++k) {
        if (k == 1 && !L.tree) continue;
        if (k == 3 && !L.overlap) continue;
        step = 1 + k;
        e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) break;
        if (k < 2 || (k == 2 && !L.overlap)) enqueue_phase(c, L, k);
        else if (k == 2) enqueue_ewald_branch(c, L, c->stream);
        else enqueue_ewald_join(c, L, c->stream);
        const hipError_t r = hipPeekAtLastError();
        const hipError_t ec = hipStreamEndCapture(c->stream, &piece[k]);  // always end it
        e = r != hipSuccess ? r : ec;
    }
    hipGraph_t parent = nullptr;
    if (e == hipSuccess) {
        step = 5;
        e = hipGraphCreate(&parent, 0);
    }
    // nodes with explicit dependencies (at most two each)
    auto add_event = [&](hipEvent_t ev, hipGraphNode_t d0, hipGraphNode_t d1) {
        hipGraphNode_t deps[2], n = nullptr;
        int nd = 0;
        if (d0) deps[nd++] = d0;
        if (d1) deps[nd++] = d1;
        if (e == hipSuccess) e = hipGraphAddEventRecordNode(&n, parent, nd ? deps : nullptr, nd, ev);
        return n;
    };
    auto add_child = [&](hipGraph_t child, hipGraphNode_t d0, hipGraphNode_t d1) {
        hipGraphNode_t deps[2], n = nullptr;
        int nd = 0;
        if (d0) deps[nd++] = d0;
        if (d1) deps[nd++] = d1;
        if (e == hipSuccess) e = hipGraphAddChildGraphNode(&n, parent, nd ? deps : nullptr, nd, child);
        return n;
    };
    if (e == hipSuccess) {
        step = 6;
        // ev_start, phase 0, ev_k0, phase 1, ev_k1, then either phase 2,
        // ev_e1, ev_end, or, with the overlap, the branch between ev_e0 and
        // ev_e1 (after ev_start or after phase 0) joined with ev_k1 by the
        // join piece, then ev_end
        hipGraphNode_t n_start = add_event(c->ev_start, nullptr, nullptr);
        hipGraphNode_t n_p0 = add_child(piece[0], n_start, nullptr);
        hipGraphNode_t n_k0 = add_event(c->ev_k0, n_p0, nullptr);
        hipGraphNode_t n_p1 = piece[1] ? add_child(piece[1], n_k0, nullptr) : n_k0;
        hipGraphNode_t n_k1 = add_event(c->ev_k1, n_p1, nullptr);
        hipGraphNode_t n_last = nullptr;
        if (L.overlap) {
            hipGraphNode_t n_e0 = add_event(c->ev_e0, L.early ? n_start : n_p0, nullptr);
            hipGraphNode_t n_br = add_child(piece[2], n_e0, nullptr);
            hipGraphNode_t n_e1 = add_event(c->ev_e1, n_br, nullptr);
            n_last = add_child(piece[3], n_k1, n_e1);
        } else {
            hipGraphNode_t n_p2 = add_child(piece[2], n_k1, nullptr);
            n_last = add_event(c->ev_e1, n_p2, nullptr);
        }
        (void)add_event(c->ev_end, n_last, nullptr);
    }
    if (e == hipSuccess) {
        step = 7;
        e = hipGraphInstantiate(&g.gexec[0], parent, nullptr, nullptr, 0);
    }
    for (hipGraph_t pc : piece)  // the parent holds copies
        if (pc) (void)hipGraphDestroy(pc);
    if (e == hipSuccess && g.gexec[0]) {
        g.graph[0] = parent;
        g.set = new LaunchSet(L);
        return;
    }
    if (parent) (void)hipGraphDestroy(parent);
    (void)hipGetLastError();
    drop_graph(c);
    c->no_graph = true;
    c->graph_error = 1000 * step + (e != hipSuccess ? int(e) : int(hipErrorUnknown));
}

mgrav_status mgrav_compute_parts(mgrav_ctx* c, int parts, float* acc, float* pot) {
    if (!c) return fail(nullptr, MGRAV_ERR_INVALID_ARG, "ctx is NULL");
    c->err.clear();
    if (!c->bound) return fail(c, MGRAV_ERR_STATE, "compute before bind");
    if (c->failed) return fail(c, MGRAV_ERR_STATE, "context failed; bind again");
    if (!acc || !pot) return fail(c, MGRAV_ERR_INVALID_ARG, "null output");
    if (parts <= 0 || parts > MGRAV_PART_ALL) return fail(c, MGRAV_ERR_INVALID_ARG, "bad parts");
    HIP_TRY(c, hipSetDevice(c->device));
    LaunchSet L;
    make_launch(c, parts, acc, pot, &L);
    mgrav_ctx::GraphSet& g = c->gs[L.stage];
    const bool same = g.set && std::memcmp(g.set, &L, sizeof(L)) == 0;
    if (!same) {
        drop_set(c, L.stage);
        if (!c->direct) capture_graphs(c, L);
    }
    if (g.gexec[0]) {
        HIP_TRY(c, hipGraphLaunch(g.gexec[0], c->stream));
    } else if (L.overlap) {
        // the exact correction on the side stream, into the double buffer,
        // beside the PP + PC kernel; then added to its sums on the stream
        // (the PP + PC kernel times itself on the device clock, so no event
        // marker sits between the phases on the stream unless the side
        // stream needs one to start after phase 0)
        HIP_TRY(c, hipEventRecord(c->ev_start, c->stream));
        auto side_ewald = [&](hipEvent_t after) -> hipError_t {
            hipError_t r = hipStreamWaitEvent(c->side, after, 0);
            if (r == hipSuccess) r = hipEventRecord(c->ev_e0, c->side);
            if (r != hipSuccess) return r;
            enqueue_ewald_branch(c, L, c->side);
            r = hipGetLastError();
            return r == hipSuccess ? hipEventRecord(c->ev_e1, c->side) : r;
        };
        if (L.early) HIP_TRY(c, side_ewald(c->ev_start));
        enqueue_phase(c, L, 0);
        HIP_TRY(c, hipGetLastError());
        if (!L.early) {
            HIP_TRY(c, hipEventRecord(c->ev_k0, c->stream));
            HIP_TRY(c, side_ewald(c->ev_k0));
        }
        enqueue_phase(c, L, 1);
        HIP_TRY(c, hipGetLastError());
        HIP_TRY(c, hipStreamWaitEvent(c->stream, c->ev_e1, 0));
        enqueue_ewald_join(c, L, c->stream);
        HIP_TRY(c, hipGetLastError());
        HIP_TRY(c, hipEventRecord(c->ev_end, c->stream));
    } else {
        const hipEvent_t marks[3] = {c->ev_k0, c->ev_k1, c->ev_e1};
        HIP_TRY(c, hipEventRecord(c->ev_start, c->stream));
        for (int ph = 0; ph < 3; ++ph) {
            enqueue_phase(c, L, ph);
            HIP_TRY(c, hipGetLastError());
            HIP_TRY(c, hipEventRecord(marks[ph], c->stream));
        }
        HIP_TRY(c, hipEventRecord(c->ev_end, c->stream));
    }
    const bool overlap = L.overlap != 0;
    c->last_overlap = overlap;
    // counters and error bits travel back with the work: the last kernel of
    // phase 2 copies the control block into pinned host memory
    c->have_run = true;
    c->stage_pending = L.stage && L.s.active != nullptr;
    c->stage_partial = c->stage_pending;
    c->last_set = L.stage;
    return MGRAV_OK;
}

mgrav_status mgrav_compute(mgrav_ctx* c, float* acc, float* pot) {
    return mgrav_compute_parts(c, MGRAV_PART_ALL, acc, pot);
}

mgrav_status mgrav_watchdog_poll(int (*query)(void* user), void* user, double timeout_s) {
    if (!query) return fail(nullptr, MGRAV_ERR_INVALID_ARG, "query is NULL");
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const int q = query(user);
        if (q == 0) return MGRAV_OK;
        if (q < 0) return fail(nullptr, MGRAV_ERR_DEVICE, "completion query failed");
        const double dt =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (timeout_s > 0.0 && dt > timeout_s)
            return fail(nullptr, MGRAV_ERR_TIMEOUT, "deadline passed before completion");
        // spin for the first 2 ms (typical steps), then back off
        if (dt > 2e-3) std::this_thread::sleep_for(std::chrono::microseconds(dt < 0.05 ? 50 : 500));
    }
}

mgrav_status mgrav_wait(mgrav_ctx* c, double timeout_s, mgrav_stats* stats) {
    if (!c) return fail(nullptr, MGRAV_ERR_INVALID_ARG, "ctx is NULL");
    c->err.clear();
    if (!c->bound) return fail(c, MGRAV_ERR_STATE, "wait before bind");
    HIP_TRY(c, hipSetDevice(c->device));
    if (c->stage_pending && !c->stage_partial) {  // bind without compute: stage now, for its checks
        const StageArgs a = stage_args(c);
        enqueue_stage(c->stream, a);
        hipLaunchKernelGGL(k_copy_control, dim3(1), dim3(kWave), 0, c->stream, a.ctl,
                           c->host_ctl);
        HIP_TRY(c, hipGetLastError());
        c->stage_pending = false;
    }
    // Watchdog: a marker event after all enqueued work, polled until done.
    hipEvent_t marker;
    HIP_TRY(c, hipEventCreateWithFlags(&marker, hipEventDisableTiming));
    hipError_t e = hipEventRecord(marker, c->stream);
    if (e != hipSuccess) {
        (void)hipEventDestroy(marker);
        return hip_fail(c, e, "hipEventRecord");
    }
    struct EventQuery {
        hipEvent_t ev;
        hipError_t err;
        static int poll(void* user) {
            EventQuery* q = static_cast<EventQuery*>(user);
            const hipError_t r = hipEventQuery(q->ev);
            if (r == hipSuccess) return 0;
            if (r == hipErrorNotReady) return 1;
            q->err = r;
            return -1;
        }
    } query{marker, hipSuccess};
    const mgrav_status ws = mgrav_watchdog_poll(&EventQuery::poll, &query, timeout_s);
    // released on every path: a marker still pending is freed by the
    // runtime once the work before it completes
    (void)hipEventDestroy(marker);
    if (ws == MGRAV_ERR_TIMEOUT) {
        c->failed = true;
        return fail(c, MGRAV_ERR_TIMEOUT, "device work did not finish before the deadline");
    }
    if (ws != MGRAV_OK) return hip_fail(c, query.err, "device work failed");
    // host_ctl was filled by the control copy at the end of the staging or
    // of the last compute
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        if (c->have_run) {
            stats->n_pp_interactions = int64_t(c->host_ctl->n_pp_int);
            stats->n_pc_interactions = int64_t(c->host_ctl->n_pc_int);
            stats->n_active_particles = int64_t(c->host_ctl->n_active_p);
            stats->n_active_buckets = int64_t(c->host_ctl->n_active_b);
            // a timing that cannot be read stays 0; its error is cleared so
            // that the next launch check does not report it
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, c->ev_start, c->ev_end) == hipSuccess)
                stats->ms_total = ms;
            // the PP + PC kernel's span from its own wall-clock stamps (the
            // events around it where the stamps are missing)
            const unsigned long long k0 = c->host_ctl->t_k0, k1 = c->host_ctl->t_k1;
            if (c->wall_khz > 0 && k0 != 0 && k1 > k0)
                stats->ms_interact = float(double(k1 - k0) / double(c->wall_khz));
            else if (!c->last_overlap && hipEventElapsedTime(&ms, c->ev_k0, c->ev_k1) == hipSuccess)
                stats->ms_interact = ms;
            if (hipEventElapsedTime(&ms, c->last_overlap ? c->ev_e0 : c->ev_k1, c->ev_e1) ==
                hipSuccess)
                stats->ms_ewald = ms;
            (void)hipGetLastError();
            const mgrav_ctx::GraphSet* g = c->last_set >= 0 ? &c->gs[c->last_set] : nullptr;
            stats->graph_replay = g && g->gexec[0] != nullptr ? 1 : 0;
            stats->graph_error = c->graph_error;
            stats->interact_variant = g && g->set ? g->set->variant : c->variant;
            stats->ewald_fallback = c->host_ctl->ew_fallback;
            stats->ewald_samples = int64_t(c->host_ctl->ew_samples);
            stats->ewald_sample_err = c->host_ctl->ew_err;
            stats->queue_local = c->host_ctl->order_local;
        }
    }
    const int err = c->host_ctl->err;
    if (err & kErrTree) return fail(c, MGRAV_ERR_BAD_TREE, "tree check failed on the device");
    if (err & kErrList) return fail(c, MGRAV_ERR_BAD_LIST, "list check failed on the device");
    if (err & kErrParticle)
        return fail(c, MGRAV_ERR_INVALID_ARG, "non-finite position or non-positive mass");
    return MGRAV_OK;
}

mgrav_status mgrav_interact_variants(int* count) {
    if (!count) return fail(nullptr, MGRAV_ERR_INVALID_ARG, "count is NULL");
    *count = kNumVariants;
    return MGRAV_OK;
}

mgrav_status mgrav_interact_variant_info(int variant, int* pp_chunk, int* waves_per_simd,
                                         int* pc_prefetch) {
    if (variant < 0 || variant >= kNumVariants)
        return fail(nullptr, MGRAV_ERR_INVALID_ARG, "variant out of range");
    if (pp_chunk) *pp_chunk = kVariantChunk[variant];
    if (waves_per_simd) *waves_per_simd = kVariantWaves[variant];
    if (pc_prefetch) *pc_prefetch = kVariantPrefetch[variant] ? 1 : 0;
    return MGRAV_OK;
}

mgrav_status mgrav_set_interact_variant(mgrav_ctx* c, int variant) {
    if (!c) return fail(nullptr, MGRAV_ERR_INVALID_ARG, "ctx is NULL");
    c->err.clear();
    if (variant < 0 || variant >= kNumVariants)
        return fail(c, MGRAV_ERR_INVALID_ARG, "variant out of range");
    c->variant = variant;
    return MGRAV_OK;
}

mgrav_status mgrav_autotune(mgrav_ctx* c, float* acc, float* pot, const char* cache_path,
                            double budget_ms, int* chosen, double* ms_per_variant) {
    if (!c) return fail(nullptr, MGRAV_ERR_INVALID_ARG, "ctx is NULL");
    c->err.clear();
    if (!c->bound) return fail(c, MGRAV_ERR_STATE, "autotune before bind");
    if (!acc || !pot) return fail(c, MGRAV_ERR_INVALID_ARG, "null output");
    if (!(budget_ms >= 0.0)) return fail(c, MGRAV_ERR_INVALID_ARG, "budget_ms must be >= 0");
    if (ms_per_variant)
        for (int v = 0; v < kNumVariants; ++v) ms_per_variant[v] = -1.0;
    // cache key: the library build (digest of its kernel sources: variant
    // indices and register strategies change between builds), device, CU
    // count, the shape of the bound lists, the Ewald mode (with exact Ewald
    // direct launches or the graph's parallel branch overlap it with the
    // PP + PC kernel) and whether a mask is set
    char key[320];
    std::snprintf(key, sizeof(key), "%s/%s/cu%d/n%lld/b%lld/pp%lld/pc%lld/img%d/ew%d/mask%d",
                  MGRAV_SOURCE_DIGEST, c->arch.c_str(), c->n_cu, (long long)c->prob.n,
                  (long long)c->prob.n_bucket, (long long)c->prob.n_pp, (long long)c->prob.n_pc,
                  c->prob.n_images, c->ewald.mode, c->active ? 1 : 0);
    if (cache_path) {
        int hit = -1;
        if (FILE* f = std::fopen(cache_path, "r")) {
            // lines "mgrav-autotune <key> <variant> <launch mode>"; other
            // lines are ignored, the last match wins
            char line[512], k[320];
            int v = -1, m = 0, hit_mode = 0;
            while (std::fgets(line, sizeof(line), f)) {
                if (std::sscanf(line, "mgrav-autotune %319s %d %d", k, &v, &m) == 3 &&
                    std::strcmp(k, key) == 0 && v >= 0 && v < kNumVariants && (m == 0 || m == 1)) {
                    hit = v;
                    hit_mode = m;
                }
            }
            std::fclose(f);
            if (hit >= 0) {
                c->variant = hit;
                c->direct = hit_mode == MGRAV_LAUNCH_DIRECT;
                if (chosen) *chosen = hit;
                return MGRAV_OK;
            }
        }
    }
    const int saved = c->variant;
    const auto t0 = std::chrono::steady_clock::now();
    double best = 0.0;
    int best_v = saved;
    double med_v[kNumVariants];
    for (int v = 0; v < kNumVariants; ++v) {
        c->variant = v;
        double ms[8];
        int got = 0;
        // the first run of a variant captures its graph and is not timed;
        // at least two timed runs each, more while the budget lasts
        for (int rep = 0; rep < 9; ++rep) {
            mgrav_status st = mgrav_compute_parts(c, MGRAV_PART_PP | MGRAV_PART_PC, acc, pot);
            mgrav_stats stats{};
            if (st == MGRAV_OK) st = mgrav_wait(c, 60.0, &stats);
            if (st != MGRAV_OK) {
                c->variant = saved;
                return st;
            }
            if (rep > 0) ms[got++] = stats.ms_interact;
            const double spent =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                    .count();
            if (got >= 2 && spent > budget_ms * (v + 1) / kNumVariants) break;
        }
        for (int i = 1; i < got; ++i)  // median of the timed runs
            for (int j = i; j > 0 && ms[j] < ms[j - 1]; --j) std::swap(ms[j], ms[j - 1]);
        const double med = got % 2 ? ms[got / 2] : 0.5 * (ms[got / 2 - 1] + ms[got / 2]);
        if (ms_per_variant) ms_per_variant[v] = med;
        med_v[v] = med;
        if (v == 0 || med < best) {
            best = med;
            best_v = v;
        }
    }
    // Variant and launch mode together: wall time of back-to-back computes of
    // every part, from a graph and from direct launches, for the fastest
    // variant by its PP + PC time and, if that one is not a 2-wave variant,
    // for the fastest 2-wave one as well: with exact Ewald and direct
    // launches only a 2-wave variant leaves each SIMD room for the
    // correction to run beside it from the start, which can outweigh a
    // slower kernel.  Graphs are kept unless direct launches are faster.
    int cand[2] = {best_v, -1};
    if (kVariantWaves[best_v] != 2) {
        for (int v = 0; v < kNumVariants; ++v)
            if (kVariantWaves[v] == 2 && (cand[1] < 0 || med_v[v] < med_v[cand[1]])) cand[1] = v;
    }
    double best_wall = 0.0;
    int final_v = best_v, final_direct = 0;
    for (int ci = 0; ci < 2; ++ci) {
        if (cand[ci] < 0) continue;
        c->variant = cand[ci];
        for (int mode = 0; mode < 2; ++mode) {
            c->direct = mode == MGRAV_LAUNCH_DIRECT;
            drop_graph(c);
            // two warm-up computes (the first captures); the second, waited
            // for, sizes the timed run: 3 to 12 computes, about a quarter
            // of the budget
            mgrav_status st = MGRAV_OK;
            double one_ms = 0.0;
            for (int rep = 0; rep < 2 && st == MGRAV_OK; ++rep) {
                const auto w0 = std::chrono::steady_clock::now();
                st = mgrav_compute_parts(c, MGRAV_PART_ALL, acc, pot);
                if (st == MGRAV_OK) st = mgrav_wait(c, 60.0, nullptr);
                one_ms = std::chrono::duration<double, std::milli>(
                             std::chrono::steady_clock::now() - w0).count();
            }
            const int reps = std::max(3, std::min(12, int(0.25 * budget_ms / (one_ms + 1e-3))));
            const auto m0 = std::chrono::steady_clock::now();
            for (int rep = 0; rep < reps && st == MGRAV_OK; ++rep)
                st = mgrav_compute_parts(c, MGRAV_PART_ALL, acc, pot);
            if (st == MGRAV_OK) st = mgrav_wait(c, 60.0, nullptr);
            if (st != MGRAV_OK) {
                c->variant = saved;
                c->direct = false;
                return st;
            }
            const double wall =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - m0)
                    .count() / reps;
            if ((ci == 0 && mode == 0) || wall < best_wall) {
                best_wall = wall;
                final_v = cand[ci];
                final_direct = mode;
            }
        }
    }
    best_v = final_v;
    c->variant = best_v;
    if (c->direct != (final_direct == 1)) drop_graph(c);
    c->direct = final_direct == 1;
    if (chosen) *chosen = best_v;
    if (cache_path) {
        FILE* f = std::fopen(cache_path, "a");
        if (!f) return fail(c, MGRAV_ERR_INVALID_ARG, "cannot append to cache_path (variant applied)");
        std::fprintf(f, "mgrav-autotune %s %d %d\n", key, best_v, c->direct ? 1 : 0);
        std::fclose(f);
    }
    return MGRAV_OK;
}

mgrav_status mgrav_set_queue_order(mgrav_ctx* c, int order) {
    if (!c) return fail(nullptr, MGRAV_ERR_INVALID_ARG, "ctx is NULL");
    c->err.clear();
    if (order != MGRAV_QUEUE_AUTO && order != MGRAV_QUEUE_LPT && order != MGRAV_QUEUE_LOCAL)
        return fail(c, MGRAV_ERR_INVALID_ARG, "order must be MGRAV_QUEUE_AUTO, _LPT or _LOCAL");
    c->queue_order = order;  // the captured launches are rebuilt when their arguments differ
    return MGRAV_OK;
}

mgrav_status mgrav_set_launch_mode(mgrav_ctx* c, int mode) {
    if (!c) return fail(nullptr, MGRAV_ERR_INVALID_ARG, "ctx is NULL");
    c->err.clear();
    if (mode != MGRAV_LAUNCH_GRAPH && mode != MGRAV_LAUNCH_DIRECT)
        return fail(c, MGRAV_ERR_INVALID_ARG, "mode must be MGRAV_LAUNCH_GRAPH or _DIRECT");
    if (c->direct != (mode == MGRAV_LAUNCH_DIRECT)) drop_graph(c);
    c->direct = mode == MGRAV_LAUNCH_DIRECT;
    return MGRAV_OK;
}

}  // extern "C"

#include "mlp_api.inc"
#include "tree_dev.inc"
#include "store.inc"
#include "fmm.inc"
