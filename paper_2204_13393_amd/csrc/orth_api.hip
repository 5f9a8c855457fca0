// C-ABI runtime: argument checks, workspace carving and the per-step launch
// sequence of TreeTSPQR (Sec. 4.1) with BCGS-PIP+ at the leaves and at the
// single reduction level (Sec. 3.1; the paper recommends BCGS-PIP+ for the
// reduction across processes, Sec. 5.2).
//
// Workspace carving (all regions 256-byte aligned, column-major FP64):
//   Qloc  the leaf bases: leaf i's m_i x kmax block at i * ldl * kmax with
//         leading dimension ldl (ld_last for the last leaf) -- one leaf's
//         columns together in memory (a few pages rather than one page per
//         column); Householder leaves and the batched form keep one
//         ldq x kmax column-major matrix
//   T     ldt x kmax     tree factors; leaf i's T_i (kmax x kmax, upper
//                        triangular) in rows [i*kmax, (i+1)*kmax)
//   Y     ldt x s        reduction-level X: leaf i's [P_i; N_i] in its rows
//   U1L   ldq x s        leaf sweep-1 block u1
//   U1R   ldt x s        reduction sweep-1 block
//   CA    ldt x 16       apply_Q scratch (per-leaf coefficient blocks)
//   partL nchunkL x (kmax+s) x s   leaf chunk partial Gram blocks
//   partR nchunkR x (kmax+s) x s   reduction chunk partials
//   smallL p x rec       per-leaf P1, N1, N1^{-1}, P2, N2^{-1}
//   smallR 1 x rec
//   status               DevStatus

#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/orth.h"
#include "../../include/orth_measure.h"
#include "orth_deflate.h"
#include "orth_internal.h"

using namespace orth;

namespace {

constexpr int64_t kAlign = 32;        // doubles (256 bytes)
constexpr int64_t kWideGrid = 256;    // workgroups per launch below which chunks shrink (one per CU)
constexpr int kApplyMB = 16;

// Scratch of orth_apply_Q_noalloc: the per-leaf coefficient blocks of one
// column block live in this file-scope device array instead of the handle's
// workspace, so that call needs no device memory of its own.  32 MiB; every
// GPU the library runs on holds its own copy until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in): static_scratch() looks up each device's address once.
constexpr int64_t kStaticScratchDoubles = (int64_t)4 << 20;
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on device dev (looked up with dev current)
hipError_t static_scratch(int dev, double **out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }
int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Leading dimension of a stored basis: an odd multiple of 256 bytes.  With a
// power-of-two column stride every column of a wide operand starts at the
// same offset modulo the memory interleave, and the Gram products (which
// read 64 columns per wave at once) measured about 14% slower at n = 2^24.
int64_t basis_ld(int64_t rows) {
    int64_t ld = round_up(rows, kAlign);
    if ((ld / kAlign) % 2 == 0) ld += kAlign;
    return ld;
}

bool valid_s(int32_t s) { return s == 1 || s == 2 || s == 4 || s == 8 || s == 16 || s == 32; }

// widest basis (k_max + s) the planner accepts
int32_t max_cols(int32_t) { return 2048; }

// levels of a reduction tree the planner accepts (fan-in >= 2 over at most
// 2^31 leaves needs at most 31)
constexpr int kMaxLevels = 32;

struct Plan {
    int64_t n;
    int32_t s, kmax, leaf_rows, p;
    // reduction tree (Sec. 4.1, "applied recursively"): nlev levels, level l
    // has nchild[l] child segments grouped into nnode[l] nodes of fan_in
    // (the last node takes the rest); level 0's children are the leaves and
    // level nlev - 1 is the single root.  fan_in = 0: one level.
    int32_t fan_in, nlev;
    int32_t nchild[kMaxLevels], nnode[kMaxLevels];
    int64_t ldtl[kMaxLevels];     // ld of level l's stacked factor, X and U1 (ldtl[0] = ldt)
    // per-level regions (level 0's factor, X and U1 are oT, oY, oU1R; the
    // root's records oSR when nlev = 1); oCl[l]: the [P2 | C] records of
    // level l's nodes, for the levels below the root
    int64_t oTl[kMaxLevels], oYl[kMaxLevels], oU1l[kMaxLevels], oSl[kMaxLevels], oCl[kMaxLevels];
    int32_t precision;           // ORTH_FP64, ORTH_MIXED_SPLIT32 (adds the FP32 copy of the leaf
                                 // bases) or ORTH_FP64_HOUSEHOLDER (reflector leaves)
    int64_t ldq, ldt;
    bool qblk;                   // leaf bases stored leaf by leaf (ldl, ld_last)
    int64_t ldl, ld_last, qcount;
    int32_t nchunkL, nchunkR;
    // chunk heights (rows per workgroup): leaf Gram, leaf row updates,
    // reduction Gram, reduction row updates
    int32_t cL, cF, cR, cRR;
    bool rowreg = false;         // leaf row updates on the register-streamed kernel at every width
    // region offsets in doubles
    int64_t oQ, oT, oY, oU1L, oU1R, oCA, oPL, oPR, oPR2, oSL, oSR, oST, oQH, oCL, oTH, oCA2, oDF, total;
    // Householder reduction (every node's stacked problem within one
    // workgroup's panel): per level the nodes' compact-WY factors and the
    // explicit new columns; the root's coefficient record and [P; N]; a
    // third apply scratch
    bool hhtree;
    int64_t oTHl[kMaxLevels], oURl[kMaxLevels], oCR, oHR, oCA3;
    int64_t slot_cap, red_cap;   // doubles of each partial-slot region and of the pre-sum region
};

int32_t default_leaf_rows(int64_t n, int32_t kmax) {
    int64_t lr = n < 4096 ? n : 4096;
    if (lr < kmax) lr = kmax;
    return (int32_t)lr;
}

// children of the widest node of tree level l
int32_t hh_node_children(const Plan &pl, int l) {
    return pl.fan_in == 0 ? pl.nchild[l] : std::min(pl.fan_in, pl.nchild[l]);
}

// tree level l for the Householder reduction: its children's k_max physical
// rows each, its nodes as the kernels' leaves
LevelGeom hh_level_geom(const Plan &pl, int l, int chunk) {
    const int64_t rows = (int64_t)pl.nchild[l] * pl.kmax;
    return make_leaf_geom(rows, (int32_t)((int64_t)hh_node_children(pl, l) * pl.kmax), pl.nnode[l], chunk);
}

bool is_pow2_in(int32_t v, int32_t lo, int32_t hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

// tile heights a caller may ask for (0: the plan's own choice)
bool valid_tiles(const orth_tiles *t) {
    if (!t) return true;
    if (t->gram_rows != 0 && !is_pow2_in(t->gram_rows, 128, 8192)) return false;
    if (t->update_rows != 0 && !is_pow2_in(t->update_rows, 64, 8192)) return false;
    return t->update_kernel == ORTH_TILE_AUTO || t->update_kernel == ORTH_TILE_REGISTER;
}

bool make_plan(int64_t n, int32_t s, int32_t kmax, int32_t leaf_rows, int32_t precision, Plan &pl,
               int *why, int32_t fan_in = 0, bool blocked = false, const orth_tiles *tiles = nullptr) {
    *why = ORTH_ERR_ARG;
    if (fan_in < 0 || fan_in == 1) return false;
    if (!valid_tiles(tiles)) return false;
    if (n < 1 || !valid_s(s) || kmax < s || kmax % s != 0) return false;
    if (precision != ORTH_FP64 && precision != ORTH_MIXED_SPLIT32 && precision != ORTH_FP64_HOUSEHOLDER)
        return false;
    if (kmax + s > max_cols(s)) { *why = ORTH_ERR_UNSUPPORTED; return false; }
    if (leaf_rows == 0) leaf_rows = default_leaf_rows(n, kmax);
    if (leaf_rows < kmax || leaf_rows > n) return false;
    if (n > ((int64_t)1 << 40)) return false;
    if (precision == ORTH_FP64_HOUSEHOLDER) {
        // the panel kernel holds a whole leaf in registers, the per-leaf
        // small products stage k_max x s blocks in LDS
        const int32_t p = std::max<int32_t>(1, (int32_t)(n / leaf_rows));
        const int64_t last = n - (int64_t)(p - 1) * leaf_rows;
        const int64_t rows_max = std::max<int64_t>(last, p > 1 ? leaf_rows : last);
        if (hh_max_leaf_rows(s) == 0 || rows_max > hh_max_leaf_rows(s) || !hh_small_fits(s, kmax)) {
            *why = ORTH_ERR_UNSUPPORTED;
            return false;
        }
    }
    pl.n = n;
    pl.s = s;
    pl.kmax = kmax;
    pl.precision = precision;
    pl.leaf_rows = leaf_rows;
    pl.p = (int32_t)(n / leaf_rows);
    if (pl.p < 1) pl.p = 1;
    pl.ldq = basis_ld(n);
    pl.ldt = basis_ld((int64_t)pl.p * kmax);
    pl.qblk = blocked && precision != ORTH_FP64_HOUSEHOLDER;
    {
        const int64_t last_rows = n - (int64_t)(pl.p - 1) * leaf_rows;
        pl.ldl = pl.qblk ? basis_ld(leaf_rows) : pl.ldq;
        pl.ld_last = pl.qblk ? basis_ld(last_rows) : pl.ldq;
        pl.qcount = pl.qblk ? ((int64_t)(pl.p - 1) * pl.ldl + pl.ld_last) * kmax : pl.ldq * kmax;
    }
    // the tree's levels: fan_in = 0 (or >= p) is the single reduction level
    pl.fan_in = (fan_in == 0 || fan_in >= pl.p) ? 0 : fan_in;
    pl.nlev = 0;
    for (int32_t count = pl.p;;) {
        if (pl.nlev == kMaxLevels) return false;
        const int32_t nodes = pl.fan_in == 0 ? 1 : (int32_t)ceil_div(count, pl.fan_in);
        pl.nchild[pl.nlev] = count;
        pl.nnode[pl.nlev] = nodes;
        pl.ldtl[pl.nlev] = basis_ld((int64_t)count * kmax);
        ++pl.nlev;
        if (nodes == 1) break;
        count = nodes;
    }
    // chunk heights: the defaults, halved (down to 128 rows for the Grams and
    // 64 for the row updates) while a launch would have fewer workgroups than
    // the chip has compute units -- a small problem is bound by each
    // workgroup's serial walk over its rows, not by its bytes
    {
        auto shrink = [](int32_t c, int32_t cmin, auto count) {
            while (c > cmin && count(c) < kWideGrid) c /= 2;
            return c;
        };
        auto leaf_chunks = [&](int32_t c) { return (int64_t)make_leaf_geom(n, leaf_rows, pl.p, c).nchunks(); };
        auto root_chunks = [&](int32_t c) { return ceil_div((int64_t)pl.p * kmax, c); };
        // (a single leaf keeps its chunks: its many slots would go through
        // the grouped pre-sums, which the batched form does not take)
        pl.cL = pl.p > 1 ? shrink(kLeafChunk, 128, leaf_chunks) : kLeafChunk;
        pl.cF = shrink(kFinalChunk, 64, leaf_chunks);
        pl.cR = shrink(kRootChunk, 128, root_chunks);
        pl.cRR = shrink(kRootRowChunk, 64, root_chunks);
        // the caller's tile heights for the leaf passes
        if (tiles && tiles->gram_rows) pl.cL = tiles->gram_rows;
        if (tiles && tiles->update_rows) pl.cF = tiles->update_rows;
        pl.rowreg = tiles && tiles->update_kernel == ORTH_TILE_REGISTER;
    }
    // the Householder reduction is offered when every node's stacked problem
    // (its children's k_max physical rows each) fits the panel kernel
    pl.hhtree = hh_max_leaf_rows(s) > 0 && hh_small_fits(s, kmax);
    for (int l = 0; l < pl.nlev && pl.hhtree; ++l)
        pl.hhtree = (int64_t)hh_node_children(pl, l) * kmax <= hh_max_leaf_rows(s);
    const int64_t last = n - (int64_t)(pl.p - 1) * leaf_rows;
    const int64_t cpl = ceil_div(leaf_rows, pl.cL), cpl_last = ceil_div(last, pl.cL);
    pl.nchunkL = (int32_t)((pl.p - 1) * cpl + cpl_last);
    pl.nchunkR = (int32_t)ceil_div((int64_t)pl.p * kmax, pl.cR);
    int64_t off = 0;
    auto take = [&](int64_t count) {
        const int64_t o = off;
        off = round_up(off + count, kAlign);
        return o;
    };
    pl.oQ = take(pl.qcount);
    pl.oT = take(pl.ldt * kmax);
    pl.oY = take(pl.ldt * s);
    pl.oU1L = take(pl.ldq * s);
    pl.oU1R = take(pl.ldt * s);
    pl.oCA = take(pl.ldt * kApplyMB);
    // partial Gram slots are packed per step: chunk c, row group g at
    // (c * RG + g) * (k + s) * s; size for the largest step
    int64_t slot_max = 0, red_max = 0;
    for (int32_t k = 0; k + s <= kmax; k += s) {
        const int32_t ncol = k + s;
        const int64_t per = (int64_t)gram_row_groups(ncol) * ncol * s;
        int64_t nR = ceil_div((int64_t)pl.p * ncol, pl.cR);
        for (int l = 0; l < pl.nlev; ++l) {
            nR = std::max(nR, (int64_t)make_tree_geom(pl.nchild[l], pl.fan_in == 0 ? pl.nchild[l] : pl.fan_in,
                                                      kmax, ncol, pl.cR).nchunks());
            // the Householder reduction's levels run over the physical rows
            if (pl.hhtree) nR = std::max(nR, (int64_t)hh_level_geom(pl, l, pl.cR).nchunks());
        }
        slot_max = std::max(slot_max, std::max((int64_t)pl.nchunkL, nR) * per);
        // pre-summed slot groups of a level with a single local problem: the
        // reduction level, and the leaf level when there is one leaf
        const int64_t nroot = ceil_div((int64_t)pl.nchild[pl.nlev - 1] * ncol, pl.cR);
        const int64_t single = pl.p == 1 ? std::max((int64_t)pl.nchunkL, nroot) : nroot;
        red_max = std::max(red_max, ceil_div(single * gram_row_groups(ncol), kReduceGroup) * ncol * s);
    }
    pl.oPL = take(slot_max);
    pl.oPR = take(slot_max);
    pl.oPR2 = take(red_max);
    pl.slot_cap = slot_max;
    pl.red_cap = red_max;
    pl.oSL = take((int64_t)pl.p * small_stride(kmax, s));
    pl.oSR = take(small_stride(kmax, s));
    pl.oST = take(sizeof(DevStatus) / sizeof(double) + 1);
    // per-leaf coefficient records [P2 | C_i], row-major (k_max x 2s per leaf)
    pl.oCL = take((int64_t)pl.p * kmax * 2 * s);
    // mixed form: FP32 copy of the leaf bases (their layout, in floats)
    pl.oQH = precision == ORTH_MIXED_SPLIT32 ? take(ceil_div(pl.qcount, 2)) : 0;
    // Householder leaves: per leaf the compact-WY factor (column- and
    // row-major) and the reflectors' top rows (row-major), k_max x k_max each
    pl.oTH = precision == ORTH_FP64_HOUSEHOLDER ? take((int64_t)3 * pl.p * kmax * kmax) : 0;
    // and orth_apply_Q's second coefficient scratch (-Z_i, or the tree's
    // down-sweep in turn with CA), like CA
    pl.oCA2 = (precision == ORTH_FP64_HOUSEHOLDER || pl.nlev > 1 || pl.hhtree) ? take(pl.ldt * kApplyMB) : 0;
    for (int l = 0; l < pl.nlev; ++l) {
        pl.oTHl[l] = pl.hhtree ? take((int64_t)3 * pl.nnode[l] * kmax * kmax) : 0;
        pl.oURl[l] = pl.hhtree ? take(pl.ldtl[l] * s) : 0;
    }
    pl.oCR = pl.hhtree ? take((int64_t)kmax * 2 * s) : 0;
    pl.oHR = pl.hhtree ? take((int64_t)kmax * s) : 0;
    // a third region: the Householder reduction's apply, and Householder
    // leaves under a tree (their -Z_i beside the down-sweep's two regions)
    pl.oCA3 = (pl.hhtree || (precision == ORTH_FP64_HOUSEHOLDER && pl.nlev > 1)) ? take(pl.ldt * kApplyMB) : 0;
    // deflation state (counters and the first sweep's s x s W), Householder leaves only
    pl.oDF = precision == ORTH_FP64_HOUSEHOLDER ? take(defl_state_doubles(s)) : 0;
    // the tree's levels: level 0 stacks the leaves' factors in T, Y, U1R;
    // every level above has its own; records per node (the root's is SR
    // for a single level)
    for (int l = 0; l < pl.nlev; ++l) {
        const bool root = l == pl.nlev - 1;
        pl.oTl[l] = l == 0 ? pl.oT : take(pl.ldtl[l] * kmax);
        pl.oYl[l] = l == 0 ? pl.oY : take(pl.ldtl[l] * s);
        pl.oU1l[l] = l == 0 ? pl.oU1R : take(pl.ldtl[l] * s);
        pl.oSl[l] = (root && pl.nlev == 1) ? pl.oSR : take((int64_t)pl.nnode[l] * small_stride(kmax, s));
        pl.oCl[l] = root ? 0 : take((int64_t)pl.nnode[l] * kmax * 2 * s);
    }
    pl.total = off;
    return true;
}

LevelGeom leaf_geom(const Plan &pl, int chunk) { return make_leaf_geom(pl.n, pl.leaf_rows, pl.p, chunk); }

// level l of the reduction tree (level 0 over the leaves)
LevelGeom tree_geom(const Plan &pl, int l, int64_t seg_len, int chunk) {
    return make_tree_geom(pl.nchild[l], pl.fan_in == 0 ? pl.nchild[l] : pl.fan_in, pl.kmax, seg_len, chunk);
}

}  // namespace

namespace {

// FlatTSPQR (Sec. 4.2): the rows in blocks of block_rows (the last takes the
// rest), the basis as the chain of per-block factors.  Factor i is stored
// with block i's m_i rows first and the chain's coordinates after them
// (F_i: rows [0, m_i) and [m_i, m_i + k_max), k_max columns, ld ldf[i]);
// the local problem of block i at width k is the PQR problem on the
// contiguous rows [0, m_i + k + s) of F_i and of Y_i = [X_i; P_{i-1};
// N_{i-1}] (a row order the PQR problem does not depend on).  Coordinate
// rows k .. k+s-1 of the old columns are the zero rows Sec. 4.2's
// extended factor inserts: the factors start at zero and those rows are
// only written by later columns.
struct FlatPlan {
    int64_t n = 0;
    int32_t s = 0, kmax = 0, block_rows = 0;
    int32_t p = 0;
    std::vector<int64_t> r0, rows, ldf, oF, oY;
    int64_t ldmax = 0;                 // ld of the shared U1 scratch
    int64_t oU1 = 0, oZ0 = 0, oZ1 = 0, oE = 0, oP = 0, oP2 = 0, oS = 0, oST = 0;
    int64_t slot_cap = 0, red_cap = 0, total = 0;
};

bool make_flat_plan(int64_t n, int32_t s, int32_t kmax, int32_t block_rows, FlatPlan &fp) {
    if (n < 1 || !valid_s(s) || kmax < s || kmax % s != 0 || kmax + s > max_cols(s)) return false;
    if (block_rows < kmax || block_rows > n || block_rows > (1 << 29)) return false;
    fp.n = n;
    fp.s = s;
    fp.kmax = kmax;
    fp.block_rows = block_rows;
    const int64_t p64 = std::max<int64_t>(1, n / block_rows);
    if (p64 > (1 << 20)) return false;
    fp.p = (int32_t)p64;
    fp.r0.assign(fp.p, 0);
    fp.rows.assign(fp.p, 0);
    fp.ldf.assign(fp.p, 0);
    fp.oF.assign(fp.p, 0);
    fp.oY.assign(fp.p, 0);
    int64_t off = 0, rows_max = 0;
    auto take = [&](int64_t count) {
        const int64_t o = off;
        off = round_up(off + count, kAlign);
        return o;
    };
    for (int32_t i = 0; i < fp.p; ++i) {
        fp.r0[i] = (int64_t)i * block_rows;
        fp.rows[i] = i == fp.p - 1 ? n - fp.r0[i] : block_rows;
        fp.ldf[i] = basis_ld(fp.rows[i] + kmax);
        rows_max = std::max(rows_max, fp.rows[i] + kmax);
        fp.oF[i] = take(fp.ldf[i] * kmax);
        fp.oY[i] = i == 0 ? 0 : take(fp.ldf[i] * s);   // block 1 reads W itself
    }
    fp.ldmax = basis_ld(rows_max);
    fp.oU1 = take(fp.ldmax * s);
    fp.oZ0 = take((int64_t)kmax * kApplyMB);     // chain coordinates of one column block
    fp.oZ1 = take((int64_t)kmax * kApplyMB);
    fp.oE = take((int64_t)(kmax + s) * s);        // [0; I_s] below k_max zero rows
    // partial slots of one local problem (a single leaf of up to rows_max rows)
    int64_t slot_max = 0, red_max = 0;
    for (int32_t k = 0; k + s <= kmax; k += s) {
        const int32_t ncol = k + s;
        const int64_t chunks = ceil_div(rows_max, kLeafChunk);
        slot_max = std::max(slot_max, chunks * gram_row_groups(ncol) * ncol * s);
        red_max = std::max(red_max, ceil_div(chunks * gram_row_groups(ncol), kReduceGroup) * ncol * s);
    }
    fp.slot_cap = slot_max;
    fp.red_cap = red_max;
    fp.oP = take(slot_max);
    fp.oP2 = take(red_max);
    fp.oS = take(small_stride(kmax, s));
    fp.oST = take(sizeof(DevStatus) / sizeof(double) + 1);
    fp.total = off;
    return true;
}

}  // namespace

struct orth_ctx {
    Plan pl;
    bool flat = false;                     // FlatTSPQR handle (orth_create_flat)
    FlatPlan fp;
    int32_t k = 0;
    int32_t variant = ORTH_PIP_PLUS;       // the leaves' subalgorithm
    int32_t variant_red = ORTH_PIP_PLUS;   // the reduction's
    double defl_delta = 0.0;               // > 0: the reduction level deflates (Sec. 3.1)
    bool poisoned = false;
    hipStream_t stream = nullptr;
    int device = 0;                        // the stream's device
    double *ws = nullptr;
    // profiler: event pairs recorded around launches
    bool prof_on = false;
    uint32_t prof_mask = ~0u;
    struct Mark { int cls; hipEvent_t a, b; };
    std::vector<Mark> marks;
    std::vector<hipEvent_t> spare;
    double prof_ms[ORTH_K_COUNT] = {};
    int64_t prof_n[ORTH_K_COUNT] = {};

    hipEvent_t get_event() {
        if (!spare.empty()) {
            hipEvent_t e = spare.back();
            spare.pop_back();
            return e;
        }
        // timing-only events: no system-scope fence (its cache writeback
        // and invalidation would slow the bracketed work); the read
        // synchronises the stream before taking the times
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
        return e;
    }
    // bracket one launch; returns the mark index or -1
    int begin(int cls) {
        if (!prof_on || !((prof_mask >> cls) & 1u)) return -1;
        Mark m{cls, get_event(), get_event()};
        if (!m.a || !m.b || hipEventRecord(m.a, stream) != hipSuccess) return -1;
        marks.push_back(m);
        return (int)marks.size() - 1;
    }
    void end(int idx) {
        if (idx >= 0) (void)hipEventRecord(marks[idx].b, stream);
    }
    ~orth_ctx() {
        for (auto &m : marks) { (void)hipEventDestroy(m.a); (void)hipEventDestroy(m.b); }
        for (auto e : spare) (void)hipEventDestroy(e);
    }

    double *Q() const { return ws + pl.oQ; }
    // the leaf bases as a kernel operand from column c0 on
    Operand Qop(int32_t c0 = 0) const {
        if (!pl.qblk) return Operand{Q() + (int64_t)c0 * pl.ldq, pl.ldq, 0, 0, 0};
        return Operand{Q(), pl.ldl, pl.ldl * pl.kmax, pl.ld_last, c0};
    }
    OutOperand Qout(int32_t c0) const {
        if (!pl.qblk) return OutOperand{Q() + (int64_t)c0 * pl.ldq, pl.ldq, 0, 0, 0};
        return OutOperand{Q(), pl.ldl, pl.ldl * pl.kmax, pl.ld_last, c0};
    }
    double *T() const { return ws + pl.oT; }
    double *Y() const { return ws + pl.oY; }
    double *U1L() const { return ws + pl.oU1L; }
    double *U1R() const { return ws + pl.oU1R; }
    double *CA() const { return ws + pl.oCA; }
    double *PL() const { return ws + pl.oPL; }
    double *CL() const { return ws + pl.oCL; }
    float *Qhi() const {
        return pl.precision == ORTH_MIXED_SPLIT32 ? reinterpret_cast<float *>(ws + pl.oQH) : nullptr;
    }
    // the copy's new columns from c0 on (a blocked copy takes c0 from Qout's operand)
    float *Qhi_at(int32_t c0) const {
        float *q = Qhi();
        return (q && !pl.qblk) ? q + (int64_t)c0 * pl.ldq : q;
    }
    double *TH() const { return pl.precision == ORTH_FP64_HOUSEHOLDER ? ws + pl.oTH : nullptr; }
    // second apply scratch: Householder leaves (-Z_i) and reduction trees (the
    // down-sweep alternates between CA and CA2)
    double *CA2() const {
        return (pl.precision == ORTH_FP64_HOUSEHOLDER || pl.nlev > 1 || pl.hhtree) ? ws + pl.oCA2 : nullptr;
    }
    // Householder reduction regions (null unless the plan offers it)
    bool hh_red() const { return variant_red == ORTH_HOUSEHOLDER; }
    double *THl(int l) const { return pl.hhtree ? ws + pl.oTHl[l] : nullptr; }
    double *URl(int l) const { return pl.hhtree ? ws + pl.oURl[l] : nullptr; }
    double *CR() const { return pl.hhtree ? ws + pl.oCR : nullptr; }
    double *HR() const { return pl.hhtree ? ws + pl.oHR : nullptr; }
    double *CA3() const {
        return (pl.hhtree || (pl.precision == ORTH_FP64_HOUSEHOLDER && pl.nlev > 1)) ? ws + pl.oCA3 : nullptr;
    }
    DeflState *DF() const {
        return pl.precision == ORTH_FP64_HOUSEHOLDER ? reinterpret_cast<DeflState *>(ws + pl.oDF) : nullptr;
    }
    double *PR() const { return ws + pl.oPR; }
    double *PR2() const { return ws + pl.oPR2; }
    // reduction tree level l: stacked factor, X, U1 scratch, node records
    double *Tl(int l) const { return ws + pl.oTl[l]; }
    double *Yl(int l) const { return ws + pl.oYl[l]; }
    double *U1l(int l) const { return ws + pl.oU1l[l]; }
    double *Sl(int l) const { return ws + pl.oSl[l]; }
    double *Cl(int l) const { return ws + pl.oCl[l]; }
    double *SL() const { return ws + pl.oSL; }
    double *SR() const { return ws + pl.oSR; }
    DevStatus *status() const { return reinterpret_cast<DevStatus *>(ws + (flat ? fp.oST : pl.oST)); }
};

extern "C" {

size_t orth_workspace_bytes(int64_t n, int32_t s, int32_t k_max, int32_t leaf_rows,
                            int32_t precision) {
    return orth_tree_workspace_bytes(n, s, k_max, leaf_rows, precision, 0);
}

size_t orth_tree_workspace_bytes(int64_t n, int32_t s, int32_t k_max, int32_t leaf_rows,
                                 int32_t precision, int32_t fan_in) {
    Plan pl;
    int why;
    if (!make_plan(n, s, k_max, leaf_rows, precision, pl, &why, fan_in, true)) return 0;
    return (size_t)pl.total * sizeof(double);
}

int orth_create(int64_t n, int32_t s, int32_t k_max, int32_t leaf_rows, int32_t precision,
                void *d_workspace, size_t workspace_bytes, void *stream, orth_t **out) {
    return orth_create_tree(n, s, k_max, leaf_rows, precision, 0, d_workspace, workspace_bytes, stream, out);
}

int orth_create_tree(int64_t n, int32_t s, int32_t k_max, int32_t leaf_rows, int32_t precision,
                     int32_t fan_in, void *d_workspace, size_t workspace_bytes, void *stream, orth_t **out) {
    return orth_create_tiles(n, s, k_max, leaf_rows, precision, fan_in, nullptr, d_workspace, workspace_bytes,
                             stream, out);
}

size_t orth_tiles_workspace_bytes(int64_t n, int32_t s, int32_t k_max, int32_t leaf_rows, int32_t precision,
                                  int32_t fan_in, const orth_tiles *tiles) {
    Plan pl;
    int why;
    if (!make_plan(n, s, k_max, leaf_rows, precision, pl, &why, fan_in, true, tiles)) return 0;
    return (size_t)pl.total * sizeof(double);
}

int orth_tiles_in_use(const orth_t *h, orth_tiles *tiles) {
    if (!h || !tiles) return ORTH_ERR_ARG;
    tiles->gram_rows = h->pl.cL;
    tiles->update_rows = h->pl.cF;
    tiles->update_kernel = h->pl.rowreg ? ORTH_TILE_REGISTER : ORTH_TILE_AUTO;
    return ORTH_OK;
}

int orth_create_tiles(int64_t n, int32_t s, int32_t k_max, int32_t leaf_rows, int32_t precision,
                      int32_t fan_in, const orth_tiles *tiles, void *d_workspace, size_t workspace_bytes,
                      void *stream, orth_t **out) {
    if (!out) return ORTH_ERR_ARG;
    *out = nullptr;
    Plan pl;
    int why;
    if (!make_plan(n, s, k_max, leaf_rows, precision, pl, &why, fan_in, true, tiles)) return why;
    if (!d_workspace || ((uintptr_t)d_workspace % 256) != 0 ||
        workspace_bytes < (size_t)pl.total * sizeof(double))
        return ORTH_ERR_WORKSPACE;
    orth_ctx *h = new (std::nothrow) orth_ctx();
    if (!h) return ORTH_ERR_HIP;
    h->pl = pl;
    h->stream = static_cast<hipStream_t>(stream);
    h->ws = static_cast<double *>(d_workspace);
    if (hipStreamGetDevice(h->stream, &h->device) != hipSuccess) {
        (void)hipGetLastError();
        delete h;
        return ORTH_ERR_HIP;
    }
    // tree factors must start at zero: the reduction level relies on the
    // zero rows below every T_i's current k x k block
    hipError_t e = prepare_kernels(pl.s);
    if (e == hipSuccess && (pl.precision == ORTH_FP64_HOUSEHOLDER || pl.hhtree)) e = prepare_hh_kernels(pl.s);
    for (int l = 0; l < pl.nlev && e == hipSuccess; ++l) {
        e = launch_fill(h->Tl(l), pl.ldtl[l] * (int64_t)pl.kmax, 0.0, h->stream);
        if (e == hipSuccess) e = launch_fill(h->Yl(l), pl.ldtl[l] * (int64_t)pl.s, 0.0, h->stream);
    }
    // Householder leaves: the compact-WY factors grow into zeros below their diagonal
    if (e == hipSuccess && h->TH())
        e = launch_fill(h->TH(), (int64_t)3 * pl.p * pl.kmax * pl.kmax, 0.0, h->stream);
    // and so do the Householder reduction's (with the reflectors' top rows)
    for (int l = 0; l < pl.nlev && e == hipSuccess && pl.hhtree; ++l)
        e = launch_fill(h->THl(l), (int64_t)3 * pl.nnode[l] * pl.kmax * pl.kmax, 0.0, h->stream);
    if (e == hipSuccess && h->DF())
        e = launch_fill_i32(reinterpret_cast<int32_t *>(h->DF()), (int64_t)(sizeof(DeflState) / sizeof(int32_t)), 0,
                            h->stream);
    if (e == hipSuccess)
        e = launch_fill_i32(reinterpret_cast<int32_t *>(h->status()),
                            (int64_t)(sizeof(DevStatus) / sizeof(int32_t)), 0, h->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete h;
        return ORTH_ERR_HIP;
    }
    *out = h;
    return ORTH_OK;
}

size_t orth_flat_workspace_bytes(int64_t n, int32_t s, int32_t k_max, int32_t block_rows) {
    FlatPlan fp;
    if (!make_flat_plan(n, s, k_max, block_rows, fp)) return 0;
    return (size_t)fp.total * sizeof(double);
}

int orth_create_flat(int64_t n, int32_t s, int32_t k_max, int32_t block_rows, void *d_workspace,
                     size_t workspace_bytes, void *stream, orth_t **out) {
    if (!out) return ORTH_ERR_ARG;
    *out = nullptr;
    FlatPlan fp;
    if (!make_flat_plan(n, s, k_max, block_rows, fp)) {
        return (valid_s(s) && k_max >= s && k_max % s == 0 && k_max + s > max_cols(s)) ? ORTH_ERR_UNSUPPORTED
                                                                                         : ORTH_ERR_ARG;
    }
    if (!d_workspace || ((uintptr_t)d_workspace % 256) != 0 ||
        workspace_bytes < (size_t)fp.total * sizeof(double))
        return ORTH_ERR_WORKSPACE;
    orth_ctx *h = new (std::nothrow) orth_ctx();
    if (!h) return ORTH_ERR_HIP;
    h->flat = true;
    h->fp = std::move(fp);
    // the level runs read the block width and capacity from the plan
    h->pl.n = n;
    h->pl.s = s;
    h->pl.kmax = k_max;
    h->pl.precision = ORTH_FP64;
    h->stream = static_cast<hipStream_t>(stream);
    h->ws = static_cast<double *>(d_workspace);
    if (hipStreamGetDevice(h->stream, &h->device) != hipSuccess) {
        (void)hipGetLastError();
        delete h;
        return ORTH_ERR_HIP;
    }
    // factors and staging start at zero (the rows a local problem inserts
    // for the newest coordinates are zero rows of the older columns); the
    // identity block of [0; I_s] sits at rows k_max .. k_max + s - 1
    const FlatPlan &f = h->fp;
    hipError_t e = prepare_kernels(s);
    if (e == hipSuccess) e = launch_fill(h->ws, f.total, 0.0, h->stream);
    for (int32_t j = 0; j < s && e == hipSuccess; ++j)
        e = launch_fill(h->ws + f.oE + (int64_t)j * (k_max + s) + k_max + j, 1, 1.0, h->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete h;
        return ORTH_ERR_HIP;
    }
    *out = h;
    return ORTH_OK;
}

int orth_set_variant(orth_t *h, int32_t variant) {
    return orth_set_level_variants(h, variant, variant);
}

int orth_set_level_variants(orth_t *h, int32_t leaf_variant, int32_t reduction_variant) {
    const auto ok = [](int32_t v) { return v == ORTH_PIP_PLUS || v == ORTH_PIP; };
    if (!h || !ok(leaf_variant) || !(ok(reduction_variant) || reduction_variant == ORTH_HOUSEHOLDER))
        return ORTH_ERR_ARG;
    if (h->poisoned) return ORTH_ERR_POISONED;
    // Householder at the reduction: single-level handles whose stacked
    // problem fits the panel kernel, not with deflation, not mid-basis
    if (reduction_variant == ORTH_HOUSEHOLDER && (h->flat || !h->pl.hhtree || h->defl_delta > 0.0))
        return ORTH_ERR_UNSUPPORTED;
    if ((reduction_variant == ORTH_HOUSEHOLDER) != (h->variant_red == ORTH_HOUSEHOLDER) && h->k > 0)
        return ORTH_ERR_UNSUPPORTED;
    // Householder leaves run Algorithm HH, which has no one-sweep variant
    if (h->pl.precision == ORTH_FP64_HOUSEHOLDER && leaf_variant != ORTH_PIP_PLUS) return ORTH_ERR_UNSUPPORTED;
    h->variant = leaf_variant;
    h->variant_red = reduction_variant;
    return ORTH_OK;
}

}  // extern "C"

namespace {

// One level of the tree: sweep-1 Gram, Cholesky, correction + sweep-2 Gram,
// Cholesky (the final one writes [P; N] to the next level's X, or H and R at
// the root).  Partial Gram slots are pre-summed in groups when a level has
// more than kReduceGroup of them per leaf.
struct LevelRun {
    Operand Q, X;
    const float *Qhi;              // mixed form, leaves: FP32 copy read by the sweep-1 Gram
    double *pc;                    // leaves: per-leaf [P2 | C] records (P2 half written by the Cholesky)
    OutOperand U1;
    LevelGeom geom;
    double *part, *part2;
    int64_t part_cap, part2_cap;   // doubles available at part and part2
    double *small;
    int level;
    // final outputs
    double *Yout;
    int64_t ldy, yseg;
    double *H;
    int64_t ldh;
    double *R;
    int64_t ldr;
    LevelGeom rgeom;      // chunks of the correction (row update) launch
    const DeflArgs *defl; // reduction level with deflation: eigen-based first sweep
};

int run_level(orth_ctx *h, const LevelRun &L, int k, bool two) {
    const Plan &pl = h->pl;
    const int32_t s = pl.s, kmax = pl.kmax, ncol = k + s;
    hipStream_t st = h->stream;
    const int64_t pstride = (int64_t)ncol * s;    // packed slot stride of this step
    const int cls0 = L.level == 0 ? 0 : 3;          // LEAF_* or ROOT_* classes
    hipError_t e;

    // host check of the Gram grid against the partial-slot region it writes
    if ((int64_t)L.geom.nchunks() * gram_row_groups(ncol) * pstride > L.part_cap) return ORTH_ERR_HIP;
    GramArgs ga{};
    ga.Q = L.Q;
    ga.Qhi = L.Qhi;
    ga.X = L.X;
    ga.k = k;
    ga.tile_groups = gram_tile_groups(ncol);
    ga.geom = L.geom;
    ga.partials = L.part;
    ga.part_stride = pstride;
    ga.status = h->status();
    ga.clear_retry = L.Qhi ? 1 : 0;
    ga.retry = &h->status()->retry;
    {
        const int pm = h->begin(cls0 + 0);
        e = launch_gram(s, ga, cls0 + 0, st);
        h->end(pm);
        if (e != hipSuccess) return ORTH_ERR_HIP;
    }
    CholArgs c{};
    c.part_stride = pstride;
    c.nleaf = L.geom.nleaf;
    c.k = k;
    c.kmax = kmax;
    c.level = L.level;
    c.final_sweep = two ? 2 : 1;
    c.small = L.small;
    c.small_stride = small_stride(kmax, s);
    c.Yout = L.Yout;
    c.ldy = L.ldy;
    c.yseg = L.yseg;
    c.H = L.H;
    c.ldh = L.ldh;
    c.R = L.R;
    c.ldr = L.ldr;
    c.instance = -1;
    c.pc = L.pc;
    c.pc_stride = (int64_t)kmax * 2 * s;
    c.status = h->status();
    c.retry = &h->status()->retry;

    // sum the slots of each leaf; pre-reduce when a single leaf owns many
    auto chol = [&](int sweep, int ppc, int cls, bool soft, bool cond) -> int {
        c.sweep = sweep;
        c.soft = soft ? 1 : 0;
        c.cond = cond ? 1 : 0;
        c.partials = L.part;
        c.slots_per_leaf = L.geom.cpl * ppc;
        c.slots_last = L.geom.cpl_last * ppc;
        if (L.geom.nleaf == 1 && c.slots_last > kReduceGroup) {
            // host check of the grid against the buffer it writes
            if (!L.part2 || ceil_div(c.slots_last, kReduceGroup) * pstride > L.part2_cap) return ORTH_ERR_HIP;
            ReduceArgs r{};
            r.in = L.part;
            r.stride = pstride;
            r.nslots = c.slots_last;
            r.group = kReduceGroup;
            r.nentries = ncol * s;
            r.out = L.part2;
            r.status = h->status();
            r.cond = cond ? 1 : 0;
            r.retry = &h->status()->retry;
            const int pm = h->begin(cls);
            e = launch_reduce(r, st);
            h->end(pm);
            if (e != hipSuccess) return ORTH_ERR_HIP;
            c.partials = L.part2;
            c.slots_per_leaf = c.slots_last = (int32_t)ceil_div(r.nslots, kReduceGroup);
        }
        const int pm = h->begin(cls);
        e = L.defl ? launch_defl(s, c, *L.defl, st) : launch_chol(s, c, st);
        h->end(pm);
        return e == hipSuccess ? ORTH_OK : ORTH_ERR_HIP;
    };
    // the mixed form's first sweep reads the FP32 copy: a failed pivot there
    // flags the step instead of breaking down
    if (int rc = chol(1, gram_row_groups(ncol), cls0 + 1, L.Qhi != nullptr, false)) return rc;
    if (L.Qhi) {
        // the fallback: redo the first sweep from the FP64 basis when flagged
        // (these launches return at once otherwise); a failure now is a breakdown
        GramArgs gf = ga;
        gf.Qhi = nullptr;
        gf.cond = 1;
        gf.clear_retry = 0;
        const int pm = h->begin(ORTH_K_LEAF_FALLBACK);
        e = launch_gram(s, gf, ORTH_K_LEAF_FALLBACK, st);
        h->end(pm);
        if (e != hipSuccess) return ORTH_ERR_HIP;
        if (int rc = chol(1, gram_row_groups(ncol), ORTH_K_LEAF_FALLBACK, false, true)) return rc;
    }

    // correction u1 = (x - q P1) N1^{-1}, stored to the level's U1 scratch
    FinalizeArgs f{};
    f.Q = L.Q;
    f.Qnew = L.U1;
    f.U1 = L.X;
    f.sweep = 1;
    f.k = k;
    f.geom = L.rgeom;
    f.reg_only = (L.level == 0 && pl.rowreg) ? 1 : 0;
    f.small = L.small;
    f.small_stride = small_stride(kmax, s);
    f.kmax = kmax;
    f.single_sweep = 0;
    f.Cptr = nullptr;
    f.status = h->status();
    {
        const int pm = h->begin(cls0 + 2);
        e = launch_finalize(s, f, cls0 + 2, st);
        if (e == hipSuccess && L.defl) {
            // after a drop the row update formed x - q P1; u1 = (x - q P1) W
            DeflRowArgs dr{};
            dr.U = L.U1.ptr;
            dr.ld = L.U1.ld;
            dr.geom = L.rgeom;
            dr.state = L.defl->state;
            dr.status = h->status();
            e = launch_defl_rows(s, dr, st);
        }
        h->end(pm);
        if (e != hipSuccess) return ORTH_ERR_HIP;
    }
    if (!two) return ORTH_OK;
    // sweep-2 Gram [Q U1]^T U1
    GramArgs g2 = ga;
    g2.Qhi = nullptr;             // the second sweep reads the FP64 basis
    g2.X = Operand{L.U1.ptr, L.U1.ld};
    {
        const int cls2 = L.level == 0 ? ORTH_K_LEAF_GRAM2 : ORTH_K_ROOT_GRAM2;
        const int pm = h->begin(cls2);
        e = launch_gram(s, g2, cls2, st);
        h->end(pm);
        if (e != hipSuccess) return ORTH_ERR_HIP;
    }
    return chol(2, gram_row_groups(ncol), cls0 + 1, false, false);
}

// Householder leaves (Sec. 2.2): w~ = Q_k^T w through the compact-WY form
// (Gram V^T w, T^T M, row update), the panel factorisation of w~[k:] in one
// workgroup per leaf ([P_i; N_i] to the reduction level, the s reflectors to
// the leaf basis), then the growth of T from [V v_new]^T v_new.
int run_leaves_hh(orth_ctx *h, const double *d_W, int64_t ldw, int k) {
    const Plan &pl = h->pl;
    const int32_t s = pl.s, kmax = pl.kmax, ncol = k + s;
    hipStream_t st = h->stream;
    const int64_t pstride = (int64_t)ncol * s;
    const LevelGeom gg = leaf_geom(pl, pl.cL);
    const int rg = gram_row_groups(ncol);
    if ((int64_t)gg.nchunks() * rg * pstride > pl.slot_cap) return ORTH_ERR_HIP;
    hipError_t e;
    HhArgs ha{};
    ha.geom = gg;
    ha.k = k;
    ha.kmax = kmax;
    ha.Q = h->Q();
    ha.ldq = pl.ldq;
    ha.T = h->TH();
    ha.partials = h->PL();
    ha.part_stride = pstride;
    ha.slots_per_leaf = gg.cpl * rg;
    ha.slots_last = gg.cpl_last * rg;
    ha.small = h->SL();
    ha.small_stride = small_stride(kmax, s);
    ha.Yout = h->Y();
    ha.ldy = pl.ldt;
    ha.yseg = kmax;
    ha.status = h->status();
    GramArgs ga{};
    ga.Q = Operand{h->Q(), pl.ldq};
    ga.k = k;
    ga.tile_groups = gram_tile_groups(ncol);
    ga.geom = gg;
    ga.partials = h->PL();
    ga.part_stride = pstride;
    ga.status = h->status();
    ha.X = d_W;
    ha.ldx = ldw;
    if (k > 0) {
        ga.X = Operand{d_W, ldw};
        int pm = h->begin(ORTH_K_LEAF_GRAM);
        e = launch_gram(s, ga, ORTH_K_LEAF_GRAM, st);
        h->end(pm);
        if (e != hipSuccess) return ORTH_ERR_HIP;
        pm = h->begin(ORTH_K_LEAF_HH_SMALL);
        e = launch_hh(s, HH_PREP, ha, st);
        h->end(pm);
        if (e != hipSuccess) return ORTH_ERR_HIP;
        // w~ = w - V (T^T M) into the leaf scratch
        FinalizeArgs f{};
        f.Q = Operand{h->Q(), pl.ldq};
        f.Qnew = OutOperand{h->U1L(), pl.ldq};
        f.U1 = Operand{d_W, ldw};
        f.sweep = 1;
        f.k = k;
        f.geom = leaf_geom(pl, pl.cF);
        f.reg_only = pl.rowreg ? 1 : 0;
        f.small = h->SL();
        f.small_stride = small_stride(kmax, s);
        f.kmax = kmax;
        f.status = h->status();
        pm = h->begin(ORTH_K_LEAF_CORRECT);
        e = launch_finalize(s, f, ORTH_K_LEAF_CORRECT, st);
        h->end(pm);
        if (e != hipSuccess) return ORTH_ERR_HIP;
        ha.X = h->U1L();
        ha.ldx = pl.ldq;
    }
    int pm = h->begin(ORTH_K_LEAF_HH_PANEL);
    e = launch_hh(s, HH_PANEL, ha, st);
    h->end(pm);
    if (e != hipSuccess) return ORTH_ERR_HIP;
    // [V v_new]^T v_new, then T grows
    ga.X = Operand{h->Q() + (int64_t)k * pl.ldq, pl.ldq};
    pm = h->begin(ORTH_K_LEAF_GRAM2);
    e = launch_gram(s, ga, ORTH_K_LEAF_GRAM2, st);
    h->end(pm);
    if (e != hipSuccess) return ORTH_ERR_HIP;
    pm = h->begin(ORTH_K_LEAF_HH_SMALL);
    e = launch_hh(s, HH_TUPD, ha, st);
    h->end(pm);
    return e == hipSuccess ? ORTH_OK : ORTH_ERR_HIP;
}

// Householder reduction (Sec. 2.2 on the reduction problems of Sec. 4.1):
// at tree level l every node's stacked [P_c; N_c] (its children's segments
// of k_max physical rows, zero past each segment's k+s rows) against the
// node's reflectors V (the level's factor storage), the nodes as the
// leaf-level kernels' leaves: M = V^T Y, Y~ = T^T M, w~ = Y - V Y~, the panel
// in one workgroup per node (pivots: the rows k .. k+s-1 of the node's first
// segment; [P_v; N_v] to the next level's X, the root's to a small scratch
// and then to H and R), [V v]^T v and the growth of each node's T.  Zero
// rows stay zero through every product, so each segment's rows
// k+s .. k+2s-1 are the zero rows the next call's new coordinates take.  The
// leaf instantiations are used: the reflectors have none of the stacked
// factor's zero structure that the reduction kernels skip.
int run_level_hh(orth_ctx *h, int l, int k, double *d_H, int64_t ldh, double *d_R, int64_t ldr) {
    const Plan &pl = h->pl;
    const int32_t s = pl.s, kmax = pl.kmax, ncol = k + s;
    const bool root = l == pl.nlev - 1;
    hipStream_t st = h->stream;
    const int64_t pstride = (int64_t)ncol * s;
    const LevelGeom gg = hh_level_geom(pl, l, pl.cR);
    const int rg = gram_row_groups(ncol);
    if (!pl.hhtree || (int64_t)gg.nchunks() * rg * pstride > pl.slot_cap) return ORTH_ERR_HIP;
    const int64_t ld = pl.ldtl[l];
    hipError_t e;
    HhArgs ha{};
    ha.geom = gg;
    ha.k = k;
    ha.kmax = kmax;
    ha.Q = h->Tl(l);
    ha.ldq = ld;
    ha.T = h->THl(l);
    ha.partials = h->PR();
    ha.part_stride = pstride;
    ha.slots_per_leaf = gg.cpl * rg;
    ha.slots_last = gg.cpl_last * rg;
    ha.small = h->Sl(l);
    ha.small_stride = small_stride(kmax, s);
    if (root) {
        ha.Yout = h->HR();
        ha.ldy = kmax;
        ha.yseg = 0;
    } else {
        ha.Yout = h->Yl(l + 1);
        ha.ldy = pl.ldtl[l + 1];
        ha.yseg = kmax;
    }
    ha.status = h->status();
    ha.X = h->Yl(l);
    ha.ldx = ld;
    GramArgs ga{};
    ga.Q = Operand{h->Tl(l), ld};
    ga.k = k;
    ga.tile_groups = gram_tile_groups(ncol);
    ga.geom = gg;
    ga.partials = h->PR();
    ga.part_stride = pstride;
    ga.status = h->status();
    if (k > 0) {
        ga.X = Operand{h->Yl(l), ld};
        int pm = h->begin(ORTH_K_ROOT_GRAM);
        e = launch_gram(s, ga, ORTH_K_LEAF_GRAM, st);
        h->end(pm);
        if (e != hipSuccess) return ORTH_ERR_HIP;
        pm = h->begin(ORTH_K_ROOT_CHOL);
        e = launch_hh(s, HH_PREP, ha, st);
        h->end(pm);
        if (e != hipSuccess) return ORTH_ERR_HIP;
        FinalizeArgs f{};
        f.Q = Operand{h->Tl(l), ld};
        f.Qnew = OutOperand{h->U1l(l), ld};
        f.U1 = Operand{h->Yl(l), ld};
        f.sweep = 1;
        f.k = k;
        f.geom = hh_level_geom(pl, l, pl.cRR);
        f.small = h->Sl(l);
        f.small_stride = small_stride(kmax, s);
        f.kmax = kmax;
        f.status = h->status();
        pm = h->begin(ORTH_K_ROOT_CORRECT);
        e = launch_finalize(s, f, ORTH_K_LEAF_CORRECT, st);
        h->end(pm);
        if (e != hipSuccess) return ORTH_ERR_HIP;
        ha.X = h->U1l(l);
    }
    int pm = h->begin(ORTH_K_ROOT_CHOL);
    e = launch_hh(s, HH_PANEL, ha, st);
    h->end(pm);
    if (e != hipSuccess) return ORTH_ERR_HIP;
    ga.X = Operand{h->Tl(l) + (int64_t)k * ld, ld};
    pm = h->begin(ORTH_K_ROOT_GRAM2);
    e = launch_gram(s, ga, ORTH_K_LEAF_GRAM2, st);
    h->end(pm);
    if (e != hipSuccess) return ORTH_ERR_HIP;
    pm = h->begin(ORTH_K_ROOT_CHOL);
    e = launch_hh(s, HH_TUPD, ha, st);
    h->end(pm);
    if (e != hipSuccess) return ORTH_ERR_HIP;
    if (root) {
        // [P; N] -> H (k x s) and R (s x s)
        if (k > 0) e = launch_copy_cols(h->HR(), kmax, RowMap{0, 0}, d_H, ldh, k, s, st);
        if (e == hipSuccess) e = launch_copy_cols(h->HR() + k, kmax, RowMap{0, 0}, d_R, ldr, s, s, st);
    }
    return e == hipSuccess ? ORTH_OK : ORTH_ERR_HIP;
}

// Down the tree: every node's new columns U_v = Q_{v,k+s} [C_v; 0] =
// -V (T V[0:k+s]^T C_v) + E C_v over its rows (C_v = [0; I_s] at the root,
// else the node's block from its parent, in the right half of its record),
// then each child segment's k+s rows -> the right half of that child's
// record (the leaves' C_i at level 0)
int finalize_level_hh(orth_ctx *h, int l, int k) {
    const Plan &pl = h->pl;
    const int32_t s = pl.s, kmax = pl.kmax, K = k + s;
    const bool root = l == pl.nlev - 1;
    hipStream_t st = h->stream;
    const int64_t cseg = (int64_t)kmax * 2 * s;
    const int64_t ld = pl.ldtl[l];
    double *rec = root ? h->CR() : h->Cl(l);
    hipError_t e = hipSuccess;
    if (root) {
        // E = [0; I_s] in the right half of the root's record
        e = launch_fill(rec, cseg, 0.0, st);
        for (int32_t j = 0; j < s && e == hipSuccess; ++j)
            e = launch_fill(rec + (int64_t)(k + j) * 2 * s + s + j, 1, 1.0, st);
        if (e != hipSuccess) return ORTH_ERR_HIP;
    }
    HhArgs ha{};
    ha.geom = hh_level_geom(pl, l, pl.cRR);
    ha.k = k;
    ha.kmax = kmax;
    ha.Q = h->Tl(l);
    ha.ldq = ld;
    ha.T = h->THl(l);
    ha.crec = rec;
    ha.cseg = cseg;
    ha.U = h->URl(l);
    ha.ldu = ld;
    ha.status = h->status();
    int pm = h->begin(ORTH_K_ROOT_CHOL);
    e = launch_hh(s, HH_COEF, ha, st);
    h->end(pm);
    if (e != hipSuccess) return ORTH_ERR_HIP;
    FinalizeArgs f{};
    f.Q = Operand{h->Tl(l), ld};
    f.Qnew = OutOperand{h->U1l(l), ld};
    f.U1 = Operand{h->Tl(l) + (int64_t)k * ld, ld};
    f.sweep = 2;
    f.k = k;
    f.geom = ha.geom;
    f.small = h->Sl(l);
    f.small_stride = small_stride(kmax, s);
    f.kmax = kmax;
    f.single_sweep = 1;
    f.Cptr = rec;
    f.cseg = cseg;
    f.Uout = OutOperand{h->URl(l), ld};
    f.status = h->status();
    pm = h->begin(ORTH_K_ROOT_FINALIZE);
    e = launch_finalize(s, f, ORTH_K_LEAF_FINALIZE, st);
    h->end(pm);
    if (e != hipSuccess) return ORTH_ERR_HIP;
    pm = h->begin(ORTH_K_ROOT_CHOL);
    e = launch_hh(s, HH_ADDEC, ha, st);
    h->end(pm);
    if (e != hipSuccess) return ORTH_ERR_HIP;
    pm = h->begin(ORTH_K_ROOT_FINALIZE);
    e = launch_rows_to_records(h->URl(l), ld, pl.nchild[l], kmax, K, s, l == 0 ? h->CL() : h->Cl(l - 1), cseg, st);
    h->end(pm);
    return e == hipSuccess ? ORTH_OK : ORTH_ERR_HIP;
}

// Householder leaves, explicit output: U|_i = Q_{k+s} [C_i; 0] =
// -V (T V[0:k+s]^T C_i) + E C_i
int finalize_leaves_hh(orth_ctx *h, double *d_U, int64_t ldu, int k) {
    const Plan &pl = h->pl;
    const int32_t s = pl.s, kmax = pl.kmax;
    hipStream_t st = h->stream;
    HhArgs ha{};
    ha.geom = leaf_geom(pl, pl.cF);
    ha.k = k;
    ha.kmax = kmax;
    ha.Q = h->Q();
    ha.ldq = pl.ldq;
    ha.T = h->TH();
    ha.crec = h->CL();
    ha.cseg = (int64_t)kmax * 2 * s;
    ha.U = d_U;
    ha.ldu = ldu;
    ha.status = h->status();
    int pm = h->begin(ORTH_K_LEAF_HH_SMALL);
    hipError_t e = launch_hh(s, HH_COEF, ha, st);
    h->end(pm);
    if (e != hipSuccess) return ORTH_ERR_HIP;
    // row update with the reflectors as basis (k + s columns: V, then v_new as
    // the "u1" block copied to the scratch unchanged) and -Z as coefficients
    FinalizeArgs f{};
    f.Q = Operand{h->Q(), pl.ldq};
    f.Qnew = OutOperand{h->U1L(), pl.ldq};
    f.U1 = Operand{h->Q() + (int64_t)k * pl.ldq, pl.ldq};
    f.sweep = 2;
    f.k = k;
    f.geom = leaf_geom(pl, pl.cF);
    f.reg_only = pl.rowreg ? 1 : 0;
    f.small = h->SL();
    f.small_stride = small_stride(kmax, s);
    f.kmax = kmax;
    f.single_sweep = 1;
    f.Cptr = h->CL();
    f.cseg = (int64_t)kmax * 2 * s;
    f.Uout = OutOperand{d_U, ldu};
    f.status = h->status();
    pm = h->begin(ORTH_K_LEAF_FINALIZE);
    e = launch_finalize(s, f, ORTH_K_LEAF_FINALIZE, st);
    h->end(pm);
    if (e != hipSuccess) return ORTH_ERR_HIP;
    pm = h->begin(ORTH_K_LEAF_HH_SMALL);
    e = launch_hh(s, HH_ADDEC, ha, st);
    h->end(pm);
    return e == hipSuccess ? ORTH_OK : ORTH_ERR_HIP;
}

// FlatTSPQR (Sec. 4.2): Q = [Q_1 U] spans the chain
//   Q = [[F_1, 0], [0, I]] [[F_2, 0], [0, I]] ... F_p
// (rows of F_i: block i's rows first, then the k coordinates of the chain
// before it).  Y = Q C right to left: block p's factor times C, its block
// rows to Y and its coordinate rows on as the next factor's C, down to
// block 1.  C: ldc-strided k x m; Y: ldy-strided n x m.
int apply_flat_impl(orth_ctx *h, const double *d_C, int64_t ldc, int32_t m, double *d_Y, int64_t ldy) {
    const FlatPlan &fp = h->fp;
    const int32_t k = h->k;
    hipStream_t st = h->stream;
    double *Z[2] = {h->ws + fp.oZ0, h->ws + fp.oZ1};
    for (int32_t j0 = 0; j0 < m; j0 += kApplyMB) {
        const int32_t mb = (m - j0) < kApplyMB ? (m - j0) : kApplyMB;
        const double *cin = d_C + (int64_t)j0 * ldc;
        int64_t ldin = ldc;
        for (int32_t i = fp.p - 1; i >= 0; --i) {
            const Operand F{h->ws + fp.oF[i], fp.ldf[i]};
            ApplyArgs a{};
            a.k = k;
            a.Cptr = cin;
            a.ldc = ldin;
            a.cseg = 0;
            a.m = mb;
            // block rows -> Y
            a.Q = F;
            a.geom = make_leaf_geom(fp.rows[i], (int32_t)fp.rows[i], 1, kFinalChunk);
            a.Y = OutOperand{d_Y + fp.r0[i] + (int64_t)j0 * ldy, ldy};
            int pm = h->begin(ORTH_K_APPLY);
            hipError_t e = launch_apply(a, st);
            h->end(pm);
            if (e != hipSuccess) return ORTH_ERR_HIP;
            if (i == 0) break;
            // coordinate rows -> the C of block i - 1
            double *out = Z[i & 1];
            a.Q = Operand{F.ptr + fp.rows[i], F.ld};
            a.geom = make_leaf_geom(k, k, 1, kFinalChunk);
            a.Y = OutOperand{out, fp.kmax};
            pm = h->begin(ORTH_K_APPLY);
            e = launch_apply(a, st);
            h->end(pm);
            if (e != hipSuccess) return ORTH_ERR_HIP;
            cin = out;
            ldin = fp.kmax;
        }
    }
    return ORTH_OK;
}

// One FlatTSPQR call: block 1's local problem [F_1 W_1] = [F_1 U_1][[I, P_1],
// [0, N_1]], then block i's on [F_i^ext Y_i], Y_i = [W_i; P_{i-1}; N_{i-1}]
// (the previous block's Cholesky writes [P; N] straight into Y_i's
// coordinate rows), U_i appended to F_i; the last block's P and N are the
// call's H and R.  The explicit U = Q [0; I_s] runs down the chain.
int step_flat(orth_ctx *h, const double *d_W, int64_t ldw, double *d_H, int64_t ldh, double *d_R,
              int64_t ldr, double *d_U, int64_t ldu) {
    const FlatPlan &fp = h->fp;
    const int32_t s = fp.s, k = h->k, kmax = fp.kmax, ncol = k + s;
    if (!d_W || !d_R || !d_U) return ORTH_ERR_ARG;
    if (ldw < fp.n || ldu < fp.n || ldr < s) return ORTH_ERR_ARG;
    if (k > 0 && (!d_H || ldh < k)) return ORTH_ERR_ARG;
    if (k + s > kmax) return ORTH_ERR_CAPACITY;
    const bool two = h->variant == ORTH_PIP_PLUS;
    hipStream_t st = h->stream;
    // W's rows of every block after the first into its staging buffer
    for (int32_t i = 1; i < fp.p; ++i) {
        const hipError_t e = launch_copy_cols(d_W + fp.r0[i], ldw, RowMap{0, 0}, h->ws + fp.oY[i], fp.ldf[i],
                                              fp.rows[i], s, st);
        if (e != hipSuccess) return ORTH_ERR_HIP;
    }
    for (int32_t i = 0; i < fp.p; ++i) {
        const bool last = i == fp.p - 1;
        const int64_t rows = i == 0 ? fp.rows[0] : fp.rows[i] + ncol;
        double *F = h->ws + fp.oF[i];
        LevelRun L{};
        L.Q = Operand{F, fp.ldf[i]};
        L.X = i == 0 ? Operand{d_W + fp.r0[0], ldw} : Operand{h->ws + fp.oY[i], fp.ldf[i]};
        L.U1 = OutOperand{h->ws + fp.oU1, fp.ldmax};
        L.geom = make_leaf_geom(rows, (int32_t)rows, 1, kLeafChunk);
        L.rgeom = make_leaf_geom(rows, (int32_t)rows, 1, kFinalChunk);
        L.part = h->ws + fp.oP;
        L.part2 = h->ws + fp.oP2;
        L.part_cap = fp.slot_cap;
        L.part2_cap = fp.red_cap;
        L.small = h->ws + fp.oS;
        L.level = 0;
        if (last) {
            L.H = k > 0 ? d_H : nullptr;
            L.ldh = ldh;
            L.R = d_R;
            L.ldr = ldr;
        } else {
            L.Yout = h->ws + fp.oY[i + 1] + fp.rows[i + 1];
            L.ldy = fp.ldf[i + 1];
            L.yseg = 0;
        }
        if (int rc = run_level(h, L, k, two)) return rc;
        // U_i -> the factor's columns k .. k+s-1 (rows [0, rows))
        FinalizeArgs f{};
        f.Q = L.Q;
        f.Qnew = OutOperand{F + (int64_t)k * fp.ldf[i], fp.ldf[i]};
        f.U1 = Operand{L.U1.ptr, L.U1.ld};
        f.sweep = 2;
        f.k = k;
        f.geom = L.rgeom;
        f.small = L.small;
        f.small_stride = small_stride(kmax, s);
        f.kmax = kmax;
        f.single_sweep = two ? 0 : 1;
        f.Cptr = nullptr;
        f.status = h->status();
        const int pm = h->begin(ORTH_K_LEAF_FINALIZE);
        const hipError_t e = launch_finalize(s, f, ORTH_K_LEAF_CORRECT, st);
        h->end(pm);
        if (e != hipSuccess) return ORTH_ERR_HIP;
    }
    h->k = k + s;
    // U = Q [0; I_s]: the identity block sits below k_max zero rows
    const double *E = h->ws + fp.oE + (kmax - k);
    if (int rc = apply_flat_impl(h, E, (int64_t)kmax + s, s, d_U, ldu)) return rc;
    return ORTH_OK;
}

}  // namespace

extern "C" {

int orth_step(orth_t *h, const double *d_W, int64_t ldw, double *d_H, int64_t ldh, double *d_R,
              int64_t ldr, double *d_U, int64_t ldu) {
    if (!h) return ORTH_ERR_ARG;
    if (h->poisoned) return ORTH_ERR_POISONED;
    if (h->flat) {
        const int rc = step_flat(h, d_W, ldw, d_H, ldh, d_R, ldr, d_U, ldu);
        if (rc) (void)hipGetLastError();
        return rc;
    }
    const Plan &pl = h->pl;
    const int32_t s = pl.s, k = h->k, kmax = pl.kmax;
    if (!d_W || !d_R || !d_U) return ORTH_ERR_ARG;
    if (ldw < pl.n || ldu < pl.n || ldr < s) return ORTH_ERR_ARG;
    if (k > 0 && (!d_H || ldh < k)) return ORTH_ERR_ARG;
    if (k + s > kmax) return ORTH_ERR_CAPACITY;
    const bool two = h->variant == ORTH_PIP_PLUS;          // leaves
    const bool two_red = h->variant_red == ORTH_PIP_PLUS;  // reduction
    hipStream_t st = h->stream;
    const int ncol = k + s;
    int rc;

    // ---- leaves: local PQR [Q_i W_i] = [Q_i U_i][[I, P_i], [0, N_i]]
    if (pl.precision == ORTH_FP64_HOUSEHOLDER) {
        if ((rc = run_leaves_hh(h, d_W, ldw, k))) goto fail;
    } else {
        LevelRun L{};
        L.Q = h->Qop();
        L.X = Operand{d_W, ldw};
        L.U1 = OutOperand{h->U1L(), pl.ldq};
        L.geom = leaf_geom(pl, pl.cL);
        L.rgeom = leaf_geom(pl, pl.cF);
        L.Qhi = h->Qhi();
        L.pc = h->CL();
        L.part = h->PL();
        L.part2 = h->PR2();          // pre-sums when a single leaf holds many slots
        L.part_cap = pl.slot_cap;
        L.part2_cap = pl.red_cap;
        L.small = h->SL();
        L.level = 0;
        L.Yout = h->Y();
        L.ldy = pl.ldt;
        L.yseg = kmax;
        if ((rc = run_level(h, L, k, two))) goto fail;
    }
    // ---- reduction: PQR on the stacked [[T_c, P_c], [0, N_c]] of each node's
    // children (segments of k+s rows), level by level up to the root
    for (int l = 0; l < pl.nlev; ++l) {
        const bool root = l == pl.nlev - 1;
        if (h->hh_red()) {                       // Householder reduction
            if ((rc = run_level_hh(h, l, k, k > 0 ? d_H : nullptr, ldh, d_R, ldr))) goto fail;
            continue;
        }
        LevelRun L{};
        L.Q = Operand{h->Tl(l), pl.ldtl[l]};
        L.X = Operand{h->Yl(l), pl.ldtl[l]};
        L.U1 = OutOperand{h->U1l(l), pl.ldtl[l]};
        L.geom = tree_geom(pl, l, ncol, pl.cR);
        L.rgeom = tree_geom(pl, l, ncol, pl.cRR);
        L.part = h->PR();
        L.part2 = h->PR2();
        L.part_cap = pl.slot_cap;
        L.part2_cap = pl.red_cap;
        L.small = h->Sl(l);
        L.level = l + 1;
        L.pc = root ? nullptr : h->Cl(l);
        if (root) {
            L.H = k > 0 ? d_H : nullptr;
            L.ldh = ldh;
            L.R = d_R;
            L.ldr = ldr;
        } else {
            L.Yout = h->Yl(l + 1);
            L.ldy = pl.ldtl[l + 1];
            L.yseg = kmax;
        }
        DeflArgs dargs{h->defl_delta * h->defl_delta, h->DF()};
        L.defl = h->defl_delta > 0.0 ? &dargs : nullptr;
        if ((rc = run_level(h, L, k, two_red))) goto fail;
    }
    // ---- down the tree: every level's new columns [P~_c; N~_c] -> its
    // factor's columns k..k+s-1; the root's are its children's coefficient
    // blocks C_c, a lower node v forms its children's C_c = [S_v,c Y~_v,c] C_v
    // (Sec. 4.1, assembly of U), down to the leaves' records
    for (int l = pl.nlev - 1; l >= 0; --l) {
        const bool root = l == pl.nlev - 1;
        if (h->hh_red()) {
            if ((rc = finalize_level_hh(h, l, k))) goto fail;
            continue;
        }
        double *below = l == 0 ? h->CL() : h->Cl(l - 1);
        FinalizeArgs f{};
        f.Q = Operand{h->Tl(l), pl.ldtl[l]};
        f.Qnew = OutOperand{h->Tl(l) + (int64_t)k * pl.ldtl[l], pl.ldtl[l]};
        f.U1 = Operand{h->U1l(l), pl.ldtl[l]};
        f.sweep = 2;
        f.k = k;
        f.geom = tree_geom(pl, l, ncol, pl.cRR);
        f.small = h->Sl(l);
        f.small_stride = small_stride(kmax, s);
        f.kmax = kmax;
        f.single_sweep = two_red ? 0 : 1;
        f.status = h->status();
        if (root) {
            f.Cptr = nullptr;
            f.Crow = below;
            f.crow_seg = (int64_t)kmax * 2 * s;
        } else {
            f.Cptr = h->Cl(l);
            f.cseg = (int64_t)kmax * 2 * s;
            f.Cout = below;
            f.cout_seg = (int64_t)kmax * 2 * s;
        }
        const int pm = h->begin(ORTH_K_ROOT_FINALIZE);
        const hipError_t e = launch_finalize(s, f, ORTH_K_ROOT_FINALIZE, st);
        h->end(pm);
        if (e != hipSuccess) { rc = ORTH_ERR_HIP; goto fail; }
    }
    // ---- leaves: U_i appended to Q_i, explicit U|_i = [Q_i U_i] [P~_i; N~_i]
    if (pl.precision == ORTH_FP64_HOUSEHOLDER) {
        if ((rc = finalize_leaves_hh(h, d_U, ldu, k))) goto fail;
    } else {
        FinalizeArgs f{};
        f.Q = h->Qop();
        f.Qnew = h->Qout(k);
        f.Qnew_hi = h->Qhi_at(k);
        f.U1 = Operand{h->U1L(), pl.ldq};
        f.sweep = 2;
        f.k = k;
        f.geom = leaf_geom(pl, pl.cF);
        f.reg_only = pl.rowreg ? 1 : 0;
        f.small = h->SL();
        f.small_stride = small_stride(kmax, s);
        f.kmax = kmax;
        f.single_sweep = two ? 0 : 1;
        f.Cptr = h->CL();
        f.cseg = (int64_t)kmax * 2 * s;
        f.Uout = OutOperand{d_U, ldu};
        f.status = h->status();
        const int pm = h->begin(ORTH_K_LEAF_FINALIZE);
        const hipError_t e = launch_finalize(s, f, ORTH_K_LEAF_FINALIZE, st);
        h->end(pm);
        if (e != hipSuccess) { rc = ORTH_ERR_HIP; goto fail; }
    }
    h->k = k + s;
    return ORTH_OK;
fail:
    (void)hipGetLastError();
    return rc;
}

}  // extern "C"

namespace {

// Y = Q C in column blocks of at most mb_max columns.  ca (and, with
// Householder leaves, ca2) hold the per-leaf coefficient blocks of one column
// block: ldt x mb_max doubles each.  prof: bracket the launches with the
// handle's profiler events.
int apply_q_impl(orth_ctx *h, const double *d_C, int64_t ldc, int32_t m, double *d_Y, int64_t ldy,
                 double *ca, double *ca2, double *ca3, int32_t mb_max, bool prof) {
    const Plan &pl = h->pl;
    const int32_t k = h->k;
    const bool hh = pl.precision == ORTH_FP64_HOUSEHOLDER;
    hipStream_t st = h->stream;
    auto begin = [&](int cls) { return prof ? h->begin(cls) : -1; };
    auto end = [&](int idx) { if (prof) h->end(idx); };
    // host check: the tree's down-sweep and the Householder products need
    // the second scratch region
    if (!ca || ((hh || pl.nlev > 1) && !ca2) || ((h->hh_red() || (hh && pl.nlev > 1)) && !ca3) || mb_max < 1)
        return ORTH_ERR_HIP;
    for (int32_t j0 = 0; j0 < m; j0 += mb_max) {
        const int32_t mb = (m - j0) < mb_max ? (m - j0) : mb_max;
        // down the reduction tree: a node's children get C_c = S_v,c C_v
        // (rows: the level's child segments of k rows); the root's C is the
        // caller's, every lower level's the level above's output, the two
        // scratch regions in turn, so level 0 leaves C_i in `cur`
        hipError_t e = hipSuccess;
        double *cur = nullptr;
        double *zleaf = ca2;                     // Householder leaves' -Z_i scratch
        if (h->hh_red()) {
            // Householder reduction, level by level from the root: a node's
            // children get [C_c] = Q_{v,k} [C_v; 0] = -V Z + E C_v over its
            // rows (Z = T V[0:k]^T C_v); three regions in turn hold C, -Z and
            // the children's blocks
            double *buf[3] = {ca, ca2, ca3};
            int ci = 0;
            e = launch_copy_cols(d_C + (int64_t)j0 * ldc, ldc, RowMap{0, 0}, buf[0], pl.ldt, k, mb, st);
            for (int l = pl.nlev - 1; l >= 0 && e == hipSuccess; --l) {
                const int zi = (ci + 1) % 3, yi = (ci + 2) % 3;
                HhArgs hr{};
                hr.geom = hh_level_geom(pl, l, pl.cRR);
                hr.k = k;
                hr.kmax = pl.kmax;
                hr.T = h->THl(l);
                hr.ca = buf[ci];
                hr.ca_out = buf[zi];
                hr.ldca = pl.ldt;
                hr.m = mb;
                hr.U = buf[yi];
                hr.ldu = pl.ldt;
                const int pm = begin(ORTH_K_APPLY);
                e = launch_hh_apply(HH_APPLY_COEF, hr, st);
                if (e == hipSuccess) {
                    ApplyArgs r{};
                    r.Q = Operand{h->Tl(l), pl.ldtl[l]};
                    r.k = k;
                    r.geom = hr.geom;
                    r.Cptr = buf[zi];
                    r.ldc = pl.ldt;
                    r.cseg = pl.kmax;
                    r.m = mb;
                    r.Y = OutOperand{buf[yi], pl.ldt};
                    e = launch_apply(r, st);
                }
                if (e == hipSuccess) e = launch_hh_apply(HH_APPLY_ADD, hr, st);
                end(pm);
                ci = yi;
            }
            if (e != hipSuccess) { (void)hipGetLastError(); return ORTH_ERR_HIP; }
            cur = buf[ci];
            zleaf = buf[(ci + 1) % 3];            // free now
        }
        for (int l = h->hh_red() ? -1 : pl.nlev - 1; l >= 0; --l) {
            double *out = (cur == ca) ? ca2 : ca;
            ApplyArgs r{};
            r.Q = Operand{h->Tl(l), pl.ldtl[l]};
            r.k = k;
            r.geom = tree_geom(pl, l, k, pl.cRR);
            if (l == pl.nlev - 1) {
                r.Cptr = d_C + (int64_t)j0 * ldc;
                r.ldc = ldc;
                r.cseg = 0;
            } else {
                r.Cptr = cur;
                r.ldc = pl.ldt;
                r.cseg = pl.kmax;
            }
            r.m = mb;
            r.Y = OutOperand{out, pl.ldt};
            const int pm0 = begin(ORTH_K_APPLY);
            e = launch_apply(r, st);
            end(pm0);
            if (e != hipSuccess) { (void)hipGetLastError(); return ORTH_ERR_HIP; }
            cur = out;
        }
        // under a tree the down-sweep may end in ca2: the leaves' -Z_i then
        // goes to the third region
        if (hh && !h->hh_red() && cur == ca2) zleaf = ca3;
        // leaves: Y_i = Q_i C_i; with Householder leaves Y_i = -V Z_i + E C_i,
        // Z_i = T (V[0:k]^T C_i)
        HhArgs ha{};
        if (hh) {
            ha.geom = leaf_geom(pl, pl.cF);
            ha.k = k;
            ha.kmax = pl.kmax;
            ha.T = h->TH();
            ha.ca = cur;            // (one level: cur == ca)
            ha.ca_out = zleaf;
            ha.ldca = pl.ldt;
            ha.m = mb;
            ha.U = d_Y + (int64_t)j0 * ldy;
            ha.ldu = ldy;
            const int pm = begin(ORTH_K_APPLY);
            e = launch_hh_apply(HH_APPLY_COEF, ha, st);
            end(pm);
            if (e != hipSuccess) { (void)hipGetLastError(); return ORTH_ERR_HIP; }
        }
        ApplyArgs a{};
        a.Q = h->Qop();
        a.k = k;
        a.geom = leaf_geom(pl, pl.cF);
        a.Cptr = hh ? zleaf : cur;
        a.ldc = pl.ldt;
        a.cseg = pl.kmax;
        a.m = mb;
        a.Y = OutOperand{d_Y + (int64_t)j0 * ldy, ldy};
        { const int pm = begin(ORTH_K_APPLY); e = launch_apply(a, st); end(pm); }
        if (e != hipSuccess) { (void)hipGetLastError(); return ORTH_ERR_HIP; }
        if (hh) {
            const int pm = begin(ORTH_K_APPLY);
            e = launch_hh_apply(HH_APPLY_ADD, ha, st);
            end(pm);
            if (e != hipSuccess) { (void)hipGetLastError(); return ORTH_ERR_HIP; }
        }
    }
    return ORTH_OK;
}

}  // namespace

extern "C" {

int orth_apply_Q(orth_t *h, const double *d_C, int64_t ldc, int32_t m, double *d_Y, int64_t ldy) {
    if (!h) return ORTH_ERR_ARG;
    if (h->poisoned) return ORTH_ERR_POISONED;
    if (h->flat) {
        if (h->k < 1 || m < 1 || !d_C || !d_Y || ldc < h->k || ldy < h->fp.n) return ORTH_ERR_ARG;
        const int rc = apply_flat_impl(h, d_C, ldc, m, d_Y, ldy);
        if (rc) (void)hipGetLastError();
        return rc;
    }
    if (h->k < 1 || m < 1 || !d_C || !d_Y || ldc < h->k || ldy < h->pl.n) return ORTH_ERR_ARG;
    return apply_q_impl(h, d_C, ldc, m, d_Y, ldy, h->CA(), h->CA2(), h->CA3(), kApplyMB, true);
}

int orth_apply_Q_noalloc(orth_t *h, const double *d_C, int64_t ldc, int32_t m, double *d_Y, int64_t ldy) {
    if (!h) return ORTH_ERR_ARG;
    if (h->poisoned) return ORTH_ERR_POISONED;
    if (h->flat) return ORTH_ERR_UNSUPPORTED;
    // one column of coefficient blocks per region (two regions with
    // Householder leaves or a reduction tree, three with the Householder
    // reduction) must fit the static scratch
    const bool hh_leaves = h->pl.precision == ORTH_FP64_HOUSEHOLDER;
    const int64_t regions =
        (h->hh_red() || (hh_leaves && h->pl.nlev > 1)) ? 3 : ((hh_leaves || h->pl.nlev > 1) ? 2 : 1);
    const int64_t cols = kStaticScratchDoubles / (regions * h->pl.ldt);
    if (cols < 1) return ORTH_ERR_SCRATCH;
    if (h->k < 1 || m < 1 || !d_C || !d_Y || ldc < h->k || ldy < h->pl.n) return ORTH_ERR_ARG;
    double *base = nullptr;
    if (static_scratch(h->device, &base) != hipSuccess) {
        (void)hipGetLastError();
        return ORTH_ERR_HIP;
    }
    const int32_t mb_max = (int32_t)std::min<int64_t>(kApplyMB, cols);
    double *ca2 = regions >= 2 ? base + h->pl.ldt * mb_max : nullptr;
    double *ca3 = regions == 3 ? base + 2 * h->pl.ldt * mb_max : nullptr;
    return apply_q_impl(h, d_C, ldc, m, d_Y, ldy, base, ca2, ca3, mb_max, false);
}

int orth_status(orth_t *h, int32_t *status, int32_t *info) {
    if (!h || !status) return ORTH_ERR_ARG;
    DevStatus ds{};
    if (hipStreamSynchronize(h->stream) != hipSuccess ||
        hipMemcpy(&ds, h->status(), sizeof(ds), hipMemcpyDeviceToHost) != hipSuccess) {
        (void)hipGetLastError();
        return ORTH_ERR_HIP;
    }
    *status = ds.code == 0 ? ORTH_OK : ORTH_ERR_BREAKDOWN;
    if (ds.code != 0) h->poisoned = true;
    if (info) {
        info[0] = ds.level;
        info[1] = ds.leaf;
        info[2] = ds.sweep;
        info[3] = ds.column;
    }
    return ORTH_OK;
}

int orth_set_deflation(orth_t *h, double delta) {
    if (!h) return ORTH_ERR_ARG;
    if (h->poisoned) return ORTH_ERR_POISONED;
    if (!(delta >= 0.0 && delta < 1.0)) return ORTH_ERR_ARG;      // NaN fails too
    // deflation is defined for the single reduction level
    // (the eigen solver of the reduction-level factorisation stops at s = 16)
    if (delta > 0.0 && (!h->DF() || h->hh_red() || h->pl.nlev > 1 || h->pl.s > 16)) return ORTH_ERR_UNSUPPORTED;
    h->defl_delta = delta;
    return ORTH_OK;
}

int orth_deflation_info(orth_t *h, int32_t *rank, int64_t *steps, int64_t *dropped) {
    if (!h) return ORTH_ERR_ARG;
    DeflState d{};
    if (h->DF()) {
        if (hipStreamSynchronize(h->stream) != hipSuccess ||
            hipMemcpy(&d, h->DF(), sizeof(d), hipMemcpyDeviceToHost) != hipSuccess) {
            (void)hipGetLastError();
            return ORTH_ERR_HIP;
        }
    }
    if (rank) *rank = h->pl.s - d.dropped;
    if (steps) *steps = d.steps;
    if (dropped) *dropped = d.total;
    return ORTH_OK;
}

int orth_mixed_fallbacks(orth_t *h, int64_t *count) {
    if (!h || !count) return ORTH_ERR_ARG;
    DevStatus ds{};
    if (hipStreamSynchronize(h->stream) != hipSuccess ||
        hipMemcpy(&ds, h->status(), sizeof(ds), hipMemcpyDeviceToHost) != hipSuccess) {
        (void)hipGetLastError();
        return ORTH_ERR_HIP;
    }
    *count = ds.fallbacks;
    return ORTH_OK;
}

int orth_basis_width(const orth_t *h, int32_t *k) {
    if (!h || !k) return ORTH_ERR_ARG;
    *k = h->k;
    return ORTH_OK;
}

int orth_leaf_count(const orth_t *h, int32_t *p, int32_t *leaf_rows) {
    if (!h) return ORTH_ERR_ARG;
    if (h->flat) {
        if (p) *p = h->fp.p;
        if (leaf_rows) *leaf_rows = h->fp.block_rows;
        return ORTH_OK;
    }
    if (p) *p = h->pl.p;
    if (leaf_rows) *leaf_rows = h->pl.leaf_rows;
    return ORTH_OK;
}

int orth_tree_levels(const orth_t *h, int32_t *levels, int32_t *fan_in) {
    if (!h) return ORTH_ERR_ARG;
    if (levels) *levels = h->pl.nlev;
    if (fan_in) *fan_in = h->pl.fan_in;
    return ORTH_OK;
}

int orth_export_tree_level(orth_t *h, int32_t level, double *d_T, int64_t ldt) {
    if (!h) return ORTH_ERR_ARG;
    if (h->flat || h->hh_red()) return ORTH_ERR_UNSUPPORTED;
    if (h->poisoned) return ORTH_ERR_POISONED;
    const Plan &pl = h->pl;
    const int32_t k = h->k;
    if (k < 1 || level < 0 || level >= pl.nlev || !d_T || ldt < (int64_t)pl.nchild[level] * k)
        return ORTH_ERR_ARG;
    const hipError_t e = launch_copy_cols(h->Tl(level), pl.ldtl[level], RowMap{k, pl.kmax}, d_T, ldt,
                                          (int64_t)pl.nchild[level] * k, k, h->stream);
    if (e != hipSuccess) { (void)hipGetLastError(); return ORTH_ERR_HIP; }
    return ORTH_OK;
}

int orth_export_local(orth_t *h, double *d_Qloc, int64_t ldq, double *d_T, int64_t ldt) {
    if (!h) return ORTH_ERR_ARG;
    if (h->flat || (d_T && h->hh_red())) return ORTH_ERR_UNSUPPORTED;
    if (h->poisoned) return ORTH_ERR_POISONED;
    const Plan &pl = h->pl;
    const int32_t k = h->k;
    if (k < 1) return ORTH_ERR_ARG;
    if (d_Qloc && ldq < pl.n) return ORTH_ERR_ARG;
    if (d_T && ldt < (int64_t)pl.p * k) return ORTH_ERR_ARG;
    hipError_t e = hipSuccess;
    if (d_Qloc)
        e = pl.qblk ? launch_copy_leafblk(h->Qop(), leaf_geom(pl, pl.cL), d_Qloc, ldq, k, h->stream)
                    : launch_copy_cols(h->Q(), pl.ldq, RowMap{0, 0}, d_Qloc, ldq, pl.n, k, h->stream);
    if (e == hipSuccess && d_T)
        e = launch_copy_cols(h->T(), pl.ldt, RowMap{k, pl.kmax}, d_T, ldt, (int64_t)pl.p * k, k,
                             h->stream);
    if (e != hipSuccess) { (void)hipGetLastError(); return ORTH_ERR_HIP; }
    return ORTH_OK;
}

int orth_profile_enable(orth_t *h, int32_t on) {
    if (!h) return ORTH_ERR_ARG;
    h->prof_on = on != 0;
    return ORTH_OK;
}

int orth_profile_select(orth_t *h, uint32_t class_mask) {
    if (!h) return ORTH_ERR_ARG;
    h->prof_mask = class_mask;
    return ORTH_OK;
}

int orth_profile_read(orth_t *h, double *total_ms, int64_t *launches) {
    if (!h || !total_ms || !launches) return ORTH_ERR_ARG;
    if (hipStreamSynchronize(h->stream) != hipSuccess) {
        (void)hipGetLastError();
        return ORTH_ERR_HIP;
    }
    for (auto &m : h->marks) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, m.a, m.b) == hipSuccess) {
            h->prof_ms[m.cls] += ms;
            h->prof_n[m.cls] += 1;
        } else {
            (void)hipGetLastError();
        }
        h->spare.push_back(m.a);
        h->spare.push_back(m.b);
    }
    h->marks.clear();
    for (int c = 0; c < ORTH_K_COUNT; ++c) {
        total_ms[c] = h->prof_ms[c];
        launches[c] = h->prof_n[c];
    }
    return ORTH_OK;
}

int orth_profile_reset(orth_t *h) {
    if (!h) return ORTH_ERR_ARG;
    if (hipStreamSynchronize(h->stream) != hipSuccess) {
        (void)hipGetLastError();
        return ORTH_ERR_HIP;
    }
    for (auto &m : h->marks) {
        h->spare.push_back(m.a);
        h->spare.push_back(m.b);
    }
    h->marks.clear();
    for (int c = 0; c < ORTH_K_COUNT; ++c) {
        h->prof_ms[c] = 0.0;
        h->prof_n[c] = 0;
    }
    return ORTH_OK;
}

int orth_destroy(orth_t *h) {
    delete h;
    return ORTH_OK;
}

int orth_laplacian_apply(const double *d_X, int64_t ldx, double *d_Y, int64_t ldy, int32_t s,
                         int32_t nx, int32_t ny, int32_t nz, double shift, void *stream) {
    if (!d_X || !d_Y || s < 1 || nx < 1 || ny < 1 || nz < 1) return ORTH_ERR_ARG;
    const int64_t n = (int64_t)nx * ny * nz;
    if (ldx < n || ldy < n) return ORTH_ERR_ARG;
    if (launch_laplacian(d_X, ldx, d_Y, ldy, s, nx, ny, nz, shift,
                         static_cast<hipStream_t>(stream)) != hipSuccess) {
        (void)hipGetLastError();
        return ORTH_ERR_HIP;
    }
    return ORTH_OK;
}

int orth_probe_copy(const double *d_src, double *d_dst, int64_t count, void *stream) {
    if (!d_src || !d_dst || count < 0 || ((uintptr_t)d_src % 16) || ((uintptr_t)d_dst % 16))
        return ORTH_ERR_ARG;
    if (launch_copy(d_src, d_dst, count, static_cast<hipStream_t>(stream)) != hipSuccess) {
        (void)hipGetLastError();
        return ORTH_ERR_HIP;
    }
    return ORTH_OK;
}

}  // extern "C"

// ============================================================ batched form
// Many independent instances (uneven n and s) advance one orth_step together:
// every phase is one grouped launch per block width present (BatchPhase
// order), so a batch step is a fixed sequence of at most BP_COUNT x widths
// launches, with no host synchronisation or allocation: a caller can capture
// whole runs in a graph.
//
// Workspace: [descriptors][block prefix tables][status][instance regions...],
// each instance region carved exactly like a single handle's workspace.  The
// prefix table of (step, phase, width) gives instances of other widths no
// blocks.

namespace {

struct BatchLayout {
    int32_t count = 0, steps_max = 0;
    std::vector<int32_t> widths;        // distinct block widths, ascending
    std::vector<Plan> plans;
    std::vector<int64_t> inst_off;      // doubles, per instance region
    int32_t precision = ORTH_FP64;
    int64_t o_desc = 0, o_prefix = 0, o_status = 0, o_retry = 0, total = 0;   // doubles
};

bool make_batch_layout(int32_t count, const int64_t *n, const int32_t *s, const int32_t *k_max,
                       const int32_t *leaf_rows, int32_t precision, BatchLayout &L, int *why) {
    *why = ORTH_ERR_ARG;
    if (count < 1 || count > (1 << 20) || !n || !s || !k_max) return false;
    if (precision != ORTH_FP64 && precision != ORTH_MIXED_SPLIT32 && precision != ORTH_FP64_HOUSEHOLDER)
        return false;
    L.precision = precision;
    L.count = count;
    L.plans.resize(count);
    L.inst_off.resize(count);
    L.steps_max = 1 << 30;
    for (int32_t i = 0; i < count; ++i) {
        if (!make_plan(n[i], s[i], k_max[i], leaf_rows ? leaf_rows[i] : 0, precision, L.plans[i], why))
            return false;
        L.steps_max = std::min(L.steps_max, k_max[i] / s[i]);
        if (std::find(L.widths.begin(), L.widths.end(), s[i]) == L.widths.end()) L.widths.push_back(s[i]);
    }
    std::sort(L.widths.begin(), L.widths.end());
    int64_t off = 0;
    auto take = [&](int64_t doubles) {
        const int64_t o = off;
        off = round_up(off + doubles, kAlign);
        return o;
    };
    L.o_desc = take(ceil_div((int64_t)count * sizeof(BatchInst), 8));
    L.o_prefix = take(ceil_div((int64_t)L.steps_max * BP_COUNT * (int64_t)L.widths.size() * (count + 1) * 4, 8));
    L.o_status = take(ceil_div(sizeof(DevStatus), 8));
    L.o_retry = take(ceil_div((int64_t)count * 4, 8));      // per-instance retry flags (mixed form)
    for (int32_t i = 0; i < count; ++i) L.inst_off[i] = take(L.plans[i].total);
    L.total = off;
    return true;
}

}  // namespace

struct orth_batch_ctx {
    BatchLayout L;
    int32_t step = 0;
    int32_t variant = ORTH_PIP_PLUS;
    bool poisoned = false;
    hipStream_t stream = nullptr;
    double *ws = nullptr;
    std::vector<BatchInst> desc;
    std::vector<int32_t> prefix;          // steps_max x BP_COUNT x widths x (count + 1)
    std::vector<size_t> lds;              // BP_COUNT x widths
    size_t row(int32_t step, int ph, size_t w) const {
        return (((size_t)step * BP_COUNT + ph) * L.widths.size() + w) * (L.count + 1);
    }
    DevStatus *status() const { return reinterpret_cast<DevStatus *>(ws + L.o_status); }
};

extern "C" {

size_t orth_batch_workspace_bytes(int32_t count, const int64_t *n, const int32_t *s, const int32_t *k_max,
                                  const int32_t *leaf_rows, int32_t precision) {
    BatchLayout L;
    int why;
    if (!make_batch_layout(count, n, s, k_max, leaf_rows, precision, L, &why)) return 0;
    return (size_t)L.total * sizeof(double);
}

int orth_batch_create(int32_t count, const int64_t *n, const int32_t *s, const int32_t *k_max,
                      const int32_t *leaf_rows, int32_t precision, void *d_workspace,
                      size_t workspace_bytes, void *stream, orth_batch_t **out) {
    if (!out) return ORTH_ERR_ARG;
    *out = nullptr;
    BatchLayout L;
    int why;
    if (!make_batch_layout(count, n, s, k_max, leaf_rows, precision, L, &why)) return why;
    if (!d_workspace || ((uintptr_t)d_workspace % 256) != 0 ||
        workspace_bytes < (size_t)L.total * sizeof(double))
        return ORTH_ERR_WORKSPACE;
    orth_batch_ctx *b = new (std::nothrow) orth_batch_ctx();
    if (!b) return ORTH_ERR_HIP;
    b->L = L;
    b->stream = static_cast<hipStream_t>(stream);
    b->ws = static_cast<double *>(d_workspace);
    for (int32_t w : L.widths) {
        if (prepare_kernels(w) != hipSuccess ||
            (precision == ORTH_FP64_HOUSEHOLDER && prepare_hh_kernels(w) != hipSuccess)) {
            (void)hipGetLastError();
            delete b;
            return ORTH_ERR_HIP;
        }
    }
    b->desc.resize(count);
    for (int32_t i = 0; i < count; ++i) {
        const Plan &pl = L.plans[i];
        double *base = b->ws + L.inst_off[i];
        BatchInst &d = b->desc[i];
        d.n = pl.n;
        d.ldq = pl.ldq;
        d.ldt = pl.ldt;
        d.s = pl.s;
        d.kmax = pl.kmax;
        d.leaf_rows = pl.leaf_rows;
        d.p = pl.p;
        d.cL = pl.cL;
        d.cR = pl.cR;
        d.Q = base + pl.oQ;
        d.T = base + pl.oT;
        d.Y = base + pl.oY;
        d.U1L = base + pl.oU1L;
        d.U1R = base + pl.oU1R;
        d.PL = base + pl.oPL;
        d.PR = base + pl.oPR;
        d.PR2 = base + pl.oPR2;
        d.SL = base + pl.oSL;
        d.SR = base + pl.oSR;
        d.CL = base + pl.oCL;
        d.Qhi = pl.precision == ORTH_MIXED_SPLIT32 ? reinterpret_cast<float *>(base + pl.oQH) : nullptr;
        d.retry = reinterpret_cast<int32_t *>(b->ws + L.o_retry) + i;
        d.TH = pl.precision == ORTH_FP64_HOUSEHOLDER ? base + pl.oTH : nullptr;
    }
    // block prefix tables of every (step, phase, width)
    const size_t nw = L.widths.size();
    b->prefix.assign(b->row(L.steps_max, 0, 0), 0);
    for (int32_t st = 0; st < L.steps_max; ++st)
        for (int ph = 0; ph < BP_COUNT; ++ph)
            for (size_t w = 0; w < nw; ++w) {
                int32_t *row = &b->prefix[b->row(st, ph, w)];
                for (int32_t i = 0; i < count; ++i)
                    row[i + 1] = row[i] + (b->desc[i].s == L.widths[w] ? batch_phase_blocks(b->desc[i], ph, st, 1) : 0);
            }
    // the LDS-staged leaf row updates for widths >= 16 whose instances all
    // start their chunks on even rows (even leaf heights, or one leaf; the
    // rest holds by construction)
    std::vector<bool> rowlds(nw, true);
    for (size_t w = 0; w < nw; ++w)
        for (int32_t i = 0; i < count; ++i)
            if (b->desc[i].s == L.widths[w] && (b->desc[i].leaf_rows & 1) && b->desc[i].p > 1) rowlds[w] = false;
    b->lds.assign((size_t)BP_COUNT * nw, 0);
    for (int ph = 0; ph < BP_COUNT; ++ph)
        for (size_t w = 0; w < nw; ++w) b->lds[ph * nw + w] = batch_phase_lds(ph, L.widths[w], rowlds[w]);
    hipError_t e = hipMemcpyAsync(b->ws + L.o_desc, b->desc.data(), count * sizeof(BatchInst),
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + L.o_prefix, b->prefix.data(), b->prefix.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, b->stream);
    for (int32_t i = 0; i < count && e == hipSuccess; ++i) {
        const Plan &pl = L.plans[i];
        e = launch_fill(b->desc[i].T, pl.ldt * (int64_t)pl.kmax, 0.0, b->stream);
        if (e == hipSuccess) e = launch_fill(b->desc[i].Y, pl.ldt * (int64_t)pl.s, 0.0, b->stream);
        // Householder leaves: the compact-WY factors grow into zeros below their diagonal
        if (e == hipSuccess && b->desc[i].TH)
            e = launch_fill(b->desc[i].TH, (int64_t)3 * pl.p * pl.kmax * pl.kmax, 0.0, b->stream);
    }
    if (e == hipSuccess)
        e = launch_fill_i32(reinterpret_cast<int32_t *>(b->status()),
                            (int64_t)(sizeof(DevStatus) / sizeof(int32_t)), 0, b->stream);
    if (e == hipSuccess) e = launch_fill_i32(reinterpret_cast<int32_t *>(b->ws + L.o_retry), count, 0, b->stream);
    // the host copies above read b->desc / b->prefix; finish before returning
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete b;
        return ORTH_ERR_HIP;
    }
    *out = b;
    return ORTH_OK;
}

int orth_batch_set_variant(orth_batch_t *b, int32_t variant) {
    if (!b || (variant != ORTH_PIP_PLUS && variant != ORTH_PIP)) return ORTH_ERR_ARG;
    if (b->poisoned) return ORTH_ERR_POISONED;
    // (the variant names both levels; Householder leaves take no CholeskyQR variant)
    if (b->L.precision == ORTH_FP64_HOUSEHOLDER && variant != ORTH_PIP_PLUS) return ORTH_ERR_UNSUPPORTED;
    b->variant = variant;
    return ORTH_OK;
}

int orth_batch_step(orth_batch_t *b, const double *const *d_W, double *const *d_U, double *const *d_Hess) {
    if (!b) return ORTH_ERR_ARG;
    if (b->poisoned) return ORTH_ERR_POISONED;
    if (!d_W || !d_U || !d_Hess) return ORTH_ERR_ARG;
    if (b->step >= b->L.steps_max) return ORTH_ERR_CAPACITY;
    const int32_t count = b->L.count;
    BatchArgs a{};
    a.inst = reinterpret_cast<const BatchInst *>(b->ws + b->L.o_desc);
    a.count = count;
    a.step = b->step;
    a.two = b->variant == ORTH_PIP_PLUS ? 1 : 0;
    a.mixed = b->L.precision == ORTH_MIXED_SPLIT32 ? 1 : 0;
    a.hh = b->L.precision == ORTH_FP64_HOUSEHOLDER ? 1 : 0;
    a.W = d_W;
    a.U = d_U;
    a.Hess = d_Hess;
    a.status = b->status();
    const int32_t *dprefix = reinterpret_cast<const int32_t *>(b->ws + b->L.o_prefix);
    const size_t nw = b->L.widths.size();
    for (int ph = 0; ph < BP_COUNT; ++ph) {
        const bool second = ph == BP_LGRAM2 || ph == BP_LCHOL2 || ph == BP_RGRAM2 || ph == BP_RRED2 ||
                            ph == BP_RCHOL2;
        if (second && !a.two) continue;
        a.phase = ph;
        for (size_t w = 0; w < nw; ++w) {
            const size_t row = b->row(b->step, ph, w);
            const int32_t blocks = b->prefix[row + count];
            if (blocks == 0) continue;
            a.prefix = dprefix + row;
            const hipError_t e = batch_hh_phase(ph) ? launch_batch_hh_phase(a, b->L.widths[w], blocks, b->stream)
                                                    : launch_batch_phase(a, b->L.widths[w], blocks, b->lds[ph * nw + w],
                                                                         b->stream);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return ORTH_ERR_HIP;
            }
        }
    }
    b->step += 1;
    return ORTH_OK;
}

int orth_batch_status(orth_batch_t *b, int32_t *status, int32_t *info) {
    if (!b || !status) return ORTH_ERR_ARG;
    DevStatus ds{};
    if (hipStreamSynchronize(b->stream) != hipSuccess ||
        hipMemcpy(&ds, b->status(), sizeof(ds), hipMemcpyDeviceToHost) != hipSuccess) {
        (void)hipGetLastError();
        return ORTH_ERR_HIP;
    }
    *status = ds.code == 0 ? ORTH_OK : ORTH_ERR_BREAKDOWN;
    if (ds.code != 0) b->poisoned = true;
    if (info) {
        info[0] = ds.instance;
        info[1] = ds.level;
        info[2] = ds.leaf;
        info[3] = ds.sweep;
        info[4] = ds.column;
    }
    return ORTH_OK;
}

int orth_batch_mixed_fallbacks(orth_batch_t *b, int64_t *count) {
    if (!b || !count) return ORTH_ERR_ARG;
    DevStatus ds{};
    if (hipStreamSynchronize(b->stream) != hipSuccess ||
        hipMemcpy(&ds, b->status(), sizeof(ds), hipMemcpyDeviceToHost) != hipSuccess) {
        (void)hipGetLastError();
        return ORTH_ERR_HIP;
    }
    *count = ds.fallbacks;
    return ORTH_OK;
}

int orth_batch_progress(const orth_batch_t *b, int32_t *steps_done, int32_t *steps_max) {
    if (!b) return ORTH_ERR_ARG;
    if (steps_done) *steps_done = b->step;
    if (steps_max) *steps_max = b->L.steps_max;
    return ORTH_OK;
}

int orth_batch_leaf_rows(const orth_batch_t *b, int32_t *leaf_rows) {
    if (!b || !leaf_rows) return ORTH_ERR_ARG;
    for (int32_t i = 0; i < b->L.count; ++i) leaf_rows[i] = b->L.plans[i].leaf_rows;
    return ORTH_OK;
}

int orth_batch_destroy(orth_batch_t *b) {
    delete b;
    return ORTH_OK;
}

}  // extern "C"

// ============================================================ leaf-height autotuner
// Times whole orth_step sequences on synthetic blocks for every candidate
// leaf height: through one handle (copies = 1) or through a batch of
// `copies` identical instances, which keeps the GPU saturated as it is in a
// large batch.  Among candidates within 2% of the fastest the tallest wins:
// fewer leaves mean a smaller reduction level.

namespace {

// leaf heights 256 .. kTuneMaxLeaf in powers of two within [k_max, n], and n
// itself when n is below the largest
constexpr int64_t kTuneMaxLeaf = 65536;

std::vector<int32_t> tune_candidates(int64_t n, int32_t kmax) {
    std::vector<int32_t> c;
    for (int64_t lr = 256; lr <= kTuneMaxLeaf; lr *= 2)
        if (lr >= kmax && lr <= n) c.push_back((int32_t)lr);
    if (n <= kTuneMaxLeaf && n >= kmax && (c.empty() || c.back() != n)) c.push_back((int32_t)n);
    return c;
}

// single:  [plan][W n x s][U n x s][H k_max x s][R s x s]
// batch:   [batch][W n x s][U copies x n x s][Hess copies x k_max x k_max][3 x copies pointers]
// (doubles; every region 256-byte aligned)
struct TuneLayout {
    int64_t head = 0, oW = 0, oU = 0, oH = 0, oR = 0, oP = 0, total = 0;
};

bool tune_layout(int64_t n, int32_t s, int32_t kmax, int32_t copies, TuneLayout &L) {
    if (copies < 1 || copies > 4096) return false;
    const std::vector<int32_t> cand = tune_candidates(n, kmax);
    if (cand.empty()) return false;
    for (int32_t lr : cand) {
        int why;
        if (copies == 1) {
            Plan pl;
            if (!make_plan(n, s, kmax, lr, ORTH_FP64, pl, &why, 0, true)) return false;
            L.head = std::max(L.head, round_up(pl.total, kAlign));
        } else {
            std::vector<int64_t> nn(copies, n);
            std::vector<int32_t> ss(copies, s), kk(copies, kmax), ll(copies, lr);
            BatchLayout B;
            if (!make_batch_layout(copies, nn.data(), ss.data(), kk.data(), ll.data(), ORTH_FP64, B, &why))
                return false;
            L.head = std::max(L.head, round_up(B.total, kAlign));
        }
    }
    L.oW = L.head;
    L.oU = L.oW + round_up(n * s, kAlign);
    if (copies == 1) {
        L.oH = L.oU + round_up(n * s, kAlign);
        L.oR = L.oH + round_up((int64_t)kmax * s, kAlign);
        L.total = L.oR + round_up((int64_t)s * s, kAlign);
    } else {
        L.oH = L.oU + round_up(n * s, kAlign) * copies;
        L.oP = L.oH + round_up((int64_t)kmax * kmax, kAlign) * copies;
        L.total = L.oP + round_up(3 * (int64_t)copies, kAlign);
    }
    return true;
}

// time of `steps` calls for one candidate; ORTH_ERR_BREAKDOWN if it broke down
int tune_one(int64_t n, int32_t s, int32_t kmax, int32_t lr, int32_t steps, int32_t copies,
             const TuneLayout &L, double *ws, hipStream_t st, hipEvent_t e0, hipEvent_t e1, double *ms_out) {
    double *W = ws + L.oW;
    double ms_total = 0.0;
    auto timed = [&](auto &&call) -> int {
        float ms = 0.0f;
        if (hipEventRecord(e0, st) != hipSuccess) return ORTH_ERR_HIP;
        const int rc = call();
        if (rc != ORTH_OK) return rc;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            return ORTH_ERR_HIP;
        ms_total += ms;
        return ORTH_OK;
    };
    int rc = ORTH_OK;
    int32_t status = ORTH_OK;
    if (copies == 1) {
        orth_t *h = nullptr;
        rc = orth_create(n, s, kmax, lr, ORTH_FP64, ws, (size_t)L.head * sizeof(double), st, &h);
        if (rc != ORTH_OK) return rc;
        double *U = ws + L.oU, *H = ws + L.oH, *R = ws + L.oR;
        for (int32_t j = 0; j < steps && rc == ORTH_OK; ++j) {
            if (launch_synth(W, n, n, s, (uint64_t)j + 1, st) != hipSuccess) { rc = ORTH_ERR_HIP; break; }
            rc = timed([&] { return orth_step(h, W, n, H, kmax, R, s, U, n); });
        }
        if (rc == ORTH_OK) rc = orth_status(h, &status, nullptr);
        (void)orth_destroy(h);
    } else {
        std::vector<int64_t> nn(copies, n);
        std::vector<int32_t> ss(copies, s), kk(copies, kmax), ll(copies, lr);
        orth_batch_t *b = nullptr;
        rc = orth_batch_create(copies, nn.data(), ss.data(), kk.data(), ll.data(), ORTH_FP64, ws,
                               (size_t)L.head * sizeof(double), st, &b);
        if (rc != ORTH_OK) return rc;
        // device pointer arrays: every copy reads the same W and writes its own U and Hess
        std::vector<double *> ptrs(3 * (size_t)copies);
        for (int32_t i = 0; i < copies; ++i) {
            ptrs[i] = W;
            ptrs[copies + i] = ws + L.oU + round_up(n * s, kAlign) * i;
            ptrs[2 * copies + i] = ws + L.oH + round_up((int64_t)kmax * kmax, kAlign) * i;
        }
        double **dptr = reinterpret_cast<double **>(ws + L.oP);
        if (hipMemcpyAsync(dptr, ptrs.data(), ptrs.size() * sizeof(double *), hipMemcpyHostToDevice, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            rc = ORTH_ERR_HIP;
        for (int32_t j = 0; j < steps && rc == ORTH_OK; ++j) {
            if (launch_synth(W, n, n, s, (uint64_t)j + 1, st) != hipSuccess) { rc = ORTH_ERR_HIP; break; }
            rc = timed([&] { return orth_batch_step(b, dptr, dptr + copies, dptr + 2 * copies); });
        }
        if (rc == ORTH_OK) rc = orth_batch_status(b, &status, nullptr);
        (void)orth_batch_destroy(b);
    }
    if (rc != ORTH_OK) return rc;
    *ms_out = ms_total;
    return status == ORTH_OK ? ORTH_OK : ORTH_ERR_BREAKDOWN;
}

// fan-in candidates for a handle of p leaves: the single level (0), then
// 2, 4, 8, ... below p
std::vector<int32_t> tune_fan_ins(int32_t p) {
    std::vector<int32_t> c{0};
    for (int32_t g = 2; g < p; g *= 2) c.push_back(g);
    return c;
}

// regions of the fan-in search: [handle workspace][W][U][H][R] (doubles)
bool tune_tree_layout(int64_t n, int32_t s, int32_t kmax, int32_t lr, TuneLayout &L) {
    Plan pl;
    int why;
    if (!make_plan(n, s, kmax, lr, ORTH_FP64, pl, &why, 0, true)) return false;
    for (int32_t g : tune_fan_ins(pl.p)) {
        Plan pg;
        if (!make_plan(n, s, kmax, lr, ORTH_FP64, pg, &why, g, true)) return false;
        L.head = std::max(L.head, round_up(pg.total, kAlign));
    }
    L.oW = L.head;
    L.oU = L.oW + round_up(n * s, kAlign);
    L.oH = L.oU + round_up(n * s, kAlign);
    L.oR = L.oH + round_up((int64_t)kmax * s, kAlign);
    L.total = L.oR + round_up((int64_t)s * s, kAlign);
    return true;
}

}  // namespace

extern "C" {

size_t orth_tune_tree_workspace_bytes(int64_t n, int32_t s, int32_t k_max, int32_t leaf_rows) {
    TuneLayout L;
    if (leaf_rows < 1 || !tune_tree_layout(n, s, k_max, leaf_rows, L)) return 0;
    return (size_t)L.total * sizeof(double);
}

int orth_tune_tree(int64_t n, int32_t s, int32_t k_max, int32_t leaf_rows, int32_t steps, void *d_workspace,
                   size_t workspace_bytes, void *stream, int32_t *best_fan_in, int32_t *cand_fan_in,
                   double *cand_ms, int32_t max_cand, int32_t *ncand) {
    if (!best_fan_in || (max_cand > 0 && (!cand_fan_in || !cand_ms))) return ORTH_ERR_ARG;
    TuneLayout L;
    if (leaf_rows < 1 || !tune_tree_layout(n, s, k_max, leaf_rows, L)) return ORTH_ERR_ARG;
    if (steps < 1 || steps > k_max / s) return ORTH_ERR_ARG;
    if (!d_workspace || ((uintptr_t)d_workspace % 256) != 0 || workspace_bytes < (size_t)L.total * sizeof(double))
        return ORTH_ERR_WORKSPACE;
    const int32_t p = (int32_t)std::max<int64_t>(1, n / leaf_rows);
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *ws = static_cast<double *>(d_workspace);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreateWithFlags(&e0, hipEventDisableSystemFence) != hipSuccess ||
        hipEventCreateWithFlags(&e1, hipEventDisableSystemFence) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipGetLastError();
        return ORTH_ERR_HIP;
    }
    const std::vector<int32_t> cand = tune_fan_ins(p);
    std::vector<double> times(cand.size(), -1.0);
    double *W = ws + L.oW, *U = ws + L.oU, *H = ws + L.oH, *R = ws + L.oR;
    int rc = ORTH_OK;
    for (size_t c = 0; c < cand.size() && rc == ORTH_OK; ++c) {
        orth_t *h = nullptr;
        rc = orth_create_tree(n, s, k_max, leaf_rows, ORTH_FP64, cand[c], ws, (size_t)L.head * sizeof(double), st,
                              &h);
        if (rc != ORTH_OK) break;
        double total = 0.0;
        for (int32_t j = 0; j < steps && rc == ORTH_OK; ++j) {
            float ms = 0.0f;
            if (launch_synth(W, n, n, s, (uint64_t)j + 1, st) != hipSuccess || hipEventRecord(e0, st) != hipSuccess) {
                rc = ORTH_ERR_HIP;
                break;
            }
            rc = orth_step(h, W, n, H, k_max, R, s, U, n);
            if (rc == ORTH_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = ORTH_ERR_HIP;
            total += ms;
        }
        int32_t status = ORTH_OK;
        if (rc == ORTH_OK) rc = orth_status(h, &status, nullptr);
        (void)orth_destroy(h);
        if (rc == ORTH_OK && status == ORTH_OK) times[c] = total;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != ORTH_OK) {
        (void)hipGetLastError();
        return rc;
    }
    // the fastest; the single level (the simplest) wins ties within 2%
    double fastest = -1.0;
    size_t best = 0;
    for (size_t c = 0; c < cand.size(); ++c)
        if (times[c] >= 0.0 && (fastest < 0.0 || times[c] < fastest)) {
            fastest = times[c];
            best = c;
        }
    if (fastest < 0.0) return ORTH_ERR_BREAKDOWN;
    if (times[0] >= 0.0 && times[0] <= 1.02 * fastest) best = 0;
    *best_fan_in = cand[best];
    for (size_t c = 0; c < cand.size() && (int32_t)c < max_cand; ++c) {
        cand_fan_in[c] = cand[c];
        cand_ms[c] = times[c];
    }
    if (ncand) *ncand = (int32_t)cand.size();
    return ORTH_OK;
}

}  // extern "C"

namespace {

// tile candidates: the plan's own choice first, then leaf Gram rows x leaf
// row-update rows per workgroup (and, from s = 16, the register-streamed
// row updates against the LDS-staged ones)
std::vector<orth_tiles> tune_tile_candidates(int32_t s) {
    std::vector<orth_tiles> c{orth_tiles{0, 0, ORTH_TILE_AUTO}};
    for (int32_t g : {1024, 2048, 4096})
        for (int32_t u : {256, 512, 1024, 2048})
            for (int32_t kern = ORTH_TILE_AUTO; kern <= (s >= 16 ? ORTH_TILE_REGISTER : ORTH_TILE_AUTO); ++kern)
                c.push_back(orth_tiles{g, u, kern});
    return c;
}

// [handle workspace (the largest candidate's)][W][U][H][R] (doubles)
bool tune_tiles_layout(int64_t n, int32_t s, int32_t kmax, int32_t lr, TuneLayout &L) {
    for (const orth_tiles &t : tune_tile_candidates(s)) {
        Plan pl;
        int why;
        if (!make_plan(n, s, kmax, lr, ORTH_FP64, pl, &why, 0, true, &t)) return false;
        L.head = std::max(L.head, round_up(pl.total, kAlign));
    }
    L.oW = L.head;
    L.oU = L.oW + round_up(n * s, kAlign);
    L.oH = L.oU + round_up(n * s, kAlign);
    L.oR = L.oH + round_up((int64_t)kmax * s, kAlign);
    L.total = L.oR + round_up((int64_t)s * s, kAlign);
    return true;
}

}  // namespace

extern "C" {

size_t orth_tune_tiles_workspace_bytes(int64_t n, int32_t s, int32_t k_max, int32_t leaf_rows) {
    TuneLayout L;
    if (leaf_rows < 1 || !tune_tiles_layout(n, s, k_max, leaf_rows, L)) return 0;
    return (size_t)L.total * sizeof(double);
}

int orth_tune_tiles(int64_t n, int32_t s, int32_t k_max, int32_t leaf_rows, int32_t steps, void *d_workspace,
                    size_t workspace_bytes, void *stream, orth_tiles *best, orth_tiles *cand, double *cand_ms,
                    int32_t max_cand, int32_t *ncand) {
    if (!best || (max_cand > 0 && (!cand || !cand_ms))) return ORTH_ERR_ARG;
    TuneLayout L;
    if (leaf_rows < 1 || !tune_tiles_layout(n, s, k_max, leaf_rows, L)) return ORTH_ERR_ARG;
    if (steps < 1 || steps > k_max / s) return ORTH_ERR_ARG;
    if (!d_workspace || ((uintptr_t)d_workspace % 256) != 0 || workspace_bytes < (size_t)L.total * sizeof(double))
        return ORTH_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *ws = static_cast<double *>(d_workspace);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreateWithFlags(&e0, hipEventDisableSystemFence) != hipSuccess ||
        hipEventCreateWithFlags(&e1, hipEventDisableSystemFence) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipGetLastError();
        return ORTH_ERR_HIP;
    }
    const std::vector<orth_tiles> tc = tune_tile_candidates(s);
    std::vector<double> times(tc.size(), -1.0);
    double *W = ws + L.oW, *U = ws + L.oU, *H = ws + L.oH, *R = ws + L.oR;
    int rc = ORTH_OK;
    for (size_t c = 0; c < tc.size() && rc == ORTH_OK; ++c) {
        orth_t *h = nullptr;
        rc = orth_create_tiles(n, s, k_max, leaf_rows, ORTH_FP64, 0, &tc[c], ws, (size_t)L.head * sizeof(double),
                               st, &h);
        if (rc != ORTH_OK) break;
        double total = 0.0;
        for (int32_t j = 0; j < steps && rc == ORTH_OK; ++j) {
            float ms = 0.0f;
            if (launch_synth(W, n, n, s, (uint64_t)j + 1, st) != hipSuccess || hipEventRecord(e0, st) != hipSuccess) {
                rc = ORTH_ERR_HIP;
                break;
            }
            rc = orth_step(h, W, n, H, k_max, R, s, U, n);
            if (rc == ORTH_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = ORTH_ERR_HIP;
            total += ms;
        }
        int32_t status = ORTH_OK;
        if (rc == ORTH_OK) rc = orth_status(h, &status, nullptr);
        (void)orth_destroy(h);
        if (rc == ORTH_OK && status == ORTH_OK) times[c] = total;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != ORTH_OK) {
        (void)hipGetLastError();
        return rc;
    }
    // the fastest; the plan's own choice wins ties within 2%
    double fastest = -1.0;
    size_t pick = 0;
    for (size_t c = 0; c < tc.size(); ++c)
        if (times[c] >= 0.0 && (fastest < 0.0 || times[c] < fastest)) {
            fastest = times[c];
            pick = c;
        }
    if (fastest < 0.0) return ORTH_ERR_BREAKDOWN;
    if (times[0] >= 0.0 && times[0] <= 1.02 * fastest) pick = 0;
    *best = tc[pick];
    for (size_t c = 0; c < tc.size() && (int32_t)c < max_cand; ++c) {
        cand[c] = tc[c];
        cand_ms[c] = times[c];
    }
    if (ncand) *ncand = (int32_t)tc.size();
    return ORTH_OK;
}

size_t orth_tune_workspace_bytes(int64_t n, int32_t s, int32_t k_max, int32_t copies) {
    TuneLayout L;
    if (!tune_layout(n, s, k_max, copies, L)) return 0;
    return (size_t)L.total * sizeof(double);
}

int orth_tune_leaf_rows(int64_t n, int32_t s, int32_t k_max, int32_t steps, int32_t copies,
                        void *d_workspace, size_t workspace_bytes, void *stream, int32_t *best_leaf_rows,
                        int32_t *cand_rows, double *cand_ms, int32_t max_cand, int32_t *ncand) {
    if (!best_leaf_rows || (max_cand > 0 && (!cand_rows || !cand_ms))) return ORTH_ERR_ARG;
    TuneLayout L;
    if (!tune_layout(n, s, k_max, copies, L)) return ORTH_ERR_ARG;
    if (steps < 1 || steps > k_max / s) return ORTH_ERR_ARG;
    if (!d_workspace || ((uintptr_t)d_workspace % 256) != 0 || workspace_bytes < (size_t)L.total * sizeof(double))
        return ORTH_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *ws = static_cast<double *>(d_workspace);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreateWithFlags(&e0, hipEventDisableSystemFence) != hipSuccess ||
        hipEventCreateWithFlags(&e1, hipEventDisableSystemFence) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipGetLastError();
        return ORTH_ERR_HIP;
    }
    const std::vector<int32_t> cand = tune_candidates(n, k_max);
    std::vector<double> times(cand.size(), -1.0);
    int rc = ORTH_OK;
    for (size_t c = 0; c < cand.size(); ++c) {
        double ms = 0.0;
        const int r = tune_one(n, s, k_max, cand[c], steps, copies, L, ws, st, e0, e1, &ms);
        if (r == ORTH_OK) times[c] = ms;
        else if (r != ORTH_ERR_BREAKDOWN) { rc = r; break; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != ORTH_OK) {
        (void)hipGetLastError();
        return rc;
    }
    double fastest = -1.0;
    for (double t : times)
        if (t >= 0.0 && (fastest < 0.0 || t < fastest)) fastest = t;
    if (fastest < 0.0) return ORTH_ERR_BREAKDOWN;
    int32_t best = 0;
    for (size_t c = 0; c < cand.size(); ++c)
        if (times[c] >= 0.0 && times[c] <= 1.02 * fastest) best = std::max(best, cand[c]);
    *best_leaf_rows = best;
    for (size_t c = 0; c < cand.size() && (int32_t)c < max_cand; ++c) {
        cand_rows[c] = cand[c];
        cand_ms[c] = times[c];
    }
    if (ncand) *ncand = (int32_t)cand.size();
    return ORTH_OK;
}

}  // extern "C"
