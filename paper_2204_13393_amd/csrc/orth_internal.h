// Internal declarations shared by the kernels and the C-ABI runtime.
//
// Row addressing.  Every kernel sees its operands as column-major matrices
// whose *logical* rows map to physical rows through a RowMap.  The leaf
// level uses the identity.  The reduction level (Sec. 4.1, the PQR problem
// on the stacked leaf coefficient blocks [[T_i, P_i], [0, N_i]]) stores leaf
// i's block in rows [i*seg_stride, i*seg_stride + seg_len) of the tree-factor
// matrix, so logical row r maps to (r / seg_len) * seg_stride + r % seg_len.
//
// Level geometry.  A level solves `nleaf` independent local PQR problems on
// consecutive row ranges of `leaf_rows` logical rows (the last one takes the
// remainder).  Each leaf is cut into chunks of `chunk_rows` rows, one
// workgroup per chunk; per-chunk partial Gram blocks are summed per leaf in
// chunk order, so results are bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace orth {

struct RowMap {
    int64_t seg_len;     // 0 = identity
    int64_t seg_stride;
    __host__ __device__ __forceinline__ int64_t phys(int64_t r) const {
        if (seg_len == 0) return r;
        const int64_t q = r / seg_len;
        return q * seg_stride + (r - q * seg_len);
    }
};

struct LevelGeom {
    int64_t nrows;       // logical rows of the level
    int64_t leaf_rows;   // logical rows of every leaf but the last
    int32_t nleaf;
    int32_t chunk_rows;
    int32_t cpl;         // chunks of a full leaf
    int32_t cpl_last;    // chunks of the last leaf
    RowMap map;

    __host__ __device__ int32_t nchunks() const { return (nleaf - 1) * cpl + cpl_last; }
    __host__ __device__ int32_t first_chunk(int32_t leaf) const { return leaf * cpl; }
    __host__ __device__ int32_t chunks_of(int32_t leaf) const {
        return leaf == nleaf - 1 ? cpl_last : cpl;
    }
    __host__ __device__ int64_t leaf_begin(int32_t leaf) const { return (int64_t)leaf * leaf_rows; }
    __host__ __device__ int64_t leaf_end(int32_t leaf) const {
        return leaf == nleaf - 1 ? nrows : (int64_t)(leaf + 1) * leaf_rows;
    }
    // chunk g -> (leaf, logical row range)
    __host__ __device__ void chunk(int32_t g, int32_t &leaf, int64_t &r0, int64_t &r1) const {
        const int32_t full = (nleaf - 1) * cpl;
        int32_t c;
        if (g < full) { leaf = g / cpl; c = g - leaf * cpl; }
        else { leaf = nleaf - 1; c = g - full; }
        r0 = leaf_begin(leaf) + (int64_t)c * chunk_rows;
        const int64_t e = leaf_end(leaf);
        r1 = r0 + chunk_rows < e ? r0 + chunk_rows : e;
    }
};

// ---- level planning shared by the runtime and the batched kernels ----
constexpr int kThreads = 256;         // threads per workgroup of every kernel
constexpr int kWaves = kThreads / 64;
constexpr int kGramTPW = 4;           // 16-column tiles per wave in the Gram kernel

// waves of a Gram workgroup that share rows (1, 2, 4), workgroups across the
// columns, and partial slots per chunk (row groups)
__host__ __device__ inline int gram_tile_groups(int ncol) {
    const int nmt = (ncol + 15) / 16;
    const int groups = (nmt + kGramTPW - 1) / kGramTPW;
    return groups <= 1 ? 1 : (groups <= 2 ? 2 : 4);
}
// At s = 32 the products outweigh the loads, so the tiles are spread evenly
// over the waves of a chunk's workgroups (at most gram_tpw of them per wave)
// rather than packed kGramTPW to a wave: packing left whole workgroups with
// one busy wave.  Each output entry still comes from one wave, summed over
// the rows in the same order, so the split does not change the bits.
__host__ __device__ constexpr int gram_tpw(int s) { return s >= 32 ? 5 : kGramTPW; }
__host__ __device__ inline int gram_col_groups(int ncol, int s) {
    const int nmt = (ncol + 15) / 16;
    if (s >= 32 && gram_tile_groups(ncol) == kWaves) return (nmt + kWaves * gram_tpw(s) - 1) / (kWaves * gram_tpw(s));
    const int groups = (nmt + kGramTPW - 1) / kGramTPW;
    return groups <= 4 ? 1 : (groups + 3) / 4;
}
// first tile and number of tiles (<= gram_tpw(s); none when <= 0) of tile
// group tg (workgroup column by, wave w: tg = by * tile_groups + w % tile_groups)
__host__ __device__ inline void gram_wave_tiles(int ncol, int s, int tg, int &tile0, int &ntl) {
    const int nmt = (ncol + 15) / 16;
    if (s >= 32 && gram_tile_groups(ncol) == kWaves) {
        const int w = kWaves * gram_col_groups(ncol, s);
        tile0 = tg * nmt / w;
        ntl = (tg + 1) * nmt / w - tile0;
    } else {
        tile0 = tg * kGramTPW;
        ntl = nmt - tile0 < kGramTPW ? nmt - tile0 : kGramTPW;
    }
}
__host__ __device__ inline int gram_row_groups(int ncol) { return kWaves / gram_tile_groups(ncol); }
constexpr int kLeafChunk = 2048;      // rows per workgroup at the leaf level
constexpr int kRootChunk = 2048;      // rows per workgroup at the reduction level
// rows per workgroup in the leaf row updates: one 512-row pass of a
// workgroup's four waves at s <= 8 (eight rows per lane); measured 2.7%
// faster per s = 8 sequence than 2048 (1% at s = 16, equal at s = 32)
constexpr int kFinalChunk = 512;
// the batched form's leaf row updates keep 2048-row chunks (1% faster there:
// its instances are short and each workgroup first locates its instance)
constexpr int kBatchFinalChunk = 2048;
// rows per workgroup in the reduction-level row updates: the reduction level
// has p (k + s) rows, and 512-row chunks give its correction and finalize
// enough workgroups (its Gram keeps 2048: more chunks mean more partial sums
// for the Cholesky to add)
constexpr int kRootRowChunk = 512;
constexpr int kReduceGroup = 16;      // slots pre-summed per group at a single-leaf level

__host__ __device__ inline int64_t ceil_div64(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Fixed-order sum p[0] + p[stride] + ... + p[(cnt-1) stride], added in slot
// order; the loads are issued sixteen (then eight, then four) at a time so
// they are in flight together (the additions, and so the bits, are those of
// the plain loop).  A small problem's leaf sums 32 slots: two rounds of
// load latency instead of four.
template <int B>
__device__ __forceinline__ void slot_sum_batches(const double *p, int64_t stride, int cnt, int &q, double &v) {
    for (; q + B <= cnt; q += B) {
        double t[B];
#pragma unroll
        for (int u = 0; u < B; ++u) t[u] = p[(int64_t)(q + u) * stride];
#pragma unroll
        for (int u = 0; u < B; ++u) v += t[u];
    }
}
__device__ __forceinline__ double slot_sum(const double *p, int64_t stride, int cnt) {
    double v = 0.0;
    int q = 0;
    slot_sum_batches<16>(p, stride, cnt, q, v);
    slot_sum_batches<8>(p, stride, cnt, q, v);
    slot_sum_batches<4>(p, stride, cnt, q, v);
    for (; q < cnt; ++q) v += p[(int64_t)q * stride];
    return v;
}

// leaves of leaf_rows rows (the last takes the remainder), identity rows
__host__ __device__ inline LevelGeom make_leaf_geom(int64_t n, int32_t leaf_rows, int32_t p, int chunk) {
    LevelGeom g{};
    g.nrows = n;
    g.leaf_rows = leaf_rows;
    g.nleaf = p;
    g.chunk_rows = chunk;
    const int64_t last = n - (int64_t)(p - 1) * leaf_rows;
    g.cpl = (int32_t)ceil_div64(leaf_rows, chunk);
    g.cpl_last = (int32_t)ceil_div64(last, chunk);
    g.map = RowMap{0, 0};
    return g;
}

// the reduction level: one local problem over p segments of seg_len rows,
// segment i stored at rows [i*kmax, i*kmax + seg_len)
__host__ __device__ inline LevelGeom make_root_geom(int32_t p, int32_t kmax, int64_t seg_len, int chunk) {
    LevelGeom g{};
    g.nrows = (int64_t)p * seg_len;
    g.leaf_rows = g.nrows;
    g.nleaf = 1;
    g.chunk_rows = chunk;
    g.cpl = (int32_t)ceil_div64(g.nrows, chunk);
    g.cpl_last = g.cpl;
    g.map = RowMap{seg_len, kmax};
    return g;
}

// a level of a reduction tree (Sec. 4.1, the reduction problem solved by
// TreeTSPQR again): nchild child segments of seg_len rows (child c stored at
// rows [c*kmax, c*kmax + seg_len)), grouped into nodes of fan_in
// consecutive children, the last node taking the rest; fan_in >= nchild is
// the single node of make_root_geom
__host__ __device__ inline LevelGeom make_tree_geom(int32_t nchild, int32_t fan_in, int32_t kmax, int64_t seg_len,
                                                    int chunk) {
    if (fan_in >= nchild) return make_root_geom(nchild, kmax, seg_len, chunk);
    LevelGeom g{};
    g.nrows = (int64_t)nchild * seg_len;
    g.nleaf = (int32_t)ceil_div64(nchild, fan_in);
    g.leaf_rows = (int64_t)fan_in * seg_len;
    g.chunk_rows = chunk;
    g.cpl = (int32_t)ceil_div64(g.leaf_rows, chunk);
    g.cpl_last = (int32_t)ceil_div64(g.nrows - (int64_t)(g.nleaf - 1) * g.leaf_rows, chunk);
    g.map = RowMap{seg_len, kmax};
    return g;
}

// Device status record (first failure wins).
struct DevStatus {
    int32_t code;        // 0 ok, 3 breakdown
    int32_t level;       // 0 leaves, 1 reduction
    int32_t leaf;
    int32_t sweep;       // CholeskyQR sweep 1 or 2
    int32_t column;      // pivot column
    int32_t instance;    // batch instance (-1 for a single handle)
    int32_t retry;       // mixed form: a first-sweep leaf pivot failed on the FP32
                         // copy in this step; the sweep is redone from the FP64 basis
    int32_t fallbacks;   // mixed form: steps that took that fallback
};

// Per-leaf small-matrix record, in doubles:
//   P1 [kmax][s] | N1 [s][s] | N1inv [s][s] | P2 [kmax][s] | N2inv [s][s]
// All stored row-major ([row][col]).
__host__ __device__ inline int64_t small_stride(int32_t kmax, int32_t s) {
    return 2 * (int64_t)kmax * s + 3 * (int64_t)s * s;
}

// Column-major matrix under a level's RowMap, or (lstride > 0, leaf level
// only) stored leaf by leaf: leaf i's rows form their own column-major block
// at ptr + i lstride with leading dimension ld (ld_last for the last leaf,
// which may be taller), so that one leaf's columns lie together in memory.
// c0: first column (blocked storage only; a plain operand's ptr already
// points at its first column).
struct Operand {
    const double *ptr;
    int64_t ld;
    int64_t lstride;
    int64_t ld_last;
    int32_t c0;
};
struct OutOperand {
    double *ptr;
    int64_t ld;
    int64_t lstride;
    int64_t ld_last;
    int32_t c0;
};

// Element offset, from an operand's ptr, of a leaf's (global row 0, column
// 0) and that leaf's leading dimension: ptr + offset + c ld_leaf + r is
// element (r, c) for every global row r of the leaf.
__host__ __device__ inline int64_t leaf_offset(int64_t ld, int64_t lstride, int64_t ld_last, int32_t c0,
                                               const LevelGeom &g, int32_t leaf, int64_t &ld_leaf) {
    if (lstride == 0) {
        ld_leaf = ld;
        return 0;
    }
    ld_leaf = leaf == g.nleaf - 1 ? ld_last : ld;
    return (int64_t)leaf * lstride + (int64_t)c0 * ld_leaf - g.leaf_begin(leaf);
}

// The operand as a plain column-major matrix over one leaf's global rows.
// The base address is formed in integers: it may lie before the block (a
// leaf's rows start at leaf_begin), every element read through it lies
// inside.
template <class Op>
__host__ __device__ inline Op leaf_view(const Op &o, const LevelGeom &g, int32_t leaf) {
    if (o.lstride == 0) return o;
    Op v = o;
    int64_t ldl;
    const int64_t off = leaf_offset(o.ld, o.lstride, o.ld_last, o.c0, g, leaf, ldl);
    v.ptr = reinterpret_cast<decltype(o.ptr)>(reinterpret_cast<uintptr_t>(o.ptr) + off * (int64_t)sizeof(double));
    v.ld = ldl;
    v.lstride = 0;
    v.ld_last = 0;
    v.c0 = 0;
    return v;
}

// The FP32 copy of a blocked operand (same element layout, floats).
template <class F, class Op>
__host__ __device__ inline F *leaf_view_hi(F *hi, const Op &o, const LevelGeom &g, int32_t leaf) {
    if (!hi || o.lstride == 0) return hi;
    int64_t ldl;
    const int64_t off = leaf_offset(o.ld, o.lstride, o.ld_last, o.c0, g, leaf, ldl);
    return reinterpret_cast<F *>(reinterpret_cast<uintptr_t>(hi) + off * (int64_t)sizeof(float));
}

// ---- kernel launch descriptors (filled by the runtime) ----

// pass A: partial [Q X]^T X per chunk (and per row group of the chunk)
struct GramArgs {
    Operand Q;            // k columns
    const float *Qhi;     // mixed form, sweep 1: read the FP32 copy of Q (same ld) instead
    Operand X;            // s columns
    int32_t k;
    int32_t tile_groups;  // waves of a workgroup sharing the rows: 1, 2 or 4
    LevelGeom geom;
    double *partials;     // slot (chunk * row_groups + rg): [k + s][s]
    int64_t part_stride;  // doubles per slot
    DevStatus *status;
    int32_t cond;         // 1: run only when *retry is set (the mixed form's fallback)
    int32_t clear_retry;  // 1: the first thread clears *retry (the step's first Gram)
    int32_t *retry;       // mixed form's retry flag: &status->retry, or a batch instance's own
};

// fixed-order pre-reduction of many partial slots of one leaf:
// out[grp][e] = sum over slots [grp*group, min((grp+1)*group, nslots)) of in[slot][e]
struct ReduceArgs {
    const double *in;
    int64_t stride;       // doubles per slot (in and out)
    int32_t nslots;
    int32_t group;
    int32_t nentries;
    double *out;
    const DevStatus *status;
    int32_t cond;         // 1: run only when *retry is set
    const int32_t *retry;
};

// per-leaf Cholesky of one sweep (and the combination after sweep 2)
struct CholArgs {
    const double *partials;   // slot (leaf * slots_per_leaf + i)
    int64_t part_stride;
    int32_t nleaf;
    int32_t slots_per_leaf;   // every leaf but the last
    int32_t slots_last;       // the last leaf
    int32_t k;
    int32_t kmax;
    int32_t sweep;        // 1 or 2
    int32_t level;        // for the status record
    int32_t final_sweep;  // sweep that produces [P; N]
    double *small;
    int64_t small_stride;
    // output of the final sweep: either the next level's stacked X (segmented)
    // or, at the root, H (k x s) and R (s x s)
    double *Yout;         // next-level X, column-major, ld = ldy, leaf i at row i*yseg
    int64_t ldy;
    int64_t yseg;
    double *H;
    int64_t ldh;
    double *R;
    int64_t ldr;
    int32_t instance;         // for the status record (-1: single handle)
    DevStatus *status;
    // leaf level, second sweep: also store P2 row-major in the left half of
    // the per-leaf coefficient record [c][2s] (nullptr: not needed)
    double *pc;
    int64_t pc_stride;        // doubles per leaf record
    int32_t soft;             // 1: a failed pivot sets *retry instead of the breakdown
    int32_t cond;             // 1: run only when *retry is set
    int32_t *retry;           // as GramArgs::retry
};

// row update: sweep 1: u1 = (x - q P1) N1^{-1} (U1 = x in, Qnew = u1 out);
// sweep 2: u = (u1 - q P2) N2^{-1} -> new basis columns, optional explicit
// Uout = [q u] C_leaf
struct FinalizeArgs {
    Operand Q;            // k columns (read)
    OutOperand Qnew;      // s output columns, same RowMap
    float *Qnew_hi;       // mixed form: also store fl32 of the new columns here (ld of Qnew)
    Operand U1;           // s input columns (x for sweep 1, u1 for sweep 2)
    int32_t sweep;        // which coefficients of the leaf record: 1 (P1, N1^-1) or 2 (P2, N2^-1)
    int32_t k;
    LevelGeom geom;
    const double *small;
    int64_t small_stride;
    int32_t kmax;
    int32_t single_sweep; // 1: u = u1 (BCGS-PIP variant)
    // leaf finalize: the per-leaf coefficient record, row-major [c][2s] with
    // P2 row c in columns 0..s-1 and C_i row c in columns s..2s-1 (C_i =
    // [P~_i; N~_i], (k+s) x s), leaf i at Cptr + i*cseg; one load per basis
    // column fetches both.  Cptr == nullptr -> no explicit output
    const double *Cptr;
    int64_t cseg;
    // reduction-level finalize: also store the new columns as the right half
    // of those records (logical row r = leaf*(k+s) + c ->
    // Crow[leaf*crow_seg + c*2s + s + j])
    double *Crow;
    int64_t crow_seg;
    OutOperand Uout;      // explicit output (identity RowMap, leaf level)
    // tree level below the root: the explicit product [q u] C goes to the
    // children's coefficient records instead (logical row r = child*(k+s) + c
    // -> Cout[child*cout_seg + c*2s + s + j]); Uout unused
    double *Cout;
    int64_t cout_seg;
    const DevStatus *status;
    int32_t reg_only;     // host-side choice: 1 keeps the register-streamed kernel for s >= 16
};

// Y = Q C_leaf for a column block of C
struct ApplyArgs {
    Operand Q;
    int32_t k;
    LevelGeom geom;
    const double *Cptr;   // element (c, j) at Cptr[j*ldc + leaf*cseg + c]
    int64_t ldc;
    int64_t cseg;         // 0: same C for all leaves
    int32_t m;            // columns of this block
    OutOperand Y;         // under geom.map
};

// ---- Householder leaves (orth_hh.hip) ----
// leaf bases as unit reflectors V_i with compact-WY factors T_i; per leaf
// three k_max x k_max blocks at T + i 3 k_max^2 (T column-major, T row-major,
// the reflectors' top rows row-major); see orth_hh.hip for the step
struct HhArgs {
    LevelGeom geom;           // leaf geometry (identity rows)
    int32_t k, kmax;
    double *Q;                // reflectors (the stored leaf bases)
    int64_t ldq;
    double *T;
    // partial Gram slots of the leaf Gram kernel ([k+s][s] each)
    const double *partials;
    int64_t part_stride;
    int32_t slots_per_leaf, slots_last;
    double *small;            // per-leaf records (sweep-1 projection and inverse normalizer)
    int64_t small_stride;
    const double *X;          // panel input: Q_k^T w (or w at k = 0)
    int64_t ldx;
    double *Yout;             // next level's X: leaf i's [P_i; N_i] at rows i*yseg
    int64_t ldy, yseg;
    double *crec;             // per-leaf [left | right] records, row-major (k+s) x 2s
    int64_t cseg;
    double *U;                // explicit output (E C term)
    int64_t ldu;
    const DevStatus *status;
    // orth_apply_Q: per-leaf coefficient blocks C_i (k x m) in, -Z_i out, element
    // (c, j) at [j * ldca + leaf * kmax + c]; m <= 16 columns
    const double *ca;
    double *ca_out;
    int64_t ldca;
    int32_t m;
};
enum HhKernel { HH_PREP = 0, HH_PANEL, HH_TUPD, HH_COEF, HH_ADDEC, HH_APPLY_COEF, HH_APPLY_ADD };
// (k + s) x 16 bound of orth_apply_Q's per-leaf coefficient blocks at full
// width (two of them within 64 KB of LDS; narrower blocks above it)
constexpr int64_t kHhMaxCoef = 4096;
// dynamic LDS a workgroup may hold (the per-leaf small products stage
// (k + s) x s blocks in it)
constexpr size_t kHhLdsMax = 160 * 1024;
// largest leaf the panel kernel holds in registers for block width s (0: unsupported s)
int64_t hh_max_leaf_rows(int s);
// the per-leaf small products' LDS staging fits for block width s at k_max columns
bool hh_small_fits(int s, int64_t kmax);
// once per handle, on its device: raise the dynamic-LDS limit of the
// Householder kernels of block width s
hipError_t prepare_hh_kernels(int s);
hipError_t launch_hh(int s, HhKernel which, const HhArgs &a, hipStream_t st);
// orth_apply_Q with Householder leaves: HH_APPLY_COEF (Z_i = T V_top^T C_i, -Z_i
// to ca_out), then the apply kernel, then HH_APPLY_ADD (Y_i[0:k] += C_i)
hipError_t launch_hh_apply(HhKernel which, const HhArgs &a, hipStream_t st);

// ---- batched form: many independent instances, one grouped launch per phase ----
// Per-instance descriptor (device memory); regions carved like a single handle.
struct BatchInst {
    int64_t n, ldq, ldt;
    int32_t s, kmax, leaf_rows, p;
    int32_t cL, cR;           // Gram chunk heights of the leaves and the reduction (the plan's)
    double *Q, *T, *Y, *U1L, *U1R, *PL, *PR, *PR2, *SL, *SR, *CL;
    float *Qhi;               // mixed form: FP32 copy of Q (same layout, floats); nullptr for FP64
    int32_t *retry;           // mixed form: this instance's retry flag
    double *TH;               // Householder leaves: per-leaf compact-WY factors (nullptr otherwise)
};

// phases of one orth_batch_step, in stream order
// (Householder leaves: the leaf Gram and correction form Q_k^T w through the
// compact-WY factor, BP_HPREP between them forms T^T M; the panel, the Gram
// of the new reflectors and the T update follow; BP_HCOEF and BP_HADDEC
// frame the finalize.  The FP64 and mixed leaves' Cholesky phases have no
// blocks there, and the H phases none for the other forms.)
enum BatchPhase {
    BP_LGRAM = 0, BP_HPREP, BP_LCHOL1,
    BP_LGRAMF, BP_LCHOLF,     // mixed form: the first sweep redone from the FP64 basis when flagged
    BP_LCORR, BP_HPANEL, BP_LGRAM2, BP_LCHOL2, BP_HTUPD,
    BP_RGRAM, BP_RRED1, BP_RCHOL1, BP_RCORR, BP_RGRAM2, BP_RRED2, BP_RCHOL2,
    BP_RFIN, BP_HCOEF, BP_LFIN, BP_HADDEC, BP_COUNT
};
__host__ __device__ inline bool batch_hh_phase(int phase) {
    return phase == BP_HPREP || phase == BP_HPANEL || phase == BP_HTUPD || phase == BP_HCOEF || phase == BP_HADDEC;
}

struct BatchArgs {
    const BatchInst *inst;
    const int32_t *prefix;    // exclusive block prefix over instances, count + 1 entries
    int32_t count;
    int32_t step;             // call index: instance i works at k = step * s_i
    int32_t phase;
    int32_t two;              // 1: BCGS-PIP+ (two sweeps), 0: BCGS-PIP
    int32_t mixed;            // 1: the instances keep FP32 copies (the first leaf Gram reads them)
    int32_t hh;               // 1: Householder leaves (the instances' TH)
    const double *const *W;   // device array: instance i's W (n_i x s_i, ld n_i)
    double *const *U;         // device array: explicit new blocks
    double *const *Hess;      // device array: K_i x K_i column-major, block `step` gets [H; R]
    DevStatus *status;
};

// workgroups instance d needs in a phase of a given step (0: phase skipped)
__host__ __device__ inline int32_t batch_phase_blocks(const BatchInst &d, int phase, int step, int two) {
    const int32_t k = step * d.s, ncol = k + d.s;
    if (d.TH) {
        // Householder leaves: Q_k^T w only past the first call; the panel,
        // the new reflectors' Gram and the T update every call
        switch (phase) {
            case BP_LGRAM:
                return k > 0 ? make_leaf_geom(d.n, d.leaf_rows, d.p, d.cL).nchunks() * gram_col_groups(ncol, d.s) : 0;
            case BP_LGRAM2:
                return make_leaf_geom(d.n, d.leaf_rows, d.p, d.cL).nchunks() * gram_col_groups(ncol, d.s);
            case BP_HPREP:
                return k > 0 ? d.p : 0;
            case BP_LCORR:
                return k > 0 ? make_leaf_geom(d.n, d.leaf_rows, d.p, kBatchFinalChunk).nchunks() : 0;
            case BP_HPANEL:
            case BP_HTUPD:
            case BP_HCOEF:
            case BP_HADDEC:
                return d.p;
            case BP_LCHOL1:
            case BP_LCHOL2:
            case BP_LGRAMF:
            case BP_LCHOLF:
                return 0;
            default:
                break;            // the reduction level and the finalize as below
        }
    } else if (batch_hh_phase(phase)) {
        return 0;
    }
    const bool second = phase == BP_LGRAM2 || phase == BP_LCHOL2 || phase == BP_RGRAM2 ||
                        phase == BP_RRED2 || phase == BP_RCHOL2;
    if (second && !two) return 0;
    switch (phase) {
        case BP_LGRAMF:
            if (!d.Qhi) return 0;
            [[fallthrough]];
        case BP_LGRAM:
        case BP_LGRAM2:
            return make_leaf_geom(d.n, d.leaf_rows, d.p, d.cL).nchunks() * gram_col_groups(ncol, d.s);
        case BP_LCHOLF:
            if (!d.Qhi) return 0;
            [[fallthrough]];
        case BP_LCHOL1:
        case BP_LCHOL2:
            return d.p;
        case BP_LCORR:
        case BP_LFIN:
            return make_leaf_geom(d.n, d.leaf_rows, d.p, kBatchFinalChunk).nchunks();
        case BP_RGRAM:
        case BP_RGRAM2:
            return make_root_geom(d.p, d.kmax, ncol, d.cR).nchunks() * gram_col_groups(ncol, d.s);
        case BP_RRED1:
        case BP_RRED2: {
            const int32_t slots = make_root_geom(d.p, d.kmax, ncol, d.cR).nchunks() * gram_row_groups(ncol);
            if (slots <= kReduceGroup) return 0;
            return (int32_t)(ceil_div64((int64_t)ncol * d.s, kThreads) * ceil_div64(slots, kReduceGroup));
        }
        case BP_RCHOL1:
        case BP_RCHOL2:
            return 1;
        case BP_RCORR:
        case BP_RFIN:
            return make_root_geom(d.p, d.kmax, ncol, kRootRowChunk).nchunks();
    }
    return 0;
}

#if defined(__HIPCC__)
// The batched kernels: workgroup b belongs to the instance whose block range
// [prefix[i], prefix[i+1]) holds b; its index within that range is `local`.
__device__ __forceinline__ void batch_locate(const BatchArgs &a, int &inst, int &local) {
    __shared__ int32_t found[2];
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    for (int i = tid; i < a.count; i += (int)blockDim.x)
        if (a.prefix[i] <= b && b < a.prefix[i + 1]) {
            found[0] = i;
            found[1] = b - a.prefix[i];
        }
    __syncthreads();
    inst = found[0];
    local = found[1];
}
#endif

// launchers (orth_kernels.hip)
hipError_t launch_gram(int s, const GramArgs &a, int cls, hipStream_t st);
hipError_t launch_reduce(const ReduceArgs &a, hipStream_t st);
hipError_t launch_chol(int s, const CholArgs &a, hipStream_t st);
hipError_t launch_finalize(int s, const FinalizeArgs &a, int cls, hipStream_t st);
// once per handle, on its device: raise the dynamic-LDS limit of the kernels
// a block width s uses beyond 64 KB
hipError_t prepare_kernels(int s);
hipError_t launch_apply(const ApplyArgs &a, hipStream_t st);
hipError_t launch_fill(double *p, int64_t count, double v, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t st);
hipError_t launch_copy_cols(const double *src, int64_t lds, RowMap smap, double *dst,
                            int64_t ldd, int64_t rows, int32_t cols, hipStream_t st);
// dst (column-major, ldd) <- the first `cols` columns of a leaf-blocked
// operand over the level's rows
hipError_t launch_copy_leafblk(const Operand &src, const LevelGeom &g, double *dst, int64_t ldd, int32_t cols,
                               hipStream_t st);
// rec[i rec_seg + c 2s + s + j] = src[i seg_rows + c + j ld] for i < nseg,
// c < rows, j < s (the right halves of per-leaf [. | C_i] records)
hipError_t launch_rows_to_records(const double *src, int64_t ld, int32_t nseg, int64_t seg_rows, int32_t rows,
                                 int32_t s, double *rec, int64_t rec_seg, hipStream_t st);
hipError_t launch_laplacian(const double *X, int64_t ldx, double *Y, int64_t ldy, int32_t s,
                            int32_t nx, int32_t ny, int32_t nz, double shift, hipStream_t st);
hipError_t launch_copy(const double *src, double *dst, int64_t count, hipStream_t st);
hipError_t launch_synth(double *W, int64_t ld, int64_t n, int32_t s, uint64_t seed, hipStream_t st);
// one phase for the instances of block width s (prefix table restricted to them)
hipError_t launch_batch_phase(const BatchArgs &a, int s, int32_t blocks, size_t lds, hipStream_t st);
// dynamic LDS one launch of a phase for width s needs; rowlds: the leaf row
// updates of s >= 16 run LDS-staged (every instance of the width has even
// leaf heights)
size_t batch_phase_lds(int phase, int s, bool rowlds);
// the Householder phases (orth_hh.hip): one launch for the instances of
// width s (all at k = step * s, which sizes the LDS staging)
hipError_t launch_batch_hh_phase(const BatchArgs &a, int s, int32_t blocks, hipStream_t st);


}  // namespace orth
