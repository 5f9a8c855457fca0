// gfx950 kernels of the TreeTSPQR step (Sec. 4.1) with BCGS-PIP+ leaves and
// reduction (Sec. 3.1).  FP64 throughout.
//
// One level (the leaves, or the reduction problem on the stacked leaf
// coefficient blocks) runs four kinds of kernels:
//
//   k_gram      sweep-1 Gram "at once" (Algorithm BCGS-PIP, first line): per
//               row chunk the partial [Q X]^T X, i.e. P1 = Q^T X and
//               G1 = X^T X in one pass over the rows.
//   k_chol      per leaf: fixed-order sum of the chunk partials, the s x s
//               Cholesky factor N of G - P^T P and its inverse; after the
//               second sweep also the combination P = P1 + P2 N1, N = N2 N1.
//   k_rowmfma   per row: the correction u1 = (x - q P1) N1^{-1} of
//               BCGS-PIP+ (its third line), whose sweep-2 Gram [Q U1]^T U1 is
//               then k_gram again; and the finalize u = (u1 - q P2) N2^{-1}
//               appended to the level's local basis, at the leaf level
//               together with the explicit new block
//               U|_i = [Q_i U_i] [P~_i; N~_i] (Sec. 4.1, assembly of U).
//
// Layout: every operand is column-major; rows are streamed with coalesced
// column reads straight into the matrix-core operands (the Gram products
// take rows as the contraction index, the row updates take them as the
// output index of a transposed product).  For blocks of 16 and more
// columns the leaf-level row update (k_rowlds) stages its basis and
// coefficient operands in LDS through direct loads instead, so that enough
// bytes stay in flight while the matrix cores, busier at those widths, work.
// No floating-point atomics: every sum has a fixed order.

#include "orth_internal.h"

namespace orth {

namespace {


typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bool failed(const DevStatus *st) { return st->code != 0; }

// One 16x16x4 FP64 matrix-core product D += A B.  Lane roles (gfx950):
// A[i][kk] is held by lane i + 16 kk, B[kk][j] by lane j + 16 kk, and
// D[i][j] by lane j + 16 (i % 4) in accumulator register i / 4.
__device__ __forceinline__ dbl4 mfma16(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ dbl4 zero4() { return dbl4{0.0, 0.0, 0.0, 0.0}; }

// R consecutive doubles / floats (as FP64) starting at p, vector loads when
// 16-byte aligned
template <int R>
__device__ __forceinline__ void load_run(const double *p, double (&v)[R]) {
    if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
#pragma unroll
        for (int u = 0; u < R / 2; ++u) {
            const double2 w = reinterpret_cast<const double2 *>(p)[u];
            v[2 * u] = w.x;
            v[2 * u + 1] = w.y;
        }
    } else {
#pragma unroll
        for (int u = 0; u < R; ++u) v[u] = p[u];
    }
}

template <int R>
__device__ __forceinline__ void load_run(const float *p, double (&v)[R]) {
    if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
#pragma unroll
        for (int u = 0; u < R / 4; ++u) {
            const float4 w = reinterpret_cast<const float4 *>(p)[u];
            v[4 * u] = w.x;
            v[4 * u + 1] = w.y;
            v[4 * u + 2] = w.z;
            v[4 * u + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int u = 0; u < R; ++u) v[u] = p[u];
    }
}

// direct loads into LDS (global_load_lds_dwordx4 takes an LDS pointer)
typedef __attribute__((address_space(1))) void global_void;
typedef __attribute__((address_space(3))) void lds_void;

// Wait until at most n vector-memory operations of this wave are
// outstanding (n a multiple of the loads per stage, below 64).
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

template <int L, int NST>
__device__ __forceinline__ void wait_stage(int ahead) {
    // ahead: stages issued after the one needed (0 .. NST - 2)
    if constexpr (NST >= 4) { if (ahead >= 2) { wait_vm<2 * L>(); return; } }
    if constexpr (NST >= 3) { if (ahead >= 1) { wait_vm<L>(); return; } }
    wait_vm<0>();
}

typedef double dbl2v __attribute__((ext_vector_type(2)));

}  // namespace

// ---------------------------------------------------------------- sweep 1
// Partial [Q X]^T X of one row chunk on the matrix cores.  The columns of
// Z = [Q X] are cut into 16-column tiles; a wave owns up to gram_tpw(s) tiles
// and one N tile per 16 columns of X.  The contraction runs over rows: in a
// macro-step of 32 rows, lane group kk = lane/16 feeds rows r + 8 kk + t to
// the t-th of 8 back-to-back products, so every lane streams 8 consecutive
// rows (64 contiguous bytes) of one column straight from HBM; no LDS.
// When the tiles do not fill all waves, the spare waves take other
// macro-steps of the chunk (row groups) and write their own partial slots.
// CLS (the launch site's profiler class) only names the instantiation, so a
// kernel trace attributes every dispatch to its role.
// rows per lane and column in one macro-step of the Gram kernel: RPL
// consecutive rows per lane give each column a contiguous run of 32 RPL bytes
// per wave
template <int S>
__host__ __device__ constexpr int gram_rpl() { return 8; }

// TZ (the reduction level): the basis is the stacked tree factor, whose
// column c holds zeros below segment row (c / s + 1) s (it was written when
// each segment had that many rows, and the rest was zero-filled at create).
// Those entries are taken as zeros without being read.
template <int S, bool TZ = false>
__device__ __forceinline__ void gram_body(const GramArgs &a, int bx, int by) {
    if (failed(a.status) || (a.cond && *a.retry == 0)) return;
    constexpr int NT = (S + 15) / 16;
    constexpr int RPL = gram_rpl<S>();
    constexpr int MS = 4 * RPL;                 // rows per macro-step
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int il = lane & 15, g = lane >> 4;
    const int k = a.k, ncol = k + S;
    const int TG = a.tile_groups, RG = kWaves / TG;
    const int tg = by * TG + wave % TG;
    const int rg = wave / TG;
    constexpr int TPW = gram_tpw(S);
    int tile0, ntl;
    gram_wave_tiles(ncol, S, tg, tile0, ntl);
    if (ntl <= 0) return;  // no columns for this wave (no barrier in this kernel)
    int leaf;
    int64_t r0, r1;
    a.geom.chunk(bx, leaf, r0, r1);
    const Operand Qv = leaf_view(a.Q, a.geom, leaf);    // the leaf's block of a blocked basis

    const double *colp[TPW];
    int cz[TPW];                                // TZ: segment rows of column c that can be nonzero
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int c = (tile0 + t) * 16 + il;
        colp[t] = t >= ntl ? nullptr
                           : (c < k ? Qv.ptr + (int64_t)c * Qv.ld
                                    : (c < ncol ? a.X.ptr + (int64_t)(c - k) * a.X.ld : nullptr));
        cz[t] = c < k ? (c / S + 1) * S : ncol;
    }
    const double *xcol[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int j = 16 * nt + il;
        xcol[nt] = j < S ? a.X.ptr + (int64_t)j * a.X.ld : nullptr;
    }
    dbl4 acc[TPW][NT];
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[t][nt] = zero4();

    const bool ident = a.geom.map.seg_len == 0;
    for (int64_t rm = r0 + MS * rg; rm < r1; rm += MS * RG) {
        double av[TPW][RPL], bv[NT][RPL];
        const int64_t rb = rm + RPL * g;
        // this lane's RPL rows are contiguous in memory: always at the leaf
        // level, and at the reduction level when they sit in one segment
        bool contig = rm + MS <= r1;
        int64_t pb = rb, rs = 0;
        if (!ident) {
            const int64_t q0 = rb / a.geom.map.seg_len;
            contig = contig && (rb + RPL - 1) / a.geom.map.seg_len == q0;
            rs = rb - q0 * a.geom.map.seg_len;
            pb = q0 * a.geom.map.seg_stride + rs;
        }
        if (contig) {
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                if (colp[t] && (!TZ || rs + RPL <= cz[t])) {
                    load_run<RPL>(colp[t] + pb, av[t]);
                } else if (TZ && S % RPL != 0 && colp[t] && rs < cz[t]) {
                    // a run across the bound (only when s < RPL: otherwise runs and
                    // bounds are both multiples of RPL within the segment)
#pragma unroll
                    for (int u = 0; u < RPL; ++u) av[t][u] = rs + u < cz[t] ? colp[t][pb + u] : 0.0;
                } else {
#pragma unroll
                    for (int u = 0; u < RPL; ++u) av[t][u] = 0.0;
                }
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                if (xcol[nt]) {
                    load_run<RPL>(xcol[nt] + pb, bv[nt]);
                } else {
#pragma unroll
                    for (int u = 0; u < RPL; ++u) bv[nt][u] = 0.0;
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < RPL; ++u) {
                const int64_t row = rb + u;
                const bool ok = row < r1;
                const int64_t prow = a.geom.map.phys(ok ? row : r0);
                const int64_t srow = TZ ? row % a.geom.map.seg_len : 0;
#pragma unroll
                for (int t = 0; t < TPW; ++t)
                    av[t][u] = (ok && colp[t] && (!TZ || srow < cz[t])) ? colp[t][prow] : 0.0;
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) bv[nt][u] = (ok && xcol[nt]) ? xcol[nt][prow] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < RPL; ++u)
#pragma unroll
            for (int t = 0; t < TPW; ++t)
                if (t < ntl)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) acc[t][nt] = mfma16(av[t][u], bv[nt][u], acc[t][nt]);
    }
    double *out = a.partials + ((int64_t)bx * RG + rg) * a.part_stride;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        if (t >= ntl) break;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int j = 16 * nt + il;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = (tile0 + t) * 16 + 4 * v + g;
                if (c < ncol && j < S) out[(int64_t)c * S + j] = acc[t][nt][v];
            }
        }
    }
}

template <int S, int CLS>
__global__ __launch_bounds__(kThreads) void k_gram(GramArgs a) {
    gram_body<S, CLS == 3 || CLS == 10>(a, blockIdx.x, blockIdx.y);   // reduction level: TZ
}

// The mixed form's sweep-1 Gram on the FP32 matrix cores
// (v_mfma_f32_16x16x4f32).  The basis columns come from the FP32 copy; X is
// read in FP64 and rounded to FP32 in registers, so every product operand
// is an FP32 number and P1 = Q^T X, G1 = X^T X carry relative errors of a
// few FP32 units (about 1e-7): the first CholeskyQR sweep only has to leave
// u1 nearly orthogonal, and the second sweep, in FP64, wins the accuracy
// back (Sec. 3.1).  The FP32 accumulators are promoted to FP64 after every
// macro-step (RPL products of 4 rows each), so rounding grows with the
// macro-step, not with the leaf height.  Same tiles, slots and launch shape
// as gram_body; each lane takes 16 consecutive rows per column.
// Lane roles of the FP32 product (gfx950): A[i][kk] at lane i + 16 kk,
// B[kk][j] at lane j + 16 kk, D[i][j] at lane j + 16 (i / 4), register i % 4.
typedef float flt4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ flt4 mfma16f(float a, float b, flt4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int R>
__device__ __forceinline__ void load_run_f(const float *p, float (&v)[R]) {
    if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
#pragma unroll
        for (int u = 0; u < R / 4; ++u) {
            const float4 w = reinterpret_cast<const float4 *>(p)[u];
            v[4 * u] = w.x;
            v[4 * u + 1] = w.y;
            v[4 * u + 2] = w.z;
            v[4 * u + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int u = 0; u < R; ++u) v[u] = p[u];
    }
}

template <int R>
__device__ __forceinline__ void load_run_f(const double *p, float (&v)[R]) {
    double d[R];
    load_run<R>(p, d);
#pragma unroll
    for (int u = 0; u < R; ++u) v[u] = (float)d[u];
}

template <int S>
__device__ __forceinline__ void gram_f32_body(const GramArgs &a, int bx, int by) {
    if (a.clear_retry && bx == 0 && by == 0 && threadIdx.x == 0) *a.retry = 0;
    if (failed(a.status)) return;
    constexpr int NT = (S + 15) / 16;
    constexpr int RPL = 16;                    // 64 contiguous bytes of the copy per lane and column
    constexpr int MS = 4 * RPL;                 // rows per macro-step
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int il = lane & 15, g = lane >> 4;
    const int k = a.k, ncol = k + S;
    const int TG = a.tile_groups, RG = kWaves / TG;
    const int tg = by * TG + wave % TG;
    const int rg = wave / TG;
    constexpr int TPW = gram_tpw(S);
    int tile0, ntl;
    gram_wave_tiles(ncol, S, tg, tile0, ntl);
    if (ntl <= 0) return;
    int leaf;
    int64_t r0, r1;
    a.geom.chunk(bx, leaf, r0, r1);
    const float *qhi = leaf_view_hi(a.Qhi, a.Q, a.geom, leaf);   // the leaf's block of the copy
    const int64_t qld = leaf_view(a.Q, a.geom, leaf).ld;

    const float *colh[TPW];
    const double *colp[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int c = (tile0 + t) * 16 + il;
        colh[t] = (t < ntl && c < k) ? qhi + (int64_t)c * qld : nullptr;
        colp[t] = (t < ntl && c >= k && c < ncol) ? a.X.ptr + (int64_t)(c - k) * a.X.ld : nullptr;
    }
    const double *xcol[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int j = 16 * nt + il;
        xcol[nt] = j < S ? a.X.ptr + (int64_t)j * a.X.ld : nullptr;
    }
    double acc[TPW][NT][4];
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[t][nt][v] = 0.0;

    const bool ident = a.geom.map.seg_len == 0;
    for (int64_t rm = r0 + MS * rg; rm < r1; rm += MS * RG) {
        float av[TPW][RPL], bv[NT][RPL];
        const int64_t rb = rm + RPL * g;
        if (ident && rm + MS <= r1) {
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                if (colh[t]) {
                    load_run_f<RPL>(colh[t] + rb, av[t]);
                } else if (colp[t]) {
                    load_run_f<RPL>(colp[t] + rb, av[t]);
                } else {
#pragma unroll
                    for (int u = 0; u < RPL; ++u) av[t][u] = 0.0f;
                }
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                if (xcol[nt]) {
                    load_run_f<RPL>(xcol[nt] + rb, bv[nt]);
                } else {
#pragma unroll
                    for (int u = 0; u < RPL; ++u) bv[nt][u] = 0.0f;
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < RPL; ++u) {
                const int64_t row = rb + u;
                const bool ok = row < r1;
                const int64_t prow = a.geom.map.phys(ok ? row : r0);
#pragma unroll
                for (int t = 0; t < TPW; ++t)
                    av[t][u] = !ok ? 0.0f : (colh[t] ? colh[t][prow] : (colp[t] ? (float)colp[t][prow] : 0.0f));
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) bv[nt][u] = (ok && xcol[nt]) ? (float)xcol[nt][prow] : 0.0f;
            }
        }
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            if (t >= ntl) continue;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                flt4 d = flt4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int u = 0; u < RPL; ++u) d = mfma16f(av[t][u], bv[nt][u], d);
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[t][nt][v] += (double)d[v];
            }
        }
    }
    double *out = a.partials + ((int64_t)bx * RG + rg) * a.part_stride;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        if (t >= ntl) break;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int j = 16 * nt + il;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = (tile0 + t) * 16 + 4 * g + v;
                if (c < ncol && j < S) out[(int64_t)c * S + j] = acc[t][nt][v];
            }
        }
    }
}

template <int S>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_gram_hi(GramArgs a) {
    gram_f32_body<S>(a, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------- reduce
// Fixed-order pre-sum of groups of partial slots (one thread per entry).
__device__ __forceinline__ void reduce_body(const ReduceArgs &a, int bx, int by) {
    if (failed(a.status) || (a.cond && *a.retry == 0)) return;
    const int e = bx * kThreads + threadIdx.x;
    if (e >= a.nentries) return;
    const int grp = by;
    const int s0 = grp * a.group;
    const int s1 = s0 + a.group < a.nslots ? s0 + a.group : a.nslots;
    const double v = slot_sum(a.in + (int64_t)s0 * a.stride + e, a.stride, s1 - s0);
    a.out[(int64_t)grp * a.stride + e] = v;
}

__global__ __launch_bounds__(kThreads) void k_reduce(ReduceArgs a) { reduce_body(a, blockIdx.x, blockIdx.y); }

// ---------------------------------------------------------------- Cholesky
// Per leaf: sum the leaf's partial Gram slots in slot order, store P to the
// leaf record, form G - P^T P in row chunks staged through LDS, factor it
// (right-looking upper Cholesky, lane j owns column j), invert the factor by
// back substitution, and after the final sweep combine the sweeps and write
// [P; N] to the next level (or H and R at the root).
constexpr int kCholCB = 64;   // P rows per LDS chunk

// A failed pivot: the first failure wins the status record (the breakdown),
// or, for the mixed form's first sweep on the FP32 copy (soft), the step is
// flagged for the FP64 redo of that sweep instead.
__device__ __forceinline__ void chol_fail(const CholArgs &a, int leaf, int column) {
    if (a.soft) {
        *a.retry = 1;
        return;
    }
    if (atomicCAS(&a.status->code, 0, 3) == 0) {
        a.status->level = a.level;
        a.status->leaf = leaf;
        a.status->sweep = a.sweep;
        a.status->column = column;
        a.status->instance = a.instance;
    }
}

// blocks of 16 and more columns: the wide form below
__host__ __device__ constexpr size_t chol_lds_bytes_s(int s) {
    return s >= 16 ? (size_t)9 * s * s * 8 + 16 : ((size_t)5 * s * s + (size_t)kCholCB * s) * 8 + 16;
}
template <int S>
__host__ __device__ constexpr size_t chol_lds_bytes() { return chol_lds_bytes_s(S); }

// a double from lane l (l wave-uniform)
__device__ __forceinline__ double readlane_d(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Steps 3-4 of the per-leaf Cholesky: N^T N = sm (upper, right-looking) and
// N^{-1}, in one wave: lane j < S owns column j in registers and the pivot
// row is broadcast with readlane, so no step needs a workgroup barrier.
// Returns false after recording a failed pivot (then nm and ni are not set).
template <int S>
__device__ __forceinline__ bool chol_factor_one_wave(const CholArgs &a, int leaf, const double *sm, double *nm,
                                                     double *ni, int &bad, int wave, int lane, int tid) {
    if (wave == 0) {
        const int j = lane;
        const bool own = j < S;
        double col[S];
#pragma unroll
        for (int i = 0; i < S; ++i) col[i] = own ? sm[i * S + j] : 0.0;
        int fail = 0;
#pragma unroll
        for (int kk = 0; kk < S; ++kk) {
            const double piv = readlane_d(col[kk], kk);
            if (!(piv > 0.0) || !isfinite(piv)) { fail = kk + 1; break; }
            const double nkk = sqrt(piv);
            const double r = j == kk ? nkk : (j > kk && own ? col[kk] / nkk : 0.0);   // N[kk][j]
            col[kk] = r;
#pragma unroll
            for (int i = kk + 1; i < S; ++i) {
                const double ri = readlane_d(r, i);                                   // N[kk][i]
                if (j >= i && own) col[i] -= ri * r;
            }
        }
        if (fail) {
            if (lane == 0) bad = fail;
        } else if (own) {
#pragma unroll
            for (int i = 0; i < S; ++i) {
                if (i > j) col[i] = 0.0;
                nm[i * S + j] = col[i];
            }
        }
    }
    __syncthreads();
    if (bad) {
        if (tid == 0) chol_fail(a, leaf, bad - 1);
        return false;
    }
    if (a.cond && leaf == 0 && tid == 0) atomicAdd(&a.status->fallbacks, 1);
    if (wave == 0 && lane < S) {
        // back substitution N x = e_j, x[l] = 0 past j; the rows of N are read
        // by every lane at once (LDS broadcast)
        const int j = lane;
        double x[S];
#pragma unroll
        for (int i = S - 1; i >= 0; --i) {
            double t = 0.0;
#pragma unroll
            for (int l = i + 1; l < S; ++l) t = fma(nm[i * S + l], x[l], t);
            x[i] = i > j ? 0.0 : (i == j ? 1.0 / nm[i * S + i] : -t / nm[i * S + i]);
        }
#pragma unroll
        for (int i = 0; i < S; ++i) ni[i * S + j] = x[i];
    }
    __syncthreads();
    return true;
}

// The same steps for s = 16, 32 with the two products whose length grows with
// k on the matrix cores: P^T P (the four waves take interleaved 4-row steps
// and their partial sums are added in wave order) and, after the second
// sweep, P = P1 + P2 N1 (16-row tiles over the waves).  The factorisation and
// the inverse run in one wave, lane j holding column j in registers: the
// pivot row is broadcast with readlane, so no step needs a workgroup barrier.
template <int S>
__device__ __forceinline__ void chol_wide_body(const CholArgs &a, int bx) {
    static_assert(S == 16 || S == 32, "wide blocks only");
    constexpr int NT = S / 16;
    if (failed(a.status) || (a.cond && *a.retry == 0)) return;
    extern __shared__ double lds[];
    double *gs = lds, *sm = gs + S * S, *nm = sm + S * S, *ni = nm + S * S, *n1 = ni + S * S;
    double *part = n1 + S * S;                                // 4 x S x S partial sums of P^T P
    int &bad = *reinterpret_cast<int *>(part + 4 * S * S);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int il = lane & 15, g = lane >> 4;
    const int leaf = bx;
    const int k = a.k, ncol = k + S;
    if (tid == 0) bad = 0;
    double *rec = a.small + (int64_t)leaf * a.small_stride;
    double *recP1 = rec;
    double *recN1 = rec + (int64_t)a.kmax * S;
    double *recN1i = recN1 + S * S;
    double *recP2 = recN1i + S * S;
    double *recN2i = recP2 + (int64_t)a.kmax * S;
    double *recP = a.sweep == 1 ? recP1 : recP2;

    // 1. fixed-order slot sum: P -> leaf record, G -> LDS
    const int first = leaf * a.slots_per_leaf;
    const int cnt = leaf == a.nleaf - 1 ? a.slots_last : a.slots_per_leaf;
    for (int e = tid; e < ncol * S; e += kThreads) {
        const double v = slot_sum(a.partials + (int64_t)first * a.part_stride + e, a.part_stride, cnt);
        if (e < k * S) {
            recP[e] = v;
            if (a.pc && a.sweep == 2) a.pc[(int64_t)leaf * a.pc_stride + (int64_t)(e / S) * 2 * S + e % S] = v;
        }
        else gs[e - k * S] = v;
    }
    if (a.sweep == 2 && a.final_sweep == 2)
        for (int e = tid; e < S * S; e += kThreads) n1[e] = recN1[e];
    __syncthreads();

    // 2. P^T P: A[i][kk] = P[c][16 ti + i], B[kk][j] = P[c][16 tj + j] for the
    //    rows c = c0 + kk of one 4-row step
    {
        dbl4 pp[NT][NT];
#pragma unroll
        for (int ti = 0; ti < NT; ++ti)
#pragma unroll
            for (int tj = 0; tj < NT; ++tj) pp[ti][tj] = zero4();
        for (int c0 = 4 * wave; c0 < k; c0 += 4 * kWaves) {
            const int c = c0 + g;
            double pv[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) pv[t] = c < k ? recP[(int64_t)c * S + 16 * t + il] : 0.0;
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int tj = 0; tj < NT; ++tj) pp[ti][tj] = mfma16(pv[ti], pv[tj], pp[ti][tj]);
        }
        double *pw = part + wave * S * S;
#pragma unroll
        for (int ti = 0; ti < NT; ++ti)
#pragma unroll
            for (int tj = 0; tj < NT; ++tj)
#pragma unroll
                for (int v = 0; v < 4; ++v) pw[(16 * ti + 4 * v + g) * S + 16 * tj + il] = pp[ti][tj][v];
    }
    __syncthreads();
    for (int e = tid; e < S * S; e += kThreads)
        sm[e] = gs[e] - (((part[e] + part[S * S + e]) + part[2 * S * S + e]) + part[3 * S * S + e]);
    __syncthreads();

    // 3-4. N^T N = sm (upper) and N^{-1}, one wave, lane j < S owns column j
    if (!chol_factor_one_wave<S>(a, leaf, sm, nm, ni, bad, wave, lane, tid)) return;
    if (a.sweep == 1) {
        for (int e = tid; e < S * S; e += kThreads) { recN1[e] = nm[e]; recN1i[e] = ni[e]; }
    } else {
        for (int e = tid; e < S * S; e += kThreads) recN2i[e] = ni[e];
    }
    if (a.sweep != a.final_sweep) return;

    // 5. [P; N] of this leaf
    const int64_t ybase = (int64_t)leaf * a.yseg;
    auto put = [&](int c, int jj, double v) {
        if (a.Yout) a.Yout[(int64_t)jj * a.ldy + ybase + c] = v;
        if (c < k) {
            if (a.H) a.H[(int64_t)jj * a.ldh + c] = v;
        } else if (a.R) {
            a.R[(int64_t)jj * a.ldr + (c - k)] = v;
        }
    };
    if (a.sweep == 1) {
        for (int e = tid; e < ncol * S; e += kThreads) {
            const int c = e / S, jj = e % S;
            put(c, jj, c < k ? recP1[e] : nm[(c - k) * S + jj]);
        }
        return;
    }
    // P = P1 + P2 N1: A[ci][kk] = P2[16 rt + ci][4 ks + kk], B[kk][j] = N1[4 ks + kk][16 tj + j]
    for (int rt = wave; 16 * rt < k; rt += kWaves) {
#pragma unroll
        for (int tj = 0; tj < NT; ++tj) {
            dbl4 d = zero4();
#pragma unroll
            for (int ks = 0; ks < S / 4; ++ks)
                d = mfma16(recP2[(int64_t)(16 * rt + il) * S + 4 * ks + g], n1[(4 * ks + g) * S + 16 * tj + il], d);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = 16 * rt + 4 * v + g, jj = 16 * tj + il;
                put(c, jj, recP1[(int64_t)c * S + jj] + d[v]);
            }
        }
    }
    // N = N2 N1
    for (int e = tid; e < S * S; e += kThreads) {
        const int i = e / S, jj = e % S;
        double v = 0.0;
        for (int l = i; l <= jj; ++l) v = fma(nm[i * S + l], n1[l * S + jj], v);
        put(k + i, jj, v);
    }
}

template <int S>
__device__ __forceinline__ void chol_narrow_body(const CholArgs &a, int bx) {
    if (failed(a.status) || (a.cond && *a.retry == 0)) return;
    constexpr int EPT = (S * S + kThreads - 1) / kThreads;   // S x S entries per thread
    extern __shared__ double lds[];
    double *gs = lds, *sm = gs + S * S, *nm = sm + S * S, *ni = nm + S * S, *n1 = ni + S * S;
    double *pc = n1 + S * S;                                  // kCholCB x S
    int &bad = *reinterpret_cast<int *>(pc + kCholCB * S);
    const int tid = threadIdx.x;
    const int leaf = bx;
    const int k = a.k, ncol = k + S;
    if (tid == 0) bad = 0;
    double *rec = a.small + (int64_t)leaf * a.small_stride;
    double *recP1 = rec;
    double *recN1 = rec + (int64_t)a.kmax * S;
    double *recN1i = recN1 + S * S;
    double *recP2 = recN1i + S * S;
    double *recN2i = recP2 + (int64_t)a.kmax * S;
    double *recP = a.sweep == 1 ? recP1 : recP2;

    // 1. fixed-order slot sum: P -> leaf record, G -> LDS (and P too when it
    //    fits one LDS chunk: step 2 then reads no global memory)
    const int first = leaf * a.slots_per_leaf;
    const int cnt = leaf == a.nleaf - 1 ? a.slots_last : a.slots_per_leaf;
    const bool p_in_lds = k <= kCholCB;
    for (int e = tid; e < ncol * S; e += kThreads) {
        const double v = slot_sum(a.partials + (int64_t)first * a.part_stride + e, a.part_stride, cnt);
        if (e < k * S) {
            recP[e] = v;
            if (p_in_lds) pc[e] = v;
            if (a.pc && a.sweep == 2) a.pc[(int64_t)leaf * a.pc_stride + (int64_t)(e / S) * 2 * S + e % S] = v;
        }
        else gs[e - k * S] = v;
    }
    if (a.sweep == 2 && a.final_sweep == 2)
        for (int e = tid; e < S * S; e += kThreads) n1[e] = recN1[e];
    __syncthreads();
    // 2. sm = G - P^T P, P streamed through LDS in row chunks
    double d[EPT];
#pragma unroll
    for (int m = 0; m < EPT; ++m) d[m] = 0.0;
    for (int c0 = 0; c0 < k; c0 += kCholCB) {
        const int cb = (k - c0) < kCholCB ? (k - c0) : kCholCB;
        if (!p_in_lds) {
            for (int e = tid; e < cb * S; e += kThreads) pc[e] = recP[(int64_t)c0 * S + e];
            __syncthreads();
        }
#pragma unroll
        for (int m = 0; m < EPT; ++m) {
            const int e = tid + kThreads * m;
            if (e < S * S) {
                const int i = e / S, j = e % S;
                for (int c = 0; c < cb; ++c) d[m] = fma(pc[c * S + i], pc[c * S + j], d[m]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
        const int e = tid + kThreads * m;
        if (e < S * S) {
            sm[e] = gs[e] - d[m];
            nm[e] = 0.0;
            ni[e] = 0.0;
        }
    }
    __syncthreads();
    // 3-4. N^T N = sm and N^{-1} in one wave (as for the wide blocks)
    {
        const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        if (!chol_factor_one_wave<S>(a, leaf, sm, nm, ni, bad, wave, lane, tid)) return;
    }
    if (a.sweep == 1) {
        for (int e = tid; e < S * S; e += kThreads) { recN1[e] = nm[e]; recN1i[e] = ni[e]; }
    } else {
        for (int e = tid; e < S * S; e += kThreads) recN2i[e] = ni[e];
    }
    if (a.sweep != a.final_sweep) return;
    // 5. [P; N] of this leaf: one sweep -> (P1, N1); two sweeps ->
    //    P = P1 + P2 N1, N = N2 N1 (the reiteration combination)
    const int64_t ybase = (int64_t)leaf * a.yseg;
    for (int e = tid; e < ncol * S; e += kThreads) {
        const int c = e / S, j = e % S;
        double v;
        if (c < k) {
            v = recP1[e];
            if (a.sweep == 2)
                for (int i = 0; i <= j; ++i) v = fma(recP2[c * S + i], n1[i * S + j], v);
        } else {
            const int i = c - k;
            if (a.sweep == 1) {
                v = nm[i * S + j];
            } else {
                v = 0.0;
                for (int l = i; l <= j; ++l) v = fma(nm[i * S + l], n1[l * S + j], v);
            }
        }
        if (a.Yout) a.Yout[(int64_t)j * a.ldy + ybase + c] = v;
        if (c < k) {
            if (a.H) a.H[(int64_t)j * a.ldh + c] = v;
        } else if (a.R) {
            a.R[(int64_t)j * a.ldr + (c - k)] = v;
        }
    }
}

template <int S>
__device__ __forceinline__ void chol_body(const CholArgs &a, int bx) {
    if constexpr (S >= 16) {
        chol_wide_body<S>(a, bx);
    } else {
        chol_narrow_body<S>(a, bx);
    }
}

template <int S>
__global__ __launch_bounds__(kThreads) void k_chol(CholArgs a) { chol_body<S>(a, blockIdx.x); }

// ---------------------------------------------------------------- row update
// Two uses of one kernel:
//   sweep 1 (correction):  u1 = (x - q P1) N1^{-1}            -> U1 scratch
//   sweep 2 (finalize):    u  = (u1 - q P2) N2^{-1}           -> new basis columns
//                          and, with EXPL, the explicit block
//                          U|_i = q P~_i + u N~_i  (C = [P~_i; N~_i]).
constexpr int kRowCB = 64;   // coefficient rows per LDS block of k_apply

// On the matrix cores.  A wave owns blocks of 16 TR rows; lane
// (il = lane % 16, g = lane / 16) streams TR rows (lane_row) of basis column
// c0 + g, the B operand of TR transposed products Y^T += Coef^T Q^T over 4
// columns at a time.  Output column m of the coefficient block
// [P | C_top] is the row index of each product, so a lane's accumulators
// hold one row (lane_row(rb, il, t)) and the
// columns m = 16 T + 4 v + g (tile T, register v).  That is exactly the
// B-operand layout of a further product over m: the per-row triangular
// factor u = (x - q P) N^{-1} and the explicit block's u C_bot term
// also run on the matrix cores, with no exchange of data between lanes
// and no LDS.  The coefficients are read through the cache (they are the
// same for every row of a leaf).
// A lane's TR rows of a block: pairs 2 il, 2 il + 1 in each 32-row slice,
// so one 16-byte access per lane covers 256 contiguous bytes per column.
__device__ __forceinline__ int64_t lane_row(int64_t rb, int il, int t) {
    return rb + 32 * (t >> 1) + 2 * il + (t & 1);
}

template <int TR>
__device__ __forceinline__ void load_rows(const double *p, double (&v)[TR]) {   // p: row rb + 2 il
    if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
#pragma unroll
        for (int u = 0; u < TR / 2; ++u) {
            const double2 w = *reinterpret_cast<const double2 *>(p + 32 * u);
            v[2 * u] = w.x;
            v[2 * u + 1] = w.y;
        }
    } else {
#pragma unroll
        for (int u = 0; u < TR / 2; ++u) {
            v[2 * u] = p[32 * u];
            v[2 * u + 1] = p[32 * u + 1];
        }
    }
}

template <int TR>
__device__ __forceinline__ void store_rows(double *p, const double (&v)[TR]) {
    if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
#pragma unroll
        for (int u = 0; u < TR / 2; ++u) *reinterpret_cast<double2 *>(p + 32 * u) = double2{v[2 * u], v[2 * u + 1]};
    } else {
#pragma unroll
        for (int u = 0; u < TR / 2; ++u) {
            p[32 * u] = v[2 * u];
            p[32 * u + 1] = v[2 * u + 1];
        }
    }
}

// rows per lane of a block: eight for narrow blocks (64 bytes of a column
// per lane in flight), fewer where the accumulators of wide blocks would
// not leave room for two waves per SIMD
template <int S, bool EXPL>
__host__ __device__ constexpr int rowmfma_tr() { return S <= 8 ? 8 : ((S >= 32 && EXPL) ? 2 : 4); }
// 4-column steps whose loads are issued ahead of the products
template <int S, bool EXPL>
__host__ __device__ constexpr int rowmfma_pf() { return 1; }

// The end of a row block, once acc holds q [P | C_top] for the lane's TR
// rows: u = (x - q P) N^{-1} on the matrix cores, stored as new basis
// columns (and as C_i rows, or as the FP32 copy), then with EXPL the
// explicit block q C_top + u C_bot.
// A row update's arguments with the basis operands (Q, the new columns and
// their FP32 copy) narrowed to one leaf's block of a blocked basis.
__device__ __forceinline__ FinalizeArgs leaf_finalize_args(const FinalizeArgs &a_in, int leaf) {
    FinalizeArgs a = a_in;
    a.Q = leaf_view(a_in.Q, a_in.geom, leaf);
    a.Qnew = leaf_view(a_in.Qnew, a_in.geom, leaf);
    a.Qnew_hi = leaf_view_hi(a_in.Qnew_hi, a_in.Qnew, a_in.geom, leaf);
    return a;
}

template <int S, bool EXPL, int TR>
__device__ __forceinline__ void rowmfma_epilogue(const FinalizeArgs &a, int k, int64_t rb, bool fast,
                                                 const bool (&ok)[TR], const int64_t (&prow)[TR],
                                                 dbl4 (&acc)[TR][EXPL ? (2 * S + 15) / 16 : (S + 15) / 16],
                                                 const double *recNi, const double *cbase, bool ident_only) {
    constexpr int M = EXPL ? 2 * S : S;
    constexpr int NTM = (M + 15) / 16;
    constexpr int NTS = (S + 15) / 16;
    constexpr int NV = S < 4 ? 1 : 4;
    constexpr int KS = (S + 3) / 4;
    const int lane = threadIdx.x & 63;
    const int il = lane & 15, g = lane >> 4;
    const int64_t rl = rb + 2 * il;
    // x - q P for the block's columns j = 16 T + 4 v + g < S, the lane's
    // TR rows of column j read (and later written) as 16-byte pairs
    double tv[TR][NTS][4];
#pragma unroll
    for (int T = 0; T < NTS; ++T)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = 16 * T + 4 * v + g;
            double x[TR];
#pragma unroll
            for (int t = 0; t < TR; ++t) x[t] = 0.0;
            if (v < NV && j < S) {
                const double *col = a.U1.ptr + (int64_t)j * a.U1.ld;
                if (fast) {
                    load_rows<TR>(col + rl, x);
                } else {
#pragma unroll
                    for (int t = 0; t < TR; ++t) x[t] = ok[t] ? col[prow[t]] : 0.0;
                }
            }
#pragma unroll
            for (int t = 0; t < TR; ++t) tv[t][T][v] = (v < NV && j < S) ? x[t] - acc[t][T][v] : 0.0;
        }
    // u = (x - q P) N^{-1}: products over l = 4 ks + g (N^{-1} upper triangular)
    dbl4 uv[TR][NTS];
#pragma unroll
    for (int T = 0; T < NTS; ++T) {
        double an[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int l = 4 * ks + g, jo = 16 * T + il;
            an[ks] = 0.0;
            if (l < S && jo < S && l <= jo) an[ks] = ident_only ? (l == jo ? 1.0 : 0.0) : recNi[l * S + jo];
        }
#pragma unroll
        for (int t = 0; t < TR; ++t) {
            uv[t][T] = zero4();
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                if (4 * ks <= 16 * T + 15) uv[t][T] = mfma16(an[ks], tv[t][ks / 4][ks % 4], uv[t][T]);
        }
    }
#pragma unroll
    for (int T = 0; T < NTS; ++T)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int j = 16 * T + 4 * v + g;
            if (j >= S) continue;
            double y[TR];
#pragma unroll
            for (int t = 0; t < TR; ++t) y[t] = uv[t][T][v];
            double *col = a.Qnew.ptr + (int64_t)j * a.Qnew.ld;
            if (fast) {
                store_rows<TR>(col + rl, y);
            } else {
#pragma unroll
                for (int t = 0; t < TR; ++t)
                    if (ok[t]) col[prow[t]] = y[t];
            }
            if (!EXPL && a.Crow) {            // C_i rows for the leaf finalize
#pragma unroll
                for (int t = 0; t < TR; ++t)
                    if (ok[t]) {
                        const int64_t r = lane_row(rb, il, t);
                        const int64_t lf = r / a.geom.map.seg_len;
                        const int64_t cc = r - lf * a.geom.map.seg_len;
                        a.Crow[lf * a.crow_seg + cc * 2 * S + S + j] = y[t];
                    }
            }
            if (EXPL && a.Qnew_hi) {          // mixed form: FP32 copy for the next sweep-1 Gram
                float *ch = a.Qnew_hi + (int64_t)j * a.Qnew.ld;
                if (fast && (reinterpret_cast<uintptr_t>(ch + rl) & 7) == 0) {
                    // the lane's row pairs as 8-byte stores
#pragma unroll
                    for (int u = 0; u < TR / 2; ++u)
                        *reinterpret_cast<float2 *>(ch + rl + 32 * u) = float2{(float)y[2 * u], (float)y[2 * u + 1]};
                } else {
#pragma unroll
                    for (int t = 0; t < TR; ++t)
                        if (ok[t]) ch[prow[t]] = (float)y[t];
                }
            }
        }
    if (EXPL) {
        // U| = q C_top + u C_bot, C_bot = C rows k..k+S-1; rows are logical
#pragma unroll
        for (int T = 0; T < NTM; ++T) {
            if (16 * T + 15 < S) continue;        // tile without C columns
            double ac[KS];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int l = 4 * ks + g, m = 16 * T + il;
                ac[ks] = (l < S && m >= S && m < 2 * S) ? cbase[(int64_t)(k + l) * 2 * S + m] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < TR; ++t)
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) acc[t][T] = mfma16(ac[ks], uv[t][ks / 4][ks % 4], acc[t][T]);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = 16 * T + 4 * v + g;
                if (m < S || m >= 2 * S) continue;
                double y[TR];
#pragma unroll
                for (int t = 0; t < TR; ++t) y[t] = acc[t][T][v];
                if (a.Cout) {                 // tree level: the children's C records
#pragma unroll
                    for (int t = 0; t < TR; ++t)
                        if (ok[t]) {
                            const int64_t r = lane_row(rb, il, t);
                            const int64_t lf = r / a.geom.map.seg_len;
                            const int64_t cc = r - lf * a.geom.map.seg_len;
                            a.Cout[lf * a.cout_seg + cc * 2 * S + m] = y[t];
                        }
                    continue;
                }
                double *col = a.Uout.ptr + (int64_t)(m - S) * a.Uout.ld;
                if (fast) {
                    store_rows<TR>(col + rl, y);
                } else {
#pragma unroll
                    for (int t = 0; t < TR; ++t)
                        if (ok[t]) col[lane_row(rb, il, t)] = y[t];
                }
            }
        }
    }
}

// TZ (the reduction level): basis column c is zero below segment row
// (c / s + 1) s and is not read there (as in gram_body).
template <int S, bool EXPL, int TR, int PF, bool TZ = false>
__device__ __forceinline__ void rowmfma_body(const FinalizeArgs &a_in, int bx) {
    if (failed(a_in.status)) return;
    constexpr int RB = 16 * TR;              // rows per wave block
    constexpr int M = EXPL ? 2 * S : S;      // coefficient columns [P | C_top]
    constexpr int NTM = (M + 15) / 16;       // 16-column output tiles
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int il = lane & 15, g = lane >> 4;
    const int k = a_in.k;
    int leaf;
    int64_t r0, r1;
    a_in.geom.chunk(bx, leaf, r0, r1);
    const FinalizeArgs a = leaf_finalize_args(a_in, leaf);
    const double *rec = a.small + (int64_t)leaf * a.small_stride;
    // record: P1 [kmax][S] | N1 | N1^{-1} | P2 [kmax][S] | N2^{-1}
    const double *recP = a.sweep == 1 ? rec : rec + (int64_t)a.kmax * S + 2 * S * S;
    const double *recNi = a.sweep == 1 ? rec + (int64_t)a.kmax * S + S * S : recP + (int64_t)a.kmax * S;
    const bool ident_only = a.single_sweep != 0;   // u = u1 (one-sweep variant)
    // the explicit form's first S coefficient columns are zero then: at
    // s >= 16 they fill whole tiles, whose products are skipped (they would
    // add exact zeros)
    const bool skip_p = EXPL && S % 16 == 0 && ident_only;
    const double *cbase = EXPL ? a.Cptr + (int64_t)leaf * a.cseg : nullptr;
    const bool ident = a.geom.map.seg_len == 0;

    for (int64_t rb = r0 + RB * wave; rb < r1; rb += RB * kWaves) {
        const int64_t rl = rb + 2 * il;              // this lane's first row
        int64_t prow[TR];
        bool ok[TR];
        int srow[TR];                                // TZ: row within its segment
#pragma unroll
        for (int t = 0; t < TR; ++t) {
            const int64_t r = lane_row(rb, il, t);
            ok[t] = r < r1;
            prow[t] = a.geom.map.phys(ok[t] ? r : r0);
            srow[t] = TZ ? (int)(r % a.geom.map.seg_len) : 0;
        }
        const bool fast = ident && rb + RB <= r1;   // the lane's rows are contiguous and present
        dbl4 acc[TR][NTM];
#pragma unroll
        for (int t = 0; t < TR; ++t)
#pragma unroll
            for (int T = 0; T < NTM; ++T) acc[t][T] = zero4();

        // operands of the 4-column step at c0: the lane's TR rows of column
        // c0 + g and the coefficients of output columns 16 T + il (zero past k)
        auto fetch = [&](int c0, double (&q)[TR], double (&cf)[NTM]) {
            const int c = c0 + g;
#pragma unroll
            for (int t = 0; t < TR; ++t) q[t] = 0.0;
#pragma unroll
            for (int T = 0; T < NTM; ++T) cf[T] = 0.0;
            if (c < k) {
                const double *col = a.Q.ptr + (int64_t)c * a.Q.ld;
                if (fast) {
                    load_rows<TR>(col + rl, q);
                } else {
                    const int cz = (c / S + 1) * S;
#pragma unroll
                    for (int t = 0; t < TR; ++t) q[t] = (ok[t] && (!TZ || srow[t] < cz)) ? col[prow[t]] : 0.0;
                }
#pragma unroll
                for (int T = 0; T < NTM; ++T) {
                    const int m = 16 * T + il;
                    if (EXPL) {
                        // one load per column: [P2 | C] row c of the leaf's record
                        if (m < 2 * S) cf[T] = (m < S && ident_only) ? 0.0 : cbase[(int64_t)c * 2 * S + m];
                    } else if (m < S) {
                        cf[T] = ident_only ? 0.0 : recP[(int64_t)c * S + m];
                    }
                }
            }
        };
        // PF steps of prefetch: the loads of the next PF steps are in
        // flight while the matrix cores work on this one
        double qs[PF + 1][TR], cs[PF + 1][NTM];
#pragma unroll
        for (int p = 0; p < PF; ++p) fetch(4 * p, qs[p], cs[p]);
        for (int c0 = 0; c0 < k; c0 += 4) {
            fetch(c0 + 4 * PF, qs[PF], cs[PF]);
#pragma unroll
            for (int t = 0; t < TR; ++t)
#pragma unroll
                for (int T = 0; T < NTM; ++T)
                    if (!skip_p || T >= S / 16) acc[t][T] = mfma16(cs[0][T], qs[0][t], acc[t][T]);
#pragma unroll
            for (int p = 0; p < PF; ++p) {
#pragma unroll
                for (int t = 0; t < TR; ++t) qs[p][t] = qs[p + 1][t];
#pragma unroll
                for (int T = 0; T < NTM; ++T) cs[p][T] = cs[p + 1][T];
            }
        }

        rowmfma_epilogue<S, EXPL, TR>(a, k, rb, fast, ok, prow, acc, recNi, cbase, ident_only);
    }
}

// ---------------------------------------------------------------- row update, LDS-staged
// The leaf-level row update with its basis and coefficient operands staged
// in LDS by direct loads (global_load_lds_dwordx4): a load in flight holds
// no register, so a workgroup keeps NST - 1 stages of BK basis columns in
// flight while the matrix cores work on the oldest one.  The workgroup
// walks its chunk in tiles of BM = 64 TR rows (16 TR per wave, the lanes'
// rows as in rowmfma_body); the stream of (tile, stage) pairs runs on
// without a break, so the first stages of the next tile load during the
// epilogue of this one.  The products, their order and the epilogue are
// those of rowmfma_body, so both kernels give the same bits.
//
// Requirements (checked by the launcher): identity row map, even chunk
// starts (16-byte row pairs), BK a multiple of 4.
// rows per lane, basis columns per stage and stages of the LDS ring (the
// fastest measured; the wide finalize keeps two rows per lane, its
// accumulators and epilogue already take the register file of two waves)
template <int S, bool EXPL>
__host__ __device__ constexpr int rowlds_tr() { return (S >= 32 && EXPL) ? 2 : 4; }
template <int S, bool EXPL>
__host__ __device__ constexpr int rowlds_bk() { return (S >= 32 && EXPL) ? 16 : 8; }
template <int S, bool EXPL>
__host__ __device__ constexpr int rowlds_nst() { return (S >= 32 && EXPL) ? 2 : 3; }

template <int S, bool EXPL, int TR, int BK, int NST>
struct RowLds {
    static constexpr int M = EXPL ? 2 * S : S;          // coefficient columns
    static constexpr int NTM = (M + 15) / 16;
    static constexpr int RW = 16 * TR;                   // rows per wave
    static constexpr int BM = kWaves * RW;               // rows per tile
    static constexpr int QN = BK * BM;                   // basis doubles per stage
    static constexpr int CN = BK * M;                    // coefficient doubles per stage
    static constexpr int LQ = QN / 128 / kWaves;         // basis loads per wave per stage
    static constexpr int CL = (CN / 2 + 64 * kWaves - 1) / (64 * kWaves);   // coefficient loads per wave
    // coefficient area: every lane of every wave loads (the wait counts
    // assume equal loads per wave), lanes past CN into the spare tail; reads
    // past column M of the last row stay inside it as well
    static constexpr int CP = (CL * 128 * kWaves > CN + 16) ? CL * 128 * kWaves : CN + 16;
    static constexpr int L = LQ + CL;                    // direct loads per wave per stage
    static constexpr size_t lds_bytes() { return (size_t)NST * (QN + CP) * 8; }
    static_assert(QN % (128 * kWaves) == 0, "basis stage must split evenly over the waves");
    static_assert(BK % 4 == 0 && TR % 2 == 0, "4-column steps, row pairs");
    static_assert((NST - 1) * L < 64, "wait counts fit the counter");
};

// LDS operands of one 4-column step: TR basis rows (TR / 2 16-byte reads at
// q + 256 u bytes) and NTM coefficients (at c + 128 T bytes), with the wait
// for them inside the same statement.
template <int TR, int NTM>
__device__ __forceinline__ void lds_step(uint32_t q, uint32_t c, double (&qv)[TR], double (&cv)[NTM]);

template <>
__device__ __forceinline__ void lds_step<2, 4>(uint32_t q, uint32_t c, double (&qv)[2], double (&cv)[4]) {
    dbl2v a;
    asm volatile("ds_read_b128 %0, %5\n\t"
                 "ds_read_b64 %1, %6\n\t"
                 "ds_read_b64 %2, %6 offset:128\n\t"
                 "ds_read_b64 %3, %6 offset:256\n\t"
                 "ds_read_b64 %4, %6 offset:384\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(a), "=&v"(cv[0]), "=&v"(cv[1]), "=&v"(cv[2]), "=&v"(cv[3])
                 : "v"(q), "v"(c) : "memory");
    qv[0] = a.x; qv[1] = a.y;
}

template <>
__device__ __forceinline__ void lds_step<4, 2>(uint32_t q, uint32_t c, double (&qv)[4], double (&cv)[2]) {
    dbl2v a, b;
    asm volatile("ds_read_b128 %0, %4\n\t"
                 "ds_read_b128 %1, %4 offset:256\n\t"
                 "ds_read_b64 %2, %5\n\t"
                 "ds_read_b64 %3, %5 offset:128\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(a), "=&v"(b), "=&v"(cv[0]), "=&v"(cv[1])
                 : "v"(q), "v"(c) : "memory");
    qv[0] = a.x; qv[1] = a.y; qv[2] = b.x; qv[3] = b.y;
}

template <>
__device__ __forceinline__ void lds_step<4, 1>(uint32_t q, uint32_t c, double (&qv)[4], double (&cv)[1]) {
    dbl2v a, b;
    asm volatile("ds_read_b128 %0, %3\n\t"
                 "ds_read_b128 %1, %3 offset:256\n\t"
                 "ds_read_b64 %2, %4\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(a), "=&v"(b), "=&v"(cv[0])
                 : "v"(q), "v"(c) : "memory");
    qv[0] = a.x; qv[1] = a.y; qv[2] = b.x; qv[3] = b.y;
}

template <>
__device__ __forceinline__ void lds_step<8, 1>(uint32_t q, uint32_t c, double (&qv)[8], double (&cv)[1]) {
    dbl2v a, b, d, e;
    asm volatile("ds_read_b128 %0, %5\n\t"
                 "ds_read_b128 %1, %5 offset:256\n\t"
                 "ds_read_b128 %2, %5 offset:512\n\t"
                 "ds_read_b128 %3, %5 offset:768\n\t"
                 "ds_read_b64 %4, %6\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(a), "=&v"(b), "=&v"(d), "=&v"(e), "=&v"(cv[0])
                 : "v"(q), "v"(c) : "memory");
    qv[0] = a.x; qv[1] = a.y; qv[2] = b.x; qv[3] = b.y;
    qv[4] = d.x; qv[5] = d.y; qv[6] = e.x; qv[7] = e.y;
}

template <>
__device__ __forceinline__ void lds_step<2, 1>(uint32_t q, uint32_t c, double (&qv)[2], double (&cv)[1]) {
    dbl2v a;
    asm volatile("ds_read_b128 %0, %2\n\t"
                 "ds_read_b64 %1, %3\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(a), "=&v"(cv[0])
                 : "v"(q), "v"(c) : "memory");
    qv[0] = a.x; qv[1] = a.y;
}

template <>
__device__ __forceinline__ void lds_step<2, 2>(uint32_t q, uint32_t c, double (&qv)[2], double (&cv)[2]) {
    dbl2v a;
    asm volatile("ds_read_b128 %0, %3\n\t"
                 "ds_read_b64 %1, %4\n\t"
                 "ds_read_b64 %2, %4 offset:128\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(a), "=&v"(cv[0]), "=&v"(cv[1])
                 : "v"(q), "v"(c) : "memory");
    qv[0] = a.x; qv[1] = a.y;
}

template <int S, bool EXPL, int TR, int BK, int NST>
__device__ __forceinline__ void rowlds_body(const FinalizeArgs &a_in, int bx, double *lds) {
    using C = RowLds<S, EXPL, TR, BK, NST>;
    constexpr int M = C::M, NTM = C::NTM, RW = C::RW, BM = C::BM;
    if (failed(a_in.status)) return;
    // the wave index in a scalar register: the tile loop's branches are uniform
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int il = lane & 15, g = lane >> 4;
    const int k = a_in.k;
    int leaf;
    int64_t r0, r1;
    a_in.geom.chunk(bx, leaf, r0, r1);
    const FinalizeArgs a = leaf_finalize_args(a_in, leaf);
    const double *rec = a.small + (int64_t)leaf * a.small_stride;
    const double *recP = a.sweep == 1 ? rec : rec + (int64_t)a.kmax * S + 2 * S * S;
    const double *recNi = a.sweep == 1 ? rec + (int64_t)a.kmax * S + S * S : recP + (int64_t)a.kmax * S;
    const bool ident_only = a.single_sweep != 0;
    const bool skip_p = EXPL && S % 16 == 0 && ident_only;   // zero tiles, as in rowmfma_body
    const double *cbase = EXPL ? a.Cptr + (int64_t)leaf * a.cseg : nullptr;
    const double *coef = EXPL ? cbase : recP;           // rows c of [P2 | C] or of P

    const int nk = (k + BK - 1) / BK;                    // stages per tile
    const int ntile = (int)((r1 - r0 + BM - 1) / BM);
    const int nz = nk * ntile;                           // (tile, stage) pairs

    // direct loads of stage z into slot z % NST: basis columns c0 .. c0 + BK - 1
    // of the tile's rows (one 1 KB load = 128 rows of one column), then the
    // coefficient rows c0 .. c0 + BK - 1 (contiguous, M doubles each)
    auto issue = [&](int z) {
        const int tile = z / nk, kb = z - tile * nk;
        const int64_t R0 = r0 + (int64_t)tile * BM;
        const int c0 = kb * BK;
        double *qs = lds + (size_t)(z % NST) * (C::QN + C::CP);
        double *cs = qs + C::QN;
#pragma unroll
        for (int j = 0; j < C::LQ; ++j) {
            const int gi = wave * C::LQ + j;             // 1 KB piece of the stage
            const int cc = gi / (BM / 128), part = gi % (BM / 128);
            int c = c0 + cc;
            if (c >= k) c = c0;                          // past k: a valid column, never used
            int64_t row = R0 + part * 128 + 2 * lane;
            if (row >= r1) row = r0;                     // past the chunk: a valid pair, never stored
            const double *src = a.Q.ptr + (int64_t)c * a.Q.ld + row;
            __builtin_amdgcn_global_load_lds((global_void *)src, (lds_void *)(qs + cc * BM + part * 128), 16, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < C::CL; ++j) {
            const int e = ((wave * C::CL + j) * 64 + lane) * 2;   // first double of this lane
            const bool use = e < C::CN && c0 + e / M < k;        // else a valid row, never read
            const double *src = coef + (int64_t)c0 * M + (use ? e : 0);
            __builtin_amdgcn_global_load_lds((global_void *)src, (lds_void *)(cs + (wave * C::CL + j) * 128), 16, 0, 0);
        }
    };

    for (int z = 0; z < NST - 1 && z < nz; ++z) issue(z);

    for (int tile = 0; tile < ntile; ++tile) {
        const int64_t R0 = r0 + (int64_t)tile * BM;
        const int64_t rb = R0 + (int64_t)wave * RW;
        int64_t prow[TR];
        bool ok[TR];
#pragma unroll
        for (int t = 0; t < TR; ++t) {
            const int64_t r = lane_row(rb, il, t);
            ok[t] = r < r1;
            prow[t] = ok[t] ? r : r0;
        }
        const bool fast = rb + RW <= r1;
        dbl4 acc[TR][NTM];
#pragma unroll
        for (int t = 0; t < TR; ++t)
#pragma unroll
            for (int T = 0; T < NTM; ++T) acc[t][T] = zero4();

        for (int kb = 0; kb < nk; ++kb) {
            const int z = tile * nk + kb;
            const int ahead = min(NST - 2, nz - 1 - z);
            wait_stage<C::L, NST>(ahead);
            __builtin_amdgcn_s_barrier();                // stage z everywhere; slot of z - 1 free
            if (z + NST - 1 < nz) issue(z + NST - 1);
            const double *qs = lds + (size_t)(z % NST) * (C::QN + C::CP);
            const double *cs = qs + C::QN;
            const uint32_t qa = (uint32_t)(uintptr_t)(lds_void *)(qs + g * BM + wave * RW + 2 * il);
            const uint32_t ca = (uint32_t)(uintptr_t)(lds_void *)(cs + g * M + il);
            const int csteps = min(BK, k - kb * BK) / 4;
#pragma unroll
            for (int st = 0; st < BK / 4; ++st) {
                if (st < csteps) {
                    double qv[TR], cv[NTM];
                    lds_step<TR, NTM>(qa + st * 4 * BM * 8, ca + st * 4 * M * 8, qv, cv);
#pragma unroll
                    for (int T = 0; T < NTM; ++T) {
                        const int m = 16 * T + il;
                        if (m >= M || (ident_only && m < S)) cv[T] = 0.0;
                    }
#pragma unroll
                    for (int t = 0; t < TR; ++t)
#pragma unroll
                        for (int T = 0; T < NTM; ++T)
                            if (!skip_p || T >= S / 16) acc[t][T] = mfma16(cv[T], qv[t], acc[t][T]);
                }
            }
        }
        rowmfma_epilogue<S, EXPL, TR>(a, k, rb, fast, ok, prow, acc, recNi, cbase, ident_only);
    }
}

template <int S, bool EXPL, int CLS>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_rowlds(FinalizeArgs a) {
    extern __shared__ double lds_dyn[];
    rowlds_body<S, EXPL, rowlds_tr<S, EXPL>(), rowlds_bk<S, EXPL>(), rowlds_nst<S, EXPL>()>(a, blockIdx.x, lds_dyn);
}

template <int S, bool EXPL, int CLS>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_rowmfma(FinalizeArgs a) {
    // the reduction level's correction and finalize (classes 5, 6): TZ
    rowmfma_body<S, EXPL, rowmfma_tr<S, EXPL>(), rowmfma_pf<S, EXPL>(), CLS == 5 || CLS == 6>(a, blockIdx.x);
}

// ---------------------------------------------------------------- apply Q C
constexpr int kApplyMB = 16;
template <int RPT>
__global__ __launch_bounds__(kThreads) void k_apply(ApplyArgs a) {
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int k = a.k, m = a.m;
    double *cl = lds;  // kRowCB x kApplyMB
    int leaf;
    int64_t r0, r1;
    a.geom.chunk(blockIdx.x, leaf, r0, r1);
    const double *cbase = a.Cptr + (int64_t)leaf * a.cseg;
    const Operand Qv = leaf_view(a.Q, a.geom, leaf);
    for (int64_t base = r0; base < r1; base += (int64_t)kThreads * RPT) {
        int64_t prow[RPT];
        bool ok[RPT];
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int64_t r = base + tid + (int64_t)kThreads * i;
            ok[i] = r < r1;
            prow[i] = a.geom.map.phys(ok[i] ? r : r0);
        }
        double acc[RPT][kApplyMB];
#pragma unroll
        for (int i = 0; i < RPT; ++i)
#pragma unroll
            for (int j = 0; j < kApplyMB; ++j) acc[i][j] = 0.0;
        for (int c0 = 0; c0 < k; c0 += kRowCB) {
            const int cb = (k - c0) < kRowCB ? (k - c0) : kRowCB;
            __syncthreads();
            for (int e = tid; e < cb * kApplyMB; e += kThreads) {
                const int c = e / kApplyMB, j = e % kApplyMB;
                cl[e] = j < m ? cbase[(int64_t)j * a.ldc + c0 + c] : 0.0;
            }
            __syncthreads();
            for (int c = 0; c < cb; ++c) {
                double q[RPT];
#pragma unroll
                for (int i = 0; i < RPT; ++i) q[i] = Qv.ptr[(int64_t)(c0 + c) * Qv.ld + prow[i]];
#pragma unroll
                for (int j = 0; j < kApplyMB; ++j) {
                    const double w = cl[c * kApplyMB + j];
#pragma unroll
                    for (int i = 0; i < RPT; ++i) acc[i][j] = fma(q[i], w, acc[i][j]);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            if (!ok[i]) continue;
            for (int j = 0; j < m; ++j) a.Y.ptr[(int64_t)j * a.Y.ld + prow[i]] = acc[i][j];
        }
    }
}

// ---------------------------------------------------------------- utilities
__global__ void k_fill(double *p, int64_t count, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_i32(int32_t *p, int64_t count, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_copy_cols(const double *src, int64_t lds_, RowMap smap, double *dst, int64_t ldd,
                            int64_t rows, int32_t cols) {
    const int64_t total = rows * cols;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / rows, r = e - c * rows;
        dst[c * ldd + r] = src[c * lds_ + smap.phys(r)];
    }
}

__global__ void k_copy_leafblk(Operand src, LevelGeom g, double *dst, int64_t ldd, int32_t cols) {
    const int64_t rows = g.nrows, total = rows * cols;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / rows, r = e - c * rows;
        int32_t leaf = (int32_t)(r / g.leaf_rows);
        if (leaf > g.nleaf - 1) leaf = g.nleaf - 1;
        const Operand v = leaf_view(src, g, leaf);
        dst[c * ldd + r] = v.ptr[c * v.ld + r];
    }
}

// the right halves of the per-leaf records [. | C_i] (row-major, 2s columns)
// from a column-major matrix holding leaf i's rows at i * seg_rows
__global__ void k_rows_to_records(const double *src, int64_t ld, int32_t nseg, int64_t seg_rows, int32_t rows,
                                  int32_t s, double *rec, int64_t rec_seg) {
    const int64_t total = (int64_t)nseg * rows * s;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / ((int64_t)rows * s);
        const int32_t rem = (int32_t)(e - i * rows * s), c = rem / s, j = rem - (rem / s) * s;
        rec[i * rec_seg + (int64_t)c * 2 * s + s + j] = src[i * seg_rows + c + (int64_t)j * ld];
    }
}

__global__ void k_laplacian(const double *X, int64_t ldx, double *Y, int64_t ldy, int32_t s,
                            int32_t nx, int32_t ny, int32_t nz, double shift) {
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t total = n * s;
    const double diag = (nz > 1 ? 6.0 : 4.0) + shift;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / n, p = e - c * n;
        const double *x = X + c * ldx;
        const int64_t i = p % nx;
        const int64_t j = (p / nx) % ny;
        const int64_t l = p / ((int64_t)nx * ny);
        double v = diag * x[p];
        if (i > 0) v -= x[p - 1];
        if (i < nx - 1) v -= x[p + 1];
        if (j > 0) v -= x[p - nx];
        if (j < ny - 1) v -= x[p + nx];
        if (nz > 1) {
            const int64_t pl = (int64_t)nx * ny;
            if (l > 0) v -= x[p - pl];
            if (l < nz - 1) v -= x[p + pl];
        }
        Y[c * ldy + p] = v;
    }
}

// Synthetic blocks for timing runs: entry (r, c) of block `seed` is a
// splitmix64 hash of (seed, c, r) mapped to a uniform value in [-1, 1).
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__global__ void k_synth(double *W, int64_t ld, int64_t n, int32_t s, uint64_t seed) {
    const int64_t total = n * s;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / n, r = e - c * n;
        const uint64_t h = splitmix64(splitmix64(seed * 0x100000001B3ull + (uint64_t)c) ^ (uint64_t)r);
        W[c * ld + r] = (double)(h >> 11) * 0x1.0p-52 - 1.0;
    }
}

__global__ __launch_bounds__(256) void k_copy(const double *__restrict__ src, double *__restrict__ dst,
                                              int64_t count) {
    const int64_t n2 = count / 2;
    const double2 *s2 = reinterpret_cast<const double2 *>(src);
    double2 *d2 = reinterpret_cast<double2 *>(dst);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n2;
         i += (int64_t)gridDim.x * blockDim.x)
        d2[i] = s2[i];
    if (blockIdx.x == 0 && threadIdx.x == 0 && (count & 1)) dst[count - 1] = src[count - 1];
}

// ---------------------------------------------------------------- batched form
// One grouped launch per phase covers every instance of a batch: workgroup b
// belongs to the instance whose block range [prefix[i], prefix[i+1]) holds b.
// The per-instance work is the same device code as the single-handle
// kernels, selected by the instance's block width.

__device__ __forceinline__ int64_t hess_offset(const BatchInst &d, int step) {
    return (int64_t)step * d.s * d.kmax;      // column block `step` of the K x K buffer
}

template <int S>
__device__ void batch_gram(const BatchArgs &a, const BatchInst &d, int inst, int local) {
    const int k = a.step * S, ncol = k + S;
    const bool leaf = a.phase == BP_LGRAM || a.phase == BP_LGRAMF || a.phase == BP_LGRAM2;
    GramArgs g{};
    g.k = k;
    g.tile_groups = gram_tile_groups(ncol);
    g.part_stride = (int64_t)ncol * S;
    g.status = a.status;
    if (leaf) {
        g.Q = Operand{d.Q, d.ldq};
        g.X = a.phase == BP_LGRAM2 ? Operand{d.U1L, d.ldq} : Operand{a.W[inst], d.n};
        // Householder leaves: the second leaf Gram is [V v_new]^T v_new, the
        // new reflectors just stored after the basis
        if (a.hh && a.phase == BP_LGRAM2) g.X = Operand{d.Q + (int64_t)k * d.ldq, d.ldq};
        g.geom = make_leaf_geom(d.n, d.leaf_rows, d.p, d.cL);
        g.partials = d.PL;
        g.retry = d.retry;
        g.cond = a.phase == BP_LGRAMF ? 1 : 0;   // the mixed form's FP64 redo, when flagged
    } else {
        g.Q = Operand{d.T, d.ldt};
        g.X = a.phase == BP_RGRAM ? Operand{d.Y, d.ldt} : Operand{d.U1R, d.ldt};
        g.geom = make_root_geom(d.p, d.kmax, ncol, d.cR);
        g.partials = d.PR;
    }
    const int cg = gram_col_groups(ncol, S);
    gram_body<S>(g, local / cg, local % cg);
}

// the mixed form's first leaf Gram, on the FP32 copy of the instance's basis;
// it clears the instance's retry flag for this step
template <int S>
__device__ void batch_gram_hi(const BatchArgs &a, const BatchInst &d, int inst, int local) {
    const int k = a.step * S, ncol = k + S;
    GramArgs g{};
    g.k = k;
    g.tile_groups = gram_tile_groups(ncol);
    g.part_stride = (int64_t)ncol * S;
    g.status = a.status;
    g.Q = Operand{d.Q, d.ldq};
    g.Qhi = d.Qhi;
    g.X = Operand{a.W[inst], d.n};
    g.geom = make_leaf_geom(d.n, d.leaf_rows, d.p, d.cL);
    g.partials = d.PL;
    g.clear_retry = 1;
    g.retry = d.retry;
    const int cg = gram_col_groups(ncol, S);
    gram_f32_body<S>(g, local / cg, local % cg);
}

template <int S>
__device__ void batch_chol(const BatchArgs &a, const BatchInst &d, int inst, int local) {
    const int k = a.step * S, ncol = k + S;
    const bool leaf = a.phase == BP_LCHOL1 || a.phase == BP_LCHOLF || a.phase == BP_LCHOL2;
    const int sweep = (a.phase == BP_LCHOL2 || a.phase == BP_RCHOL2) ? 2 : 1;
    CholArgs c{};
    c.part_stride = (int64_t)ncol * S;
    c.k = k;
    c.kmax = d.kmax;
    c.sweep = sweep;
    c.level = leaf ? 0 : 1;
    c.final_sweep = a.two ? 2 : 1;
    c.small_stride = small_stride(d.kmax, S);
    c.instance = inst;
    c.status = a.status;
    const int rg = gram_row_groups(ncol);
    if (leaf) {
        const LevelGeom gl = make_leaf_geom(d.n, d.leaf_rows, d.p, d.cL);
        c.partials = d.PL;
        c.nleaf = d.p;
        c.slots_per_leaf = gl.cpl * rg;
        c.slots_last = gl.cpl_last * rg;
        c.small = d.SL;
        c.Yout = d.Y;
        c.ldy = d.ldt;
        c.yseg = d.kmax;
        c.pc = d.CL;
        c.pc_stride = (int64_t)d.kmax * 2 * S;
        // mixed form: a failed pivot on the FP32 copy flags the instance's
        // FP64 redo (BP_LGRAMF, BP_LCHOLF), which runs only when flagged
        c.retry = d.retry;
        c.soft = (a.phase == BP_LCHOL1 && d.Qhi) ? 1 : 0;
        c.cond = a.phase == BP_LCHOLF ? 1 : 0;
    } else {
        const LevelGeom gr = make_root_geom(d.p, d.kmax, ncol, d.cR);
        const int slots = gr.nchunks() * rg;
        c.partials = slots > kReduceGroup ? d.PR2 : d.PR;
        c.nleaf = 1;
        c.slots_per_leaf = c.slots_last = slots > kReduceGroup ? (int32_t)ceil_div64(slots, kReduceGroup) : slots;
        c.small = d.SR;
        double *col = a.Hess[inst] + hess_offset(d, a.step);
        c.H = k > 0 ? col : nullptr;
        c.ldh = d.kmax;
        c.R = col + k;
        c.ldr = d.kmax;
    }
    chol_body<S>(c, local);
}

__device__ void batch_reduce(const BatchArgs &a, const BatchInst &d, int local) {
    const int k = a.step * d.s, ncol = k + d.s;
    const int slots = make_root_geom(d.p, d.kmax, ncol, d.cR).nchunks() * gram_row_groups(ncol);
    ReduceArgs r{};
    r.in = d.PR;
    r.stride = (int64_t)ncol * d.s;
    r.nslots = slots;
    r.group = kReduceGroup;
    r.nentries = ncol * d.s;
    r.out = d.PR2;
    r.status = a.status;
    const int eb = (int)ceil_div64(r.nentries, kThreads);
    reduce_body(r, local % eb, local / eb);
}

// the leaf row updates' arguments for instance d: the correction (BP_LCORR)
// or the finalize with the explicit block (BP_LFIN)
template <int S>
__device__ __forceinline__ FinalizeArgs batch_leaf_rowupdate_args(const BatchArgs &a, const BatchInst &d, int inst) {
    const int k = a.step * S;
    FinalizeArgs f{};
    f.k = k;
    f.kmax = d.kmax;
    f.small_stride = small_stride(d.kmax, S);
    f.status = a.status;
    f.geom = make_leaf_geom(d.n, d.leaf_rows, d.p, kBatchFinalChunk);
    f.small = d.SL;
    if (a.phase == BP_LCORR) {
        f.Q = Operand{d.Q, d.ldq};
        f.Qnew = OutOperand{d.U1L, d.ldq};
        f.U1 = Operand{a.W[inst], d.n};
        f.sweep = 1;
    } else {
        f.Q = Operand{d.Q, d.ldq};
        f.Qnew = OutOperand{d.Q + (int64_t)k * d.ldq, d.ldq};
        f.Qnew_hi = d.Qhi ? d.Qhi + (int64_t)k * d.ldq : nullptr;   // mixed form: FP32 copy
        f.U1 = Operand{d.U1L, d.ldq};
        f.sweep = 2;
        f.single_sweep = a.two ? 0 : 1;
        f.Cptr = d.CL;
        f.cseg = (int64_t)d.kmax * 2 * S;
        f.Uout = OutOperand{a.U[inst], d.n};
        if (a.hh) {
            // Householder leaves: -V Z over the k + s reflectors (the new
            // ones as the "u1" block, copied to the scratch unchanged)
            f.Qnew = OutOperand{d.U1L, d.ldq};
            f.Qnew_hi = nullptr;
            f.U1 = Operand{d.Q + (int64_t)k * d.ldq, d.ldq};
            f.single_sweep = 1;
        }
    }
    return f;
}

template <int S>
__device__ void batch_rowupdate(const BatchArgs &a, const BatchInst &d, int inst, int local) {
    const int k = a.step * S, ncol = k + S;
    FinalizeArgs f{};
    f.k = k;
    f.kmax = d.kmax;
    f.small_stride = small_stride(d.kmax, S);
    f.status = a.status;
    switch (a.phase) {
        case BP_LCORR:
            f.Q = Operand{d.Q, d.ldq};
            f.Qnew = OutOperand{d.U1L, d.ldq};
            f.U1 = Operand{a.W[inst], d.n};
            f.sweep = 1;
            f.geom = make_leaf_geom(d.n, d.leaf_rows, d.p, kBatchFinalChunk);
            f.small = d.SL;
            rowmfma_body<S, false, rowmfma_tr<S, false>(), rowmfma_pf<S, false>()>(f, local);
            return;
        case BP_RCORR:
            f.Q = Operand{d.T, d.ldt};
            f.Qnew = OutOperand{d.U1R, d.ldt};
            f.U1 = Operand{d.Y, d.ldt};
            f.sweep = 1;
            f.geom = make_root_geom(d.p, d.kmax, ncol, kRootRowChunk);
            f.small = d.SR;
            rowmfma_body<S, false, rowmfma_tr<S, false>(), rowmfma_pf<S, false>()>(f, local);
            return;
        case BP_RFIN:
            f.Q = Operand{d.T, d.ldt};
            f.Qnew = OutOperand{d.T + (int64_t)k * d.ldt, d.ldt};
            f.U1 = Operand{d.U1R, d.ldt};
            f.sweep = 2;
            f.single_sweep = a.two ? 0 : 1;
            f.geom = make_root_geom(d.p, d.kmax, ncol, kRootRowChunk);
            f.small = d.SR;
            f.Crow = d.CL;
            f.crow_seg = (int64_t)d.kmax * 2 * S;
            rowmfma_body<S, false, rowmfma_tr<S, false>(), rowmfma_pf<S, false>()>(f, local);
            return;
        default:   // BP_LFIN
            f.Q = Operand{d.Q, d.ldq};
            f.Qnew = OutOperand{d.Q + (int64_t)k * d.ldq, d.ldq};
            f.Qnew_hi = d.Qhi ? d.Qhi + (int64_t)k * d.ldq : nullptr;
            f.U1 = Operand{d.U1L, d.ldq};
            f.sweep = 2;
            f.single_sweep = a.two ? 0 : 1;
            if (a.hh) {      // Householder leaves, as in batch_leaf_rowupdate_args
                f.Qnew = OutOperand{d.U1L, d.ldq};
                f.Qnew_hi = nullptr;
                f.U1 = Operand{d.Q + (int64_t)k * d.ldq, d.ldq};
                f.single_sweep = 1;
            }
            f.geom = make_leaf_geom(d.n, d.leaf_rows, d.p, kBatchFinalChunk);
            f.small = d.SL;
            f.Cptr = d.CL;
            f.cseg = (int64_t)d.kmax * 2 * S;
            f.Uout = OutOperand{a.U[inst], d.n};
            rowmfma_body<S, true, rowmfma_tr<S, true>(), rowmfma_pf<S, true>()>(f, local);
            return;
    }
}

// One kernel per block width: the host launches a phase once for every
// width present in the batch, with a block prefix table that gives the
// other widths' instances no blocks, so each width keeps its own register
// allocation.
template <int S>
__global__ __launch_bounds__(kThreads) void kb_gram(BatchArgs a) {
    int inst, local;
    batch_locate(a, inst, local);
    const BatchInst d = a.inst[inst];
    batch_gram<S>(a, d, inst, local);
}

template <int S>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void kb_gram_hi(BatchArgs a) {
    int inst, local;
    batch_locate(a, inst, local);
    const BatchInst d = a.inst[inst];
    batch_gram_hi<S>(a, d, inst, local);
}

template <int S>
__global__ __launch_bounds__(kThreads) void kb_chol(BatchArgs a) {
    int inst, local;
    batch_locate(a, inst, local);
    const BatchInst d = a.inst[inst];
    batch_chol<S>(a, d, inst, local);
}

__global__ __launch_bounds__(kThreads) void kb_reduce(BatchArgs a) {
    int inst, local;
    batch_locate(a, inst, local);
    const BatchInst d = a.inst[inst];
    batch_reduce(a, d, local);
}

template <int S>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void kb_rowupdate(BatchArgs a) {
    int inst, local;
    batch_locate(a, inst, local);
    const BatchInst d = a.inst[inst];
    batch_rowupdate<S>(a, d, inst, local);
}

// the leaf row updates of blocks of 16 and more columns, LDS-staged as the
// single handles' (k_rowlds: same products, same bits); the host uses it
// when every instance of the width meets rowlds_body's requirements (even
// chunk starts: even leaf heights or a single leaf; the rest holds by
// construction)
template <int S, bool EXPL>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void kb_rowlds(BatchArgs a) {
    extern __shared__ double lds_dyn[];
    int inst, local;
    batch_locate(a, inst, local);
    const BatchInst d = a.inst[inst];
    const FinalizeArgs f = batch_leaf_rowupdate_args<S>(a, d, inst);
    rowlds_body<S, EXPL, rowlds_tr<S, EXPL>(), rowlds_bk<S, EXPL>(), rowlds_nst<S, EXPL>()>(f, local, lds_dyn);
}

// ---------------------------------------------------------------- launchers
static int grid_for(int64_t count, int threads) {
    int64_t b = (count + threads - 1) / threads;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (int)b;
}

template <int S>
static hipError_t gram_s(const GramArgs &a, int cls, hipStream_t st) {
    const int ncol = a.k + S;
    const dim3 grid(a.geom.nchunks(), gram_col_groups(ncol, S));
    switch (cls) {
        case 0: hipLaunchKernelGGL((k_gram<S, 0>), grid, dim3(kThreads), 0, st, a); break;
        case 3: hipLaunchKernelGGL((k_gram<S, 3>), grid, dim3(kThreads), 0, st, a); break;
        case 9: hipLaunchKernelGGL((k_gram<S, 9>), grid, dim3(kThreads), 0, st, a); break;
        case 11: hipLaunchKernelGGL((k_gram<S, 11>), grid, dim3(kThreads), 0, st, a); break;
        default: hipLaunchKernelGGL((k_gram<S, 10>), grid, dim3(kThreads), 0, st, a); break;
    }
    return hipGetLastError();
}

template <int S>
static hipError_t gram_hi_s(const GramArgs &a, hipStream_t st) {
    const dim3 grid(a.geom.nchunks(), gram_col_groups(a.k + S, S));
    hipLaunchKernelGGL((k_gram_hi<S>), grid, dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_gram(int s, const GramArgs &a, int cls, hipStream_t st) {
    if (a.Qhi) {                      // mixed form, leaf sweep-1 Gram
        if (cls != 0) return hipErrorInvalidValue;
        switch (s) {
            case 1: return gram_hi_s<1>(a, st);
            case 2: return gram_hi_s<2>(a, st);
            case 4: return gram_hi_s<4>(a, st);
            case 8: return gram_hi_s<8>(a, st);
            case 16: return gram_hi_s<16>(a, st);
            case 32: return gram_hi_s<32>(a, st);
        }
        return hipErrorInvalidValue;
    }
    switch (s) {
        case 1: return gram_s<1>(a, cls, st);
        case 2: return gram_s<2>(a, cls, st);
        case 4: return gram_s<4>(a, cls, st);
        case 8: return gram_s<8>(a, cls, st);
        case 16: return gram_s<16>(a, cls, st);
        case 32: return gram_s<32>(a, cls, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_reduce(const ReduceArgs &a, hipStream_t st) {
    const int ngrp = (a.nslots + a.group - 1) / a.group;
    const dim3 grid((a.nentries + kThreads - 1) / kThreads, ngrp);
    hipLaunchKernelGGL(k_reduce, grid, dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

template <int S>
static hipError_t chol_s(const CholArgs &a, hipStream_t st) {
    hipLaunchKernelGGL((k_chol<S>), dim3(a.nleaf), dim3(kThreads), chol_lds_bytes<S>(), st, a);
    return hipGetLastError();
}

hipError_t launch_chol(int s, const CholArgs &a, hipStream_t st) {
    switch (s) {
        case 1: return chol_s<1>(a, st);
        case 2: return chol_s<2>(a, st);
        case 4: return chol_s<4>(a, st);
        case 8: return chol_s<8>(a, st);
        case 16: return chol_s<16>(a, st);
        case 32: return chol_s<32>(a, st);
    }
    return hipErrorInvalidValue;
}

// the LDS-staged kernel takes leaf-level launches of blocks of 16 and more
// columns (narrower blocks run at the streaming rate without it) whose row
// pairs and coefficient rows are 16-byte aligned
static bool rowlds_eligible(const FinalizeArgs &a, int s) {
    const auto al16 = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    if (s < 16 || a.geom.map.seg_len != 0) return false;
    // even chunk starts: even chunks, and even leaf heights unless one leaf
    if (((a.geom.leaf_rows & 1) && a.geom.nleaf > 1) || (a.geom.chunk_rows & 1) || (a.Q.ld & 1) ||
        !al16(a.Q.ptr))
        return false;
    if (!al16(a.small) || (a.small_stride & 1) || ((int64_t)a.kmax * s & 1)) return false;
    if (a.Cptr && (!al16(a.Cptr) || (a.cseg & 1))) return false;
    return true;
}

template <int S, bool EXPL, int CLS>
static hipError_t launch_rowlds(const FinalizeArgs &a, hipStream_t st) {
    using C = RowLds<S, EXPL, rowlds_tr<S, EXPL>(), rowlds_bk<S, EXPL>(), rowlds_nst<S, EXPL>()>;
    hipLaunchKernelGGL((k_rowlds<S, EXPL, CLS>), dim3(a.geom.nchunks()), dim3(kThreads), C::lds_bytes(), st, a);
    return hipGetLastError();
}

template <int S>
static hipError_t rowupdate_s(const FinalizeArgs &a, int cls, hipStream_t st) {
    const dim3 grid(a.geom.nchunks());
    if constexpr (S >= 16) {
        if (!a.reg_only && rowlds_eligible(a, S)) {
            if (a.Cptr != nullptr) return launch_rowlds<S, true, 7>(a, st);
            return launch_rowlds<S, false, 2>(a, st);   // the leaf correction is the only leaf-level one
        }
    }
    if (a.Cptr != nullptr && cls == 6) {
        // a tree level below the root: explicit product into the children's
        // records, stacked tree-factor rows (zero rows skipped)
        if (!a.Cout || a.geom.map.seg_len == 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_rowmfma<S, true, 6>), grid, dim3(kThreads), 0, st, a);
    } else if (a.Cptr != nullptr) {
        hipLaunchKernelGGL((k_rowmfma<S, true, 7>), grid, dim3(kThreads), 0, st, a);
    } else {
        switch (cls) {
            case 2: hipLaunchKernelGGL((k_rowmfma<S, false, 2>), grid, dim3(kThreads), 0, st, a); break;
            case 5: hipLaunchKernelGGL((k_rowmfma<S, false, 5>), grid, dim3(kThreads), 0, st, a); break;
            default: hipLaunchKernelGGL((k_rowmfma<S, false, 6>), grid, dim3(kThreads), 0, st, a); break;
        }
    }
    return hipGetLastError();
}

// Kernels whose dynamic LDS exceeds 64 KB need the limit raised once per
// function on the current device (host-side, outside any stream, so never
// inside a captured graph): the LDS-staged row updates and the wide Cholesky
// at s = 32.
template <int S, bool EXPL, int CLS>
static hipError_t raise_rowlds_lds() {
    using C = RowLds<S, EXPL, rowlds_tr<S, EXPL>(), rowlds_bk<S, EXPL>(), rowlds_nst<S, EXPL>()>;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rowlds<S, EXPL, CLS>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)C::lds_bytes());
}

template <int S>
static hipError_t raise_wide_lds() {
    hipError_t e = raise_rowlds_lds<S, true, 7>();
    if (e == hipSuccess) e = raise_rowlds_lds<S, false, 2>();
    using CF = RowLds<S, true, rowlds_tr<S, true>(), rowlds_bk<S, true>(), rowlds_nst<S, true>()>;
    using CC = RowLds<S, false, rowlds_tr<S, false>(), rowlds_bk<S, false>(), rowlds_nst<S, false>()>;
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&kb_rowlds<S, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)CF::lds_bytes());
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&kb_rowlds<S, false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)CC::lds_bytes());
    if (e == hipSuccess && chol_lds_bytes<S>() > 65536)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_chol<S>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)chol_lds_bytes<S>());
    if (e == hipSuccess && chol_lds_bytes<S>() > 65536)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&kb_chol<S>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)chol_lds_bytes<S>());
    return e;
}

hipError_t prepare_kernels(int s) {
    switch (s) {
        case 16: return raise_wide_lds<16>();
        case 32: return raise_wide_lds<32>();
    }
    return hipSuccess;
}

hipError_t launch_finalize(int s, const FinalizeArgs &a, int cls, hipStream_t st) {
    switch (s) {
        case 1: return rowupdate_s<1>(a, cls, st);
        case 2: return rowupdate_s<2>(a, cls, st);
        case 4: return rowupdate_s<4>(a, cls, st);
        case 8: return rowupdate_s<8>(a, cls, st);
        case 16: return rowupdate_s<16>(a, cls, st);
        case 32: return rowupdate_s<32>(a, cls, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_apply(const ApplyArgs &a, hipStream_t st) {
    if (a.m < 1 || a.m > kApplyMB) return hipErrorInvalidValue;
    const size_t lds = (size_t)kRowCB * kApplyMB * 8;
    hipLaunchKernelGGL((k_apply<1>), dim3(a.geom.nchunks()), dim3(kThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_fill(double *p, int64_t count, double v, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(count, 256)), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(count, 256)), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}

hipError_t launch_copy_cols(const double *src, int64_t lds_, RowMap smap, double *dst, int64_t ldd,
                            int64_t rows, int32_t cols, hipStream_t st) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_cols, dim3(grid_for(rows * cols, 256)), dim3(256), 0, st, src, lds_,
                       smap, dst, ldd, rows, cols);
    return hipGetLastError();
}

hipError_t launch_copy_leafblk(const Operand &src, const LevelGeom &g, double *dst, int64_t ldd, int32_t cols,
                               hipStream_t st) {
    const int64_t total = g.nrows * cols;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_leafblk, dim3(grid_for(total, 256)), dim3(256), 0, st, src, g, dst, ldd, cols);
    return hipGetLastError();
}

hipError_t launch_rows_to_records(const double *src, int64_t ld, int32_t nseg, int64_t seg_rows, int32_t rows,
                                 int32_t s, double *rec, int64_t rec_seg, hipStream_t st) {
    const int64_t total = (int64_t)nseg * rows * s;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rows_to_records, dim3(grid_for(total, 256)), dim3(256), 0, st, src, ld, nseg, seg_rows, rows,
                       s, rec, rec_seg);
    return hipGetLastError();
}

hipError_t launch_laplacian(const double *X, int64_t ldx, double *Y, int64_t ldy, int32_t s,
                            int32_t nx, int32_t ny, int32_t nz, double shift, hipStream_t st) {
    const int64_t total = (int64_t)nx * ny * nz * s;
    hipLaunchKernelGGL(k_laplacian, dim3(grid_for(total, 256)), dim3(256), 0, st, X, ldx, Y, ldy, s,
                       nx, ny, nz, shift);
    return hipGetLastError();
}

hipError_t launch_synth(double *W, int64_t ld, int64_t n, int32_t s, uint64_t seed, hipStream_t st) {
    if (n <= 0 || s <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_synth, dim3(grid_for(n * s, 256)), dim3(256), 0, st, W, ld, n, s, seed);
    return hipGetLastError();
}

hipError_t launch_copy(const double *src, double *dst, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy, dim3(grid_for(count / 2 + 1, 256)), dim3(256), 0, st, src, dst, count);
    return hipGetLastError();
}

}  // namespace orth

namespace orth {

template <int S, bool EXPL>
static size_t rowlds_lds_bytes() {
    return RowLds<S, EXPL, rowlds_tr<S, EXPL>(), rowlds_bk<S, EXPL>(), rowlds_nst<S, EXPL>()>::lds_bytes();
}

size_t batch_phase_lds(int phase, int s, bool rowlds) {
    auto chol = [](int s) -> size_t { return chol_lds_bytes_s(s); };
    switch (phase) {
        case BP_LCHOL1: case BP_LCHOLF: case BP_LCHOL2: case BP_RCHOL1: case BP_RCHOL2:
            return chol(s);
        case BP_LCORR: case BP_LFIN:
            if (!rowlds || s < 16) return 0;
            if (s == 16) return phase == BP_LFIN ? rowlds_lds_bytes<16, true>() : rowlds_lds_bytes<16, false>();
            return phase == BP_LFIN ? rowlds_lds_bytes<32, true>() : rowlds_lds_bytes<32, false>();
    }
    return 0;
}

template <int S>
static hipError_t batch_phase_s(const BatchArgs &a, int32_t blocks, size_t lds, hipStream_t st) {
    if (batch_hh_phase(a.phase)) return hipErrorInvalidValue;   // launch_batch_hh_phase
    switch (a.phase) {
        case BP_LGRAM:
            if (a.mixed) {       // its own kernel: the FP64 Grams keep their register budget
                hipLaunchKernelGGL((kb_gram_hi<S>), dim3(blocks), dim3(kThreads), lds, st, a);
                break;
            }
            [[fallthrough]];
        case BP_LGRAMF: case BP_LGRAM2: case BP_RGRAM: case BP_RGRAM2:
            hipLaunchKernelGGL((kb_gram<S>), dim3(blocks), dim3(kThreads), lds, st, a);
            break;
        case BP_LCHOL1: case BP_LCHOLF: case BP_LCHOL2: case BP_RCHOL1: case BP_RCHOL2:
            hipLaunchKernelGGL((kb_chol<S>), dim3(blocks), dim3(kThreads), lds, st, a);
            break;
        case BP_RRED1: case BP_RRED2:
            hipLaunchKernelGGL(kb_reduce, dim3(blocks), dim3(kThreads), lds, st, a);
            break;
        default:
            if constexpr (S >= 16) {
                // a nonzero LDS size for a leaf row update selects the LDS-staged kernel
                if (lds > 0 && a.phase == BP_LCORR) {
                    hipLaunchKernelGGL((kb_rowlds<S, false>), dim3(blocks), dim3(kThreads), lds, st, a);
                    break;
                }
                if (lds > 0 && a.phase == BP_LFIN) {
                    hipLaunchKernelGGL((kb_rowlds<S, true>), dim3(blocks), dim3(kThreads), lds, st, a);
                    break;
                }
            }
            hipLaunchKernelGGL((kb_rowupdate<S>), dim3(blocks), dim3(kThreads), lds, st, a);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_batch_phase(const BatchArgs &a, int s, int32_t blocks, size_t lds, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    switch (s) {
        case 1: return batch_phase_s<1>(a, blocks, lds, st);
        case 2: return batch_phase_s<2>(a, blocks, lds, st);
        case 4: return batch_phase_s<4>(a, blocks, lds, st);
        case 8: return batch_phase_s<8>(a, blocks, lds, st);
        case 16: return batch_phase_s<16>(a, blocks, lds, st);
        case 32: return batch_phase_s<32>(a, blocks, lds, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace orth
