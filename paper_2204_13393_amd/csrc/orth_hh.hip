// Householder leaves (Sec. 2.2, Algorithm "HH"; the node-level method of the
// paper's proposed design, Sec. 5.2): every leaf basis is held as unit
// reflectors V_i (n_i x k, column c zero above leaf row c) with the
// compact-WY factor T_i (k x k upper triangular, Q = I - V T V^T for the
// product H_0 ... H_{k-1}, H_c = I - 2 v_c v_c^T).  A step on leaf i:
//
//   M = V^T w                       leaf Gram kernel (basis V)
//   Y = T^T M                       k_hh_prep        (this file)
//   w~ = w - V Y = Q_k^T w          row-update kernel (coefficients Y, identity)
//   P = w~[0:k]; Householder QR of w~[k:] -> s reflectors, N (s x s)
//                                   k_hh_panel       (this file)
//   [V v_new]^T v_new               leaf Gram kernel (block v_new)
//   T grows: T[0:k, k:k+s] = -T W T_s, T_s from v_new^T v_new
//                                   k_hh_tupd        (this file)
//   ... reduction level (BCGS-PIP+, unchanged) gives C_i ((k+s) x s) ...
//   Z = T (V[0:k+s]^T C_i)          k_hh_coef        (this file)
//   U|_i = -V Z                     row-update kernel (coefficients -Z)
//   U|_i[0:k+s] += C_i              k_hh_addec       (this file)
//
// The explicit block U|_i = Q_{k+s} [C_i; 0] = (I - V T V^T) [C_i; 0].  Every
// kernel here runs one workgroup per leaf and sums partial Gram slots in slot
// order, so results are bitwise reproducible.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "orth_internal.h"

namespace orth {
namespace {

__device__ __forceinline__ bool hh_failed(const DevStatus *st) { return st->code != 0; }

// sum over the 64 lanes of a wave (every lane gets the same value: the
// butterfly adds the same two operands on both partners)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// acc[j] += sum over c in [c0, c1) of t(c) L[c ls + j], c in order: the
// contraction loop of the per-leaf products for blocks of 32 columns.
// These kernels run one wave per SIMD (their LDS staging takes up to
// 160 KB), so the loads of t (T or V, from global memory) are issued
// kHhRing columns ahead; the scheduling barrier keeps each column's LDS
// reads next to its products (hoisted, they would take the registers of
// all the columns in flight).
// t(c) = valid ? p[c stride] : 0; every load is unconditional (p is a valid
// row for every lane, c is clamped into [c0, c1)) so that no value is
// needed before its use.
constexpr int kHhRing = 8;
template <int NJ>
__device__ __forceinline__ void hh_ring_contract(double (&acc)[NJ], int c0, int c1, const double *p, int64_t stride,
                                                 bool valid, const double *L, int ls) {
    // the range is the same for the whole wave: scalar loop control
    c0 = __builtin_amdgcn_readfirstlane(c0);
    c1 = __builtin_amdgcn_readfirstlane(c1);
    if (c0 >= c1) return;
    double ring[kHhRing];
    // (issued in ring order, as in the loop, so that the waits before each
    // use count the loads still in flight)
#pragma unroll
    for (int u = 0; u < kHhRing; ++u) {
        ring[u] = p[(int64_t)min(c0 + u, c1 - 1) * stride];
        __builtin_amdgcn_sched_barrier(0);
    }
    // whole groups of kHhRing columns, no branch inside a group: a column
    // past c1 adds t = 0 times a finite entry of row c1 - 1, which leaves
    // every sum as it is.  The LDS row of the next column is read while the
    // current one is multiplied.
    double cur[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) cur[j] = L[c0 * ls + j];
    for (int c = c0; c < c1; c += kHhRing) {
#pragma unroll
        for (int u = 0; u < kHhRing; ++u) {
            const int cc = c + u;
            const double t = (valid && cc < c1) ? ring[u] : 0.0;
            ring[u] = p[(int64_t)min(cc + kHhRing, c1 - 1) * stride];
            const double *Ln = L + min(cc + 1, c1 - 1) * ls;
            double nx[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j) nx[j] = Ln[j];
#pragma unroll
            for (int j = 0; j < NJ; ++j) acc[j] = fma(t, cur[j], acc[j]);
#pragma unroll
            for (int j = 0; j < NJ; ++j) cur[j] = nx[j];
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Per-leaf small matrices, k_max x k_max doubles each, at T + leaf 3 k_max^2:
//   Tc  the compact-WY factor T, column-major (element (r, c) at c k_max + r)
//   Tr  the same factor row-major (element (r, c) at r k_max + c)
//   Vr  the top k_max rows of the leaf's reflectors, row-major
// Each product below keeps one output row per lane and walks the
// contraction index with one coalesced load per step (the copy whose
// contiguous direction runs along the lanes), the other operand broadcast
// from LDS.  Entries below (T) or above (V) the diagonal are stored zeros,
// so a wave walks one range for all its lanes.
__device__ __forceinline__ double *hh_tc(const HhArgs &a, int leaf) {
    return a.T + (int64_t)leaf * 3 * a.kmax * a.kmax;
}

// ------------------------------------------------------------ T^T M
// Y = T_k^T M, M = V^T w from the leaf's partial slots (rows 0..k-1 of each
// [k+s][s] slot); Y goes to the leaf record's first-sweep projection and the
// record's first-sweep inverse normalizer is set to I, so the row-update
// kernel's sweep-1 pass computes w - V Y.
template <int S>
__device__ __forceinline__ void hh_prep_body(const HhArgs &a, int leaf) {
    if (hh_failed(a.status)) return;
    extern __shared__ double lds[];                 // M, k x S row-major
    const int tid = threadIdx.x, k = a.k;
    const int first = leaf * a.slots_per_leaf;
    const int cnt = leaf == a.geom.nleaf - 1 ? a.slots_last : a.slots_per_leaf;
    for (int e = tid; e < k * S; e += kThreads) {
        const double v = slot_sum(a.partials + (int64_t)first * a.part_stride + e, a.part_stride, cnt);
        lds[e] = v;
    }
    __syncthreads();
    const int64_t km = a.kmax;
    const double *Tr = hh_tc(a, leaf) + km * km;
    double *rec = a.small + (int64_t)leaf * a.small_stride;
    for (int rb = 0; rb < k; rb += kThreads) {
        const int r = rb + tid;
        // Y[r] = sum over c <= r of T(c, r) M[c]: T row c, lanes along r
        const int wmax = rb + (tid & ~63) + 63;
        // (a wave whose rows all lie past k has nothing to form)
        const int cend = rb + (tid & ~63) >= k ? 0 : (wmax + 1 < k ? wmax + 1 : k);
        double acc[S];
#pragma unroll
        for (int j = 0; j < S; ++j) acc[j] = 0.0;
        if constexpr (S >= 32) {
            hh_ring_contract(acc, 0, cend, Tr + (r < k ? r : k - 1), km, r < k, lds, S);
        } else {
            #pragma unroll 4      // four loads in flight per lane
            for (int c = 0; c < cend; ++c) {
                const double t = r < k ? Tr[(int64_t)c * km + r] : 0.0;
#pragma unroll
                for (int j = 0; j < S; ++j) acc[j] = fma(t, lds[c * S + j], acc[j]);
            }
        }
        if (r < k) {
#pragma unroll
            for (int j = 0; j < S; ++j) rec[(int64_t)r * S + j] = acc[j];
        }
    }
    double *n1i = rec + km * S + S * S;
    for (int e = tid; e < S * S; e += kThreads) n1i[e] = (e / S == e % S) ? 1.0 : 0.0;
}

template <int S>
__global__ __launch_bounds__(kThreads) void k_hh_prep(HhArgs a) { hh_prep_body<S>(a, blockIdx.x); }

// ------------------------------------------------------------ panel
// One workgroup factors leaf i's block w~ (n_i x s) held in registers: rows
// below k form the projection P, rows k.. the panel, triangularised column by
// column as in Algorithm "HH" (sign opposite to the pivot entry, sgn 0 = +1;
// a column that is zero from its pivot down gets the reflector e_pivot and a
// zero diagonal).  Each column costs one workgroup reduction: the dot
// products of the column with itself and the later columns over the rows
// from the pivot down, plus the pivot row's entries.
constexpr int kHhThreads = 512;
constexpr int kHhWaves = kHhThreads / 64;

template <int S>
__host__ __device__ constexpr int hh_rpt() { return S <= 4 ? 16 : (S == 8 ? 8 : 2); }
// sub-panel width: blocks wider than 16 columns are factored 8 columns at a
// time (k_hh_panel_sub)
template <int S>
__host__ __device__ constexpr int hh_sub() { return S <= 16 ? S : 8; }

template <int S>
__device__ __forceinline__ void hh_panel_body(const HhArgs &a, int leaf) {
    if (hh_failed(a.status)) return;
    constexpr int RPT = hh_rpt<S>();
    __shared__ double red[2][kHhWaves][S];
    __shared__ double rowv[2][S];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t r0 = a.geom.leaf_begin(leaf);
    const int nl = (int)(a.geom.leaf_end(leaf) - r0);
    const int k = a.k;

    double x[RPT][S];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int row = tid + kHhThreads * q;
#pragma unroll
        for (int c = 0; c < S; ++c) x[q][c] = row < nl ? a.X[(r0 + row) + (int64_t)c * a.ldx] : 0.0;
    }
    double *Yl = a.Yout + (int64_t)leaf * a.yseg;   // [P; N] of this leaf, column c at Yl + c ldy
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int row = tid + kHhThreads * q;
        if (row < k) {
#pragma unroll
            for (int c = 0; c < S; ++c) Yl[row + (int64_t)c * a.ldy] = x[q][c];
        }
    }

#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int pj = k + j, b = j & 1;
        double part[S];
#pragma unroll
        for (int c = 0; c < S; ++c) part[c] = 0.0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int row = tid + kHhThreads * q;
            if (row >= pj && row < nl) {
#pragma unroll
                for (int c = j; c < S; ++c) part[c] = fma(x[q][j], x[q][c], part[c]);
            }
        }
#pragma unroll
        for (int c = j; c < S; ++c) part[c] = wave_sum(part[c]);
        if (lane == 0) {
#pragma unroll
            for (int c = j; c < S; ++c) red[b][wave][c] = part[c];
        }
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            if (tid + kHhThreads * q == pj) {
#pragma unroll
                for (int c = j; c < S; ++c) rowv[b][c] = x[q][c];
            }
        }
        __syncthreads();
        double d[S], av[S];
#pragma unroll
        for (int c = j; c < S; ++c) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < kHhWaves; ++w) t += red[b][w][c];
            d[c] = t;
            av[c] = rowv[b][c];
        }
        const double lam = sqrt(d[j]);
        const double u0 = av[j];
        const bool zero = lam == 0.0;
        // v~ = (rows from the pivot down) - sigma lambda e_pivot, ||v~||^2 =
        // 2 lambda (lambda + |u0|); a NaN column runs the general branch
        const double njj = zero ? 0.0 : (u0 >= 0.0 ? -lam : lam);
        const double v0 = zero ? 1.0 : u0 - njj;
        const double nv2 = zero ? 1.0 : 2.0 * lam * (lam + fabs(u0));
        double coef[S];
#pragma unroll
        for (int c = j + 1; c < S; ++c) {
            const double w = zero ? av[c] : d[c] - njj * av[c];   // v~^T (column c)
            coef[c] = 2.0 * w / nv2;
        }
        if (tid == 0) {
            double *yr = Yl + k + j;
#pragma unroll
            for (int c = 0; c < S; ++c) {
                double v = 0.0;
                if (c == j) v = njj;
                else if (c > j) v = av[c] - v0 * coef[c];
                yr[(int64_t)c * a.ldy] = v;
            }
        }
        const double vn = sqrt(nv2);
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int row = tid + kHhThreads * q;
            if (row >= pj && row < nl) {
                const double vi = row == pj ? v0 : x[q][j];
#pragma unroll
                for (int c = j + 1; c < S; ++c) x[q][c] = fma(-vi, coef[c], x[q][c]);
                x[q][j] = vi / vn;
            }
        }
    }
    // the s reflectors, zero above their pivot rows
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int row = tid + kHhThreads * q;
        if (row < nl) {
#pragma unroll
            for (int c = 0; c < S; ++c)
                a.Q[(r0 + row) + (int64_t)(k + c) * a.ldq] = row >= k + c ? x[q][c] : 0.0;
        }
    }
}

template <int S>
__global__ __launch_bounds__(kHhThreads) void k_hh_panel(HhArgs a) { hh_panel_body<S>(a, blockIdx.x); }

// Blocks wider than the register budget (s = 32): the same factorisation in
// sub-panels of SB columns, in a kernel of 1024 threads holding 4 rows each
// (4096 rows; an 8-column sub-panel takes 64 registers per thread).  A
// sub-panel is loaded, the reflectors of the earlier sub-panels are applied
// to it one at a time, H_0 first (x -= 2 v (v^T x) with the stored unit
// reflector, whose rows a thread reads back from the ones it stored
// itself), so its rows k .. k + cb - 1 hold N's rows above it; it is then
// factored from row k + cb down as in k_hh_panel.  Each reduction takes two
// barriers: after the waves' partial sums, one wave forms the column's
// scalars and coefficients in LDS, which every thread then reads.
constexpr int kHhSubThreads = 1024;
constexpr int kHhSubWaves = kHhSubThreads / 64;
constexpr int kHhSubRows = 4;

template <int SB>
struct HhSubShared {
    double red[2][kHhSubWaves][SB];   // the waves' partial sums
    double rowv[2][SB];               // the pivot row
    double cf[2][SB];                 // per-column coefficients of the update
    double v0[2], vn[2];              // pivot entry of v~ and ||v~||
};

template <int SB>
struct HhSubCtx {
    const HhArgs &a;
    double *Yl;
    HhSubShared<SB> &sh;
    int k, cb, nl, it, tid, lane, wave;
};

// The wave sums of eight values per lane with ten exchanges instead of
// eight butterflies of six: at each of the first three steps a lane keeps
// half of its values and adds its partner's matching half, so afterwards
// lane l holds value (l >> 3) & 7 summed over the eight lanes that differ in
// bits 3..5; three more steps add over bits 0..2.  Lanes with l & 7 == 0
// end with the sum of value l >> 3 over the wave.
__device__ __forceinline__ double wave_sum8_transposed(const double (&v)[8], int lane) {
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
    double w[4], x[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double keep = b5 ? v[4 + i] : v[i], give = b5 ? v[i] : v[4 + i];
        w[i] = keep + __shfl_xor(give, 32, 64);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double keep = b4 ? w[2 + i] : w[i], give = b4 ? w[i] : w[2 + i];
        x[i] = keep + __shfl_xor(give, 16, 64);
    }
    double y = (b3 ? x[1] : x[0]) + __shfl_xor(b3 ? x[0] : x[1], 8, 64);
    y += __shfl_xor(y, 4, 64);
    y += __shfl_xor(y, 2, 64);
    y += __shfl_xor(y, 1, 64);
    return y;
}

// the waves' partial sums part[c] (c >= J0; the others are not used) into
// sh.red[b] (then a barrier)
template <int SB, int J0>
__device__ __forceinline__ void hh_sub_partials(double (&part)[SB], HhSubShared<SB> &sh, int b, int lane, int wave) {
    static_assert(SB == 8, "eight values per lane");
#pragma unroll
    for (int c = 0; c < J0; ++c) part[c] = 0.0;
    const double y = wave_sum8_transposed(part, lane);
    if ((lane & 7) == 0) sh.red[b][wave][lane >> 3] = y;
}

// One column J of a sub-panel (the steps of k_hh_panel's column loop), as a
// template so that every index into the register block is a constant.
template <int SB, int RPT, int J>
__device__ __forceinline__ void hh_sub_column(double (&x)[RPT][SB], const HhSubCtx<SB> &g) {
    const HhArgs &a = g.a;
    HhSubShared<SB> &sh = g.sh;
    const int k = g.k, cb = g.cb, nl = g.nl, tid = g.tid, lane = g.lane, wave = g.wave;
    const int pj = k + cb + J, b = (g.it + J) & 1;
    {
        double part[SB];
#pragma unroll
        for (int c = J; c < SB; ++c) part[c] = 0.0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int row = tid + kHhSubThreads * q;
            if (row >= pj && row < nl) {
#pragma unroll
                for (int c = J; c < SB; ++c) part[c] = fma(x[q][J], x[q][c], part[c]);
            }
        }
        hh_sub_partials<SB, J>(part, sh, b, lane, wave);
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            if (tid + kHhSubThreads * q == pj) {
#pragma unroll
                for (int c = J; c < SB; ++c) sh.rowv[b][c] = x[q][c];
            }
        }
    }
    __syncthreads();
    if (wave == 0) {
        // lane c < SB: column c's dot product with column J (fixed wave order)
        // and its pivot-row entry
        const int c = lane < SB ? lane : SB - 1;
        double d = 0.0;
#pragma unroll
        for (int w = 0; w < kHhSubWaves; ++w) d += sh.red[b][w][c < J ? J : c];
        const double av = sh.rowv[b][c < J ? J : c];
        const double dj = __shfl(d, J, 64), u0 = __shfl(av, J, 64);
        const double lam = sqrt(dj);
        const bool zero = lam == 0.0;
        const double njj = zero ? 0.0 : (u0 >= 0.0 ? -lam : lam);
        const double v0 = zero ? 1.0 : u0 - njj;
        const double nv2 = zero ? 1.0 : 2.0 * lam * (lam + fabs(u0));
        const double cf = 2.0 * (zero ? av : d - njj * av) / nv2;
        if (lane > J && lane < SB) sh.cf[b][lane] = cf;
        if (lane == 0) {
            sh.v0[b] = v0;
            sh.vn[b] = sqrt(nv2);
        }
        // row pj of N: zero left of the diagonal, this sub-panel's entries
        // (the later sub-panels write theirs when loaded)
        double *yr = g.Yl + pj;
        if (lane < cb + J) yr[(int64_t)lane * a.ldy] = 0.0;
        if (lane >= J && lane < SB) yr[(int64_t)(cb + lane) * a.ldy] = lane == J ? njj : av - v0 * cf;
    }
    __syncthreads();
    const double v0 = sh.v0[b], vn = sh.vn[b];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int row = tid + kHhSubThreads * q;
        if (row >= pj && row < nl) {
            const double vi = row == pj ? v0 : x[q][J];
#pragma unroll
            for (int c = J + 1; c < SB; ++c) x[q][c] = fma(-vi, sh.cf[b][c], x[q][c]);
            x[q][J] = vi / vn;
        }
    }
}

template <int SB, int RPT, int J>
struct HhSubCols {
    static __device__ __forceinline__ void run(double (&x)[RPT][SB], const HhSubCtx<SB> &g) {
        hh_sub_column<SB, RPT, J>(x, g);
        HhSubCols<SB, RPT, J + 1>::run(x, g);
    }
};
template <int SB, int RPT>
struct HhSubCols<SB, RPT, SB> {
    static __device__ __forceinline__ void run(double (&)[RPT][SB], const HhSubCtx<SB> &) {}
};

template <int S, int SB>
__device__ __forceinline__ void hh_panel_sub_body(const HhArgs &a, int leaf) {
    static_assert(S % SB == 0 && SB <= 64, "whole sub-panels, a column per lane");
    if (hh_failed(a.status)) return;
    constexpr int RPT = kHhSubRows;
    __shared__ HhSubShared<SB> sh;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t r0 = a.geom.leaf_begin(leaf);
    const int nl = (int)(a.geom.leaf_end(leaf) - r0);
    const int k = a.k;
    double *Yl = a.Yout + (int64_t)leaf * a.yseg;   // [P; N] of this leaf, column c at Yl + c ldy
    int it = 0;                                      // reductions so far (LDS buffer it & 1)

    for (int cb = 0; cb < S; cb += SB) {
        double x[RPT][SB];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int row = tid + kHhSubThreads * q;
#pragma unroll
            for (int c = 0; c < SB; ++c)
                x[q][c] = row < nl ? a.X[(r0 + row) + (int64_t)(cb + c) * a.ldx] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int row = tid + kHhSubThreads * q;
            if (row < k) {
#pragma unroll
                for (int c = 0; c < SB; ++c) Yl[row + (int64_t)(cb + c) * a.ldy] = x[q][c];
            }
        }
        // the earlier sub-panels' reflectors, H_0 first
#pragma unroll 1
        for (int j = 0; j < cb; ++j, ++it) {
            const int b = it & 1;
            double v[RPT];
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int row = tid + kHhSubThreads * q;
                v[q] = row < nl ? a.Q[(r0 + row) + (int64_t)(k + j) * a.ldq] : 0.0;
            }
            {
                double part[SB];
#pragma unroll
                for (int c = 0; c < SB; ++c) {
                    double t = 0.0;
#pragma unroll
                    for (int q = 0; q < RPT; ++q) t = fma(v[q], x[q][c], t);
                    part[c] = t;
                }
                hh_sub_partials<SB, 0>(part, sh, b, lane, wave);
            }
            __syncthreads();
            if (wave == 0 && lane < SB) {
                double t = 0.0;
#pragma unroll
                for (int w = 0; w < kHhSubWaves; ++w) t += sh.red[b][w][lane];
                sh.cf[b][lane] = 2.0 * t;
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < SB; ++c) {
                const double tw = sh.cf[b][c];
#pragma unroll
                for (int q = 0; q < RPT; ++q) x[q][c] = fma(-v[q], tw, x[q][c]);
            }
        }
        // rows k .. k + cb - 1: N's entries above this sub-panel
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int row = tid + kHhSubThreads * q;
            if (row >= k && row < k + cb) {
#pragma unroll
                for (int c = 0; c < SB; ++c) Yl[row + (int64_t)(cb + c) * a.ldy] = x[q][c];
            }
        }
        HhSubCols<SB, RPT, 0>::run(x, HhSubCtx<SB>{a, Yl, sh, k, cb, nl, it, tid, lane, wave});
        it += SB;
        // this sub-panel's reflectors, zero above their pivot rows
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int row = tid + kHhSubThreads * q;
            if (row < nl) {
#pragma unroll
                for (int c = 0; c < SB; ++c)
                    a.Q[(r0 + row) + (int64_t)(k + cb + c) * a.ldq] = row >= k + cb + c ? x[q][c] : 0.0;
            }
        }
    }
}

template <int S, int SB>
__global__ __launch_bounds__(kHhSubThreads) void k_hh_panel_sub(HhArgs a) { hh_panel_sub_body<S, SB>(a, blockIdx.x); }

// ------------------------------------------------------------ T update
// From the slots of [V v_new]^T v_new: W = V^T v_new (k x s) and
// G = v_new^T v_new.  T_s (s x s, upper): diagonal 2, column j above the
// diagonal -2 T_s[0:j, 0:j] G[0:j, j]; then T[0:k, k:k+s] = -T (W T_s), in
// both copies of T.  Also copies the reflectors' new top rows k..k+s-1 to
// the row-major Vr.
template <int S>
__device__ __forceinline__ void hh_tupd_body(const HhArgs &a, int leaf) {
    if (hh_failed(a.status)) return;
    extern __shared__ double lds[];
    const int tid = threadIdx.x, k = a.k, K = k + S;
    double *W = lds;                    // K x S row-major: W (rows < k), G (rows k..)
    double *Ts = W + K * S;             // S x S row-major
    const int first = leaf * a.slots_per_leaf;
    const int cnt = leaf == a.geom.nleaf - 1 ? a.slots_last : a.slots_per_leaf;
    for (int e = tid; e < K * S; e += kThreads) {
        const double v = slot_sum(a.partials + (int64_t)first * a.part_stride + e, a.part_stride, cnt);
        W[e] = v;
    }
    for (int e = tid; e < S * S; e += kThreads) Ts[e] = (e / S == e % S) ? 2.0 : 0.0;
    __syncthreads();
    const double *G = W + k * S;
    for (int j = 1; j < S; ++j) {
        if (tid < j) {
            const int i = tid;
            double v = 0.0;
            for (int l = i; l < j; ++l) v = fma(Ts[i * S + l], G[l * S + j], v);
            Ts[i * S + j] = -2.0 * v;
        }
        __syncthreads();
    }
    // B = W T_s, in place row by row (a row belongs to one thread)
    for (int r = tid; r < k; r += kThreads) {
        double bv[S];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            double v = 0.0;
#pragma unroll
            for (int l = 0; l <= j; ++l) v = fma(W[r * S + l], Ts[l * S + j], v);
            bv[j] = v;
        }
#pragma unroll
        for (int j = 0; j < S; ++j) W[r * S + j] = bv[j];
    }
    __syncthreads();
    const int64_t km = a.kmax;
    double *Tc = hh_tc(a, leaf), *Tr = Tc + km * km, *Vr = Tr + km * km;
    for (int rb = 0; rb < k; rb += kThreads) {
        const int r = rb + tid;
        // -(T B)[r] = -sum over c >= r of T(r, c) B[c]: T column c, lanes along r
        const int wmin = rb + (tid & ~63);
        double acc[S];
#pragma unroll
        for (int j = 0; j < S; ++j) acc[j] = 0.0;
        if constexpr (S >= 32) {
            hh_ring_contract(acc, wmin, k, Tc + (r < k ? r : k - 1), km, r < k, W, S);
        } else {
            #pragma unroll 4      // four loads in flight per lane
            for (int c = wmin; c < k; ++c) {
                const double t = r < k ? Tc[(int64_t)c * km + r] : 0.0;
#pragma unroll
                for (int j = 0; j < S; ++j) acc[j] = fma(t, W[c * S + j], acc[j]);
            }
        }
        if (r < k) {
#pragma unroll
            for (int j = 0; j < S; ++j) {
                Tc[(int64_t)(k + j) * km + r] = -acc[j];
                Tr[(int64_t)r * km + k + j] = -acc[j];
            }
        }
    }
    for (int e = tid; e < S * S; e += kThreads) {
        const int j = e / S, i = e - (e / S) * S;
        const double v = i <= j ? Ts[i * S + j] : 0.0;
        Tc[(int64_t)(k + j) * km + k + i] = v;
        Tr[(int64_t)(k + i) * km + k + j] = v;
    }
    const int64_t r0 = a.geom.leaf_begin(leaf);
    for (int e = tid; e < S * K; e += kThreads) {
        const int i = e / K, c = e - (e / K) * K;
        Vr[(int64_t)(k + i) * km + c] = a.Q[(r0 + k + i) + (int64_t)c * a.ldq];
    }
}

template <int S>
__global__ __launch_bounds__(kThreads) void k_hh_tupd(HhArgs a) { hh_tupd_body<S>(a, blockIdx.x); }

// ------------------------------------------------------------ coefficients
// C_i (the leaf's (k+s) x s block from the reduction, right half of its
// record) -> Z = T (V[0:k+s]^T C_i); the record's right half becomes -Z (the
// row-update kernel then forms -V Z) and its left half keeps C_i for the
// final E C_i term.
// CB columns of C_i at a time (CB = S, or S / 2 when two K x S blocks do
// not fit the LDS); every output column is the same sum either way.
template <int S, int CB>
__device__ __forceinline__ void hh_coef_body(const HhArgs &a, int leaf) {
    static_assert(S % CB == 0, "whole column blocks");
    if (hh_failed(a.status)) return;
    extern __shared__ double lds[];
    const int tid = threadIdx.x, K = a.k + S;
    double *C = lds, *B = lds + K * CB;            // K x CB row-major each
    double *rec = a.crec + (int64_t)leaf * a.cseg;  // row c: [left S | right S]
    const int64_t km = a.kmax;
    const double *Tc = hh_tc(a, leaf), *Vr = Tc + 2 * km * km;
    for (int j0 = 0; j0 < S; j0 += CB) {
        for (int e = tid; e < K * CB; e += kThreads) {
            const int r = e / CB, j = e - (e / CB) * CB;
            const double v = rec[(int64_t)r * 2 * S + S + j0 + j];
            C[e] = v;
            rec[(int64_t)r * 2 * S + j0 + j] = v;
        }
        __syncthreads();
        for (int cb = 0; cb < K; cb += kThreads) {
            const int c = cb + tid;
            // B[c] = sum over r >= c of V(r, c) C[r]: V row r, lanes along c
            const int wmin = cb + (tid & ~63);
            double acc[CB];
#pragma unroll
            for (int j = 0; j < CB; ++j) acc[j] = 0.0;
            if constexpr (S >= 32) {
                hh_ring_contract(acc, wmin, K, Vr + (c < K ? c : K - 1), km, c < K, C, CB);
            } else {
                #pragma unroll 4      // four loads in flight per lane
                for (int r = wmin; r < K; ++r) {
                    const double v = c < K ? Vr[(int64_t)r * km + c] : 0.0;
#pragma unroll
                    for (int j = 0; j < CB; ++j) acc[j] = fma(v, C[r * CB + j], acc[j]);
                }
            }
            if (c < K) {
#pragma unroll
                for (int j = 0; j < CB; ++j) B[c * CB + j] = acc[j];
            }
        }
        __syncthreads();
        for (int rb = 0; rb < K; rb += kThreads) {
            const int r = rb + tid;
            // Z[r] = sum over c >= r of T(r, c) B[c]: T column c, lanes along r
            const int wmin = rb + (tid & ~63);
            double acc[CB];
#pragma unroll
            for (int j = 0; j < CB; ++j) acc[j] = 0.0;
            if constexpr (S >= 32) {
                hh_ring_contract(acc, wmin, K, Tc + (r < K ? r : K - 1), km, r < K, B, CB);
            } else {
                #pragma unroll 4      // four loads in flight per lane
                for (int c = wmin; c < K; ++c) {
                    const double t = r < K ? Tc[(int64_t)c * km + r] : 0.0;
#pragma unroll
                    for (int j = 0; j < CB; ++j) acc[j] = fma(t, B[c * CB + j], acc[j]);
                }
            }
            if (r < K) {
#pragma unroll
                for (int j = 0; j < CB; ++j) rec[(int64_t)r * 2 * S + S + j0 + j] = -acc[j];
            }
        }
        __syncthreads();      // the next block overwrites C and B
    }
}

template <int S, int CB>
__global__ __launch_bounds__(kThreads) void k_hh_coef(HhArgs a) { hh_coef_body<S, CB>(a, blockIdx.x); }

// U|_i[0:k+s] += C_i (left half of the leaf's record)
template <int S>
__device__ __forceinline__ void hh_addec_body(const HhArgs &a, int leaf) {
    if (hh_failed(a.status)) return;
    const int tid = threadIdx.x, K = a.k + S;
    const double *rec = a.crec + (int64_t)leaf * a.cseg;
    const int64_t r0 = a.geom.leaf_begin(leaf);
    for (int e = tid; e < K * S; e += kThreads) {
        const int r = e / S, j = e - (e / S) * S;
        a.U[(r0 + r) + (int64_t)j * a.ldu] += rec[(int64_t)r * 2 * S + j];
    }
}

template <int S>
__global__ __launch_bounds__(kThreads) void k_hh_addec(HhArgs a) { hh_addec_body<S>(a, blockIdx.x); }

// ------------------------------------------------------------ apply
// orth_apply_Q: Y_i = Q_k [C_i; 0] = -V Z_i + E C_i with Z_i = T (V[0:k]^T C_i),
// C_i the leaf's coefficient block (k x m) from the reduction level.  MBI
// columns at a time, so the two k x MBI LDS blocks fit in 64 KB.
template <int MBI>
__global__ __launch_bounds__(kThreads) void k_hh_apply_coef(HhArgs a) {
    extern __shared__ double lds[];
    const int leaf = blockIdx.x, tid = threadIdx.x, k = a.k;
    const int64_t km = a.kmax;
    double *C = lds, *B = lds + (int64_t)k * MBI;   // k x MBI row-major each
    const double *Tc = hh_tc(a, leaf), *Vr = Tc + 2 * km * km;
    const double *cin = a.ca + leaf * km;
    double *cout = a.ca_out + leaf * km;
    for (int j0 = 0; j0 < a.m; j0 += MBI) {
        const int nb = a.m - j0 < MBI ? a.m - j0 : MBI;
        for (int e = tid; e < k * MBI; e += kThreads) {
            const int c = e / MBI, jj = e - (e / MBI) * MBI;
            C[e] = jj < nb ? cin[(int64_t)(j0 + jj) * a.ldca + c] : 0.0;
        }
        __syncthreads();
        for (int cb = 0; cb < k; cb += kThreads) {
            const int c = cb + tid;
            const int wmin = cb + (tid & ~63);
            double acc[MBI];
#pragma unroll
            for (int j = 0; j < MBI; ++j) acc[j] = 0.0;
            #pragma unroll 4      // four loads in flight per lane
            for (int r = wmin; r < k; ++r) {
                const double v = c < k ? Vr[(int64_t)r * km + c] : 0.0;
#pragma unroll
                for (int j = 0; j < MBI; ++j) acc[j] = fma(v, C[r * MBI + j], acc[j]);
            }
            if (c < k) {
#pragma unroll
                for (int j = 0; j < MBI; ++j) B[c * MBI + j] = acc[j];
            }
        }
        __syncthreads();
        for (int rb = 0; rb < k; rb += kThreads) {
            const int r = rb + tid;
            const int wmin = rb + (tid & ~63);
            double acc[MBI];
#pragma unroll
            for (int j = 0; j < MBI; ++j) acc[j] = 0.0;
            #pragma unroll 4      // four loads in flight per lane
            for (int c = wmin; c < k; ++c) {
                const double t = r < k ? Tc[(int64_t)c * km + r] : 0.0;
#pragma unroll
                for (int j = 0; j < MBI; ++j) acc[j] = fma(t, B[c * MBI + j], acc[j]);
            }
            if (r < k) {
#pragma unroll
                for (int j = 0; j < MBI; ++j)
                    if (j < nb) cout[(int64_t)(j0 + j) * a.ldca + r] = -acc[j];
            }
        }
        __syncthreads();
    }
}

// Y_i[0:k] += C_i
__global__ __launch_bounds__(kThreads) void k_hh_apply_add(HhArgs a) {
    const int leaf = blockIdx.x, tid = threadIdx.x, k = a.k;
    const double *cin = a.ca + leaf * (int64_t)a.kmax;
    const int64_t r0 = a.geom.leaf_begin(leaf);
    for (int e = tid; e < k * a.m; e += kThreads) {
        const int j = e / k, c = e - (e / k) * k;
        a.U[(r0 + c) + (int64_t)j * a.ldu] += cin[(int64_t)j * a.ldca + c];
    }
}

// dynamic LDS of the per-leaf small products for block width s at K = k + s
// columns (0: the K x s staging does not fit); coef_cb: the coefficient
// kernel's column block
size_t hh_prep_lds(int s, int64_t K) { return (size_t)(K - s) * s * 8; }
size_t hh_tupd_lds(int s, int64_t K) { return (size_t)(K * s + (int64_t)s * s) * 8; }
int hh_coef_cb(int s, int64_t K) {
    if ((size_t)2 * K * s * 8 <= kHhLdsMax) return s;
    if (s > 1 && (size_t)2 * K * (s / 2) * 8 <= kHhLdsMax) return s / 2;
    return 0;
}

// ------------------------------------------------------------ batched form
// The per-leaf Householder kernels for a batch: workgroup b is leaf `local`
// of the instance batch_locate finds, with the arguments a single handle of
// that instance's plan would pass (its leaf Gram geometry for the partial
// slots; the leaf bounds are those of every geometry).
// The instance of workgroup b without shared memory (these kernels keep the
// whole 160 KB of LDS for their staging): the last i with prefix[i] <= b,
// which is the i with prefix[i] <= b < prefix[i + 1] (instances with no
// blocks repeat their neighbour's entry).  Every lane takes the same path.
__device__ __forceinline__ void batch_locate_nolds(const BatchArgs &a, int &inst, int &local) {
    const int b = blockIdx.x;
    int lo = 0, hi = a.count - 1;          // prefix[0] = 0 <= b, prefix[count] > b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.prefix[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    inst = lo;
    local = b - a.prefix[lo];
}

template <int S>
__device__ __forceinline__ HhArgs batch_hh_args(const BatchArgs &a, const BatchInst &d, int inst) {
    const int k = a.step * S, ncol = k + S;
    const LevelGeom gg = make_leaf_geom(d.n, d.leaf_rows, d.p, d.cL);
    const int rg = gram_row_groups(ncol);
    HhArgs h{};
    h.geom = gg;
    h.k = k;
    h.kmax = d.kmax;
    h.Q = d.Q;
    h.ldq = d.ldq;
    h.T = d.TH;
    h.partials = d.PL;
    h.part_stride = (int64_t)ncol * S;
    h.slots_per_leaf = gg.cpl * rg;
    h.slots_last = gg.cpl_last * rg;
    h.small = d.SL;
    h.small_stride = small_stride(d.kmax, S);
    h.X = k > 0 ? d.U1L : a.W[inst];        // Q_k^T w (or w at k = 0)
    h.ldx = k > 0 ? d.ldq : d.n;
    h.Yout = d.Y;
    h.ldy = d.ldt;
    h.yseg = d.kmax;
    h.crec = d.CL;
    h.cseg = (int64_t)d.kmax * 2 * S;
    h.U = a.U[inst];
    h.ldu = d.n;
    h.status = a.status;
    return h;
}

template <int S>
__global__ __launch_bounds__(kThreads) void kb_hh_prep(BatchArgs a) {
    int inst, local;
    batch_locate_nolds(a, inst, local);
    const BatchInst d = a.inst[inst];
    hh_prep_body<S>(batch_hh_args<S>(a, d, inst), local);
}

template <int S>
__global__ __launch_bounds__(kHhThreads) void kb_hh_panel(BatchArgs a) {
    int inst, local;
    batch_locate_nolds(a, inst, local);
    const BatchInst d = a.inst[inst];
    hh_panel_body<S>(batch_hh_args<S>(a, d, inst), local);
}

template <int S, int SB>
__global__ __launch_bounds__(kHhSubThreads) void kb_hh_panel_sub(BatchArgs a) {
    int inst, local;
    batch_locate_nolds(a, inst, local);
    const BatchInst d = a.inst[inst];
    hh_panel_sub_body<S, SB>(batch_hh_args<S>(a, d, inst), local);
}

template <int S>
__global__ __launch_bounds__(kThreads) void kb_hh_tupd(BatchArgs a) {
    int inst, local;
    batch_locate_nolds(a, inst, local);
    const BatchInst d = a.inst[inst];
    hh_tupd_body<S>(batch_hh_args<S>(a, d, inst), local);
}

template <int S, int CB>
__global__ __launch_bounds__(kThreads) void kb_hh_coef(BatchArgs a) {
    int inst, local;
    batch_locate_nolds(a, inst, local);
    const BatchInst d = a.inst[inst];
    hh_coef_body<S, CB>(batch_hh_args<S>(a, d, inst), local);
}

template <int S>
__global__ __launch_bounds__(kThreads) void kb_hh_addec(BatchArgs a) {
    int inst, local;
    batch_locate_nolds(a, inst, local);
    const BatchInst d = a.inst[inst];
    hh_addec_body<S>(batch_hh_args<S>(a, d, inst), local);
}

template <int S>
hipError_t batch_hh_s(const BatchArgs &a, int32_t blocks, hipStream_t st) {
    const int K = a.step * S + S;
    if (!hh_small_fits(S, K)) return hipErrorInvalidValue;
    switch (a.phase) {
        case BP_HPREP:
            hipLaunchKernelGGL((kb_hh_prep<S>), dim3(blocks), dim3(kThreads), hh_prep_lds(S, K), st, a);
            break;
        case BP_HPANEL:
            if constexpr (S > 16) {
                hipLaunchKernelGGL((kb_hh_panel_sub<S, hh_sub<S>()>), dim3(blocks), dim3(kHhSubThreads), 0, st, a);
            } else {
                hipLaunchKernelGGL((kb_hh_panel<S>), dim3(blocks), dim3(kHhThreads), 0, st, a);
            }
            break;
        case BP_HTUPD:
            hipLaunchKernelGGL((kb_hh_tupd<S>), dim3(blocks), dim3(kThreads), hh_tupd_lds(S, K), st, a);
            break;
        case BP_HCOEF:
            if (hh_coef_cb(S, K) == S) {
                hipLaunchKernelGGL((kb_hh_coef<S, S>), dim3(blocks), dim3(kThreads), (size_t)2 * K * S * 8, st, a);
            } else if constexpr (S > 1) {
                hipLaunchKernelGGL((kb_hh_coef<S, S / 2>), dim3(blocks), dim3(kThreads), (size_t)K * S * 8, st, a);
            }
            break;
        case BP_HADDEC:
            hipLaunchKernelGGL((kb_hh_addec<S>), dim3(blocks), dim3(kThreads), 0, st, a);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int S>
hipError_t hh_launch(HhKernel which, const HhArgs &a, hipStream_t st) {
    const int nleaf = a.geom.nleaf;
    const int K = a.k + S;
    switch (which) {
        case HH_PREP:
            if (a.k < 1) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_hh_prep<S>), dim3(nleaf), dim3(kThreads), hh_prep_lds(S, K), st, a);
            break;
        case HH_PANEL:
            if constexpr (S > 16) {
                hipLaunchKernelGGL((k_hh_panel_sub<S, hh_sub<S>()>), dim3(nleaf), dim3(kHhSubThreads), 0, st, a);
            } else {
                hipLaunchKernelGGL((k_hh_panel<S>), dim3(nleaf), dim3(kHhThreads), 0, st, a);
            }
            break;
        case HH_TUPD:
            hipLaunchKernelGGL((k_hh_tupd<S>), dim3(nleaf), dim3(kThreads), hh_tupd_lds(S, K), st, a);
            break;
        case HH_COEF:
            if (hh_coef_cb(S, K) == S) {
                hipLaunchKernelGGL((k_hh_coef<S, S>), dim3(nleaf), dim3(kThreads), (size_t)2 * K * S * 8, st, a);
            } else if constexpr (S > 1) {
                hipLaunchKernelGGL((k_hh_coef<S, S / 2>), dim3(nleaf), dim3(kThreads), (size_t)K * S * 8, st, a);
            }
            break;
        case HH_ADDEC:
            hipLaunchKernelGGL((k_hh_addec<S>), dim3(nleaf), dim3(kThreads), 0, st, a);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_hh_apply(HhKernel which, const HhArgs &a, hipStream_t st) {
    if (a.geom.nleaf < 1 || a.k < 1 || a.k > a.kmax || a.m < 1 || a.m > 16) return hipErrorInvalidValue;
    const int nleaf = a.geom.nleaf;
    if (which == HH_APPLY_ADD) {
        hipLaunchKernelGGL(k_hh_apply_add, dim3(nleaf), dim3(kThreads), 0, st, a);
        return hipGetLastError();
    }
    if (which != HH_APPLY_COEF) return hipErrorInvalidValue;
    // columns per pass: two k x MBI blocks within 64 KB of LDS
    const int64_t k = a.k;
    if (k * 16 <= kHhMaxCoef) {
        hipLaunchKernelGGL((k_hh_apply_coef<16>), dim3(nleaf), dim3(kThreads), (size_t)(2 * k * 16 * 8), st, a);
    } else if (k * 8 <= kHhMaxCoef) {
        hipLaunchKernelGGL((k_hh_apply_coef<8>), dim3(nleaf), dim3(kThreads), (size_t)(2 * k * 8 * 8), st, a);
    } else if (k * 4 <= kHhMaxCoef) {
        hipLaunchKernelGGL((k_hh_apply_coef<4>), dim3(nleaf), dim3(kThreads), (size_t)(2 * k * 4 * 8), st, a);
    } else if (k * 2 <= kHhMaxCoef) {
        hipLaunchKernelGGL((k_hh_apply_coef<2>), dim3(nleaf), dim3(kThreads), (size_t)(2 * k * 2 * 8), st, a);
    } else if (k <= kHhMaxCoef) {
        hipLaunchKernelGGL((k_hh_apply_coef<1>), dim3(nleaf), dim3(kThreads), (size_t)(2 * k * 8), st, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int64_t hh_max_leaf_rows(int s) {
    switch (s) {
        case 1: return (int64_t)kHhThreads * hh_rpt<1>();
        case 2: return (int64_t)kHhThreads * hh_rpt<2>();
        case 4: return (int64_t)kHhThreads * hh_rpt<4>();
        case 8: return (int64_t)kHhThreads * hh_rpt<8>();
        case 16: return (int64_t)kHhThreads * hh_rpt<16>();
        case 32: return (int64_t)kHhSubThreads * kHhSubRows;
    }
    return 0;
}

bool hh_small_fits(int s, int64_t kmax) {
    return hh_prep_lds(s, kmax) <= kHhLdsMax && hh_tupd_lds(s, kmax) <= kHhLdsMax && hh_coef_cb(s, kmax) > 0;
}

template <int S>
static hipError_t raise_hh_lds() {
    const int lim = (int)kHhLdsMax;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_hh_prep<S>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_hh_tupd<S>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_hh_coef<S, S>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    if constexpr (S > 1) {
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_hh_coef<S, S / 2>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    }
    // and the batched forms of the same kernels
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&kb_hh_prep<S>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&kb_hh_tupd<S>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&kb_hh_coef<S, S>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    if constexpr (S > 1) {
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(&kb_hh_coef<S, S / 2>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    }
    return e;
}

hipError_t launch_batch_hh_phase(const BatchArgs &a, int s, int32_t blocks, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    switch (s) {
        case 1: return batch_hh_s<1>(a, blocks, st);
        case 2: return batch_hh_s<2>(a, blocks, st);
        case 4: return batch_hh_s<4>(a, blocks, st);
        case 8: return batch_hh_s<8>(a, blocks, st);
        case 16: return batch_hh_s<16>(a, blocks, st);
        case 32: return batch_hh_s<32>(a, blocks, st);
    }
    return hipErrorInvalidValue;
}

hipError_t prepare_hh_kernels(int s) {
    switch (s) {
        case 1: return raise_hh_lds<1>();
        case 2: return raise_hh_lds<2>();
        case 4: return raise_hh_lds<4>();
        case 8: return raise_hh_lds<8>();
        case 16: return raise_hh_lds<16>();
        case 32: return raise_hh_lds<32>();
    }
    return hipErrorInvalidValue;
}

hipError_t launch_hh(int s, HhKernel which, const HhArgs &a, hipStream_t st) {
    // host checks of the launch against what the kernels assume
    if (a.geom.nleaf < 1 || a.k < 0 || !hh_small_fits(s, (int64_t)a.k + s)) return hipErrorInvalidValue;
    if (which == HH_PANEL) {
        const int64_t last = a.geom.leaf_end(a.geom.nleaf - 1) - a.geom.leaf_begin(a.geom.nleaf - 1);
        const int64_t full = a.geom.nleaf > 1 ? a.geom.leaf_rows : last;
        if (std::max(last, full) > hh_max_leaf_rows(s) || std::min(last, full) < a.k + s) return hipErrorInvalidValue;
    }
    switch (s) {
        case 1: return hh_launch<1>(which, a, st);
        case 2: return hh_launch<2>(which, a, st);
        case 4: return hh_launch<4>(which, a, st);
        case 8: return hh_launch<8>(which, a, st);
        case 16: return hh_launch<16>(which, a, st);
        case 32: return hh_launch<32>(which, a, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace orth
