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
//   k_correct   sweep 2 (BCGS-PIP+, lines 3-4): u1 = (x - q P1) N1^{-1} row
//               by row, stored, and the partial [Q U1]^T U1 of the same rows
//               while the row tile is still in LDS.
//   k_finalize  per row: u = (u1 - q P2) N2^{-1} appended to the level's
//               local basis, and at the leaf level the explicit new block
//               U|_i = [Q_i U_i] [P~_i; N~_i] (Sec. 4.1, assembly of U).
//
// Layout: every operand is column-major; rows are streamed in tiles with
// coalesced column reads (consecutive lanes = consecutive rows) and staged
// in LDS as row-major tiles so the Gram products can give each lane whole
// columns while the s coefficients of a row are LDS broadcasts.
// No floating-point atomics: every sum has a fixed order.

#include "orth_internal.h"

namespace orth {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ bool failed(const DevStatus *st) {
    return __builtin_nontemporal_load(&st->code) != 0;
}

__host__ __device__ __forceinline__ int odd_ld(int ncol) { return ncol | 1; }

// Cross-wave fixed-order reduction of acc[CPT][S] (lanes = columns) and store
// of the chunk's partial Gram block.  `red` needs kWaves*64*S doubles.
template <int S, int CPT>
__device__ __forceinline__ void store_partial(double (&acc)[CPT][S], double *red, int ncol,
                                              double *out) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < S; ++j) red[(wave * 64 + lane) * S + j] = acc[q][j];
        __syncthreads();
        for (int e = tid; e < 64 * S; e += kThreads) {
            const int c = e / S + 64 * q;
            if (c < ncol) {
                double v = red[e];
#pragma unroll
                for (int w = 1; w < kWaves; ++w) v += red[w * 64 * S + e];
                out[64 * q * S + e] = v;
            }
        }
    }
}

// Load rows [rt, rt+nr) of [A B] (ka columns of A then S of B) into a row-major
// LDS tile tile[r*ldt + c]; rows >= nr are zero.
template <int S>
__device__ __forceinline__ void load_tile(const Operand &A, const Operand &B, int ka, int64_t rt,
                                          int nr, int TR, const RowMap &map, double *tile,
                                          int ldt, double *bt) {
    const int tid = threadIdx.x;
    const int rr = tid % TR;
    const int cstep = kThreads / TR;
    const bool rok = rr < nr;
    const int64_t prow = map.phys(rt + (rok ? rr : 0));
    const int ncol = ka + S;
    for (int c = tid / TR; c < ncol; c += cstep) {
        double v = 0.0;
        if (rok) v = (c < ka) ? A.ptr[(int64_t)c * A.ld + prow] : B.ptr[(int64_t)(c - ka) * B.ld + prow];
        tile[rr * ldt + c] = v;
        if (c >= ka) bt[rr * S + (c - ka)] = v;
    }
}

}  // namespace

// ---------------------------------------------------------------- sweep 1
template <int S, int CPT>
__global__ __launch_bounds__(kThreads) void k_gram(GramArgs a) {
    if (failed(a.status)) return;
    extern __shared__ double lds[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int k = a.k, ncol = k + S, TR = a.tile_rows, LDT = odd_ld(ncol);
    double *tile = lds;
    double *xt = lds + TR * LDT;
    int leaf;
    int64_t r0, r1;
    a.geom.chunk(blockIdx.x, leaf, r0, r1);

    double acc[CPT][S];
#pragma unroll
    for (int q = 0; q < CPT; ++q)
#pragma unroll
        for (int j = 0; j < S; ++j) acc[q][j] = 0.0;

    for (int64_t rt = r0; rt < r1; rt += TR) {
        const int nr = (int)((r1 - rt) < TR ? (r1 - rt) : TR);
        __syncthreads();
        load_tile<S>(a.Q, a.X, k, rt, nr, TR, a.geom.map, tile, LDT, xt);
        __syncthreads();
        for (int r = wave; r < nr; r += kWaves) {
            double xv[S];
#pragma unroll
            for (int j = 0; j < S; ++j) xv[j] = xt[r * S + j];
#pragma unroll
            for (int q = 0; q < CPT; ++q) {
                const int c = lane + 64 * q;
                const double v = (c < ncol) ? tile[r * LDT + c] : 0.0;
#pragma unroll
                for (int j = 0; j < S; ++j) acc[q][j] = fma(v, xv[j], acc[q][j]);
            }
        }
    }
    store_partial<S, CPT>(acc, lds, ncol, a.partials + (int64_t)blockIdx.x * a.part_stride);
}

// ---------------------------------------------------------------- sweep 2
// Projection lane layout: G = 256/TR lanes share one tile row and split the k
// columns (c = g, g+G, ...); their partial sums meet in a butterfly over the
// G lanes, which sit in the same wave (64/G rows per wave).
template <int S, int CPT>
__global__ __launch_bounds__(kThreads) void k_correct(CorrectArgs a) {
    if (failed(a.status)) return;
    extern __shared__ double lds[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int k = a.k, ncol = k + S, TR = a.tile_rows, LDT = odd_ld(ncol);
    const int G = kThreads / TR;
    double *tile = lds;                       // TR x LDT
    double *xt = tile + TR * LDT;             // TR x S
    double *ut = xt + TR * S;                 // TR x S
    double *p1 = ut + TR * S;                 // k x S
    double *n1i = p1 + (int64_t)k * S;        // S x S
    int leaf;
    int64_t r0, r1;
    a.geom.chunk(blockIdx.x, leaf, r0, r1);
    const double *rec = a.small + (int64_t)leaf * a.small_stride;
    for (int e = tid; e < k * S; e += kThreads) p1[e] = rec[e];
    for (int e = tid; e < S * S; e += kThreads) n1i[e] = rec[(int64_t)a.kmax * S + S * S + e];

    double acc[CPT][S];
#pragma unroll
    for (int q = 0; q < CPT; ++q)
#pragma unroll
        for (int j = 0; j < S; ++j) acc[q][j] = 0.0;

    // projection role of this thread: tile row pr, column phase g
    const int g = lane % G;
    const int pr = wave * (64 / G) + lane / G;

    for (int64_t rt = r0; rt < r1; rt += TR) {
        const int nr = (int)((r1 - rt) < TR ? (r1 - rt) : TR);
        __syncthreads();
        load_tile<S>(a.Q, a.X, k, rt, nr, TR, a.geom.map, tile, LDT, xt);
        __syncthreads();
        // y = x - q P1 (partial over this lane's columns, then butterfly)
        double y[S];
#pragma unroll
        for (int j = 0; j < S; ++j) y[j] = 0.0;
        for (int c = g; c < k; c += G) {
            const double v = tile[pr * LDT + c];
#pragma unroll
            for (int j = 0; j < S; ++j) y[j] = fma(v, p1[c * S + j], y[j]);
        }
        for (int off = 1; off < G; off <<= 1) {
#pragma unroll
            for (int j = 0; j < S; ++j) y[j] += __shfl_xor(y[j], off, 64);
        }
        if (g == 0) {
            double t[S];
#pragma unroll
            for (int j = 0; j < S; ++j) t[j] = xt[pr * S + j] - y[j];
            // u1 = t N1^{-1} (upper triangular)
#pragma unroll
            for (int j = 0; j < S; ++j) {
                double u = 0.0;
#pragma unroll
                for (int i = 0; i <= j; ++i) u = fma(t[i], n1i[i * S + j], u);
                ut[pr * S + j] = u;
            }
            if (pr < nr) {
                const int64_t prow = a.geom.map.phys(rt + pr);
#pragma unroll
                for (int j = 0; j < S; ++j) a.U1.ptr[(int64_t)j * a.U1.ld + prow] = ut[pr * S + j];
            }
        }
        __syncthreads();
        if (a.write_gram) {
            for (int r = wave; r < nr; r += kWaves) {
                double uv[S];
#pragma unroll
                for (int j = 0; j < S; ++j) uv[j] = ut[r * S + j];
#pragma unroll
                for (int q = 0; q < CPT; ++q) {
                    const int c = lane + 64 * q;
                    double v = 0.0;
                    if (c < k) v = tile[r * LDT + c];
                    else if (c < ncol) v = ut[r * S + (c - k)];
#pragma unroll
                    for (int j = 0; j < S; ++j) acc[q][j] = fma(v, uv[j], acc[q][j]);
                }
            }
        }
    }
    if (a.write_gram)
        store_partial<S, CPT>(acc, lds, ncol, a.partials + (int64_t)blockIdx.x * a.part_stride);
}

// ---------------------------------------------------------------- Cholesky
template <int S>
__global__ __launch_bounds__(kThreads) void k_chol(CholArgs a) {
    if (failed(a.status)) return;
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int leaf = blockIdx.x;
    const int k = a.k, ncol = k + S;
    double *pg = lds;                         // ncol x S : [P; G]
    double *sm = pg + (int64_t)ncol * S;      // S x S work (G - P^T P, then updated)
    double *nm = sm + S * S;                  // N
    double *ni = nm + S * S;                  // N^{-1}
    __shared__ int bad;
    if (tid == 0) bad = 0;

    const int first = a.geom.first_chunk(leaf), cnt = a.geom.chunks_of(leaf);
    for (int e = tid; e < ncol * S; e += kThreads) {
        double v = 0.0;
        for (int p = 0; p < cnt; ++p) v += a.partials[(int64_t)(first + p) * a.part_stride + e];
        pg[e] = v;
    }
    __syncthreads();
    for (int e = tid; e < S * S; e += kThreads) {
        const int i = e / S, j = e % S;
        double d = 0.0;
        for (int c = 0; c < k; ++c) d = fma(pg[c * S + i], pg[c * S + j], d);
        sm[e] = pg[(k + i) * S + j] - d;
        nm[e] = 0.0;
        ni[e] = 0.0;
    }
    __syncthreads();
    // right-looking upper Cholesky: N^T N = sm, lane j owns column j
    for (int kk = 0; kk < S; ++kk) {
        if (tid == kk) {
            const double piv = sm[kk * S + kk];
            if (!(piv > 0.0) || !isfinite(piv)) bad = kk + 1;
            else nm[kk * S + kk] = sqrt(piv);
        }
        __syncthreads();
        if (bad) break;
        if (tid > kk && tid < S) nm[kk * S + tid] = sm[kk * S + tid] / nm[kk * S + kk];
        __syncthreads();
        if (tid > kk && tid < S) {
            const int j = tid;
            const double nkj = nm[kk * S + j];
            for (int i = kk + 1; i <= j; ++i) sm[i * S + j] -= nm[kk * S + i] * nkj;
        }
        __syncthreads();
    }
    if (bad) {
        if (tid == 0 && atomicCAS(&a.status->code, 0, 3) == 0) {
            a.status->level = a.level;
            a.status->leaf = leaf;
            a.status->sweep = a.sweep;
            a.status->column = bad - 1;
        }
        return;
    }
    // N^{-1}, lane j owns column j (back substitution)
    if (tid < S) {
        const int j = tid;
        ni[j * S + j] = 1.0 / nm[j * S + j];
        for (int i = j - 1; i >= 0; --i) {
            double t = 0.0;
            for (int l = i + 1; l <= j; ++l) t = fma(nm[i * S + l], ni[l * S + j], t);
            ni[i * S + j] = -t / nm[i * S + i];
        }
    }
    __syncthreads();
    double *rec = a.small + (int64_t)leaf * a.small_stride;
    double *recP1 = rec;
    double *recN1 = rec + (int64_t)a.kmax * S;
    double *recN1i = recN1 + S * S;
    double *recP2 = recN1i + S * S;
    double *recN2i = recP2 + (int64_t)a.kmax * S;
    if (a.sweep == 1) {
        for (int e = tid; e < k * S; e += kThreads) recP1[e] = pg[e];
        for (int e = tid; e < S * S; e += kThreads) { recN1[e] = nm[e]; recN1i[e] = ni[e]; }
    } else {
        for (int e = tid; e < k * S; e += kThreads) recP2[e] = pg[e];
        for (int e = tid; e < S * S; e += kThreads) recN2i[e] = ni[e];
    }
    if (a.sweep != a.final_sweep) return;
    // [P; N] of this leaf:  sweep 1 only -> (P1, N1);  two sweeps ->
    // P = P1 + P2 N1, N = N2 N1 (the reiteration combination).
    const int64_t ybase = (int64_t)leaf * a.yseg;
    for (int e = tid; e < ncol * S; e += kThreads) {
        const int c = e / S, j = e % S;
        double v;
        if (c < k) {
            if (a.sweep == 1) {
                v = pg[e];
            } else {
                v = recP1[e];
                for (int i = 0; i <= j; ++i) v = fma(pg[c * S + i], recN1[i * S + j], v);
            }
        } else {
            const int i = c - k;
            if (a.sweep == 1) {
                v = nm[i * S + j];
            } else {
                v = 0.0;
                for (int l = i; l <= j; ++l) v = fma(nm[i * S + l], recN1[l * S + j], v);
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

// ---------------------------------------------------------------- finalize
template <int S, int RPT>
__global__ __launch_bounds__(kThreads) void k_finalize(FinalizeArgs a) {
    if (failed(a.status)) return;
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int k = a.k;
    double *p2 = lds;                         // k x S
    double *cq = p2 + (int64_t)k * S;         // k x S   (C rows 0..k-1)
    double *cn = cq + (int64_t)k * S;         // S x S   (C rows k..k+S-1)
    double *n2i = cn + S * S;                 // S x S
    int leaf;
    int64_t r0, r1;
    a.geom.chunk(blockIdx.x, leaf, r0, r1);
    const double *rec = a.small + (int64_t)leaf * a.small_stride;
    const double *recP2 = rec + (int64_t)a.kmax * S + 2 * S * S;
    const double *recN2i = recP2 + (int64_t)a.kmax * S;
    const bool explicit_out = a.Cptr != nullptr;
    for (int e = tid; e < k * S; e += kThreads) {
        p2[e] = a.single_sweep ? 0.0 : recP2[e];
        if (explicit_out) {
            const int c = e / S, j = e % S;
            cq[e] = a.Cptr[(int64_t)j * a.ldc + (int64_t)leaf * a.cseg + c];
        }
    }
    for (int e = tid; e < S * S; e += kThreads) {
        const int i = e / S, j = e % S;
        n2i[e] = a.single_sweep ? (i == j ? 1.0 : 0.0) : recN2i[e];
        if (explicit_out) cn[e] = a.Cptr[(int64_t)j * a.ldc + (int64_t)leaf * a.cseg + k + i];
    }
    __syncthreads();

    for (int64_t base = r0; base < r1; base += (int64_t)kThreads * RPT) {
        int64_t prow[RPT];
        bool ok[RPT];
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int64_t r = base + tid + (int64_t)kThreads * i;
            ok[i] = r < r1;
            prow[i] = a.geom.map.phys(ok[i] ? r : r0);
        }
        double pa[RPT][S], pb[RPT][S];
#pragma unroll
        for (int i = 0; i < RPT; ++i)
#pragma unroll
            for (int j = 0; j < S; ++j) { pa[i][j] = 0.0; pb[i][j] = 0.0; }
#pragma unroll 2
        for (int c = 0; c < k; ++c) {
            double q[RPT];
#pragma unroll
            for (int i = 0; i < RPT; ++i) q[i] = a.Q.ptr[(int64_t)c * a.Q.ld + prow[i]];
#pragma unroll
            for (int j = 0; j < S; ++j) {
                const double vp = p2[c * S + j];
                const double vc = cq[c * S + j];
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    pa[i][j] = fma(q[i], vp, pa[i][j]);
                    pb[i][j] = fma(q[i], vc, pb[i][j]);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            if (!ok[i]) continue;
            double t[S], u[S];
#pragma unroll
            for (int j = 0; j < S; ++j) t[j] = a.U1.ptr[(int64_t)j * a.U1.ld + prow[i]] - pa[i][j];
#pragma unroll
            for (int j = 0; j < S; ++j) {
                double v = 0.0;
#pragma unroll
                for (int l = 0; l <= j; ++l) v = fma(t[l], n2i[l * S + j], v);
                u[j] = v;
                a.Qnew.ptr[(int64_t)j * a.Qnew.ld + prow[i]] = v;
            }
            if (explicit_out) {
                const int64_t r = base + tid + (int64_t)kThreads * i;
#pragma unroll
                for (int j = 0; j < S; ++j) {
                    double v = pb[i][j];
#pragma unroll
                    for (int l = 0; l <= j; ++l) v = fma(u[l], cn[l * S + j], v);
                    a.Uout.ptr[(int64_t)j * a.Uout.ld + r] = v;
                }
            }
        }
    }
}

// ---------------------------------------------------------------- apply Q C
constexpr int kApplyMB = 16;
template <int RPT>
__global__ __launch_bounds__(kThreads) void k_apply(ApplyArgs a) {
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int k = a.k, m = a.m;
    double *cl = lds;  // k x kApplyMB
    int leaf;
    int64_t r0, r1;
    a.geom.chunk(blockIdx.x, leaf, r0, r1);
    for (int e = tid; e < k * kApplyMB; e += kThreads) {
        const int c = e / kApplyMB, j = e % kApplyMB;
        cl[e] = j < m ? a.Cptr[(int64_t)j * a.ldc + (int64_t)leaf * a.cseg + c] : 0.0;
    }
    __syncthreads();
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
        for (int c = 0; c < k; ++c) {
            double q[RPT];
#pragma unroll
            for (int i = 0; i < RPT; ++i) q[i] = a.Q.ptr[(int64_t)c * a.Q.ld + prow[i]];
#pragma unroll
            for (int j = 0; j < kApplyMB; ++j) {
                const double w = cl[c * kApplyMB + j];
#pragma unroll
                for (int i = 0; i < RPT; ++i) acc[i][j] = fma(q[i], w, acc[i][j]);
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

// ---------------------------------------------------------------- launchers
static int grid_for(int64_t count, int threads) {
    int64_t b = (count + threads - 1) / threads;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (int)b;
}

int gram_tile_rows(int ncol, int s) {
    const int ldt = odd_ld(ncol);
    const int budget = 40 * 1024;
    for (int tr = 64; tr >= 8; tr >>= 1)
        if ((size_t)tr * (ldt + 2 * s) * 8 <= (size_t)budget) return tr;
    return 8;
}

size_t gram_lds_bytes(int ncol, int s, int tr) {
    const size_t tile = (size_t)tr * (odd_ld(ncol) + s) * 8;
    const size_t red = (size_t)kWaves * 64 * s * 8;
    return tile > red ? tile : red;
}

size_t correct_lds_bytes(int ncol, int s, int kmax, int tr) {
    (void)kmax;
    const int k = ncol - s;
    const size_t tile = ((size_t)tr * (odd_ld(ncol) + 2 * s) + (size_t)k * s + (size_t)s * s) * 8;
    const size_t red = (size_t)kWaves * 64 * s * 8;
    return tile > red ? tile : red;
}

int correct_tile_rows(int ncol, int s) {
    for (int tr = 16; tr >= 8; tr >>= 1)
        if (correct_lds_bytes(ncol, s, 0, tr) <= 60 * 1024) return tr;
    return 8;
}

static int cpt_for(int ncol) {
    const int c = (ncol + 63) / 64;
    if (c <= 1) return 1;
    if (c <= 2) return 2;
    if (c <= 4) return 4;
    return 8;
}

#define ORTH_DISPATCH_CPT(KERNEL, S, CPT, ARGS, LDS, GRID, ST)                                  \
    switch (CPT) {                                                                              \
        case 1: hipLaunchKernelGGL((KERNEL<S, 1>), GRID, dim3(kThreads), LDS, ST, ARGS); break; \
        case 2: hipLaunchKernelGGL((KERNEL<S, 2>), GRID, dim3(kThreads), LDS, ST, ARGS); break; \
        case 4: hipLaunchKernelGGL((KERNEL<S, 4>), GRID, dim3(kThreads), LDS, ST, ARGS); break; \
        default:                                                                                \
            if (8 * S > 64) return hipErrorInvalidValue;                                        \
            hipLaunchKernelGGL((KERNEL<S, (8 * S > 64 ? 1 : 8)>), GRID, dim3(kThreads), LDS, ST, \
                               ARGS);                                                           \
            break;                                                                              \
    }

template <int S>
static hipError_t gram_s(const GramArgs &a, hipStream_t st) {
    const int ncol = a.k + S;
    const size_t lds = gram_lds_bytes(ncol, S, a.tile_rows);
    const dim3 grid(a.geom.nchunks());
    ORTH_DISPATCH_CPT(k_gram, S, cpt_for(ncol), a, lds, grid, st);
    return hipGetLastError();
}

template <int S>
static hipError_t correct_s(const CorrectArgs &a, hipStream_t st) {
    const int ncol = a.k + S;
    const size_t lds = correct_lds_bytes(ncol, S, a.kmax, a.tile_rows);
    const dim3 grid(a.geom.nchunks());
    ORTH_DISPATCH_CPT(k_correct, S, cpt_for(ncol), a, lds, grid, st);
    return hipGetLastError();
}

hipError_t launch_gram(int s, const GramArgs &a, int, hipStream_t st) {
    switch (s) {
        case 1: return gram_s<1>(a, st);
        case 2: return gram_s<2>(a, st);
        case 4: return gram_s<4>(a, st);
        case 8: return gram_s<8>(a, st);
        case 16: return gram_s<16>(a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_correct(int s, const CorrectArgs &a, int, hipStream_t st) {
    switch (s) {
        case 1: return correct_s<1>(a, st);
        case 2: return correct_s<2>(a, st);
        case 4: return correct_s<4>(a, st);
        case 8: return correct_s<8>(a, st);
        case 16: return correct_s<16>(a, st);
    }
    return hipErrorInvalidValue;
}

template <int S>
static hipError_t chol_s(const CholArgs &a, hipStream_t st) {
    const size_t lds = ((size_t)(a.k + S) * S + 3 * S * S) * 8;
    hipLaunchKernelGGL((k_chol<S>), dim3(a.geom.nleaf), dim3(kThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_chol(int s, const CholArgs &a, hipStream_t st) {
    switch (s) {
        case 1: return chol_s<1>(a, st);
        case 2: return chol_s<2>(a, st);
        case 4: return chol_s<4>(a, st);
        case 8: return chol_s<8>(a, st);
        case 16: return chol_s<16>(a, st);
    }
    return hipErrorInvalidValue;
}

template <int S>
static hipError_t finalize_s(const FinalizeArgs &a, hipStream_t st) {
    const size_t lds = ((size_t)2 * a.k * S + 2 * S * S) * 8;
    constexpr int RPT = S >= 16 ? 1 : 2;
    hipLaunchKernelGGL((k_finalize<S, RPT>), dim3(a.geom.nchunks()), dim3(kThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_finalize(int s, const FinalizeArgs &a, hipStream_t st) {
    switch (s) {
        case 1: return finalize_s<1>(a, st);
        case 2: return finalize_s<2>(a, st);
        case 4: return finalize_s<4>(a, st);
        case 8: return finalize_s<8>(a, st);
        case 16: return finalize_s<16>(a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_apply(const ApplyArgs &a, hipStream_t st) {
    if (a.m < 1 || a.m > kApplyMB) return hipErrorInvalidValue;
    const size_t lds = (size_t)a.k * kApplyMB * 8;
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

hipError_t launch_laplacian(const double *X, int64_t ldx, double *Y, int64_t ldy, int32_t s,
                            int32_t nx, int32_t ny, int32_t nz, double shift, hipStream_t st) {
    const int64_t total = (int64_t)nx * ny * nz * s;
    hipLaunchKernelGGL(k_laplacian, dim3(grid_for(total, 256)), dim3(256), 0, st, X, ldx, Y, ldy, s,
                       nx, ny, nz, shift);
    return hipGetLastError();
}

hipError_t launch_copy(const double *src, double *dst, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy, dim3(grid_for(count / 2 + 1, 256)), dim3(256), 0, st, src, dst, count);
    return hipGetLastError();
}

}  // namespace orth
