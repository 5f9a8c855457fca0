// Deflation at the reduction level (Sec. 3.1).  The Cholesky factorisation
// cannot tell a rank-deficient G - P^T P from a full-rank one, so the
// reduction level's first sweep takes its eigen decomposition
// V Lambda V^T instead and keeps the t eigenvalues above
// delta^2 ||X||_F^2 (||X||_F^2 = trace G at the reduction level):
//
//   t = s:  the plain Cholesky step (nothing changes for a full-rank block);
//   t < s:  N1 = [Lambda~^{1/2} V~^T; 0] (kept eigenvalues in decreasing
//           order, each eigenvector turned so that its entry of largest
//           magnitude is positive), u1 = (x - q P1) W with
//           W = [V~ Lambda~^{-1/2}, 0]: the row-update kernel computes
//           x - q P1 (identity in place of N1^{-1}) and k_defl_rows applies W.
//
// The second sweep factors the t kept columns of u1 by Cholesky (its other
// columns are exact zeros), N2 = diag(L, 0), and the combination is the
// usual P = P1 + P2 N1, N = N2 N1, with full products since N1 is not
// triangular after a drop.  The block keeps width s: the dropped columns of
// U and rows of N are zero, and a later zero column is dropped again.
//
// The eigen decomposition is cyclic Jacobi with the round-robin ordering:
// s/2 disjoint rotations per round, s - 1 rounds per sweep, until every
// off-diagonal entry is negligible against its diagonal pair, at most
// kJacobiSweeps sweeps (so every launch ends).

#include <hip/hip_runtime.h>

#include "orth_deflate.h"

namespace orth {
namespace {

constexpr int kJacobiSweeps = 14;

__device__ void defl_fail(const CholArgs &a, int column) {
    if (atomicCAS(&a.status->code, 0, 3) == 0) {
        a.status->level = a.level;
        a.status->leaf = 0;
        a.status->sweep = a.sweep;
        a.status->column = column;
        a.status->instance = a.instance;
    }
}

// Upper Cholesky N^T N = sm on the leading m x m block (sm is overwritten),
// then N^{-1} by back substitution; entries outside the block stay as the
// caller set them.  Returns 0, or 1 + the failing column.
template <int S>
__device__ int defl_chol(double *sm, double *nm, double *ni, int m, int &bad) {
    const int tid = threadIdx.x;
    for (int kk = 0; kk < m; ++kk) {
        if (tid == kk) {
            const double piv = sm[kk * S + kk];
            if (!(piv > 0.0) || !isfinite(piv)) bad = kk + 1;
            else nm[kk * S + kk] = sqrt(piv);
        }
        __syncthreads();
        if (bad) break;
        if (tid > kk && tid < m) nm[kk * S + tid] = sm[kk * S + tid] / nm[kk * S + kk];
        __syncthreads();
        if (tid > kk && tid < m) {
            const double nkj = nm[kk * S + tid];
            for (int i = kk + 1; i <= tid; ++i) sm[i * S + tid] -= nm[kk * S + i] * nkj;
        }
        __syncthreads();
    }
    const int b = bad;
    if (b) return b;
    if (tid < m) {
        const int j = tid;
        ni[j * S + j] = 1.0 / nm[j * S + j];
        for (int i = j - 1; i >= 0; --i) {
            double t = 0.0;
            for (int l = i + 1; l <= j; ++l) t = fma(nm[i * S + l], ni[l * S + j], t);
            ni[i * S + j] = -t / nm[i * S + i];
        }
    }
    __syncthreads();
    return 0;
}

// rotation (c, s) with J = [[c, s], [-s, c]] on (p, q) such that J^T A J has
// a zero (p, q) entry (the symmetric 2 x 2 Schur decomposition, Golub & Van
// Loan Sec. 8.5); the smaller of the two angles
__device__ void sym_schur2(double app, double apq, double aqq, double &c, double &s) {
    c = 1.0;
    s = 0.0;
    if (apq == 0.0) return;
    const double tau = (aqq - app) / (2.0 * apq);
    double t;
    if (fabs(tau) > 1e150) t = 0.5 / tau;
    else t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    c = 1.0 / sqrt(1.0 + t * t);
    s = t * c;
}

template <int S>
__global__ __launch_bounds__(kThreads) void k_defl(CholArgs a, DeflArgs d) {
    if (a.status->code != 0) return;
    __shared__ double gs[S * S], sm[S * S], AV[2 * S * S], nm[S * S], ni[S * S], n1[S * S];
    double *A = AV, *V = AV + S * S;
    __shared__ double lam[S], rc[S], rsn[S];
    __shared__ int rp[S], rq[S], ord[S];
    __shared__ int t_sh, bad, done;
    const int tid = threadIdx.x;
    const int k = a.k, ncol = k + S;
    DeflState *ds = d.state;
    double *rec = a.small;                       // one reduction node: record 0
    double *recP1 = rec;
    double *recN1 = rec + (int64_t)a.kmax * S;
    double *recN1i = recN1 + S * S;
    double *recP2 = recN1i + S * S;
    double *recN2i = recP2 + (int64_t)a.kmax * S;
    double *recP = a.sweep == 1 ? recP1 : recP2;
    if (tid == 0) {
        bad = 0;
        t_sh = a.sweep == 1 ? S : S - ds->dropped;
    }
    // 1. fixed-order sum of the Gram slots: P -> record, G -> LDS
    for (int e = tid; e < ncol * S; e += kThreads) {
        double v = 0.0;
        for (int q = 0; q < a.slots_last; ++q) v += a.partials[(int64_t)q * a.part_stride + e];
        if (e < k * S) recP[e] = v;
        else gs[e - k * S] = v;
    }
    if (a.sweep == 2)
        for (int e = tid; e < S * S; e += kThreads) n1[e] = recN1[e];
    __syncthreads();
    // 2. sm = G - P^T P, P staged through LDS (A and V, free until step 3)
    //    in chunks of 2 S rows; each entry sums its rows in increasing order
    constexpr int EPT = (S * S + kThreads - 1) / kThreads;
    constexpr int CB = 2 * S;
    double acc[EPT];
#pragma unroll
    for (int m = 0; m < EPT; ++m) acc[m] = 0.0;
    for (int c0 = 0; c0 < k; c0 += CB) {
        const int cb = k - c0 < CB ? k - c0 : CB;
        for (int e = tid; e < cb * S; e += kThreads) A[e] = recP[(int64_t)c0 * S + e];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < EPT; ++m) {
            const int e = tid + kThreads * m;
            if (e < S * S) {
                const int i = e / S, j = e % S;
                for (int c = 0; c < cb; ++c) acc[m] = fma(A[c * S + i], A[c * S + j], acc[m]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
        const int e = tid + kThreads * m;
        if (e < S * S) {
            sm[e] = gs[e] - acc[m];
            nm[e] = 0.0;
            ni[e] = 0.0;
        }
    }
    __syncthreads();

    if (a.sweep == 1) {
        // 3. eigen decomposition of the symmetric part of sm
        for (int e = tid; e < S * S; e += kThreads) {
            const int i = e / S, j = e % S;
            A[e] = 0.5 * (sm[i * S + j] + sm[j * S + i]);
            V[e] = i == j ? 1.0 : 0.0;
        }
        __syncthreads();
        if constexpr (S > 1) {
            constexpr int H = S / 2;
            if (tid == 0) done = 0;
            for (int sw = 0; sw < kJacobiSweeps; ++sw) {
                for (int r = 0; r < S - 1; ++r) {
                    // round r pairs S-1 with r and (r + i) with (r - i) mod S-1
                    if (tid < H) {
                        int p = tid == 0 ? S - 1 : (r + tid) % (S - 1);
                        int q = tid == 0 ? r : (r - tid + (S - 1)) % (S - 1);
                        if (p > q) { const int x = p; p = q; q = x; }
                        double c, sn;
                        sym_schur2(A[p * S + p], A[p * S + q], A[q * S + q], c, sn);
                        rp[tid] = p;
                        rq[tid] = q;
                        rc[tid] = c;
                        rsn[tid] = sn;
                    }
                    __syncthreads();
                    for (int w = tid; w < H * S; w += kThreads) {        // rows: J^T A
                        const int i = w / S, j = w % S;
                        const int p = rp[i], q = rq[i];
                        const double c = rc[i], sn = rsn[i];
                        const double ap = A[p * S + j], aq = A[q * S + j];
                        A[p * S + j] = c * ap - sn * aq;
                        A[q * S + j] = sn * ap + c * aq;
                    }
                    __syncthreads();
                    for (int w = tid; w < H * S; w += kThreads) {        // columns: A J, V J
                        const int i = w / S, j = w % S;
                        const int p = rp[i], q = rq[i];
                        const double c = rc[i], sn = rsn[i];
                        const double ap = A[j * S + p], aq = A[j * S + q];
                        A[j * S + p] = c * ap - sn * aq;
                        A[j * S + q] = sn * ap + c * aq;
                        const double vp = V[j * S + p], vq = V[j * S + q];
                        V[j * S + p] = c * vp - sn * vq;
                        V[j * S + q] = sn * vp + c * vq;
                    }
                    __syncthreads();
                }
                // converged: every off-diagonal entry below 1e-18 of the
                // geometric mean of its diagonal pair (or exactly zero)
                if (tid == 0) {
                    int conv = 1;
                    for (int i = 0; i < S && conv; ++i)
                        for (int j = i + 1; j < S; ++j) {
                            const double a = fabs(A[i * S + j]);
                            if (a != 0.0 && !(a <= 1e-18 * sqrt(fabs(A[i * S + i]) * fabs(A[j * S + j])))) {
                                conv = 0;
                                break;
                            }
                        }
                    done = conv;
                }
                __syncthreads();
                if (done) break;
            }
        }
        // 4. order, rank, and the breakdown of a non-finite block
        if (tid == 0) {
            double tr = 0.0;
            for (int j = 0; j < S; ++j) tr += gs[j * S + j];
            bool fin = isfinite(tr);
            for (int j = 0; j < S; ++j) {
                lam[j] = A[j * S + j];
                fin = fin && isfinite(lam[j]);
                ord[j] = j;
            }
            for (int j = 1; j < S; ++j) {                   // stable, decreasing
                const int o = ord[j];
                int i = j;
                while (i > 0 && lam[ord[i - 1]] < lam[o]) {
                    ord[i] = ord[i - 1];
                    --i;
                }
                ord[i] = o;
            }
            const double thr = d.delta2 * tr;
            int t = 0;
            while (t < S && lam[ord[t]] > thr) ++t;
            t_sh = t;
            if (!fin) bad = 1;
        }
        __syncthreads();
        if (bad) {
            if (tid == 0) defl_fail(a, 0);
            return;
        }
        const int t = t_sh;
        if (t == S) {
            const int b = defl_chol<S>(sm, nm, ni, S, bad);
            if (b) {
                if (tid == 0) defl_fail(a, b - 1);
                return;
            }
        } else {
            double *W = defl_W(ds);
            if (tid < S) {
                const int r = tid;
                if (r < t) {
                    const int col = ord[r];
                    int im = 0;
                    for (int l = 1; l < S; ++l)
                        if (fabs(V[l * S + col]) > fabs(V[im * S + col])) im = l;
                    const double sg = V[im * S + col] < 0.0 ? -1.0 : 1.0;
                    const double sq = sqrt(lam[col]);
                    for (int l = 0; l < S; ++l) {
                        const double v = sg * V[l * S + col];
                        nm[r * S + l] = sq * v;
                        W[l * S + r] = v / sq;
                    }
                } else {
                    for (int l = 0; l < S; ++l) W[l * S + r] = 0.0;
                }
                ni[r * S + r] = 1.0;             // the row update forms x - q P1
            }
            __syncthreads();
        }
        for (int e = tid; e < S * S; e += kThreads) {
            recN1[e] = nm[e];
            recN1i[e] = ni[e];
        }
        if (tid == 0) {
            ds->dropped = S - t;
            if (t < S) {
                ds->steps += 1;
                ds->total += S - t;
            }
        }
    } else {
        // 3'. Cholesky of the t kept columns (the others are exact zeros)
        const int t = t_sh;
        const int b = defl_chol<S>(sm, nm, ni, t, bad);
        if (b) {
            if (tid == 0) defl_fail(a, b - 1);
            return;
        }
        for (int e = tid; e < S * S; e += kThreads) recN2i[e] = ni[e];
    }
    if (a.sweep != a.final_sweep) return;
    // 5. [P; N]: one sweep -> (P1, N1); two -> P = P1 + P2 N1, N = N2 N1
    for (int e = tid; e < ncol * S; e += kThreads) {
        const int c = e / S, j = e % S;
        double v;
        if (c < k) {
            v = recP1[e];
            if (a.sweep == 2)
                for (int i = 0; i < S; ++i) v = fma(recP2[(int64_t)c * S + i], n1[i * S + j], v);
        } else {
            const int i = c - k;
            if (a.sweep == 1) {
                v = nm[i * S + j];
            } else {
                v = 0.0;
                for (int l = i; l < S; ++l) v = fma(nm[i * S + l], n1[l * S + j], v);
            }
        }
        if (a.Yout) a.Yout[(int64_t)j * a.ldy + c] = v;
        if (c < k) {
            if (a.H) a.H[(int64_t)j * a.ldh + c] = v;
        } else if (a.R) {
            a.R[(int64_t)j * a.ldr + (c - k)] = v;
        }
    }
}

template <int S>
__global__ __launch_bounds__(kThreads) void k_defl_rows(DeflRowArgs a) {
    if (a.status->code != 0 || a.state->dropped == 0) return;
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r >= a.geom.nrows) return;
    const int64_t pr = a.geom.map.phys(r);
    const double *W = defl_W(a.state);
    double x[S];
#pragma unroll
    for (int l = 0; l < S; ++l) x[l] = a.U[(int64_t)l * a.ld + pr];
#pragma unroll
    for (int j = 0; j < S; ++j) {
        double y = 0.0;
#pragma unroll
        for (int l = 0; l < S; ++l) y = fma(x[l], W[l * S + j], y);
        a.U[(int64_t)j * a.ld + pr] = y;
    }
}

template <int S>
hipError_t defl_s(const CholArgs &a, const DeflArgs &d, hipStream_t st) {
    hipLaunchKernelGGL((k_defl<S>), dim3(1), dim3(kThreads), 0, st, a, d);
    return hipGetLastError();
}

template <int S>
hipError_t defl_rows_s(const DeflRowArgs &a, hipStream_t st) {
    const int64_t blocks = (a.geom.nrows + kThreads - 1) / kThreads;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_defl_rows<S>), dim3((unsigned)blocks), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_defl(int s, const CholArgs &a, const DeflArgs &d, hipStream_t st) {
    if (a.nleaf != 1 || !d.state || !a.small || !a.partials) return hipErrorInvalidValue;
    switch (s) {
        case 1: return defl_s<1>(a, d, st);
        case 2: return defl_s<2>(a, d, st);
        case 4: return defl_s<4>(a, d, st);
        case 8: return defl_s<8>(a, d, st);
        case 16: return defl_s<16>(a, d, st);
    }
    // s = 32: orth_set_deflation refuses it (the eigen solver holds s <= 16 columns)
    return hipErrorInvalidValue;
}

hipError_t launch_defl_rows(int s, const DeflRowArgs &a, hipStream_t st) {
    if (!a.U || !a.state) return hipErrorInvalidValue;
    switch (s) {
        case 1: return defl_rows_s<1>(a, st);
        case 2: return defl_rows_s<2>(a, st);
        case 4: return defl_rows_s<4>(a, st);
        case 8: return defl_rows_s<8>(a, st);
        case 16: return defl_rows_s<16>(a, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace orth
