// Workgroup-level dense complex kernels for CDNA4 (64-wide wavefronts, 256-thread workgroups):
// partial LU with row pivoting restricted to the fully-summed rows, split into its panel step
// (one workgroup) and its trailing-update tiles (any number of workgroups), so that a large
// front can spread its Schur-complement update over the whole chip while small fronts run the
// whole factorisation inside one workgroup.
//
// Complex arithmetic here uses four real multiplies per product, so the rounding of every
// product is the textbook one (the large fronts' trailing GEMM on the matrix cores, gemm.cuh,
// uses three).
#pragma once

#include <hip/hip_runtime.h>

namespace cr {

template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// c - a * b
template <typename T>
__device__ __forceinline__ cx<T> cfms(cx<T> c, cx<T> a, cx<T> b) {
    return {c.re - a.re * b.re + a.im * b.im, c.im - a.re * b.im - a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> crecip(cx<T> a) {
    // 1 / a with scaling against overflow (Smith's algorithm)
    if (fabs(a.re) >= fabs(a.im)) {
        T r = a.im / a.re, d = a.re + a.im * r;
        return {T(1) / d, -r / d};
    } else {
        T r = a.re / a.im, d = a.im + a.re * r;
        return {r / d, T(-1) / d};
    }
}
template <typename T>
__device__ __forceinline__ T cabs1(cx<T> a) { return fabs(a.re) + fabs(a.im); }

constexpr int kWG = 256;     // threads per workgroup (4 wavefronts)
constexpr int kNB = 16;      // panel width
constexpr int kTile = 64;    // trailing-update tile (64 x 64, 4 x 4 per thread)

// Element loop over [0, n) with stride NT in batches of U iterations: the loads of all U
// iterations are issued before any of their stores. The callers' iterations touch disjoint
// addresses, which the compiler cannot prove, so without the batching every iteration would
// wait for its own loads.
template <int NT, int U, typename Load, typename Store>
__device__ __forceinline__ void batched_for(int n, Load ld, Store st) {
    using V = decltype(ld(0));
    for (int base = threadIdx.x; base < n; base += NT * U) {
        V v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + u * NT;
            if (e < n) v[u] = ld(e);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + u * NT;
            if (e < n) st(e, v[u]);
        }
    }
}

// Workgroup barrier that orders LDS only: outstanding global loads (prefetches of later steps)
// stay in flight across it, which a full __syncthreads (a workgroup fence on all memory) would
// wait for. For points where the threads share data through LDS alone; the global loads must
// then be global-address-space ones (flat loads are counted with LDS accesses and would be
// waited for as well).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Workgroup max-reduction of (value, index); lowest index wins ties. Uses red_v/red_i in LDS
// (kWG / 64 + 1 entries each). All threads receive the result.
template <typename T>
__device__ __forceinline__ void wg_argmax(T v, int i, T* red_v, int* red_i, T& out_v, int& out_i) {
    const int t = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) {
        T ov = __shfl_xor(v, off);
        int oi = __shfl_xor(i, off);
        if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
    }
    if ((t & 63) == 0) { red_v[t >> 6] = v; red_i[t >> 6] = i; }
    __syncthreads();
    if (t == 0) {
        T bv = red_v[0];
        int bi = red_i[0];
        for (int w = 1; w < kWG / 64; ++w)
            if (red_v[w] > bv || (red_v[w] == bv && red_i[w] < bi)) { bv = red_v[w]; bi = red_i[w]; }
        red_v[kWG / 64] = bv;
        red_i[kWG / 64] = bi;
    }
    __syncthreads();
    out_v = red_v[kWG / 64];
    out_i = red_i[kWG / 64];
    __syncthreads();
}

// Composite permutation of one panel's row swaps (at most 2 kNB rows are touched).
struct SwapShared {
    int row[2 * kNB], src[2 * kNB], n;
};

template <typename T>
struct LuShared {
    cx<T> a[kTile][kNB + 1];     // trailing update: L panel tile
    cx<T> b[kNB][kTile + 1];     // trailing update: U panel tile
    T red_v[kWG / 64 + 1];
    int red_i[kWG / 64 + 1];
    SwapShared sw;
};
// the part of LuShared a panel step uses (pivot search and row swaps)
template <typename T>
struct PanelShared {
    T red_v[kWG / 64 + 1];
    int red_i[kWG / 64 + 1];
    SwapShared sw;
};

// The row swaps ipiv[k0..k1) (row k exchanged with row ipiv[k], in order; absolute row indices)
// applied to columns [ca, cb) of A as one gather: thread 0 composes them into "row r now holds
// old row src(r)" for the touched rows, then every moved entry is read before any is written
// (a barrier between), so a panel's swaps cost one memory round trip on these columns instead
// of one per swap. Same result as the swaps one by one. Called by the whole workgroup; ipiv
// entries must be visible to thread 0 (it wrote them, or they come from an earlier kernel).
template <typename T, int U = 4>
__device__ void wg_apply_swaps(cx<T>* __restrict__ A, int lda, const int* ipiv, int k0, int k1, int ca, int cb,
                               SwapShared& sw) {
    const int t = threadIdx.x;
    __syncthreads();   // an earlier call's readers of sw are done
    if (t < 64) {
        // the first wave composes them in registers: lane j < 16 stands for row k0 + j, lane
        // 16 + j for row ipiv[k0 + j] (one load for all of them); val = the row whose value is
        // at the lane's row so far. A row held by several lanes is tracked in the lowest one.
        const int nk = k1 - k0;
        int row = -1;
        if (t < nk) row = k0 + t;
        else if (t >= kNB && t - kNB < nk) row = ipiv[k0 + t - kNB];
        int val = row;
        for (int k = 0; k < nk; ++k) {
            const int rk = k0 + k, pk = __builtin_amdgcn_readlane(row, kNB + k);
            if (pk == rk) continue;
            const int la = __ffsll((unsigned long long)__ballot(row == rk)) - 1;
            const int lb = __ffsll((unsigned long long)__ballot(row == pk)) - 1;
            const int va = __builtin_amdgcn_readlane(val, la), vb = __builtin_amdgcn_readlane(val, lb);
            if (t == la) val = vb;
            if (t == lb) val = va;
        }
        bool dup = false;
        for (int q = 0; q < 2 * kNB; ++q) {
            const int other = __builtin_amdgcn_readlane(row, q);
            dup = dup || (q < t && other == row);
        }
        const bool keep = row >= 0 && !dup && val != row;
        const unsigned long long kb = (unsigned long long)__ballot(keep);
        const int slot = __builtin_amdgcn_mbcnt_hi((unsigned)(kb >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)kb, 0u));
        if (keep) {
            sw.row[slot] = row;
            sw.src[slot] = val;
        }
        if (t == 0) sw.n = __popcll(kb);
    }
    __syncthreads();
    const int n = sw.n;
    if (n == 0) return;
    // whole columns per pass: every source row of a column is read before any row of that column
    // is written
    const int cpi = (U * kWG) / n;
    for (int c0 = ca; c0 < cb; c0 += cpi) {
        const int tot = n * min(cpi, cb - c0);
        cx<T> v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = u * kWG + t;
            if (e < tot) v[u] = A[sw.src[e % n] + (size_t)(c0 + e / n) * lda];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = u * kWG + t;
            if (e < tot) A[sw.row[e % n] + (size_t)(c0 + e / n) * lda] = v[u];
        }
        __syncthreads();
    }
}

// Panel step of the partial LU of the m x m column-major A (leading dimension lda): factor
// columns [k0, k1) over rows [k0, rend) with pivots searched among the fully-summed rows [k, p)
// (ipiv[k] = row swapped with k; the swap is applied to columns [sw0, sw1) of the two rows: the
// panel's own columns at once, the others composed into one gather after the panel),
// then, when trsm is set, U12 rows [k0, k1) x columns [k1, m) = L_kk^{-1} A (unit lower).
// rend = m factors the whole panel; rend = p leaves the rows [p, m), which never take part in
// pivoting, to a separate triangular solve with the panel's U (the large-front row-strip
// kernel). On long columns one pass over the rows scales the column, applies its rank-1
// update to the rest of the panel and takes the next column's pivot candidates on the way.
// Pivots with cabs1 <= tiny (or NaN) are replaced by tiny in their own direction and counted
// in *nperturb.
// LEAN = true keeps the long-column loop register-light (one row in flight per thread) for
// callers whose occupancy matters more than memory-level parallelism (the reduced-model sweep).
template <typename T, bool LEAN = false, typename SH = LuShared<T>>
__device__ __forceinline__ void wg_panel(cx<T>* __restrict__ A, int lda, int m, int p, int k0, int k1, int* __restrict__ ipiv, T tiny,
                         int* nperturb, SH& sh, int sw0, int sw1, bool trsm, int rend) {
    const int t = threadIdx.x;
    T best = T(-1);
    int bi = k0;
    bool have = false;   // pivot candidates of column k already taken by the previous pass
    for (int k = k0; k < k1; ++k) {
        if (!have) {
            best = T(-1);
            bi = k;
            for (int i = k + t; i < p; i += kWG) {
                const T v = cabs1(A[i + (size_t)k * lda]);
                if (v > best) { best = v; bi = i; }
            }
        }
        T pv;
        int pi;
        wg_argmax(best, bi, sh.red_v, sh.red_i, pv, pi);
        if (t == 0) ipiv[k] = pi;
        if (pi != k) {
            // the panel's own columns now; the other columns of [sw0, sw1) after the panel
            for (int j = max(sw0, k0) + t; j < min(sw1, k1); j += kWG) {
                cx<T> x = A[k + (size_t)j * lda], y = A[pi + (size_t)j * lda];
                A[k + (size_t)j * lda] = y;
                A[pi + (size_t)j * lda] = x;
            }
            __syncthreads();
        }
        cx<T> d = A[k + (size_t)k * lda];
        if (!(pv > tiny)) {   // tiny or NaN pivot: static perturbation
            T mag = cabs1(d);
            if (mag > T(0)) { d.re = d.re / mag * tiny; d.im = d.im / mag * tiny; }
            else { d.re = tiny; d.im = T(0); }
            __syncthreads();
            if (t == 0) { A[k + (size_t)k * lda] = d; atomicAdd(nperturb, 1); }
        }
        const cx<T> r = crecip(d);
        const int nc = k1 - k - 1;
        const int rows = rend - k - 1;
        have = rows >= kWG;
        if (have) {
            // long columns: one pass per column, one row per thread at a time; the row of U is
            // held in registers and the next column's pivot candidates are taken on the way
            cx<T> u[kNB - 1];
#pragma unroll
            for (int jj = 0; jj < kNB - 1; ++jj) u[jj] = jj < nc ? A[k + (size_t)(k + 1 + jj) * lda] : cx<T>{T(0), T(0)};
            best = T(-1);
            bi = k + 1;
            for (int i = k + 1 + t; i < rend; i += kWG) {
                if constexpr (LEAN) {
                    const cx<T> l = cmul(A[i + (size_t)k * lda], r);
                    A[i + (size_t)k * lda] = l;
#pragma unroll
                    for (int jj = 0; jj < kNB - 1; ++jj) {
                        if (jj < nc) {
                            cx<T>& x = A[i + (size_t)(k + 1 + jj) * lda];
                            const cx<T> y = cfms(x, l, u[jj]);
                            x = y;
                            if (jj == 0 && i < p) {
                                const T v = cabs1(y);
                                if (v > best) { best = v; bi = i; }
                            }
                        }
                    }
                    continue;
                }
                // the row's entries are all loaded before any store (one memory latency per row)
                const cx<T> a0 = A[i + (size_t)k * lda];
                cx<T> xv[kNB - 1];
#pragma unroll
                for (int jj = 0; jj < kNB - 1; ++jj)
                    xv[jj] = jj < nc ? A[i + (size_t)(k + 1 + jj) * lda] : cx<T>{T(0), T(0)};
                const cx<T> l = cmul(a0, r);
                A[i + (size_t)k * lda] = l;
#pragma unroll
                for (int jj = 0; jj < kNB - 1; ++jj) {
                    if (jj < nc) {
                        const cx<T> y = cfms(xv[jj], l, u[jj]);
                        A[i + (size_t)(k + 1 + jj) * lda] = y;
                        if (jj == 0 && i < p) {
                            const T v = cabs1(y);
                            if (v > best) { best = v; bi = i; }
                        }
                    }
                }
            }
        } else {
            // short columns (small fronts, reduced models): scale, then every (row, column) pair
            // of the rank-1 update is one thread's work so that all threads stay busy
            for (int i = k + 1 + t; i < rend; i += kWG) A[i + (size_t)k * lda] = cmul(A[i + (size_t)k * lda], r);
            __syncthreads();
            batched_for<kWG, 4>(rows * nc,
                [&](int e) {
                    const int i = k + 1 + e % rows, j = k + 1 + e / rows;
                    return cfms(A[i + (size_t)j * lda], A[i + (size_t)k * lda], A[k + (size_t)j * lda]);
                },
                [&](int e, cx<T> v) { A[k + 1 + e % rows + (size_t)(k + 1 + e / rows) * lda] = v; });
        }
        __syncthreads();
    }
    wg_apply_swaps<T, LEAN ? 1 : 4>(A, lda, ipiv, k0, k1, sw0, min(sw1, k0), sh.sw);
    wg_apply_swaps<T, LEAN ? 1 : 4>(A, lda, ipiv, k0, k1, max(sw0, k1), sw1, sh.sw);
    if (!trsm || k1 >= m) return;
    // U12 block: solve L_kk X = A[k0:k1, k1:m] (unit lower)
    for (int j = k1 + t; j < m; j += kWG) {
        cx<T> x[kNB];
#pragma unroll
        for (int r = 0; r < kNB; ++r)
            if (k0 + r < k1) x[r] = A[k0 + r + (size_t)j * lda];
#pragma unroll
        for (int r = 0; r < kNB; ++r) {
            if (k0 + r >= k1) break;
#pragma unroll
            for (int s = 0; s < r; ++s) x[r] = cfms(x[r], A[k0 + r + (size_t)(k0 + s) * lda], x[s]);
        }
#pragma unroll
        for (int r = 0; r < kNB; ++r)
            if (k0 + r < k1) A[k0 + r + (size_t)j * lda] = x[r];
    }
    __syncthreads();
}

// Panel step as wg_panel with rend = p and no U12 solve, for panels whose fully-summed rows fit in
// LDS (p - k0 <= R): the 16 columns are staged in LDS, factored there, and written back; the row
// swaps reach the block's earlier columns [sw0, k0) in global memory after the panel, composed
// into one gather. Same arithmetic, same order.
template <typename T, int R, typename SH>
__device__ void wg_panel_lds(cx<T>* __restrict__ A, int lda, int p, int k0, int k1, int* __restrict__ ipiv, T tiny,
                             int* nperturb, SH& sh, cx<T> (*P)[kNB + 1], int sw0) {
    const int t = threadIdx.x;
    const int rows = p - k0, nb = k1 - k0;
    // eight loads in flight per thread (a plain strided loop waits for each load in turn)
    batched_for<kWG, 8>(rows * nb, [&](int e) { return A[k0 + e % rows + (size_t)(k0 + e / rows) * lda]; },
                        [&](int e, cx<T> v) { P[e % rows][e / rows] = v; });
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
        T best = T(-1);
        int bi = k;
        for (int i = k + t; i < rows; i += kWG) {
            const T v = cabs1(P[i][k]);
            if (v > best) { best = v; bi = i; }
        }
        T pv;
        int pi;
        wg_argmax(best, bi, sh.red_v, sh.red_i, pv, pi);
        if (t == 0) ipiv[k0 + k] = k0 + pi;
        if (pi != k) {
            if (t < nb) { cx<T> x = P[k][t]; P[k][t] = P[pi][t]; P[pi][t] = x; }
            __syncthreads();
        }
        cx<T> d = P[k][k];
        if (!(pv > tiny)) {
            T mag = cabs1(d);
            if (mag > T(0)) { d.re = d.re / mag * tiny; d.im = d.im / mag * tiny; }
            else { d.re = tiny; d.im = T(0); }
            __syncthreads();
            if (t == 0) { P[k][k] = d; atomicAdd(nperturb, 1); }
        }
        const cx<T> r = crecip(d);
        for (int i = k + 1 + t; i < rows; i += kWG) {
            const cx<T> l = cmul(P[i][k], r);
            P[i][k] = l;
            for (int jj = k + 1; jj < nb; ++jj) P[i][jj] = cfms(P[i][jj], l, P[k][jj]);
        }
        __syncthreads();
    }
    for (int e = t; e < rows * nb; e += kWG) {
        const int i = e % rows, c = e / rows;
        A[k0 + i + (size_t)(k0 + c) * lda] = P[i][c];
    }
    // the swaps reach the block's earlier columns once, after the panel
    wg_apply_swaps<T>(A, lda, ipiv, k0, k1, sw0, k0, sh.sw);
}

// One 64 x 64 tile (rows i0.., columns j0..) of the trailing update
// A[k1:m, k1:m] -= A[k1:m, k0:k1] A[k0:k1, k1:m], with k1 - k0 <= kNB.
template <typename T, int U = kTile * kNB / kWG>
__device__ void wg_tile_update(cx<T>* __restrict__ A, int lda, int m, int k0, int k1, int i0, int j0, LuShared<T>& sh) {
    const int t = threadIdx.x;
    const int nbk = k1 - k0;
    const int tx = t & 15, ty = t >> 4;   // 16 x 16 threads, 4 x 4 each
    // both tiles staged with U loads in flight per thread (all of them by default)
    batched_for<kWG, U>(kTile * kNB,
        [&](int e) {
            const int r = e % kTile, c = e / kTile;
            return (i0 + r < m && c < nbk) ? A[i0 + r + (size_t)(k0 + c) * lda] : cx<T>{T(0), T(0)};
        },
        [&](int e, cx<T> v) { sh.a[e % kTile][e / kTile] = v; });
    batched_for<kWG, U>(kTile * kNB,
        [&](int e) {
            const int r = e % kNB, c = e / kNB;
            return (j0 + c < m && r < nbk) ? A[k0 + r + (size_t)(j0 + c) * lda] : cx<T>{T(0), T(0)};
        },
        [&](int e, cx<T> v) { sh.b[e % kNB][e / kNB] = v; });
    __syncthreads();
    cx<T> acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = {T(0), T(0)};
    for (int c = 0; c < nbk; ++c) {
        cx<T> av[4], bv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) av[a] = sh.a[tx + 16 * a][c];
#pragma unroll
        for (int b = 0; b < 4; ++b) bv[b] = sh.b[c][ty + 16 * b];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                acc[a][b].re += av[a].re * bv[b].re - av[a].im * bv[b].im;
                acc[a][b].im += av[a].re * bv[b].im + av[a].im * bv[b].re;
            }
    }
    // all 16 entries of the thread are loaded before the first store (one memory latency)
    cx<T> cv[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = i0 + tx + 16 * a, j = j0 + ty + 16 * b;
            cv[a][b] = (i < m && j < m) ? A[i + (size_t)j * lda] : cx<T>{T(0), T(0)};
        }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = i0 + tx + 16 * a, j = j0 + ty + 16 * b;
            if (i < m && j < m) A[i + (size_t)j * lda] = {cv[a][b].re - acc[a][b].re, cv[a][b].im - acc[a][b].im};
        }
    __syncthreads();
}

// Whole partial LU inside one workgroup: P A = L U on the leading p columns with the trailing
// (m-p) x (m-p) block replaced by its Schur complement.
template <typename T, bool LEAN = false>
__device__ void wg_getrf(cx<T>* __restrict__ A, int lda, int m, int p, int* __restrict__ ipiv, T tiny, int* nperturb,
                         LuShared<T>& sh) {
    for (int k0 = 0; k0 < p; k0 += kNB) {
        const int k1 = min(k0 + kNB, p);
        wg_panel<T, LEAN>(A, lda, m, p, k0, k1, ipiv, tiny, nperturb, sh, 0, m, true, m);
        if (k1 >= m) break;
        const int tiles = (m - k1 + kTile - 1) / kTile;
        for (int tile = 0; tile < tiles * tiles; ++tile)
            wg_tile_update<T, LEAN ? 1 : kTile * kNB / kWG>(A, lda, m, k0, k1, k1 + (tile % tiles) * kTile,
                                                              k1 + (tile / tiles) * kTile, sh);
    }
    __syncthreads();
}

}  // namespace cr
