// Blocked trailing updates of a large front's partial LU on the matrix cores.
//
// A large front is factored by outer blocks of kOB = 128 pivot columns, each made of eight
// 16-column panels (wg_panel). Inside an outer block the updates are deferred: before panel s
// the L-shaped strip it needs -- its own 16 columns below the diagonal and its 16 rows to the
// right -- receives the contributions of panels 0..s-1 of the block (wg_strip_update); after
// the block the trailing matrix receives all 128 columns at once, S -= L21 U12 with K = 128
// (wg_gemm_tile), a complex GEMM on MFMA: v_mfma_f32_16x16x4f32 for complex-FP32 fronts and
// v_mfma_f64_16x16x4f64 for FP64 fronts, each complex product as three real products
// (Ar Br, Ai Bi, (Ar + Ai)(Br + Bi)): a quarter fewer matrix-core operations than four, with a
// normwise error bound of the same order (the imaginary part's bound grows from
// |Ar||Bi| + |Ai||Br| to (|Ar| + |Ai|)(|Br| + |Bi|) times u); the factor is only ever used
// under FP64 refinement with a certified backward error.
//
// MFMA 16x16x4 operand layout (lane l of a 64-wide wavefront, checked on gfx950): A[i][k] with
// i = l % 16, k = l / 16; B[k][j] with j = l % 16, k = l / 16; the accumulator's item r is
// D[4 (l / 16) + r][l % 16] for the FP32 instruction and D[l / 16 + 4 r][l % 16] for FP64.
#pragma once

#include "dense.cuh"

namespace cr {

constexpr int kOB = 128;     // outer block (pivot columns per trailing GEMM)
constexpr int kST = 64;      // strip update tile (rows or columns per workgroup)
constexpr int kGT = 64;      // GEMM output tile (kGT x kGT per workgroup, 32 x 32 per wave)

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct MfmaAcc;
template <>
struct MfmaAcc<float> {
    typedef f32x4 type;
    static __device__ __forceinline__ f32x4 mfma(float a, float b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <>
struct MfmaAcc<double> {
    typedef f64x4 type;
    static __device__ __forceinline__ f64x4 mfma(double a, double b, f64x4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <typename T, int TW = kGT>
struct GemmShared {
    static constexpr int KC = sizeof(T) == 4 ? 32 : 16;   // K chunk staged in LDS (35 KB at TW = 64, 68 KB at 128)
    cx<T> a[KC][TW + 4];   // L21 chunk, a[k][i]
    // U12 chunk, b[k][j]; it is written along k (one column of U12 per lane run), so an odd row
    // pitch spreads those writes over the LDS banks
    cx<T> b[KC][TW + 1];
};

// C[i0:i0+TW, j0:j0+TW] -= A[i0:, k0:k0+K] A[k0:k0+K, j0:] inside the m x m column-major front
// (rows >= m and columns >= jend <= m are skipped). 256 threads; wave w owns the (TW/2) x (TW/2) quadrant
// ((TW/2) (w & 1), (TW/2) (w >> 1)) as BI x BI blocks of 16 x 16 (BI = TW / 32).
template <typename T, int TW = kGT>
__device__ void wg_gemm_tile(cx<T>* __restrict__ A, int lda, int m, int k0, int K, int i0, int j0,
                             GemmShared<T, TW>& sh, int jend) {
    typedef typename MfmaAcc<T>::type acc_t;
    constexpr int BI = TW / 32;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wi = (TW / 2) * (w & 1), wj = (TW / 2) * (w >> 1);
    // three real products per complex one: p1 = sum Ar Br, p2 = sum Ai Bi,
    // p3 = sum (Ar + Ai)(Br + Bi); Re = p1 - p2, Im = p3 - p1 - p2
    acc_t p1[BI][BI], p2[BI][BI], p3[BI][BI];
#pragma unroll
    for (int a = 0; a < BI; ++a)
#pragma unroll
        for (int b = 0; b < BI; ++b) {
            p1[a][b] = acc_t{0, 0, 0, 0};
            p2[a][b] = acc_t{0, 0, 0, 0};
            p3[a][b] = acc_t{0, 0, 0, 0};
        }
    constexpr int KC = GemmShared<T, TW>::KC;
    constexpr int PER = TW * KC / kWG;   // entries of each operand chunk per thread
    // software pipeline: chunk c + 1 is fetched into registers (all loads in flight together)
    // while chunk c is multiplied from LDS
    cx<T> ra[PER], rb[PER];
    auto fetch = [&](int kc) {
        const int nk = min(KC, K - kc);
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + q * kWG;
            const int i = e % TW, k = e / TW;
            ra[q] = (k < nk && i0 + i < m) ? A[i0 + i + (size_t)(k0 + kc + k) * lda] : cx<T>{T(0), T(0)};
            const int k2 = e % KC, j = e / KC;
            rb[q] = (k2 < nk && j0 + j < jend) ? A[k0 + kc + k2 + (size_t)(j0 + j) * lda] : cx<T>{T(0), T(0)};
        }
    };
    fetch(0);
    for (int kc = 0; kc < K; kc += KC) {
        const int nk = min(KC, K - kc);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + q * kWG;
            sh.a[e / TW][e % TW] = ra[q];   // L21 chunk, coalesced down the columns
            sh.b[e % KC][e / KC] = rb[q];   // U12 chunk, coalesced down the columns
        }
        __syncthreads();
        if (kc + KC < K) fetch(kc + KC);
        const int li = lane & 15, lk = lane >> 4;
        for (int kk = 0; kk < nk; kk += 4) {
            cx<T> av[BI], bv[BI];
            T as[BI], bs[BI];
#pragma unroll
            for (int a = 0; a < BI; ++a) {
                av[a] = sh.a[kk + lk][wi + 16 * a + li];
                as[a] = av[a].re + av[a].im;
            }
#pragma unroll
            for (int b = 0; b < BI; ++b) {
                bv[b] = sh.b[kk + lk][wj + 16 * b + li];
                bs[b] = bv[b].re + bv[b].im;
            }
#pragma unroll
            for (int a = 0; a < BI; ++a)
#pragma unroll
                for (int b = 0; b < BI; ++b) {
                    p1[a][b] = MfmaAcc<T>::mfma(av[a].re, bv[b].re, p1[a][b]);
                    p2[a][b] = MfmaAcc<T>::mfma(av[a].im, bv[b].im, p2[a][b]);
                    p3[a][b] = MfmaAcc<T>::mfma(as[a], bs[b], p3[a][b]);
                }
        }
    }
    // epilogue: each lane owns 4 rows of one column per 16 x 16 block; a row of blocks at a time,
    // all of its C entries are loaded before the first store (entries outside the front read a
    // clamped address and are not stored)
    const int lj = lane & 15;
#pragma unroll
    for (int a = 0; a < BI; ++a) {
        cx<T> cv[BI][4];
#pragma unroll
        for (int b = 0; b < BI; ++b) {
            const int j = min(j0 + wj + 16 * b + lj, jend - 1);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = min(i0 + wi + 16 * a + MfmaAcc<T>::row(lane, r), m - 1);
                cv[b][r] = A[i + (size_t)j * lda];
            }
        }
#pragma unroll
        for (int b = 0; b < BI; ++b) {
            const int j = j0 + wj + 16 * b + lj;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wi + 16 * a + MfmaAcc<T>::row(lane, r);
                if (i < m && j < jend) {
                    cx<T> x = cv[b][r];
                    const T s1 = p1[a][b][r], s2 = p2[a][b][r];
                    x.re -= s1 - s2;
                    x.im -= p3[a][b][r] - s1 - s2;
                    A[i + (size_t)j * lda] = x;
                }
            }
        }
    }
}

// C[r0:r0+nr, c0:c0+nc] -= A[r0:r0+nr, k0:k0+K] A[k0:k0+K, c0:c0+nc] with nr, nc <= 64 and K a
// multiple of 4 (the in-block updates of the panel chain): 16 x 16 output tiles, one per wave at a
// time, on the matrix cores with three real products per complex one (as the trailing GEMM);
// each wave loads its operands straight from memory, eight K steps at a time, so the update
// needs no LDS and no workgroup barrier. The caller synchronises before another wave reads C.
template <typename T>
__device__ void wg_strip_update(cx<T>* __restrict__ A, int lda, int r0, int nr, int c0, int nc, int k0, int K) {
    typedef typename MfmaAcc<T>::type acc_t;
    constexpr int H = 8;   // K steps (of 4) whose loads are issued together
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int tr = (nr + 15) / 16, ntile = tr * ((nc + 15) / 16);
    for (int tile = wave; tile < ntile; tile += kWG / 64) {
        const int R0 = r0 + 16 * (tile % tr), C0 = c0 + 16 * (tile / tr);
        const int trows = min(16, r0 + nr - R0), tcols = min(16, c0 + nc - C0);
        acc_t p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
        const bool aok = li < trows, bok = li < tcols;
        for (int s0 = 0; 4 * s0 < K; s0 += H) {
            cx<T> av[H], bv[H];
#pragma unroll
            for (int s = 0; s < H; ++s) {
                const int k = 4 * (s0 + s) + lk;
                const bool kin = k < K;
                av[s] = (aok && kin) ? A[R0 + li + (size_t)(k0 + k) * lda] : cx<T>{T(0), T(0)};
                bv[s] = (bok && kin) ? A[k0 + k + (size_t)(C0 + li) * lda] : cx<T>{T(0), T(0)};
            }
#pragma unroll
            for (int s = 0; s < H; ++s) {
                p1 = MfmaAcc<T>::mfma(av[s].re, bv[s].re, p1);
                p2 = MfmaAcc<T>::mfma(av[s].im, bv[s].im, p2);
                p3 = MfmaAcc<T>::mfma(av[s].re + av[s].im, bv[s].re + bv[s].im, p3);
            }
        }
        // item r of the accumulators: row MfmaAcc<T>::row(lane, r) of the tile, column li
        cx<T> cv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ro = MfmaAcc<T>::row(lane, r);
            cv[r] = (ro < trows && li < tcols) ? A[R0 + ro + (size_t)(C0 + li) * lda] : cx<T>{T(0), T(0)};
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ro = MfmaAcc<T>::row(lane, r);
            if (ro < trows && li < tcols) {
                const T s1 = p1[r], s2 = p2[r];
                cv[r].re -= s1 - s2;
                cv[r].im -= p3[r] - s1 - s2;
                A[R0 + ro + (size_t)(C0 + li) * lda] = cv[r];
            }
        }
    }
}

}  // namespace cr
