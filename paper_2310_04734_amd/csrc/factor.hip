// Multifrontal LU of the shifted system A_j = K~ - w_j^2 M~ (Jacobi-scaled) at an expansion
// point, and the forward/backward solves with the stored factor (paper Section 3.3: one
// factorisation per expansion point, reused for every moment at that point).
//
// Fronts are processed level by level from the leaves of the nested-dissection tree to the
// root; every front of a level is one workgroup:
//   assemble:  zero the m x m front, scatter the original entries (formed in FP64 and rounded
//              to the factor precision), add the children's contribution blocks (pull, in
//              child order: deterministic, no atomics);
//   factor:    partial LU of the p fully-summed columns (pivoting among fully-summed rows),
//              leaving the Schur complement in the trailing (m-p) x (m-p) block.
// The fronts stay resident in one device arena (HBM is large enough that the contribution
// blocks need no stack), so the L and U parts are the factor used by the solves.
#include <algorithm>
#include <utility>
#include <chrono>
#include <cmath>

#include <cstring>

#include "dense.cuh"
#include "gemm.cuh"
#include "internal.h"
#include "util.cuh"

namespace cr {
namespace {

// Front assembly: zero the front, scatter A = K~ - sigma M~ (FP64, rounded once), add the
// children's contribution blocks. gridDim.y workgroups share one front by owning the parent
// columns j with j % gridDim.y == blockIdx.y, so no two workgroups touch the same entry.
template <typename T>
__global__ void __launch_bounds__(kWG) k_front_assemble(
    const int32_t* __restrict__ level_fronts, const int32_t* __restrict__ fsize, const int64_t* __restrict__ front_off,
    const int32_t* __restrict__ child_off, const int32_t* __restrict__ child_list, const int32_t* __restrict__ npiv,
    const int64_t* __restrict__ cmap_off, const int32_t* __restrict__ cmap, const int64_t* __restrict__ ent_off,
    const int64_t* __restrict__ ent_src, const int32_t* __restrict__ ent_dst, const zd* __restrict__ K,
    const zd* __restrict__ M, double sigma, cx<T>* __restrict__ arena) {
    const int f = level_fronts[blockIdx.x];
    const int m = fsize[f];
    const int S = gridDim.y, y = blockIdx.y, t = threadIdx.x;
    cx<T>* F = arena + front_off[f];
    if (S == 1) {
        const int64_t mm = (int64_t)m * m;
        for (int64_t e = t; e < mm; e += kWG) F[e] = {T(0), T(0)};
    } else {
        for (int j = y; j < m; j += S)
            for (int i = t; i < m; i += kWG) F[i + (size_t)j * m] = {T(0), T(0)};
    }
    __syncthreads();
    const int64_t e0 = ent_off[f];
    const int ne = (int)(ent_off[f + 1] - e0);
    auto mine = [&](int32_t d) { return S == 1 || (d / m) % S == y; };
    batched_for<kWG, 4>(ne,
        [&](int e) {
            const int32_t d = ent_dst[e0 + e];
            if (!mine(d)) return cx<T>{T(0), T(0)};
            const int64_t s = ent_src[e0 + e];
            const zd k = K[s], mv = M[s];
            return cx<T>{T(k.re - sigma * mv.re), T(k.im - sigma * mv.im)};   // FP64, rounded once
        },
        [&](int e, cx<T> v) {
            const int32_t d = ent_dst[e0 + e];
            if (mine(d)) F[d] = v;
        });
    __syncthreads();
    for (int ci = child_off[f]; ci < child_off[f + 1]; ++ci) {
        const int c = child_list[ci];
        const int mc = fsize[c], pc = npiv[c], nc = mc - pc;
        const cx<T>* C = arena + front_off[c];
        const int32_t* map = cmap + cmap_off[c];
        if (S == 1) {
            batched_for<kWG, 4>(nc * nc,
                [&](int e) {
                    const int r = e % nc, s = e / nc;
                    const cx<T> v = C[(pc + r) + (size_t)(pc + s) * mc], d = F[map[r] + (size_t)map[s] * m];
                    return cx<T>{d.re + v.re, d.im + v.im};
                },
                [&](int e, cx<T> v) { F[map[e % nc] + (size_t)map[e / nc] * m] = v; });
        } else {
            for (int s = 0; s < nc; ++s) {
                const int js = map[s];
                if (js % S != y) continue;
                const cx<T>* Cs = C + pc + (size_t)(pc + s) * mc;
                cx<T>* Fs = F + (size_t)js * m;
                batched_for<kWG, 4>(nc,
                    [&](int r) {
                        const cx<T> v = Cs[r], d = Fs[map[r]];
                        return cx<T>{d.re + v.re, d.im + v.im};
                    },
                    [&](int r, cx<T> v) { Fs[map[r]] = v; });
            }
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(kWG) k_front_factor(const int32_t* __restrict__ level_fronts,
                                                     const int32_t* __restrict__ fsize, const int32_t* __restrict__ npiv,
                                                     const int32_t* __restrict__ first, const int64_t* __restrict__ front_off,
                                                     cx<T>* __restrict__ arena, int32_t* __restrict__ ipiv, T tiny,
                                                     int32_t* nperturb, const int32_t* __restrict__ big) {
    __shared__ LuShared<T> sh;
    const int f = level_fronts[blockIdx.x];
    const int m = fsize[f], p = npiv[f];
    if (p == 0 || big[f]) return;
    wg_getrf<T>(arena + front_off[f], m, m, p, ipiv + first[f], tiny, nperturb, sh);
}

// Large fronts are factored by 128-column blocks of eight 16-column panels. Panel step j:
//   k_front_colstrip  (not the block's first panel) the panel's columns, rows [k0, m), receive
//                     the block's earlier panels (rows tiled over workgroups);
//   k_front_panel     one workgroup per front: pivots, scaling and the in-panel updates of the
//                     fully-summed rows [k0, p), row swaps inside the block's columns [K0, k1);
//   k_front_rowstrip  the panel's row swaps on the block's later columns [k1, Kend), whose rows
//                     [k0, k1) then receive the block's earlier panels and are solved with the
//                     panel's unit-lower diagonal block; and rows [p, m) of the panel (one row per
//                     thread) solved with its U.
// After the block's panels:
//   k_front_rowblock  the same row strips for the columns outside the block (the block's swaps
//                     on [0, K0) and on [Kend, m), and U12 rows of the block on [Kend, m));
//   k_front_gemm      trailing GEMM with K = 128 on MFMA: first the next block's columns, then
//                     the rest on the context's second stream, where it overlaps the next
//                     block's panels (which touch only that block's columns).
// Swaps are applied before any update of the current block touches the swapped rows outside
// the block's columns, so both rows of a swap are always in the same state.
// LDS for a panel's fully-summed rows (16 columns): small enough that the panel fits on a
// compute unit beside one workgroup of the overlapping trailing GEMM
constexpr int kPanelLdsBytes = 48 * 1024;

// Two variants, each taking the fronts of its class and skipping the others: LDS = true stages
// the fully-summed rows in LDS (p - k0 <= panel_lds_rows<T>()); LDS = false works on the front in
// memory and needs only the small shared state, so it fits on a compute unit beside the trailing
// GEMM's workgroups of the previous block.
template <typename T>
constexpr int panel_lds_rows() { return kPanelLdsBytes / (int)sizeof(cx<T>) / (kNB + 1); }

// Split panels (k_front_panel_coop below): rows per workgroup, limits, and the class rule shared
// by the host and the kernels.
constexpr int kCoopRPT = 1;          // panel rows per thread (in registers)
constexpr int kCoopRows = kCoopRPT * kWG;   // panel rows per workgroup
constexpr int kCoopMaxG = 64;        // workgroups per front
constexpr int kCoopMaxWG = 256;      // workgroups of one launch (all must be resident at once)
constexpr int kCoopSpins = 1 << 20;  // default bound on a barrier wait's polls (about a second)

__host__ __device__ constexpr int coop_groups(int rows, int min_rows) {
    return (min_rows > 0 && rows >= min_rows && (rows + kCoopRows - 1) / kCoopRows <= kCoopMaxG)
               ? (rows + kCoopRows - 1) / kCoopRows : 0;
}

template <typename T, bool LDS>
__global__ void __launch_bounds__(kWG) k_front_panel(const int32_t* __restrict__ big_list, int step, int split_rows,
                                                    const int32_t* __restrict__ fsize, const int32_t* __restrict__ npiv,
                                                    const int32_t* __restrict__ first, const int64_t* __restrict__ front_off,
                                                    cx<T>* __restrict__ arena, int32_t* __restrict__ ipiv, T tiny,
                                                    int32_t* nperturb) {
    constexpr int R = panel_lds_rows<T>();
    __shared__ PanelShared<T> sh;
    const int f = big_list[blockIdx.x];
    const int m = fsize[f], p = npiv[f], k0 = step * kNB;
    if (k0 >= p || (p - k0 <= R) != LDS || coop_groups(p - k0, split_rows) > 0) return;
    const int K0 = (k0 / kOB) * kOB, k1 = min(k0 + kNB, p);
    if constexpr (LDS) {
        __shared__ cx<T> pl[R][kNB + 1];
        wg_panel_lds<T, R>(arena + front_off[f], m, p, k0, k1, ipiv + first[f], tiny, nperturb, sh, pl, K0);
    } else {
        wg_panel<T>(arena + front_off[f], m, m, p, k0, k1, ipiv + first[f], tiny, nperturb, sh, K0, k1, false, p);
    }
}

// Panels with many fully-summed rows (p - k0 >= the system's split threshold) are spread over
// G = ceil((p - k0) / kCoopRows) workgroups that hold the panel's rows in registers (kCoopRPT
// rows of 16 entries per thread) for the whole panel: the single-workgroup panel streams the
// panel through one compute unit once per column, at that unit's share of the L2 bandwidth.
// Per column k, every workgroup publishes its best pivot candidate (largest cabs1 among its rows
// >= k, lowest row on ties), that candidate's row and, for the owner of row k, row k itself;
// after a barrier of the front's G workgroups every workgroup takes the same winner (same rule),
// swaps, scales and updates its rows with the same complex operations in the same order as
// wg_panel, so the factor is bit-identical to the single-workgroup panel. Publications
// alternate between two buffers by column parity: a workgroup reads column k's buffer before it
// arrives at column k + 1's barrier, which no workgroup passes before every one has arrived.
template <typename T>
struct CoopPub {
    T cand_v[2][kCoopMaxG];
    int cand_i[2][kCoopMaxG];
    cx<T> row[2][kCoopMaxG][kNB];
    cx<T> rowk[2][kNB];
};
constexpr int kCoopBarInts = 64;   // per front slot: one 64-bit barrier word (256-byte stride)

// Barrier of one front's G workgroups on one 64-bit word: generation << 32 | arrivals. The
// arrival is one acquire-release add that returns the generation; the last arrival advances the
// generation and takes the arrivals back to zero with a second (release) add; the others poll
// the generation (acquire). Stores before the barrier are visible to every workgroup of the
// front after it. Waits are bounded: a wait past max_polls polls sets *fail and returns false,
// so the kernel always ends (the host then reports the factor invalid).
__device__ bool coop_barrier(unsigned long long* word, int G, int max_polls, int* fail) {
    __shared__ int ok_sh;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned long long old = __hip_atomic_fetch_add(word, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned g0 = (unsigned)(old >> 32);
        if ((unsigned)old == (unsigned)(G - 1)) {
            __hip_atomic_fetch_add(word, (1ull << 32) - (unsigned long long)G, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            for (int spins = 0;
                 (unsigned)(__hip_atomic_load(word, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >> 32) == g0;) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > max_polls) {
                    atomicExch(fail, 1);
                    ok = 0;
                    break;
                }
            }
        }
        ok_sh = ok;
    }
    __syncthreads();
    return ok_sh != 0;
}

// f(integral_constant<int, 0>), ..., f(integral_constant<int, N - 1>) in order
template <typename F, int... I>
__device__ __forceinline__ void static_for_seq(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_seq(f, std::make_integer_sequence<int, N>{});
}

// grid (max G, fronts of the level): blockIdx.y = the front's slot in pub and bar
template <typename T>
__global__ void __launch_bounds__(kWG) k_front_panel_coop(const int32_t* __restrict__ big_list, int step, int min_rows,
                                                         const int32_t* __restrict__ fsize, const int32_t* __restrict__ npiv,
                                                         const int32_t* __restrict__ first, const int64_t* __restrict__ front_off,
                                                         cx<T>* __restrict__ arena, int32_t* __restrict__ ipiv, T tiny,
                                                         int32_t* nperturb, CoopPub<T>* __restrict__ pub, int* bar, int max_polls,
                                                         int* fail) {
    __shared__ PanelShared<T> sh;
    // the column's publications, loaded in one batch after its barrier
    __shared__ T s_cv[kCoopMaxG];
    __shared__ int s_ci[kCoopMaxG];
    __shared__ cx<T> s_rows[kCoopMaxG + 1][kNB];   // candidate rows, then row k
    __shared__ T s_pv;
    __shared__ int s_pi, s_w;
    const int f = big_list[blockIdx.y];
    const int m = fsize[f], p = npiv[f], k0 = step * kNB;
    if (k0 >= p) return;
    const int G = coop_groups(p - k0, min_rows);
    const int g = blockIdx.x, t = threadIdx.x;
    if (g >= G) return;
    const int K0 = (k0 / kOB) * kOB, k1 = min(k0 + kNB, p), nb = k1 - k0;
    cx<T>* A = arena + front_off[f];
    int32_t* piv = ipiv + first[f];
    // identity pivots first: a factorisation whose barrier wait failed (then every later split
    // panel is skipped) still leaves valid rows for the swap kernels that follow; the workgroup
    // overwrites them with the real pivots as it goes
    if (g == 0 && t < nb) piv[k0 + t] = k0 + t;
    if (__hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    CoopPub<T>& P = pub[blockIdx.y];
    unsigned long long* word = reinterpret_cast<unsigned long long*>(bar + kCoopBarInts * blockIdx.y);
    int ir[kCoopRPT];
    bool own[kCoopRPT];
    cx<T> a[kCoopRPT][kNB];
    T best = T(-1);
    int bi = k0;
#pragma unroll
    for (int r = 0; r < kCoopRPT; ++r) {
        ir[r] = k0 + g * kCoopRows + r * kWG + t;
        own[r] = ir[r] < p;
#pragma unroll
        for (int jj = 0; jj < kNB; ++jj)
            a[r][jj] = (own[r] && jj < nb) ? A[ir[r] + (size_t)(k0 + jj) * m] : cx<T>{T(0), T(0)};
        if (own[r]) {
            const T v = cabs1(a[r][0]);
            if (v > best) { best = v; bi = ir[r]; }
        }
    }
    bool alive = true;   // false once a barrier wait has failed: the remaining steps are skipped
    // the column steps are instantiated one by one (a loop, even under an unroll pragma, is too
    // large for the unroller and would index a[][] at run time, i.e. in scratch)
    static_for<kNB>([&](auto kc) {
        constexpr int kk = decltype(kc)::value;
        const int k = k0 + kk, par = kk & 1;
        if (kk < nb && alive) {
            T lv;
            int li;
            wg_argmax(best, bi, sh.red_v, sh.red_i, lv, li);
            if (t == 0) {
                P.cand_v[par][g] = lv;
                P.cand_i[par][g] = li;
            }
#pragma unroll
            for (int r = 0; r < kCoopRPT; ++r) {
                if (own[r] && ir[r] == li)
#pragma unroll
                    for (int jj = 0; jj < kNB; ++jj) P.row[par][g][jj] = a[r][jj];
                if (own[r] && ir[r] == k)
#pragma unroll
                    for (int jj = 0; jj < kNB; ++jj) P.rowk[par][jj] = a[r][jj];
            }
            alive = coop_barrier(word, G, max_polls, fail);   // uniform over the workgroup
        }
        if (kk < nb && alive) {
            // every candidate with its row, and row k, in one round of loads
            if (t < G) {
                s_cv[t] = P.cand_v[par][t];
                s_ci[t] = P.cand_i[par][t];
            }
            for (int e = t; e < (G + 1) * kNB; e += kWG)
                s_rows[e / kNB][e % kNB] = e < G * kNB ? P.row[par][e / kNB][e % kNB] : P.rowk[par][e % kNB];
            __syncthreads();
            if (t < 64) {
                // the winner among the G candidates: largest value, lowest row
                T v = T(-1);
                int i = k, w = 0;
                if (t < G) {
                    v = s_cv[t];
                    i = s_ci[t];
                    w = t;
                }
                for (int off = 32; off > 0; off >>= 1) {
                    const T ov = __shfl_xor(v, off);
                    const int oi = __shfl_xor(i, off), ow = __shfl_xor(w, off);
                    if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; w = ow; }
                }
                if (t == 0) { s_pv = v; s_pi = i; s_w = w; }
            }
            __syncthreads();
            const T pv = s_pv;
            const int pi = min(max(s_pi, k), p - 1);   // always so; the clamp keeps ipiv a row of the front
            const cx<T>* su = s_rows[pi == k ? G : s_w];   // the pivot row
            // the swap of rows k and pi over the panel's columns
#pragma unroll
            for (int r = 0; r < kCoopRPT; ++r) {
                if (own[r] && ir[r] == k) {
#pragma unroll
                    for (int jj = 0; jj < kNB; ++jj) a[r][jj] = su[jj];
                } else if (own[r] && ir[r] == pi) {
#pragma unroll
                    for (int jj = 0; jj < kNB; ++jj) a[r][jj] = s_rows[G][jj];
                }
            }
            cx<T> d = su[kk];
            if (!(pv > tiny)) {   // tiny or NaN pivot: static perturbation (as wg_panel)
                const T mag = cabs1(d);
                if (mag > T(0)) { d.re = d.re / mag * tiny; d.im = d.im / mag * tiny; }
                else { d.re = tiny; d.im = T(0); }
                if (g == 0 && t == 0) atomicAdd(nperturb, 1);
            }
            if (g == 0 && t == 0) piv[k] = pi;
            const cx<T> rc = crecip(d);
            best = T(-1);
            bi = k + 1;
#pragma unroll
            for (int r = 0; r < kCoopRPT; ++r) {
                if (own[r] && ir[r] == k) a[r][kk] = d;
                if (own[r] && ir[r] > k) {
                    const cx<T> l = cmul(a[r][kk], rc);
                    a[r][kk] = l;
#pragma unroll
                    for (int jj = kk + 1; jj < kNB; ++jj) a[r][jj] = cfms(a[r][jj], l, su[jj]);
                    if (kk + 1 < kNB) {
                        const T v = cabs1(a[r][kk + 1]);
                        if (v > best) { best = v; bi = ir[r]; }
                    }
                }
            }
            __syncthreads();   // s_rows is rewritten at the next column
        }
    });
    if (!alive) return;
#pragma unroll
    for (int r = 0; r < kCoopRPT; ++r)
#pragma unroll
        for (int jj = 0; jj < kNB; ++jj)
            if (own[r] && jj < nb) A[ir[r] + (size_t)(k0 + jj) * m] = a[r][jj];
    // the panel's swaps on the block's earlier columns [K0, k0), as one gather
    if (g == 0 && K0 < k0) wg_apply_swaps<T>(A, m, piv, k0, k1, K0, k0, sh.sw);
}

// rows of a column strip per workgroup (8 MFMA tiles, two per wave; 128 rows measured faster than
// 32 or 64 on the fuselage fronts, while the row tiles keep kST = 64 columns)
constexpr int kCST = 128;

template <typename T>
__global__ void __launch_bounds__(kWG) k_front_colstrip(const int32_t* __restrict__ big_list, int step,
                                                       const int32_t* __restrict__ fsize, const int32_t* __restrict__ npiv,
                                                       const int64_t* __restrict__ front_off, cx<T>* __restrict__ arena) {
    const int f = big_list[blockIdx.y];
    const int m = fsize[f], p = npiv[f], k0 = step * kNB;
    if (k0 >= p) return;
    const int K0 = (k0 / kOB) * kOB, k1 = min(k0 + kNB, p);
    const int r0 = k0 + kCST * (int)blockIdx.x;
    if (r0 >= m || K0 == k0) return;
    wg_strip_update<T>(arena + front_off[f], m, r0, min(kCST, m - r0), k0, k1 - k0, K0, k0 - K0);
}

// col[k0:k0+16] <- D^{-1} col[k0:k0+16] with D unit lower (d, zero-padded past the panel's nb
// rows and columns). The rows past nb solve to their own values (their rows of d are zero) and
// are written back unchanged, so that loads and stores need no row conditions: the caller owns
// the whole column, and rows at or past m (only possible past nb) are clamped to row m - 1,
// which is past the panel as well. Branch-free stores keep the compiler from hoisting every
// read of d into registers.
template <typename T>
__device__ __forceinline__ void unit_lower16(cx<T>* __restrict__ col, int k0, int m, const cx<T> (*d)[kNB + 1]) {
    cx<T> xv[kNB];
#pragma unroll
    for (int r = 0; r < kNB; ++r) xv[r] = col[min(k0 + r, m - 1)];
#pragma unroll
    for (int r = 1; r < kNB; ++r)
#pragma unroll
        for (int q = 0; q < r; ++q) xv[r] = cfms(xv[r], d[r][q], xv[q]);
#pragma unroll
    for (int r = 0; r < kNB; ++r) col[min(k0 + r, m - 1)] = xv[r];
}

template <typename T>
struct RowStripShared {
    cx<T> d[kNB][kNB + 1];   // diagonal block of the panel (unit-lower L and U)
    cx<T> rd[kNB];           // reciprocals of U's diagonal
    SwapShared sw;
};

// The row strip of a panel (see above). The factorisation defers the part outside the panel's
// 128-column block (the swaps on columns [0, K0) and [Kend, m), and the rows [k0, k1) of U12
// beyond the block) to k_front_rowblock, so that the next block's panels touch only their own
// columns: the right columns here are [k1, Kend) with Kend the block's last pivot column + 1.
// The rows [p, m) part loads and stores without column conditions (a conditional store after the
// unrolled solve makes the compiler hoist every read of the diagonal block into registers and
// spill): a panel of nb < 16 columns reads column k0 + nb - 1 in place of the missing ones and
// stores the columns in reverse order, so that column's last store is its own solved value.
template <typename T>
__global__ void __launch_bounds__(kWG) k_front_rowstrip(const int32_t* __restrict__ big_list, int step,
                                                       const int32_t* __restrict__ fsize, const int32_t* __restrict__ npiv,
                                                       const int32_t* __restrict__ first, const int64_t* __restrict__ front_off,
                                                       const int32_t* __restrict__ ipiv, cx<T>* __restrict__ arena) {
    __shared__ RowStripShared<T> sh;
    const int f = big_list[blockIdx.y];
    const int m = fsize[f], p = npiv[f], k0 = step * kNB;
    if (k0 >= p) return;
    const int K0 = (k0 / kOB) * kOB, k1 = min(k0 + kNB, p), nb = k1 - k0;
    const int Kend = min(K0 + kOB, p);
    const int nright = (Kend - k1 + kST - 1) / kST, nleft = 0;
    const int nl21 = (m - p + kWG - 1) / kWG;
    const int x = blockIdx.x;
    if (x >= nright + nleft + nl21) return;
    const int t = threadIdx.x;
    cx<T>* A = arena + front_off[f];
    if (x >= nright + nleft) {
        // rows [p, m) of the panel: l_ik = (a_ik - sum_{k' < k} l_ik' u_k'k) / u_kk, in the
        // order and rounding of the panel's own column steps
        for (int e = t; e < kNB * kNB; e += kWG) {
            const int i = e % kNB, k = e / kNB;
            sh.d[i][k] = (i < nb && k < nb) ? A[k0 + i + (size_t)(k0 + k) * m] : cx<T>{T(1), T(0)};
        }
        __syncthreads();
        if (t < kNB) sh.rd[t] = crecip(sh.d[t][t]);
        __syncthreads();
        const int i = p + kWG * (x - nright - nleft) + t;
        if (i >= m) return;
        cx<T> a[kNB];
#pragma unroll
        for (int k = 0; k < kNB; ++k) a[k] = A[i + (size_t)(k0 + min(k, nb - 1)) * m];
#pragma unroll
        for (int k = 0; k < kNB; ++k) {
            a[k] = cmul(a[k], sh.rd[k]);
#pragma unroll
            for (int j = k + 1; j < kNB; ++j) a[j] = cfms(a[j], a[k], sh.d[k][j]);
        }
#pragma unroll
        for (int k = kNB - 1; k >= 0; --k) A[i + (size_t)(k0 + min(k, nb - 1)) * m] = a[k];
        return;
    }
    const bool right = x < nright;
    const int c0 = right ? k1 + kST * x : kST * (x - nright);
    const int nc = right ? min(kST, Kend - c0) : min(kST, K0 - c0);
    const int32_t* pv = ipiv + first[f];
    // the panel's swaps on this tile's columns, composed into one gather
    wg_apply_swaps<T>(A, m, pv, k0, k1, c0, c0 + nc, sh.sw);
    if (!right) return;
    if (K0 < k0) wg_strip_update<T>(A, m, k0, nb, c0, nc, K0, k0 - K0);
    for (int e = t; e < kNB * kNB; e += kWG) {
        const int i = e % kNB, k = e / kNB;
        sh.d[i][k] = (i < nb && k < nb) ? A[k0 + i + (size_t)(k0 + k) * m] : cx<T>{T(0), T(0)};
    }
    __syncthreads();
    if (t < nc) unit_lower16(A + (size_t)(c0 + t) * m, k0, m, sh.d);
}

// After the panels of 128-column block [K0, K1): the block's deferred row strips, one
// workgroup per 64-column tile (blockIdx.y = front). Right tiles (columns [K1, m)): for each
// panel in order, its row swaps, then rows [k0, k1) receive the block's earlier panels and are
// solved with the panel's unit-lower diagonal block (U12 = L_bb^{-1} P A[K0:K1, K1:m]). Left tiles
// (columns [0, K0), the factor's earlier L columns): the block's row swaps. Every tile's work
// stays in its own columns.
template <typename T>
__global__ void __launch_bounds__(kWG) k_front_rowblock(const int32_t* __restrict__ big_list, int blk,
                                                       const int32_t* __restrict__ fsize, const int32_t* __restrict__ npiv,
                                                       const int32_t* __restrict__ first, const int64_t* __restrict__ front_off,
                                                       const int32_t* __restrict__ ipiv, cx<T>* __restrict__ arena) {
    __shared__ RowStripShared<T> sh;
    const int f = big_list[blockIdx.y];
    const int m = fsize[f], p = npiv[f], K0 = blk * kOB;
    if (K0 >= p) return;
    const int K1 = min(K0 + kOB, p);
    const int nright = (m - K1 + kST - 1) / kST, nleft = (K0 + kST - 1) / kST;
    const int x = blockIdx.x;
    if (x >= nright + nleft) return;
    const int t = threadIdx.x;
    cx<T>* A = arena + front_off[f];
    const int32_t* pv = ipiv + first[f];
    const bool right = x < nright;
    const int c0 = right ? K1 + kST * x : kST * (x - nright);
    const int nc = right ? min(kST, m - c0) : min(kST, K0 - c0);
    for (int k0 = K0; k0 < K1; k0 += kNB) {
        const int k1 = min(k0 + kNB, K1), nb = k1 - k0;
        wg_apply_swaps<T>(A, m, pv, k0, k1, c0, c0 + nc, sh.sw);
        if (!right) continue;
        if (K0 < k0) wg_strip_update<T>(A, m, k0, nb, c0, nc, K0, k0 - K0);
        __syncthreads();
        for (int e = t; e < kNB * kNB; e += kWG) {
            const int i = e % kNB, k = e / kNB;
            sh.d[i][k] = (i < nb && k < nb) ? A[k0 + i + (size_t)(k0 + k) * m] : cx<T>{T(0), T(0)};
        }
        __syncthreads();
        if (t < nc) unit_lower16(A + (size_t)(c0 + t) * m, k0, m, sh.d);
        __syncthreads();
    }
}

// large fronts, after 128-column block [K0, K1): trailing GEMM S -= L21 U12 on MFMA over rows
// [K1, m) and a column range, one TW x TW tile per workgroup (blockIdx.y = front). cols 0: all
// of [K1, m); 1: the next block's pivot columns [K1, K2), K2 = min(K1 + 128, p); 2: [K2, m).
template <typename T, int TW>
__global__ void __launch_bounds__(kWG) k_front_gemm(const int32_t* __restrict__ big_list, int blk, int cols,
                                                   const int32_t* __restrict__ fsize, const int32_t* __restrict__ npiv,
                                                   const int64_t* __restrict__ front_off, cx<T>* __restrict__ arena) {
    __shared__ GemmShared<T, TW> sh;
    const int f = big_list[blockIdx.y];
    const int m = fsize[f], p = npiv[f], K0 = blk * kOB;
    if (K0 >= p) return;
    const int K1 = min(K0 + kOB, p);
    if (K1 >= m) return;
    const int K2 = max(K1, min(K1 + kOB, p));
    const int jlo = cols == 2 ? K2 : K1, jhi = cols == 1 ? K2 : m;
    if (jhi <= jlo) return;
    const int nr = (m - K1 + TW - 1) / TW, ncl = (jhi - jlo + TW - 1) / TW;
    const int x = blockIdx.x;
    if (x >= nr * ncl) return;
    wg_gemm_tile<T, TW>(arena + front_off[f], m, m, K0, K1 - K0, K1 + TW * (x % nr), jlo + TW * (x / nr), sh, jhi);
}

// ------------------------------------------------------------------ solves
// Both solves are blocked by 64 pivots (one wavefront): the 64 x 64 diagonal block is staged in
// LDS and solved by one wave per right-hand side with one row per lane (each solved value is
// broadcast from its lane with v_readlane, no barriers); the solved values are staged in LDS and the rest of the
// front vector is updated by the whole workgroup with the block's column panel, whose loads
// are independent of each other (unrolled). Two barriers per 64 pivots.

constexpr int kWideSolve = 1024;   // threads per workgroup for the solve levels with large fronts
constexpr int kSB = 64;     // solve block (= wavefront size)
constexpr int kSR = 16;     // right-hand sides per pass

// The value of lane k (k wave-uniform) in every lane: v_readlane into a scalar register, which
// costs a few cycles where a shuffle takes an LDS-crossbar round trip per 32-bit half; the
// diagonal-block chains take one such broadcast per pivot.
__device__ __forceinline__ float lane_value(float v, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ __forceinline__ double lane_value(double v, int k) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned int lo = (unsigned int)__builtin_amdgcn_readlane((int)(unsigned int)b, k);
    const unsigned int hi = (unsigned int)__builtin_amdgcn_readlane((int)(unsigned int)(b >> 32), k);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <typename T>
__device__ __forceinline__ cx<T> lane_cx(cx<T> v, int k) {
    return {lane_value(v.re, k), lane_value(v.im, k)};
}


template <typename T>
struct SolveShared {
    cx<T> d[kSB][kSB + 1];   // diagonal block
    cx<T> y[kSB][kSR];       // solved block values
    cx<T> rd[kSB];           // reciprocals of U's diagonal in the block (backward solves)
    cx<T> red[kWideSolve];   // partial sums of the column-split panel products
};

// Diagonal-block solves by one wave, lane i holding row i of the right-hand side. The lane's
// entries of the block are read from LDS kChain at a time into registers ahead of the dependent
// chain (one LDS wait per kChain steps), and the lane's update is a select rather than a branch.
// Unit lower: wi <- L^{-1} wi over nb pivots.
constexpr int kChain = 4;   // (8 trips a code-generation error in this compiler release)
template <typename T, int R>
__device__ __forceinline__ void wave_lower_solve(cx<T> (&wi)[R], const SolveShared<T>& sh, int nb, int lane) {
    for (int k0 = 0; k0 < nb - 1; k0 += kChain) {
        cx<T> dr[kChain];
#pragma unroll
        for (int j = 0; j < kChain; ++j) dr[j] = sh.d[lane][min(k0 + j, kSB - 1)];
#pragma unroll
        for (int j = 0; j < kChain; ++j) {
            const int k = k0 + j;
            if (k < nb - 1) {
                const bool upd = lane > k;
#pragma unroll
                for (int r = 0; r < R; ++r) {   // independent chains interleaved
                    const cx<T> wk = lane_cx(wi[r], k);
                    const cx<T> u = cfms(wi[r], dr[j], wk);
                    wi[r].re = upd ? u.re : wi[r].re;   // per component: a select of the values
                    wi[r].im = upd ? u.im : wi[r].im;
                }
            }
        }
    }
}
// Upper: wi <- U^{-1} wi, sh.rd holding the reciprocals of U's diagonal.
template <typename T, int R>
__device__ __forceinline__ void wave_upper_solve(cx<T> (&wi)[R], const SolveShared<T>& sh, int nb, int lane) {
    for (int k1 = nb - 1; k1 >= 0; k1 -= kChain) {
        cx<T> dr[kChain], rr[kChain];
#pragma unroll
        for (int j = 0; j < kChain; ++j) {
            dr[j] = sh.d[lane][max(k1 - j, 0)];
            rr[j] = sh.rd[max(k1 - j, 0)];
        }
#pragma unroll
        for (int j = 0; j < kChain; ++j) {
            const int k = k1 - j;
            if (k >= 0) {
                const bool piv = lane == k, upd = lane < k;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const cx<T> xk = cmul(lane_cx(wi[r], k), rr[j]);
                    const cx<T> u = cfms(wi[r], dr[j], xk);
                    wi[r].re = piv ? xk.re : (upd ? u.re : wi[r].re);
                    wi[r].im = piv ? xk.im : (upd ? u.im : wi[r].im);
                }
            }
        }
    }
}

// The block's right-hand sides [l0, l0 + nr) of the front vector w (column stride m) through the
// diagonal solve: wave v takes right-hand sides v, v + W, v + 2 W, ... (W waves), up to R of them
// interleaved in one pass; the solved values go back to w (pivot rows < nb) and to sh.y.
template <typename T, int NT, bool UPPER>
__device__ __forceinline__ void wave_diag_solve(cx<T>* w, int64_t m, int kb, int nb, int l0, int nr,
                                                SolveShared<T>& sh) {
    constexpr int W = NT / 64, R = (kSR + W - 1) / W;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cnt = nr > wave ? (nr - wave + W - 1) / W : 0;   // right-hand sides of this wave
    if (cnt == 0) return;
    if (cnt == 1) {
        cx<T> wi[1];
        cx<T>* wl = w + (size_t)(l0 + wave) * m;
        wi[0] = lane < nb ? wl[kb + lane] : cx<T>{T(0), T(0)};
        if (UPPER) wave_upper_solve<T, 1>(wi, sh, nb, lane);
        else wave_lower_solve<T, 1>(wi, sh, nb, lane);
        if (lane < nb) wl[kb + lane] = wi[0];
        sh.y[lane][wave] = wi[0];
        return;
    }
    cx<T> wi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int lr = wave + r * W;
        wi[r] = (r < cnt && lane < nb) ? w[kb + lane + (size_t)(l0 + lr) * m] : cx<T>{T(0), T(0)};
    }
    if (UPPER) wave_upper_solve<T, R>(wi, sh, nb, lane);
    else wave_lower_solve<T, R>(wi, sh, nb, lane);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int lr = wave + r * W;
        if (r < cnt) {
            if (lane < nb) w[kb + lane + (size_t)(l0 + lr) * m] = wi[r];
            sh.y[lane][lr] = wi[r];
        }
    }
}

// Column split of a panel product over few rows: with ne = rows x right-hand sides entries and
// NT threads, the workgroup forms G groups of NT / G threads (G a power of two, at most 16, and
// 1 when the entries fill half the workgroup); group g sums its own contiguous share of the
// panel's columns, so a thread issues ncols / G loads instead of ncols, and the G partial sums
// are added through LDS.
template <int NT>
__device__ __forceinline__ int split_groups(int ne) {
    const int r = (ne + 63) & ~63;
    int G = 1;
    while (G < 16 && 2 * G * r <= NT) G *= 2;
    return G;
}

// acc - sum_{k < nb} Fr[k m] y[k][lr] for nb <= 64, summed in k order; the panel's entries of the
// row are loaded 32 at a time with all loads of a batch in flight before the first product
template <typename T, int BATCH = 32>
__device__ __forceinline__ cx<T> row_panel_fms(cx<T> acc, const cx<T>* __restrict__ Fr, int64_t m, int nb,
                                               const cx<T> (*y)[kSR], int lr) {
#pragma unroll
    for (int h = 0; h < kSB; h += BATCH) {
        if (h >= nb) break;
        // unconditional loads (past nb the last column is read again and not used), so that
        // the batch is issued without branches
        cx<T> f[BATCH];
#pragma unroll
        for (int k = 0; k < BATCH; ++k) f[k] = Fr[(size_t)min(h + k, nb - 1) * m];
#pragma unroll
        for (int k = 0; k < BATCH; ++k)
            if (h + k < nb) acc = cfms(acc, f[k], y[h + k][lr]);
    }
    return acc;
}

// Partial product of group g (of G) over columns [0, ncols <= 64) of a panel: returns
// -sum_{k in group's share} Fr[k m] y[k][lr]; the share is wave-uniform, so the loads of a
// share are issued together under scalar branches, at most BATCH at a time (register budget of
// the 1024-thread workgroups).
template <typename T, int BATCH>
__device__ __forceinline__ cx<T> group_panel_partial(const cx<T>* __restrict__ Fr, int64_t m, int ncols, int g,
                                                     int G, const cx<T> (*y)[kSR], int lr) {
    const int per = (ncols + G - 1) / G, ka = g * per, cnt = min(per, ncols - ka);
    cx<T> acc = {T(0), T(0)};
#pragma unroll
    for (int h = 0; h < kSB / 2; h += BATCH) {
        if (h >= cnt) break;
        cx<T> f[BATCH];
#pragma unroll
        for (int k = 0; k < BATCH; ++k)
            if (h + k < cnt) f[k] = Fr[(size_t)(ka + h + k) * m];
#pragma unroll
        for (int k = 0; k < BATCH; ++k)
            if (h + k < cnt) acc = cfms(acc, f[k], y[ka + h + k][lr]);
    }
    return acc;
}

// ---- multi-RHS panel products on the matrix cores: W[rows, nr] -= F[rows, ncols] Y[ncols, nr]
// for nr <= 16 as 16 x 16 output tiles (one per wave at a time), each complex product as four
// real MFMA 16x16x4 products; every panel entry is loaded once (not once per right-hand side).
// Lane l supplies the A operand F[row0 + l % 16][k0 + l / 16] and the B operand
// Y[k0 + l / 16][l % 16] (zero past ncols or nr); item r of the accumulators is row
// MfmaAcc<T>::row(l, r), column l % 16 of the tile.
constexpr int kMfmaRhs = 4;   // right-hand sides from which the panel products use the matrix cores

template <typename T, int H = 8>   // H: K steps whose loads are issued together
__device__ __forceinline__ void mfma_panel_accum(typename MfmaAcc<T>::type& dre, typename MfmaAcc<T>::type& dim,
                                                 const cx<T>* __restrict__ Frow, int64_t ldf, bool rok, int ncols,
                                                 const cx<T> (*y)[kSR], int nr) {
    const int lane = threadIdx.x & 63, i = lane & 15, kk = lane >> 4;
#pragma unroll
    for (int s0 = 0; s0 < kSB / 4; s0 += H) {
        if (4 * s0 >= ncols) break;
        cx<T> av[H];
#pragma unroll
        for (int s = 0; s < H; ++s) {
            const int k = 4 * (s0 + s) + kk;
            av[s] = (rok && k < ncols) ? Frow[(size_t)k * ldf] : cx<T>{T(0), T(0)};
        }
#pragma unroll
        for (int s = 0; s < H; ++s) {
            const int k = 4 * (s0 + s) + kk;
            const cx<T> b = (k < ncols && i < nr) ? y[k][i] : cx<T>{T(0), T(0)};
            dre = MfmaAcc<T>::mfma(av[s].re, b.re, dre);
            dre = MfmaAcc<T>::mfma(-av[s].im, b.im, dre);
            dim = MfmaAcc<T>::mfma(av[s].re, b.im, dim);
            dim = MfmaAcc<T>::mfma(av[s].im, b.re, dim);
        }
    }
}

// w[tr0 + row + j ldw] -= D[row][j] for row < trows, j < nr (one wave), in two halves so that the
// tile's entries can be loaded before its products are formed
template <typename T>
__device__ __forceinline__ void mfma_tile_load(cx<T> (&cv)[4], const cx<T>* w, int64_t ldw, int tr0, int trows, int nr) {
    const int lane = threadIdx.x & 63, j = lane & 15;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ro = MfmaAcc<T>::row(lane, r);
        cv[r] = (ro < trows && j < nr) ? w[tr0 + ro + (size_t)j * ldw] : cx<T>{T(0), T(0)};
    }
}
template <typename T>
__device__ __forceinline__ void mfma_tile_store(cx<T> (&cv)[4], cx<T>* w, int64_t ldw, int tr0, int trows, int nr,
                                                const typename MfmaAcc<T>::type& dre,
                                                const typename MfmaAcc<T>::type& dim) {
    const int lane = threadIdx.x & 63, j = lane & 15;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ro = MfmaAcc<T>::row(lane, r);
        if (ro < trows && j < nr) {
            cv[r].re -= dre[r];
            cv[r].im -= dim[r];
            w[tr0 + ro + (size_t)j * ldw] = cv[r];
        }
    }
}
template <typename T>
__device__ __forceinline__ void mfma_tile_sub(cx<T>* w, int64_t ldw, int tr0, int trows, int nr,
                                              const typename MfmaAcc<T>::type& dre,
                                              const typename MfmaAcc<T>::type& dim) {
    cx<T> cv[4];
    mfma_tile_load<T>(cv, w, ldw, tr0, trows, nr);
    mfma_tile_store<T>(cv, w, ldw, tr0, trows, nr, dre, dim);
}

// w[r + j ldw] -= sum_{k < ncols} Fc[r + k ldf] y[k][j] for r in [r0, r0 + rows), j < nr
template <typename T, int NT>
__device__ __forceinline__ void mfma_rows_update(cx<T>* w, int64_t ldw, int r0, int rows, int nr, const cx<T>* Fc, int64_t ldf,
                                 int ncols, const cx<T> (*y)[kSR]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, i = lane & 15;
    const int ntile = rows > 0 ? (rows + 15) / 16 : 0;
    // the 512-thread super-block kernel has the registers to issue all 16 K steps' loads at once
    constexpr int H = NT == 512 ? 16 : 8;
    for (int tile = wave; tile < ntile; tile += NT / 64) {
        typename MfmaAcc<T>::type dre = {0, 0, 0, 0}, dim = {0, 0, 0, 0};
        const int tr0 = r0 + 16 * tile, trows = min(16, rows - 16 * tile);
        cx<T> cv[4];
        mfma_tile_load<T>(cv, w, ldw, tr0, trows, nr);
        mfma_panel_accum<T, H>(dre, dim, Fc + tr0 + i, ldf, i < trows, ncols, y, nr);
        mfma_tile_store<T>(cv, w, ldw, tr0, trows, nr, dre, dim);
    }
}

// w[r0 + i + lr m] -= sum_{k < ncols} Fc[r0 + i + k m] y[k][lr] for i < rows, lr < nr
// (ncols <= 64, y in LDS); column-split over thread groups when the rows are few. The caller
// synchronises before y or w is reused.
// MR (kernels built for several right-hand sides): from kMfmaRhs of them the product runs on the
// matrix cores; single right-hand-side kernels carry no MFMA code (lower register pressure).
template <typename T, int NT, int BATCH, bool MR>
__device__ __forceinline__ void panel_fms(cx<T>* __restrict__ w, int64_t m, int r0, int rows, int nr, const cx<T>* __restrict__ Fc,
                          int ncols, SolveShared<T>& sh) {
    const int t = threadIdx.x, ne = rows * nr;
    if (ne == 0) return;
    if constexpr (MR) {
        if (nr >= kMfmaRhs) {
            mfma_rows_update<T, NT>(w, m, r0, rows, nr, Fc, m, ncols, sh.y);
            return;
        }
    }
    const int G = split_groups<NT>(ne);
    if (G == 1) {
        for (int e = t; e < ne; e += NT) {
            const int r = r0 + e % rows, lr = e / rows;
            cx<T> acc = w[r + (size_t)lr * m];
            const cx<T>* Fr = Fc + r;
            if (BATCH > 0) {
                acc = row_panel_fms<T, (BATCH > 0 ? BATCH : 32)>(acc, Fr, m, ncols, sh.y, lr);
            } else {
#pragma unroll 16
                for (int k = 0; k < ncols; ++k) acc = cfms(acc, Fr[(size_t)k * m], sh.y[k][lr]);
            }
            w[r + (size_t)lr * m] = acc;
        }
        return;
    }
    const int S = NT / G, g = t / S, e = t % S;
    cx<T> part = {T(0), T(0)};
    if (e < ne) part = group_panel_partial<T, (NT > 256 ? 16 : 32)>(Fc + r0 + e % rows, m, ncols, g, G, sh.y, e / rows);
    sh.red[t] = part;
    __syncthreads();
    if (g == 0 && e < ne) {
        const int r = r0 + e % rows, lr = e / rows;
        cx<T> acc = w[r + (size_t)lr * m];
        for (int h = 0; h < G; ++h) {
            acc.re += sh.red[h * S + e].re;
            acc.im += sh.red[h * S + e].im;
        }
        w[r + (size_t)lr * m] = acc;
    }
}

// Forward: per front, w (m x nrhs, column stride m) = [b_piv ; 0] + children's contributions,
// row swaps on the pivot part, y = L11^{-1} w_piv, w_cb -= L21 y; y is written to x (new
// numbering) and w_cb stays in the front's work slot for the parent.
template <typename T>
struct SolveArgs {
    const int32_t *fsize, *npiv, *first, *child_off, *child_list, *cmap, *idx, *parent, *ipiv;
    const int32_t* huge;     // per front: 1 = triangular parts done by the multi-workgroup kernels
    const int32_t* psrc;     // per pivot: source row of the front's composed row swaps
    const int64_t *front_off, *idx_off, *cmap_off;
    const cx<T>* arena;
    cx<T>* x;
    int64_t ldx;
    int nrhs;
    cx<T>* work;
};

template <typename T, int NT, bool MR>
__device__ void front_fwd_body(int f, const SolveArgs<T>& a, SolveShared<T>& sh) {
    const int32_t *fsize = a.fsize, *npiv = a.npiv, *first = a.first, *child_off = a.child_off,
                  *child_list = a.child_list, *cmap = a.cmap;
    const int64_t *front_off = a.front_off, *idx_off = a.idx_off, *cmap_off = a.cmap_off;
    const cx<T>* arena = a.arena;
    cx<T>* x = a.x;
    cx<T>* work = a.work;
    const int64_t ldx = a.ldx;
    const int nrhs = a.nrhs;
    const int m = fsize[f], p = npiv[f], f0 = first[f];
    const cx<T>* F = arena + front_off[f];
    cx<T>* w = work + idx_off[f] * nrhs;   // m x nrhs
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    batched_for<NT, 4>(m * nrhs,
        [&](int e) { const int r = e % m, l = e / m; return r < p ? x[f0 + r + (size_t)l * ldx] : cx<T>{T(0), T(0)}; },
        [&](int e, cx<T> v) { w[e] = v; });
    __syncthreads();
    for (int ci = child_off[f]; ci < child_off[f + 1]; ++ci) {
        const int c = child_list[ci];
        const int mc = fsize[c], pc = npiv[c], nc = mc - pc;
        const cx<T>* wc = work + idx_off[c] * nrhs;
        const int32_t* map = cmap + cmap_off[c];
        batched_for<NT, 4>(nc * nrhs,
            [&](int e) {
                const int r = e % nc, l = e / nc;
                const cx<T> v = wc[pc + r + (size_t)l * mc], d = w[map[r] + (size_t)l * m];
                return cx<T>{d.re + v.re, d.im + v.im};
            },
            [&](int e, cx<T> v) { w[map[e % nc] + (size_t)(e / nc) * m] = v; });
        __syncthreads();
    }
    if (p == 0) return;
    // the front's row swaps as one gather, w_piv[k] <- w_piv[psrc[k]], staged through the
    // front's own (not yet written) pivot slots of x
    const int32_t* src = a.psrc + f0;
    batched_for<NT, 4>(p * nrhs, [&](int e) { return w[e % p + (size_t)(e / p) * m]; },
                       [&](int e, cx<T> v) { x[f0 + e % p + (size_t)(e / p) * ldx] = v; });
    __syncthreads();
    batched_for<NT, 4>(p * nrhs, [&](int e) { return x[f0 + src[e % p] + (size_t)(e / p) * ldx]; },
                       [&](int e, cx<T> v) { w[e % p + (size_t)(e / p) * m] = v; });
    __syncthreads();
    if (a.huge[f]) return;
    // Wide single-right-hand-side kernels hold the next diagonal block in registers (U entries
    // a thread): its loads are issued before the current block's chain and panel, so that they
    // share a memory round trip with the chain's own loads instead of starting one of their own.
    constexpr int U = kSB * kSB / NT;
    constexpr bool kAhead = NT >= 1024 && !MR;
    cx<T> ahead[kAhead ? U : 1];
    auto load_diag = [&](int kb, int nb, cx<T>* v) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = t + u * NT, i = e % kSB, k = e / kSB;
            v[u] = (i < nb && k < nb) ? F[kb + i + (size_t)(kb + k) * m] : cx<T>{T(0), T(0)};
        }
    };
    if constexpr (kAhead) load_diag(0, min(kSB, p), ahead);
    for (int kb = 0; kb < p; kb += kSB) {
        const int nb = min(kSB, p - kb);
        if constexpr (kAhead) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = t + u * NT;
                sh.d[e % kSB][e / kSB] = ahead[u];
            }
            if (kb + kSB < p) load_diag(kb + kSB, min(kSB, p - kb - kSB), ahead);
        } else {
            // the diagonal block to LDS with all of a thread's loads in flight at once
            batched_for<NT, U>(kSB * kSB,
                [&](int e) {
                    const int i = e % kSB, k = e / kSB;
                    return (i < nb && k < nb) ? F[kb + i + (size_t)(kb + k) * m] : cx<T>{T(0), T(0)};
                },
                [&](int e, cx<T> v) { sh.d[e % kSB][e / kSB] = v; });
        }
        for (int l0 = 0; l0 < nrhs; l0 += kSR) {
            const int nr = min(kSR, nrhs - l0);
            __syncthreads();
            // diagonal block: unit lower triangular, right-hand sides spread over the waves
            wave_diag_solve<T, NT, false>(w, m, kb, nb, l0, nr, sh);
            __syncthreads();
            // rows below the block: w[r] -= F[r, kb:kb+nb] y
            panel_fms<T, NT, (NT > 256 ? 16 : 32), MR>(w + (size_t)l0 * m, m, kb + nb, m - kb - nb, nr,
                                                   F + (size_t)kb * m, nb, sh);
        }
        __syncthreads();
    }
    batched_for<NT, 4>(p * nrhs, [&](int e) { return w[e % p + (size_t)(e / p) * m]; },
                       [&](int e, cx<T> v) { x[f0 + e % p + (size_t)(e / p) * ldx] = v; });
}


// Backward: x_piv = U11^{-1} (y - U12 x_cb), x_cb gathered from already-solved ancestors.
template <typename T, int NT, bool MR>
__device__ void front_bwd_body(int f, const SolveArgs<T>& a, SolveShared<T>& sh) {
    const int32_t *fsize = a.fsize, *npiv = a.npiv, *first = a.first, *idx = a.idx;
    const int64_t *front_off = a.front_off, *idx_off = a.idx_off;
    const cx<T>* arena = a.arena;
    cx<T>* x = a.x;
    const int64_t ldx = a.ldx;
    const int nrhs = a.nrhs;
    const int m = fsize[f], p = npiv[f], f0 = first[f];
    if (p == 0) return;
    const cx<T>* F = arena + front_off[f];
    const int32_t* ix = idx + idx_off[f];
    cx<T>* w = a.work + idx_off[f] * nrhs;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    batched_for<NT, 4>(m * nrhs, [&](int e) { return x[ix[e % m] + (size_t)(e / m) * ldx]; },
                       [&](int e, cx<T> v) { w[e] = v; });
    if (a.huge[f]) return;
    __syncthreads();
    // y_piv -= U12 x_cb, the contribution columns taken kSB at a time through LDS
    const int c = m - p;
    for (int l0 = 0; l0 < nrhs && c > 0; l0 += kSR) {
        const int nr = min(kSR, nrhs - l0);
        if constexpr (MR) {
            if (nr >= kMfmaRhs) {
                // 16-row tiles of the pivot rows on the matrix cores, accumulated over all columns
                const int ntile = (p + 15) / 16, nw = NT / 64, i = lane & 15;
                for (int pass = 0; pass < (ntile + nw - 1) / nw; ++pass) {
                    const int tile = pass * nw + wave, tr0 = 16 * tile;
                    const int trows = tile < ntile ? min(16, p - tr0) : 0;
                    typename MfmaAcc<T>::type dre = {0, 0, 0, 0}, dim = {0, 0, 0, 0};
                    for (int s0 = 0; s0 < c; s0 += kSB) {
                        const int ns = min(kSB, c - s0);
                        __syncthreads();
                        for (int q = t; q < kSB * kSR; q += NT) {
                            const int sidx = q % kSB, lr = q / kSB;
                            sh.y[sidx][lr] =
                                (sidx < ns && lr < nr) ? w[p + s0 + sidx + (size_t)(l0 + lr) * m] : cx<T>{T(0), T(0)};
                        }
                        __syncthreads();
                        if (trows > 0)
                            mfma_panel_accum<T>(dre, dim, F + tr0 + i + (size_t)(p + s0) * m, m, i < trows, ns, sh.y, nr);
                    }
                    if (trows > 0) mfma_tile_sub<T>(w + (size_t)l0 * m, m, tr0, trows, nr, dre, dim);
                }
                continue;
            }
        }
        const int G = split_groups<NT>(p * nr);
        if (G > 1) {
            // few pivot rows: the contribution columns are split over G thread groups
            const int S = NT / G, g = t / S, e = t % S;
            cx<T> part = {T(0), T(0)};
            if (c * nr <= kSB * (kSB + 1)) {
                // x_cb staged once, in the diagonal-block buffer (unused until the diagonal
                // solves); group g then runs through its contiguous share of the columns with
                // no barrier in between
                cx<T>* xs = &sh.d[0][0];
                __syncthreads();
                for (int q = t; q < c * nr; q += NT) xs[q] = w[p + q % c + (size_t)(l0 + q / c) * m];
                __syncthreads();
                if (e < p * nr) {
                    constexpr int BATCH = NT > 256 ? 8 : 16;
                    const int per = (c + G - 1) / G, ka = g * per, cnt = min(per, c - ka);
                    const cx<T>* Fr = F + e % p + (size_t)(p + ka) * m;
                    const cx<T>* xl = xs + (size_t)(e / p) * c + ka;
                    for (int h = 0; h < cnt; h += BATCH) {
                        cx<T> fv[BATCH];
#pragma unroll
                        for (int k = 0; k < BATCH; ++k)
                            if (h + k < cnt) fv[k] = Fr[(size_t)(h + k) * m];
#pragma unroll
                        for (int k = 0; k < BATCH; ++k)
                            if (h + k < cnt) part = cfms(part, fv[k], xl[h + k]);
                    }
                }
            } else {
                for (int s0 = 0; s0 < c; s0 += kSB) {
                    const int ns = min(kSB, c - s0);
                    __syncthreads();
                    for (int q = t; q < kSB * kSR; q += NT) {
                        const int sidx = q % kSB, lr = q / kSB;
                        sh.y[sidx][lr] =
                            (sidx < ns && lr < nr) ? w[p + s0 + sidx + (size_t)(l0 + lr) * m] : cx<T>{T(0), T(0)};
                    }
                    __syncthreads();
                    if (e < p * nr) {
                        const cx<T> d = group_panel_partial<T, (NT > 256 ? 16 : 32)>(F + e % p + (size_t)(p + s0) * m, m,
                                                                                     ns, g, G, sh.y, e / p);
                        part.re += d.re;
                        part.im += d.im;
                    }
                }
            }
            sh.red[t] = part;
            __syncthreads();
            if (g == 0 && e < p * nr) {
                cx<T>* wr = w + e % p + (size_t)(l0 + e / p) * m;
                cx<T> acc = *wr;
                for (int h = 0; h < G; ++h) {
                    acc.re += sh.red[h * S + e].re;
                    acc.im += sh.red[h * S + e].im;
                }
                *wr = acc;
            }
            continue;
        }
        for (int base = 0; base < p * nr; base += 4 * NT) {
            cx<T> acc[4];
            for (int g = 0; g < 4; ++g) {
                const int e = base + g * NT + t;
                acc[g] = e < p * nr ? w[e % p + (size_t)(l0 + e / p) * m] : cx<T>{T(0), T(0)};
            }
            for (int s0 = 0; s0 < c; s0 += kSB) {
                const int ns = min(kSB, c - s0);
                __syncthreads();
                for (int e = t; e < kSB * kSR; e += NT) {
                    const int sidx = e % kSB, lr = e / kSB;
                    sh.y[sidx][lr] = (sidx < ns && lr < nr) ? w[p + s0 + sidx + (size_t)(l0 + lr) * m] : cx<T>{T(0), T(0)};
                }
                __syncthreads();
                for (int g = 0; g < 4; ++g) {
                    const int e = base + g * NT + t;
                    if (e >= p * nr) break;
                    const int r = e % p, lr = e / p;
                    const cx<T>* Fr = F + r + (size_t)(p + s0) * m;
                    cx<T> a = acc[g];
#pragma unroll 16
                    for (int k = 0; k < ns; ++k) a = cfms(a, Fr[(size_t)k * m], sh.y[k][lr]);
                    acc[g] = a;
                }
            }
            __syncthreads();
            for (int g = 0; g < 4; ++g) {
                const int e = base + g * NT + t;
                if (e < p * nr) w[e % p + (size_t)(l0 + e / p) * m] = acc[g];
            }
        }
    }
    __syncthreads();
    for (int kb = ((p - 1) / kSB) * kSB; kb >= 0; kb -= kSB) {
        const int nb = min(kSB, p - kb);
        batched_for<NT, kSB * kSB / NT>(kSB * kSB,
            [&](int e) {
                const int i = e % kSB, k = e / kSB;
                return (i < nb && k < nb) ? F[kb + i + (size_t)(kb + k) * m] : cx<T>{T(1), T(0)};
            },
            [&](int e, cx<T> v) { sh.d[e % kSB][e / kSB] = v; });
        // the divisions leave the sequential chain: all reciprocals of the block's diagonal at once
        if (t < kSB) sh.rd[t] = t < nb ? crecip(F[kb + t + (size_t)(kb + t) * m]) : cx<T>{T(1), T(0)};
        for (int l0 = 0; l0 < nrhs; l0 += kSR) {
            const int nr = min(kSR, nrhs - l0);
            __syncthreads();
            wave_diag_solve<T, NT, true>(w, m, kb, nb, l0, nr, sh);
            __syncthreads();
            // rows above the block: w[r] -= F[r, kb:kb+nb] x_blk
            panel_fms<T, NT, 0, MR>(w + (size_t)l0 * m, m, 0, kb, nr, F + (size_t)kb * m, nb, sh);
        }
        __syncthreads();
    }
    batched_for<NT, 4>(p * nrhs, [&](int e) { return w[e % p + (size_t)(e / p) * m]; },
                       [&](int e, cx<T> v) { x[f0 + e % p + (size_t)(e / p) * ldx] = v; });
}

// One launch per tree level and direction; every front of the level is one workgroup.
template <typename T, int NT, bool MR>
__global__ void __launch_bounds__(NT) k_front_fwd(const int32_t* __restrict__ level_fronts, SolveArgs<T> a) {
    __shared__ SolveShared<T> sh;
    front_fwd_body<T, NT, MR>(level_fronts[blockIdx.x], a, sh);
}
template <typename T, int NT, bool MR>
__global__ void __launch_bounds__(NT) k_front_bwd(const int32_t* __restrict__ level_fronts, SolveArgs<T> a) {
    __shared__ SolveShared<T> sh;
    front_bwd_body<T, NT, MR>(level_fronts[blockIdx.x], a, sh);
}

// ---- the largest fronts: triangular solves by super-blocks of kHugeSB pivots. Per super-block
// two launches: k_huge_diag, one workgroup per front, solves the super-block's four 64-pivot
// diagonal blocks in order (each as in the per-level solves: diagonal block in LDS, right-hand
// sides spread over the waves, then the rest of the super-block updated with the block's panel)
// and stores the solved values to w and x; then k_huge_rows spreads the rows outside the
// super-block over workgroups of 64 rows, each subtracting F[rows, super-block] times the solved
// values (MFMA tiles with several right-hand sides). The backward direction first subtracts
// U12 x_cb from the pivot rows (k_huge_rows over the contribution columns).
constexpr int kHugeSB = 4 * kSB;
constexpr int kHugeDiagWG = 512;   // threads of k_huge_diag: two waves per SIMD, two right-hand sides per wave

// w[r0 + i] -= F[r0 + i, c0:c0+nc] w[c0:c0+nc] for i < rows <= 64 (all right-hand sides); the
// solved values are staged 64 columns at a time through sh.y
template <typename T>
__device__ void huge_rows_update(const cx<T>* __restrict__ F, cx<T>* __restrict__ w, int m, int nrhs, int r0, int rows,
                                 int c0, int nc, SolveShared<T>& sh, int lbeg, int lend) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int l0 = lbeg; l0 < min(lend, nrhs); l0 += kSR) {
        const int nr = min(kSR, nrhs - l0);
        if (nr >= kMfmaRhs) {
            // wave w: rows [r0 + 16 w, +16) on the matrix cores, accumulated over all columns
            const int tr0 = r0 + 16 * wave, trows = min(16, rows - 16 * wave), i = lane & 15;
            typename MfmaAcc<T>::type dre = {0, 0, 0, 0}, dim = {0, 0, 0, 0};
            for (int s0 = 0; s0 < nc; s0 += kSB) {
                const int ns = min(kSB, nc - s0);
                __syncthreads();
                for (int e = t; e < kSB * kSR; e += kWG) {
                    const int si = e % kSB, lr = e / kSB;
                    sh.y[si][lr] = (si < ns && lr < nr) ? w[c0 + s0 + si + (size_t)(l0 + lr) * m] : cx<T>{T(0), T(0)};
                }
                __syncthreads();
                if (trows > 0)
                    mfma_panel_accum<T>(dre, dim, F + tr0 + i + (size_t)(c0 + s0) * m, m, i < trows, ns, sh.y, nr);
            }
            if (trows > 0) mfma_tile_sub<T>(w + (size_t)l0 * m, m, tr0, trows, nr, dre, dim);
            __syncthreads();
            continue;
        }
        // each thread owns up to 4 (row, rhs) pairs of this workgroup's 64 x nr outputs
        cx<T> acc[4];
        for (int g = 0; g < 4; ++g) {
            const int e = g * kWG + t;
            acc[g] = e < rows * nr ? w[r0 + e % rows + (size_t)(l0 + e / rows) * m] : cx<T>{T(0), T(0)};
        }
        for (int s0 = 0; s0 < nc; s0 += kSB) {
            const int ns = min(kSB, nc - s0);
            __syncthreads();
            for (int e = t; e < kSB * kSR; e += kWG) {
                const int si = e % kSB, lr = e / kSB;
                sh.y[si][lr] = (si < ns && lr < nr) ? w[c0 + s0 + si + (size_t)(l0 + lr) * m] : cx<T>{T(0), T(0)};
            }
            __syncthreads();
            for (int g = 0; g < 4; ++g) {
                const int e = g * kWG + t;
                if (e >= rows * nr) break;
                const int r = r0 + e % rows, lr = e / rows;
                const cx<T>* Fr = F + r + (size_t)(c0 + s0) * m;
                cx<T> v = acc[g];
#pragma unroll 16
                for (int k = 0; k < ns; ++k) v = cfms(v, Fr[(size_t)k * m], sh.y[k][lr]);
                acc[g] = v;
            }
        }
        for (int g = 0; g < 4; ++g) {
            const int e = g * kWG + t;
            if (e < rows * nr) w[r0 + e % rows + (size_t)(l0 + e / rows) * m] = acc[g];
        }
        __syncthreads();
    }
}

// mode 0 (forward): rows [K1, m) receive the super-block [K0, K1); mode 1 (backward): rows
// [0, K0) receive it; mode 2 (backward, first): rows [0, p) receive the contribution columns
// [p, m) (U12 x_cb). A workgroup takes 64 rows and kSR right-hand sides. The workgroups of one
// row tile's right-hand-side chunks get block indices 8 apart: the dispatcher deals consecutive
// indices round-robin to the 8 XCDs, so they run on one XCD and share its L2 copy of the rows.
__device__ __forceinline__ void huge_tile_of(int bid, int nch, int* rowtile, int* chunk) {
    const int rest = bid >> 3;
    *chunk = rest % nch;
    *rowtile = (rest / nch) * 8 + (bid & 7);
}
static unsigned huge_grid_x(unsigned rowtiles, int nrhs) {
    const unsigned nch = (unsigned)((nrhs + kSR - 1) / kSR);
    return ((rowtiles + 7) / 8) * 8 * nch;
}
template <typename T>
__global__ void __launch_bounds__(kWG) k_huge_rows(const int32_t* __restrict__ huge_list, int mode, int K0,
                                                   SolveArgs<T> a) {
    __shared__ SolveShared<T> sh;
    const int f = huge_list[blockIdx.y];
    int rowtile, chunk;
    huge_tile_of((int)blockIdx.x, (a.nrhs + kSR - 1) / kSR, &rowtile, &chunk);
    const int m = a.fsize[f], p = a.npiv[f];
    int rb, re, c0, nc;
    if (mode == 2) {
        rb = 0, re = p, c0 = p, nc = m - p;
    } else {
        if (K0 >= p) return;
        const int K1 = min(K0 + kHugeSB, p);
        c0 = K0, nc = K1 - K0;
        rb = mode == 0 ? K1 : 0;
        re = mode == 0 ? m : K0;
    }
    const int r0 = rb + kSB * rowtile;
    if (r0 >= re || nc <= 0) return;
    huge_rows_update<T>(a.arena + a.front_off[f], a.work + a.idx_off[f] * a.nrhs, m, a.nrhs, r0, min(kSB, re - r0), c0,
                        nc, sh, chunk * kSR, (chunk + 1) * kSR);
}

// The same row updates for kMfmaRhs or more right-hand sides, on the matrix cores: a workgroup
// takes 16 rows and kSR right-hand sides, wave v sums the 64-column chunks v, v + 4, ... of the
// source columns with all of a chunk's loads (F rows and solved values) in flight together, and
// the four partial 16 x 16 tiles are added in LDS in wave order. Four times as many workgroups
// as 64-row tiles, and one memory round trip per chunk instead of one per 32 columns.
template <typename T>
__global__ void __launch_bounds__(kWG) k_huge_rows_mfma(const int32_t* __restrict__ huge_list, int mode, int K0,
                                                        SolveArgs<T> a) {
    typedef typename MfmaAcc<T>::type acc_t;
    __shared__ acc_t red_re[kWG / 64][64], red_im[kWG / 64][64];
    const int f = huge_list[blockIdx.y];
    int rowtile, chunk;
    huge_tile_of((int)blockIdx.x, (a.nrhs + kSR - 1) / kSR, &rowtile, &chunk);
    const int m = a.fsize[f], p = a.npiv[f];
    int rb, re, c0, nc;
    if (mode == 2) {
        rb = 0, re = p, c0 = p, nc = m - p;
    } else {
        if (K0 >= p) return;
        const int K1 = min(K0 + kHugeSB, p);
        c0 = K0, nc = K1 - K0;
        rb = mode == 0 ? K1 : 0;
        re = mode == 0 ? m : K0;
    }
    const int r0 = rb + 16 * rowtile;
    if (r0 >= re || nc <= 0) return;
    const int rows = min(16, re - r0), l0 = chunk * kSR, nr = min(kSR, a.nrhs - l0);
    const cx<T>* F = a.arena + a.front_off[f];
    cx<T>* w = a.work + a.idx_off[f] * a.nrhs;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, i = lane & 15, kk = lane >> 4;
    acc_t dre = {0, 0, 0, 0}, dim = {0, 0, 0, 0};
    for (int s0 = 64 * wave; s0 < nc; s0 += 64 * (kWG / 64)) {
        const int ns = min(64, nc - s0);
        cx<T> av[16], bv[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int k = 4 * s + kk;
            av[s] = (i < rows && k < ns) ? F[r0 + i + (size_t)(c0 + s0 + k) * m] : cx<T>{T(0), T(0)};
            bv[s] = (k < ns && i < nr) ? w[c0 + s0 + k + (size_t)(l0 + i) * m] : cx<T>{T(0), T(0)};
        }
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            dre = MfmaAcc<T>::mfma(av[s].re, bv[s].re, dre);
            dre = MfmaAcc<T>::mfma(-av[s].im, bv[s].im, dre);
            dim = MfmaAcc<T>::mfma(av[s].re, bv[s].im, dim);
            dim = MfmaAcc<T>::mfma(av[s].im, bv[s].re, dim);
        }
    }
    red_re[wave][lane] = dre;
    red_im[wave][lane] = dim;
    __syncthreads();
    if (wave == 0) {
        acc_t sr = red_re[0][lane], si = red_im[0][lane];
#pragma unroll
        for (int v = 1; v < kWG / 64; ++v) {
            sr += red_re[v][lane];
            si += red_im[v][lane];
        }
        mfma_tile_sub<T>(w + (size_t)l0 * m, m, r0, rows, nr, sr, si);
    }
}

// the super-block [K0, K1) of one front (grid: one workgroup per huge front and chunk of kSR
// right-hand sides; the chunks are independent)
template <typename T, bool UPPER>
__global__ void __launch_bounds__(kHugeDiagWG) k_huge_diag(const int32_t* __restrict__ huge_list, int K0, SolveArgs<T> a) {
    constexpr int NT = kHugeDiagWG;
    __shared__ SolveShared<T> sh;
    const int f = huge_list[blockIdx.x];
    const int m = a.fsize[f], p = a.npiv[f], f0 = a.first[f];
    if (K0 >= p) return;
    const int K1 = min(K0 + kHugeSB, p), t = threadIdx.x;
    const cx<T>* F = a.arena + a.front_off[f];
    cx<T>* w = a.work + a.idx_off[f] * a.nrhs;
    const int nrhs = a.nrhs;
    const int lc = (int)blockIdx.y * kSR;
    // the diagonal blocks do not depend on the solve: the next one is loaded into registers while
    // the current one is solved and its panel applied
    constexpr int DPER = kSB * kSB / NT;
    cx<T> dn[DPER];
    auto fetch_d = [&](int kb) {
        const int nb = min(kSB, K1 - kb);
#pragma unroll
        for (int u = 0; u < DPER; ++u) {
            const int e = t + u * NT, i = e % kSB, k = e / kSB;
            dn[u] = (i < nb && k < nb) ? F[kb + i + (size_t)(kb + k) * m] : (UPPER ? cx<T>{T(1), T(0)} : cx<T>{T(0), T(0)});
        }
    };
    for (int l0 = lc; l0 < min(nrhs, lc + kSR); l0 += kSR) {
        const int nr = min(kSR, nrhs - l0);
        const int kfirst = UPPER ? K0 + ((K1 - 1 - K0) / kSB) * kSB : K0;
        fetch_d(kfirst);
        for (int kb = kfirst; UPPER ? kb >= K0 : kb < K1; kb += UPPER ? -kSB : kSB) {
            const int nb = min(kSB, K1 - kb);
            __syncthreads();
#pragma unroll
            for (int u = 0; u < DPER; ++u) {
                const int e = t + u * NT;
                sh.d[e % kSB][e / kSB] = dn[u];
            }
            if (UPPER && t < kSB) sh.rd[t] = t < nb ? crecip(F[kb + t + (size_t)(kb + t) * m]) : cx<T>{T(1), T(0)};
            const int knext = kb + (UPPER ? -kSB : kSB);
            if (UPPER ? knext >= K0 : knext < K1) fetch_d(knext);
            lds_barrier();   // the block in LDS (the prefetch stays in flight)
            wave_diag_solve<T, NT, UPPER>(w, m, kb, nb, l0, nr, sh);
            lds_barrier();   // the solved values in sh.y; the panel below reads no row the solve wrote
            // the rest of the super-block with the block's panel
            if (UPPER)
                panel_fms<T, NT, 0, true>(w + (size_t)l0 * m, m, K0, kb - K0, nr, F + (size_t)kb * m, nb, sh);
            else
                panel_fms<T, NT, 16, true>(w + (size_t)l0 * m, m, kb + nb, K1 - kb - nb, nr, F + (size_t)kb * m, nb,
                                           sh);
        }
    }
    __syncthreads();
    const int nk = K1 - K0, nrc = min(kSR, nrhs - lc);
    batched_for<NT, 4>(nk * nrc, [&](int e) { return w[K0 + e % nk + (size_t)(lc + e / nk) * m]; },
                        [&](int e, cx<T> v) { a.x[f0 + K0 + e % nk + (size_t)(lc + e / nk) * a.ldx] = v; });
}

// gather (with precision change) B (old numbering, n x nrhs FP64) -> xp (new numbering, T)
template <typename T>
__global__ void k_gather_perm(const zd* __restrict__ B, int64_t ldb, const int32_t* __restrict__ perm, int64_t n, int nrhs,
                              cx<T>* __restrict__ xp) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * nrhs) return;
    const int64_t i = e % n, l = e / n;
    const zd v = B[perm[i] + l * ldb];
    xp[e] = {T(v.re), T(v.im)};
}

// X (old numbering) (+)= xp (new numbering); accumulate when add != 0
template <typename T>
__global__ void k_scatter_perm(const cx<T>* __restrict__ xp, const int32_t* __restrict__ perm, int64_t n, int nrhs,
                               zd* __restrict__ X, int64_t ldx, int add) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * nrhs) return;
    const int64_t i = e % n, l = e / n;
    const cx<T> v = xp[e];
    zd& d = X[perm[i] + l * ldx];
    if (add) { d.re += (double)v.re; d.im += (double)v.im; }
    else { d.re = (double)v.re; d.im = (double)v.im; }
}

// out = sum_t c_t p_t entry by entry (FP64): the shifted matrix or the mass matrix at one frequency
// for systems with a damping matrix or frequency-dependent terms
struct Comb {
    const zd* p[3 + kMaxTerms];
    zd c[3 + kMaxTerms];
    int n;
};
__global__ void k_combine(int64_t nnz, Comb cb, zd* __restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        double re = 0, im = 0;
        for (int t = 0; t < cb.n; ++t) {
            const zd v = cb.p[t][e], c = cb.c[t];
            re += c.re * v.re - c.im * v.im;
            im += c.re * v.im + c.im * v.re;
        }
        out[e] = {re, im};
    }
}

__global__ void k_maxabs_entries(const zd* __restrict__ K, const zd* __restrict__ M, int64_t nnz, double sigma,
                                 unsigned long long* out) {
    double m = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        double re = K[e].re - sigma * M[e].re, im = K[e].im - sigma * M[e].im;
        m = fmax(m, fabs(re) + fabs(im));
    }
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

// Per front, the composition of its row swaps (ipiv[k] swapped with k, k = 0..p-1) as a gather
// map: psrc[k] = the row whose value ends at k. Done once per factorisation so that every solve
// applies the swaps in one parallel gather; the sequential composition runs in LDS.
constexpr int kComposeLds = 16384;   // pivots composed in LDS (64 KB); larger fronts use global memory
__global__ void __launch_bounds__(kWG) k_compose_pivots(const int32_t* __restrict__ npiv, const int32_t* __restrict__ first,
                                                       const int32_t* __restrict__ ipiv, int32_t* __restrict__ psrc) {
    __shared__ int32_t perm[kComposeLds];
    const int f = blockIdx.x;
    const int p = npiv[f], f0 = first[f];
    const int32_t* iv = ipiv + f0;
    int32_t* out = psrc + f0;
    if (p <= kComposeLds) {
        for (int k = threadIdx.x; k < p; k += kWG) perm[k] = k;
        __syncthreads();
        if (threadIdx.x == 0)
            for (int k = 0; k < p; ++k) {
                const int r = iv[k];
                const int32_t tmp = perm[k];
                perm[k] = perm[r];
                perm[r] = tmp;
            }
        __syncthreads();
        for (int k = threadIdx.x; k < p; k += kWG) out[k] = perm[k];
    } else {
        for (int k = threadIdx.x; k < p; k += kWG) out[k] = k;
        __syncthreads();
        if (threadIdx.x == 0)
            for (int k = 0; k < p; ++k) {
                const int r = iv[k];
                const int32_t tmp = out[k];
                out[k] = out[r];
                out[r] = tmp;
            }
    }
}

template <typename T>
void run_factor(Factor& f, cr_sys sys, double sigma, cx<T>* arena, T tiny, hipStream_t s) {
    const Symbolic& S = *sys->sym;
    const DevSymbolic& D = *sys->dsym;
    hipStream_t aux = S.big_list.empty() ? nullptr : aux_stream(sys->ctx);
    const int split_rows = sys->fclass.split_rows;
    if (split_rows > 0 && !S.big_list.empty()) {
        // split-panel publications and barrier counters, one slot per large front of a level
        size_t slots = 0;
        for (int l = 0; l < S.nlevel; ++l) slots = std::max(slots, (size_t)(S.big_off[l + 1] - S.big_off[l]));
        f.coop_pub.reserve((slots * sizeof(CoopPub<T>) + sizeof(double) - 1) / sizeof(double));
        f.coop_bar.reserve(slots * kCoopBarInts);
        fill_zero(f.coop_bar.p, (int64_t)(slots * kCoopBarInts), s);
    }
    for (int l = 0; l < S.nlevel; ++l) {
        const int nf = S.level_off[l + 1] - S.level_off[l];
        const int32_t* lf = D.level_fronts.p + S.level_off[l];
        {
            // workgroups per front: one per 32 columns of the level's largest front, at most 256
            // (the top fronts are the largest memory traffic of the assembly: m^2 entries zeroed
            // and the children's contribution blocks added, which 64 workgroups cannot stream at
            // the memory's rate; on the fuselage fronts 32 columns per workgroup measured faster
            // than 8, 16 or 64, and a cap of 256 faster than 128, 512 or 1024)
            int mmax = 0;
            for (int q = S.level_off[l]; q < S.level_off[l + 1]; ++q) mmax = std::max(mmax, S.fsize[S.level_fronts[q]]);
            const unsigned split = (unsigned)std::min(256, std::max(1, mmax / 32));
            ProfScope ps(sys->ctx, "front_assemble", s);
            hipLaunchKernelGGL(k_front_assemble<T>, dim3(nf, split), dim3(kWG), 0, s, lf, D.fsize.p, D.front_off.p, D.child_off.p,
                               D.child_list.p, D.npiv.p, D.cmap_off.p, D.cmap.p, D.ent_off.p, D.ent_src.p, D.ent_dst.p,
                               f.opK, f.opM, sigma, arena);
        }
        {
            ProfScope ps(sys->ctx, "front_factor", s);
            hipLaunchKernelGGL(k_front_factor<T>, dim3(nf), dim3(kWG), 0, s, lf, D.fsize.p, D.npiv.p, D.first.p,
                               D.front_off.p, arena, f.ipiv.p, tiny, f.nperturb.p, D.big.p);
        }
        const int nbig = S.big_off[l + 1] - S.big_off[l];
        if (nbig == 0) continue;
        const int32_t* bl = D.big_list.p + S.big_off[l];
        // Blocks of 128 columns with one block of look-ahead: block b's panels (library stream)
        // touch only the block's own columns, so they run while the trailing update of block
        // b - 1 beyond b's columns runs on the second stream; then the deferred row strips of
        // block b and the update of block b + 1's columns (library stream), and the rest of
        // block b's update goes to the second stream.
        const int per = kOB / kNB, nblk = (S.nsteps[l] + per - 1) / per;
        const bool overlap = aux != nullptr;
        bool pending = false;   // a trailing update is in flight on the second stream
        for (int blk = 0; blk < nblk; ++blk) {
            for (int j = blk * per; j < std::min(S.nsteps[l], (blk + 1) * per); ++j) {
                unsigned gcol = 0, grow = 0, gsplit = 0;
                bool any_lds = false, any_mem = false, any_split = false;
                int nsplit = 0;   // workgroups of the split panels
                for (int q = S.big_off[l]; q < S.big_off[l + 1]; ++q) {
                    const int f = S.big_list[q], m = S.fsize[f], p = S.npiv[f], k0 = j * kNB;
                    if (k0 >= p) continue;
                    const int G = p - k0 <= panel_lds_rows<T>() ? 0 : coop_groups(p - k0, split_rows);
                    if (p - k0 <= panel_lds_rows<T>()) any_lds = true;
                    else if (G == 0) any_mem = true;
                    else {
                        any_split = true;
                        nsplit += G;
                        gsplit = std::max(gsplit, (unsigned)G);
                    }
                    const int K0 = (k0 / kOB) * kOB, k1 = std::min(k0 + kNB, p), Kend = std::min(K0 + kOB, p);
                    gcol = std::max(gcol, (unsigned)((m - k0 + kCST - 1) / kCST));
                    grow = std::max(grow, (unsigned)((Kend - k1 + kST - 1) / kST + (m - p + kWG - 1) / kWG));
                }
                if (j % per != 0 && gcol) {
                    ProfScope ps(sys->ctx, "front_colstrip", s);
                    hipLaunchKernelGGL(k_front_colstrip<T>, dim3(gcol, nbig), dim3(kWG), 0, s, bl, j, D.fsize.p,
                                       D.npiv.p, D.front_off.p, arena);
                }
                // every workgroup of a split launch must be resident at once: beyond kCoopMaxWG the
                // step's panels all take the single-workgroup kernel
                const int split = nsplit <= kCoopMaxWG ? split_rows : 0;
                if (any_split && !split) any_mem = true;
                if (any_split && split) {
                    ProfScope ps(sys->ctx, "front_panel", s);
                    hipLaunchKernelGGL(k_front_panel_coop<T>, dim3(gsplit, nbig), dim3(kWG), 0, s, bl, j, split, D.fsize.p,
                                       D.npiv.p, D.first.p, D.front_off.p, arena, f.ipiv.p, tiny, f.nperturb.p,
                                       reinterpret_cast<CoopPub<T>*>(f.coop_pub.p), f.coop_bar.p,
                                       sys->fclass.split_polls > 0 ? sys->fclass.split_polls : kCoopSpins, f.nperturb.p + 1);
                }
                if (any_mem) {
                    ProfScope ps(sys->ctx, "front_panel", s);
                    hipLaunchKernelGGL((k_front_panel<T, false>), dim3(nbig), dim3(kWG), 0, s, bl, j, split, D.fsize.p,
                                       D.npiv.p, D.first.p, D.front_off.p, arena, f.ipiv.p, tiny, f.nperturb.p);
                }
                if (any_lds) {
                    ProfScope ps(sys->ctx, "front_panel", s);
                    hipLaunchKernelGGL((k_front_panel<T, true>), dim3(nbig), dim3(kWG), 0, s, bl, j, split, D.fsize.p,
                                       D.npiv.p, D.first.p, D.front_off.p, arena, f.ipiv.p, tiny, f.nperturb.p);
                }
                if (grow) {
                    ProfScope ps(sys->ctx, "front_rowstrip", s);
                    hipLaunchKernelGGL(k_front_rowstrip<T>, dim3(grow, nbig), dim3(kWG), 0, s, bl, j, D.fsize.p,
                                       D.npiv.p, D.first.p, D.front_off.p, f.ipiv.p, arena);
                }
            }
            if (pending) {
                CR_HIP(hipStreamWaitEvent(s, sys->ctx->ev_join, 0));
                pending = false;
            }
            unsigned gblk = 0, t_next = 0, t_rest = 0;
            for (int q = S.big_off[l]; q < S.big_off[l + 1]; ++q) {
                const int f = S.big_list[q], m = S.fsize[f], p = S.npiv[f], K0 = blk * kOB;
                if (K0 >= p) continue;
                const int K1 = std::min(K0 + kOB, p), K2 = std::max(K1, std::min(K1 + kOB, p));
                gblk = std::max(gblk, (unsigned)((m - K1 + kST - 1) / kST + (K0 + kST - 1) / kST));
                const unsigned nr = (unsigned)((m - K1 + kGT - 1) / kGT);
                t_next = std::max(t_next, nr * (unsigned)((K2 - K1 + kGT - 1) / kGT));
                t_rest = std::max(t_rest, nr * (unsigned)((m - K2 + kGT - 1) / kGT));
            }
            if (gblk) {
                ProfScope ps(sys->ctx, "front_rowblock", s);
                hipLaunchKernelGGL(k_front_rowblock<T>, dim3(gblk, nbig), dim3(kWG), 0, s, bl, blk, D.fsize.p, D.npiv.p,
                                   D.first.p, D.front_off.p, f.ipiv.p, arena);
            }
            // 64 x 64 tiles: 128 x 128 tiles (one wave per SIMD for their accumulators) were
            // measured slower on the fuselage fronts
            if (t_next) {
                ProfScope ps(sys->ctx, "front_gemm", s);
                hipLaunchKernelGGL((k_front_gemm<T, kGT>), dim3(t_next, nbig), dim3(kWG), 0, s, bl, blk, 1, D.fsize.p,
                                   D.npiv.p, D.front_off.p, arena);
            }
            if (t_rest) {
                hipStream_t gs = s;
                if (overlap) {
                    CR_HIP(hipEventRecord(sys->ctx->ev_fork, s));
                    CR_HIP(hipStreamWaitEvent(aux, sys->ctx->ev_fork, 0));
                    gs = aux;
                }
                {
                    ProfScope ps(sys->ctx, "front_gemm", gs);
                    hipLaunchKernelGGL((k_front_gemm<T, kGT>), dim3(t_rest, nbig), dim3(kWG), 0, gs, bl, blk, 2,
                                       D.fsize.p, D.npiv.p, D.front_off.p, arena);
                }
                if (overlap) {
                    CR_HIP(hipEventRecord(sys->ctx->ev_join, aux));
                    pending = true;
                }
            }
        }
        if (pending) CR_HIP(hipStreamWaitEvent(s, sys->ctx->ev_join, 0));
    }
    hipLaunchKernelGGL(k_compose_pivots, dim3(S.nfront), dim3(kWG), 0, s, D.npiv.p, D.first.p, f.ipiv.p, f.psrc.p);
    CR_HIP(hipGetLastError());
}

// one solve level: the kernel variant for the right-hand-side count (MR)
template <typename T, int NT>
void launch_level(bool fwd, bool mr, int nf, hipStream_t s, const int32_t* lf, const SolveArgs<T>& a) {
    if (fwd) {
        if (mr) hipLaunchKernelGGL((k_front_fwd<T, NT, true>), dim3(nf), dim3(NT), 0, s, lf, a);
        else hipLaunchKernelGGL((k_front_fwd<T, NT, false>), dim3(nf), dim3(NT), 0, s, lf, a);
    } else {
        if (mr) hipLaunchKernelGGL((k_front_bwd<T, NT, true>), dim3(nf), dim3(NT), 0, s, lf, a);
        else hipLaunchKernelGGL((k_front_bwd<T, NT, false>), dim3(nf), dim3(NT), 0, s, lf, a);
    }
}

// one launch of the huge-front row updates: the matrix-core kernel (16-row tiles) from kMfmaRhs
// right-hand sides on, else the 64-row kernel
template <typename T>
void huge_rows(const int32_t* hl, int nh, int mode, int K0, unsigned tiles16, unsigned tiles64, const SolveArgs<T>& a,
               hipStream_t s) {
    if (a.nrhs >= kMfmaRhs)
        hipLaunchKernelGGL(k_huge_rows_mfma<T>, dim3(huge_grid_x(tiles16, a.nrhs), nh), dim3(kWG), 0, s, hl, mode, K0, a);
    else
        hipLaunchKernelGGL(k_huge_rows<T>, dim3(huge_grid_x(tiles64, a.nrhs), nh), dim3(kWG), 0, s, hl, mode, K0, a);
}

template <typename T>
void run_solve(const Factor& f, int nrhs, cx<T>* xp, cx<T>* work, hipStream_t s, const cx<T>* arena) {
    cr_sys sys = f.sys;
    const Symbolic& S = *sys->sym;
    const DevSymbolic& D = *sys->dsym;
    SolveArgs<T> a;
    a.fsize = D.fsize.p;
    a.npiv = D.npiv.p;
    a.first = D.first.p;
    a.child_off = D.child_off.p;
    a.child_list = D.child_list.p;
    a.cmap = D.cmap.p;
    a.idx = D.idx.p;
    a.parent = D.parent.p;
    a.ipiv = f.ipiv.p;
    a.huge = D.huge.p;
    a.psrc = f.psrc.p;
    a.front_off = D.front_off.p;
    a.idx_off = D.idx_off.p;
    a.cmap_off = D.cmap_off.p;
    a.arena = arena;
    a.x = xp;
    a.ldx = (int64_t)S.n;
    a.nrhs = nrhs;
    a.work = const_cast<cx<T>*>(work);
    const unsigned nch = (unsigned)((nrhs + kSR - 1) / kSR);
    {
        for (int l = 0; l < S.nlevel; ++l) {
            const int nf = S.level_off[l + 1] - S.level_off[l];
            {
                ProfScope ps(sys->ctx, "front_fwd", s);
                const int32_t* lf = D.level_fronts.p + S.level_off[l];
                const bool mr = nrhs >= kMfmaRhs;
                if (S.wide_solve[l] & (mr ? 1 : 2)) launch_level<T, kWideSolve>(true, mr, nf, s, lf, a);
                else launch_level<T, kWG>(true, mr, nf, s, lf, a);
            }
            const int nh = S.huge_off[l + 1] - S.huge_off[l];
            const int32_t* hl = D.huge_list.p + S.huge_off[l];
            for (int K0 = 0; K0 < S.huge_piv[l]; K0 += kHugeSB) {
                unsigned gx = 1, gx16 = 1;
                for (int q = S.huge_off[l]; q < S.huge_off[l + 1]; ++q) {
                    const int hf = S.huge_list[q], m = S.fsize[hf], p = S.npiv[hf];
                    if (K0 >= p) continue;
                    gx = std::max(gx, (unsigned)((m - std::min(K0 + kHugeSB, p) + kSB - 1) / kSB));
                    gx16 = std::max(gx16, (unsigned)((m - std::min(K0 + kHugeSB, p) + 15) / 16));
                }
                ProfScope ps(sys->ctx, "front_fwd_huge", s);
                hipLaunchKernelGGL((k_huge_diag<T, false>), dim3(nh, nch), dim3(kHugeDiagWG), 0, s, hl, K0, a);
                huge_rows(hl, nh, 0, K0, gx16, gx, a, s);
            }
        }
        for (int l = S.nlevel - 1; l >= 0; --l) {
            const int nf = S.level_off[l + 1] - S.level_off[l];
            {
                ProfScope ps(sys->ctx, "front_bwd", s);
                const int32_t* lf = D.level_fronts.p + S.level_off[l];
                const bool mr = nrhs >= kMfmaRhs;
                if (S.wide_solve[l] & (mr ? 1 : 2)) launch_level<T, kWideSolve>(false, mr, nf, s, lf, a);
                else launch_level<T, kWG>(false, mr, nf, s, lf, a);
            }
            const int nh = S.huge_off[l + 1] - S.huge_off[l];
            if (nh == 0) continue;
            const int32_t* hl = D.huge_list.p + S.huge_off[l];
            {
                ProfScope ps(sys->ctx, "front_bwd_huge", s);
                huge_rows(hl, nh, 2, 0, (unsigned)((S.huge_piv[l] + 15) / 16), (unsigned)((S.huge_piv[l] + kSB - 1) / kSB),
                          a, s);
            }
            for (int K0 = ((S.huge_piv[l] - 1) / kHugeSB) * kHugeSB; K0 >= 0; K0 -= kHugeSB) {
                ProfScope ps(sys->ctx, "front_bwd_huge", s);
                hipLaunchKernelGGL((k_huge_diag<T, true>), dim3(nh, nch), dim3(kHugeDiagWG), 0, s, hl, K0, a);
                if (K0 > 0) huge_rows(hl, nh, 1, K0, (unsigned)((K0 + 15) / 16), (unsigned)((K0 + kSB - 1) / kSB), a, s);
            }
        }
    }
    CR_HIP(hipGetLastError());
}

}  // namespace

void upload_symbolic(cr_sys sys) {
    const Symbolic& S = *sys->sym;
    auto D = std::make_unique<DevSymbolic>();
    hipStream_t s = sys->ctx->stream;
    upload(D->first, S.first, s);
    upload(D->npiv, S.npiv, s);
    upload(D->fsize, S.fsize, s);
    upload(D->parent, S.parent, s);
    upload(D->child_off, S.child_off, s);
    upload(D->child_list, S.child_list, s);
    upload(D->level_fronts, S.level_fronts, s);
    upload(D->idx, S.idx, s);
    upload(D->cmap, S.cmap, s);
    upload(D->ent_dst, S.ent_dst, s);
    upload(D->idx_off, S.idx_off, s);
    upload(D->front_off, S.front_off, s);
    upload(D->cmap_off, S.cmap_off, s);
    upload(D->ent_off, S.ent_off, s);
    upload(D->ent_src, S.ent_src, s);
    upload(D->perm, S.perm, s);
    upload(D->iperm, S.iperm, s);
    upload(D->big, S.big, s);
    upload(D->big_list, S.big_list, s);
    upload(D->huge, S.huge, s);
    upload(D->huge_list, S.huge_list, s);
    CR_HIP(hipStreamSynchronize(s));
    sys->dsym = std::move(D);
}

void numeric_factor(Factor& f, cr_sys sys, double omega, cr_precision prec, hipStream_t s) {
    CR_REQUIRE(sys->sym && sys->dsym, CR_E_STATE, "factor before analyse");
    const Symbolic& S = *sys->sym;
    f.sys = sys;
    f.omega = omega;
    f.prec = prec;
    f.ipiv.reserve(S.n);
    f.psrc.reserve(S.n);
    f.nperturb.reserve(2);
    const int64_t nnz = sys->rowptr[sys->n];
    if (!sys->D.empty() || !sys->terms.empty()) {
        // A(w) = K~ + sum_K-terms c_t T_t + i w D~ - w^2 (M~ + sum_M-terms c_t T_t)
        Comb a{}, m{};
        const double w2 = omega * omega;
        a.p[a.n] = sys->d_K.p; a.c[a.n++] = {1.0, 0.0};
        a.p[a.n] = sys->d_M.p; a.c[a.n++] = {-w2, 0.0};
        if (!sys->D.empty()) { a.p[a.n] = sys->d_D.p; a.c[a.n++] = {0.0, omega}; }
        m.p[m.n] = sys->d_M.p; m.c[m.n++] = {1.0, 0.0};
        for (const FreqTerm& t : sys->terms) {
            const zd c = t.coef(omega);
            if (t.kind == 0) { a.p[a.n] = t.d_vals.p; a.c[a.n++] = c; }
            else {
                a.p[a.n] = t.d_vals.p; a.c[a.n++] = {-w2 * c.re, -w2 * c.im};
                m.p[m.n] = t.d_vals.p; m.c[m.n++] = c;
            }
        }
        f.aval.reserve(nnz);
        hipLaunchKernelGGL(k_combine, dim3(1024), dim3(256), 0, s, nnz, a, f.aval.p);
        f.opK = f.aval.p;
        f.opM = f.aval.p;
        f.opS = 0.0;
        if (m.n > 1) {
            f.mval.reserve(nnz);
            hipLaunchKernelGGL(k_combine, dim3(1024), dim3(256), 0, s, nnz, m, f.mval.p);
            f.opMass = f.mval.p;
        } else {
            f.mval.release();
            f.opMass = sys->d_M.p;
        }
    } else {
        // the shifted operator pre-formed for the refinement residual; the front assembly reads
        // K~ and M~ directly
        Comb a{};
        a.p[a.n] = sys->d_K.p; a.c[a.n++] = {1.0, 0.0};
        a.p[a.n] = sys->d_M.p; a.c[a.n++] = {-omega * omega, 0.0};
        f.aval.reserve(nnz);
        hipLaunchKernelGGL(k_combine, dim3(1024), dim3(256), 0, s, nnz, a, f.aval.p);
        f.mval.release();
        f.opK = sys->d_K.p;
        f.opM = sys->d_M.p;
        f.opS = omega * omega;
        f.opMass = sys->d_M.p;
    }
    f.opA = f.aval.p;
    f.anorm_omega = -1;
    const double sigma = f.opS;
    // largest |entry| of the shifted matrix sets the perturbation threshold
    f.amax.reserve(1);
    fill_zero(f.amax.p, 1, s);
    fill_zero(f.nperturb.p, 2, s);
    hipLaunchKernelGGL(k_maxabs_entries, dim3(256), dim3(256), 0, s, f.opK, f.opM, nnz, sigma, f.amax.p);
    unsigned long long hm = 0;
    CR_HIP(hipMemcpyAsync(&hm, f.amax.p, sizeof(hm), hipMemcpyDeviceToHost, s));
    CR_HIP(hipStreamSynchronize(s));
    double amax;
    std::memcpy(&amax, &hm, sizeof(amax));
    CR_REQUIRE(amax > 0 && std::isfinite(amax), CR_E_SINGULAR,
               "the shifted matrix at this frequency has no nonzero entry or a non-finite one: no pivot can be perturbed");
    if (prec == CR_MIXED) {
        f.arena64.release();
        f.arena32.reserve(S.arena);
        run_factor<float>(f, sys, sigma, reinterpret_cast<cx<float>*>(f.arena32.p), (float)(3e-4 * amax), s);
    } else {
        f.arena32.release();
        f.arena64.reserve(S.arena);
        run_factor<double>(f, sys, sigma, reinterpret_cast<cx<double>*>(f.arena64.p), 1e-8 * amax, s);
    }
    int32_t np[2] = {0, 0};
    CR_HIP(hipMemcpyAsync(np, f.nperturb.p, sizeof(np), hipMemcpyDeviceToHost, s));
    CR_HIP(hipStreamSynchronize(s));
    CR_REQUIRE(np[1] == 0, CR_E_HIP,
               "a split panel's workgroups were not resident together (barrier wait timed out): the factor is invalid");
    f.n_perturbed = np[0];
}

// one application of the stored factor: Xout = A~^{-1} B (both FP64, old numbering)
void apply_factor(const Factor& f, int nrhs, const zd* B, int64_t ldb, zd* X, int64_t ldx, int add, SolveWork& w,
                  hipStream_t s) {
    cr_sys sys = f.sys;
    const Symbolic& S = *sys->sym;
    const int64_t n = S.n;
    const int64_t tot = n * nrhs;
    const int nb = (int)((tot + 255) / 256);
    if (f.prec == CR_MIXED) {
        w.w32.reserve((size_t)S.idx_off[S.nfront] * nrhs + n * nrhs);
        cx<float>* xp = reinterpret_cast<cx<float>*>(w.w32.p);
        cx<float>* work = xp + n * nrhs;
        hipLaunchKernelGGL(k_gather_perm<float>, dim3(nb), dim3(256), 0, s, B, ldb, sys->dsym->perm.p, n, nrhs, xp);
        run_solve<float>(f, nrhs, xp, work, s, reinterpret_cast<const cx<float>*>(f.arena32.p));
        hipLaunchKernelGGL(k_scatter_perm<float>, dim3(nb), dim3(256), 0, s, xp, sys->dsym->perm.p, n, nrhs, X, ldx, add);
    } else {
        w.w64.reserve((size_t)S.idx_off[S.nfront] * nrhs + n * nrhs);
        cx<double>* xp = reinterpret_cast<cx<double>*>(w.w64.p);
        cx<double>* work = xp + n * nrhs;
        hipLaunchKernelGGL(k_gather_perm<double>, dim3(nb), dim3(256), 0, s, B, ldb, sys->dsym->perm.p, n, nrhs, xp);
        run_solve<double>(f, nrhs, xp, work, s, reinterpret_cast<const cx<double>*>(f.arena64.p));
        hipLaunchKernelGGL(k_scatter_perm<double>, dim3(nb), dim3(256), 0, s, xp, sys->dsym->perm.p, n, nrhs, X, ldx, add);
    }
    CR_HIP(hipGetLastError());
}

}  // namespace cr

