// Reduced frequency sweep (the MOR online phase, paper Section 3.3, reduced system of Eq. (11)):
// for every frequency w of every reduced model,
//     A_R(w) = K_R + i w D_R - w^2 M_R    (formed in FP64, rounded once to the LU precision)
//     P A_R = L U                         (dense, partial pivoting; complex FP32 or FP64)
//     X = A_R^{-1} F_R (i w)^flags        (+ FP64 iterative refinement with K_R, M_R, D_R)
//     Y = C_R X                           (FP64)
//
// One persistent launch: each workgroup owns a workspace slot and takes (model, frequency)
// items from a queue ordered by q^3 descending (longest first), so uneven model orders balance
// across the 256 compute units. The same kernel serves the single-model sweep, the batched
// sweep, and the greedy's candidate solves (which write X instead of Y).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>

#include "dense.cuh"
#include "internal.h"
#include "sweep.h"
#include "util.cuh"

namespace cr {
namespace {

// B (q x L, ld q) <- A^{-1} B with the LU factor in A (ld lda) and row pivots ipiv
template <typename T>
__device__ void wg_lu_solve(const cx<T>* __restrict__ A, int lda, int q, const int* __restrict__ ipiv,
                            cx<T>* __restrict__ B, int L) {
    const int t = threadIdx.x;
    for (int l = t; l < L; l += kWG) {
        cx<T>* b = B + (size_t)l * q;
        for (int k = 0; k < q; ++k) {
            const int r = ipiv[k];
            if (r != k) { cx<T> a = b[k]; b[k] = b[r]; b[r] = a; }
        }
    }
    __syncthreads();
    // column-oriented substitutions over independent (row, right-hand side) entries; within a
    // step row k of B is only read, so each thread's entries are loaded before any is stored
    // (four at a time) instead of one memory round trip per entry
    for (int k = 0; k < q - 1; ++k) {
        const int rows = q - k - 1;
        batched_for<kWG, 4>(rows * L,
            [&](int e) {
                const int i = k + 1 + e % rows, l = e / rows;
                return cfms(B[i + (size_t)l * q], A[i + (size_t)k * lda], B[k + (size_t)l * q]);
            },
            [&](int e, cx<T> v) { B[k + 1 + e % rows + (size_t)(e / rows) * q] = v; });
        __syncthreads();
    }
    for (int k = q - 1; k >= 0; --k) {
        const cx<T> d = crecip(A[k + (size_t)k * lda]);
        for (int l = t; l < L; l += kWG) B[k + (size_t)l * q] = cmul(B[k + (size_t)l * q], d);
        __syncthreads();
        batched_for<kWG, 4>(k * L,
            [&](int e) {
                const int i = e % k, l = e / k;
                return cfms(B[i + (size_t)l * q], A[i + (size_t)k * lda], B[k + (size_t)l * q]);
            },
            [&](int e, cx<T> v) { B[e % k + (size_t)(e / k) * q] = v; });
        __syncthreads();
    }
}

template <typename T>
__device__ __forceinline__ T wg_sum(T v, T* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    T s = ((red[0] + red[1]) + red[2]) + red[3];
    return s;
}
template <typename T>
__device__ __forceinline__ T wg_max(T v, T* red) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// Per load column l of the q x L column-major arrays (ld q): the largest entry magnitude of each of
// three arrays, into out[0][l], out[1][l], out[2][l] (LDS, L <= kMaxLoads). One wave per column
// (columns dealt round-robin to the four waves), lanes strided over the rows, then a shuffle
// reduction; ends with a barrier.
constexpr int kMaxLoads = 64;
template <typename TA, typename TB, typename TC>
__device__ void col_max3(const TA* __restrict__ a, const TB* __restrict__ b, const TC* __restrict__ c, int q, int L,
                         double (*out)[kMaxLoads]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int l = wave; l < L; l += kWG / 64) {
        double ma = 0, mb = 0, mc = 0;
        for (int i = lane; i < q; i += 64) {
            const size_t e = i + (size_t)l * q;
            ma = fmax(ma, hypot((double)a[e].re, (double)a[e].im));
            mb = fmax(mb, hypot((double)b[e].re, (double)b[e].im));
            mc = fmax(mc, hypot((double)c[e].re, (double)c[e].im));
        }
        for (int off = 32; off > 0; off >>= 1) {
            ma = fmax(ma, __shfl_xor(ma, off));
            mb = fmax(mb, __shfl_xor(mb, off));
            mc = fmax(mc, __shfl_xor(mc, off));
        }
        if (lane == 0) { out[0][l] = ma; out[1][l] = mb; out[2][l] = mc; }
    }
    __syncthreads();
}

// Factor and solve one reduced system in precision T: A_R(w) rounded to T, LU with partial
// pivoting over every row, X = A_R^{-1} B with FP64 refinement (refine) or a single solve.
// Only a pivot that is zero, non-finite or below eps_T^2 max|A_R| (numerically singular) is
// perturbed, and a perturbed factor is always refined in FP64 so that its solution is either
// certified or reported. Refinement stops per load column: column l has converged when its
// normwise backward error ||r_l|| / (||A_R|| ||x_l|| + ||b_l||) <= tol or when the last
// correction is below tol ||x_l|| (infinity norms); with a complex-FP32 factor the backward
// error test also needs a last correction below 1e-12 ||x_l||. The item converges when every
// column has.
// It stops unconverged after max_iter corrections or when the largest backward error of the
// unconverged columns fails to halve. Returns whether the item converged.
constexpr double kDxF32 = 1e-12;
// entry o of A_R(w) = K_R + i w D_R - w^2 M_R + sum_t c_t T_t in FP64 (tc: this frequency's c_t)
__device__ __forceinline__ zd ar_entry(const RomDesc& rd, size_t o, double w, double w2, const zd* tc) {
    const zd k = rd.KR[o], m = rd.MR[o];
    double re = k.re - w2 * m.re, im = k.im - w2 * m.im;
    if (rd.DR) { const zd d = rd.DR[o]; re -= w * d.im; im += w * d.re; }
    for (int t = 0; t < rd.nterm; ++t) {
        const zd c = tc[t], v = rd.T[t][o];
        re += c.re * v.re - c.im * v.im;
        im += c.re * v.im + c.im * v.re;
    }
    return {re, im};
}

template <typename T>
__device__ bool solve_item(const RomDesc& rd, double w, const zd* tc, cx<T>* __restrict__ A, int* __restrict__ ipiv, zd* __restrict__ X,
                           zd* __restrict__ R, const zd* __restrict__ Bv, cx<T>* __restrict__ D, bool refine, int max_iter,
                           double tol, LuShared<T>& sh, double* red, int* s_perturb, int* its_out,
                           double (*cm)[kMaxLoads], double* s_bn) {
    const int t = threadIdx.x;
    const int q = rd.q, L = rd.L;
    const double w2 = w * w;
    double amax = 0;
    for (int e = t; e < q * q; e += kWG) {
        const zd a = ar_entry(rd, e, w, w2, tc);
        A[e] = {T(a.re), T(a.im)};
        amax = fmax(amax, fabs(a.re) + fabs(a.im));
    }
    amax = wg_max(amax, red);
    for (int e = t; e < q * L; e += kWG) {
        X[e] = {0.0, 0.0};
        R[e] = Bv[e];
    }
    if (t == 0) *s_perturb = 0;
    __syncthreads();
    constexpr double eps = sizeof(T) == 4 ? 5.96e-8 : 1.11e-16;
    const T tiny = amax > 0 ? T(amax * eps * eps) : T(sizeof(T) == 4 ? 1e-37 : 1e-307);
    wg_getrf<T, true>(A, q, q, q, ipiv, tiny, s_perturb, sh);
    refine = refine || *s_perturb > 0;
    int its = 0;
    double prev = 1e300, an = 0;
    bool conv = false;
    for (;;) {
        for (int e = t; e < q * L; e += kWG) D[e] = {T(R[e].re), T(R[e].im)};
        __syncthreads();
        wg_lu_solve<T>(A, q, q, ipiv, D, L);
        for (int e = t; e < q * L; e += kWG) { X[e].re += (double)D[e].re; X[e].im += (double)D[e].im; }
        __syncthreads();
        if (!refine) { conv = true; break; }
        // R = B - A_R X in FP64. One thread per row reads K_R, M_R (and D_R) once per
        // refinement step for up to kLc load columns; X comes through LDS kJc rows at a time.
        constexpr int kLc = 16, kJc = 32;
        __shared__ zd xs[kJc][kLc];
        double anorm_part = 0;
        for (int l0 = 0; l0 < L; l0 += kLc) {
            const int nl = min(kLc, L - l0);
            for (int i0 = 0; i0 < q; i0 += kWG) {
                const int i = i0 + t;
                const bool act = i < q;
                double rr[kLc], ri[kLc], rowsum = 0;
#pragma unroll
                for (int c = 0; c < kLc; ++c) {
                    rr[c] = (act && c < nl) ? Bv[i + (size_t)(l0 + c) * q].re : 0.0;
                    ri[c] = (act && c < nl) ? Bv[i + (size_t)(l0 + c) * q].im : 0.0;
                }
                for (int j0 = 0; j0 < q; j0 += kJc) {
                    const int nj = min(kJc, q - j0);
                    __syncthreads();
                    for (int e = t; e < kJc * kLc; e += kWG) {
                        const int jj = e % kJc, c = e / kJc;
                        xs[jj][c] = (jj < nj && c < nl) ? X[j0 + jj + (size_t)(l0 + c) * q] : zd{0.0, 0.0};
                    }
                    __syncthreads();
                    if (act) {
                        for (int jj = 0; jj < nj; ++jj) {
                            const size_t o = i + (size_t)(j0 + jj) * q;
                            const zd a = ar_entry(rd, o, w, w2, tc);
                            const double ar = a.re, ai = a.im;
                            if (its == 0 && l0 == 0) rowsum += hypot(ar, ai);
#pragma unroll
                            for (int c = 0; c < kLc; ++c) {
                                const zd x = xs[jj][c];
                                rr[c] -= ar * x.re - ai * x.im;
                                ri[c] -= ar * x.im + ai * x.re;
                            }
                        }
                    }
                }
                if (act) {
                    anorm_part = fmax(anorm_part, rowsum);
#pragma unroll
                    for (int c = 0; c < kLc; ++c)
                        if (c < nl) R[i + (size_t)(l0 + c) * q] = {rr[c], ri[c]};
                }
            }
        }
        if (its == 0) an = wg_max(anorm_part, red);
        __syncthreads();
        // per column: cm[0] = ||r_l||, cm[1] = ||x_l||, cm[2] = ||d_l|| (last correction)
        col_max3(R, X, D, q, L, cm);
        bool all = true;
        double worst = 0;
        for (int l = 0; l < L; ++l) {
            const double be = cm[0][l] / (an * cm[1][l] + s_bn[l]);
            // a complex-FP32 factor contracts the error by about kappa u_32 per correction, so a
            // small backward error alone leaves up to kappa tol in x: its columns must also have
            // taken a correction below kDxF32 ||x|| (the remaining error is a fraction of it)
            const bool ok = sizeof(T) == 8 ? (be <= tol || cm[2][l] <= tol * cm[1][l])
                                           : (be <= tol && cm[2][l] <= kDxF32 * cm[1][l]) || cm[2][l] <= tol * cm[1][l];
            all = all && ok;
            if (!ok) worst = fmax(worst, be);
        }
        __syncthreads();
        if (all) { conv = true; break; }
        if (its >= max_iter || !(worst < 0.5 * prev)) break;
        prev = worst;
        ++its;
    }
    *its_out = its;
    return conv;
}

// stats: [0] max refinement iterations, [1] not converged, [2] perturbed pivots,
//        [3] FP64 fallbacks, [4] work-queue counter
template <typename T>
__global__ void __launch_bounds__(kWG) k_sweep(const RomDesc* __restrict__ roms, const int2* __restrict__ items, int nitems,
                                               int64_t slot_a, int64_t slot_v, zd* __restrict__ wsA, int* __restrict__ wsP,
                                               zd* __restrict__ wsX, zd* __restrict__ wsR, zd* __restrict__ wsB,
                                               zd* __restrict__ wsD, int refine, int max_iter, double tol,
                                               int* __restrict__ stats, int q_lds) {
    __shared__ LuShared<double> sh;   // large enough for the FP32 variant as well
    extern __shared__ double dyn_lds[];   // reduced matrix of orders q <= q_lds (LDS-resident variant)
    __shared__ double red[8];
    __shared__ int s_item;
    __shared__ int s_perturb;
    __shared__ double s_cm[3][kMaxLoads];   // per-column norms of the refinement
    __shared__ double s_bn[kMaxLoads];      // ||b_l||_inf of the current item
    const int t = threadIdx.x;
    zd* Aslot = wsA + (size_t)blockIdx.x * slot_a;   // slot_a complex128 entries (fits either precision)
    int* ipiv = wsP + (size_t)blockIdx.x * 4096;
    zd* X = wsX + (size_t)blockIdx.x * slot_v;
    zd* R = wsR + (size_t)blockIdx.x * slot_v;
    zd* Bv = wsB + (size_t)blockIdx.x * slot_v;
    zd* Dslot = wsD + (size_t)blockIdx.x * slot_v;
    int* counter = stats + 4;
    for (;;) {
        if (t == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int next = s_item;
        __syncthreads();
        if (next >= nitems) break;
        const int2 it = items[next];
        const RomDesc rd = roms[it.x];
        const int q = rd.q, L = rd.L;
        const double w = rd.omegas[it.y];
        for (int e = t; e < q * L; e += kWG) {
            const int l = e / q;
            const zd f = rd.FR[e];
            Bv[e] = rd.flags[l] ? zd{-w * f.im, w * f.re} : f;
        }
        __syncthreads();
        col_max3(Bv, Bv, Bv, q, L, s_cm);
        for (int l = t; l < L; l += kWG) s_bn[l] = s_cm[0][l];
        __syncthreads();
        int its = 0, fell_back = 0, nperturbed = 0;
        cx<T>* Awork = q <= q_lds ? reinterpret_cast<cx<T>*>(dyn_lds) : reinterpret_cast<cx<T>*>(Aslot);
        const zd* tc = rd.nterm ? rd.tcoef + (size_t)it.y * rd.nterm : nullptr;
        bool conv = solve_item<T>(rd, w, tc, Awork, ipiv, X, R, Bv, reinterpret_cast<cx<T>*>(Dslot),
                                  refine != 0, max_iter, tol, reinterpret_cast<LuShared<T>&>(sh), red, &s_perturb, &its,
                                  s_cm, s_bn);
        nperturbed = s_perturb;
        if (!conv && sizeof(T) == 4) {
            // complex-FP32 LU too inaccurate for refinement to converge (kappa(A_R) u_32 >~ 1):
            // redo this frequency with a complex-FP64 LU
            fell_back = 1;
            int its2 = 0;
            conv = solve_item<double>(rd, w, tc, reinterpret_cast<cx<double>*>(Aslot), ipiv, X, R, Bv,
                                      reinterpret_cast<cx<double>*>(Dslot), true, max_iter, tol, sh, red, &s_perturb, &its2,
                                      s_cm, s_bn);
            nperturbed += s_perturb;
            its += its2;
        }
        if (rd.out_x) {
            zd* o = rd.out + (size_t)it.y * q * L;
            for (int e = t; e < q * L; e += kWG) o[e] = X[e];
        } else {
            // Y = C_R X: one thread per (receiver, group of 4 loads); C_R read once per group
            const int no = rd.n_o;
            zd* o = rd.out + (size_t)it.y * L * no;
            const int ng = (L + 3) / 4;
            for (int e = t; e < no * ng; e += kWG) {
                const int oo = e % no, l0 = 4 * (e / no);
                const int nl = min(4, L - l0);
                double yr[4] = {0, 0, 0, 0}, yi[4] = {0, 0, 0, 0};
                for (int k = 0; k < q; ++k) {
                    const zd c = rd.CR[oo + (size_t)k * no];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        if (j < nl) {
                            const zd x = X[k + (size_t)(l0 + j) * q];
                            yr[j] += c.re * x.re - c.im * x.im;
                            yi[j] += c.re * x.im + c.im * x.re;
                        }
                    }
                }
                for (int j = 0; j < nl; ++j) o[oo + (size_t)(l0 + j) * no] = {yr[j], yi[j]};
            }
        }
        if (t == 0) {
            atomicMax(stats + 0, its);
            if (!conv) atomicAdd(stats + 1, 1);
            if (nperturbed) atomicAdd(stats + 2, nperturbed);
            if (fell_back) atomicAdd(stats + 3, 1);
        }
        __syncthreads();
    }
}

}  // namespace

// LDS-resident variant: the reduced matrix stays in LDS when q^2 entries fit the budget
static int q_lds_for(cr_precision prec, int lds_bytes) {
    const int elt = prec == CR_MIXED ? (int)sizeof(cx<float>) : (int)sizeof(cx<double>);
    int q = 0;
    while ((q + 1) * (q + 1) * elt <= lds_bytes) ++q;
    return q;
}

void SweepEngine::prepare(const std::vector<RomDesc>& roms, const std::vector<int2>& items, hipStream_t s) {
    qmax = 0;
    Lmax = 0;
    for (const RomDesc& r : roms) {
        qmax = std::max(qmax, r.q);
        Lmax = std::max(Lmax, r.L);
    }
    CR_REQUIRE(qmax <= 4096, CR_E_UNSUPPORTED, "reduced order above 4096");
    CR_REQUIRE(Lmax <= 64, CR_E_UNSUPPORTED, "more than 64 load columns in a reduced model");
    nitems = (int)items.size();
    d_roms.reserve(roms.size());
    d_items.reserve(items.size());
    d_stats.reserve(8);
    if (!roms.empty())
        CR_HIP(hipMemcpyAsync(d_roms.p, roms.data(), roms.size() * sizeof(RomDesc), hipMemcpyHostToDevice, s));
    if (!items.empty())
        CR_HIP(hipMemcpyAsync(d_items.p, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    CR_HIP(hipStreamSynchronize(s));
}

// Launch the prepared items with grid = min(items, grid_per_cu * CUs) resident workgroups and an
// LDS budget for the LDS-resident variant. Only kernels are enqueued (no memset / memcpy), so
// the launch can be captured in a graph.
void SweepEngine::launch(cr_precision prec, bool refine, int grid_per_cu, int lds_bytes, hipStream_t s) {
    if (nitems == 0) return;
    const int64_t slot_a = (int64_t)qmax * qmax, slot_v = (int64_t)qmax * std::max(Lmax, 1);
    const int grid = std::min<int>(nitems, std::max(1, grid_per_cu) * num_cu);
    wsA.reserve((size_t)grid * slot_a);
    wsP.reserve((size_t)grid * 4096);
    wsX.reserve((size_t)grid * slot_v);
    wsR.reserve((size_t)grid * slot_v);
    wsB.reserve((size_t)grid * slot_v);
    wsD.reserve((size_t)grid * slot_v);
    fill_zero(d_stats.p, 8, s);
    const int q_lds = q_lds_for(prec, lds_bytes);
    const size_t dyn = q_lds > 0 ? (size_t)lds_bytes : 0;
    ProfScope ps(ctx, "sweep", s);
    if (prec == CR_MIXED) {
        if (dyn > 65536) CR_HIP(hipFuncSetAttribute((const void*)k_sweep<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
        hipLaunchKernelGGL(k_sweep<float>, dim3(grid), dim3(kWG), dyn, s, d_roms.p, d_items.p, nitems, slot_a, slot_v,
                           wsA.p, wsP.p, wsX.p, wsR.p, wsB.p, wsD.p, 1, 10, 1e-14, d_stats.p, q_lds);
    } else {
        if (dyn > 65536) CR_HIP(hipFuncSetAttribute((const void*)k_sweep<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
        hipLaunchKernelGGL(k_sweep<double>, dim3(grid), dim3(kWG), dyn, s, d_roms.p, d_items.p, nitems, slot_a, slot_v,
                           wsA.p, wsP.p, wsX.p, wsR.p, wsB.p, wsD.p, refine ? 1 : 0, 10, 1e-14, d_stats.p, q_lds);
    }
    CR_HIP(hipGetLastError());
}

void SweepEngine::read_stats(hipStream_t s, int* max_its, int* not_conv, int* perturbed, int* fallbacks) {
    int st[8] = {0};
    if (nitems > 0) CR_HIP(hipMemcpyAsync(st, d_stats.p, sizeof(st), hipMemcpyDeviceToHost, s));
    CR_HIP(hipStreamSynchronize(s));
    *max_its = st[0];
    *not_conv = st[1];
    *perturbed = st[2];
    if (fallbacks) *fallbacks = st[3];
}

void SweepEngine::run(const std::vector<RomDesc>& roms, const std::vector<int2>& items, cr_precision prec, bool refine,
                      hipStream_t s, int* max_its, int* not_conv, int* perturbed, int grid_override, int* fallbacks) {
    prepare(roms, items, s);
    const int gpc = grid_override > 0 ? std::max(1, grid_override / num_cu) : 2;
    launch(prec, refine, gpc, 0, s);
    read_stats(s, max_its, not_conv, perturbed, fallbacks);
}

// Autotune the launch shape on a stratified sample of the prepared items (every k-th item, so
// the sample keeps the order mix): workgroups per CU in {1, 2, 4} x LDS budget in
// {0, 32 KB, 64 KB, 120 KB}. Returns the best (grid_per_cu, lds_bytes) and fills the timings.
void SweepEngine::autotune(const std::vector<RomDesc>& roms, const std::vector<int2>& items, cr_precision prec,
                           bool refine, hipStream_t s, int* best_gpc, int* best_lds, std::vector<double>* ms) {
    const int target = 32 * num_cu;   // enough items that every shape runs several per workgroup
    std::vector<int2> sample;
    const size_t stride = std::max<size_t>(1, items.size() / (size_t)target);
    for (size_t i = 0; i < items.size(); i += stride) sample.push_back(items[i]);
    prepare(roms, sample, s);
    const int gpcs[3] = {1, 2, 4};
    const int ldss[4] = {0, 32768, 65536, 98304};   // static LDS of the kernel is ~50 KB of 160 KB
    hipEvent_t e0, e1;
    CR_HIP(hipEventCreate(&e0));
    CR_HIP(hipEventCreate(&e1));
    double best = 1e300;
    *best_gpc = 2;
    *best_lds = 0;
    if (ms) ms->clear();
    for (int g : gpcs)
        for (int l : ldss) {
            float t = 0;
            try {
                launch(prec, refine, g, l, s);   // warm (allocation, code load)
                CR_HIP(hipEventRecord(e0, s));
                launch(prec, refine, g, l, s);
                CR_HIP(hipEventRecord(e1, s));
                CR_HIP(hipEventSynchronize(e1));
                CR_HIP(hipEventElapsedTime(&t, e0, e1));
            } catch (const Error&) {
                (void)hipGetLastError();   // a shape the device refuses (e.g. LDS budget): skip it
                CR_HIP(hipStreamSynchronize(s));
                if (ms) ms->push_back(-1.0);
                continue;
            }
            if (ms) ms->push_back(t);
            if (t < best) { best = t; *best_gpc = g; *best_lds = l; }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    prepare(roms, items, s);
}


// ---------------------------------------------------------------- allocation-free sweep
// cr_sweep_noalloc keeps everything the sweep needs beyond its inputs and outputs (the model
// descriptor, the work queue, the statistics, the frequencies and the per-workgroup workspaces)
// in one static device array instead of library allocations. Each device holds its own copy for
// the life of the process; host code reaches it only through the address hipGetSymbolAddress
// returns for that device (the array's name is a host-side stand-in, not a device address).
constexpr size_t kNoallocScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_dev[kMaxDevices] = {};

__global__ void k_items_iota(int2* __restrict__ items, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) items[i] = make_int2(0, i);
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
}  // namespace

void noalloc_scratch_init(int device) {
    CR_REQUIRE(device >= 0 && device < kMaxDevices, CR_E_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[device]) return;
    void* p = nullptr;
    CR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    CR_REQUIRE(p != nullptr, CR_E_HIP, "hipGetSymbolAddress returned no address for the sweep scratch");
    g_scratch_dev[device] = static_cast<unsigned char*>(p);
}

size_t noalloc_scratch_bytes() { return kNoallocScratchBytes; }

void sweep_noalloc(int device, int num_cu, const RomDesc& rd_in, const double* omegas_host, int nfreq, cr_precision prec,
                   hipStream_t s, int* max_its, int* not_conv, int* perturbed, int* fallbacks) {
    unsigned char* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (device >= 0 && device < kMaxDevices) base = g_scratch_dev[device];
    }
    CR_REQUIRE(base != nullptr, CR_E_STATE, "cr_sweep_noalloc: the device's scratch was not set up (cr_ctx_create)");
    *max_its = *not_conv = *perturbed = *fallbacks = 0;
    if (nfreq == 0) return;
    const int q = rd_in.q, L = rd_in.L;
    CR_REQUIRE(q >= 1 && q <= 4096 && L >= 1 && L <= kMaxLoads, CR_E_UNSUPPORTED,
               "cr_sweep_noalloc: reduced order or load count out of range");
    // layout: descriptor | statistics | frequencies | work queue | per-workgroup workspaces
    const size_t o_desc = 0, o_stats = 256, o_om = 512;
    const size_t o_items = align256(o_om + sizeof(double) * (size_t)nfreq);
    const size_t head = align256(o_items + sizeof(int2) * (size_t)nfreq);
    const int64_t slot_a = (int64_t)q * q, slot_v = (int64_t)q * L;
    const size_t per_wg = sizeof(zd) * (size_t)slot_a + sizeof(int) * 4096 + 4 * sizeof(zd) * (size_t)slot_v;
    CR_REQUIRE(head + per_wg <= kNoallocScratchBytes, CR_E_UNSUPPORTED,
               "cr_sweep_noalloc: " + std::to_string(nfreq) + " frequencies at order " + std::to_string(q) + " with " +
                   std::to_string(L) + " loads need " + std::to_string(head + per_wg) +
                   " bytes of scratch for one workgroup; the static scratch holds " +
                   std::to_string(kNoallocScratchBytes) + " bytes");
    const int cap = (int)std::min<size_t>((kNoallocScratchBytes - head) / per_wg, (size_t)1 << 20);
    const int grid = std::max(1, std::min({nfreq, 2 * num_cu, cap}));
    RomDesc rd = rd_in;
    rd.omegas = reinterpret_cast<const double*>(base + o_om);
    RomDesc* d_desc = reinterpret_cast<RomDesc*>(base + o_desc);
    int* d_stats = reinterpret_cast<int*>(base + o_stats);
    int2* d_items = reinterpret_cast<int2*>(base + o_items);
    unsigned char* w = base + head;
    zd* wsA = reinterpret_cast<zd*>(w);
    w += sizeof(zd) * (size_t)slot_a * grid;
    int* wsP = reinterpret_cast<int*>(w);
    w += sizeof(int) * (size_t)4096 * grid;
    zd* wsX = reinterpret_cast<zd*>(w);
    zd* wsR = wsX + (size_t)slot_v * grid;
    zd* wsB = wsR + (size_t)slot_v * grid;
    zd* wsD = wsB + (size_t)slot_v * grid;
    CR_HIP(hipMemcpyAsync(d_desc, &rd, sizeof(RomDesc), hipMemcpyHostToDevice, s));
    CR_HIP(hipMemcpyAsync(base + o_om, omegas_host, sizeof(double) * (size_t)nfreq, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_items_iota, dim3(std::min(1024, (nfreq + 255) / 256)), dim3(256), 0, s, d_items, nfreq);
    fill_zero(d_stats, 8, s);
    if (prec == CR_MIXED)
        hipLaunchKernelGGL(k_sweep<float>, dim3(grid), dim3(kWG), 0, s, d_desc, d_items, nfreq, slot_a, slot_v, wsA, wsP,
                           wsX, wsR, wsB, wsD, 1, 10, 1e-14, d_stats, 0);
    else
        hipLaunchKernelGGL(k_sweep<double>, dim3(grid), dim3(kWG), 0, s, d_desc, d_items, nfreq, slot_a, slot_v, wsA, wsP,
                           wsX, wsR, wsB, wsD, 0, 10, 1e-14, d_stats, 0);
    CR_HIP(hipGetLastError());
    int st[8];
    CR_HIP(hipMemcpyAsync(st, d_stats, sizeof(st), hipMemcpyDeviceToHost, s));
    CR_HIP(hipStreamSynchronize(s));
    *max_its = st[0];
    *not_conv = st[1];
    *perturbed = st[2];
    *fallbacks = st[3];
}

}  // namespace cr
