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
//        [3] FP64 fallbacks, [4] dense work-queue counter, [5] Hessenberg work-queue counter
//        (orders <= 256), [6] Hessenberg items handed to the dense path, [7] their work-queue
//        counter, [8] Hessenberg work-queue counter (orders above 256)
// nitems_dev (when not null) holds the item count on the device (the redo list of the Hessenberg
// sweep); qctr is the stats index of this launch's work-queue counter.
template <typename T>
__global__ void __launch_bounds__(kWG) k_sweep(const RomDesc* __restrict__ roms, const int2* __restrict__ items, int nitems,
                                               int64_t slot_a, int64_t slot_v, zd* __restrict__ wsA, int* __restrict__ wsP,
                                               zd* __restrict__ wsX, zd* __restrict__ wsR, zd* __restrict__ wsB,
                                               zd* __restrict__ wsD, int refine, int max_iter, double tol,
                                               int* __restrict__ stats, int q_lds, const int* nitems_dev, int qctr) {
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
    int* counter = stats + qctr;
    if (nitems_dev) nitems = *nitems_dev;
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

// ------------------------------------------------------------ Hessenberg-triangular sweep
// For a model without D_R and frequency-dependent terms the pencil is reduced once to
// Hessenberg-triangular form (unitary Q, Z): Q^H K_R Z = H upper Hessenberg, Q^H M_R Z = Th upper
// triangular; then A_R(w) = Q (H - w^2 Th) Z^H and y = C_R A_R^{-1} b = (C_R Z) (H - w^2 Th)^{-1}
// (Q^H b). Each frequency is an O(q^2) solve with an upper Hessenberg matrix instead of an
// O(q^3) dense LU; the reduction costs O(q^3) once per model.

__device__ __forceinline__ zd zmul(zd a, zd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ zd zconjmul(zd a, zd b) { return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; }   // conj(a) b
__device__ __forceinline__ double zabs1(zd a) { return fabs(a.re) + fabs(a.im); }

// Rotation G = [[c, s], [-conj(s), c]] (c real) with G [a; b] = [r; 0]
__device__ __forceinline__ void givens(zd a, zd b, double& c, zd& s, zd& r) {
    const double aa = hypot(a.re, a.im), bb = hypot(b.re, b.im);
    if (bb == 0.0) {
        c = 1.0;
        s = {0.0, 0.0};
        r = a;
        return;
    }
    if (aa == 0.0) {
        c = 0.0;
        s = {b.re / bb, -b.im / bb};   // conj(b) / |b|
        r = {bb, 0.0};
        return;
    }
    const double nr = hypot(aa, bb);
    c = aa / nr;
    const zd ph = {a.re / aa, a.im / aa};
    s = zmul(ph, zd{b.re / nr, -b.im / nr});   // (a / |a|) conj(b) / r
    r = {ph.re * nr, ph.im * nr};
}

// Moler-Stewart reduction of one model per workgroup (all data in global memory):
//   phase 1: Th upper triangular by row rotations (rows i-1, i), column by column bottom-up, applied
//            to Th, H and Ft (the rotations of a column are chained through that column only, so
//            one thread computes them and every thread then streams its own columns);
//   phase 2: for each column j of H and i = q-1 .. j+2: a row rotation zeroes H[i][j] (applied to
//            H, Th, Ft) and creates Th[i][i-1], which a column rotation on (i-1, i) zeroes
//            (applied to Th, H and Ct). The row rotations of column j are chained through column j
//            of H only (the column rotations touch columns > j), so they are computed up front.
__global__ void __launch_bounds__(kWG) k_ht_reduce(const HtJob* __restrict__ jobs) {
    __shared__ double rc[kHtMaxQ];
    __shared__ zd rs[kHtMaxQ];
    __shared__ zd tpair[2];   // Th[i][i] and Th[i][i-1] after the row rotation of a phase-2 step
    __shared__ double red[8];
    const HtJob jb = jobs[blockIdx.x];
    const int q = jb.q, L = jb.L, no = jb.n_o, t = threadIdx.x;
    zd* __restrict__ H = jb.H;
    zd* __restrict__ T = jb.Th;
    zd* __restrict__ Ft = jb.Ft;
    zd* __restrict__ Ct = jb.Ct;
    for (int e = t; e < q * q; e += kWG) {
        H[e] = jb.KR[e];
        T[e] = jb.MR[e];
    }
    for (int e = t; e < q * L; e += kWG) Ft[e] = jb.FR[e];
    for (int e = t; e < no * q; e += kWG) Ct[e] = jb.CR[e];
    __syncthreads();
    // ---- phase 1
    for (int j = 0; j < q - 1; ++j) {
        if (t == 0) {
            zd b = T[(q - 1) + (size_t)j * q];
            for (int i = q - 1; i > j; --i) {
                const zd a = T[(i - 1) + (size_t)j * q];
                zd r;
                givens(a, b, rc[i], rs[i], r);
                T[i + (size_t)j * q] = {0.0, 0.0};
                b = r;
            }
            T[j + (size_t)j * q] = b;
        }
        __syncthreads();
        const int nT = q - 1 - j, ncol = nT + q + L;
        for (int ci = t; ci < ncol; ci += kWG) {
            zd* x = ci < nT ? T + (size_t)(j + 1 + ci) * q : ci < nT + q ? H + (size_t)(ci - nT) * q : Ft + (size_t)(ci - nT - q) * q;
            zd carry = x[q - 1];
            for (int i = q - 1; i > j; --i) {
                const zd xa = x[i - 1];
                const double c = rc[i];
                const zd s = rs[i];
                const zd sx = zconjmul(s, xa);   // conj(s) xa
                x[i] = {c * carry.re - sx.re, c * carry.im - sx.im};
                const zd sc = zmul(s, carry);
                carry = {c * xa.re + sc.re, c * xa.im + sc.im};
            }
            x[j] = carry;
        }
        __syncthreads();
    }
    // ---- phase 2
    for (int j = 0; j + 2 < q; ++j) {
        if (t == 0) {
            zd b = H[(q - 1) + (size_t)j * q];
            for (int i = q - 1; i > j + 1; --i) {
                const zd a = H[(i - 1) + (size_t)j * q];
                zd r;
                givens(a, b, rc[i], rs[i], r);
                H[i + (size_t)j * q] = {0.0, 0.0};
                b = r;
            }
            H[(j + 1) + (size_t)j * q] = b;
        }
        __syncthreads();
        for (int i = q - 1; i > j + 1; --i) {
            const double c = rc[i];
            const zd s = rs[i];
            // row rotation on rows (i-1, i): H columns j+1..q-1, Th columns i-1..q-1, Ft columns
            const int nH = q - 1 - j, nT = q - i + 1, ncol = nH + nT + L;
            for (int ci = t; ci < ncol; ci += kWG) {
                int col;
                zd* x;
                if (ci < nH) { col = j + 1 + ci; x = H + (size_t)col * q; }
                else if (ci < nH + nT) { col = i - 1 + (ci - nH); x = T + (size_t)col * q; }
                else { col = -1; x = Ft + (size_t)(ci - nH - nT) * q; }
                const zd xa = x[i - 1], xb = x[i];
                const zd sb = zmul(s, xb), sa = zconjmul(s, xa);
                const zd na = {c * xa.re + sb.re, c * xa.im + sb.im};
                const zd nb = {c * xb.re - sa.re, c * xb.im - sa.im};
                x[i - 1] = na;
                x[i] = nb;
                if (ci >= nH && ci < nH + nT) {
                    if (col == i) tpair[0] = nb;        // Th[i][i]
                    if (col == i - 1) tpair[1] = nb;    // Th[i][i-1] (the fill)
                }
            }
            __syncthreads();
            // column rotation on (i-1, i) zeroing Th[i][i-1]: [x_{i-1}, x_i] G with G [Th_ii; Th_i,i-1] = [r; 0]
            double c2;
            zd s2, r2;
            givens(tpair[0], tpair[1], c2, s2, r2);
            const int nrow = (i + 1) + q + no;
            for (int ri = t; ri < nrow; ri += kWG) {
                zd *x0, *x1;
                if (ri <= i) { x0 = T + ri + (size_t)(i - 1) * q; x1 = T + ri + (size_t)i * q; }
                else if (ri < i + 1 + q) { const int rr = ri - (i + 1); x0 = H + rr + (size_t)(i - 1) * q; x1 = H + rr + (size_t)i * q; }
                else { const int rr = ri - (i + 1) - q; x0 = Ct + rr + (size_t)(i - 1) * no; x1 = Ct + rr + (size_t)i * no; }
                const zd a0 = *x0, a1 = *x1;
                const zd sc = zconjmul(s2, a1);   // conj(s) x_i
                const zd sa = zmul(s2, a0);
                *x0 = {c2 * a0.re - sc.re, c2 * a0.im - sc.im};
                *x1 = {sa.re + c2 * a1.re, sa.im + c2 * a1.im};
                if (ri == i) *x0 = {0.0, 0.0};   // Th[i][i-1], zero up to rounding
            }
            __syncthreads();
        }
    }
    // largest entries of the Hessenberg and triangular parts (the pivot threshold of the sweep)
    double hm = 0, tm = 0;
    for (int e = t; e < q * q; e += kWG) {
        const int i = e % q, jj = e / q;
        if (i <= jj + 1) hm = fmax(hm, zabs1(H[e]));
        if (i <= jj) tm = fmax(tm, zabs1(T[e]));
    }
    for (int off = 32; off > 0; off >>= 1) {
        hm = fmax(hm, __shfl_xor(hm, off));
        tm = fmax(tm, __shfl_xor(tm, off));
    }
    if ((t & 63) == 0) { red[t >> 6] = hm; red[4 + (t >> 6)] = tm; }
    __syncthreads();
    if (t == 0) {
        jb.htnorm[0] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        jb.htnorm[1] = fmax(fmax(red[4], red[5]), fmax(red[6], red[7]));
    }
}

// A pointer read from a descriptor in memory is a generic one, and loads through it are flat
// memory instructions, which also count against the LDS wait counter; the kernels' descriptors
// hold global-memory arrays only, so they say so.
#if defined(__HIP_DEVICE_COMPILE__)
#define CR_GLOBAL_AS __attribute__((address_space(1)))
#else
#define CR_GLOBAL_AS   // the host pass only parses kernel bodies
#endif
template <typename T>
__device__ __forceinline__ const CR_GLOBAL_AS T* gp(const T* p) {
    return (const CR_GLOBAL_AS T*)p;
}
template <typename T>
__device__ __forceinline__ CR_GLOBAL_AS T* gpw(T* p) {
    return (CR_GLOBAL_AS T*)p;
}


// One (model, frequency) item of a Hessenberg model per workgroup pass: A = H - w^2 Th (upper
// Hessenberg). Column elimination from the bottom: at step k = q-1 .. 1 the columns (k-1, k) are
// swapped when |A[k][k-1]| > |A[k][k]| (partial pivoting on row k) and column k-1 loses mu times
// column k so that A[k][k-1] = 0; column k and row k are then final (A E = A' upper triangular,
// E the product of the column operations), so y_k = b_k / A'[k][k] and b_i -= A'[i][k] y_k
// (i < k) at once: back substitution fused with the elimination, nothing stored. The outputs
// Y = (C_R Z) x = (C_R Z E) y: the same column operations on Ct's columns, whose final column k
// multiplies y_k. NT threads (q <= NT): thread t owns row t of A and b, and the top n_o threads
// own the output rows (threads NT - n_o + o), so that they hold no row of A when q + n_o <= NT.
// A pivot below eps^2 max|A| (numerically singular) is replaced in its direction and the item
// is listed in `redo` for the dense path with FP64 refinement. qctr: stats index of the queue.
template <int NT>
__global__ void __launch_bounds__(NT) k_sweep_hess(const RomDesc* __restrict__ roms, const int2* __restrict__ items,
                                                   int nitems, int* __restrict__ stats, int2* __restrict__ redo, int qctr) {
    constexpr int R = 1;
    __shared__ int s_item;
    __shared__ zd s_y[2][kHtMaxL];
    __shared__ zd s_mu[2];
    __shared__ int s_sw[2];
    __shared__ int s_pert;
    const int t = threadIdx.x;
    int* counter = stats + qctr;
    for (;;) {
        if (t == 0) {
            s_item = atomicAdd(counter, 1);
            s_pert = 0;
        }
        __syncthreads();
        const int next = s_item;
        __syncthreads();
        if (next >= nitems) break;
        const int2 it = items[next];
        const RomDesc rd = roms[it.x];
        const int q = rd.q, L = rd.L, no = rd.n_o;
        const double w = rd.omegas[it.y], w2 = w * w;
        const auto H = gp(rd.H);
        const auto Th = gp(rd.Th);
        const auto Ct = gp(rd.Ct);
        const auto Ft = gp(rd.Ft);
        const auto flags = gp(rd.flags);
        const double tiny = (gp(rd.htnorm)[0] + w2 * gp(rd.htnorm)[1]) * 1.23e-32;   // eps^2 max|A|
        auto aval = [&](int i, int jj) -> zd {
            const zd h = H[i + (size_t)jj * q];
            if (i > jj) return h;
            const zd tt = Th[i + (size_t)jj * q];
            return {h.re - w2 * tt.re, h.im - w2 * tt.im};
        };
        // u[r]: row i of the original column k-1 at step k; u1, u2: columns k-2, k-3 (loaded
        // three steps ahead of their use)
        zd c[R], u[R], u1[R], u2[R], b[R][kHtMaxL];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = t + NT * r;
            c[r] = u[r] = u1[r] = u2[r] = zd{0.0, 0.0};
#pragma unroll
            for (int l = 0; l < kHtMaxL; ++l) b[r][l] = zd{0.0, 0.0};
            if (i < q) {
                c[r] = aval(i, q - 1);
                if (q >= 2) u[r] = aval(i, q - 2);
                if (q >= 3 && i <= q - 2) u1[r] = aval(i, q - 3);
                if (q >= 4 && i <= q - 3) u2[r] = aval(i, q - 4);
#pragma unroll
                for (int l = 0; l < kHtMaxL; ++l) {
                    if (l < L) {
                        const zd f = Ft[i + (size_t)l * q];
                        b[r][l] = flags[l] ? zd{-w * f.im, w * f.re} : f;
                    }
                }
            }
        }
        const int o = t - (NT - no);   // output row of this thread, if o >= 0
        const bool orow = o >= 0;
        zd cw = {0.0, 0.0}, uw = {0.0, 0.0}, uw1 = {0.0, 0.0}, uw2 = {0.0, 0.0}, yo[kHtMaxL];
#pragma unroll
        for (int l = 0; l < kHtMaxL; ++l) yo[l] = zd{0.0, 0.0};
        if (orow) {
            cw = Ct[o + (size_t)(q - 1) * no];
            if (q >= 2) uw = Ct[o + (size_t)(q - 2) * no];
            if (q >= 3) uw1 = Ct[o + (size_t)(q - 3) * no];
            if (q >= 4) uw2 = Ct[o + (size_t)(q - 4) * no];
        }
        for (int k = q - 1; k >= 0; --k) {
            const int sl = k & 1;
            // the owner of row k: pivot, multiplier and y_k
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (t + NT * r != k) continue;
                zd piv = c[r], oth = u[r];
                int sw = 0;
                if (k > 0 && zabs1(oth) > zabs1(piv)) {
                    const zd x = piv;
                    piv = oth;
                    oth = x;
                    sw = 1;
                }
                if (!(zabs1(piv) > tiny)) {
                    const double mg = zabs1(piv);
                    piv = mg > 0 ? zd{piv.re / mg * tiny, piv.im / mg * tiny} : zd{tiny, 0.0};
                    s_pert = 1;
                }
                const double den = piv.re * piv.re + piv.im * piv.im;
                const zd inv = {piv.re / den, -piv.im / den};
                s_mu[sl] = zmul(oth, inv);
                s_sw[sl] = sw;
#pragma unroll
                for (int l = 0; l < kHtMaxL; ++l)
                    if (l < L) s_y[sl][l] = zmul(b[r][l], inv);
            }
            lds_barrier();   // the step's pivot data; column prefetches stay in flight
            const zd mu = s_mu[sl];
            const int sw = s_sw[sl];
            // column operation on the thread's rows and output row: cc[r] / ccw = final column k
            zd cc[R], ccw = {0.0, 0.0};
            bool act[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = t + NT * r;
                act[r] = i < k;
                cc[r] = zd{0.0, 0.0};
                if (!act[r]) continue;
                zd uu = u[r], c0 = c[r];
                if (sw) { const zd x = uu; uu = c0; c0 = x; }
                const zd m = zmul(mu, c0);
                c[r] = {uu.re - m.re, uu.im - m.im};   // column k-1 after the operation
                cc[r] = c0;
                u[r] = u1[r];
                u1[r] = u2[r];
                if (k >= 4 && i <= k - 3) u2[r] = aval(i, k - 4);   // used at step k - 3
            }
            if (orow) {
                zd uu = uw, c0 = cw;
                if (sw) { const zd x = uu; uu = c0; c0 = x; }
                if (k > 0) {
                    const zd m = zmul(mu, c0);
                    cw = {uu.re - m.re, uu.im - m.im};
                }
                ccw = c0;
                uw = uw1;
                uw1 = uw2;
                if (k >= 4) uw2 = Ct[o + (size_t)(k - 4) * no];
            }
            // b_i -= A'[i][k] y_k and Y_o += W'[o][k] y_k, y_k read from LDS load by load
#pragma unroll
            for (int l = 0; l < kHtMaxL; ++l) {
                const zd yl = l < L ? s_y[sl][l] : zd{0.0, 0.0};
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const zd p = zmul(cc[r], yl);
                    b[r][l] = {b[r][l].re - p.re, b[r][l].im - p.im};
                }
                const zd p = zmul(ccw, yl);
                yo[l] = {yo[l].re + p.re, yo[l].im + p.im};
            }
        }
        __syncthreads();
        if (s_pert) {
            if (t == 0) {
                const int slot = atomicAdd(stats + 6, 1);
                redo[slot] = it;
                atomicAdd(stats + 2, 1);
            }
        } else if (orow) {
            auto yout = gpw(rd.out + (size_t)it.y * L * no);
#pragma unroll
            for (int l = 0; l < kHtMaxL; ++l)
                if (l < L) yout[o + (size_t)l * no] = yo[l];
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
    qht = 0;
    for (const RomDesc& r : roms) {
        qmax = std::max(qmax, r.q);
        Lmax = std::max(Lmax, r.L);
        if (r.H) qht = std::max(qht, r.q);
    }
    CR_REQUIRE(qmax <= 4096, CR_E_UNSUPPORTED, "reduced order above 4096");
    CR_REQUIRE(Lmax <= 64, CR_E_UNSUPPORTED, "more than 64 load columns in a reduced model");
    // dense-LU items first (in the given order), then the Hessenberg models' items of order above
    // 256, then the other Hessenberg items
    std::vector<int2> ordered;
    ordered.reserve(items.size());
    for (const int2& it : items)
        if (!roms[it.x].H) ordered.push_back(it);
    nitems = (int)ordered.size();
    for (const int2& it : items)
        if (roms[it.x].H && roms[it.x].q > kWG) ordered.push_back(it);
    nht_big = (int)ordered.size() - nitems;
    for (const int2& it : items)
        if (roms[it.x].H && roms[it.x].q <= kWG) ordered.push_back(it);
    nht = (int)ordered.size() - nitems;
    d_roms.reserve(roms.size());
    d_items.reserve(ordered.size());
    d_redo.reserve(std::max(nht, 1));
    d_stats.reserve(16);
    if (!roms.empty())
        CR_HIP(hipMemcpyAsync(d_roms.p, roms.data(), roms.size() * sizeof(RomDesc), hipMemcpyHostToDevice, s));
    if (!ordered.empty())
        CR_HIP(hipMemcpyAsync(d_items.p, ordered.data(), ordered.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    CR_HIP(hipStreamSynchronize(s));
}

// Launch the prepared items with grid = min(items, grid_per_cu * CUs) resident workgroups and an
// LDS budget for the LDS-resident variant. Only kernels are enqueued (no memset / memcpy), so
// the launch can be captured in a graph.
void SweepEngine::launch(cr_precision prec, bool refine, int grid_per_cu, int lds_bytes, hipStream_t s) {
    if (nitems + nht == 0) return;
    const int64_t slot_a = (int64_t)qmax * qmax, slot_v = (int64_t)qmax * std::max(Lmax, 1);
    const int grid = std::min<int>(std::max(nitems, nht), std::max(1, grid_per_cu) * num_cu);
    wsA.reserve((size_t)grid * slot_a);
    wsP.reserve((size_t)grid * 4096);
    wsX.reserve((size_t)grid * slot_v);
    wsR.reserve((size_t)grid * slot_v);
    wsB.reserve((size_t)grid * slot_v);
    wsD.reserve((size_t)grid * slot_v);
    fill_zero(d_stats.p, 16, s);
    const int q_lds = q_lds_for(prec, lds_bytes);
    const size_t dyn = q_lds > 0 ? (size_t)lds_bytes : 0;
    ProfScope ps(ctx, "sweep", s);
    if (nitems > 0) {
        const int g = std::min(grid, nitems);
        if (prec == CR_MIXED) {
            if (dyn > 65536) CR_HIP(hipFuncSetAttribute((const void*)k_sweep<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
            hipLaunchKernelGGL(k_sweep<float>, dim3(g), dim3(kWG), dyn, s, d_roms.p, d_items.p, nitems, slot_a, slot_v,
                               wsA.p, wsP.p, wsX.p, wsR.p, wsB.p, wsD.p, 1, 10, 1e-14, d_stats.p, q_lds, nullptr, 4);
        } else {
            if (dyn > 65536) CR_HIP(hipFuncSetAttribute((const void*)k_sweep<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
            hipLaunchKernelGGL(k_sweep<double>, dim3(g), dim3(kWG), dyn, s, d_roms.p, d_items.p, nitems, slot_a, slot_v,
                               wsA.p, wsP.p, wsX.p, wsR.p, wsB.p, wsD.p, refine ? 1 : 0, 10, 1e-14, d_stats.p, q_lds,
                               nullptr, 4);
        }
    }
    if (nht > 0) {
        // Hessenberg models (FP64, no refinement requested): one item per workgroup pass, then
        // the items with a numerically singular pivot through the dense path with refinement
        // orders above 256 first (512-thread workgroups, one per compute unit), then the others
        const int g = std::min(nht, std::max(1, grid_per_cu) * num_cu);
        if (nht_big > 0)
            hipLaunchKernelGGL(k_sweep_hess<2 * kWG>, dim3(std::min(nht_big, num_cu)), dim3(2 * kWG), 0, s, d_roms.p,
                               d_items.p + nitems, nht_big, d_stats.p, d_redo.p, 8);
        if (nht > nht_big)
            hipLaunchKernelGGL(k_sweep_hess<kWG>, dim3(std::min(g, nht - nht_big)), dim3(kWG), 0, s, d_roms.p,
                               d_items.p + nitems + nht_big, nht - nht_big, d_stats.p, d_redo.p, 5);
        hipLaunchKernelGGL(k_sweep<double>, dim3(std::min(g, num_cu)), dim3(kWG), 0, s, d_roms.p, d_redo.p, 0, slot_a,
                           slot_v, wsA.p, wsP.p, wsX.p, wsR.p, wsB.p, wsD.p, 1, 10, 1e-14, d_stats.p, 0,
                           d_stats.p + 6, 7);
    }
    CR_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- reduction to HT form
void ht_reduce(const std::vector<HtJob>& jobs, hipStream_t s) {
    if (jobs.empty()) return;
    for (const HtJob& j : jobs)
        CR_REQUIRE(j.q >= 1 && j.q <= kHtMaxQ && j.L >= 1 && j.L <= kHtMaxL && j.n_o >= 1 && j.n_o <= kHtMaxOut,
                   CR_E_UNSUPPORTED, "Hessenberg-triangular reduction: model out of range");
    DevBuf<HtJob> d;
    d.alloc(jobs.size());
    CR_HIP(hipMemcpyAsync(d.p, jobs.data(), jobs.size() * sizeof(HtJob), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_ht_reduce, dim3((unsigned)jobs.size()), dim3(kWG), 0, s, d.p);
    CR_HIP(hipGetLastError());
    CR_HIP(hipStreamSynchronize(s));
}

void SweepEngine::read_stats(hipStream_t s, int* max_its, int* not_conv, int* perturbed, int* fallbacks) {
    int st[8] = {0};
    if (nitems + nht > 0) CR_HIP(hipMemcpyAsync(st, d_stats.p, sizeof(st), hipMemcpyDeviceToHost, s));
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
                           wsX, wsR, wsB, wsD, 1, 10, 1e-14, d_stats, 0, nullptr, 4);
    else
        hipLaunchKernelGGL(k_sweep<double>, dim3(grid), dim3(kWG), 0, s, d_desc, d_items, nfreq, slot_a, slot_v, wsA, wsP,
                           wsX, wsR, wsB, wsD, 0, 10, 1e-14, d_stats, 0, nullptr, 4);
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
