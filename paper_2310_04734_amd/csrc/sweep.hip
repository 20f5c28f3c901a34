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
    for (int k = 0; k < q - 1; ++k) {
        const int rows = q - k - 1;
        for (int e = t; e < rows * L; e += kWG) {
            const int i = k + 1 + e % rows, l = e / rows;
            B[i + (size_t)l * q] = cfms(B[i + (size_t)l * q], A[i + (size_t)k * lda], B[k + (size_t)l * q]);
        }
        __syncthreads();
    }
    for (int k = q - 1; k >= 0; --k) {
        const cx<T> d = crecip(A[k + (size_t)k * lda]);
        for (int l = t; l < L; l += kWG) B[k + (size_t)l * q] = cmul(B[k + (size_t)l * q], d);
        __syncthreads();
        for (int e = t; e < k * L; e += kWG) {
            const int i = e % k, l = e / k;
            B[i + (size_t)l * q] = cfms(B[i + (size_t)l * q], A[i + (size_t)k * lda], B[k + (size_t)l * q]);
        }
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

// Factor and solve one reduced system in precision T: A_R(w) rounded to T, LU with partial
// pivoting, X = A_R^{-1} B with FP64 refinement (refine) or a single solve. Returns whether the
// normwise backward error reached tol (always true without refinement).
template <typename T>
__device__ bool solve_item(const RomDesc& rd, double w, cx<T>* __restrict__ A, int* __restrict__ ipiv, zd* __restrict__ X,
                           zd* __restrict__ R, const zd* __restrict__ Bv, cx<T>* __restrict__ D, bool refine, int max_iter,
                           double tol, LuShared<T>& sh, double* red, int* s_perturb, int* its_out) {
    const int t = threadIdx.x;
    const int q = rd.q, L = rd.L;
    const double w2 = w * w;
    double amax = 0;
    for (int e = t; e < q * q; e += kWG) {
        const zd k = rd.KR[e], m = rd.MR[e];
        double re = k.re - w2 * m.re, im = k.im - w2 * m.im;
        if (rd.DR) { const zd d = rd.DR[e]; re -= w * d.im; im += w * d.re; }
        A[e] = {T(re), T(im)};
        amax = fmax(amax, fabs(re) + fabs(im));
    }
    amax = wg_max(amax, red);
    for (int e = t; e < q * L; e += kWG) {
        X[e] = {0.0, 0.0};
        R[e] = Bv[e];
    }
    if (t == 0) *s_perturb = 0;
    __syncthreads();
    const T tiny = sizeof(T) == 4 ? T(3e-4 * amax) : T(1e-8 * amax);
    wg_getrf<T>(A, q, q, q, ipiv, tiny, s_perturb, sh);
    int its = 0;
    double prev = 1e300;
    bool conv = false;
    for (;;) {
        for (int e = t; e < q * L; e += kWG) D[e] = {T(R[e].re), T(R[e].im)};
        __syncthreads();
        wg_lu_solve<T>(A, q, q, ipiv, D, L);
        for (int e = t; e < q * L; e += kWG) { X[e].re += (double)D[e].re; X[e].im += (double)D[e].im; }
        __syncthreads();
        if (!refine) { conv = true; break; }
        // R = B - A_R X in FP64; backward error max ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf),
        // pooled over the load columns
        double anorm_part = 0, rmax = 0, xmax = 0, bmax = 0;
        for (int e = t; e < q * L; e += kWG) {
            const int i = e % q, l = e / q;
            double rr = Bv[e].re, ri = Bv[e].im, rowsum = 0;
            for (int j = 0; j < q; ++j) {
                const zd k = rd.KR[i + (size_t)j * q], m = rd.MR[i + (size_t)j * q];
                double ar = k.re - w2 * m.re, ai = k.im - w2 * m.im;
                if (rd.DR) { const zd d = rd.DR[i + (size_t)j * q]; ar -= w * d.im; ai += w * d.re; }
                const zd x = X[j + (size_t)l * q];
                rr -= ar * x.re - ai * x.im;
                ri -= ar * x.im + ai * x.re;
                if (l == 0) rowsum += hypot(ar, ai);
            }
            R[e] = {rr, ri};
            anorm_part = fmax(anorm_part, rowsum);
            rmax = fmax(rmax, hypot(rr, ri));
            xmax = fmax(xmax, hypot(X[e].re, X[e].im));
            bmax = fmax(bmax, hypot(Bv[e].re, Bv[e].im));
        }
        const double an = wg_max(anorm_part, red);
        const double rn = wg_max(rmax, red);
        const double xn = wg_max(xmax, red);
        const double bn = wg_max(bmax, red);
        const double be = rn / (an * xn + bn);
        if (be <= tol) { conv = true; break; }
        if (its >= max_iter || !(be < 0.5 * prev)) break;
        prev = be;
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
                                               int* __restrict__ stats) {
    __shared__ LuShared<double> sh;   // large enough for the FP32 variant as well
    __shared__ double red[8];
    __shared__ int s_item;
    __shared__ int s_perturb;
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
        int its = 0, fell_back = 0;
        bool conv = solve_item<T>(rd, w, reinterpret_cast<cx<T>*>(Aslot), ipiv, X, R, Bv, reinterpret_cast<cx<T>*>(Dslot),
                                  refine != 0, max_iter, tol, reinterpret_cast<LuShared<T>&>(sh), red, &s_perturb, &its);
        if (!conv && sizeof(T) == 4) {
            // complex-FP32 LU too inaccurate for refinement to converge (kappa(A_R) u_32 >~ 1):
            // redo this frequency with a complex-FP64 LU
            fell_back = 1;
            int its2 = 0;
            conv = solve_item<double>(rd, w, reinterpret_cast<cx<double>*>(Aslot), ipiv, X, R, Bv,
                                      reinterpret_cast<cx<double>*>(Dslot), true, max_iter, tol, sh, red, &s_perturb, &its2);
            its += its2;
        }
        if (rd.out_x) {
            zd* o = rd.out + (size_t)it.y * q * L;
            for (int e = t; e < q * L; e += kWG) o[e] = X[e];
        } else {
            const int no = rd.n_o;
            zd* o = rd.out + (size_t)it.y * L * no;
            for (int e = t; e < no * L; e += kWG) {
                const int oo = e % no, l = e / no;
                double yr = 0, yi = 0;
                for (int k = 0; k < q; ++k) {
                    const zd c = rd.CR[oo + (size_t)k * no], x = X[k + (size_t)l * q];
                    yr += c.re * x.re - c.im * x.im;
                    yi += c.re * x.im + c.im * x.re;
                }
                o[oo + (size_t)l * no] = {yr, yi};
            }
        }
        if (t == 0) {
            atomicMax(stats + 0, its);
            if (!conv) atomicAdd(stats + 1, 1);
            if (s_perturb) atomicAdd(stats + 2, s_perturb);
            if (fell_back) atomicAdd(stats + 3, 1);
        }
        __syncthreads();
    }
}

}  // namespace

void SweepEngine::run(const std::vector<RomDesc>& roms, const std::vector<int2>& items, cr_precision prec, bool refine,
                      hipStream_t s, int* max_its, int* not_conv, int* perturbed, int grid_override, int* fallbacks) {
    if (fallbacks) *fallbacks = 0;
    if (items.empty()) {
        *max_its = *not_conv = *perturbed = 0;
        return;
    }
    int qmax = 0, Lmax = 0;
    for (const RomDesc& r : roms) {
        qmax = std::max(qmax, r.q);
        Lmax = std::max(Lmax, r.L);
    }
    CR_REQUIRE(qmax <= 4096, CR_E_UNSUPPORTED, "reduced order above 4096");
    const int64_t slot_a = (int64_t)qmax * qmax, slot_v = (int64_t)qmax * std::max(Lmax, 1);
    const int grid = grid_override > 0 ? std::min<int>((int)items.size(), grid_override)
                                       : std::min<int>((int)items.size(), 2 * num_cu);
    d_roms.reserve(roms.size());
    d_items.reserve(items.size());
    d_stats.reserve(8);
    CR_HIP(hipMemcpyAsync(d_roms.p, roms.data(), roms.size() * sizeof(RomDesc), hipMemcpyHostToDevice, s));
    CR_HIP(hipMemcpyAsync(d_items.p, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    fill_zero(d_stats.p, 8, s);
    wsA.reserve((size_t)grid * slot_a);
    wsP.reserve((size_t)grid * 4096);
    wsX.reserve((size_t)grid * slot_v);
    wsR.reserve((size_t)grid * slot_v);
    wsB.reserve((size_t)grid * slot_v);
    wsD.reserve((size_t)grid * slot_v);
    ProfScope ps(ctx, "sweep", s);
    if (prec == CR_MIXED) {
        hipLaunchKernelGGL(k_sweep<float>, dim3(grid), dim3(kWG), 0, s, d_roms.p, d_items.p, (int)items.size(), slot_a,
                           slot_v, wsA.p, wsP.p, wsX.p, wsR.p, wsB.p, wsD.p, 1, 10, 1e-14, d_stats.p);
    } else {
        hipLaunchKernelGGL(k_sweep<double>, dim3(grid), dim3(kWG), 0, s, d_roms.p, d_items.p, (int)items.size(), slot_a,
                           slot_v, wsA.p, wsP.p, wsX.p, wsR.p, wsB.p, wsD.p, refine ? 1 : 0, 10, 1e-14, d_stats.p);
    }
    CR_HIP(hipGetLastError());
    int st[8];
    CR_HIP(hipMemcpyAsync(st, d_stats.p, sizeof(st), hipMemcpyDeviceToHost, s));
    CR_HIP(hipStreamSynchronize(s));
    *max_its = st[0];
    *not_conv = st[1];
    *perturbed = st[2];
    if (fallbacks) *fallbacks = st[3];
}

}  // namespace cr
