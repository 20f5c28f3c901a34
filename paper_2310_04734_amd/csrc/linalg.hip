// FP64 sparse and tall-skinny kernels of the basis build:
//   * CSR SpMM with the scaled K~ and M~ (shared pattern): (K~ - s M~) X, the refinement
//     residual B - (K~ - s M~) X, and the pair K~ X, M~ X for the projection;
//   * column norms for the backward error of the refinement;
//   * Gram products H = A^H B of tall-skinny blocks (two passes of these plus the update
//     W -= V H make the block classical Gram-Schmidt, CGS2);
//   * the receiver gather C_R = S_recv V_recv and the candidate residual norms of the greedy.
// Reductions are two-stage with a fixed order (per-workgroup partials, then one ordered sum),
// so every result is bit-reproducible from run to run.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <complex>
#include <cstring>

#include "dense.cuh"
#include "internal.h"
#include "util.cuh"

namespace cr {
namespace {

constexpr int kRowLanes = 8;   // lanes per CSR row

// MODE 0: Y = (K - s M) X     MODE 1: Y = B - (K - s M) X     MODE 2: Y = K X, Y2 = M X     MODE 3: Y = M X
// M may be null in modes 0 and 1 (K then holds the pre-formed operator). RC right-hand sides per
// pass over a row: every matrix entry and column index is read once per RC columns of X.
template <int MODE, int RC>
__global__ void __launch_bounds__(256) k_spmm(int64_t n, const int64_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ col, const zd* __restrict__ K,
                                              const zd* __restrict__ M, double s, int nrhs, const zd* __restrict__ X,
                                              int64_t ldx, const zd* __restrict__ B, int64_t ldb, zd* __restrict__ Y,
                                              zd* __restrict__ Y2, int64_t ldy) {
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kRowLanes;
    const int lane = threadIdx.x % kRowLanes;
    const bool valid = row < n;
    const int64_t b = valid ? rowptr[row] : 0, e = valid ? rowptr[row + 1] : 0;
    const bool single = (MODE == 0 || MODE == 1) && M == nullptr;
    for (int l0 = 0; l0 < nrhs; l0 += RC) {
        double ar[RC], ai[RC], br[MODE == 2 ? RC : 1], bi[MODE == 2 ? RC : 1];
#pragma unroll
        for (int c = 0; c < RC; ++c) ar[c] = ai[c] = 0;
#pragma unroll
        for (int c = 0; c < (MODE == 2 ? RC : 1); ++c) br[c] = bi[c] = 0;
        for (int64_t k = b + lane; k < e; k += kRowLanes) {
            const int32_t j = col[k];
            double vr, vi;
            zd mv{0, 0};
            if (MODE == 3) { mv = M[k]; vr = mv.re; vi = mv.im; }
            else {
                const zd kv = K[k];
                if (MODE == 2) { mv = M[k]; vr = kv.re; vi = kv.im; }
                else if (single) { vr = kv.re; vi = kv.im; }
                else { mv = M[k]; vr = kv.re - s * mv.re; vi = kv.im - s * mv.im; }
            }
#pragma unroll
            for (int c = 0; c < RC; ++c) {
                if (l0 + c >= nrhs) break;
                const zd x = X[j + (l0 + c) * ldx];
                ar[c] += vr * x.re - vi * x.im;
                ai[c] += vr * x.im + vi * x.re;
                if (MODE == 2) {
                    br[c] += mv.re * x.re - mv.im * x.im;
                    bi[c] += mv.re * x.im + mv.im * x.re;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < RC; ++c) {
            for (int off = kRowLanes / 2; off > 0; off >>= 1) {
                ar[c] += __shfl_xor(ar[c], off, kRowLanes);
                ai[c] += __shfl_xor(ai[c], off, kRowLanes);
                if (MODE == 2) {
                    br[c] += __shfl_xor(br[c], off, kRowLanes);
                    bi[c] += __shfl_xor(bi[c], off, kRowLanes);
                }
            }
        }
        if (valid && lane == 0) {
#pragma unroll
            for (int c = 0; c < RC; ++c) {
                if (l0 + c >= nrhs) break;
                const int64_t o = row + (l0 + c) * ldy;
                if (MODE == 0 || MODE == 3) Y[o] = {ar[c], ai[c]};
                if (MODE == 1) { const zd bb = B[row + (l0 + c) * ldb]; Y[o] = {bb.re - ar[c], bb.im - ai[c]}; }
                if (MODE == 2) { Y[o] = {ar[c], ai[c]}; Y2[o] = {br[c], bi[c]}; }
            }
        }
    }
}

// out[3*l + {0,1,2}] = max_i |R_il|, |X_il|, |B_il| (atomicMax on the bits of non-negative doubles)
__global__ void k_colmax3(int64_t n, int nrhs, const zd* __restrict__ R, const zd* __restrict__ X, const zd* __restrict__ B,
                          int64_t ld, unsigned long long* out) {
    const int l = blockIdx.y;
    double m0 = 0, m1 = 0, m2 = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const zd r = R[i + l * ld], x = X[i + l * ld], b = B[i + l * ld];
        m0 = fmax(m0, hypot(r.re, r.im));
        m1 = fmax(m1, hypot(x.re, x.im));
        m2 = fmax(m2, hypot(b.re, b.im));
    }
    for (int off = 32; off > 0; off >>= 1) {
        m0 = fmax(m0, __shfl_xor(m0, off));
        m1 = fmax(m1, __shfl_xor(m1, off));
        m2 = fmax(m2, __shfl_xor(m2, off));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(out + 3 * l + 0, (unsigned long long)__double_as_longlong(m0));
        atomicMax(out + 3 * l + 1, (unsigned long long)__double_as_longlong(m1));
        atomicMax(out + 3 * l + 2, (unsigned long long)__double_as_longlong(m2));
    }
}

// ||K~ - s M~||_inf
__global__ void k_rownorm(int64_t n, const int64_t* __restrict__ rowptr, const zd* __restrict__ K, const zd* __restrict__ M,
                          double s, unsigned long long* out) {
    double m = 0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0;
        for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k)
            acc += M ? hypot(K[k].re - s * M[k].re, K[k].im - s * M[k].im) : hypot(K[k].re, K[k].im);
        m = fmax(m, acc);
    }
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

__global__ void k_axpy_copy(int64_t n, const zd* __restrict__ src, zd* __restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace

// ------------------------------------------------------------------ SpMM front-ends
static inline unsigned spmm_blocks(int64_t n) { return (unsigned)((n * kRowLanes + 255) / 256); }

// one launch of k_spmm<MODE, RC> with RC the smallest chunk of {4, 8, 16} that covers nrhs
template <int MODE>
static void spmm_launch(cr_sys sys, const zd* Kv, const zd* Mv, double sigma, int nrhs, const zd* X, int64_t ldx,
                        const zd* B, int64_t ldb, zd* Y, zd* Y2, int64_t ldy, hipStream_t s) {
    ProfScope ps(sys->ctx, "spmm", s);
    const dim3 grid(spmm_blocks(sys->n)), blk(256);
    if (nrhs <= 4 || MODE == 2)
        hipLaunchKernelGGL((k_spmm<MODE, 4>), grid, blk, 0, s, sys->n, sys->d_rowptr.p, sys->d_col.p, Kv, Mv, sigma, nrhs,
                           X, ldx, B, ldb, Y, Y2, ldy);
    else if (nrhs <= 8)
        hipLaunchKernelGGL((k_spmm<MODE, 8>), grid, blk, 0, s, sys->n, sys->d_rowptr.p, sys->d_col.p, Kv, Mv, sigma, nrhs,
                           X, ldx, B, ldb, Y, Y2, ldy);
    else
        hipLaunchKernelGGL((k_spmm<MODE, 16>), grid, blk, 0, s, sys->n, sys->d_rowptr.p, sys->d_col.p, Kv, Mv, sigma,
                           nrhs, X, ldx, B, ldb, Y, Y2, ldy);
}

void spmm_shifted(cr_sys sys, const zd* Kv, const zd* Mv, double sigma, int nrhs, const zd* X, int64_t ldx, zd* Y,
                  int64_t ldy, hipStream_t s) {
    spmm_launch<0>(sys, Kv, Mv, sigma, nrhs, X, ldx, nullptr, 0, Y, nullptr, ldy, s);
}
void spmm_km(cr_sys sys, int nrhs, const zd* X, int64_t ldx, zd* KX, zd* MX, int64_t ldy, hipStream_t s) {
    spmm_launch<2>(sys, sys->d_K.p, sys->d_M.p, 0.0, nrhs, X, ldx, nullptr, 0, KX, MX, ldy, s);
}
void spmm_m(cr_sys sys, int nrhs, const zd* X, int64_t ldx, zd* Y, int64_t ldy, hipStream_t s) {
    spmm_launch<3>(sys, sys->d_K.p, sys->d_M.p, 0.0, nrhs, X, ldx, nullptr, 0, Y, nullptr, ldy, s);
}
void spmm_residual(cr_sys sys, const zd* Kv, const zd* Mv, double sigma, int nrhs, const zd* X, int64_t ldx,
                   const zd* B, int64_t ldb, zd* R, int64_t ldr, hipStream_t s) {
    spmm_launch<1>(sys, Kv, Mv, sigma, nrhs, X, ldx, B, ldb, R, nullptr, ldr, s);
}

double shifted_norm_inf(cr_sys sys, const zd* Kv, const zd* Mv, double sigma, DevBuf<unsigned long long>& scratch,
                        hipStream_t s) {
    scratch.reserve(1);
    fill_zero(scratch.p, 1, s);
    hipLaunchKernelGGL(k_rownorm, dim3(256), dim3(256), 0, s, sys->n, sys->d_rowptr.p, Kv, Mv, sigma, scratch.p);
    unsigned long long h = 0;
    CR_HIP(hipMemcpyAsync(&h, scratch.p, sizeof(h), hipMemcpyDeviceToHost, s));
    CR_HIP(hipStreamSynchronize(s));
    double v;
    std::memcpy(&v, &h, sizeof(v));
    return v;
}

// ------------------------------------------------------------------ batched column kernels
// (one independent vector per right-hand side: basis V_k[:, l] at Vb + k*n*nrhs + l*n)
namespace {

// partial[(chunk * nrhs + l) * kk + k] = sum_{i in chunk} conj(V_k[i, l]) w[i, l]
__global__ void __launch_bounds__(256) k_bdot_partial(int64_t n, int nrhs, int kk, const zd* __restrict__ Vb,
                                                      const zd* __restrict__ w, zd* __restrict__ partial) {
    __shared__ double sr[4], si[4];
    const int l = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const zd wv = i < n ? w[i + (int64_t)l * n] : zd{0, 0};
    for (int k = 0; k < kk; ++k) {
        double r = 0, im = 0;
        if (i < n) {
            const zd v = Vb[(int64_t)k * n * nrhs + (int64_t)l * n + i];
            r = v.re * wv.re + v.im * wv.im;
            im = v.re * wv.im - v.im * wv.re;
        }
        for (int off = 32; off > 0; off >>= 1) {
            r += __shfl_xor(r, off);
            im += __shfl_xor(im, off);
        }
        if ((threadIdx.x & 63) == 0) { sr[threadIdx.x >> 6] = r; si[threadIdx.x >> 6] = im; }
        __syncthreads();
        if (threadIdx.x == 0)
            partial[((size_t)blockIdx.x * nrhs + l) * kk + k] = {((sr[0] + sr[1]) + sr[2]) + sr[3],
                                                                 ((si[0] + si[1]) + si[2]) + si[3]};
        __syncthreads();
    }
}

__global__ void k_bdot_reduce(int nchunk, int nrhs, int kk, const zd* __restrict__ partial, zd* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;   // e = l * kk + k
    if (e >= nrhs * kk) return;
    double r = 0, im = 0;
    for (int c = 0; c < nchunk; ++c) {
        const zd v = partial[(size_t)c * nrhs * kk + e];
        r += v.re;
        im += v.im;
    }
    out[e] = {r, im};
}

// w[i, l] += sign * sum_k V_k[i, l] h[l * kk + k]
__global__ void k_baxpy(int64_t n, int nrhs, int kk, const zd* __restrict__ Vb, const zd* __restrict__ h, double sign,
                        zd* __restrict__ w) {
    const int l = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double ar = 0, ai = 0;
    for (int k = 0; k < kk; ++k) {
        const zd v = Vb[(int64_t)k * n * nrhs + (int64_t)l * n + i], c = h[l * kk + k];
        ar += v.re * c.re - v.im * c.im;
        ai += v.re * c.im + v.im * c.re;
    }
    zd& d = w[i + (int64_t)l * n];
    d.re += sign * ar;
    d.im += sign * ai;
}

__global__ void k_bscale_into(int64_t n, int nrhs, const zd* __restrict__ src, const double* __restrict__ inv,
                              zd* __restrict__ dst) {
    const int l = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const zd v = src[i + (int64_t)l * n];
    dst[i + (int64_t)l * n] = {v.re * inv[l], v.im * inv[l]};
}

}  // namespace

struct BatchCols {
    int64_t n;
    int nrhs;
    DevBuf<zd> partial, dots;
    std::vector<zd> hd;
    void dot(const zd* Vb, int kk, const zd* w, hipStream_t s, std::vector<zd>& out) {
        const int nchunk = (int)((n + 255) / 256);
        partial.reserve((size_t)nchunk * nrhs * kk);
        dots.reserve((size_t)nrhs * kk);
        hipLaunchKernelGGL(k_bdot_partial, dim3(nchunk, nrhs), dim3(256), 0, s, n, nrhs, kk, Vb, w, partial.p);
        hipLaunchKernelGGL(k_bdot_reduce, dim3((nrhs * kk + 255) / 256), dim3(256), 0, s, nchunk, nrhs, kk, partial.p,
                           dots.p);
        out.resize((size_t)nrhs * kk);
        CR_HIP(hipMemcpyAsync(out.data(), dots.p, out.size() * sizeof(zd), hipMemcpyDeviceToHost, s));
        CR_HIP(hipStreamSynchronize(s));
    }
    void axpy(const zd* Vb, int kk, const std::vector<zd>& h, double sign, zd* w, hipStream_t s) {
        dots.reserve((size_t)nrhs * kk);
        CR_HIP(hipMemcpyAsync(dots.p, h.data(), (size_t)nrhs * kk * sizeof(zd), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_baxpy, dim3((unsigned)((n + 255) / 256), nrhs), dim3(256), 0, s, n, nrhs, kk, Vb, dots.p,
                           sign, w);
        CR_HIP(hipStreamSynchronize(s));
    }
};

// One GMRES(m) cycle on the left-preconditioned system (LU)^{-1} A~ d = (LU)^{-1} r, every
// right-hand side with its own Krylov basis (FP64 vectors, CGS2, Givens rotations on the host);
// X += d. Returns the number of preconditioned operator applications.
static int gmres_cycle(Factor& f, int nrhs, const zd* R, zd* X, int m, double rtol, SolveWork& w, hipStream_t s) {
    cr_sys sys = f.sys;
    const int64_t n = sys->n;
    const size_t blk = (size_t)n * nrhs;
    w.kry.reserve(blk * (m + 1));
    w.d.reserve(blk);
    zd* Vb = w.kry.p;
    zd* tmp = w.d.p;
    BatchCols bc{n, nrhs};
    DevBuf<double> inv(nrhs);
    std::vector<double> hinv(nrhs);
    // v0 = z / ||z||, z = LU^{-1} r
    apply_factor(f, nrhs, R, n, tmp, n, 0, w, s);
    std::vector<zd> dd;
    bc.dot(tmp, 1, tmp, s, dd);   // ||z_l||^2 (Vb slot 0 used as a one-vector basis: tmp)
    std::vector<double> beta(nrhs);
    for (int l = 0; l < nrhs; ++l) {
        beta[l] = std::sqrt(std::max(dd[l].re, 0.0));
        hinv[l] = beta[l] > 0 ? 1.0 / beta[l] : 0.0;
    }
    CR_HIP(hipMemcpyAsync(inv.p, hinv.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_bscale_into, dim3((unsigned)((n + 255) / 256), nrhs), dim3(256), 0, s, n, nrhs, tmp, inv.p, Vb);
    // Hessenberg columns and Givens rotations per right-hand side
    std::vector<std::vector<std::complex<double>>> H(nrhs, std::vector<std::complex<double>>((size_t)(m + 1) * m));
    std::vector<std::vector<std::complex<double>>> g(nrhs, std::vector<std::complex<double>>(m + 1));
    std::vector<std::vector<double>> cs(nrhs, std::vector<double>(m));
    std::vector<std::vector<std::complex<double>>> sn(nrhs, std::vector<std::complex<double>>(m));
    for (int l = 0; l < nrhs; ++l) g[l][0] = beta[l];
    std::vector<char> done(nrhs, 0);
    for (int l = 0; l < nrhs; ++l) done[l] = beta[l] == 0;
    int j = 0, applications = 1;
    for (; j < m; ++j) {
        bool all = true;
        for (int l = 0; l < nrhs; ++l) all = all && done[l];
        if (all) break;
        zd* vj = Vb + blk * j;
        zd* vn = Vb + blk * (j + 1);
        spmm_shifted(sys, f.opA, nullptr, 0.0, nrhs, vj, n, w.r.p, n, s);   // A v_j (FP64)
        apply_factor(f, nrhs, w.r.p, n, vn, n, 0, w, s);            // (LU)^{-1} A v_j
        ++applications;
        std::vector<zd> h1, h2;
        bc.dot(Vb, j + 1, vn, s, h1);
        bc.axpy(Vb, j + 1, h1, -1.0, vn, s);
        bc.dot(Vb, j + 1, vn, s, h2);
        bc.axpy(Vb, j + 1, h2, -1.0, vn, s);
        bc.dot(vn, 1, vn, s, dd);
        for (int l = 0; l < nrhs; ++l) {
            const double hn = std::sqrt(std::max(dd[l].re, 0.0));
            hinv[l] = (hn > 0 && !done[l]) ? 1.0 / hn : 0.0;
            auto& Hl = H[l];
            for (int k = 0; k <= j; ++k)
                Hl[k + (size_t)j * (m + 1)] = {h1[l * (j + 1) + k].re + h2[l * (j + 1) + k].re,
                                               h1[l * (j + 1) + k].im + h2[l * (j + 1) + k].im};
            Hl[j + 1 + (size_t)j * (m + 1)] = hn;
            // apply previous rotations, then a new one zeroing H[j+1, j]
            for (int k = 0; k < j; ++k) {
                const std::complex<double> a = Hl[k + (size_t)j * (m + 1)], b = Hl[k + 1 + (size_t)j * (m + 1)];
                Hl[k + (size_t)j * (m + 1)] = cs[l][k] * a + sn[l][k] * b;
                Hl[k + 1 + (size_t)j * (m + 1)] = -std::conj(sn[l][k]) * a + cs[l][k] * b;
            }
            const std::complex<double> a = Hl[j + (size_t)j * (m + 1)];
            const double bb = hn;
            const double r = std::sqrt(std::norm(a) + bb * bb);
            if (r > 0) {
                cs[l][j] = std::abs(a) / r;
                const std::complex<double> ph = std::abs(a) > 0 ? a / std::abs(a) : std::complex<double>(1.0, 0.0);
                sn[l][j] = ph * bb / r;
                Hl[j + (size_t)j * (m + 1)] = ph * r;
            } else {
                cs[l][j] = 1.0;
                sn[l][j] = 0.0;
            }
            Hl[j + 1 + (size_t)j * (m + 1)] = 0.0;
            g[l][j + 1] = -std::conj(sn[l][j]) * g[l][j];
            g[l][j] = cs[l][j] * g[l][j];
            if (!done[l] && (std::abs(g[l][j + 1]) <= rtol * beta[l] || hn == 0)) done[l] = 2;
        }
        CR_HIP(hipMemcpyAsync(inv.p, hinv.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_bscale_into, dim3((unsigned)((n + 255) / 256), nrhs), dim3(256), 0, s, n, nrhs, vn, inv.p, vn);
    }
    // y = H^{-1} g per right-hand side (back substitution over the columns each one used), X += V y
    const int kk = j;
    if (kk > 0) {
        std::vector<zd> y((size_t)nrhs * kk, zd{0, 0});
        for (int l = 0; l < nrhs; ++l) {
            if (beta[l] == 0) continue;
            std::vector<std::complex<double>> yl(kk);
            for (int k = kk - 1; k >= 0; --k) {
                std::complex<double> acc = g[l][k];
                for (int c = k + 1; c < kk; ++c) acc -= H[l][k + (size_t)c * (m + 1)] * yl[c];
                const std::complex<double> dgl = H[l][k + (size_t)k * (m + 1)];
                yl[k] = std::abs(dgl) > 0 ? acc / dgl : 0.0;
            }
            for (int k = 0; k < kk; ++k) y[(size_t)l * kk + k] = {yl[k].real(), yl[k].imag()};
        }
        bc.axpy(Vb, kk, y, 1.0, X, s);
    }
    return applications;
}

// Solve A~ X = B with the stored factor: X = (LU)^{-1} B, then FP64 refinement. Classic
// corrections X += (LU)^{-1}(B - A~ X) while they at least halve the normwise backward error
// max_l ||r_l|| / (||A~|| ||x_l|| + ||b_l||); when one does not, GMRES-refinement cycles take
// over (the low-precision factor as preconditioner of an FP64 GMRES on the correction
// equation). Stops at tol or after max_iter refinement steps.
int solve_scaled(Factor& f, int nrhs, const zd* B, zd* X, int max_iter, double tol, double* berr, SolveWork& w,
                 hipStream_t s, bool strict, bool allow_krylov) {

    cr_sys sys = f.sys;
    const int64_t n = sys->n;
    if (f.anorm_omega != f.omega) {
        f.anorm = shifted_norm_inf(sys, f.opA, nullptr, 0.0, w.sc, s);
        f.anorm_omega = f.omega;
    }
    const double anorm = f.anorm;
    w.r.reserve((size_t)n * nrhs);
    w.res.reserve((size_t)n * nrhs);
    w.red.reserve(3 * (size_t)nrhs);
    w.hred.resize(3 * (size_t)nrhs);
    unsigned long long* nrm = reinterpret_cast<unsigned long long*>(w.red.p);
    apply_factor(f, nrhs, B, n, X, n, 0, w, s);
    int it = 0;
    double prev = 1e300, be = 1e300;
    bool krylov = false;
    for (;;) {
        spmm_residual(sys, f.opA, nullptr, 0.0, nrhs, X, n, B, n, w.res.p, n, s);
        fill_zero(nrm, 3 * nrhs, s);
        hipLaunchKernelGGL(k_colmax3, dim3(64, nrhs), dim3(256), 0, s, n, nrhs, w.res.p, X, B, n, nrm);
        CR_HIP(hipMemcpyAsync(w.hred.data(), nrm, 3 * nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
        CR_HIP(hipStreamSynchronize(s));
        be = 0;
        for (int l = 0; l < nrhs; ++l) {
            const double rn = w.hred[3 * l], xn = w.hred[3 * l + 1], bn = w.hred[3 * l + 2];
            const double den = anorm * xn + bn;
            be = std::max(be, den > 0 ? rn / den : 0.0);
        }
        if (be <= tol || it >= max_iter) break;
        if (!krylov && !(be < 0.5 * prev)) {
            if (!allow_krylov) break;   // caller decides (e.g. refactor in FP64)
            krylov = true;
        }
        if (krylov && f.prec == CR_FP64 && !(be < 0.5 * prev)) break;   // FP64 factor: nothing left to gain
        prev = be;
        if (!krylov) {
            apply_factor(f, nrhs, w.res.p, n, X, n, 1, w, s);
        } else {
            gmres_cycle(f, nrhs, w.res.p, X, 30, 1e-6, w, s);
        }
        ++it;
    }
    *berr = be;
    if (strict && !(be <= tol))
    {
        char buf[96];
        std::snprintf(buf, sizeof(buf), "iterative refinement stopped at backward error %.3e after %d steps", be, it);
        throw Error(CR_E_NOT_CONVERGED, buf);
    }
    return it;
}

// ------------------------------------------------------------------ Gram / update (CGS2)
namespace {

constexpr int kGramRows = 256;   // rows per workgroup chunk
constexpr int kGramB = 16;       // max columns of the staged operand

// Sum over the 64 lanes of a wave of V doubles per lane (V a power of two <= 64), as a
// reduce-scatter: each exchange step sends half of the values still held to the partner lane and
// keeps the other half, so the wave does V - 1 + (6 - log2 V) shuffles instead of 6 V. On return
// v[0] of lane l is the wave's total of value wave_sum_index<V>(l); every value has 64 / V lanes
// holding it, the one with wave_sum_writer<V>(l) true writes it.
template <int V, int H = V / 2, int D = 32>
__device__ __forceinline__ void wave_sum_scatter(double (&v)[V], int lane) {
    if constexpr (H >= 1) {
        const bool up = lane & D;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const double send = up ? v[i] : v[i + H];
            const double keep = up ? v[i + H] : v[i];
            v[i] = keep + __shfl_xor(send, D);
        }
        wave_sum_scatter<V, H / 2, D / 2>(v, lane);
    } else {
        // distances below the last halving step: plain sums
#pragma unroll
        for (int d = D; d >= 1; d /= 2) v[0] += __shfl_xor(v[0], d);
    }
}
template <int V>
__device__ __forceinline__ int wave_sum_index(int lane) {
    int idx = 0;
    for (int h = V / 2, d = 32; h >= 1; h /= 2, d /= 2)
        if (lane & d) idx += h;
    return idx;
}
template <int V>
__device__ __forceinline__ bool wave_sum_writer(int lane) {
    return (lane & (64 / V - 1)) == 0;
}

// partial[chunk][k][c] = sum_{i in chunk} conj(A[i,k]) B[i,c],  k < qa, c < b (b <= 16)
// B = the staged column count rounded up (1 or 4; wider blocks go to the matrix-core kernel below);
// blockIdx.y strides over the columns of A so that short tall matrices still fill the chip.
// The chunk of B is staged column by column (lane-consecutive rows: no LDS bank conflicts).
template <int B>
__global__ void __launch_bounds__(256) k_gram_partial(int64_t n, int qa, int b, const zd* __restrict__ A, int64_t lda,
                                                      const zd* __restrict__ Bm, int64_t ldb, zd* __restrict__ partial) {
    __shared__ zd sb[B][kGramRows];
    const int64_t i0 = (int64_t)blockIdx.x * kGramRows;
    const int rows = (int)std::min<int64_t>(kGramRows, n - i0);
    for (int e = threadIdx.x; e < kGramRows * B; e += 256) {
        const int r = e % kGramRows, c = e / kGramRows;
        sb[c][r] = (r < rows && c < b) ? Bm[i0 + r + c * ldb] : zd{0, 0};
    }
    __syncthreads();
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    zd* out = partial + (size_t)blockIdx.x * qa * b;
    for (int k = blockIdx.y * 4 + wave; k < qa; k += 4 * gridDim.y) {
        double v[2 * B];
#pragma unroll
        for (int c = 0; c < 2 * B; ++c) v[c] = 0;
        zd a[kGramRows / 64];
#pragma unroll
        for (int j = 0; j < kGramRows / 64; ++j) {
            const int r = lane + 64 * j;
            a[j] = r < rows ? A[i0 + r + k * lda] : zd{0, 0};
        }
#pragma unroll
        for (int j = 0; j < kGramRows / 64; ++j) {
            const int r = lane + 64 * j;
#pragma unroll
            for (int c = 0; c < B; ++c) {
                const zd w = sb[c][r];
                v[2 * c] += a[j].re * w.re + a[j].im * w.im;   // conj(a) * w
                v[2 * c + 1] += a[j].re * w.im - a[j].im * w.re;
            }
        }
        wave_sum_scatter<2 * B>(v, lane);
        const int idx = wave_sum_index<2 * B>(lane), c = idx / 2;
        if (wave_sum_writer<2 * B>(lane) && c < b) {
            double* o = reinterpret_cast<double*>(out + k + (size_t)c * qa);
            o[idx & 1] = v[0];
        }
    }
}

constexpr int kGramRowsM = 512;   // rows per wave of the matrix-core Gram
constexpr int kGramTPW = 4;        // 16-column tiles of A per wave

typedef double f64x4_t __attribute__((ext_vector_type(4)));

// partial[chunk][k][c] as k_gram_partial, for blocks of 5..16 columns, on the matrix cores
// (v_mfma_f64_16x16x4f64): one wave per (chunk of kGramRowsM rows, group of kGramTPW 16-column
// tiles of A), no LDS and no barrier. A step takes 4 rows; lane l supplies the A operand
// A[row][k0 + l % 16] and the B operand B[row][l % 16] of row r0 + l / 16, and conj(A)^T B is
// formed as four real products into separate real and imaginary accumulators, which stay in
// registers over the whole chunk (item r of lane l holds k = k0 + l / 16 + 4 r, c = l % 16).
__global__ void __launch_bounds__(256) k_gram_mfma(int64_t n, int qa, int b, const zd* __restrict__ A, int64_t lda,
                                                   const zd* __restrict__ Bm, int64_t ldb, zd* __restrict__ partial,
                                                   int nchunk, int ntg) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wid >= (int64_t)nchunk * ntg) return;
    const int chunk = (int)(wid % nchunk), tg = (int)(wid / nchunk);
    const int64_t rb = (int64_t)chunk * kGramRowsM, rend = std::min<int64_t>(n, rb + kGramRowsM);
    const int i = lane & 15, kk = lane >> 4, kbase = tg * kGramTPW * 16;
    f64x4_t hre[kGramTPW], him[kGramTPW];
#pragma unroll
    for (int t = 0; t < kGramTPW; ++t) {
        hre[t] = f64x4_t{0, 0, 0, 0};
        him[t] = f64x4_t{0, 0, 0, 0};
    }
    constexpr int U = 4;   // 4-row steps whose loads are issued together
    for (int64_t r0 = rb; r0 < rend; r0 += 4 * U) {
        zd bv[U], av[U][kGramTPW];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = r0 + 4 * u + kk;
            const bool ok = row < rend;
            bv[u] = (ok && i < b) ? Bm[row + (int64_t)i * ldb] : zd{0, 0};
#pragma unroll
            for (int t = 0; t < kGramTPW; ++t) {
                const int col = kbase + 16 * t + i;
                av[u][t] = (ok && col < qa) ? A[row + (int64_t)col * lda] : zd{0, 0};
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int t = 0; t < kGramTPW; ++t) {
                // conj(a) b = (ar br + ai bi) + i (ar bi - ai br)
                hre[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][t].re, bv[u].re, hre[t], 0, 0, 0);
                hre[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][t].im, bv[u].im, hre[t], 0, 0, 0);
                him[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][t].re, bv[u].im, him[t], 0, 0, 0);
                him[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[u][t].im, bv[u].re, him[t], 0, 0, 0);
            }
    }
    zd* out = partial + (size_t)chunk * qa * b;
#pragma unroll
    for (int t = 0; t < kGramTPW; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = kbase + 16 * t + kk + 4 * r;
            if (k < qa && i < b) out[k + (size_t)i * qa] = {hre[t][r], him[t][r]};
        }
}

// H[k + c*ldh] = sum of the nchunk partials of output o = k + c qa (conj_t: conj into
// H[c + k*ldh]), in a fixed order: thread t takes output o0 + t % OB and the chunks
// ch = t / OB (mod 1024 / OB) in increasing order, four running sums; the 1024 / OB sums of an
// output are then added by a fixed tree in LDS.
template <int OB>
__global__ void __launch_bounds__(1024) k_gram_reduce(int nchunk, int qa, int b, const zd* __restrict__ partial,
                                                      zd* __restrict__ H, int64_t ldh, int conj_t) {
    constexpr int NS = 1024 / OB;
    __shared__ zd red[1024];
    const int t = threadIdx.x, lo = t % OB, sg = t / OB;
    const int no = qa * b, o = blockIdx.x * OB + lo;
    zd acc = {0, 0};
    if (o < no) {
        zd s4[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
        int ch = sg;
        for (; ch + 3 * NS < nchunk; ch += 4 * NS) {
            zd v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = partial[(size_t)(ch + u * NS) * no + o];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                s4[u].re += v[u].re;
                s4[u].im += v[u].im;
            }
        }
        for (; ch < nchunk; ch += NS) {
            const zd v = partial[(size_t)ch * no + o];
            s4[0].re += v.re;
            s4[0].im += v.im;
        }
        acc = {(s4[0].re + s4[1].re) + (s4[2].re + s4[3].re), (s4[0].im + s4[1].im) + (s4[2].im + s4[3].im)};
    }
    red[t] = acc;
    __syncthreads();
#pragma unroll
    for (int h = NS / 2; h >= 1; h /= 2) {
        if (sg < h) {
            red[t].re += red[t + h * OB].re;
            red[t].im += red[t + h * OB].im;
        }
        __syncthreads();
    }
    if (sg == 0 && o < no) {
        const int k = o % qa, c = o / qa;
        if (conj_t) H[c + (size_t)k * ldh] = {red[t].re, -red[t].im};
        else H[k + (size_t)c * ldh] = red[t];
    }
}

// W[:, c] -= V[:, 0:q] H[0:q, c] for c < b (b <= 16); H staged through LDS in chunks of 64 rows
__global__ void __launch_bounds__(256) k_update(int64_t n, int q, int b, const zd* __restrict__ V, int64_t ldv,
                                                const zd* __restrict__ H, int64_t ldh, zd* __restrict__ W, int64_t ldw) {
    __shared__ zd sh[64][kGramB];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double ar[kGramB], ai[kGramB];
#pragma unroll
    for (int c = 0; c < kGramB; ++c) ar[c] = ai[c] = 0;
    for (int k0 = 0; k0 < q; k0 += 64) {
        const int kn = min(64, q - k0);
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * kGramB; e += 256) {
            const int r = e % 64, c = e / 64;
            sh[r][c] = (r < kn && c < b) ? H[k0 + r + (size_t)c * ldh] : zd{0, 0};
        }
        __syncthreads();
        if (i < n) {
            for (int r = 0; r < kn; ++r) {
                const zd v = V[i + (int64_t)(k0 + r) * ldv];
#pragma unroll
                for (int c = 0; c < kGramB; ++c) {
                    const zd h = sh[r][c];
                    ar[c] += v.re * h.re - v.im * h.im;
                    ai[c] += v.re * h.im + v.im * h.re;
                }
            }
        }
    }
    if (i < n)
        for (int c = 0; c < b; ++c) {
            zd& w = W[i + (int64_t)c * ldw];
            w.re -= ar[c];
            w.im -= ai[c];
        }
}

__global__ void k_gather_recv(int n_o, int q, const int64_t* __restrict__ recv, const double* __restrict__ scale,
                              const zd* __restrict__ V, int64_t ldv, zd* __restrict__ CR) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_o * q) return;
    const int o = e % n_o, k = e / n_o;
    const int64_t r = recv[o];
    const zd v = V[r + (int64_t)k * ldv];
    CR[o + (size_t)k * n_o] = {scale[r] * v.re, scale[r] * v.im};
}

__global__ void k_scale_cols(int64_t n, int b, zd* __restrict__ W, int64_t ldw, const double* __restrict__ inv) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * b) return;
    const int64_t i = e % n;
    const int c = (int)(e / n);
    W[i + c * ldw].re *= inv[c];
    W[i + c * ldw].im *= inv[c];
}

}  // namespace

// H (qa x b, ld ldh) = A^H B, A n x qa, B n x b; conj_t stores H^H (b x qa) instead.
void gram(int64_t n, int qa, int b, const zd* A, int64_t lda, const zd* B, int64_t ldb, zd* H, int64_t ldh, int conj_t,
          DevBuf<zd>& partial, hipStream_t s) {
    if (qa <= 0 || b <= 0) return;
    for (int c0 = 0; c0 < b; c0 += kGramB) {
        const int bc = std::min(kGramB, b - c0);
        const bool mat = bc > 4;   // wide blocks on the matrix cores
        const int nchunk = (int)((n + (mat ? kGramRowsM : kGramRows) - 1) / (mat ? kGramRowsM : kGramRows));
        partial.reserve((size_t)nchunk * qa * bc);
        // at least ~1024 workgroups when the columns of A allow it
        const unsigned gy = (unsigned)std::max(1, std::min((qa + 3) / 4, (1024 + nchunk - 1) / nchunk));
        const dim3 grid(nchunk, gy);
        if (mat) {
            const int ntg = (qa + 16 * kGramTPW - 1) / (16 * kGramTPW);
            const int64_t waves = (int64_t)nchunk * ntg;
            hipLaunchKernelGGL(k_gram_mfma, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, n, qa, bc, A, lda,
                               B + (int64_t)c0 * ldb, ldb, partial.p, nchunk, ntg);
        } else if (bc == 1)
            hipLaunchKernelGGL(k_gram_partial<1>, grid, dim3(256), 0, s, n, qa, bc, A, lda, B + (int64_t)c0 * ldb, ldb,
                               partial.p);
        else
            hipLaunchKernelGGL(k_gram_partial<4>, grid, dim3(256), 0, s, n, qa, bc, A, lda, B + (int64_t)c0 * ldb, ldb,
                               partial.p);
        zd* Hc = conj_t ? H + c0 : H + (int64_t)c0 * ldh;
        const int no = qa * bc;
        if (no == 1)
            hipLaunchKernelGGL(k_gram_reduce<1>, dim3(1), dim3(1024), 0, s, nchunk, qa, bc, partial.p, Hc, ldh, conj_t);
        else if (no <= 16)
            hipLaunchKernelGGL(k_gram_reduce<16>, dim3(1), dim3(1024), 0, s, nchunk, qa, bc, partial.p, Hc, ldh, conj_t);
        else
            hipLaunchKernelGGL(k_gram_reduce<64>, dim3((no + 63) / 64), dim3(1024), 0, s, nchunk, qa, bc, partial.p, Hc,
                               ldh, conj_t);
    }
}

void update(int64_t n, int q, int b, const zd* V, int64_t ldv, const zd* H, int64_t ldh, zd* W, int64_t ldw, hipStream_t s) {
    if (q <= 0 || b <= 0) return;
    for (int c0 = 0; c0 < b; c0 += kGramB) {
        const int bc = std::min(kGramB, b - c0);
        hipLaunchKernelGGL(k_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, q, bc, V, ldv,
                           H + (int64_t)c0 * ldh, ldh, W + (int64_t)c0 * ldw, ldw);
    }
}

void gather_recv(cr_sys sys, int q, const zd* V, int64_t ldv, zd* CR, hipStream_t s) {
    if (sys->n_o == 0 || q == 0) return;
    hipLaunchKernelGGL(k_gather_recv, dim3((sys->n_o * q + 255) / 256), dim3(256), 0, s, sys->n_o, q, sys->d_recv.p,
                       sys->d_scale.p, V, ldv, CR);
}

void scale_cols(int64_t n, int b, zd* W, int64_t ldw, const double* inv_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_cols, dim3((unsigned)((n * b + 255) / 256)), dim3(256), 0, s, n, b, W, ldw, inv_dev);
}

void copy_dev(int64_t n, const zd* src, zd* dst, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_axpy_copy, dim3(1024), dim3(256), 0, s, n, src, dst);
}

namespace {
__global__ void k_copy_scaled(int64_t n, const zd* __restrict__ src, zd* __restrict__ dst, double f) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = {src[i].re * f, src[i].im * f};
}
__global__ void k_copy_2d(int rows, int cols, const zd* __restrict__ src, int64_t lds, zd* __restrict__ dst, int64_t ldd) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * cols) return;
    const int64_t r = e % rows, c = e / rows;
    dst[r + c * ldd] = src[r + c * lds];
}
__global__ void k_scale_rows(int64_t n, int nrhs, const zd* __restrict__ src, const double* __restrict__ sc,
                             zd* __restrict__ dst) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * nrhs) return;
    const double f = sc[e % n];
    dst[e] = {src[e].re * f, src[e].im * f};
}
}  // namespace

namespace {
// O = a X + c Y over b columns (complex scalars; O may alias X or Y)
__global__ void k_comb(int64_t n, int b, zd a, const zd* X, int64_t ldx, zd c, const zd* Y, int64_t ldy, zd* O,
                       int64_t ldo) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * b) return;
    const int64_t i = e % n, j = e / n;
    const zd x = X[i + j * ldx], y = Y[i + j * ldy];
    O[i + j * ldo] = {a.re * x.re - a.im * x.im + c.re * y.re - c.im * y.im,
                      a.re * x.im + a.im * x.re + c.re * y.im + c.im * y.re};
}

// X[:, c] = diag(scale) V XR[:, c] for c < b (b <= kGramB); XR staged through LDS in chunks of 64 rows
__global__ void __launch_bounds__(256) k_lift(int64_t n, int q, int b, const zd* __restrict__ V, int64_t ldv,
                                              const zd* __restrict__ XR, int64_t ldr, const double* __restrict__ scale,
                                              zd* __restrict__ X, int64_t ldx) {
    __shared__ zd sh[64][kGramB];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double ar[kGramB], ai[kGramB];
#pragma unroll
    for (int c = 0; c < kGramB; ++c) ar[c] = ai[c] = 0;
    for (int k0 = 0; k0 < q; k0 += 64) {
        const int kn = min(64, q - k0);
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * kGramB; e += 256) {
            const int r = e % 64, c = e / 64;
            sh[r][c] = (r < kn && c < b) ? XR[k0 + r + (size_t)c * ldr] : zd{0, 0};
        }
        __syncthreads();
        if (i < n) {
            for (int r = 0; r < kn; ++r) {
                const zd v = V[i + (int64_t)(k0 + r) * ldv];
#pragma unroll
                for (int c = 0; c < kGramB; ++c) {
                    const zd h = sh[r][c];
                    ar[c] += v.re * h.re - v.im * h.im;
                    ai[c] += v.re * h.im + v.im * h.re;
                }
            }
        }
    }
    if (i < n) {
        const double f = scale ? scale[i] : 1.0;
        for (int c = 0; c < b; ++c) X[i + (int64_t)c * ldx] = {f * ar[c], f * ai[c]};
    }
}
}  // namespace

namespace {
// dst[i] = src[idx[i]] for i < m
__global__ void k_gather_idx(int64_t m, const int32_t* __restrict__ idx, const zd* __restrict__ src, zd* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) dst[i] = src[idx[i]];
}
// dst[tgt[i]] (+)= src[pos[i]] for i < m (distinct targets within one call)
__global__ void k_scatter_idx(int64_t m, const int32_t* __restrict__ pos, const int32_t* __restrict__ tgt,
                              const zd* __restrict__ src, zd* __restrict__ dst, int add) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const zd v = src[pos[i]];
    zd& d = dst[tgt[i]];
    if (add) { d.re += v.re; d.im += v.im; }
    else d = v;
}
}  // namespace

void gather_idx(int64_t m, const int32_t* idx, const zd* src, zd* dst, hipStream_t s) {
    if (m > 0) hipLaunchKernelGGL(k_gather_idx, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, m, idx, src, dst);
}
void scatter_idx(int64_t m, const int32_t* pos, const int32_t* tgt, const zd* src, zd* dst, int add, hipStream_t s) {
    if (m > 0)
        hipLaunchKernelGGL(k_scatter_idx, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, m, pos, tgt, src, dst, add);
}

void comb(int64_t n, int b, zd a, const zd* X, int64_t ldx, zd c, const zd* Y, int64_t ldy, zd* O, int64_t ldo,
          hipStream_t s) {
    const int64_t tot = n * b;
    if (tot <= 0) return;
    hipLaunchKernelGGL(k_comb, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, b, a, X, ldx, c, Y, ldy, O, ldo);
}

void lift(int64_t n, int q, int ncol, const zd* V, int64_t ldv, const zd* XR, int64_t ldr, const double* scale, zd* X,
          int64_t ldx, hipStream_t s) {
    for (int c0 = 0; c0 < ncol; c0 += kGramB) {
        const int bc = std::min(kGramB, ncol - c0);
        hipLaunchKernelGGL(k_lift, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, q, bc, V, ldv,
                           XR + (int64_t)c0 * ldr, ldr, scale, X + (int64_t)c0 * ldx, ldx);
    }
}

void copy_cols_scaled(int64_t n, const zd* src, zd* dst, double factor, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_scaled, dim3((unsigned)std::min<int64_t>(1024, (n + 255) / 256)), dim3(256), 0, s, n, src,
                       dst, factor);
}
void copy_2d(int rows, int cols, const zd* src, int64_t lds, zd* dst, int64_t ldd, hipStream_t s) {
    const int64_t tot = (int64_t)rows * cols;
    if (tot <= 0) return;
    hipLaunchKernelGGL(k_copy_2d, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, rows, cols, src, lds, dst, ldd);
}
void scale_rows(int64_t n, int nrhs, const zd* src, const double* sc, zd* dst, hipStream_t s) {
    const int64_t tot = n * nrhs;
    if (tot <= 0) return;
    hipLaunchKernelGGL(k_scale_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, nrhs, src, sc, dst);
}

// ------------------------------------------------------------------ candidate residuals
namespace {

constexpr int kCandChunk = 8;

// partial[chunk][c] = sum_i sum_l | s_cl F[i,l] - sum_k (KV[i,k] - w_c^2 MV[i,k]) X[k, l, c] |^2
// X: q x L x ncand (ld q, then L); scal[c*L + l] = (i w_c)^flag
__global__ void __launch_bounds__(256) k_resid_partial(int64_t n, int q, int L, int ncand, const zd* __restrict__ KV,
                                                       const zd* __restrict__ MV, int64_t ldv, const zd* __restrict__ F,
                                                       const zd* __restrict__ X, const zd* __restrict__ scal,
                                                       const double* __restrict__ w2, double* __restrict__ partial) {
    extern __shared__ zd sx[];   // q x L x kCandChunk
    const int c0 = blockIdx.y * kCandChunk;
    const int nc = min(kCandChunk, ncand - c0);
    for (int e = threadIdx.x; e < q * L * nc; e += 256) sx[e] = X[(size_t)c0 * q * L + e];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double acc2[kCandChunk];
#pragma unroll
    for (int c = 0; c < kCandChunk; ++c) acc2[c] = 0;
    if (i < n) {
        for (int l = 0; l < L; ++l) {
            double rr[kCandChunk], ri[kCandChunk];
            const zd f = F[i + (int64_t)l * n];
#pragma unroll
            for (int c = 0; c < kCandChunk; ++c) {
                if (c < nc) {
                    const zd sc = scal[(c0 + c) * L + l];
                    rr[c] = f.re * sc.re - f.im * sc.im;
                    ri[c] = f.re * sc.im + f.im * sc.re;
                } else rr[c] = ri[c] = 0;
            }
            for (int k = 0; k < q; ++k) {
                const zd kv = KV[i + (int64_t)k * ldv], mv = MV[i + (int64_t)k * ldv];
#pragma unroll
                for (int c = 0; c < kCandChunk; ++c) {
                    if (c >= nc) break;
                    const double a_r = kv.re - w2[c0 + c] * mv.re, a_i = kv.im - w2[c0 + c] * mv.im;
                    const zd x = sx[(size_t)c * q * L + (size_t)l * q + k];
                    rr[c] -= a_r * x.re - a_i * x.im;
                    ri[c] -= a_r * x.im + a_i * x.re;
                }
            }
#pragma unroll
            for (int c = 0; c < kCandChunk; ++c) acc2[c] += rr[c] * rr[c] + ri[c] * ri[c];
        }
    }
    __shared__ double red[4][kCandChunk];
#pragma unroll
    for (int c = 0; c < kCandChunk; ++c) {
        double v = acc2[c];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64][c] = v;
    }
    __syncthreads();
    if (threadIdx.x < nc) {
        const int c = threadIdx.x;
        partial[(size_t)blockIdx.x * ncand + c0 + c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
    }
}

// Large q x L on the matrix cores: a workgroup takes 64 rows (16 per wave) and kRG candidates;
// for each candidate c the wave forms its A operand (K~V - w_c^2 M~V)[rows, k..k+4) from one read
// of K~V and M~V (shared by the kRG candidates) and multiplies it with X_c[k..k+4, 16 loads],
// v_mfma_f64_16x16x4f64, each complex product as three real ones (Ar Br, Ai Bi,
// (Ar + Ai)(Br + Bi)); the epilogue subtracts the product from s_c F and sums |.|^2. X, its
// re + im sums and the wave's K~V, M~V rows pass through LDS kRK columns at a time (held in
// registers they would be indexed by the loop counter and spill to scratch).
constexpr int kRG = 8;   // candidates per workgroup
constexpr int kRK = 8;   // columns of the basis per chunk
typedef double rf64x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_resid_mfma(int64_t n, int q, int L, int ncand, const zd* __restrict__ KV,
                                                    const zd* __restrict__ MV, int64_t ldv, const zd* __restrict__ F,
                                                    const zd* __restrict__ X, const zd* __restrict__ scal,
                                                    const double* __restrict__ w2, double* __restrict__ partial) {
    __shared__ zd sx[kRG][kRK][16];
    __shared__ double sxs[kRG][kRK][16];   // re + im of sx (three real products per complex one)
    __shared__ zd sa[4][2][kRK][16];       // per wave: K~V and M~V [column][row]
    __shared__ double red[4][kRG];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int li = lane & 15, lk = lane >> 4;
    // flat grid, candidate group fastest: the groups of one row chunk are dispatched together
    const int ngroup = (ncand + kRG - 1) / kRG;
    const int64_t chunk = blockIdx.x / ngroup;
    const int c0 = (int)(blockIdx.x % ngroup) * kRG, nc = min(kRG, ncand - c0);
    const int64_t rbase = chunk * 64 + 16 * wave;
    const int64_t arow = rbase + li;   // the row this lane supplies to the A operand
    const bool aok = arow < n;
    double w2c[kRG], acc2[kRG];
#pragma unroll
    for (int c = 0; c < kRG; ++c) {
        w2c[c] = c < nc ? w2[c0 + c] : 0.0;
        acc2[c] = 0.0;
    }
    for (int l0 = 0; l0 < L; l0 += 16) {
        const int nl = min(16, L - l0);
        // p1 = sum ar br, p2 = sum ai bi, p3 = sum (ar + ai)(br + bi): Re = p1 - p2, Im = p3 - p1 - p2
        rf64x4 p1[kRG], p2[kRG], p3[kRG];
#pragma unroll
        for (int c = 0; c < kRG; ++c) {
            p1[c] = rf64x4{0, 0, 0, 0};
            p2[c] = rf64x4{0, 0, 0, 0};
            p3[c] = rf64x4{0, 0, 0, 0};
        }
        // software pipeline: the next chunk's X entries and A-operand rows are loaded into
        // registers while the current chunk is multiplied
        constexpr int XPER = kRG * kRK * 16 / 256;
        zd xr[XPER], kvn[kRK / 4], mvn[kRK / 4];
        auto fetch = [&](int k0) {
#pragma unroll
            for (int u = 0; u < XPER; ++u) {
                const int e = t + 256 * u;
                const int l = e % 16, k = (e / 16) % kRK, c = e / (16 * kRK);
                xr[u] = (c < nc && k0 + k < q && l < nl) ? X[((size_t)(c0 + c) * L + l0 + l) * q + k0 + k]
                                                         : zd{0.0, 0.0};
            }
#pragma unroll
            for (int s = 0; s < kRK / 4; ++s) {
                const int k = k0 + 4 * s + lk;
                const bool ok = aok && k < q;
                kvn[s] = ok ? KV[arow + (int64_t)k * ldv] : zd{0.0, 0.0};
                mvn[s] = ok ? MV[arow + (int64_t)k * ldv] : zd{0.0, 0.0};
            }
        };
        fetch(0);
        for (int k0 = 0; k0 < q; k0 += kRK) {
            __syncthreads();
#pragma unroll
            for (int u = 0; u < XPER; ++u) {
                const int e = t + 256 * u;
                sx[e / (16 * kRK)][(e / 16) % kRK][e % 16] = xr[u];
                sxs[e / (16 * kRK)][(e / 16) % kRK][e % 16] = xr[u].re + xr[u].im;
            }
#pragma unroll
            for (int s = 0; s < kRK / 4; ++s) {
                sa[wave][0][4 * s + lk][li] = kvn[s];
                sa[wave][1][4 * s + lk][li] = mvn[s];
            }
            __syncthreads();
            if (k0 + kRK < q) fetch(k0 + kRK);
#pragma unroll 1
            for (int s = 0; s < kRK / 4; ++s) {
                const zd kv = sa[wave][0][4 * s + lk][li], mv = sa[wave][1][4 * s + lk][li];
                const double kvs = kv.re + kv.im, mvs = mv.re + mv.im;
#pragma unroll
                for (int c = 0; c < kRG; ++c) {
                    const zd b = sx[c][4 * s + lk][li];
                    const double bsum = sxs[c][4 * s + lk][li];
                    const double ar = kv.re - w2c[c] * mv.re, ai = kv.im - w2c[c] * mv.im;
                    const double asum = kvs - w2c[c] * mvs;
                    p1[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, b.re, p1[c], 0, 0, 0);
                    p2[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, b.im, p2[c], 0, 0, 0);
                    p3[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(asum, bsum, p3[c], 0, 0, 0);
                }
            }
        }
        // accumulator item r of lane l: row lk + 4 r of the wave's 16, load column li
        zd fv[4];
        bool rok[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = rbase + lk + 4 * r;
            rok[r] = row < n && li < nl;
            fv[r] = rok[r] ? F[row + (int64_t)(l0 + li) * n] : zd{0.0, 0.0};
        }
#pragma unroll
        for (int c = 0; c < kRG; ++c) {
            const zd sc = (c < nc && li < nl) ? scal[(c0 + c) * L + l0 + li] : zd{0.0, 0.0};
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double s1 = p1[c][r], s2 = p2[c][r];
                const double rr = fv[r].re * sc.re - fv[r].im * sc.im - (s1 - s2);
                const double ri = fv[r].re * sc.im + fv[r].im * sc.re - (p3[c][r] - s1 - s2);
                if (rok[r] && c < nc) acc2[c] += rr * rr + ri * ri;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < kRG; ++c) {
        double v = acc2[c];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[wave][c] = v;
    }
    __syncthreads();
    if (t < nc) partial[(size_t)chunk * ncand + c0 + t] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
}

__global__ void k_resid_reduce(int nchunk, int ncand, const double* __restrict__ partial, double* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncand) return;
    double s = 0;
    for (int k = 0; k < nchunk; ++k) s += partial[(size_t)k * ncand + c];
    out[c] = s;
}

}  // namespace

// res2[c] = || scal_c .* F - (KV - w_c^2 MV) X_c ||_F^2 for every candidate
void candidate_residuals(int64_t n, int q, int L, int ncand, const zd* KV, const zd* MV, int64_t ldv, const zd* F,
                         const zd* X, const zd* scal, const double* w2, double* res2, DevBuf<double>& partial,
                         hipStream_t s) {
    const size_t shmem = (size_t)q * L * kCandChunk * sizeof(zd);
    int nchunk;
    if (shmem <= 64 * 1024) {
        nchunk = (int)((n + 255) / 256);
        partial.reserve((size_t)nchunk * ncand);
        hipLaunchKernelGGL(k_resid_partial, dim3(nchunk, (ncand + kCandChunk - 1) / kCandChunk), dim3(256), shmem, s, n,
                           q, L, ncand, KV, MV, ldv, F, X, scal, w2, partial.p);
    } else {
        const int64_t nch = (n + 63) / 64, ngroup = (ncand + kRG - 1) / kRG;
        CR_REQUIRE(nch * ngroup * 256 < ((int64_t)1 << 32), CR_E_UNSUPPORTED,
                   "candidate residuals: rows x candidates beyond one launch");
        nchunk = (int)nch;
        partial.reserve((size_t)nchunk * ncand);
        hipLaunchKernelGGL(k_resid_mfma, dim3((unsigned)(nch * ngroup)), dim3(256), 0, s, n, q, L, ncand, KV, MV, ldv, F,
                           X, scal, w2, partial.p);
    }
    hipLaunchKernelGGL(k_resid_reduce, dim3((ncand + 255) / 256), dim3(256), 0, s, nchunk, ncand, partial.p, res2);
}

}  // namespace cr
