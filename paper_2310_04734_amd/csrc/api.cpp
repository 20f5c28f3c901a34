// C ABI of the library: contexts, systems, analysis, factorisation and solves, the rational
// Krylov basis (fixed and greedy expansion points), the Galerkin projection, and reduced
// models. Kernels live in factor.hip, linalg.hip and sweep.hip.
#include <algorithm>
#include <cfloat>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

#include "internal.h"
#include "sweep.h"
#include "util.cuh"

namespace cr {
void gram(int64_t n, int qa, int b, const zd* A, int64_t lda, const zd* B, int64_t ldb, zd* H, int64_t ldh, int conj_t,
          DevBuf<zd>& partial, hipStream_t s);
void update(int64_t n, int q, int b, const zd* V, int64_t ldv, const zd* H, int64_t ldh, zd* W, int64_t ldw, hipStream_t s);
void gather_recv(cr_sys sys, int q, const zd* V, int64_t ldv, zd* CR, hipStream_t s);
void copy_dev(int64_t n, const zd* src, zd* dst, hipStream_t s);
void candidate_residuals(int64_t n, int q, int L, int ncand, const zd* KV, const zd* MV, int64_t ldv, const zd* F,
                         const zd* X, const zd* scal, const double* w2, double* res2, DevBuf<double>& partial,
                         hipStream_t s);
void copy_cols_scaled(int64_t n, const zd* src, zd* dst, double factor, hipStream_t s);
void copy_2d(int rows, int cols, const zd* src, int64_t lds, zd* dst, int64_t ldd, hipStream_t s);
void comb(int64_t n, int b, zd a, const zd* X, int64_t ldx, zd c, const zd* Y, int64_t ldy, zd* O, int64_t ldo,
          hipStream_t s);
void scale_rows(int64_t n, int nrhs, const zd* src, const double* sc, zd* dst, hipStream_t s);
}  // namespace cr

namespace cr {
thread_local const cr_allocator* tl_alloc = nullptr;
void lift(int64_t n, int q, int ncol, const zd* V, int64_t ldv, const zd* XR, int64_t ldr, const double* scale, zd* X,
          int64_t ldx, hipStream_t s);
}  // namespace cr

using namespace cr;

struct cr_fact_s {
    Factor f;
    SolveWork w;
};

struct cr_rom_s {
    cr_ctx ctx = nullptr;
    int q = 0, L = 0, n_o = 0;
    bool has_d = false;
    DevBuf<zd> KR, MR, DR, FR, CR;
    DevBuf<int32_t> flags;
    // frequency-dependent parts: A_R(w) gains sum_t c_t(w) TR[t] (kind 0: c = 1 + i eta(w);
    // kind 1: c = -w^2 / (c^2 (1 + i eta(w))))
    std::vector<TermMeta> tmeta;
    std::vector<DevBuf<zd>> TR;
    DevBuf<zd> tcoef;   // per-call coefficient table (nfreq x nterm)
    // Hessenberg-triangular form of (K_R, M_R) for FP64 sweeps (built on first use)
    bool ht_ready = false;
    DevBuf<zd> htH, htT, htF, htC;
    DevBuf<double> htN;
};

struct cr_basis_s {
    cr_sys sys = nullptr;
    int q = 0, cap = 0;
    DevBuf<zd> V, KV, MV, DV;    // n x cap (DV only for a system with a damping matrix)
    DevBuf<zd> KR, MR, DR;       // cap x cap (incremental Galerkin projection)
    std::vector<DevBuf<zd>> TV, TR;   // per frequency-dependent term: T V (n x cap), V^H T V (cap x cap)
    std::vector<double> shifts;
    int deflated = 0;
    int ir_iterations = 0;
    double max_berr = 0;
    int n_perturbed = 0;
    int fp64_refactorizations = 0;
    // scratch
    DevBuf<zd> W, H, Hn, partial, RHS;
    std::vector<zd> hH;
};

namespace {

std::string g_create_error;

SweepEngine& engine(cr_ctx ctx) {
    if (!ctx->sweep) {
        ctx->sweep = new SweepEngine();
        ctx->sweep->num_cu = ctx->num_cu;
        ctx->sweep->ctx = ctx;
    }
    return *ctx->sweep;
}

double now() { return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count(); }

// ---------------------------------------------------------------- basis growth
void ensure_capacity(cr_basis B, int need) {
    if (need <= B->cap) return;
    cr_sys sys = B->sys;
    hipStream_t s = sys->ctx->stream;
    const int64_t n = sys->n;
    const bool hd = !sys->D.empty();
    int cap = std::max(need, std::max(16, 2 * B->cap));
    DevBuf<zd> V((size_t)n * cap), KV((size_t)n * cap), MV((size_t)n * cap), KR((size_t)cap * cap), MR((size_t)cap * cap);
    DevBuf<zd> DV(hd ? (size_t)n * cap : 0), DR(hd ? (size_t)cap * cap : 0);
    const size_t nt = sys->terms.size();
    std::vector<DevBuf<zd>> TV(nt), TR(nt);
    for (size_t t = 0; t < nt; ++t) {
        TV[t].alloc((size_t)n * cap);
        TR[t].alloc((size_t)cap * cap);
        if (B->q > 0) {
            copy_dev(n * B->q, B->TV[t].p, TV[t].p, s);
            copy_2d(B->q, B->q, B->TR[t].p, B->cap, TR[t].p, cap, s);
        }
    }
    if (B->q > 0) {
        copy_dev(n * B->q, B->V.p, V.p, s);
        copy_dev(n * B->q, B->KV.p, KV.p, s);
        copy_dev(n * B->q, B->MV.p, MV.p, s);
        copy_2d(B->q, B->q, B->KR.p, B->cap, KR.p, cap, s);
        copy_2d(B->q, B->q, B->MR.p, B->cap, MR.p, cap, s);
        if (hd) {
            copy_dev(n * B->q, B->DV.p, DV.p, s);
            copy_2d(B->q, B->q, B->DR.p, B->cap, DR.p, cap, s);
        }
    }
    CR_HIP(hipStreamSynchronize(s));
    B->V = std::move(V);
    B->KV = std::move(KV);
    B->MV = std::move(MV);
    B->KR = std::move(KR);
    B->MR = std::move(MR);
    B->DV = std::move(DV);
    B->DR = std::move(DR);
    B->TV = std::move(TV);
    B->TR = std::move(TR);
    B->cap = cap;
}

// squared column norms of W (n x b) via the Gram diagonal
std::vector<double> col_norms2(cr_basis B, const zd* W, int b) {
    cr_sys sys = B->sys;
    hipStream_t s = sys->ctx->stream;
    B->H.reserve((size_t)b * b);
    gram(sys->n, b, b, W, sys->n, W, sys->n, B->H.p, b, 0, B->partial, s);
    B->hH.resize((size_t)b * b);
    CR_HIP(hipMemcpyAsync(B->hH.data(), B->H.p, (size_t)b * b * sizeof(zd), hipMemcpyDeviceToHost, s));
    CR_HIP(hipStreamSynchronize(s));
    std::vector<double> out(b);
    for (int c = 0; c < b; ++c) out[c] = B->hH[(size_t)c * b + c].re;
    return out;
}

// incremental Galerkin projection of the new columns [q0, q1)
void project_new(cr_basis B, int q0, int q1) {
    cr_sys sys = B->sys;
    hipStream_t s = sys->ctx->stream;
    const int64_t n = sys->n;
    const int nb = q1 - q0;
    if (nb <= 0) return;
    spmm_km(sys, nb, B->V.p + n * q0, n, B->KV.p + n * q0, B->MV.p + n * q0, n, s);
    const bool hd = !sys->D.empty();
    if (hd) spmm_shifted(sys, sys->d_D.p, sys->d_D.p, 0.0, nb, B->V.p + n * q0, n, B->DV.p + n * q0, n, s);
    const int64_t ld = B->cap;
    // columns: R[0:q1, q0:q1] = V[:, 0:q1]^H (KV)[:, q0:q1]
    gram(n, q1, nb, B->V.p, n, B->KV.p + n * q0, n, B->KR.p + ld * q0, ld, 0, B->partial, s);
    gram(n, q1, nb, B->V.p, n, B->MV.p + n * q0, n, B->MR.p + ld * q0, ld, 0, B->partial, s);
    if (hd) gram(n, q1, nb, B->V.p, n, B->DV.p + n * q0, n, B->DR.p + ld * q0, ld, 0, B->partial, s);
    for (size_t t = 0; t < sys->terms.size(); ++t) {
        const zd* T = sys->terms[t].d_vals.p;
        spmm_shifted(sys, T, T, 0.0, nb, B->V.p + n * q0, n, B->TV[t].p + n * q0, n, s);
        gram(n, q1, nb, B->V.p, n, B->TV[t].p + n * q0, n, B->TR[t].p + ld * q0, ld, 0, B->partial, s);
        if (q0 > 0) gram(n, q0, nb, B->TV[t].p, n, B->V.p + n * q0, n, B->TR[t].p + q0, ld, 1, B->partial, s);
    }
    // rows: R[q0:q1, 0:q0] = conj((KV)[:, 0:q0]^H V[:, q0:q1])^T
    if (q0 > 0) {
        gram(n, q0, nb, B->KV.p, n, B->V.p + n * q0, n, B->KR.p + q0, ld, 1, B->partial, s);
        gram(n, q0, nb, B->MV.p, n, B->V.p + n * q0, n, B->MR.p + q0, ld, 1, B->partial, s);
        if (hd) gram(n, q0, nb, B->DV.p, n, B->V.p + n * q0, n, B->DR.p + q0, ld, 1, B->partial, s);
    }
}

// Orthonormalise the b columns of W against V and each other (block CGS2 in FP64, then two
// passes per column inside the block) and append the accepted ones. Returns accepted count.
int orthonormalise_append(cr_basis B, zd* W, int b) {
    cr_sys sys = B->sys;
    hipStream_t s = sys->ctx->stream;
    const int64_t n = sys->n;
    // norms before orthogonalisation (diagonal of W^H W) stay on the device until the first
    // column's norm after it is read, so that each column costs one host round trip
    B->Hn.reserve((size_t)b * b + 1);
    gram(n, b, b, W, n, W, n, B->Hn.p, b, 0, B->partial, s);
    std::vector<double> before(b, 0.0);
    const int q0 = B->q;
    if (q0 > 0) {
        B->H.reserve((size_t)q0 * b);
        for (int pass = 0; pass < 2; ++pass) {
            gram(n, q0, b, B->V.p, n, W, n, B->H.p, q0, 0, B->partial, s);
            update(n, q0, b, B->V.p, n, B->H.p, q0, W, n, s);
        }
    }
    ensure_capacity(B, q0 + b);
    int q = q0;
    for (int c = 0; c < b; ++c) {
        zd* w = W + n * c;
        const int na = q - q0;   // columns accepted from this block so far
        if (na > 0) {
            B->H.reserve((size_t)na);
            for (int pass = 0; pass < 2; ++pass) {
                gram(n, na, 1, B->V.p + n * q0, n, w, n, B->H.p, na, 0, B->partial, s);
                update(n, na, 1, B->V.p + n * q0, n, B->H.p, na, w, n, s);
            }
        }
        gram(n, 1, 1, w, n, w, n, B->Hn.p + (size_t)b * b, 1, 0, B->partial, s);
        const size_t nread = c == 0 ? (size_t)b * b + 1 : 1;
        B->hH.resize((size_t)b * b + 1);
        CR_HIP(hipMemcpyAsync(B->hH.data() + (b * b + 1 - nread), B->Hn.p + (b * b + 1 - nread), nread * sizeof(zd),
                              hipMemcpyDeviceToHost, s));
        CR_HIP(hipStreamSynchronize(s));
        if (c == 0)
            for (int k = 0; k < b; ++k) before[k] = B->hH[(size_t)k * b + k].re;
        const double after2 = B->hH[(size_t)b * b].re;
        const double ratio = std::sqrt(after2 / std::max(before[c], 1e-300));
        if (!(before[c] > 0) || !(ratio >= 1e-10)) {
            B->deflated++;
            continue;
        }
        copy_cols_scaled(n, w, B->V.p + n * q, 1.0 / std::sqrt(after2), s);
        ++q;
    }
    B->q = q;
    project_new(B, q0, q);
    return q - q0;
}

// Y = M(w_j) X with the mass matrix of the factor's frequency
void mass_apply(const Factor& fac, cr_sys sys, int b, const zd* X, int64_t ldx, zd* Y, int64_t ldy, hipStream_t s) {
    if (fac.opMass == sys->d_M.p) spmm_m(sys, b, X, ldx, Y, ldy, s);
    else spmm_shifted(sys, fac.opMass, fac.opMass, 0.0, b, X, ldx, Y, ldy, s);
}

// X = A_j^{-1} B for b columns with FP64 refinement until the normwise backward error is at most
// max(1e-14, sqrt(n) eps), the stopping rule of LAPACK's mixed-precision solver (dsgesv:
// ||r|| <= sqrt(n) eps ||A|| ||x||): below it a correction is under the rounding level of a
// backward-stable solve at this size. A complex-FP32 factor whose classic refinement stalls
// (kappa(A_j) u_32 >~ 1) is refactored in complex FP64 once, which is cheaper than a Krylov
// refinement of every one of its solves.
void shifted_solve(cr_basis B, Factor& fac, SolveWork& sw, double omega, int b, const zd* rhs, zd* X) {
    cr_sys sys = B->sys;
    hipStream_t s = sys->ctx->stream;
    const double tol = std::max(1e-14, std::sqrt((double)sys->n) * DBL_EPSILON);
    double berr = 0;
    int its = solve_scaled(fac, b, rhs, X, 10, tol, &berr, sw, s, false, fac.prec == CR_FP64);
    if (!(berr <= tol) && fac.prec == CR_MIXED) {
        numeric_factor(fac, sys, omega, CR_FP64, s);
        B->n_perturbed += fac.n_perturbed;
        B->fp64_refactorizations++;
        its += solve_scaled(fac, b, rhs, X, 10, tol, &berr, sw, s, false);
    }
    B->ir_iterations += its;
    B->max_berr = std::max(B->max_berr, berr);
}

// Orthonormalise the b columns of W (length m, leading dimension m) against Z[:, 0:nz] (block CGS2)
// and each other (two passes per column), appending the accepted columns to Z; the deflation
// rule of the basis. Returns the number appended.
int orth_append_local(int64_t m, zd* Z, int& nz, zd* W, int b, cr_basis B, hipStream_t s) {
    DevBuf<zd> H((size_t)std::max(nz + b, 1) * b), nrm(2);
    std::vector<zd> h(1);
    auto norm2 = [&](const zd* w) {
        gram(m, 1, 1, w, m, w, m, nrm.p, 1, 0, B->partial, s);
        CR_HIP(hipMemcpyAsync(h.data(), nrm.p, sizeof(zd), hipMemcpyDeviceToHost, s));
        CR_HIP(hipStreamSynchronize(s));
        return h[0].re;
    };
    const int z0 = nz;
    for (int c = 0; c < b; ++c) {
        zd* w = W + m * c;
        const double before = norm2(w);
        for (int pass = 0; pass < 2; ++pass)
            if (nz > 0) {
                gram(m, nz, 1, Z, m, w, m, H.p, nz, 0, B->partial, s);
                update(m, nz, 1, Z, m, H.p, nz, w, m, s);
            }
        const double after = norm2(w);
        if (!(before > 0) || !(std::sqrt(after / before) >= 1e-10)) continue;
        copy_cols_scaled(m, w, Z + m * nz, 1.0 / std::sqrt(after), s);
        ++nz;
    }
    return nz - z0;
}

// Krylov blocks at one expansion point: X = A^{-1} F~, then X = A^{-1} M~ Q (Eq. (10))
void add_shift(cr_basis B, Factor& fac, SolveWork& sw, double omega, int blocks, cr_precision prec) {
    cr_sys sys = B->sys;
    hipStream_t s = sys->ctx->stream;
    const int64_t n = sys->n;
    numeric_factor(fac, sys, omega, prec, s);
    B->n_perturbed += fac.n_perturbed;
    B->shifts.push_back(omega);
    const int L = sys->L;
    B->RHS.reserve((size_t)n * std::max(L, 1));
    B->W.reserve((size_t)n * std::max(L, 1));
    int b = L;
    copy_dev(n * L, sys->d_F.p, B->RHS.p, s);
    if (!sys->terms.empty()) {
        // frequency-dependent matrices: the pencils of different expansion points differ, so the
        // recurrence continues from this point's own vectors (orthonormalised among themselves)
        // and each block is then appended to the basis
        DevBuf<zd> Z((size_t)n * std::max(blocks * L, 1));
        int nz = 0;
        for (int blk = 0; blk < blocks && b > 0; ++blk) {
            if (blk > 0) mass_apply(fac, sys, b, Z.p + n * (nz - b), n, B->RHS.p, n, s);
            shifted_solve(B, fac, sw, omega, b, B->RHS.p, B->W.p);
            const int z0 = nz;
            b = orth_append_local(n, Z.p, nz, B->W.p, b, B, s);
            if (b == 0) break;
            copy_dev(n * b, Z.p + n * z0, B->W.p, s);
            orthonormalise_append(B, B->W.p, b);
        }
        return;
    }
    for (int blk = 0; blk < blocks && b > 0; ++blk) {
        if (blk > 0) mass_apply(fac, sys, b, B->V.p + n * (B->q - b), n, B->RHS.p, n, s);
        shifted_solve(B, fac, sw, omega, b, B->RHS.p, B->W.p);
        b = orthonormalise_append(B, B->W.p, b);
    }
}

// Second-order Krylov blocks at one expansion point for a system with a damping matrix
// (Section 3.3, Eq. (9)): with A_j = K~ + i w_j D~ - w_j^2 M~, D_j = 2 i w_j M~ + D~ and M_j = M~, the
// space of r_0 = A_j^{-1} F~, r_1 = -A_j^{-1} D_j r_0, r_i = -A_j^{-1} (D_j r_(i-1) + M_j r_(i-2)),
// built as an Arnoldi process on the linearisation [u; v] -> [-A_j^{-1} (M~ (2 i w_j u + v) + D~ u); u]
// started from [r_0; 0] (the upper halves of its Krylov vectors are the r_i). The upper halves
// of each orthonormalised block are appended to the basis with CGS2.
void add_shift_soar(cr_basis B, Factor& fac, SolveWork& sw, double omega, int blocks, cr_precision prec) {
    cr_sys sys = B->sys;
    hipStream_t s = sys->ctx->stream;
    const int64_t n = sys->n, m = 2 * n;
    numeric_factor(fac, sys, omega, prec, s);
    B->n_perturbed += fac.n_perturbed;
    B->shifts.push_back(omega);
    const int L = sys->L;
    B->RHS.reserve((size_t)n * std::max(L, 1));
    B->W.reserve((size_t)n * std::max(L, 1));
    DevBuf<zd> Z((size_t)m * std::max(blocks * L, 1)), W((size_t)m * L), T((size_t)n * L), Y((size_t)n * L);
    int nz = 0, last0 = 0, b = L;
    for (int blk = 0; blk < blocks && b > 0; ++blk) {
        if (blk == 0) {
            shifted_solve(B, fac, sw, omega, b, sys->d_F.p, B->W.p);
            fill_zero(W.p, m * b, s);
        } else {
            const zd* U = Z.p + m * last0;       // upper halves of the latest block (leading dimension m)
            const zd* Vv = U + n;                // lower halves
            comb(n, b, zd{0.0, 2.0 * omega}, U, m, zd{1.0, 0.0}, Vv, m, T.p, n, s);      // t = 2 i w u + v
            mass_apply(fac, sys, b, T.p, n, Y.p, n, s);                                  // M~ t
            spmm_shifted(sys, sys->d_D.p, sys->d_D.p, 0.0, b, U, m, B->RHS.p, n, s);     // D~ u
            comb(n, b, zd{-1.0, 0.0}, Y.p, n, zd{-1.0, 0.0}, B->RHS.p, n, B->RHS.p, n, s);
            shifted_solve(B, fac, sw, omega, b, B->RHS.p, B->W.p);
            copy_2d((int)n, b, U, m, W.p + n, m, s);                                     // lower half = u
        }
        copy_2d((int)n, b, B->W.p, n, W.p, m, s);                                        // upper half
        last0 = nz;
        b = orth_append_local(m, Z.p, nz, W.p, b, B, s);
        if (b == 0) break;
        copy_2d((int)n, b, Z.p + m * last0, m, B->W.p, n, s);
        orthonormalise_append(B, B->W.p, b);
    }
}

// independent copy of a basis and its incremental projection (for look-ahead trials)
std::unique_ptr<cr_basis_s> clone_basis(cr_basis B) {
    cr_sys sys = B->sys;
    hipStream_t s = sys->ctx->stream;
    const int64_t n = sys->n;
    auto C = std::make_unique<cr_basis_s>();
    C->sys = sys;
    ensure_capacity(C.get(), B->cap);
    copy_dev(n * B->q, B->V.p, C->V.p, s);
    copy_dev(n * B->q, B->KV.p, C->KV.p, s);
    copy_dev(n * B->q, B->MV.p, C->MV.p, s);
    copy_2d(B->q, B->q, B->KR.p, B->cap, C->KR.p, C->cap, s);
    copy_2d(B->q, B->q, B->MR.p, B->cap, C->MR.p, C->cap, s);
    if (!sys->D.empty()) {
        copy_dev(n * B->q, B->DV.p, C->DV.p, s);
        copy_2d(B->q, B->q, B->DR.p, B->cap, C->DR.p, C->cap, s);
    }
    CR_HIP(hipStreamSynchronize(s));
    C->q = B->q;
    C->shifts = B->shifts;
    return C;
}

void fill_info(cr_basis B, cr_basis_info* info, double t0) {
    if (!info) return;
    info->q = B->q;
    info->deflated = B->deflated;
    info->n_shifts = (int)B->shifts.size();
    info->ir_iterations = B->ir_iterations;
    info->max_backward_error = B->max_berr;
    info->n_perturbed = B->n_perturbed;
    info->fp64_refactorizations = B->fp64_refactorizations;
    info->seconds = now() - t0;
}

// reduced model from the basis' incremental projection (packed to ld = q)
std::unique_ptr<cr_rom_s> rom_from_basis(cr_basis B) {
    cr_sys sys = B->sys;
    hipStream_t s = sys->ctx->stream;
    const int64_t n = sys->n;
    const int q = B->q, L = sys->L;
    auto r = std::make_unique<cr_rom_s>();
    r->ctx = sys->ctx;
    r->q = q;
    r->L = L;
    r->n_o = sys->n_o;
    r->KR.alloc((size_t)q * q);
    r->MR.alloc((size_t)q * q);
    r->FR.alloc((size_t)q * std::max(L, 1));
    r->CR.alloc((size_t)std::max(sys->n_o, 1) * q);
    r->flags.alloc(std::max(L, 1));
    copy_2d(q, q, B->KR.p, B->cap, r->KR.p, q, s);
    copy_2d(q, q, B->MR.p, B->cap, r->MR.p, q, s);
    if (!sys->D.empty()) {
        r->has_d = true;
        r->DR.alloc((size_t)q * q);
        copy_2d(q, q, B->DR.p, B->cap, r->DR.p, q, s);
    }
    for (size_t t = 0; t < sys->terms.size(); ++t) {
        r->tmeta.push_back(static_cast<const TermMeta&>(sys->terms[t]));
        r->TR.emplace_back((size_t)q * q);
        copy_2d(q, q, B->TR[t].p, B->cap, r->TR.back().p, q, s);
    }
    gram(n, q, L, B->V.p, n, sys->d_F.p, n, r->FR.p, q, 0, B->partial, s);
    gather_recv(sys, q, B->V.p, n, r->CR.p, s);
    if (L > 0) CR_HIP(hipMemcpyAsync(r->flags.p, sys->d_flags.p, L * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    CR_HIP(hipStreamSynchronize(s));
    return r;
}

void fill_sweep_info(cr_sweep_info* info, int mi, int nc, int fb, int np, double secs) {
    if (!info) return;
    info->max_ir_iterations = mi;
    info->not_converged = nc;
    info->fp64_fallbacks = fb;
    info->n_perturbed = np;
    info->seconds = secs;
}

// whether a sweep of r in this precision (and with refinement requested or not) takes the
// Hessenberg-triangular path
bool use_ht(const cr_rom_s* r, cr_precision prec, bool refine, int out_x) {
    return prec == CR_FP64 && !refine && !out_x && ht_eligible(r->q, r->L, r->n_o, r->has_d, (int)r->tmeta.size());
}

// Reduce the models that take the Hessenberg-triangular path and have no reduced form yet, one
// workgroup per model in one launch.
void ensure_ht(const std::vector<cr_rom_s*>& roms, hipStream_t s) {
    std::vector<HtJob> jobs;
    std::vector<cr_rom_s*> todo;
    for (cr_rom_s* r : roms) {
        if (r->ht_ready || std::find(todo.begin(), todo.end(), r) != todo.end()) continue;
        const size_t q = (size_t)r->q;
        r->htH.alloc(q * q);
        r->htT.alloc(q * q);
        r->htF.alloc(q * (size_t)r->L);
        r->htC.alloc((size_t)r->n_o * q);
        r->htN.alloc(2);
        jobs.push_back(HtJob{r->KR.p, r->MR.p, r->FR.p, r->CR.p, r->htH.p, r->htT.p, r->htF.p, r->htC.p, r->htN.p,
                             r->q, r->L, r->n_o});
        todo.push_back(r);
    }
    ht_reduce(jobs, s);
    for (cr_rom_s* r : todo) r->ht_ready = true;
}

RomDesc desc_of(const cr_rom_s* r, const double* omegas_dev, zd* out, int out_x) {
    RomDesc d;
    d.KR = r->KR.p;
    d.MR = r->MR.p;
    d.DR = r->has_d ? r->DR.p : nullptr;
    d.FR = r->FR.p;
    d.CR = r->CR.p;
    d.flags = r->flags.p;
    d.omegas = omegas_dev;
    d.out = out;
    d.q = r->q;
    d.L = r->L;
    d.n_o = r->n_o;
    d.out_x = out_x;
    d.nterm = 0;
    for (int t = 0; t < kMaxTerms; ++t) d.T[t] = nullptr;
    d.tcoef = nullptr;
    d.H = d.Th = d.Ft = d.Ct = nullptr;
    d.htnorm = nullptr;
    return d;
}

// point the descriptor at the model's Hessenberg-triangular form (built by ensure_ht)
void attach_ht(const cr_rom_s* r, RomDesc& d) {
    d.H = r->htH.p;
    d.Th = r->htT.p;
    d.Ft = r->htF.p;
    d.Ct = r->htC.p;
    d.htnorm = r->htN.p;
}

// Frequency-dependent terms of a reduced model: upload the coefficient table of the given host
// frequencies (kind 0: 1 + i eta(w); kind 1: -w^2 / (c^2 (1 + i eta(w)))) into the model's
// buffer and point the descriptor at it; off is the table offset of this call's first frequency.
void attach_terms(cr_rom_s* r, RomDesc& d, const double* omegas, int nfreq, hipStream_t s) {
    const int nt = (int)r->tmeta.size();
    if (nt == 0 || nfreq == 0) return;
    std::vector<zd> tab((size_t)nfreq * nt);
    for (int i = 0; i < nfreq; ++i)
        for (int t = 0; t < nt; ++t) {
            const TermMeta& m = r->tmeta[t];
            zd c = m.coef(omegas[i]);
            if (m.kind == 1) c = {-omegas[i] * omegas[i] * c.re, -omegas[i] * omegas[i] * c.im};
            tab[(size_t)i * nt + t] = c;
        }
    r->tcoef.reserve(tab.size());
    CR_HIP(hipMemcpyAsync(r->tcoef.p, tab.data(), tab.size() * sizeof(zd), hipMemcpyHostToDevice, s));
    CR_HIP(hipStreamSynchronize(s));
    d.nterm = nt;
    for (int t = 0; t < nt; ++t) d.T[t] = r->TR[t].p;
    d.tcoef = r->tcoef.p;
}

}  // namespace

namespace cr {
void finalize_sys(cr_sys sys) {
    const int64_t n = sys->n, nnz = sys->rowptr[n];
    hipStream_t s = sys->ctx->stream;
    sys->scale.assign(n, 1.0);
    // stiffness of frequency-dependent solids taken with loss factor zero (coefficient 1)
    for (int64_t r = 0; r < n; ++r) {
        double d = 0;
        for (int64_t k = sys->rowptr[r]; k < sys->rowptr[r + 1]; ++k)
            if (sys->col[k] == r) {
                double re = sys->K[k].re, im = sys->K[k].im;
                for (const FreqTerm& t : sys->terms)
                    if (t.kind == 0) { re += t.vals[k].re; im += t.vals[k].im; }
                d = std::hypot(re, im);
            }
        CR_REQUIRE(d > 0, CR_E_INVALID, "zero diagonal of K at DoF " + std::to_string(r));
        sys->scale[r] = 1.0 / std::sqrt(d);
    }
    const bool hd = !sys->D.empty();
    std::vector<zd> Ks(nnz), Ms(nnz), Ds(hd ? nnz : 0), Fs(sys->F.size());
    for (int64_t r = 0; r < n; ++r)
        for (int64_t k = sys->rowptr[r]; k < sys->rowptr[r + 1]; ++k) {
            const double f = sys->scale[r] * sys->scale[sys->col[k]];
            Ks[k] = {sys->K[k].re * f, sys->K[k].im * f};
            Ms[k] = {sys->M[k].re * f, sys->M[k].im * f};
            if (hd) Ds[k] = {sys->D[k].re * f, sys->D[k].im * f};
        }
    for (int l = 0; l < sys->L; ++l)
        for (int64_t r = 0; r < n; ++r) {
            const zd v = sys->F[(size_t)l * n + r];
            Fs[(size_t)l * n + r] = {v.re * sys->scale[r], v.im * sys->scale[r]};
        }
    upload(sys->d_rowptr, sys->rowptr, s);
    upload(sys->d_col, sys->col, s);
    upload(sys->d_K, Ks, s);
    upload(sys->d_M, Ms, s);
    if (hd) upload(sys->d_D, Ds, s);
    for (FreqTerm& t : sys->terms) {
        std::vector<zd> Ts(nnz);
        for (int64_t r = 0; r < n; ++r)
            for (int64_t k = sys->rowptr[r]; k < sys->rowptr[r + 1]; ++k) {
                const double f = sys->scale[r] * sys->scale[sys->col[k]];
                Ts[k] = {t.vals[k].re * f, t.vals[k].im * f};
            }
        upload(t.d_vals, Ts, s);
    }
    upload(sys->d_F, Fs, s);
    upload(sys->d_scale, sys->scale, s);
    upload(sys->d_recv, sys->recv, s);
    upload(sys->d_flags, sys->flags, s);
    CR_HIP(hipStreamSynchronize(s));
}
}  // namespace cr

// =============================================================== C ABI
extern "C" {

cr_status cr_ctx_create(int device, void* hip_stream, const cr_allocator* allocator, cr_ctx* out) {
    if (!out) return CR_E_INVALID;
    if (allocator && (!allocator->alloc || !allocator->free)) {
        g_create_error = "allocator without alloc or free function";
        return CR_E_INVALID;
    }
    try {
        int count = 0;
        hipError_t e = hipGetDeviceCount(&count);
        if (e != hipSuccess || count == 0) {
            g_create_error = "no HIP device available";
            return CR_E_HIP;
        }
        if (device < 0 || device >= count) {
            g_create_error = "device index out of range";
            return CR_E_INVALID;
        }
        CR_HIP(hipSetDevice(device));
        auto c = std::make_unique<cr_ctx_s>();
        c->device = device;
        c->stream = reinterpret_cast<hipStream_t>(hip_stream);
        hipDeviceProp_t prop;
        CR_HIP(hipGetDeviceProperties(&prop, device));
        c->num_cu = prop.multiProcessorCount;
        if (allocator) {
            c->alloc = *allocator;
            c->has_alloc = true;
        }
        noalloc_scratch_init(device);   // address of this device's static sweep scratch
        *out = c.release();
        return CR_OK;
    } catch (const cr::Error& e) {
        g_create_error = e.what();
        return e.code;
    }
}

void cr_ctx_destroy(cr_ctx ctx) {
    if (!ctx) return;
    if (ctx->aux) {
        (void)hipStreamSynchronize(ctx->aux);
        (void)hipEventDestroy(ctx->ev_fork);
        (void)hipEventDestroy(ctx->ev_join);
        (void)hipStreamDestroy(ctx->aux);
    }
    delete ctx->sweep;
    delete ctx;
}

const char* cr_last_error(cr_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }
const char* cr_create_error(void) { return g_create_error.c_str(); }

cr_status cr_sys_get_dims(cr_sys sys, cr_sys_dims* out) {
    if (!sys || !out) return CR_E_INVALID;
    out->n = sys->n;
    out->nnz = sys->rowptr[sys->n];
    out->n_u = sys->n_u;
    out->L = sys->L;
    out->n_o = sys->n_o;
    return CR_OK;
}

cr_status cr_sys_export(cr_sys sys, int64_t* rowptr, int32_t* col, cr_z* K, cr_z* M, cr_z* F, int32_t* flags,
                        int64_t* recv_dofs) {
    if (!sys) return CR_E_INVALID;
    const int64_t n = sys->n, nnz = sys->rowptr[n];
    if (rowptr) std::memcpy(rowptr, sys->rowptr.data(), (n + 1) * sizeof(int64_t));
    if (col) std::memcpy(col, sys->col.data(), nnz * sizeof(int32_t));
    if (K) std::memcpy(K, sys->K.data(), nnz * sizeof(cr_z));
    if (M) std::memcpy(M, sys->M.data(), nnz * sizeof(cr_z));
    if (F && !sys->F.empty()) std::memcpy(F, sys->F.data(), sys->F.size() * sizeof(cr_z));
    if (flags && sys->L) std::memcpy(flags, sys->flags.data(), sys->L * sizeof(int32_t));
    if (recv_dofs && sys->n_o) std::memcpy(recv_dofs, sys->recv.data(), sys->n_o * sizeof(int64_t));
    return CR_OK;
}

void cr_sys_destroy(cr_sys sys) { delete sys; }

cr_status cr_sys_import_csr(cr_ctx ctx, int64_t n, const int64_t* rowptr, const int32_t* col, const cr_z* K,
                            const cr_z* D, const cr_z* M, int32_t L, const cr_z* F, const int32_t* flags, int32_t n_o,
                            const int64_t* recv_dofs, const double* coords, cr_sys* out) {
    if (!ctx) return CR_E_INVALID;
    return cr_guard(ctx, [&] {
        CR_REQUIRE(out && n > 0 && n < (int64_t)INT32_MAX && rowptr && col && K && M && L >= 0 && L <= 4096 &&
                       (L == 0 || (F && flags)) && n_o >= 0 && (n_o == 0 || recv_dofs),
                   CR_E_INVALID, "cr_sys_import_csr: bad arguments");
        CR_REQUIRE(rowptr[0] == 0, CR_E_INVALID, "cr_sys_import_csr: rowptr[0] must be 0");
        for (int64_t r = 0; r < n; ++r)
            CR_REQUIRE(rowptr[r + 1] >= rowptr[r], CR_E_INVALID, "cr_sys_import_csr: rowptr not monotone");
        const int64_t nnz = rowptr[n];
        const bool hd = D != nullptr;
        auto finite = [](const cr_z& z) { return std::isfinite(z.re) && std::isfinite(z.im); };
        // entries and transposed explicit zeros, sorted by (row, column); duplicates summed
        std::vector<std::pair<uint64_t, int64_t>> ent;
        ent.reserve((size_t)(2 * nnz));
        for (int64_t r = 0; r < n; ++r)
            for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k) {
                const int64_t c = col[k];
                CR_REQUIRE(c >= 0 && c < n, CR_E_INVALID, "cr_sys_import_csr: column index out of range");
                CR_REQUIRE(finite(K[k]) && finite(M[k]) && (!hd || finite(D[k])), CR_E_INVALID,
                           "cr_sys_import_csr: non-finite matrix value");
                ent.push_back({((uint64_t)r << 32) | (uint64_t)c, k});
                if (c != r) ent.push_back({((uint64_t)c << 32) | (uint64_t)r, -1});
            }
        std::sort(ent.begin(), ent.end());
        auto sys = std::make_unique<cr_sys_s>();
        sys->ctx = ctx;
        sys->n = n;
        sys->n_u = 0;
        sys->L = L;
        sys->n_o = n_o;
        sys->rowptr.assign(n + 1, 0);
        for (size_t e = 0; e < ent.size();) {
            const uint64_t key = ent[e].first;
            const int64_t r = (int64_t)(key >> 32);
            const int32_t c = (int32_t)(key & 0xffffffffu);
            zd kv{0, 0}, mv{0, 0}, dv{0, 0};
            for (; e < ent.size() && ent[e].first == key; ++e) {
                const int64_t k = ent[e].second;
                if (k < 0) continue;
                kv.re += K[k].re; kv.im += K[k].im;
                mv.re += M[k].re; mv.im += M[k].im;
                if (hd) { dv.re += D[k].re; dv.im += D[k].im; }
            }
            sys->col.push_back(c);
            sys->K.push_back(kv);
            sys->M.push_back(mv);
            if (hd) sys->D.push_back(dv);
            sys->rowptr[r + 1]++;
        }
        for (int64_t r = 0; r < n; ++r) sys->rowptr[r + 1] += sys->rowptr[r];
        sys->F.resize((size_t)n * L);
        for (size_t e = 0; e < sys->F.size(); ++e) {
            CR_REQUIRE(finite(F[e]), CR_E_INVALID, "cr_sys_import_csr: non-finite load value");
            sys->F[e] = {F[e].re, F[e].im};
        }
        sys->flags.assign(flags, flags + L);
        for (int32_t f : sys->flags) CR_REQUIRE(f == 0 || f == 1, CR_E_INVALID, "cr_sys_import_csr: flags must be 0 or 1");
        sys->recv.assign(recv_dofs, recv_dofs + n_o);
        for (int64_t r : sys->recv) CR_REQUIRE(r >= 0 && r < n, CR_E_INVALID, "cr_sys_import_csr: receiver DoF out of range");
        if (coords) {
            sys->coords.assign(coords, coords + 3 * n);
            for (double x : sys->coords) CR_REQUIRE(std::isfinite(x), CR_E_INVALID, "cr_sys_import_csr: non-finite coordinate");
        }
        finalize_sys(sys.get());
        *out = sys.release();
    });
}

cr_status cr_set_front_classes(cr_sys sys, int32_t big_m, int32_t huge_m) {
    if (!sys) return CR_E_INVALID;
    return cr_guard(sys->ctx, [&] {
        CR_REQUIRE(!sys->sym, CR_E_STATE, "cr_set_front_classes: call before cr_analyse");
        CR_REQUIRE(big_m >= 32 && huge_m >= 64, CR_E_INVALID, "cr_set_front_classes: thresholds too small");
        sys->fclass.big_m = big_m;
        sys->fclass.huge_m = huge_m;
    });
}

cr_status cr_set_panel_split(cr_sys sys, int32_t min_rows, int32_t max_polls) {
    if (!sys) return CR_E_INVALID;
    return cr_guard(sys->ctx, [&] {
        CR_REQUIRE(min_rows == 0 || min_rows >= 512, CR_E_INVALID, "cr_set_panel_split: min_rows must be 0 or >= 512");
        CR_REQUIRE(max_polls >= 0, CR_E_INVALID, "cr_set_panel_split: max_polls must be >= 0");
        sys->fclass.split_rows = min_rows;
        sys->fclass.split_polls = max_polls;
    });
}

cr_status cr_analyse(cr_sys sys, cr_analysis_info* info) {
    if (!sys) return CR_E_INVALID;
    return cr_guard(sys->ctx, [&] {
        if (!sys->sym) {
            sys->sym = analyse_pattern(sys->n, sys->rowptr, sys->col, sys->coords, sys->fclass);
            upload_symbolic(sys);
        }
        if (info) {
            const Symbolic& S = *sys->sym;
            info->n_fronts = S.nfront;
            info->n_levels = S.nlevel;
            info->max_front = S.max_front;
            info->max_pivots = S.max_piv;
            info->factor_entries = S.factor_entries;
            info->factor_flops = S.factor_flops;
            info->gemm_flops = S.gemm_flops;
            info->seconds = S.seconds;
        }
    });
}

cr_status cr_factor(cr_sys sys, double omega, cr_precision prec, cr_fact* out, cr_factor_info* info) {
    if (!sys) return CR_E_INVALID;
    return cr_guard(sys->ctx, [&] {
        CR_REQUIRE(out && std::isfinite(omega) && (prec == CR_FP64 || prec == CR_MIXED), CR_E_INVALID, "cr_factor: bad arguments");
        CR_REQUIRE(sys->sym, CR_E_STATE, "cr_factor: call cr_analyse first");
        const double t0 = now();
        auto f = std::make_unique<cr_fact_s>();
        numeric_factor(f->f, sys, omega, prec, sys->ctx->stream);
        if (info) {
            info->n_perturbed = f->f.n_perturbed;
            info->seconds = now() - t0;
        }
        *out = f.release();
    });
}

void cr_fact_destroy(cr_fact f) { delete f; }

cr_status cr_solve(cr_fact f, int32_t nrhs, const cr_z* B_dev, cr_z* X_dev, const cr_ir_opts* opts, cr_solve_info* info) {
    if (!f) return CR_E_INVALID;
    cr_sys sys = f->f.sys;
    return cr_guard(sys->ctx, [&] {
        CR_REQUIRE(nrhs >= 0 && (nrhs == 0 || (B_dev && X_dev)), CR_E_INVALID, "cr_solve: bad arguments");
        if (nrhs == 0) return;
        hipStream_t s = sys->ctx->stream;
        const int64_t n = sys->n;
        const int max_iter = opts ? opts->max_iter : 10;
        const double tol = opts ? opts->tol : 1e-14;
        // A = S^{-1} A~ S^{-1}: X = S (A~^{-1} (S B))
        DevBuf<zd> Bs((size_t)n * nrhs), Xs((size_t)n * nrhs);
        scale_rows(n, nrhs, reinterpret_cast<const zd*>(B_dev), sys->d_scale.p, Bs.p, s);
        double berr = 0;
        int its = 0;
        cr_status st = CR_OK;
        std::string msg;
        try {
            its = solve_scaled(f->f, nrhs, Bs.p, Xs.p, max_iter, tol, &berr, f->w, s, true);
        } catch (const cr::Error& e) {
            if (e.code != CR_E_NOT_CONVERGED) throw;
            st = e.code;
            msg = e.what();
        }
        scale_rows(n, nrhs, Xs.p, sys->d_scale.p, reinterpret_cast<zd*>(X_dev), s);
        CR_HIP(hipStreamSynchronize(s));
        if (info) {
            info->iterations = its;
            info->backward_error = berr;
        }
        if (st != CR_OK) throw cr::Error(st, msg);
    });
}

cr_status cr_basis_build(cr_sys sys, int32_t nshift, const double* omegas, const int32_t* blocks, cr_precision prec,
                         cr_basis* out, cr_basis_info* info) {
    if (!sys) return CR_E_INVALID;
    return cr_guard(sys->ctx, [&] {
        CR_REQUIRE(out && nshift > 0 && omegas && blocks, CR_E_INVALID, "cr_basis_build: bad arguments");
        CR_REQUIRE(prec == CR_FP64 || prec == CR_MIXED, CR_E_INVALID, "cr_basis_build: bad precision");
        CR_REQUIRE(sys->sym, CR_E_STATE, "cr_basis_build: call cr_analyse first");
        CR_REQUIRE(sys->L > 0, CR_E_INVALID, "cr_basis_build: system has no loads");
        const double t0 = now();
        auto B = std::make_unique<cr_basis_s>();
        B->sys = sys;
        int total = 0;
        for (int j = 0; j < nshift; ++j) {
            CR_REQUIRE(blocks[j] >= 0 && std::isfinite(omegas[j]), CR_E_INVALID, "cr_basis_build: bad shift");
            total += blocks[j] * sys->L;
        }
        ensure_capacity(B.get(), std::max(total, 1));
        Factor fac;
        SolveWork sw;
        for (int j = 0; j < nshift; ++j) {
            if (sys->D.empty()) add_shift(B.get(), fac, sw, omegas[j], blocks[j], prec);
            else add_shift_soar(B.get(), fac, sw, omegas[j], blocks[j], prec);
        }
        fill_info(B.get(), info, t0);
        *out = B.release();
    });
}

}  // extern "C"

namespace {
// The residual-maximum greedy (Section 3.3, after Eq. (9)) on the candidate grid of o; options
// already validated. maxres_out receives the largest candidate residual after each point.
std::unique_ptr<cr_basis_s> run_greedy(cr_sys sys, const cr_greedy_opts* o, cr_precision prec, cr_greedy_trace* trace,
                                       std::vector<double>* maxres_out) {
    hipStream_t s = sys->ctx->stream;
    const int nc = o->n_cand, L = sys->L;
    const int64_t n = sys->n;
    // candidates as numpy.linspace computes them (start + i * step, last = stop exactly)
    std::vector<double> cand(nc), cw(nc), w2(nc);
    const double step = (o->f_hi_hz - o->f_lo_hz) / (nc - 1);
    for (int i = 0; i < nc; ++i) cand[i] = i * step + o->f_lo_hz;
    cand[nc - 1] = o->f_hi_hz;
    for (int i = 0; i < nc; ++i) {
        cw[i] = (2.0 * M_PI) * cand[i];
        w2[i] = cw[i] * cw[i];
    }
    const double centre = 0.5 * (cand[0] + cand[nc - 1]);
    int j = 0;
    for (int i = 1; i < nc; ++i)
        if (std::fabs(cand[i] - centre) < std::fabs(cand[j] - centre)) j = i;
    auto B = std::make_unique<cr_basis_s>();
    B->sys = sys;
    ensure_capacity(B.get(), o->blocks * L * std::min(o->max_shifts, 64));
    Factor fac;
    SolveWork sw;
    SweepEngine& E = engine(sys->ctx);
    // load scales (i w_c)^flag and ||S f(w_c)||_F^2
    std::vector<zd> scal((size_t)nc * L);
    std::vector<double> fn2(nc, 0.0);
    std::vector<double> f2 = col_norms2(B.get(), sys->d_F.p, L);
    for (int c = 0; c < nc; ++c)
        for (int l = 0; l < L; ++l) {
            scal[(size_t)c * L + l] = sys->flags[l] ? zd{0.0, cw[c]} : zd{1.0, 0.0};
            fn2[c] += (sys->flags[l] ? w2[c] : 1.0) * f2[l];
        }
    DevBuf<zd> d_scal(scal.size());
    DevBuf<double> d_w2(nc), d_cw(nc), d_res2(nc), partial;
    CR_HIP(hipMemcpyAsync(d_scal.p, scal.data(), scal.size() * sizeof(zd), hipMemcpyHostToDevice, s));
    CR_HIP(hipMemcpyAsync(d_w2.p, w2.data(), nc * sizeof(double), hipMemcpyHostToDevice, s));
    CR_HIP(hipMemcpyAsync(d_cw.p, cw.data(), nc * sizeof(double), hipMemcpyHostToDevice, s));
    DevBuf<zd> Xc;
    std::vector<int> used;
    std::vector<double> maxres, res(nc, 0.0);
    std::vector<int> mlp_used;
    std::vector<int2> items(nc);
    for (int c = 0; c < nc; ++c) items[c] = make_int2(0, c);
    int stalled = 0;
    for (int it = 0; it < o->max_shifts; ++it) {
        used.push_back(j);
        const int q_before = B->q;
        add_shift(B.get(), fac, sw, cw[j], o->blocks, prec);
        stalled = B->q == q_before ? stalled + 1 : 0;
        auto rom = rom_from_basis(B.get());
        const int q = B->q;
        Xc.reserve((size_t)nc * q * L);
        std::vector<RomDesc> rd{desc_of(rom.get(), d_cw.p, Xc.p, 1)};
        int mi, ncv, np;
        E.run(rd, items, CR_FP64, false, s, &mi, &ncv, &np);
        {
            ProfScope ps(sys->ctx, "resid", s);
            candidate_residuals(n, q, L, nc, B->KV.p, B->MV.p, n, sys->d_F.p, Xc.p, d_scal.p, d_w2.p, d_res2.p, partial, s);
        }
        CR_HIP(hipMemcpyAsync(res.data(), d_res2.p, nc * sizeof(double), hipMemcpyDeviceToHost, s));
        CR_HIP(hipStreamSynchronize(s));
        double mx = 0;
        for (int c = 0; c < nc; ++c) {
            res[c] = std::sqrt(res[c] / fn2[c]);
            mx = std::max(mx, res[c]);
        }
        if (trace && trace->res_hist) std::copy(res.begin(), res.end(), trace->res_hist + (size_t)it * nc);
        maxres.push_back(mx);
        if (mx <= o->tol) break;
        if (o->stall_stop > 0 && stalled >= o->stall_stop) break;
        if (o->lookahead > 0) {
            // one-step look-ahead over the K largest residual peaks, each tried on a copy
            const int K = o->lookahead;
            std::vector<int> idx(nc);
            std::iota(idx.begin(), idx.end(), 0);
            std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return res[a] > res[b]; });
            std::vector<int> picks;
            for (int c : idx) {
                if ((int)picks.size() >= K) break;
                bool bad = false;
                for (int u : used) bad = bad || std::abs(u - c) <= 1;
                for (int pk : picks) bad = bad || std::abs(pk - c) < 3;
                if (!bad) picks.push_back(c);
            }
            std::vector<double> rtmp(nc);
            for (int k = 0; k < K; ++k) {
                double best_after = -1.0;
                const int c = k < (int)picks.size() ? picks[k] : -1;
                if (c >= 0) {
                    auto Bc = clone_basis(B.get());
                    add_shift(Bc.get(), fac, sw, cw[c], o->blocks, prec);
                    auto romc = rom_from_basis(Bc.get());
                    const int qc = Bc->q;
                    Xc.reserve((size_t)nc * qc * L);
                    std::vector<RomDesc> rdc{desc_of(romc.get(), d_cw.p, Xc.p, 1)};
                    int mi2, ncv2, np2;
                    E.run(rdc, items, CR_FP64, false, s, &mi2, &ncv2, &np2);
                    candidate_residuals(n, qc, L, nc, Bc->KV.p, Bc->MV.p, n, sys->d_F.p, Xc.p, d_scal.p, d_w2.p,
                                        d_res2.p, partial, s);
                    CR_HIP(hipMemcpyAsync(rtmp.data(), d_res2.p, nc * sizeof(double), hipMemcpyDeviceToHost, s));
                    CR_HIP(hipStreamSynchronize(s));
                    best_after = 0;
                    for (int cc = 0; cc < nc; ++cc) best_after = std::max(best_after, std::sqrt(rtmp[cc] / fn2[cc]));
                }
                if (trace && trace->la_cand) trace->la_cand[(size_t)it * K + k] = c;
                if (trace && trace->la_res) trace->la_res[(size_t)it * K + k] = best_after;
            }
        }
        int best = -1;
        for (int c = 0; c < nc; ++c) {
            if (std::find(used.begin(), used.end(), c) != used.end()) continue;
            if (best < 0 || res[c] > res[best]) best = c;
        }
        if (best < 0) break;
        int choice = best, took_mlp = 0;
        if (o->policy == CR_POLICY_MLP) {
            const int prop = mlp_propose(o->mlp, res, used, o->geom);
            if (prop >= 0 && res[prop] >= 0.1 * mx) { choice = prop; took_mlp = 1; }
        }
        mlp_used.push_back(took_mlp);
        j = choice;
    }
    if (trace) {
        trace->n_iter = (int)used.size();
        for (size_t k = 0; k < used.size(); ++k) {
            if (trace->shift_idx) trace->shift_idx[k] = used[k];
            if (trace->max_res) trace->max_res[k] = maxres[k];
            if (trace->mlp_used) trace->mlp_used[k] = (k >= 1 && k - 1 < mlp_used.size()) ? mlp_used[k - 1] : 0;
        }
        if (trace->res) std::copy(res.begin(), res.end(), trace->res);
    }
    if (maxres_out) *maxres_out = maxres;
    return B;
}

void check_greedy_opts(cr_sys sys, const cr_greedy_opts* o, cr_precision prec) {
    CR_REQUIRE(o, CR_E_INVALID, "cr_basis_build_greedy: bad arguments");
    CR_REQUIRE(o->n_cand >= 2 && o->n_cand <= 4096 && o->blocks >= 1 && o->max_shifts >= 1 && o->tol > 0 &&
                   o->stall_stop >= 0 && o->lookahead >= 0 &&
                   std::isfinite(o->f_lo_hz) && std::isfinite(o->f_hi_hz) && o->f_hi_hz > o->f_lo_hz && o->f_lo_hz >= 0,
               CR_E_INVALID, "cr_basis_build_greedy: bad options");
    CR_REQUIRE(prec == CR_FP64 || prec == CR_MIXED, CR_E_INVALID, "cr_basis_build_greedy: bad precision");
    CR_REQUIRE(o->policy == CR_POLICY_GREEDY || (o->policy == CR_POLICY_MLP && o->mlp), CR_E_INVALID,
               "cr_basis_build_greedy: MLP policy needs a network");
    CR_REQUIRE(sys->sym, CR_E_STATE, "cr_basis_build_greedy: call cr_analyse first");
    CR_REQUIRE(sys->D.empty() && sys->terms.empty(), CR_E_UNSUPPORTED,
               "cr_basis_build_greedy: systems with a damping matrix or frequency-dependent materials take fixed "
               "expansion points (cr_basis_build)");
    CR_REQUIRE(sys->L > 0, CR_E_INVALID, "cr_basis_build_greedy: system has no loads");
}
}  // namespace

extern "C" {

cr_status cr_basis_build_greedy(cr_sys sys, const cr_greedy_opts* o, cr_precision prec, cr_basis* out,
                                cr_greedy_trace* trace, cr_basis_info* info) {
    if (!sys) return CR_E_INVALID;
    return cr_guard(sys->ctx, [&] {
        CR_REQUIRE(o && out, CR_E_INVALID, "cr_basis_build_greedy: bad arguments");
        check_greedy_opts(sys, o, prec);
        const double t0 = now();
        auto B = run_greedy(sys, o, prec, trace, nullptr);
        fill_info(B.get(), info, t0);
        *out = B.release();
    });
}

cr_status cr_build_local_roms(cr_sys sys, const cr_window_opts* o, cr_precision prec, int32_t* n_windows,
                              int32_t* win_cand, double* win_hi_hz, double* win_max_res, cr_rom* roms,
                              cr_window_info* info) {
    if (!sys) return CR_E_INVALID;
    std::vector<cr_rom> made;
    cr_status st = cr_guard(sys->ctx, [&] {
        CR_REQUIRE(o && n_windows && win_cand && win_hi_hz && roms && o->max_windows >= 1 && o->min_cand >= 2,
                   CR_E_INVALID, "cr_build_local_roms: bad arguments");
        cr_greedy_opts g{};
        g.f_lo_hz = o->f_lo_hz;
        g.f_hi_hz = o->f_hi_hz;
        g.n_cand = o->n_cand;
        g.blocks = o->blocks;
        g.tol = o->tol;
        g.max_shifts = o->max_shifts;
        g.policy = CR_POLICY_GREEDY;
        check_greedy_opts(sys, &g, prec);
        const double t0 = now();
        const int nc = o->n_cand;
        std::vector<double> cand(nc);
        const double step = (o->f_hi_hz - o->f_lo_hz) / (nc - 1);
        for (int i = 0; i < nc; ++i) cand[i] = i * step + o->f_lo_hz;
        cand[nc - 1] = o->f_hi_hz;
        int attempted = 0, unconv = 0, qmax = 0, kept_shifts = 0;
        // bisection: a window whose greedy misses tol within max_shifts points is split at its
        // middle candidate (shared by both halves) while both halves keep min_cand candidates
        std::vector<std::pair<int, int>> todo{{0, nc - 1}};
        while (!todo.empty()) {
            const auto [i0, i1] = todo.back();
            todo.pop_back();
            const int k = i1 - i0 + 1;
            cr_greedy_opts gw = g;
            gw.f_lo_hz = cand[i0];
            gw.f_hi_hz = cand[i1];
            gw.n_cand = k;
            std::vector<double> mres;
            auto B = run_greedy(sys, &gw, prec, nullptr, &mres);
            attempted += (int)B->shifts.size();
            const bool conv = !mres.empty() && mres.back() <= o->tol;
            if (conv || k < 2 * o->min_cand - 1) {
                CR_REQUIRE((int)made.size() < o->max_windows, CR_E_INVALID,
                           "cr_build_local_roms: more windows than max_windows");
                const int w = (int)made.size();
                win_cand[2 * w] = i0;
                win_cand[2 * w + 1] = i1;
                win_hi_hz[w] = cand[i1];
                if (win_max_res) win_max_res[w] = mres.empty() ? 0.0 : mres.back();
                unconv += conv ? 0 : 1;
                qmax = std::max(qmax, B->q);
                kept_shifts += (int)B->shifts.size();
                made.push_back(rom_from_basis(B.get()).release());
                continue;
            }
            const int mid = (i0 + i1) / 2;
            todo.push_back({mid, i1});   // left half first
            todo.push_back({i0, mid});
        }
        *n_windows = (int32_t)made.size();
        for (size_t w = 0; w < made.size(); ++w) roms[w] = made[w];
        if (info) {
            info->n_windows = (int32_t)made.size();
            info->expansion_points = kept_shifts;
            info->attempted_points = attempted;
            info->max_q = qmax;
            info->unconverged = unconv;
            info->seconds = now() - t0;
        }
    });
    if (st != CR_OK)
        for (cr_rom r : made) delete r;
    return st;
}

cr_status cr_sweep_windows(int32_t nwin, const cr_rom* roms, const double* win_hi_hz, int32_t nfreq,
                           const double* omegas, cr_precision prec, cr_z* Y_dev, cr_sweep_info* info) {
    if (nwin < 1 || !roms || !roms[0]) return CR_E_INVALID;
    cr_ctx ctx = roms[0]->ctx;
    return cr_guard(ctx, [&] {
        CR_REQUIRE(win_hi_hz && nfreq >= 0 && (nfreq == 0 || (omegas && Y_dev)), CR_E_INVALID,
                   "cr_sweep_windows: bad arguments");
        CR_REQUIRE(prec == CR_FP64 || prec == CR_MIXED, CR_E_INVALID, "cr_sweep_windows: bad precision");
        for (int k = 0; k < nwin; ++k) {
            CR_REQUIRE(roms[k] && roms[k]->ctx == ctx && roms[k]->L == roms[0]->L && roms[k]->n_o == roms[0]->n_o,
                       CR_E_INVALID, "cr_sweep_windows: windows of different systems");
            CR_REQUIRE(k == 0 || win_hi_hz[k] >= win_hi_hz[k - 1], CR_E_INVALID,
                       "cr_sweep_windows: window edges not increasing");
        }
        for (int i = 0; i < nfreq; ++i)
            CR_REQUIRE(std::isfinite(omegas[i]), CR_E_INVALID, "cr_sweep_windows: non-finite frequency");
        const double t0 = now();
        hipStream_t s = ctx->stream;
        SweepEngine& E = engine(ctx);
        E.d_omega.reserve(std::max(nfreq, 1));
        if (nfreq) CR_HIP(hipMemcpyAsync(E.d_omega.p, omegas, nfreq * sizeof(double), hipMemcpyHostToDevice, s));
        std::vector<RomDesc> ds(nwin);
        for (int k = 0; k < nwin; ++k) {
            CR_REQUIRE(roms[k]->tmeta.empty(), CR_E_UNSUPPORTED,
                       "cr_sweep_windows: reduced models with frequency-dependent terms need cr_sweep");
            ds[k] = desc_of(roms[k], E.d_omega.p, reinterpret_cast<zd*>(Y_dev), 0);
        }
        // each frequency to the first window whose upper edge is not below it (the last above
        // the band); items ordered by the window's q^3, longest first
        std::vector<int2> items(nfreq);
        for (int i = 0; i < nfreq; ++i) {
            const double f = omegas[i] / (2.0 * M_PI);
            int k = 0;
            while (k < nwin - 1 && f > win_hi_hz[k]) ++k;
            items[i] = make_int2(k, i);
        }
        std::stable_sort(items.begin(), items.end(), [&](int2 a, int2 b) { return ds[a.x].q > ds[b.x].q; });
        int mi = 0, nc = 0, np = 0, fb = 0;
        E.run(ds, items, prec, prec == CR_MIXED, s, &mi, &nc, &np, 0, &fb);
        fill_sweep_info(info, mi, nc, fb, np, now() - t0);
        CR_REQUIRE(nc == 0, CR_E_NOT_CONVERGED,
                   "cr_sweep_windows: refinement did not reach its tolerance at " + std::to_string(nc) + " frequencies");
    });
}

cr_status cr_basis_dims(cr_basis b, int32_t* q) {
    if (!b || !q) return CR_E_INVALID;
    *q = b->q;
    return CR_OK;
}

cr_status cr_basis_copy(cr_basis b, cr_z* V_dev) {
    if (!b) return CR_E_INVALID;
    return cr_guard(b->sys->ctx, [&] {
        CR_REQUIRE(V_dev || b->q == 0, CR_E_INVALID, "cr_basis_copy: null output");
        copy_dev(b->sys->n * b->q, b->V.p, reinterpret_cast<zd*>(V_dev), b->sys->ctx->stream);
        CR_HIP(hipStreamSynchronize(b->sys->ctx->stream));
    });
}

void cr_basis_destroy(cr_basis b) { delete b; }

cr_status cr_recover_field(cr_basis b, int64_t ncol, const cr_z* XR_dev, cr_z* X_dev) {
    if (!b) return CR_E_INVALID;
    return cr_guard(b->sys->ctx, [&] {
        CR_REQUIRE(ncol >= 0 && (ncol == 0 || (XR_dev && X_dev)) && ncol <= (int64_t)INT32_MAX, CR_E_INVALID,
                   "cr_recover_field: bad arguments");
        CR_REQUIRE(b->q > 0 || ncol == 0, CR_E_INVALID, "cr_recover_field: empty basis");
        if (ncol == 0) return;
        cr_sys sys = b->sys;
        hipStream_t s = sys->ctx->stream;
        lift(sys->n, b->q, (int)ncol, b->V.p, sys->n, reinterpret_cast<const zd*>(XR_dev), b->q, sys->d_scale.p,
             reinterpret_cast<zd*>(X_dev), sys->n, s);
        CR_HIP(hipGetLastError());
        CR_HIP(hipStreamSynchronize(s));
    });
}

cr_status cr_project(cr_sys sys, cr_basis b, cr_rom* out) {
    if (!sys || !b) return CR_E_INVALID;
    return cr_guard(sys->ctx, [&] {
        CR_REQUIRE(out && b->sys == sys, CR_E_INVALID, "cr_project: basis of another system");
        CR_REQUIRE(b->q > 0, CR_E_INVALID, "cr_project: empty basis");
        *out = rom_from_basis(b).release();
    });
}

cr_status cr_rom_import(cr_ctx ctx, int32_t q, int32_t L, int32_t n_o, const cr_z* KR, const cr_z* DR, const cr_z* MR,
                        const cr_z* FR, const cr_z* CR, const int32_t* flags, cr_rom* out) {
    if (!ctx) return CR_E_INVALID;
    return cr_guard(ctx, [&] {
        CR_REQUIRE(out && q > 0 && q <= 4096 && L > 0 && n_o >= 0 && KR && MR && FR && flags && (n_o == 0 || CR),
                   CR_E_INVALID, "cr_rom_import: bad arguments");
        hipStream_t s = ctx->stream;
        auto r = std::make_unique<cr_rom_s>();
        r->ctx = ctx;
        r->q = q;
        r->L = L;
        r->n_o = n_o;
        r->KR.alloc((size_t)q * q);
        r->MR.alloc((size_t)q * q);
        r->FR.alloc((size_t)q * L);
        r->CR.alloc((size_t)std::max(n_o, 1) * q);
        r->flags.alloc(L);
        CR_HIP(hipMemcpyAsync(r->KR.p, KR, (size_t)q * q * sizeof(zd), hipMemcpyHostToDevice, s));
        CR_HIP(hipMemcpyAsync(r->MR.p, MR, (size_t)q * q * sizeof(zd), hipMemcpyHostToDevice, s));
        CR_HIP(hipMemcpyAsync(r->FR.p, FR, (size_t)q * L * sizeof(zd), hipMemcpyHostToDevice, s));
        if (n_o) CR_HIP(hipMemcpyAsync(r->CR.p, CR, (size_t)n_o * q * sizeof(zd), hipMemcpyHostToDevice, s));
        CR_HIP(hipMemcpyAsync(r->flags.p, flags, L * sizeof(int32_t), hipMemcpyHostToDevice, s));
        if (DR) {
            r->has_d = true;
            r->DR.alloc((size_t)q * q);
            CR_HIP(hipMemcpyAsync(r->DR.p, DR, (size_t)q * q * sizeof(zd), hipMemcpyHostToDevice, s));
        }
        CR_HIP(hipStreamSynchronize(s));
        *out = r.release();
    });
}

cr_status cr_rom_dims(cr_rom r, int32_t* q, int32_t* L, int32_t* n_o) {
    if (!r) return CR_E_INVALID;
    if (q) *q = r->q;
    if (L) *L = r->L;
    if (n_o) *n_o = r->n_o;
    return CR_OK;
}

cr_status cr_rom_export(cr_rom r, cr_z* KR, cr_z* MR, cr_z* FR, cr_z* CR) {
    if (!r) return CR_E_INVALID;
    return cr_guard(r->ctx, [&] {
        hipStream_t s = r->ctx->stream;
        const size_t q = r->q;
        if (KR) CR_HIP(hipMemcpyAsync(KR, r->KR.p, q * q * sizeof(zd), hipMemcpyDeviceToHost, s));
        if (MR) CR_HIP(hipMemcpyAsync(MR, r->MR.p, q * q * sizeof(zd), hipMemcpyDeviceToHost, s));
        if (FR) CR_HIP(hipMemcpyAsync(FR, r->FR.p, q * r->L * sizeof(zd), hipMemcpyDeviceToHost, s));
        if (CR && r->n_o) CR_HIP(hipMemcpyAsync(CR, r->CR.p, q * r->n_o * sizeof(zd), hipMemcpyDeviceToHost, s));
        CR_HIP(hipStreamSynchronize(s));
    });
}

void cr_rom_destroy(cr_rom r) { delete r; }

cr_status cr_sweep(cr_rom r, int32_t nfreq, const double* omegas, cr_precision prec, cr_z* Y_dev, cr_sweep_info* info) {
    if (!r) return CR_E_INVALID;
    return cr_guard(r->ctx, [&] {
        CR_REQUIRE(nfreq >= 0 && (nfreq == 0 || (omegas && Y_dev)), CR_E_INVALID, "cr_sweep: bad arguments");
        CR_REQUIRE(prec == CR_FP64 || prec == CR_MIXED, CR_E_INVALID, "cr_sweep: bad precision");
        for (int i = 0; i < nfreq; ++i) CR_REQUIRE(std::isfinite(omegas[i]), CR_E_INVALID, "cr_sweep: non-finite frequency");
        const double t0 = now();
        hipStream_t s = r->ctx->stream;
        SweepEngine& E = engine(r->ctx);
        E.d_omega.reserve(std::max(nfreq, 1));
        if (nfreq) CR_HIP(hipMemcpyAsync(E.d_omega.p, omegas, nfreq * sizeof(double), hipMemcpyHostToDevice, s));
        std::vector<RomDesc> roms{desc_of(r, E.d_omega.p, reinterpret_cast<zd*>(Y_dev), 0)};
        attach_terms(r, roms[0], omegas, nfreq, s);
        if (nfreq && use_ht(r, prec, prec == CR_MIXED, 0)) {
            ensure_ht({r}, s);
            attach_ht(r, roms[0]);
        }
        std::vector<int2> items(nfreq);
        for (int i = 0; i < nfreq; ++i) items[i] = make_int2(0, i);
        int mi = 0, nc = 0, np = 0, fb = 0;
        E.run(roms, items, prec, prec == CR_MIXED, s, &mi, &nc, &np, 0, &fb);
        fill_sweep_info(info, mi, nc, fb, np, now() - t0);
        CR_REQUIRE(nc == 0, CR_E_NOT_CONVERGED,
                   "cr_sweep: refinement did not reach its tolerance at " + std::to_string(nc) + " frequencies");
    });
}

cr_status cr_sweep_states(cr_rom r, int32_t nfreq, const double* omegas, cr_precision prec, cr_z* XR_dev,
                          cr_sweep_info* info) {
    if (!r) return CR_E_INVALID;
    return cr_guard(r->ctx, [&] {
        CR_REQUIRE(nfreq >= 0 && (nfreq == 0 || (omegas && XR_dev)), CR_E_INVALID, "cr_sweep_states: bad arguments");
        CR_REQUIRE(prec == CR_FP64 || prec == CR_MIXED, CR_E_INVALID, "cr_sweep_states: bad precision");
        for (int i = 0; i < nfreq; ++i)
            CR_REQUIRE(std::isfinite(omegas[i]), CR_E_INVALID, "cr_sweep_states: non-finite frequency");
        const double t0 = now();
        hipStream_t s = r->ctx->stream;
        SweepEngine& E = engine(r->ctx);
        E.d_omega.reserve(std::max(nfreq, 1));
        if (nfreq) CR_HIP(hipMemcpyAsync(E.d_omega.p, omegas, nfreq * sizeof(double), hipMemcpyHostToDevice, s));
        std::vector<RomDesc> roms{desc_of(r, E.d_omega.p, reinterpret_cast<zd*>(XR_dev), 1)};
        attach_terms(r, roms[0], omegas, nfreq, s);
        std::vector<int2> items(nfreq);
        for (int i = 0; i < nfreq; ++i) items[i] = make_int2(0, i);
        int mi = 0, nc = 0, np = 0, fb = 0;
        E.run(roms, items, prec, prec == CR_MIXED, s, &mi, &nc, &np, 0, &fb);
        fill_sweep_info(info, mi, nc, fb, np, now() - t0);
        CR_REQUIRE(nc == 0, CR_E_NOT_CONVERGED,
                   "cr_sweep_states: refinement did not reach its tolerance at " + std::to_string(nc) + " frequencies");
    });
}

cr_status cr_sweep_noalloc(cr_rom r, int32_t nfreq, const double* omegas, cr_precision prec, cr_z* Y_dev,
                           cr_sweep_info* info) {
    if (!r) return CR_E_INVALID;
    return cr_guard(r->ctx, [&] {
        CR_REQUIRE(nfreq >= 0 && (nfreq == 0 || (omegas && Y_dev)), CR_E_INVALID, "cr_sweep_noalloc: bad arguments");
        CR_REQUIRE(prec == CR_FP64 || prec == CR_MIXED, CR_E_INVALID, "cr_sweep_noalloc: bad precision");
        for (int i = 0; i < nfreq; ++i)
            CR_REQUIRE(std::isfinite(omegas[i]), CR_E_INVALID, "cr_sweep_noalloc: non-finite frequency");
        const double t0 = now();
        CR_REQUIRE(r->tmeta.empty(), CR_E_UNSUPPORTED,
                   "cr_sweep_noalloc: reduced models with frequency-dependent terms need cr_sweep");
        const RomDesc d = desc_of(r, nullptr, reinterpret_cast<zd*>(Y_dev), 0);
        int mi = 0, nc = 0, np = 0, fb = 0;
        sweep_noalloc(r->ctx->device, r->ctx->num_cu, d, omegas, nfreq, prec, r->ctx->stream, &mi, &nc, &np, &fb);
        fill_sweep_info(info, mi, nc, fb, np, now() - t0);
        CR_REQUIRE(nc == 0, CR_E_NOT_CONVERGED,
                   "cr_sweep_noalloc: refinement did not reach its tolerance at " + std::to_string(nc) + " frequencies");
    });
}

cr_status cr_sweep_batched(cr_ctx ctx, int32_t nrom, const cr_rom* roms, int32_t nfreq, const double* omegas,
                           cr_precision prec, cr_z* const* Y_dev, const cr_tune* tune, cr_sweep_info* info) {
    if (!ctx) return CR_E_INVALID;
    return cr_guard(ctx, [&] {
        CR_REQUIRE(nrom >= 0 && nfreq >= 0 && (nrom == 0 || (roms && Y_dev)) && (nfreq == 0 || omegas), CR_E_INVALID,
                   "cr_sweep_batched: bad arguments");
        CR_REQUIRE(prec == CR_FP64 || prec == CR_MIXED, CR_E_INVALID, "cr_sweep_batched: bad precision");
        CR_REQUIRE(!tune || (tune->variant >= 0 && tune->variant <= 2 && tune->grid_per_cu >= 0 && tune->nb >= 0 &&
                             tune->nb <= 150),
                   CR_E_INVALID, "cr_sweep_batched: bad tuning");
        const double t0 = now();
        hipStream_t s = ctx->stream;
        SweepEngine& E = engine(ctx);
        const size_t nw = (size_t)nrom * nfreq;
        for (size_t i = 0; i < nw; ++i) CR_REQUIRE(std::isfinite(omegas[i]), CR_E_INVALID, "cr_sweep_batched: non-finite frequency");
        E.d_omega.reserve(std::max<size_t>(nw, 1));
        if (nw) CR_HIP(hipMemcpyAsync(E.d_omega.p, omegas, nw * sizeof(double), hipMemcpyHostToDevice, s));
        std::vector<RomDesc> ds(nrom);
        for (int m = 0; m < nrom; ++m) {
            CR_REQUIRE(roms[m] && roms[m]->ctx == ctx && Y_dev[m], CR_E_INVALID, "cr_sweep_batched: bad model");
            ds[m] = desc_of(roms[m], E.d_omega.p + (size_t)m * nfreq, reinterpret_cast<zd*>(Y_dev[m]), 0);
            // a model with frequency-dependent terms keeps one coefficient table per call
            for (int m2 = 0; m2 < m && !roms[m]->tmeta.empty(); ++m2)
                CR_REQUIRE(roms[m2] != roms[m], CR_E_INVALID,
                           "cr_sweep_batched: a model with frequency-dependent terms appears twice");
            attach_terms(roms[m], ds[m], omegas + (size_t)m * nfreq, nfreq, s);
        }
        const bool refine = prec == CR_MIXED || (tune && tune->refine);
        {
            std::vector<cr_rom_s*> hts;
            for (int m = 0; m < nrom; ++m)
                if (nfreq && use_ht(roms[m], prec, refine, 0)) hts.push_back(roms[m]);
            ensure_ht(hts, s);
            for (int m = 0; m < nrom; ++m)
                if (nfreq && use_ht(roms[m], prec, refine, 0)) attach_ht(roms[m], ds[m]);
        }
        // longest first: q^3 descending, then model index, then frequency
        std::vector<int> order(nrom);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ds[a].q > ds[b].q; });
        std::vector<int2> items;
        items.reserve(nw);
        for (int m : order)
            for (int i = 0; i < nfreq; ++i) items.push_back(make_int2(m, i));
        int mi = 0, nc = 0, np = 0, fb = 0;
        const int gpc = tune && tune->grid_per_cu > 0 ? tune->grid_per_cu : 2;
        const int lds = tune && tune->variant == 1 ? tune->nb * 1024 : 0;
        E.prepare(ds, items, s);
        E.launch(prec, refine, gpc, lds, s);
        E.read_stats(s, &mi, &nc, &np, &fb);
        fill_sweep_info(info, mi, nc, fb, np, now() - t0);
        CR_REQUIRE(nc == 0, CR_E_NOT_CONVERGED,
                   "cr_sweep_batched: refinement did not reach its tolerance at " + std::to_string(nc) + " items");
    });
}

}  // extern "C"

extern "C" cr_status cr_profile_enable(cr_ctx ctx, int32_t on) {
    if (!ctx) return CR_E_INVALID;
    return cr_guard(ctx, [&] {
        CR_HIP(hipStreamSynchronize(ctx->stream));
        ctx->prof.clear();
        ctx->prof.on = on != 0;
    });
}

extern "C" cr_status cr_profile_select(cr_ctx ctx, const char* names) {
    if (!ctx) return CR_E_INVALID;
    return cr_guard(ctx, [&] {
        ctx->prof.only.clear();
        if (!names) return;
        std::string cur;
        for (const char* c = names;; ++c) {
            if (*c == ',' || *c == 0) {
                if (!cur.empty()) ctx->prof.only.push_back(cur);
                cur.clear();
                if (*c == 0) break;
            } else if (*c != ' ') {
                cur.push_back(*c);
            }
        }
    });
}

extern "C" cr_status cr_profile_read(cr_ctx ctx, int32_t max, char* names, int32_t* counts, double* total_ms, int32_t* n) {
    if (!ctx) return CR_E_INVALID;
    return cr_guard(ctx, [&] {
        CR_REQUIRE(max >= 0 && n && (max == 0 || (names && counts && total_ms)), CR_E_INVALID, "cr_profile_read: bad arguments");
        CR_HIP(hipStreamSynchronize(ctx->stream));
        std::vector<std::string> keys;
        std::vector<int> cnt;
        std::vector<double> tot;
        for (const auto& r : ctx->prof.recs) {
            float ms = 0;
            CR_HIP(hipEventElapsedTime(&ms, r.a, r.b));
            size_t k = std::find(keys.begin(), keys.end(), std::string(r.name)) - keys.begin();
            if (k == keys.size()) {
                keys.push_back(r.name);
                cnt.push_back(0);
                tot.push_back(0.0);
            }
            cnt[k]++;
            tot[k] += ms;
        }
        *n = (int32_t)keys.size();
        for (int i = 0; i < (int)keys.size() && i < max; ++i) {
            std::strncpy(names + 32 * i, keys[i].c_str(), 31);
            names[32 * i + 31] = 0;
            counts[i] = cnt[i];
            total_ms[i] = tot[i];
        }
    });
}

// ---------------------------------------------------------------- sweep plans (graph replay)
struct cr_sweep_plan_s {
    cr_ctx ctx = nullptr;
    cr_precision prec = CR_MIXED;
    std::unique_ptr<SweepEngine> eng;
    DevBuf<double> omegas;
    int gpc = 2, lds = 0;
    std::vector<double> tune_ms;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~cr_sweep_plan_s() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

extern "C" cr_status cr_sweep_plan_create(cr_ctx ctx, int32_t nrom, const cr_rom* roms, int32_t nfreq,
                                          const double* omegas, cr_precision prec, cr_z* const* Y_dev,
                                          const cr_tune* tune, cr_sweep_plan* out) {
    if (!ctx) return CR_E_INVALID;
    return cr_guard(ctx, [&] {
        CR_REQUIRE(out && nrom > 0 && nfreq > 0 && roms && omegas && Y_dev, CR_E_INVALID, "cr_sweep_plan_create: bad arguments");
        CR_REQUIRE(prec == CR_FP64 || prec == CR_MIXED, CR_E_INVALID, "cr_sweep_plan_create: bad precision");
        hipStream_t s = ctx->stream;
        auto P = std::make_unique<cr_sweep_plan_s>();
        P->ctx = ctx;
        P->prec = prec;
        P->eng = std::make_unique<SweepEngine>();
        P->eng->num_cu = ctx->num_cu;
        P->eng->ctx = ctx;
        const size_t nw = (size_t)nrom * nfreq;
        P->omegas.alloc(nw);
        CR_HIP(hipMemcpyAsync(P->omegas.p, omegas, nw * sizeof(double), hipMemcpyHostToDevice, s));
        std::vector<RomDesc> ds(nrom);
        for (int m = 0; m < nrom; ++m) {
            CR_REQUIRE(roms[m] && roms[m]->ctx == ctx && Y_dev[m], CR_E_INVALID, "cr_sweep_plan_create: bad model");
            CR_REQUIRE(roms[m]->tmeta.empty(), CR_E_UNSUPPORTED,
                       "cr_sweep_plan_create: reduced models with frequency-dependent terms need cr_sweep");
            ds[m] = desc_of(roms[m], P->omegas.p + (size_t)m * nfreq, reinterpret_cast<zd*>(Y_dev[m]), 0);
        }
        const bool refine = prec == CR_MIXED || (tune && tune->refine);
        {
            std::vector<cr_rom_s*> hts;
            for (int m = 0; m < nrom; ++m)
                if (use_ht(roms[m], prec, refine, 0)) hts.push_back(roms[m]);
            ensure_ht(hts, s);
            for (int m = 0; m < nrom; ++m)
                if (use_ht(roms[m], prec, refine, 0)) attach_ht(roms[m], ds[m]);
        }
        std::vector<int> order(nrom);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ds[a].q > ds[b].q; });
        std::vector<int2> items;
        items.reserve(nw);
        for (int m : order)
            for (int i = 0; i < nfreq; ++i) items.push_back(make_int2(m, i));
        if (!tune || tune->variant == 0) {
            P->eng->autotune(ds, items, prec, refine, s, &P->gpc, &P->lds, &P->tune_ms);
        } else {
            P->gpc = tune->grid_per_cu > 0 ? tune->grid_per_cu : 2;
            P->lds = tune->variant == 1 ? std::max(0, tune->nb) * 1024 : 0;
        }
        P->eng->prepare(ds, items, s);
        P->eng->launch(prec, refine, P->gpc, P->lds, s);   // eager run: allocates the workspaces
        CR_HIP(hipStreamSynchronize(s));
        CR_HIP(hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking));
        const bool prof = ctx->prof.on;
        ctx->prof.on = false;
        CR_HIP(hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal));
        try {
            P->eng->launch(prec, refine, P->gpc, P->lds, P->cap);
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(P->cap, &g);
            if (g) (void)hipGraphDestroy(g);
            ctx->prof.on = prof;
            throw;
        }
        CR_HIP(hipStreamEndCapture(P->cap, &P->graph));
        ctx->prof.on = prof;
        CR_HIP(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
        *out = P.release();
    });
}

extern "C" cr_status cr_sweep_plan_execute(cr_sweep_plan plan, cr_sweep_info* info) {
    if (!plan) return CR_E_INVALID;
    return cr_guard(plan->ctx, [&] {
        const double t0 = now();
        hipStream_t s = plan->ctx->stream;
        {
            ProfScope ps(plan->ctx, "sweep_graph", s);
            CR_HIP(hipGraphLaunch(plan->exec, s));
        }
        int mi = 0, nc = 0, np = 0, fb = 0;
        plan->eng->read_stats(s, &mi, &nc, &np, &fb);
        fill_sweep_info(info, mi, nc, fb, np, now() - t0);
        CR_REQUIRE(nc == 0, CR_E_NOT_CONVERGED,
                   "cr_sweep_plan_execute: refinement did not reach its tolerance at " + std::to_string(nc) + " items");
    });
}

extern "C" cr_status cr_sweep_plan_tuning(cr_sweep_plan plan, cr_tune* chosen, double* ms, int32_t max, int32_t* n) {
    if (!plan) return CR_E_INVALID;
    if (chosen) {
        chosen->variant = plan->lds > 0 ? 1 : 0;
        chosen->grid_per_cu = plan->gpc;
        chosen->nb = plan->lds / 1024;
    }
    if (n) *n = (int32_t)plan->tune_ms.size();
    for (int i = 0; ms && i < max && i < (int)plan->tune_ms.size(); ++i) ms[i] = plan->tune_ms[i];
    return CR_OK;
}

extern "C" void cr_sweep_plan_destroy(cr_sweep_plan plan) { delete plan; }
