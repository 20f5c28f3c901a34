// Domain decomposition for the shifted solves (paper Section 3.2): GMRES preconditioned by an
// additive Schwarz sum over physics-based subdomains, each subdomain matrix factored by the
// library's multifrontal LU. The memory-lean alternative to one full factorisation per frequency:
// only the (overlapping) subdomain factors are stored.
//
//   subdomains: the structure DoFs and the fluid DoFs (the physical domains), each grown by
//               `overlap` layers of neighbours in the graph of A;
//   M^{-1} r = sum_j R~_j^T A_j^{-1} R_j r,  A_j = R_j A~ R_j^T   (restricted: R~_j writes only
//               the DoFs subdomain j owned before growing; basic: R~_j = R_j);
//   right-preconditioned GMRES(restart) in FP64 on the Jacobi-scaled system, CGS2 Arnoldi,
//               Givens rotations on the host, stop at ||b - A x|| <= tol ||b|| per column.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>

#include "internal.h"
#include "util.cuh"

namespace cr {
void gram(int64_t n, int qa, int b, const zd* A, int64_t lda, const zd* B, int64_t ldb, zd* H, int64_t ldh, int conj_t,
          DevBuf<zd>& partial, hipStream_t s);
void update(int64_t n, int q, int b, const zd* V, int64_t ldv, const zd* H, int64_t ldh, zd* W, int64_t ldw, hipStream_t s);
void copy_dev(int64_t n, const zd* src, zd* dst, hipStream_t s);
void copy_cols_scaled(int64_t n, const zd* src, zd* dst, double factor, hipStream_t s);
void scale_rows(int64_t n, int nrhs, const zd* src, const double* sc, zd* dst, hipStream_t s);
void gather_idx(int64_t m, const int32_t* idx, const zd* src, zd* dst, hipStream_t s);
void scatter_idx(int64_t m, const int32_t* pos, const int32_t* tgt, const zd* src, zd* dst, int add, hipStream_t s);
void spmm_residual(cr_sys sys, const zd* Kv, const zd* Mv, double sigma, int nrhs, const zd* X, int64_t ldx,
                   const zd* B, int64_t ldb, zd* R, int64_t ldr, hipStream_t s);
}  // namespace cr

using namespace cr;

struct cr_dd_s {
    cr_sys sys = nullptr;
    cr_dd_opts o{};
    struct Sub {
        std::unique_ptr<cr_sys_s> s;
        DevBuf<int32_t> idx;           // subdomain DoF -> global DoF
        DevBuf<int32_t> pos, tgt;      // prolongation: sub position -> global DoF (owned or all)
        int64_t nw = 0;                // prolongated entries
        Factor f;
        SolveWork w;
        DevBuf<zd> r, z;
    };
    std::vector<std::unique_ptr<Sub>> subs;
    double omega = -1;
    cr_precision prec = CR_FP64;
    int64_t sub_entries = 0;
    DevBuf<zd> partial;
};

namespace {

double now() { return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count(); }

void factor_subs(cr_dd dd, double omega, cr_precision prec) {
    if (dd->omega == omega && dd->prec == prec) return;
    for (auto& sb : dd->subs) numeric_factor(sb->f, sb->s.get(), omega, prec, dd->sys->ctx->stream);
    dd->omega = omega;
    dd->prec = prec;
}

// Z = M^{-1} R for nrhs columns (n x nrhs, leading dimension n), scaled coordinates
void precondition(cr_dd dd, int nrhs, const zd* R, zd* Z, hipStream_t s) {
    const int64_t n = dd->sys->n;
    fill_zero(Z, n * nrhs, s);
    for (auto& sb : dd->subs) {
        const int64_t m = sb->s->n;
        sb->r.reserve((size_t)m * nrhs);
        sb->z.reserve((size_t)m * nrhs);
        for (int c = 0; c < nrhs; ++c) gather_idx(m, sb->idx.p, R + n * c, sb->r.p + m * c, s);
        // exact subdomain solves (the paper applies a full LU per subdomain): FP64 refinement to a
        // backward error of 1e-14, GMRES refinement when a perturbed pivot stalls it
        double berr = 0;
        solve_scaled(sb->f, nrhs, sb->r.p, sb->z.p, 10, 1e-14, &berr, sb->w, s, false, true);
        for (int c = 0; c < nrhs; ++c) scatter_idx(sb->nw, sb->pos.p, sb->tgt.p, sb->z.p + m * c, Z + n * c, 1, s);
    }
}

double norm2(cr_dd dd, const zd* x, hipStream_t s, DevBuf<zd>& h) {
    gram(dd->sys->n, 1, 1, x, dd->sys->n, x, dd->sys->n, h.p, 1, 0, dd->partial, s);
    zd v;
    CR_HIP(hipMemcpyAsync(&v, h.p, sizeof(zd), hipMemcpyDeviceToHost, s));
    CR_HIP(hipStreamSynchronize(s));
    return std::sqrt(std::max(v.re, 0.0));
}

// one column: right-preconditioned GMRES(restart); returns iterations, sets the final relative residual
int gmres_column(cr_dd dd, const zd* b, zd* x, double* relres, hipStream_t s) {
    cr_sys sys = dd->sys;
    const int64_t n = sys->n;
    const int m = dd->o.restart;
    const double w2 = dd->omega * dd->omega;
    DevBuf<zd> V((size_t)n * (m + 1)), Zb((size_t)n * m), r(n), h((size_t)m + 2), y((size_t)m);
    fill_zero(x, n, s);
    const double bn = norm2(dd, b, s, h);
    int its = 0;
    *relres = 0;
    if (!(bn > 0)) return 0;
    std::vector<zd> hh((size_t)m + 2);
    for (;;) {
        spmm_residual(sys, sys->d_K.p, sys->d_M.p, w2, 1, x, n, b, n, r.p, n, s);
        const double beta = norm2(dd, r.p, s, h);
        *relres = beta / bn;
        if (beta <= dd->o.tol * bn || its >= dd->o.max_iter) break;
        copy_cols_scaled(n, r.p, V.p, 1.0 / beta, s);
        std::vector<std::complex<double>> H((size_t)(m + 1) * m, 0.0), g(m + 1, 0.0), sn(m);
        std::vector<double> cs(m);
        g[0] = beta;
        int k = 0;
        for (; k < m && its < dd->o.max_iter; ++k) {
            precondition(dd, 1, V.p + n * k, Zb.p + n * k, s);
            zd* wv = V.p + n * (k + 1);
            // w = A z_k  (as 0 - (0 - A z_k) with the residual kernel and a zero right-hand side)
            fill_zero(r.p, n, s);
            spmm_residual(sys, sys->d_K.p, sys->d_M.p, w2, 1, Zb.p + n * k, n, r.p, n, wv, n, s);
            // wv holds -A z_k; the sign is absorbed below by negating the Hessenberg column
            std::vector<std::complex<double>> hc(k + 2, 0.0);
            for (int pass = 0; pass < 2; ++pass) {
                gram(n, k + 1, 1, V.p, n, wv, n, h.p, k + 1, 0, dd->partial, s);
                update(n, k + 1, 1, V.p, n, h.p, k + 1, wv, n, s);
                CR_HIP(hipMemcpyAsync(hh.data(), h.p, (k + 1) * sizeof(zd), hipMemcpyDeviceToHost, s));
                CR_HIP(hipStreamSynchronize(s));
                for (int i = 0; i <= k; ++i) hc[i] -= std::complex<double>(hh[i].re, hh[i].im);
            }
            const double hn = norm2(dd, wv, s, h);
            hc[k + 1] = hn;
            if (hn > 0) copy_cols_scaled(n, wv, wv, -1.0 / hn, s);   // v_(k+1) = (A z_k - V h) / hn
            ++its;
            for (int i = 0; i < k; ++i) {
                const std::complex<double> a = hc[i], bb = hc[i + 1];
                hc[i] = cs[i] * a + sn[i] * bb;
                hc[i + 1] = -std::conj(sn[i]) * a + cs[i] * bb;
            }
            const std::complex<double> a = hc[k];
            const double rr = std::sqrt(std::norm(a) + hn * hn);
            if (rr > 0) {
                cs[k] = std::abs(a) / rr;
                const std::complex<double> ph = std::abs(a) > 0 ? a / std::abs(a) : 1.0;
                sn[k] = ph * hn / rr;
                hc[k] = ph * rr;
            } else {
                cs[k] = 1.0;
                sn[k] = 0.0;
            }
            hc[k + 1] = 0.0;
            for (int i = 0; i <= k; ++i) H[i + (size_t)k * (m + 1)] = hc[i];
            g[k + 1] = -std::conj(sn[k]) * g[k];
            g[k] = cs[k] * g[k];
            if (std::abs(g[k + 1]) <= dd->o.tol * bn || hn == 0) { ++k; break; }
        }
        // y = H^{-1} g (upper triangular k x k), x += Z y
        std::vector<std::complex<double>> yy(k);
        for (int i = k - 1; i >= 0; --i) {
            std::complex<double> acc = g[i];
            for (int c = i + 1; c < k; ++c) acc -= H[i + (size_t)c * (m + 1)] * yy[c];
            yy[i] = std::abs(H[i + (size_t)i * (m + 1)]) > 0 ? acc / H[i + (size_t)i * (m + 1)] : 0.0;
        }
        std::vector<zd> ny(k);
        for (int i = 0; i < k; ++i) ny[i] = {-yy[i].real(), -yy[i].imag()};
        if (k > 0) {
            CR_HIP(hipMemcpyAsync(y.p, ny.data(), k * sizeof(zd), hipMemcpyHostToDevice, s));
            update(n, k, 1, Zb.p, n, y.p, k, x, n, s);   // x -= Z (-y)
        }
    }
    return its;
}

}  // namespace

extern "C" {

cr_status cr_dd_create(cr_sys sys, const cr_dd_opts* o, cr_dd* out) {
    if (!sys) return CR_E_INVALID;
    return cr_guard(sys->ctx, [&] {
        CR_REQUIRE(o && out && o->overlap >= 0 && o->overlap <= 16 && o->restart >= 1 && o->restart <= 1000 &&
                       o->max_iter >= 1 && o->tol > 0,
                   CR_E_INVALID, "cr_dd_create: bad options");
        CR_REQUIRE(sys->D.empty() && sys->terms.empty(), CR_E_UNSUPPORTED,
                   "cr_dd_create: systems with a damping matrix or frequency-dependent materials are not supported");
        hipStream_t s = sys->ctx->stream;
        const int64_t n = sys->n, nu = sys->n_u;
        auto dd = std::make_unique<cr_dd_s>();
        dd->sys = sys;
        dd->o = *o;
        std::vector<std::pair<int64_t, int64_t>> ranges;
        if (nu > 0) ranges.push_back({0, nu});
        if (n > nu) ranges.push_back({nu, n});
        CR_REQUIRE(nu > 0, CR_E_UNSUPPORTED, "cr_dd_create: the physics-based split needs structure DoFs (n_u > 0)");
        for (auto [lo, hi] : ranges) {
            std::vector<char> mark(n, 0);
            for (int64_t i = lo; i < hi; ++i) mark[i] = 1;
            for (int l = 0; l < o->overlap; ++l) {
                std::vector<char> nxt = mark;
                for (int64_t r = 0; r < n; ++r)
                    if (mark[r])
                        for (int64_t k = sys->rowptr[r]; k < sys->rowptr[r + 1]; ++k) nxt[sys->col[k]] = 1;
                mark.swap(nxt);
            }
            std::vector<int32_t> idx, loc(n, -1);
            for (int64_t i = 0; i < n; ++i)
                if (mark[i]) { loc[i] = (int32_t)idx.size(); idx.push_back((int32_t)i); }
            auto sb = std::make_unique<cr_dd_s::Sub>();
            auto ss = std::make_unique<cr_sys_s>();
            ss->ctx = sys->ctx;
            ss->n = (int64_t)idx.size();
            ss->rowptr.assign(ss->n + 1, 0);
            for (size_t a = 0; a < idx.size(); ++a) {
                const int64_t r = idx[a];
                for (int64_t k = sys->rowptr[r]; k < sys->rowptr[r + 1]; ++k)
                    if (loc[sys->col[k]] >= 0) {
                        ss->col.push_back(loc[sys->col[k]]);
                        ss->K.push_back(sys->K[k]);
                        ss->M.push_back(sys->M[k]);
                    }
                ss->rowptr[a + 1] = (int64_t)ss->col.size();
            }
            if (!sys->coords.empty()) {
                ss->coords.resize(3 * idx.size());
                for (size_t a = 0; a < idx.size(); ++a)
                    for (int j = 0; j < 3; ++j) ss->coords[3 * a + j] = sys->coords[3 * (size_t)idx[a] + j];
            }
            finalize_sys(ss.get());
            ss->fclass = sys->fclass;
            ss->sym = analyse_pattern(ss->n, ss->rowptr, ss->col, ss->coords, ss->fclass);
            upload_symbolic(ss.get());
            dd->sub_entries += ss->sym->factor_entries;
            std::vector<int32_t> pos, tgt;
            for (size_t a = 0; a < idx.size(); ++a)
                if (!o->restricted || (idx[a] >= lo && idx[a] < hi)) { pos.push_back((int32_t)a); tgt.push_back(idx[a]); }
            upload(sb->idx, idx, s);
            upload(sb->pos, pos, s);
            upload(sb->tgt, tgt, s);
            sb->nw = (int64_t)pos.size();
            sb->s = std::move(ss);
            dd->subs.push_back(std::move(sb));
        }
        CR_HIP(hipStreamSynchronize(s));
        *out = dd.release();
    });
}

void cr_dd_destroy(cr_dd dd) { delete dd; }

cr_status cr_dd_solve(cr_dd dd, double omega, cr_precision sub_prec, int32_t nrhs, const cr_z* B_dev, cr_z* X_dev,
                      cr_dd_info* info) {
    if (!dd) return CR_E_INVALID;
    cr_sys sys = dd->sys;
    return cr_guard(sys->ctx, [&] {
        CR_REQUIRE(std::isfinite(omega) && (sub_prec == CR_FP64 || sub_prec == CR_MIXED) && nrhs >= 0 &&
                       (nrhs == 0 || (B_dev && X_dev)),
                   CR_E_INVALID, "cr_dd_solve: bad arguments");
        const double t0 = now();
        hipStream_t s = sys->ctx->stream;
        const int64_t n = sys->n;
        factor_subs(dd, omega, sub_prec);
        DevBuf<zd> Bs((size_t)n * std::max(nrhs, 1)), Xs((size_t)n * std::max(nrhs, 1));
        if (nrhs) scale_rows(n, nrhs, reinterpret_cast<const zd*>(B_dev), sys->d_scale.p, Bs.p, s);
        int itmax = 0;
        double worst = 0;
        for (int c = 0; c < nrhs; ++c) {
            double rr = 0;
            itmax = std::max(itmax, gmres_column(dd, Bs.p + n * c, Xs.p + n * c, &rr, s));
            worst = std::max(worst, rr);
        }
        if (nrhs) scale_rows(n, nrhs, Xs.p, sys->d_scale.p, reinterpret_cast<zd*>(X_dev), s);
        CR_HIP(hipStreamSynchronize(s));
        if (info) {
            info->iterations = itmax;
            info->rel_residual = worst;
            info->n_sub = (int32_t)dd->subs.size();
            info->sub_factor_entries = dd->sub_entries;
            info->seconds = now() - t0;
        }
        CR_REQUIRE(!(worst > dd->o.tol), CR_E_NOT_CONVERGED,
                   "cr_dd_solve: GMRES stopped at relative residual " + std::to_string(worst));
    });
}

cr_status cr_dd_precondition(cr_dd dd, double omega, cr_precision sub_prec, int32_t nrhs, const cr_z* R_dev,
                             cr_z* Z_dev) {
    if (!dd) return CR_E_INVALID;
    cr_sys sys = dd->sys;
    return cr_guard(sys->ctx, [&] {
        CR_REQUIRE(std::isfinite(omega) && (sub_prec == CR_FP64 || sub_prec == CR_MIXED) && nrhs >= 0 &&
                       (nrhs == 0 || (R_dev && Z_dev)),
                   CR_E_INVALID, "cr_dd_precondition: bad arguments");
        factor_subs(dd, omega, sub_prec);
        precondition(dd, nrhs, reinterpret_cast<const zd*>(R_dev), reinterpret_cast<zd*>(Z_dev), sys->ctx->stream);
        CR_HIP(hipStreamSynchronize(sys->ctx->stream));
    });
}

}  // extern "C"
