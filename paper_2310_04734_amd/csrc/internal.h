// Internal declarations shared by the library's translation units (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/cabinrom.h"

namespace cr {

// ------------------------------------------------------------------------- errors
struct Error : std::runtime_error {
    cr_status code;
    Error(cr_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define CR_HIP(call)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            throw ::cr::Error(CR_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define CR_REQUIRE(cond, code, msg)                        \
    do {                                                   \
        if (!(cond)) throw ::cr::Error((code), (msg));     \
    } while (0)

// ------------------------------------------------------------------------- device buffers
// Allocator of the context whose API call is running on this thread (set by cr_guard), or null
// for hipMalloc / hipFree. A buffer remembers the allocator that produced it and frees through it.
extern thread_local const cr_allocator* tl_alloc;

// Owning device allocation; movable, not copyable.
template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    const cr_allocator* al = nullptr;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), al(o.al) { o.p = nullptr; o.n = 0; o.al = nullptr; }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; al = o.al; o.p = nullptr; o.n = 0; o.al = nullptr; }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (count == 0) return;
        const size_t bytes = count * sizeof(T);
        if (tl_alloc) {
            void* q = tl_alloc->alloc(bytes, tl_alloc->user);
            if (!q) throw Error(CR_E_OOM, "the context's allocator returned no memory for " + std::to_string(bytes) + " bytes");
            p = static_cast<T*>(q);
            al = tl_alloc;
        } else {
            hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), bytes);
            if (e != hipSuccess) {
                p = nullptr;
                (void)hipGetLastError();
                throw Error(CR_E_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
            }
            al = nullptr;
        }
        n = count;
    }
    // grow (contents not preserved) when smaller than count
    void reserve(size_t count) { if (count > n) alloc(count); }
    void release() {
        if (p) {
            if (al) al->free(p, al->user);
            else (void)hipFree(p);
        }
        p = nullptr;
        n = 0;
        al = nullptr;
    }
    size_t bytes() const { return n * sizeof(T); }
};

template <typename T>
void upload(DevBuf<T>& d, const std::vector<T>& h, hipStream_t s) {
    d.alloc(h.size());
    if (!h.empty()) CR_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// ------------------------------------------------------------------------- complex helpers
struct zd { double re, im; };   // host/device complex128 storage
struct zf { float re, im; };    // complex64 storage

// ------------------------------------------------------------------------- analysis
struct Symbolic {
    int64_t n = 0;
    std::vector<int32_t> perm;     // new -> old
    std::vector<int32_t> iperm;    // old -> new
    // fronts in postorder (children before parents)
    int32_t nfront = 0;
    std::vector<int32_t> first;    // first pivot (new index)
    std::vector<int32_t> npiv;
    std::vector<int32_t> fsize;    // m = npiv + ncb
    std::vector<int64_t> idx_off;  // offset of the front's row index list (length m) in idx
    std::vector<int32_t> idx;      // new indices: pivots then contribution rows (sorted)
    std::vector<int32_t> parent;   // -1 for roots
    std::vector<int32_t> child_off, child_list;  // CSR of children
    std::vector<int32_t> level;    // 0 = leaves ... height
    int32_t nlevel = 0;
    std::vector<int32_t> level_off, level_fronts;  // fronts grouped by level
    std::vector<int64_t> front_off;  // offset (complex entries) of front f in the arena
    int64_t arena = 0;               // total complex entries
    std::vector<int64_t> piv_off;    // = first[f] (pivot rows are globally numbered)
    // child contribution -> parent local index maps (int32 per child CB row)
    std::vector<int64_t> cmap_off;   // per front (as child): offset into cmap, length ncb
    std::vector<int32_t> cmap;
    // original-entry scatter: per front, list of (csr position, local row, local col)
    std::vector<int64_t> ent_off;    // per front
    std::vector<int64_t> ent_src;    // csr position
    std::vector<int32_t> ent_dst;    // local row + local col * m (fits: m^2 < 2^31)
    int32_t max_front = 0, max_piv = 0, max_children = 0;
    // large fronts are factored panel by panel with the trailing updates spread over many
    // workgroups: per level the list of large fronts and the number of 16-column panel steps
    std::vector<int32_t> big;                  // per front: 1 = large
    std::vector<int32_t> big_off, big_list;    // per level
    std::vector<int32_t> nsteps;               // per level
    // the largest fronts are solved block by block with the rows spread over many workgroups
    std::vector<int32_t> huge;                 // per front: 1 = multi-workgroup solve
    std::vector<int32_t> huge_off, huge_list;  // per level
    std::vector<int32_t> huge_piv;             // per level: max pivots of its huge fronts
    std::vector<int32_t> wide_solve;           // per level: 1024-thread solve workgroups (bit 0: multi-RHS, bit 1: one RHS)
    int64_t factor_entries = 0;
    double factor_flops = 0;
    double gemm_flops = 0;         // trailing-GEMM part of factor_flops (large fronts)
    double seconds = 0;
};

// Device copy of the symbolic data used by the numeric kernels.
struct DevSymbolic {
    DevBuf<int32_t> first, npiv, fsize, parent, child_off, child_list, level_fronts, idx, cmap, ent_dst;
    DevBuf<int64_t> idx_off, front_off, cmap_off, ent_off, ent_src;
    DevBuf<int32_t> perm, iperm;
    DevBuf<int32_t> big, big_list, huge, huge_list;
};

// A frequency-dependent part of K(w) or M(w): a material whose loss factor follows a table.
// kind 0 (solid stiffness with real E): contributes (1 + i eta(f)) T to K(w);
// kind 1 (fluid mass int N^T N):         contributes T / (c^2 (1 + i eta(f))) to M(w).
struct TermMeta {
    int kind = 0;
    double c = 0;
    std::vector<double> f_hz, eta;
    double eta_at(double f) const {
        if (f <= f_hz.front()) return eta.front();
        if (f >= f_hz.back()) return eta.back();
        size_t k = 1;
        while (f_hz[k] < f) ++k;
        const double t = (f - f_hz[k - 1]) / (f_hz[k] - f_hz[k - 1]);
        return eta[k - 1] + t * (eta[k] - eta[k - 1]);
    }
    // coefficient of the term in K(w) (kind 0) or in M(w) (kind 1) at angular frequency w
    zd coef(double omega) const {
        const double e = eta_at(omega / (2.0 * 3.14159265358979323846));
        if (kind == 0) return {1.0, e};
        const double d = c * c * (1.0 + e * e);   // 1 / (c^2 (1 + i e)) = (1 - i e) / (c^2 (1 + e^2))
        return {1.0 / d, -e / d};
    }
};
struct FreqTerm : TermMeta {
    std::vector<zd> vals;   // host, unscaled, on the system's pattern
    DevBuf<zd> d_vals;      // device, Jacobi-scaled
};
constexpr int kMaxTerms = 4;

// scale, scaled device copies and norms of a freshly assembled or imported system
void finalize_sys(cr_sys sys);

// size thresholds of the front classes: m >= big_m factored with many workgroups, m >= huge_m
// solved with many workgroups
struct FrontClasses {
    int32_t big_m = 192, huge_m = 1024;
    int32_t split_rows = 1024;   // panels with this many fully-summed rows use several workgroups (0: never)
    int32_t split_polls = 0;     // bound on a split panel's barrier polls (0: the default, about a second)
};

std::unique_ptr<Symbolic> analyse_pattern(int64_t n, const std::vector<int64_t>& rowptr,
                                          const std::vector<int32_t>& col,
                                          const std::vector<double>& coords /* n*3 or empty */,
                                          const FrontClasses& fc);

}  // namespace cr

// ------------------------------------------------------------------------- handles
namespace cr {
struct SweepEngine;

// Event-bracketed kernel timing (off unless enabled through cr_profile_enable).
struct Profiler {
    bool on = false;
    std::vector<std::string> only;   // kernel names to time (empty: all)
    bool wants(const char* name) const {
        if (only.empty()) return true;
        for (const auto& o : only)
            if (o == name) return true;
        return false;
    }
    struct Rec {
        const char* name;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t take() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void clear() {
        for (auto& r : recs) { pool.push_back(r.a); pool.push_back(r.b); }
        recs.clear();
    }
    ~Profiler() {
        clear();
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};
}  // namespace cr

struct cr_ctx_s {
    int device = 0;
    bool has_alloc = false;
    cr_allocator alloc{};               // device-memory hook (has_alloc)
    hipStream_t stream = nullptr;
    std::string err;
    int num_cu = 256;
    cr::SweepEngine* sweep = nullptr;   // persistent sweep workspaces (owned)
    cr::Profiler prof;
    // second stream (default priority) for work that overlaps the library stream, with the
    // events that order the two; created on first use, owned
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

namespace cr {
// the context's second stream and its fork / join events, created on first use
inline hipStream_t aux_stream(cr_ctx_s* ctx) {
    if (!ctx->aux) {
        CR_HIP(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
        CR_HIP(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
        CR_HIP(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
    }
    return ctx->aux;
}

// RAII bracket of one kernel launch (no-op while profiling is off)
struct ProfScope {
    cr_ctx_s* ctx;
    hipStream_t s;
    const char* name;
    hipEvent_t a = nullptr;
    ProfScope(cr_ctx_s* c, const char* n, hipStream_t st) : ctx(c), s(st), name(n) {
        if (ctx && ctx->prof.on && ctx->prof.wants(name)) {
            a = ctx->prof.take();
            if (a) (void)hipEventRecord(a, s);
        }
    }
    ~ProfScope() {
        if (a) {
            hipEvent_t b = ctx->prof.take();
            if (b) {
                (void)hipEventRecord(b, s);
                ctx->prof.recs.push_back({name, a, b});
            }
        }
    }
};
}  // namespace cr

struct cr_sys_s {
    cr_ctx ctx = nullptr;
    int64_t n = 0, n_u = 0;
    int32_t L = 0, n_o = 0;
    // host, unscaled
    std::vector<int64_t> rowptr;
    std::vector<int32_t> col;
    std::vector<cr::zd> K, M, F;   // F: n x L column-major
    std::vector<cr::zd> D;         // viscous damping on the same pattern, or empty (D = 0)
    std::vector<cr::FreqTerm> terms;   // frequency-dependent parts of K(w), M(w) (K, M hold the rest)
    std::vector<int32_t> flags;
    std::vector<int64_t> recv;
    std::vector<double> coords;    // n x 3 DoF coordinates (for nested dissection)
    std::vector<double> scale;     // S = |K_ii|^{-1/2}
    double anorm_inf = 0;          // max over rows of sum |K~| (scaled) for backward errors
    double mnorm_inf = 0;          // same for M~
    // device, scaled
    cr::DevBuf<int64_t> d_rowptr;
    cr::DevBuf<int32_t> d_col;
    cr::DevBuf<cr::zd> d_K, d_M, d_F, d_D;
    cr::DevBuf<double> d_scale;
    cr::DevBuf<int64_t> d_recv;
    cr::DevBuf<int32_t> d_flags;
    // analysis
    cr::FrontClasses fclass;
    std::unique_ptr<cr::Symbolic> sym;
    std::unique_ptr<cr::DevSymbolic> dsym;
};

namespace cr {

// ------------------------------------------------------------------------- factor internals
struct Factor {
    cr_sys sys = nullptr;
    double omega = 0;
    cr_precision prec = CR_FP64;
    DevBuf<zd> arena64;   // complex128 fronts (FP64)
    DevBuf<zf> arena32;   // complex64 fronts (MIXED)
    DevBuf<int32_t> ipiv; // local pivot row per pivot (n)
    DevBuf<int32_t> psrc; // per pivot: source row of the front's composed swaps (n)
    DevBuf<int32_t> nperturb;   // [0] perturbed pivots, [1] a split panel's barrier wait failed
    DevBuf<unsigned long long> amax;
    DevBuf<double> coop_pub;    // split panels: pivot candidates and rows published per front slot
    DevBuf<int32_t> coop_bar;   // split panels: barrier counters per front slot
    int32_t n_perturbed = 0;
    double anorm = 0, anorm_omega = -1;   // ||A~||_inf at the factored shift
    // the shifted operator A~ = opK - opS opM on the system's pattern: (K~, M~, w^2), or for a
    // system with damping the pre-formed values aval = K~ + i w D~ - w^2 M~ with (aval, aval, 0)
    DevBuf<zd> aval;
    const zd* opA = nullptr;   // A~ pre-formed (FP64): the refinement residual reads 20 B per entry
    const zd* opK = nullptr;
    const zd* opM = nullptr;
    double opS = 0;
    // M(w_j) for the Krylov recurrence: M~, or pre-formed with the frequency-dependent terms
    DevBuf<zd> mval;
    const zd* opMass = nullptr;
};

void upload_symbolic(cr_sys sys);
// X (+)= A~^{-1} B with the stored factor (FP64 in and out, old numbering)
void apply_factor(const Factor& f, int nrhs, const zd* B, int64_t ldb, zd* X, int64_t ldx, int add,
                  struct SolveWork& w, hipStream_t s);

// numeric factorisation into an existing Factor (arena reused when large enough)
void numeric_factor(Factor& f, cr_sys sys, double omega, cr_precision prec, hipStream_t s);

// workspace for solves
struct SolveWork {
    DevBuf<zd> w64;    // front work vectors (arena of sum m * nrhs), FP64 solve
    DevBuf<zf> w32;    // same, FP32 solve
    DevBuf<zd> xperm;  // permuted RHS / solution n x nrhs
    DevBuf<zd> r;      // operator products n x nrhs
    DevBuf<zd> res;    // refinement residual n x nrhs
    DevBuf<zd> d;      // correction n x nrhs
    DevBuf<zd> kry;    // GMRES bases (m + 1) x n x nrhs
    DevBuf<unsigned long long> sc;
    DevBuf<double> red;  // reduction scratch
    std::vector<double> hred;
};

// Solve A~ X = B for the scaled system (device, n x nrhs, ld n) with FP64 refinement.
// Returns iterations; sets backward error. Throws CR_E_NOT_CONVERGED only when `strict`.
int solve_scaled(Factor& f, int nrhs, const zd* B, zd* X, int max_iter, double tol, double* berr,
                 SolveWork& w, hipStream_t s, bool strict, bool allow_krylov = true);


// Greedy hook: the network's proposed next candidate (-1 when it proposes none); residuals res
// of every candidate, candidates already used, geometry features (or null).
int mlp_propose(cr_mlp m, const std::vector<double>& res, const std::vector<int>& used, const double* geom);

// y = (Kv - sigma Mv) x with values Kv, Mv on the system's pattern (or two outputs Kx, Mx) on the
// device, FP64 CSR.
void spmm_shifted(cr_sys sys, const zd* Kv, const zd* Mv, double sigma, int nrhs, const zd* X, int64_t ldx, zd* Y,
                  int64_t ldy, hipStream_t s);
void spmm_km(cr_sys sys, int nrhs, const zd* X, int64_t ldx, zd* KX, zd* MX, int64_t ldy, hipStream_t s);
void spmm_m(cr_sys sys, int nrhs, const zd* X, int64_t ldx, zd* Y, int64_t ldy, hipStream_t s);

}  // namespace cr

// Run `body`, converting exceptions to a status and ctx->err.
template <typename F>
static inline cr_status cr_guard(cr_ctx ctx, F&& body) {
    struct AllocScope {
        const cr_allocator* prev;
        explicit AllocScope(const cr_allocator* a) : prev(cr::tl_alloc) { cr::tl_alloc = a; }
        ~AllocScope() { cr::tl_alloc = prev; }
    } scope(ctx && ctx->has_alloc ? &ctx->alloc : nullptr);
    try {
        if (ctx) ctx->err.clear();
        body();
        return CR_OK;
    } catch (const cr::Error& e) {
        if (ctx) ctx->err = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        if (ctx) ctx->err = "host allocation failed";
        return CR_E_OOM;
    } catch (const std::exception& e) {
        if (ctx) ctx->err = e.what();
        return CR_E_INVALID;
    }
}
