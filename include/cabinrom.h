/*
 * cabinrom: rational-Arnoldi model-order reduction of the coupled structural-acoustic (u-p)
 * finite-element system, and its frequency sweep, on one AMD Instinct MI355X (gfx950).
 *
 * The full-order model is the paper's problem statement (Section 3.3, Eq. (8)) with damping
 * carried by complex stiffness (text after Eq. (8)), so D = 0:
 *
 *     (K - w^2 M) x(w) = f(w),   y(w) = C^T x(w)
 *
 * with the block structure of Section 2, Eq. (2)-(3) (two domains: structure u, fluid p):
 *
 *     K = [ K_s  -C  ]      M = [ M_s        0   ]
 *         [ 0    K_f ]          [ rho0 C^T   M_f ]
 *
 * The reduced model (Section 3.3, Eq. (10)-(11)) is the Galerkin projection onto the rational
 * Krylov space  U_j K_{k_j}(A_j^{-1} M, A_j^{-1} F),  A_j = K - w_j^2 M.
 *
 * Conventions for every entry point:
 *  - Angular frequencies w are in rad/s. Time convention e^{+i w t}.
 *  - Complex numbers are cr_z {re, im} (layout-compatible with C99 double _Complex and
 *    numpy.complex128). Dense arrays are column-major.
 *  - Pointers named *_dev are device pointers on the context's device, owned by the caller.
 *    Every other pointer is a host pointer, borrowed for the duration of the call and copied.
 *  - Handles (cr_ctx, cr_sys, cr_fact, cr_basis, cr_rom, cr_mlp) are owned by the library and
 *    released by the matching *_destroy. A cr_fact or cr_basis must be destroyed before the
 *    cr_sys it was made from; a cr_sys before its cr_ctx.
 *  - All device work is enqueued on the stream given to cr_ctx_create; every call returns after
 *    that stream has completed the call's work.
 *  - Errors: every call returns a cr_status. On failure the outputs are left untouched (unless
 *    stated otherwise) and cr_last_error(ctx) holds a message until the next call on that ctx.
 *  - Global DoF order: displacement DoFs (x, y, z) of every non-clamped solid node in
 *    increasing node id, then the pressure DoF of every fluid node in increasing node id.
 *  - Loads: column l of F is the load direction; the load at frequency w is
 *    f_l(w) = (i w)^flags[l] * F[:, l].
 */
#ifndef CABINROM_H
#define CABINROM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CR_OK = 0,
    CR_E_INVALID = -1,        /* bad argument (null pointer, size out of range, wrong state) */
    CR_E_OOM = -2,            /* device or host allocation failed */
    CR_E_HIP = -3,            /* a HIP runtime call failed */
    CR_E_SINGULAR = -4,       /* the shifted matrix has no nonzero entry (or a non-finite one), so
                                 no pivot can be perturbed */
    CR_E_NOT_CONVERGED = -5,  /* iterative refinement did not reach its tolerance */
    CR_E_UNSUPPORTED = -6,    /* input outside what this build supports */
    CR_E_STATE = -7           /* call order violated (e.g. factor before analyse) */
} cr_status;

typedef enum {
    CR_FP64 = 0,   /* plain method: complex-FP64 factorisation and solves */
    CR_MIXED = 1   /* complex-FP32 factorisation / reduced LU, FP64 iterative refinement */
} cr_precision;

typedef struct { double re, im; } cr_z;

typedef struct cr_ctx_s* cr_ctx;
typedef struct cr_sys_s* cr_sys;
typedef struct cr_fact_s* cr_fact;
typedef struct cr_basis_s* cr_basis;
typedef struct cr_rom_s* cr_rom;
typedef struct cr_mlp_s* cr_mlp;

/* ---------------------------------------------------------------- context ---------------- */

/* Device-memory hook: every device buffer the library allocates for work on a context comes
   from alloc(bytes, user) and goes back through free(p, user) (the pointer alloc returned, on the
   same device; free may be called after the call that allocated returned, e.g. from a
   *_destroy). alloc returning NULL makes the call fail with CR_E_OOM. The struct is copied. */
typedef struct {
    void* (*alloc)(size_t bytes, void* user);
    void (*free)(void* p, void* user);
    void* user;
} cr_allocator;

/* Bind to HIP device `device` and stream `hip_stream` (a hipStream_t; NULL = the null stream).
   allocator: NULL = hipMalloc / hipFree. Also sets up the device's static sweep scratch
   (cr_sweep_noalloc). */
cr_status cr_ctx_create(int device, void* hip_stream, const cr_allocator* allocator, cr_ctx* out);
void cr_ctx_destroy(cr_ctx ctx);
/* Message of the last failed call on ctx ("" if none). Valid until the next call on ctx. */
const char* cr_last_error(cr_ctx ctx);
/* Message of the last failed cr_ctx_create in this process. */
const char* cr_create_error(void);

/* Kernel timing: when enabled, every launch of the library's hot kernels on ctx is bracketed
   by HIP events on the context stream. cr_profile_enable clears the records. cr_profile_read
   synchronises the stream and aggregates by kernel name: up to max entries, names as
   NUL-terminated strings of at most 31 characters in names[32 * i]; counts[i] launches;
   total_ms[i] summed event durations; *n receives the number of distinct names. */
cr_status cr_profile_enable(cr_ctx ctx, int32_t on);
cr_status cr_profile_read(cr_ctx ctx, int32_t max, char* names, int32_t* counts, double* total_ms, int32_t* n);
/* Restricts the timing to the kernels named in names (comma-separated, e.g. "front_bwd,front_gemm";
   NULL or "" times every hot kernel again), so that a timed run carries events only around the
   launches it reports. Takes effect for launches after the call; the records are kept. Host
   string, copied. */
cr_status cr_profile_select(cr_ctx ctx, const char* names);

/* Achievable-peak probes for the rooflines (measurement support, not part of the method).
   cr_probe_copy: a streaming device-to-device copy of `bytes` (a multiple of 16) through a plain
   kernel, reps times after one warm-up; *gbs = bytes read + written per second. cr_probe_mfma:
   back-to-back 16x16x4 MFMA instructions (complex-free, FP64 for CR_FP64, FP32 for CR_MIXED) on 8
   workgroups per compute unit, reps launches after one warm-up; *tflops = flops per second.
   Both allocate their own device buffers and synchronise the context stream. */
cr_status cr_probe_copy(cr_ctx ctx, int64_t bytes, int32_t reps, double* gbs);
cr_status cr_probe_mfma(cr_ctx ctx, cr_precision prec, int32_t reps, double* tflops);

/* ---------------------------------------------------------------- assembly (Section 2) --- */

enum { CR_FLUID = 0, CR_SOLID = 1 };
enum { CR_LOAD_VOLUME_VELOCITY = 0, CR_LOAD_POINT_FORCE = 1, CR_LOAD_SKIN_PRESSURE = 2 };

/* Material: fluid {rho, eta, c} with c~^2 = c^2 (1 + i eta); solid {rho, eta, E, nu} with
   E~ = E (1 + i eta) (complex stiffness, Section 3.3 after Eq. (8)).
   Frequency-dependent loss factor (Section 3.3, text after Eq. (8): K(w) = K^ (1 + i eta(w))):
   with n_eta > 0, eta(f) is the piecewise-linear interpolant of (eta_f_hz[i], eta_val[i]) (f in Hz,
   increasing; constant beyond the ends) and eta is ignored. A solid's stiffness is then kept as a
   separate term K_m with coefficient 1 + i eta(f), a fluid's mass int N^T N as a term with
   coefficient 1 / (c^2 (1 + i eta(f))); at most 4 such materials. Systems with such terms take
   fixed expansion points (cr_basis_build, each point factoring A(w_j) = K(w_j) - w_j^2 M(w_j) and
   applying M(w_j) in Eq. (10)); their reduced model keeps V^H K_m V per term and forms
   K_R(w) = V^H K(w) V, M_R(w) = V^H M(w) V exactly at every swept frequency (the reduced system
   after Eq. (10)). */
typedef struct {
    int32_t kind;
    double rho, eta, c, E, nu;
    int32_t n_eta;
    const double* eta_f_hz;
    const double* eta_val;
} cr_material;

/* hex8 mesh. coords: n_nodes x 3 (row-major); elems: n_el x 8 node ids in the order
   (-,-,-) (+,-,-) (+,+,-) (-,+,-) (-,-,+) (+,-,+) (+,+,+) (-,+,+) of natural coordinates;
   elem_mat: material index per element; clamped: nodes whose displacements are fixed;
   iface: n_iface x 4 node ids of fluid-solid faces, ordered so that (x1-x0) x (x3-x0) points
   out of the fluid. Nodes on the interface are shared by the fluid and the solid elements. */
typedef struct {
    int64_t n_nodes;
    const double* coords;
    int64_t n_el;
    const int64_t* elems;
    const int32_t* elem_mat;
    int64_t n_clamped;
    const int64_t* clamped;
    int64_t n_iface;
    const int64_t* iface;
} cr_mesh;

/* One load column. VOLUME_VELOCITY: Q = value at fluid `node` (F = rho0 Q e_p(node), flag 1).
   POINT_FORCE: value along axis `dir` at solid `node` (flag 0). SKIN_PRESSURE: nodal pressure
   amplitudes amp[n_nodes] interpolated bilinearly on faces[n_faces x 4] whose right-hand
   normal points away from the structure; F = -int N^T p n dGamma (flag 0). */
typedef struct {
    int32_t kind;
    int32_t dir;
    int64_t node;
    cr_z value;
    int64_t n_faces;
    const int64_t* faces;
    const cr_z* amp;
} cr_load;

/* Assemble K, M (complex FP64 CSR), F and the receiver map (pressure DoFs of recv_nodes) on the
   host (hex8, 2x2x2 Gauss; interface quads 2x2 Gauss), then upload the Jacobi-scaled system
   S K S, S M S, S F with S = diag(|K_ii|^{-1/2}) to the device. Exactly one fluid material. */
cr_status cr_assemble(cr_ctx ctx, const cr_mesh* mesh, const cr_material* mats, int32_t nmat,
                      const cr_load* loads, int32_t nload, const int64_t* recv_nodes, int32_t n_o,
                      cr_sys* out);

typedef struct { int64_t n, nnz, n_u; int32_t L, n_o; } cr_sys_dims;
cr_status cr_sys_get_dims(cr_sys sys, cr_sys_dims* out);
/* Copy the unscaled assembled system to host arrays (rowptr n+1, col nnz, K nnz, M nnz,
   F n x L, flags L, recv_dofs n_o). Any pointer may be NULL to skip that array. */
cr_status cr_sys_export(cr_sys sys, int64_t* rowptr, int32_t* col, cr_z* K, cr_z* M, cr_z* F,
                        int32_t* flags, int64_t* recv_dofs);
void cr_sys_destroy(cr_sys sys);

/* A system given directly as matrices of the problem statement (Section 3.3, Eq. (8): (K + i w D -
   w^2 M) x = f(w), y = C^T x), for models assembled elsewhere. CSR with 0-based int64 row pointers
   (rowptr[n + 1]) and int32 columns; K, D, M are complex128 values on that one pattern (D may be
   NULL: D = 0, damping carried by complex K). Duplicate entries are summed, columns need not be
   sorted, and the pattern is completed to a structurally symmetric one with explicit zeros (the
   multifrontal analysis needs it). F: n x L column-major, flags[L] (load column l is
   F[:, l] (i w)^flags[l]), recv_dofs[n_o]: the DoFs y reads (C = unit columns). coords: n x 3
   DoF positions for the nested dissection, or NULL (graph bisection by breadth-first levels).
   Every diagonal entry of K must be nonzero (the library scales by |K_ii|^{-1/2}). All arrays are
   host arrays, copied. n_u of the result is 0. Errors: CR_E_INVALID for out-of-range indices,
   non-finite values, a zero diagonal or n, L, n_o out of range. */
cr_status cr_sys_import_csr(cr_ctx ctx, int64_t n, const int64_t* rowptr, const int32_t* col, const cr_z* K,
                            const cr_z* D, const cr_z* M, int32_t L, const cr_z* F, const int32_t* flags,
                            int32_t n_o, const int64_t* recv_dofs, const double* coords, cr_sys* out);

/* ---------------------------------------------------------------- analysis --------------- */

typedef struct {
    int32_t n_fronts, n_levels, max_front, max_pivots;
    int64_t factor_entries;   /* stored L + U entries (complex)                           */
    double factor_flops;      /* real flops of one numeric factorisation (complex, 4M)    */
    double gemm_flops;        /* the part of factor_flops done by the trailing GEMMs of the
                                 large fronts (on the matrix cores)                        */
    double seconds;
} cr_analysis_info;

/* Symbolic analysis, once per sparsity pattern (the paper reuses its analysis across
   frequencies, Section 3.2): nested dissection by coordinate bisection with vertex separators,
   assembly tree, front index maps. Idempotent. */
cr_status cr_analyse(cr_sys sys, cr_analysis_info* info);

/* Front classes used by the numeric kernels, set before cr_analyse (CR_E_STATE after): fronts of
   order m >= big_m (default 192, >= 32) are factored by 16-column panels with their updates spread
   over many workgroups and the trailing update as a complex GEMM on the matrix cores; fronts with
   m >= huge_m (default 1024, >= 64) are solved 64 pivots at a time with their rows spread over
   many workgroups. Smaller fronts are factored and solved by one workgroup each. The classes
   change the schedule, not the arithmetic's definition (same pivots up to rounding). */
cr_status cr_set_front_classes(cr_sys sys, int32_t big_m, int32_t huge_m);

/* Panel split of the large fronts, any time before cr_factor: a 16-column panel with at least
   min_rows fully-summed rows at or below it (default 1024; 0 = never, else >= 512) is factored
   by ceil(rows / 256) workgroups, at most 64 per front and 256 per launch, that keep its rows in
   registers and meet at a device-wide barrier per column; otherwise one workgroup per front
   streams the panel. Same pivots and the same operations in the same order: the factor is
   bit-identical either way. Every barrier wait is bounded by max_polls polls of the barrier word
   (0 = the default, 2^20 polls, about a second): a wait that runs out ends its workgroup, the
   split panels of that factorisation are skipped, and cr_factor fails with CR_E_HIP (the factor
   is not used; the next cr_factor starts afresh). A small max_polls forces that path for tests.
   CR_E_INVALID for 0 < min_rows < 512 or max_polls < 0. */
cr_status cr_set_panel_split(cr_sys sys, int32_t min_rows, int32_t max_polls);

/* ---------------------------------------------------------------- factor / solve --------- */

typedef struct { int32_t n_perturbed; double seconds; } cr_factor_info;

/* Multifrontal LU of A(w) = K + i w D - w^2 M (Section 3.3, Eq. (8); D = 0 unless the system was
   imported with one) at omega (rad/s), in complex FP64 (CR_FP64) or complex FP32 (CR_MIXED),
   partial pivoting inside each front's fully-summed block; pivots below 1e-8 max|A| (FP64) or
   3e-4 max|A| (FP32) are perturbed to that size (counted in info) and repaired by the FP64
   refinement of cr_solve. The factor is kept on the device and reused by every solve at this
   expansion point (Section 3.3, offline phase). Requires cr_analyse. CR_E_SINGULAR when A(w) has
   no nonzero entry. */
cr_status cr_factor(cr_sys sys, double omega, cr_precision prec, cr_fact* out, cr_factor_info* info);
void cr_fact_destroy(cr_fact f);

typedef struct { int32_t max_iter; double tol; } cr_ir_opts;   /* defaults: 10, 1e-14 */
typedef struct { int32_t iterations; double backward_error; } cr_solve_info;

/* Solve A X = B for nrhs columns (n x nrhs, leading dimension n, device, complex128), with FP64
   iterative refinement: R = B - A X in FP64, D = LU^{-1} R, X += D, until the normwise backward
   error max_l ||r_l|| / (||A||_inf ||x_l|| + ||b_l||) <= tol. CR_E_NOT_CONVERGED if max_iter
   corrections do not reach tol (X then holds the last iterate). */
cr_status cr_solve(cr_fact f, int32_t nrhs, const cr_z* B_dev, cr_z* X_dev, const cr_ir_opts* opts,
                   cr_solve_info* info);

/* ---------------------------------------------------------------- domain decomposition -- */

/* Iterative shifted solves by domain decomposition (Section 3.2): GMRES with an additive Schwarz
   preconditioner M^{-1} = sum_j R~_j^T A_j^{-1} R_j (Section 3.2) over physics-based subdomains
   (the structure DoFs and the fluid DoFs, as the paper splits by physical domain), each grown by
   `overlap` layers of neighbours in the graph of A; A_j = R_j A R_j^T is factored by the
   multifrontal LU of cr_factor (only the subdomain factors are stored: sub_factor_entries against
   the full factor's cr_analysis_info.factor_entries). restricted = 1: R~_j writes only the DoFs
   subdomain j owned before growing (restricted additive Schwarz), 0: R~_j = R_j; overlap 0 is
   block Jacobi. Right-preconditioned GMRES(restart) in FP64 on the Jacobi-scaled system, one
   Krylov space per right-hand side, CGS2 Arnoldi, stop when ||b - A x|| <= tol ||b|| (scaled
   2-norms) or after max_iter iterations. Plain systems only (CR_E_UNSUPPORTED with a damping
   matrix or frequency-dependent materials, or without structure DoFs). */
typedef struct cr_dd_s* cr_dd;
typedef struct { int32_t overlap, restricted, restart, max_iter; double tol; } cr_dd_opts;
typedef struct {
    int32_t iterations;        /* largest over the right-hand sides                          */
    double rel_residual;       /* largest final ||b - A x|| / ||b|| (scaled)                  */
    int32_t n_sub;
    int64_t sub_factor_entries;
    double seconds;
} cr_dd_info;

/* Subdomains and their symbolic analyses (once per system). */
cr_status cr_dd_create(cr_sys sys, const cr_dd_opts* opts, cr_dd* out);
void cr_dd_destroy(cr_dd dd);
/* Solve A(w) X = B (n x nrhs device arrays, leading dimension n, unscaled DoFs as cr_solve):
   factors the subdomains at omega in sub_prec (kept for the next call at the same omega), then
   GMRES. CR_E_NOT_CONVERGED when a column misses tol (X holds the last iterate, info filled). */
cr_status cr_dd_solve(cr_dd dd, double omega, cr_precision sub_prec, int32_t nrhs, const cr_z* B_dev, cr_z* X_dev,
                      cr_dd_info* info);
/* Z = M^{-1} R in the scaled coordinates of the system (for checks of the preconditioner). */
cr_status cr_dd_precondition(cr_dd dd, double omega, cr_precision sub_prec, int32_t nrhs, const cr_z* R_dev,
                             cr_z* Z_dev);

/* ---------------------------------------------------------------- basis / projection ----- */

typedef struct {
    int32_t q;                 /* basis columns kept                                       */
    int32_t deflated;          /* columns dropped by the 1e-10 norm-ratio rule             */
    int32_t n_shifts;
    int32_t ir_iterations;     /* total refinement corrections over all solves             */
    double max_backward_error; /* over all shifted solves; each is refined in FP64 until its
                                  normwise backward error is <= max(1e-14, sqrt(n) eps), the
                                  stopping rule of LAPACK's mixed-precision solver          */
    int32_t n_perturbed;
    int32_t fp64_refactorizations; /* CR_MIXED expansion points refactored in complex FP64
                                      because FP64 refinement of the FP32 factor stalled   */
    double seconds;
} cr_basis_info;

/* Rational Krylov basis at fixed expansion points omegas[nshift] (rad/s) with blocks[j] Krylov
   blocks at point j (Eq. (10)): factor A_j once, X = A_j^{-1} F, then X = A_j^{-1} M Q with Q
   the latest orthonormalised block; block classical Gram-Schmidt twice (CGS2) against the basis
   in FP64, columns whose norm falls below 1e-10 of their norm before orthogonalisation are
   dropped. The basis is orthonormal for the Jacobi-scaled system. For a system with a damping
   matrix D the blocks span the second-order Krylov space of Eq. (9) instead: r_0 = A_j^{-1} F,
   r_1 = -A_j^{-1} D_j r_0, r_i = -A_j^{-1} (D_j r_(i-1) + M r_(i-2)) with D_j = 2 i w_j M + D, built
   by an Arnoldi process on the linearisation [u; v] -> [-A_j^{-1} (D_j u + M v); u] whose upper
   halves are appended to the basis; cr_project then adds D_R = V^H D V. */
cr_status cr_basis_build(cr_sys sys, int32_t nshift, const double* omegas, const int32_t* blocks,
                         cr_precision prec, cr_basis* out, cr_basis_info* info);

enum { CR_POLICY_GREEDY = 0, CR_POLICY_MLP = 1 };

typedef struct {
    double f_lo_hz, f_hi_hz;   /* candidate band                                          */
    int32_t n_cand;            /* candidates linspace(f_lo, f_hi, n_cand), <= 4096         */
    int32_t blocks;            /* Krylov blocks per expansion point                        */
    double tol;                /* stop when max relative residual <= tol                   */
    int32_t max_shifts;
    int32_t policy;            /* CR_POLICY_GREEDY or CR_POLICY_MLP                        */
    cr_mlp mlp;                /* network for CR_POLICY_MLP                                */
    const double* geom;        /* geometry features for the network (mlp input tail)       */
    int32_t lookahead;         /* 0, or K > 0: after each unconverged iteration try the K
                                  largest residual peaks (at least 3 candidates apart, not
                                  next to a used point) on a copy of the basis and record
                                  the max residual each would leave (training labels)      */
    int32_t stall_stop;        /* 0, or S > 0: stop once S expansion points in a row added no
                                  basis column (every new Krylov column fell under the
                                  deflation ratio, so the reduced model cannot change)      */
} cr_greedy_opts;

typedef struct {
    int32_t n_iter;            /* expansion points used                                    */
    int32_t* shift_idx;        /* [max_shifts] candidate index per iteration (caller-owned) */
    double* max_res;           /* [max_shifts] max residual after each iteration           */
    double* res;               /* [n_cand] candidate residuals after the last iteration    */
    int32_t* mlp_used;         /* [max_shifts] 1 where the network's proposal was accepted  */
    double* res_hist;          /* [max_shifts x n_cand] residuals after each iteration, or NULL */
    int32_t* la_cand;          /* [max_shifts x lookahead] tried candidates (-1 = none), or NULL */
    double* la_res;            /* [max_shifts x lookahead] max residual after each trial, or NULL */
} cr_greedy_trace;

/* Greedy adaptive expansion points (Section 3.3, after Eq. (9)): start at the candidate nearest
   the band centre; after each point, build the Galerkin model and evaluate the relative
   residual r(w_c) = ||S f(w_c) - S A(w_c) V x_R(w_c)||_F / ||S f(w_c)||_F at every candidate
   (FP64); stop when max r <= tol, else take the unused candidate of largest r (ties: lower
   index) or, with CR_POLICY_MLP, the network's proposal unless its residual is below 0.1 max r. */
cr_status cr_basis_build_greedy(cr_sys sys, const cr_greedy_opts* opts, cr_precision prec,
                                cr_basis* out, cr_greedy_trace* trace, cr_basis_info* info);
/* Local reduced models on frequency windows (l-fROMs; Section 3.3, the local-fROM paragraph and
   its schematic figure, windows of Tab. 4) with an automated partition (the paper partitioned by
   hand): the candidates linspace(f_lo, f_hi, n_cand) are split by bisection. A window [i0, i1] of
   candidate indices runs the greedy of cr_basis_build_greedy on its own candidates
   linspace(cand[i0], cand[i1], i1 - i0 + 1) with at most max_shifts expansion points; if its
   largest candidate residual stays above tol and it holds at least 2 min_cand - 1 candidates, it
   is split at its middle candidate (which both halves share) and both halves are built, left
   first; otherwise the window is kept with its reduced model. */
typedef struct {
    double f_lo_hz, f_hi_hz;
    int32_t n_cand;            /* <= 4096                                                    */
    int32_t blocks;            /* Krylov blocks per expansion point                          */
    double tol;
    int32_t max_shifts;        /* expansion-point cap per window                             */
    int32_t min_cand;          /* >= 2                                                       */
    int32_t max_windows;       /* capacity of the output arrays                              */
} cr_window_opts;

typedef struct {
    int32_t n_windows, expansion_points; /* kept windows, their expansion points             */
    int32_t attempted_points;            /* including windows that were split                */
    int32_t max_q, unconverged;          /* largest order; windows kept at the minimum size
                                            with residual above tol                          */
    double seconds;
} cr_window_info;

/* Outputs (host arrays of max_windows entries, in increasing frequency): win_cand[2 w], [2 w + 1]
   = i0, i1; win_hi_hz[w] = cand[i1]; win_max_res[w] (may be NULL) = the window's largest
   candidate residual; roms[w] = its reduced model (caller destroys). Errors as the greedy's;
   CR_E_INVALID when more than max_windows windows are needed (no model is returned then). */
cr_status cr_build_local_roms(cr_sys sys, const cr_window_opts* opts, cr_precision prec, int32_t* n_windows,
                              int32_t* win_cand, double* win_hi_hz, double* win_max_res, cr_rom* roms,
                              cr_window_info* info);

cr_status cr_basis_dims(cr_basis b, int32_t* q);
/* Copy the basis (n x q, complex128, scaled coordinates) to a device array with leading dim n. */
cr_status cr_basis_copy(cr_basis b, cr_z* V_dev);
/* Full-field recovery from reduced states (Section 3.3, the Galerkin ansatz x = V x_R behind
   Eq. (11)): X = S V XR for ncol columns, XR_dev q x ncol (leading dimension q), X_dev n x ncol
   (leading dimension n), both complex128 on the device; S the system's diagonal scaling, so X is
   in the unscaled DoFs of the system. XR_dev may hold the states of cr_sweep_states for one
   frequency (ncol = L) or for several consecutive ones (ncol = L nfreq). */
cr_status cr_recover_field(cr_basis b, int64_t ncol, const cr_z* XR_dev, cr_z* X_dev);
void cr_basis_destroy(cr_basis b);

/* Galerkin reduced model (Eq. (11)): K_R = V^H K V, M_R = V^H M V, F_R = V^H F (the printed
   V^T f read as V^H f), C_R = C^T V (rows of the unscaled basis at the receivers). FP64. */
cr_status cr_project(cr_sys sys, cr_basis b, cr_rom* out);

/* A reduced model of the form of Eq. (11) (Section 3.3; D_R = V^H D V of the reduced system, or
   the Rayleigh form alpha M_R + beta K_R given after Eq. (11)) from host FP64 column-major arrays:
   K_R, M_R (q x q), D_R (q x q or NULL for D_R = 0), F_R (q x L), C_R (n_o x q), flags[L]
   (load column l is F_R[:, l] (i w)^flags[l]). 1 <= q <= 4096, L >= 1. Arrays are copied. */
cr_status cr_rom_import(cr_ctx ctx, int32_t q, int32_t L, int32_t n_o, const cr_z* KR,
                        const cr_z* DR, const cr_z* MR, const cr_z* FR, const cr_z* CR,
                        const int32_t* flags, cr_rom* out);
cr_status cr_rom_dims(cr_rom r, int32_t* q, int32_t* L, int32_t* n_o);
/* Copy the reduced matrices to host arrays (any may be NULL). */
cr_status cr_rom_export(cr_rom r, cr_z* KR, cr_z* MR, cr_z* FR, cr_z* CR);
void cr_rom_destroy(cr_rom r);

/* ---------------------------------------------------------------- sweep (online phase) --- */

typedef struct {
    int32_t max_ir_iterations; /* over all (w): FP64 refinement corrections of the reduced LU */
    int32_t not_converged;     /* frequencies whose refinement missed 1e-14                  */
    int32_t fp64_fallbacks;    /* CR_MIXED frequencies redone with a complex-FP64 LU because
                                  refinement of the complex-FP32 LU stalled                  */
    int32_t n_perturbed;       /* pivots of the reduced LU that were zero, non-finite or below
                                  eps^2 max|A_R| (numerically singular) and were perturbed;
                                  such a frequency is always refined in FP64                 */
    double seconds;
} cr_sweep_info;

/* Reduced sweep, the online phase of the MOR (Section 3.3, reduced system of Eq. (11), with
   y = C^T x of Eq. (8)): for each w, A_R = K_R + i w D_R - w^2 M_R formed in FP64, dense LU with
   partial pivoting over every row (complex FP32 under CR_MIXED, complex FP64 under CR_FP64),
   solve for the L load columns F_R (i w)^flags, then Y = C_R X_R. CR_MIXED refines every
   frequency in FP64 with FP64 K_R, M_R, D_R until each load column's normwise backward error
   ||r_l||_inf / (||A_R||_inf ||x_l||_inf + ||b_l||_inf) <= 1e-14 and its last correction is below
   1e-12 ||x_l||_inf (or that correction is below 1e-14 ||x_l||_inf): a backward error alone would
   leave up to kappa(A_R) 1e-14 in X. A frequency whose refinement stalls or runs out of
   corrections is redone with a complex-FP64 LU (counted in fp64_fallbacks). CR_FP64
   solves once, and refines only a frequency whose LU had to perturb a pivot.
   CR_FP64 models without D_R and frequency-dependent terms, with q <= 512, L <= 16 and
   n_o <= 256 are solved through the Hessenberg-triangular form of the pencil instead (the same
   result up to rounding): on first use the library reduces (K_R, M_R) with unitary Q, Z to
   Q^H K_R Z = H upper Hessenberg, Q^H M_R Z = T upper triangular (kept with the model, 2 q^2 +
   q (L + n_o) complex entries of device memory), and each frequency solves
   (H - w^2 T) x~ = Q^H F_R (i w)^flags with partial pivoting in O(q^2), Y = (C_R Z) x~. A
   numerically singular pivot sends that frequency to the dense LU with FP64 refinement.
   Y_dev: nfreq x L x n_o complex128, receiver index fastest ([w][l][o]).
   Errors: CR_E_NOT_CONVERGED when a refined frequency misses the tolerance (Y and info are
   still written); CR_E_UNSUPPORTED for q > 4096 or L > 64. */
cr_status cr_sweep(cr_rom r, int32_t nfreq, const double* omegas, cr_precision prec, cr_z* Y_dev,
                   cr_sweep_info* info);

/* Reduced states instead of receiver outputs: as cr_sweep, but XR_dev (nfreq x L x q complex128,
   [w][l][k] with k fastest) receives x_R(w) for every load column, for cr_recover_field. */
cr_status cr_sweep_states(cr_rom r, int32_t nfreq, const double* omegas, cr_precision prec, cr_z* XR_dev,
                          cr_sweep_info* info);

/* Stitched sweep of local models: frequency w goes to the first window k with w / (2 pi) <=
   win_hi_hz[k] (the last window above the band); all windows in one persistent launch. Y_dev
   nfreq x L x n_o as cr_sweep; models must share L and n_o. Errors as cr_sweep. */
cr_status cr_sweep_windows(int32_t nwin, const cr_rom* roms, const double* win_hi_hz, int32_t nfreq,
                           const double* omegas, cr_precision prec, cr_z* Y_dev, cr_sweep_info* info);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
   loops, harnesses that forbid hipMalloc): cr_sweep with the same arguments, results (always
   through the dense LU: for CR_FP64 models that cr_sweep solves through the Hessenberg form, the
   two agree to rounding) and errors,
   but every buffer it needs beyond the reduced model, omegas and Y_dev (model descriptor, work
   queue, statistics, a device copy of the frequencies, per-workgroup LU and refinement
   workspaces) lives in a static device array of 128 MiB that each device holds from its first
   cr_ctx_create until the process ends; the call makes no device allocation. It needs
   512 + 16 nfreq bytes (rounded up to 256) plus, per resident workgroup,
   16 q^2 + 16384 + 64 q L bytes, with at least one workgroup; larger requests fail with
   CR_E_UNSUPPORTED and a message naming the sizes. All calls on one device share the array:
   calls that overlap on one device (several threads or streams) race and must be serialised by
   the caller. Each call clears what must start at zero (the statistics) itself. */
cr_status cr_sweep_noalloc(cr_rom r, int32_t nfreq, const double* omegas, cr_precision prec, cr_z* Y_dev,
                           cr_sweep_info* info);

/* Launch shape of the batched sweep: variant (0 = default, 1 = reduced matrix LDS-resident for
   orders whose q^2 entries fit nb KiB of LDS, 2 = global-memory workspace only), resident
   workgroups per compute unit (0 = 2), nb (KiB, <= 150, variant 1 only), and refine (1 = also refine
   CR_FP64 sweeps with FP64 residuals, e.g. to serve as a reference). */
typedef struct { int32_t variant, grid_per_cu, nb, refine; } cr_tune;

/* Batched sweep (the paper's online phase, Section 3.3, run for many reduced models at once):
   nrom reduced models of uneven order in one persistent launch. omegas: nrom x nfreq
   (row-major, host); Y_dev: host array of nrom device pointers, each nfreq x L_m x n_o_m. Work
   items (model, w) are taken longest-first (q^3 descending). Per item exactly as cr_sweep.
   tune may be NULL (2 workgroups per compute unit, global-memory workspace); the autotuned
   launch shape and graph replay are cr_sweep_plan_create's. Errors as cr_sweep. */
cr_status cr_sweep_batched(cr_ctx ctx, int32_t nrom, const cr_rom* roms, int32_t nfreq,
                           const double* omegas, cr_precision prec, cr_z* const* Y_dev,
                           const cr_tune* tune, cr_sweep_info* info);

/* A batched sweep prepared for repeated execution (the online phase run again and again, e.g.
   for parameter studies): descriptors and work queue uploaded once; the launch shape
   (workgroups per CU, LDS budget of the LDS-resident variant for small orders) chosen by
   timing candidate shapes on a stratified sample of the work items when tune is NULL or
   tune->variant == 0 (otherwise taken from tune: grid_per_cu, nb = LDS budget in KiB); one
   eager execution, then the launch captured in a HIP graph that execute replays. Arguments as
   cr_sweep_batched; the roms, omegas and Y_dev buffers must stay valid while the plan exists. */
typedef struct cr_sweep_plan_s* cr_sweep_plan;
cr_status cr_sweep_plan_create(cr_ctx ctx, int32_t nrom, const cr_rom* roms, int32_t nfreq, const double* omegas,
                               cr_precision prec, cr_z* const* Y_dev, const cr_tune* tune, cr_sweep_plan* out);
cr_status cr_sweep_plan_execute(cr_sweep_plan plan, cr_sweep_info* info);
/* The chosen shape (variant = 1 when the LDS-resident variant is enabled) and, when autotuned,
   the sample times in ms of every candidate (up to max entries; *n receives the count). */
cr_status cr_sweep_plan_tuning(cr_sweep_plan plan, cr_tune* chosen, double* ms, int32_t max, int32_t* n);
void cr_sweep_plan_destroy(cr_sweep_plan plan);

/* ---------------------------------------------------------------- learned shift proposer -- */

/* MLP  n_in -> 3 x hidden (ReLU) -> n_out logits, BF16 weights with FP32 master copies and FP32
   accumulation, trained with softmax cross-entropy and Adam by the library's own kernels. */
cr_status cr_mlp_create(cr_ctx ctx, int32_t n_in, int32_t hidden, int32_t n_out, uint64_t seed,
                        cr_mlp* out);
void cr_mlp_destroy(cr_mlp m);
/* Forward pass: X_dev batch x n_in (row-major, float32) -> logits_dev batch x n_out (float32). */
cr_status cr_mlp_forward(cr_mlp m, int32_t batch, const float* X_dev, float* logits_dev);
/* One Adam step on a minibatch with integer labels and per-sample masks (mask_dev batch x n_out,
   1 = allowed class, or NULL). loss_out (host) receives the mean cross-entropy. */
cr_status cr_mlp_train_step(cr_mlp m, int32_t batch, const float* X_dev, const int32_t* labels_dev,
                            const float* mask_dev, float lr, float* loss_out);
/* Gradients of the mean loss w.r.t. the FP32 master parameters, without an update (for checks).
   grad_dev: n_params floats in the order of cr_mlp_get_params. */
cr_status cr_mlp_gradients(cr_mlp m, int32_t batch, const float* X_dev, const int32_t* labels_dev,
                           const float* mask_dev, float* grad_dev, float* loss_out);
/* Parameter count and host copies of the FP32 master parameters
   (W1, b1, W2, b2, W3, b3, W4, b4; W_l row-major out x in). */
/* Network input for one greedy state (host arrays, no device work): x[c] = log10 r_c - max_c log10 r_c
   for the n_cand candidate residuals res (values below 1e-300 are clamped), then the n_geom geometry
   features; mask (n_cand floats, or NULL) is 0 at every used candidate index and its two
   neighbours, 1 elsewhere. The greedy's CR_POLICY_MLP builds its input with the same function, so
   training data and inference agree. x must hold n_cand + n_geom floats. */
cr_status cr_mlp_features(int32_t n_cand, const double* res, int32_t n_used, const int32_t* used, int32_t n_geom,
                          const double* geom, float* x, float* mask);
cr_status cr_mlp_num_params(cr_mlp m, int64_t* n);
cr_status cr_mlp_get_params(cr_mlp m, float* params);
cr_status cr_mlp_set_params(cr_mlp m, const float* params);

#ifdef __cplusplus
}
#endif
#endif /* CABINROM_H */
