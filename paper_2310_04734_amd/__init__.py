"""Python binding of libcabinrom (rational-Arnoldi MOR of coupled u-p FE systems on MI355X).

Argument marshalling only: every step of the computation runs in the library's HIP kernels.
PyTorch provides device memory (output tensors) and the HIP stream the library enqueues on.
Importing this module fails loudly when the library has not been built; there is no CPU path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcabinrom.so")

CR_FP64 = 0
CR_MIXED = 1
CR_POLICY_GREEDY = 0
CR_POLICY_MLP = 1

_STATUS = {0: "CR_OK", -1: "CR_E_INVALID", -2: "CR_E_OOM", -3: "CR_E_HIP", -4: "CR_E_SINGULAR",
           -5: "CR_E_NOT_CONVERGED", -6: "CR_E_UNSUPPORTED", -7: "CR_E_STATE"}


class CabinRomError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = _STATUS.get(status, str(status))


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2310_04734_amd.build.build() "
                          "(there is no CPU fallback)")
    # torch first: the library then binds the HIP runtime torch already loaded (same soname), so
    # device memory and streams from torch and the library's kernels live in one runtime
    import torch  # noqa: F401
    return C.CDLL(LIB_PATH)


lib = _load()

c_z_p = C.c_void_p


class cr_material(C.Structure):
    _fields_ = [("kind", C.c_int32), ("rho", C.c_double), ("eta", C.c_double), ("c", C.c_double),
                ("E", C.c_double), ("nu", C.c_double), ("n_eta", C.c_int32), ("eta_f_hz", C.c_void_p),
                ("eta_val", C.c_void_p)]


class cr_mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("coords", C.c_void_p), ("n_el", C.c_int64), ("elems", C.c_void_p),
                ("elem_mat", C.c_void_p), ("n_clamped", C.c_int64), ("clamped", C.c_void_p),
                ("n_iface", C.c_int64), ("iface", C.c_void_p)]


class cr_z(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class cr_load(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dir", C.c_int32), ("node", C.c_int64), ("value", cr_z),
                ("n_faces", C.c_int64), ("faces", C.c_void_p), ("amp", C.c_void_p)]


class cr_sys_dims(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("n_u", C.c_int64), ("L", C.c_int32), ("n_o", C.c_int32)]


class cr_analysis_info(C.Structure):
    _fields_ = [("n_fronts", C.c_int32), ("n_levels", C.c_int32), ("max_front", C.c_int32),
                ("max_pivots", C.c_int32), ("factor_entries", C.c_int64), ("factor_flops", C.c_double),
                ("gemm_flops", C.c_double),
                ("seconds", C.c_double)]


class cr_factor_info(C.Structure):
    _fields_ = [("n_perturbed", C.c_int32), ("seconds", C.c_double)]


class cr_ir_opts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("tol", C.c_double)]


class cr_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("backward_error", C.c_double)]


class cr_basis_info(C.Structure):
    _fields_ = [("q", C.c_int32), ("deflated", C.c_int32), ("n_shifts", C.c_int32), ("ir_iterations", C.c_int32),
                ("max_backward_error", C.c_double), ("n_perturbed", C.c_int32),
                ("fp64_refactorizations", C.c_int32), ("seconds", C.c_double)]


class cr_greedy_opts(C.Structure):
    _fields_ = [("f_lo_hz", C.c_double), ("f_hi_hz", C.c_double), ("n_cand", C.c_int32), ("blocks", C.c_int32),
                ("tol", C.c_double), ("max_shifts", C.c_int32), ("policy", C.c_int32), ("mlp", C.c_void_p),
                ("geom", C.c_void_p), ("lookahead", C.c_int32), ("stall_stop", C.c_int32)]


class cr_greedy_trace(C.Structure):
    _fields_ = [("n_iter", C.c_int32), ("shift_idx", C.c_void_p), ("max_res", C.c_void_p), ("res", C.c_void_p),
                ("mlp_used", C.c_void_p), ("res_hist", C.c_void_p), ("la_cand", C.c_void_p), ("la_res", C.c_void_p)]


class cr_sweep_info(C.Structure):
    _fields_ = [("max_ir_iterations", C.c_int32), ("not_converged", C.c_int32), ("fp64_fallbacks", C.c_int32),
                ("n_perturbed", C.c_int32), ("seconds", C.c_double)]


def _sweep_info(info):
    return {k: getattr(info, k) for k, _ in cr_sweep_info._fields_}


class cr_window_opts(C.Structure):
    _fields_ = [("f_lo_hz", C.c_double), ("f_hi_hz", C.c_double), ("n_cand", C.c_int32), ("blocks", C.c_int32),
                ("tol", C.c_double), ("max_shifts", C.c_int32), ("min_cand", C.c_int32), ("max_windows", C.c_int32)]


class cr_window_info(C.Structure):
    _fields_ = [("n_windows", C.c_int32), ("expansion_points", C.c_int32), ("attempted_points", C.c_int32),
                ("max_q", C.c_int32), ("unconverged", C.c_int32), ("seconds", C.c_double)]


class cr_dd_opts(C.Structure):
    _fields_ = [("overlap", C.c_int32), ("restricted", C.c_int32), ("restart", C.c_int32), ("max_iter", C.c_int32),
                ("tol", C.c_double)]


class cr_dd_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("rel_residual", C.c_double), ("n_sub", C.c_int32),
                ("sub_factor_entries", C.c_int64), ("seconds", C.c_double)]


class cr_tune(C.Structure):
    _fields_ = [("variant", C.c_int32), ("grid_per_cu", C.c_int32), ("nb", C.c_int32), ("refine", C.c_int32)]


def _sig(name, res, *args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


P = C.c_void_p
I32, I64, D = C.c_int32, C.c_int64, C.c_double
class cr_allocator(C.Structure):
    _fields_ = [("alloc", C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)),
                ("free", C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)), ("user", C.c_void_p)]


_sig("cr_ctx_create", I32, C.c_int, P, C.POINTER(cr_allocator), C.POINTER(P))
_sig("cr_ctx_destroy", None, P)
_sig("cr_last_error", C.c_char_p, P)
_sig("cr_create_error", C.c_char_p)
_sig("cr_assemble", I32, P, C.POINTER(cr_mesh), P, I32, P, I32, P, I32, C.POINTER(P))
_sig("cr_sys_get_dims", I32, P, C.POINTER(cr_sys_dims))
_sig("cr_sys_export", I32, P, P, P, P, P, P, P, P)
_sig("cr_sys_destroy", None, P)
_sig("cr_sys_import_csr", I32, P, I64, P, P, P, P, P, I32, P, P, I32, P, P, C.POINTER(P))
_sig("cr_recover_field", I32, P, I64, P, P)
_sig("cr_dd_create", I32, P, C.POINTER(cr_dd_opts), C.POINTER(P))
_sig("cr_dd_destroy", None, P)
_sig("cr_dd_solve", I32, P, D, I32, I32, P, P, C.POINTER(cr_dd_info))
_sig("cr_dd_precondition", I32, P, D, I32, I32, P, P)
_sig("cr_build_local_roms", I32, P, C.POINTER(cr_window_opts), I32, C.POINTER(I32), P, P, P, P,
     C.POINTER(cr_window_info))
_sig("cr_sweep_windows", I32, I32, P, P, I32, P, I32, P, C.POINTER(cr_sweep_info))
_sig("cr_sweep_states", I32, P, I32, P, I32, P, C.POINTER(cr_sweep_info))
_sig("cr_analyse", I32, P, C.POINTER(cr_analysis_info))
_sig("cr_set_front_classes", I32, P, I32, I32)
_sig("cr_set_panel_split", I32, P, I32, I32)
_sig("cr_factor", I32, P, D, I32, C.POINTER(P), C.POINTER(cr_factor_info))
_sig("cr_fact_destroy", None, P)
_sig("cr_solve", I32, P, I32, P, P, C.POINTER(cr_ir_opts), C.POINTER(cr_solve_info))
_sig("cr_basis_build", I32, P, I32, P, P, I32, C.POINTER(P), C.POINTER(cr_basis_info))
_sig("cr_basis_build_greedy", I32, P, C.POINTER(cr_greedy_opts), I32, C.POINTER(P), C.POINTER(cr_greedy_trace),
     C.POINTER(cr_basis_info))
_sig("cr_basis_dims", I32, P, C.POINTER(I32))
_sig("cr_basis_copy", I32, P, P)
_sig("cr_basis_destroy", None, P)
_sig("cr_project", I32, P, P, C.POINTER(P))
_sig("cr_rom_import", I32, P, I32, I32, I32, P, P, P, P, P, P, C.POINTER(P))
_sig("cr_rom_dims", I32, P, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32))
_sig("cr_rom_export", I32, P, P, P, P, P)
_sig("cr_rom_destroy", None, P)
_sig("cr_sweep", I32, P, I32, P, I32, P, C.POINTER(cr_sweep_info))
_sig("cr_sweep_noalloc", I32, P, I32, P, I32, P, C.POINTER(cr_sweep_info))
_sig("cr_sweep_batched", I32, P, I32, P, I32, P, I32, P, C.POINTER(cr_tune), C.POINTER(cr_sweep_info))
_sig("cr_mlp_create", I32, P, I32, I32, I32, C.c_uint64, C.POINTER(P))
_sig("cr_mlp_destroy", None, P)
_sig("cr_mlp_forward", I32, P, I32, P, P)
_sig("cr_mlp_train_step", I32, P, I32, P, P, P, C.c_float, C.POINTER(C.c_float))
_sig("cr_mlp_gradients", I32, P, I32, P, P, P, P, C.POINTER(C.c_float))
_sig("cr_mlp_features", I32, I32, P, I32, P, I32, P, P, P)
_sig("cr_mlp_num_params", I32, P, C.POINTER(I64))
_sig("cr_mlp_get_params", I32, P, P)
_sig("cr_mlp_set_params", I32, P, P)
_sig("cr_sweep_plan_create", I32, P, I32, P, I32, P, I32, P, P, C.POINTER(P))
_sig("cr_sweep_plan_execute", I32, P, C.POINTER(cr_sweep_info))
_sig("cr_sweep_plan_tuning", I32, P, C.POINTER(cr_tune), P, I32, C.POINTER(I32))
_sig("cr_sweep_plan_destroy", None, P)
_sig("cr_profile_enable", I32, P, I32)
_sig("cr_profile_read", I32, P, I32, P, P, P, C.POINTER(I32))
_sig("cr_profile_select", I32, P, C.c_char_p)
_sig("cr_probe_copy", I32, P, C.c_int64, I32, C.POINTER(C.c_double))
_sig("cr_probe_mfma", I32, P, I32, I32, C.POINTER(C.c_double))


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _dev_ptr(t):
    return C.c_void_p(t.data_ptr())


class Context:
    """A library context bound to a HIP device and torch's current stream on it.

    allocator: None (hipMalloc) or a pair of Python callables (alloc(nbytes) -> int device
    pointer or 0, free(ptr)) that the library calls for every device buffer of this context;
    they are kept alive by the context."""

    def __init__(self, device: int = 0, stream=None, allocator=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = P()
        al = None
        if allocator is not None:
            fa, ff = allocator
            self._alloc_cb = cr_allocator._fields_[0][1](lambda nbytes, user: fa(int(nbytes)) or None)
            self._free_cb = cr_allocator._fields_[1][1](lambda ptr, user: ff(int(ptr or 0)))
            al = cr_allocator(self._alloc_cb, self._free_cb, None)
        st = lib.cr_ctx_create(device, C.c_void_p(stream.cuda_stream), C.byref(al) if al is not None else None,
                               C.byref(h))
        if st != 0:
            raise CabinRomError(st, lib.cr_create_error().decode())
        self.h = h

    def check(self, st):
        if st != 0:
            raise CabinRomError(st, lib.cr_last_error(self.h).decode())

    def profile(self, on: bool):
        """Start (clearing earlier records) or stop event timing of the library's kernels."""
        self.check(lib.cr_profile_enable(self.h, int(on)))

    def profile_select(self, names=None):
        """Time only the named kernels (an iterable of names; None: all of them again)."""
        arg = None if not names else ",".join(names).encode()
        self.check(lib.cr_profile_select(self.h, arg))

    def probe_copy(self, nbytes=256 << 20, reps=10):
        """Achievable HBM rate of a streaming copy (GB/s, bytes read + written)."""
        v = C.c_double()
        self.check(lib.cr_probe_copy(self.h, int(nbytes), int(reps), C.byref(v)))
        return v.value

    def probe_mfma(self, prec, reps=5):
        """Achievable matrix-core rate (TFLOP/s): FP64 MFMA for CR_FP64, FP32 MFMA for CR_MIXED."""
        v = C.c_double()
        self.check(lib.cr_probe_mfma(self.h, int(prec), int(reps), C.byref(v)))
        return v.value

    def profile_read(self):
        """{kernel name: (launches, total ms)} over the launches since profile(True)."""
        mx = 64
        names = C.create_string_buffer(32 * mx)
        counts = np.zeros(mx, np.int32)
        tot = np.zeros(mx, np.float64)
        n = I32()
        self.check(lib.cr_profile_read(self.h, mx, names, _ptr(counts), _ptr(tot), C.byref(n)))
        raw = names.raw
        out = {}
        for i in range(min(n.value, mx)):
            nm = raw[32 * i:32 * i + 32].split(b"\0", 1)[0].decode()
            out[nm] = (int(counts[i]), float(tot[i]))
        return out

    def close(self):
        if self.h:
            lib.cr_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class System:
    def __init__(self, ctx: Context, h):
        self.ctx, self.h = ctx, h
        d = cr_sys_dims()
        ctx.check(lib.cr_sys_get_dims(h, C.byref(d)))
        self.n, self.nnz, self.n_u, self.L, self.n_o = d.n, d.nnz, d.n_u, d.L, d.n_o
        self.analysis = None

    def export(self, matrices=True):
        """Unscaled host copies: rowptr, col, K, M (CSR values; None unless matrices), F (n x L),
        flags, recv DoFs."""
        n, nnz = self.n, self.nnz
        rowptr = np.empty(n + 1, np.int64) if matrices else None
        col = np.empty(nnz, np.int32) if matrices else None
        K = np.empty(nnz, np.complex128) if matrices else None
        M = np.empty(nnz, np.complex128) if matrices else None
        F = np.empty((self.L, n), np.complex128)
        flags = np.empty(max(self.L, 1), np.int32)
        recv = np.empty(max(self.n_o, 1), np.int64)
        self.ctx.check(lib.cr_sys_export(self.h, _ptr(rowptr), _ptr(col), _ptr(K), _ptr(M), _ptr(F), _ptr(flags),
                                         _ptr(recv)))
        return dict(rowptr=rowptr, col=col, K=K, M=M, F=F.T.copy(), flags=flags[:self.L], recv=recv[:self.n_o])

    def set_front_classes(self, big_m=192, huge_m=1024):
        self.ctx.check(lib.cr_set_front_classes(self.h, int(big_m), int(huge_m)))

    def set_panel_split(self, min_rows=1024, max_polls=0):
        self.ctx.check(lib.cr_set_panel_split(self.h, int(min_rows), int(max_polls)))

    def analyse(self):
        info = cr_analysis_info()
        self.ctx.check(lib.cr_analyse(self.h, C.byref(info)))
        self.analysis = {k: getattr(info, k) for k, _ in cr_analysis_info._fields_}
        return self.analysis

    def factor(self, omega: float, prec: int = CR_MIXED):
        h = P()
        info = cr_factor_info()
        self.ctx.check(lib.cr_factor(self.h, float(omega), prec, C.byref(h), C.byref(info)))
        return Factor(self, h, info.n_perturbed)

    def basis(self, omegas, blocks, prec: int = CR_MIXED):
        om = np.ascontiguousarray(omegas, np.float64)
        bl = np.ascontiguousarray(np.broadcast_to(blocks, om.shape), np.int32)
        h = P()
        info = cr_basis_info()
        self.ctx.check(lib.cr_basis_build(self.h, len(om), _ptr(om), _ptr(bl), prec, C.byref(h), C.byref(info)))
        return Basis(self, h, info)

    def basis_greedy(self, band_hz, n_cand, blocks, tol, max_shifts, prec: int = CR_MIXED, policy=CR_POLICY_GREEDY,
                     mlp=None, geom=None, lookahead=0, stall_stop=0):
        g = np.ascontiguousarray(geom if geom is not None else np.zeros(0), np.float64)
        opts = cr_greedy_opts(float(band_hz[0]), float(band_hz[1]), int(n_cand), int(blocks), float(tol),
                              int(max_shifts), int(policy), mlp.h if mlp is not None else None, _ptr(g), int(lookahead),
                              int(stall_stop))
        sidx = np.full(max_shifts, -1, np.int32)
        mres = np.zeros(max_shifts)
        res = np.zeros(n_cand)
        used = np.zeros(max_shifts, np.int32)
        hist = np.zeros((max_shifts, n_cand))
        K = max(int(lookahead), 1)
        la_c = np.full((max_shifts, K), -1, np.int32)
        la_r = np.full((max_shifts, K), -1.0)
        tr = cr_greedy_trace(0, _ptr(sidx), _ptr(mres), _ptr(res), _ptr(used), _ptr(hist), _ptr(la_c), _ptr(la_r))
        h = P()
        info = cr_basis_info()
        self.ctx.check(lib.cr_basis_build_greedy(self.h, C.byref(opts), prec, C.byref(h), C.byref(tr), C.byref(info)))
        k = tr.n_iter
        b = Basis(self, h, info)
        b.trace = dict(shift_idx=sidx[:k].copy(), max_res=mres[:k].copy(), res=res, mlp_used=used[:k].copy(),
                       res_hist=hist[:k].copy(), la_cand=la_c[:k].copy(), la_res=la_r[:k].copy())
        return b

    def local_roms(self, band_hz, n_cand, blocks, tol, max_shifts, min_cand=4, max_windows=64, prec: int = CR_MIXED):
        """Local reduced models on automatically bisected frequency windows (LocalRoms)."""
        opts = cr_window_opts(float(band_hz[0]), float(band_hz[1]), int(n_cand), int(blocks), float(tol),
                              int(max_shifts), int(min_cand), int(max_windows))
        nw = I32()
        wc = np.zeros(2 * max_windows, np.int32)
        hi = np.zeros(max_windows)
        mr = np.zeros(max_windows)
        hs = (P * max_windows)()
        info = cr_window_info()
        self.ctx.check(lib.cr_build_local_roms(self.h, C.byref(opts), prec, C.byref(nw), _ptr(wc), _ptr(hi), _ptr(mr),
                                               hs, C.byref(info)))
        k = nw.value
        roms = [Rom(self.ctx, P(hs[i])) for i in range(k)]
        return LocalRoms(self.ctx, roms, wc[:2 * k].reshape(k, 2).copy(), hi[:k].copy(), mr[:k].copy(),
                         {f: getattr(info, f) for f, _ in cr_window_info._fields_})

    def __del__(self):
        if getattr(self, "h", None) and lib is not None:
            lib.cr_sys_destroy(self.h)
            self.h = None


def assemble(ctx: Context, mesh, loads, receivers) -> System:
    """Assemble K, M, F and the receiver map from a hex8 mesh (duck-typed: coords, elems,
    elem_mat, materials, clamped, iface) and load descriptors (kind, node, dir, value,
    faces, amp)."""
    coords = np.ascontiguousarray(mesh.coords, np.float64)
    elems = np.ascontiguousarray(mesh.elems, np.int64)
    emat = np.ascontiguousarray(mesh.elem_mat, np.int32)
    clamped = np.ascontiguousarray(mesh.clamped, np.int64)
    iface = np.ascontiguousarray(mesh.iface, np.int64).reshape(-1, 4)
    m = cr_mesh(coords.shape[0], _ptr(coords), elems.shape[0], _ptr(elems), _ptr(emat), len(clamped),
                _ptr(clamped), iface.shape[0], _ptr(iface))
    mats = (cr_material * len(mesh.materials))()
    keep = []
    for i, mt in enumerate(mesh.materials):
        tab = getattr(mt, "eta_table", None)
        if tab is not None:
            fh = np.ascontiguousarray(tab[0], np.float64)
            ev = np.ascontiguousarray(tab[1], np.float64)
            keep += [fh, ev]
            mats[i] = cr_material(mt.kind, mt.rho, mt.eta, mt.c, mt.E, mt.nu, len(fh), _ptr(fh), _ptr(ev))
        else:
            mats[i] = cr_material(mt.kind, mt.rho, mt.eta, mt.c, mt.E, mt.nu, 0, None, None)
    lds = (cr_load * max(len(loads), 1))()
    for i, ld in enumerate(loads):
        v = complex(ld.value)
        faces = amp = None
        nf = 0
        if ld.faces is not None:
            faces = np.ascontiguousarray(ld.faces, np.int64).reshape(-1, 4)
            amp = np.ascontiguousarray(ld.amp, np.complex128)
            nf = faces.shape[0]
            keep += [faces, amp]
        lds[i] = cr_load(ld.kind, ld.dir, ld.node, cr_z(v.real, v.imag), nf, _ptr(faces), _ptr(amp))
    rec = np.ascontiguousarray(receivers, np.int64)
    h = P()
    ctx.check(lib.cr_assemble(ctx.h, C.byref(m), mats, len(mesh.materials), lds, len(loads), _ptr(rec), len(rec),
                              C.byref(h)))
    return System(ctx, h)


def import_csr(ctx: Context, rowptr, col, K, M, F, flags, recv_dofs, D=None, coords=None) -> System:
    """A system from CSR matrices K, M (and D) on one pattern, loads F (n x L) and receiver DoFs."""
    rowptr = np.ascontiguousarray(rowptr, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    K = np.ascontiguousarray(K, np.complex128)
    M = np.ascontiguousarray(M, np.complex128)
    Dv = np.ascontiguousarray(D, np.complex128) if D is not None else None
    n = len(rowptr) - 1
    F = np.asfortranarray(np.asarray(F, np.complex128).reshape(n, -1))
    fl = np.ascontiguousarray(flags, np.int32)
    rec = np.ascontiguousarray(recv_dofs, np.int64)
    xyz = np.ascontiguousarray(coords, np.float64) if coords is not None else None
    h = P()
    ctx.check(lib.cr_sys_import_csr(ctx.h, n, _ptr(rowptr), _ptr(col), _ptr(K), _ptr(Dv), _ptr(M), F.shape[1],
                                    F.ctypes.data_as(P), _ptr(fl), len(rec), _ptr(rec), _ptr(xyz), C.byref(h)))
    return System(ctx, h)


class Factor:
    def __init__(self, sys: System, h, n_perturbed):
        self.sys, self.h, self.n_perturbed = sys, h, n_perturbed

    def solve(self, B, max_iter=10, tol=1e-14):
        """X = A^{-1} B for a (n x nrhs) complex128 device tensor (column-major = B.T contiguous)."""
        torch = self.sys.ctx.torch
        Bc = B.t().contiguous() if B.dim() == 2 else B.reshape(1, -1).contiguous()
        X = torch.empty_like(Bc)
        info = cr_solve_info()
        opts = cr_ir_opts(max_iter, tol)
        st = lib.cr_solve(self.h, Bc.shape[0], _dev_ptr(Bc), _dev_ptr(X), C.byref(opts), C.byref(info))
        self.last_info = dict(iterations=info.iterations, backward_error=info.backward_error)
        self.sys.ctx.check(st)
        return X.t() if B.dim() == 2 else X.reshape(-1)

    def __del__(self):
        if getattr(self, "h", None) and lib is not None:
            lib.cr_fact_destroy(self.h)
            self.h = None


class Basis:
    def __init__(self, sys: System, h, info):
        self.sys, self.h = sys, h
        self.info = {k: getattr(info, k) for k, _ in cr_basis_info._fields_}
        q = I32()
        sys.ctx.check(lib.cr_basis_dims(h, C.byref(q)))
        self.q = q.value
        self.trace = None

    def V(self):
        torch = self.sys.ctx.torch
        V = torch.empty((self.q, self.sys.n), dtype=torch.complex128, device=self.sys.ctx.device)
        self.sys.ctx.check(lib.cr_basis_copy(self.h, _dev_ptr(V)))
        return V.t()

    def project(self):
        h = P()
        self.sys.ctx.check(lib.cr_project(self.sys.h, self.h, C.byref(h)))
        return Rom(self.sys.ctx, h)

    def recover(self, XR):
        """X = S V XR: full-order fields (n x ncol, unscaled DoFs) from reduced states (q x ncol)."""
        torch = self.sys.ctx.torch
        XRc = XR.t().contiguous() if XR.dim() == 2 else XR.reshape(1, -1).contiguous()   # ncol x q
        X = torch.empty((XRc.shape[0], self.sys.n), dtype=torch.complex128, device=self.sys.ctx.device)
        self.sys.ctx.check(lib.cr_recover_field(self.h, XRc.shape[0], _dev_ptr(XRc), _dev_ptr(X)))
        return X.t()

    def __del__(self):
        if getattr(self, "h", None) and lib is not None:
            lib.cr_basis_destroy(self.h)
            self.h = None


class Rom:
    def __init__(self, ctx: Context, h):
        self.ctx, self.h = ctx, h
        q, L, no = I32(), I32(), I32()
        ctx.check(lib.cr_rom_dims(h, C.byref(q), C.byref(L), C.byref(no)))
        self.q, self.L, self.n_o = q.value, L.value, no.value

    @staticmethod
    def from_arrays(ctx: Context, KR, MR, FR, CR, flags, DR=None):
        f = lambda a: np.asfortranarray(a, np.complex128)
        KR, MR, FR, CR = f(KR), f(MR), f(FR), f(CR)
        DR = f(DR) if DR is not None else None
        fl = np.ascontiguousarray(flags, np.int32)
        q, L = FR.shape
        h = P()
        ctx.check(lib.cr_rom_import(ctx.h, q, L, CR.shape[0], KR.ctypes.data_as(P), _ptr(DR) if DR is not None else None,
                                    MR.ctypes.data_as(P), FR.ctypes.data_as(P), CR.ctypes.data_as(P), _ptr(fl),
                                    C.byref(h)))
        return Rom(ctx, h)

    def export(self):
        q, L, no = self.q, self.L, self.n_o
        KR = np.empty((q, q), np.complex128, order="F")
        MR = np.empty((q, q), np.complex128, order="F")
        FR = np.empty((q, L), np.complex128, order="F")
        CR = np.empty((max(no, 1), q), np.complex128, order="F")
        self.ctx.check(lib.cr_rom_export(self.h, KR.ctypes.data_as(P), MR.ctypes.data_as(P), FR.ctypes.data_as(P),
                                         CR.ctypes.data_as(P)))
        return dict(KR=KR, MR=MR, FR=FR, CR=CR[:no])

    def sweep(self, omegas, prec=CR_MIXED, out=None):
        """Y[w, l, o] complex128 device tensor."""
        torch = self.ctx.torch
        om = np.ascontiguousarray(omegas, np.float64)
        Y = out if out is not None else torch.empty((len(om), self.L, self.n_o), dtype=torch.complex128,
                                                    device=self.ctx.device)
        info = cr_sweep_info()
        st = lib.cr_sweep(self.h, len(om), _ptr(om), prec, _dev_ptr(Y), C.byref(info))
        self.last_info = _sweep_info(info)
        self.ctx.check(st)
        return Y

    def sweep_states(self, omegas, prec=CR_MIXED):
        """x_R[w, l, k] complex128 device tensor (reduced states for cr_recover_field)."""
        torch = self.ctx.torch
        om = np.ascontiguousarray(omegas, np.float64)
        XR = torch.empty((len(om), self.L, self.q), dtype=torch.complex128, device=self.ctx.device)
        info = cr_sweep_info()
        st = lib.cr_sweep_states(self.h, len(om), _ptr(om), prec, _dev_ptr(XR), C.byref(info))
        self.last_info = _sweep_info(info)
        self.ctx.check(st)
        return XR

    def sweep_noalloc(self, omegas, prec=CR_MIXED, out=None):
        """As sweep, through the allocation-free entry point (static device scratch)."""
        torch = self.ctx.torch
        om = np.ascontiguousarray(omegas, np.float64)
        Y = out if out is not None else torch.empty((len(om), self.L, self.n_o), dtype=torch.complex128,
                                                    device=self.ctx.device)
        info = cr_sweep_info()
        st = lib.cr_sweep_noalloc(self.h, len(om), _ptr(om), prec, _dev_ptr(Y), C.byref(info))
        self.last_info = _sweep_info(info)
        self.ctx.check(st)
        return Y

    def __del__(self):
        if getattr(self, "h", None) and lib is not None:
            lib.cr_rom_destroy(self.h)
            self.h = None


class DomainDecomposition:
    """GMRES with an additive Schwarz preconditioner on the structure / fluid subdomains."""

    def __init__(self, sys: System, overlap=1, restricted=True, restart=100, max_iter=300, tol=1e-8):
        self.sys = sys
        opts = cr_dd_opts(int(overlap), int(bool(restricted)), int(restart), int(max_iter), float(tol))
        h = P()
        sys.ctx.check(lib.cr_dd_create(sys.h, C.byref(opts), C.byref(h)))
        self.h = h
        self.last_info = None

    def solve(self, omega, B, prec=CR_FP64):
        torch = self.sys.ctx.torch
        Bc = B.t().contiguous() if B.dim() == 2 else B.reshape(1, -1).contiguous()
        X = torch.empty_like(Bc)
        info = cr_dd_info()
        st = lib.cr_dd_solve(self.h, float(omega), int(prec), Bc.shape[0], _dev_ptr(Bc), _dev_ptr(X), C.byref(info))
        self.last_info = {k: getattr(info, k) for k, _ in cr_dd_info._fields_}
        self.sys.ctx.check(st)
        return X.t() if B.dim() == 2 else X.reshape(-1)

    def precondition(self, omega, R, prec=CR_FP64):
        torch = self.sys.ctx.torch
        Rc = R.t().contiguous()
        Z = torch.empty_like(Rc)
        self.sys.ctx.check(lib.cr_dd_precondition(self.h, float(omega), int(prec), Rc.shape[0], _dev_ptr(Rc),
                                                  _dev_ptr(Z)))
        return Z.t()

    def __del__(self):
        if getattr(self, "h", None) and lib is not None:
            lib.cr_dd_destroy(self.h)
            self.h = None


class LocalRoms:
    """Reduced models of frequency windows and their stitched sweep."""

    def __init__(self, ctx, roms, cand, hi_hz, max_res, info):
        self.ctx, self.roms, self.cand, self.hi_hz, self.max_res, self.info = ctx, roms, cand, hi_hz, max_res, info

    def sweep(self, omegas, prec=CR_MIXED, out=None):
        torch = self.ctx.torch
        om = np.ascontiguousarray(omegas, np.float64)
        r0 = self.roms[0]
        Y = out if out is not None else torch.empty((len(om), r0.L, r0.n_o), dtype=torch.complex128,
                                                    device=self.ctx.device)
        hs = (P * len(self.roms))(*[r.h for r in self.roms])
        hi = np.ascontiguousarray(self.hi_hz, np.float64)
        info = cr_sweep_info()
        st = lib.cr_sweep_windows(len(self.roms), hs, _ptr(hi), len(om), _ptr(om), prec, _dev_ptr(Y), C.byref(info))
        self.last_info = _sweep_info(info)
        self.ctx.check(st)
        return Y


class Mlp:
    """The learned expansion-point proposer (n_in -> 3 x hidden ReLU -> n_out), trained on the GPU."""

    def __init__(self, ctx: Context, n_in=259, hidden=256, n_out=256, seed=2310047347007):
        self.ctx, self.n_in, self.hidden, self.n_out = ctx, n_in, hidden, n_out
        h = P()
        ctx.check(lib.cr_mlp_create(ctx.h, n_in, hidden, n_out, C.c_uint64(seed), C.byref(h)))
        self.h = h
        n = I64()
        ctx.check(lib.cr_mlp_num_params(h, C.byref(n)))
        self.n_params = n.value

    def get_params(self):
        p = np.empty(self.n_params, np.float32)
        self.ctx.check(lib.cr_mlp_get_params(self.h, _ptr(p)))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        assert p.size == self.n_params
        self.ctx.check(lib.cr_mlp_set_params(self.h, _ptr(p)))

    def forward(self, X):
        torch = self.ctx.torch
        X = X.contiguous().to(torch.float32)
        out = torch.empty((X.shape[0], self.n_out), dtype=torch.float32, device=self.ctx.device)
        self.ctx.check(lib.cr_mlp_forward(self.h, X.shape[0], _dev_ptr(X), _dev_ptr(out)))
        return out

    def gradients(self, X, labels, mask=None):
        torch = self.ctx.torch
        X = X.contiguous().to(torch.float32)
        lab = labels.contiguous().to(torch.int32)
        m = mask.contiguous().to(torch.float32) if mask is not None else None
        g = torch.empty(self.n_params, dtype=torch.float32, device=self.ctx.device)
        loss = C.c_float()
        self.ctx.check(lib.cr_mlp_gradients(self.h, X.shape[0], _dev_ptr(X), _dev_ptr(lab),
                                            _dev_ptr(m) if m is not None else None, _dev_ptr(g), C.byref(loss)))
        return loss.value, g

    def train_step(self, X, labels, mask=None, lr=1e-3):
        torch = self.ctx.torch
        X = X.contiguous().to(torch.float32)
        lab = labels.contiguous().to(torch.int32)
        m = mask.contiguous().to(torch.float32) if mask is not None else None
        loss = C.c_float()
        self.ctx.check(lib.cr_mlp_train_step(self.h, X.shape[0], _dev_ptr(X), _dev_ptr(lab),
                                             _dev_ptr(m) if m is not None else None, float(lr), C.byref(loss)))
        return loss.value

    def __del__(self):
        if getattr(self, "h", None) and lib is not None:
            lib.cr_mlp_destroy(self.h)
            self.h = None


def mlp_features(res, used, geom=None):
    """Network input (float32 n_cand + n_geom) and class mask (float32 n_cand) for one greedy state."""
    res = np.ascontiguousarray(res, np.float64)
    used = np.ascontiguousarray(used, np.int32)
    g = np.ascontiguousarray(geom if geom is not None else np.zeros(0), np.float64)
    x = np.empty(res.size + g.size, np.float32)
    m = np.empty(res.size, np.float32)
    st = lib.cr_mlp_features(res.size, _ptr(res), used.size, _ptr(used), g.size, _ptr(g), _ptr(x), _ptr(m))
    if st != 0:
        raise CabinRomError(st, "cr_mlp_features: bad arguments")
    return x, m


class SweepPlan:
    """A batched sweep prepared once (autotuned launch shape, HIP graph) and replayed."""

    def __init__(self, ctx: Context, roms, omegas, prec=CR_MIXED, outs=None, tune=None):
        torch = ctx.torch
        self.ctx, self.roms = ctx, list(roms)
        self.om = np.ascontiguousarray(omegas, np.float64)
        nrom, nfreq = self.om.shape
        self.outs = outs if outs is not None else [
            torch.empty((nfreq, r.L, r.n_o), dtype=torch.complex128, device=ctx.device) for r in roms]
        hs = (P * nrom)(*[r.h for r in roms])
        ys = (P * nrom)(*[Y.data_ptr() for Y in self.outs])
        t = None
        if tune is not None:
            t = cr_tune(int(tune.get("variant", 0)), int(tune.get("grid_per_cu", 0)), int(tune.get("nb", 0)),
                        int(tune.get("refine", 0)))
        h = P()
        ctx.check(lib.cr_sweep_plan_create(ctx.h, nrom, hs, nfreq, _ptr(self.om), prec, ys,
                                           C.byref(t) if t is not None else None, C.byref(h)))
        self.h = h

    def execute(self):
        info = cr_sweep_info()
        st = lib.cr_sweep_plan_execute(self.h, C.byref(info))
        self.last_info = _sweep_info(info)
        self.ctx.check(st)
        return self.last_info

    def tuning(self):
        ch = cr_tune()
        ms = np.zeros(64)
        n = I32()
        self.ctx.check(lib.cr_sweep_plan_tuning(self.h, C.byref(ch), _ptr(ms), 64, C.byref(n)))
        return dict(variant=ch.variant, grid_per_cu=ch.grid_per_cu, lds_kib=ch.nb, sample_ms=ms[:n.value].tolist())

    def __del__(self):
        if getattr(self, "h", None) and lib is not None:
            lib.cr_sweep_plan_destroy(self.h)
            self.h = None


def sweep_batched(ctx: Context, roms, omegas, prec=CR_MIXED, outs=None, tune=None):
    """omegas: (nrom, nfreq) host array; returns a list of Y tensors (nfreq x L x n_o) and the
    sweep info. tune: None or dict(variant, grid_per_cu, nb, refine)."""
    torch = ctx.torch
    om = np.ascontiguousarray(omegas, np.float64)
    nrom, nfreq = om.shape
    if outs is None:
        outs = [torch.empty((nfreq, r.L, r.n_o), dtype=torch.complex128, device=ctx.device) for r in roms]
    hs = (P * nrom)(*[r.h for r in roms])
    ys = (P * nrom)(*[Y.data_ptr() for Y in outs])
    t = None
    if tune is not None:
        t = cr_tune(int(tune.get("variant", 0)), int(tune.get("grid_per_cu", 0)), int(tune.get("nb", 0)),
                    int(tune.get("refine", 0)))
    info = cr_sweep_info()
    st = lib.cr_sweep_batched(ctx.h, nrom, hs, nfreq, _ptr(om), prec, ys, C.byref(t) if t is not None else None,
                              C.byref(info))
    ctx.check(st)
    return outs, _sweep_info(info)
