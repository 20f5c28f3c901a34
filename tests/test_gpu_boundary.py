"""The rest of the C ABI through the binding: CSR import (with and without coordinates, duplicate
and unsorted entries), full-field recovery from reduced states, the allocator hook, the
second-order (damped) basis against the oracle, and every status code the library returns that
can be forced from the host without faulting the GPU."""
import ctypes as C

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import assembly, krylov, rom, soar, solve

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _flush(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def P():
    import paper_2310_04734_amd as P
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    return P


@pytest.fixture(scope="module")
def ctx(P):
    return P.Context(0)


@pytest.fixture(scope="module")
def small():
    w = W.small_plate_cavity()
    return w, assembly.assemble(w.mesh, w.loads, w.receivers)


def _csr(A):
    A = A.tocsr()
    A.sort_indices()
    return A


def _import(P, ctx, s, D=None, coords=None, shuffle=False):
    K, M = _csr(s["K"]), _csr(s["M"])
    Dm = _csr(D) if D is not None else None
    pat = (abs(K) + abs(M) + (abs(Dm) if Dm is not None else 0)).tocsr()
    pat.sort_indices()
    rows = np.repeat(np.arange(pat.shape[0]), np.diff(pat.indptr))
    cols = pat.indices
    kv = np.asarray(K[rows, cols]).ravel()
    mv = np.asarray(M[rows, cols]).ravel()
    dv = np.asarray(Dm[rows, cols]).ravel() if Dm is not None else None
    rowptr = pat.indptr.astype(np.int64)
    if shuffle:
        # every entry split into two halves stored as duplicates, columns in reverse order per row
        rp, cc, kk, mm, dd = [0], [], [], [], []
        for r in range(pat.shape[0]):
            sl = slice(rowptr[r], rowptr[r + 1])
            for c, a, b, e in zip(cols[sl][::-1], kv[sl][::-1], mv[sl][::-1],
                                  (dv[sl][::-1] if dv is not None else [None] * (rowptr[r + 1] - rowptr[r]))):
                for part in (0.25, 0.75):
                    cc.append(c)
                    kk.append(a * part)
                    mm.append(b * part)
                    dd.append(e * part if e is not None else 0)
            rp.append(len(cc))
        rowptr, cols, kv, mv = np.array(rp), np.array(cc), np.array(kk), np.array(mm)
        dv = np.array(dd) if dv is not None else None
    return P.import_csr(ctx, rowptr, cols, kv, mv, s["F"], s["flags"], s["recv"], D=dv, coords=coords)


def _backward_error(A, x, b):
    r = b - A @ x
    return np.abs(r).max() / (abs(A).sum(axis=1).max() * np.abs(x).max() + np.abs(b).max())


@pytest.mark.parametrize("shuffle", [False, True])
def test_import_csr_factor_solve(P, ctx, small, shuffle):
    """An imported system (no coordinates: graph bisection) solves like the oracle's SuperLU."""
    _flush(f"import csr shuffle={shuffle}")
    w, s = small
    g = _import(P, ctx, s, shuffle=shuffle)
    assert (g.n, g.L, g.n_o, g.n_u) == (s["K"].shape[0], 1, len(s["recv"]), 0)
    e = g.export()
    Kg = sp.csr_matrix((e["K"], e["col"], e["rowptr"]), shape=(g.n, g.n))
    assert abs(Kg - s["K"]).max() <= 1e-14 * abs(s["K"]).max()
    g.analyse()
    om = 2 * np.pi * 171.0
    b = solve.load_at(s["F"], s["flags"], om)
    x = g.factor(om, P.CR_FP64).solve(torch.from_numpy(b).to(ctx.device)).cpu().numpy()
    A = (s["K"] - om ** 2 * s["M"]).tocsr()
    assert _backward_error(A, x, b) <= 1e-14
    xo = solve.full_solve(s["K"], s["M"], s["F"], s["flags"], om)
    assert np.abs(x - xo).max() <= 1e-6 * np.abs(xo).max()


def test_recover_field_from_reduced_states(P, ctx):
    """x = S V x_R: at an expansion point the recovered field equals the full solve (moment
    matching of order zero), and its receiver rows equal the sweep's outputs."""
    _flush("recover field")
    w = W.box()
    s = assembly.assemble(w.mesh, w.loads, w.receivers)
    g = P.assemble(ctx, w.mesh, w.loads, w.receivers)
    g.analyse()
    shifts = 2 * np.pi * w.rom["shifts_hz"]
    B = g.basis(shifts, w.rom["blocks"], prec=P.CR_FP64)
    R = B.project()
    oms = np.array([shifts[1], 2 * np.pi * 123.4])
    XR = R.sweep_states(oms, prec=P.CR_FP64)                 # nfreq x L x q
    Y = R.sweep(oms, prec=P.CR_FP64).cpu().numpy()
    assert XR.shape == (2, 1, B.q)
    for k, om in enumerate(oms):
        X = B.recover(XR[k].t()).cpu().numpy()               # n x L
        assert np.abs(X[s["recv"], 0] - Y[k, 0]).max() <= 1e-12 * np.abs(Y[k, 0]).max()
        if k == 0:
            xo = solve.full_solve(s["K"], s["M"], s["F"], s["flags"], om)
            assert np.abs(X - xo).max() <= 1e-8 * np.abs(xo).max()
    # the oracle's own lift of the same states with the exported basis
    V = B.V().cpu().numpy()
    Xo = krylov.jacobi_scaled(s)["scale"][:, None] * (V @ XR[1].t().cpu().numpy())
    assert np.abs(B.recover(XR[1].t()).cpu().numpy() - Xo).max() <= 1e-12 * np.abs(Xo).max()


def test_allocator_hook_and_oom(P):
    """Every device buffer of a context comes from its allocator and goes back to it; an
    allocator that returns nothing makes the call fail with CR_E_OOM."""
    _flush("allocator hook")
    hip = C.CDLL("libamdhip64.so")
    live, count = {}, [0]

    def alloc(nbytes):
        p = C.c_void_p()
        if hip.hipMalloc(C.byref(p), C.c_size_t(nbytes)) != 0:
            return 0
        live[p.value] = nbytes
        count[0] += 1
        return p.value

    def free(ptr):
        assert ptr in live
        del live[ptr]
        hip.hipFree(C.c_void_p(ptr))

    w = W.box()
    c = P.Context(0, allocator=(alloc, free))
    g = P.assemble(c, w.mesh, w.loads, w.receivers)
    g.analyse()
    R = g.basis(2 * np.pi * w.rom["shifts_hz"], w.rom["blocks"], prec=P.CR_FP64).project()
    Y = R.sweep(w.omegas[:50], prec=P.CR_FP64)
    torch.cuda.synchronize()
    assert count[0] > 10 and len(live) > 0
    del R, g
    c.close()
    assert not live, f"{len(live)} buffers not returned"
    c2 = P.Context(0, allocator=(lambda n: 0, lambda p: None))
    with pytest.raises(P.CabinRomError) as e:
        P.assemble(c2, w.mesh, w.loads, w.receivers)
    assert e.value.name == "CR_E_OOM"
    assert torch.isfinite(torch.view_as_real(Y)).all()


def test_damped_second_order_basis_matches_oracle(P, ctx, small):
    """Structure-only Rayleigh damping imported as D: the second-order basis (Eq. (9)) spans the
    oracle's space, and the damped reduced model's outputs agree within 1e-6."""
    _flush("second-order basis")
    w, s = small
    sd = soar.rayleigh(s, 40.0, 2e-5, structure_only=True)
    coords = None
    g = _import(P, ctx, s, D=sd["D"], coords=coords)
    g.analyse()
    shifts = 2 * np.pi * np.array([60.0, 250.0])
    k = 4
    B = g.basis(shifts, k, prec=P.CR_FP64)
    ss = soar.jacobi_scaled_d(sd)
    rb = soar.build_basis(ss, shifts, k)
    assert B.q == rb.q == 8
    import scipy.linalg as sla
    sv = sla.svdvals(rb.basis.conj().T @ B.V().cpu().numpy())
    assert sv.min() > 1 - 1e-8
    R = B.project()
    ro = soar.project(ss, rb.basis)
    om = 2 * np.pi * np.linspace(10, 400, 97)
    Y = R.sweep(om, prec=P.CR_FP64).cpu().numpy()
    assert rom.relative_error(Y, rom.sweep(ro, om, DR=ro["DR"])).max() <= 1e-6
    for wj in shifts:
        y = soar.full_solve(sd, wj)[s["recv"]].T[None]
        assert rom.relative_error(R.sweep([wj], prec=P.CR_FP64).cpu().numpy(), y).max() < 1e-8


def test_status_codes(P, ctx, small):
    """Each status the library reports, forced from the host."""
    _flush("status codes")
    w, s = small
    # CR_E_SINGULAR: K = M = I imported, factored at w = 1 rad/s (A = 0)
    n = 3
    I3 = sp.identity(n, format="csr", dtype=complex)
    g = P.import_csr(ctx, I3.indptr, I3.indices, I3.data, I3.data, np.ones((n, 1)), [0], [0])
    with pytest.raises(P.CabinRomError) as e:
        g.factor(1.0, P.CR_FP64)
    assert e.value.name == "CR_E_STATE"          # factor before analyse
    g.analyse()
    with pytest.raises(P.CabinRomError) as e:
        g.factor(1.0, P.CR_FP64)
    assert e.value.name == "CR_E_SINGULAR"
    # a zero pivot is perturbed (counted) and refinement then cannot converge
    Kd = sp.diags([1.0, 4.0, 9.0]).tocsr().astype(complex)
    g2 = P.import_csr(ctx, Kd.indptr, Kd.indices, Kd.data, I3.data, np.ones((n, 1)), [0], [0])
    g2.analyse()
    f = g2.factor(1.0, P.CR_FP64)
    assert f.n_perturbed == 1
    with pytest.raises(P.CabinRomError) as e:
        f.solve(torch.ones(n, 1, dtype=torch.complex128, device=ctx.device))
    assert e.value.name == "CR_E_NOT_CONVERGED"
    x = f.solve(torch.tensor([[0.0], [1.0], [1.0]], dtype=torch.complex128, device=ctx.device))
    assert np.allclose(x.cpu().numpy().ravel(), [0.0, 1 / 3, 1 / 8], rtol=1e-14)
    # CR_E_NOT_CONVERGED: one refinement step cannot reach 1e-15 from a complex-FP32 factor
    gp = P.assemble(ctx, w.mesh, w.loads, w.receivers)
    gp.analyse()
    om = 2 * np.pi * 211.0
    fac = gp.factor(om, P.CR_MIXED)
    b = torch.from_numpy(solve.load_at(s["F"], s["flags"], om)).to(ctx.device)
    with pytest.raises(P.CabinRomError) as e:
        fac.solve(b, max_iter=1, tol=1e-15)
    assert e.value.name == "CR_E_NOT_CONVERGED"
    # CR_E_INVALID: bad arguments
    with pytest.raises(P.CabinRomError) as e:
        P.import_csr(ctx, [0, 1], [5], [1.0], [1.0], np.ones((1, 1)), [0], [0])
    assert e.value.name == "CR_E_INVALID"
    with pytest.raises(P.CabinRomError) as e:
        gp.factor(float("nan"), P.CR_FP64)
    assert e.value.name == "CR_E_INVALID"
    with pytest.raises(P.CabinRomError) as e:
        gp.basis(np.zeros(0), 1, prec=P.CR_FP64)
    assert e.value.name == "CR_E_INVALID"
    with pytest.raises(P.CabinRomError) as e:
        gp.basis([om], 1, prec=7)
    assert e.value.name == "CR_E_INVALID"
    R = gp.basis([om], 2, prec=P.CR_FP64).project()
    with pytest.raises(P.CabinRomError) as e:
        R.sweep([float("inf")], prec=P.CR_FP64)
    assert e.value.name == "CR_E_INVALID"
    with pytest.raises(P.CabinRomError) as e:
        P.Rom.from_arrays(ctx, np.zeros((0, 0)), np.zeros((0, 0)), np.zeros((0, 1)), np.zeros((1, 0)), [0])
    assert e.value.name == "CR_E_INVALID"
    # CR_E_STATE: front classes after the analysis
    with pytest.raises(P.CabinRomError) as e:
        gp.set_front_classes(256, 1024)
    assert e.value.name == "CR_E_STATE"
    # CR_E_UNSUPPORTED: greedy on a system with a damping matrix; more than 64 loads in a sweep
    sd = soar.rayleigh(s, 1.0, 0.0)
    gd = _import(P, ctx, s, D=sd["D"])
    gd.analyse()
    with pytest.raises(P.CabinRomError) as e:
        gd.basis_greedy((10.0, 400.0), 16, 2, 1e-6, 2, prec=P.CR_FP64)
    assert e.value.name == "CR_E_UNSUPPORTED"
    q, L = 3, 65
    Rw = P.Rom.from_arrays(ctx, np.eye(q), 1e-6 * np.eye(q), np.ones((q, L)), np.ones((1, q)), np.zeros(L))
    with pytest.raises(P.CabinRomError) as e:
        Rw.sweep([100.0], prec=P.CR_FP64)
    assert e.value.name == "CR_E_UNSUPPORTED"
