"""Learned expansion-point proposer for the greedy rational-Krylov basis (Section 3.3).

The greedy picks the candidate of largest ROM residual as the next expansion point. The proposer
is a small network that looks at the whole residual curve (and a few geometry parameters of the
model) and proposes a point instead; the greedy's residual-max choice stays the fallback
(proposal rejected when its residual is below 0.1 of the maximum) and the stopping test.

Training data come from the method itself: greedy runs with a one-step look-ahead
(cr_greedy_opts.lookahead) try the K largest residual peaks at every iteration, each on a copy of
the basis, and record the maximum residual each would leave. The label of the state (residual
curve after the iteration, used points, geometry) is the peak that leaves the smallest maximum.
The network is trained on the GPU by the library's own forward/backward/Adam kernels
(cr_mlp_train_step) and judged by the number of expansion points -- full-order factorisations
and block solves -- that the greedy needs to reach the tolerance with and without it.

    python -m paper_2310_04734_amd.proposer --out DIR [--variants 64] [--lookahead 8]

generates the seeded fuselage variants, collects the look-ahead data on the 48 training variants,
trains, evaluates both policies on the 16 test variants and writes DIR/proposer_weights.npy,
DIR/proposer_data.npz and DIR/proposer_eval.json.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import CR_FP64, CR_POLICY_GREEDY, CR_POLICY_MLP, Context, Mlp, assemble, mlp_features

WEIGHTS = os.path.join(os.path.dirname(__file__), "data", "proposer_fuselage.npy")


def _log(msg):
    print(msg, flush=True)


def build_system(ctx, w):
    s = assemble(ctx, w.mesh, w.loads, w.receivers)
    s.analyse()
    return s


def greedy_run(ctx, w, geom, policy=CR_POLICY_GREEDY, mlp=None, lookahead=0, prec=CR_FP64, sys_=None):
    """One greedy basis build on workload w; returns (trace, info dict, seconds)."""
    s = sys_ if sys_ is not None else build_system(ctx, w)
    r = w.rom
    t0 = time.perf_counter()
    b = s.basis_greedy(r["band_hz"], r["n_cand"], r["blocks"], r["tol"], r["max_shifts"], prec=prec,
                       policy=policy, mlp=mlp, geom=geom, lookahead=lookahead)
    dt = time.perf_counter() - t0
    return b.trace, dict(b.info), dt


def samples_from_trace(tr, geom):
    """(X, mask, label) rows of one look-ahead trace: one row per iteration that tried peaks."""
    X, M, Y = [], [], []
    used = tr["shift_idx"]
    for it in range(len(used)):
        cands, vals = tr["la_cand"][it], tr["la_res"][it]
        ok = (cands >= 0) & (vals >= 0)
        if not ok.any():
            continue
        k = int(np.argmin(np.where(ok, vals, np.inf)))
        x, m = mlp_features(tr["res_hist"][it], used[:it + 1], geom)
        if m[cands[k]] == 0:
            continue
        X.append(x)
        M.append(m)
        Y.append(int(cands[k]))
    return X, M, Y


def collect(ctx, variants, idx, lookahead=8, prec=CR_FP64):
    X, M, Y, stats = [], [], [], []
    for j, m in enumerate(idx):
        w, geom = variants[m]
        t0 = time.perf_counter()
        tr, info, _ = greedy_run(ctx, w, geom, lookahead=lookahead, prec=prec)
        x, mk, y = samples_from_trace(tr, geom)
        X += x
        M += mk
        Y += y
        agree = float(np.mean([y_ == s_ for y_, s_ in zip(y, tr["shift_idx"][1:])])) if y else 0.0
        stats.append(dict(variant=int(m), shifts=int(len(tr["shift_idx"])), samples=len(y), greedy_agrees=agree))
        _log(f"collect {j + 1}/{len(idx)} variant {m}: n={w.mesh.coords.shape[0]} nodes, {len(tr['shift_idx'])} "
             f"shifts, {len(y)} samples, label=greedy {agree:.2f}, {time.perf_counter() - t0:.1f} s")
    return np.array(X, np.float32), np.array(M, np.float32), np.array(Y, np.int32), stats


def train(ctx, X, M, Y, epochs=300, batch=64, lr=1e-3, seed=2310047347007):
    """Adam on minibatches drawn in a seeded order; returns the network and the loss history."""
    import torch
    from workloads.rng import SplitMix64
    net = Mlp(ctx, n_in=X.shape[1], hidden=256, n_out=M.shape[1], seed=seed)
    dev = ctx.device
    Xd = torch.from_numpy(X).to(dev)
    Md = torch.from_numpy(M).to(dev)
    Yd = torch.from_numpy(Y).to(dev)
    rng = SplitMix64(seed + 1)
    hist = []
    n = X.shape[0]
    for ep in range(epochs):
        order = rng.sample(np.arange(n), n)
        tot = 0.0
        for s0 in range(0, n, batch):
            sel = torch.from_numpy(np.ascontiguousarray(order[s0:s0 + batch], np.int64)).to(dev)
            tot += net.train_step(Xd[sel], Yd[sel], Md[sel], lr=lr) * len(sel)
        hist.append(tot / n)
        if ep % 50 == 0 or ep == epochs - 1:
            _log(f"train epoch {ep}: loss {hist[-1]:.4f}")
    return net, hist


def accuracy(net, X, M, Y):
    import torch
    lg = net.forward(torch.from_numpy(X).to(net.ctx.device)).cpu().numpy()
    lg = np.where(M > 0, lg, -np.inf)
    return float(np.mean(np.argmax(lg, axis=1) == Y))


def compare(ctx, variants, idx, net, prec=CR_FP64):
    """Shifts (full-order factorisations) to reach the tolerance: greedy vs greedy + proposer."""
    rows = []
    for m in idx:
        w, geom = variants[m]
        s = build_system(ctx, w)
        tg, ig, dg = greedy_run(ctx, w, geom, prec=prec, sys_=s)
        tm, im, dm = greedy_run(ctx, w, geom, policy=CR_POLICY_MLP, mlp=net, prec=prec, sys_=s)
        tol = w.rom["tol"]
        rows.append(dict(variant=int(m), greedy_shifts=int(len(tg["shift_idx"])), mlp_shifts=int(len(tm["shift_idx"])),
                         greedy_converged=bool(tg["max_res"][-1] <= tol), mlp_converged=bool(tm["max_res"][-1] <= tol),
                         greedy_maxres=float(tg["max_res"][-1]), mlp_maxres=float(tm["max_res"][-1]),
                         greedy_factorizations=int(len(tg["shift_idx"]) + ig["fp64_refactorizations"]),
                         mlp_factorizations=int(len(tm["shift_idx"]) + im["fp64_refactorizations"]),
                         greedy_block_solves=int(len(tg["shift_idx"]) * w.rom["blocks"]),
                         mlp_block_solves=int(len(tm["shift_idx"]) * w.rom["blocks"]),
                         greedy_q=int(ig["q"]), mlp_q=int(im["q"]), mlp_accepted=int(tm["mlp_used"].sum()),
                         greedy_s=dg, mlp_s=dm))
        _log(f"compare variant {m}: greedy {rows[-1]['greedy_shifts']} shifts ({dg:.2f} s), proposer "
             f"{rows[-1]['mlp_shifts']} shifts ({dm:.2f} s, {rows[-1]['mlp_accepted']} accepted)")
    return rows


def load_trained(ctx, path=WEIGHTS):
    p = np.load(path, allow_pickle=False)
    net = Mlp(ctx, n_in=259, hidden=256, n_out=256)
    net.set_params(p)
    return net


def main(argv=None):
    import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--variants", type=int, default=64)
    ap.add_argument("--lookahead", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=150)
    ap.add_argument("--n-core", type=int, default=6)
    ap.add_argument("--n-ring", type=int, default=3)
    ap.add_argument("--h-z", type=float, default=0.25)
    ap.add_argument("--limit-train", type=int, default=0)
    a = ap.parse_args(argv)
    os.makedirs(a.out, exist_ok=True)
    ctx = Context(0)
    variants, tr_idx, te_idx = W.fuselage_variants(n_var=a.variants, n_core=a.n_core, n_ring=a.n_ring, h_z=a.h_z)
    if a.limit_train:
        tr_idx = tr_idx[:a.limit_train]
    t0 = time.perf_counter()
    X, M, Y, cstats = collect(ctx, variants, tr_idx, lookahead=a.lookahead)
    t_collect = time.perf_counter() - t0
    np.savez(os.path.join(a.out, "proposer_data.npz"), X=X, M=M, Y=Y)
    _log(f"collected {len(Y)} samples in {t_collect:.1f} s")
    t0 = time.perf_counter()
    net, hist = train(ctx, X, M, Y, epochs=a.epochs)
    t_train = time.perf_counter() - t0
    np.save(os.path.join(a.out, "proposer_weights.npy"), net.get_params())
    acc = accuracy(net, X, M, Y)
    rows = compare(ctx, variants, te_idx, net)
    res = dict(samples=int(len(Y)), collect_s=t_collect, train_s=t_train, train_loss_first=hist[0],
               train_loss_last=hist[-1], train_accuracy=acc, collect=cstats, test=rows,
               greedy_shifts=int(sum(r["greedy_shifts"] for r in rows)),
               mlp_shifts=int(sum(r["mlp_shifts"] for r in rows)),
               mesh=dict(n_core=a.n_core, n_ring=a.n_ring, h_z=a.h_z), lookahead=a.lookahead)
    with open(os.path.join(a.out, "proposer_eval.json"), "w") as f:
        json.dump(res, f, indent=1)
    _log(f"test variants: greedy {res['greedy_shifts']} shifts, proposer {res['mlp_shifts']} shifts "
         f"(converged {sum(r['greedy_converged'] for r in rows)} / {sum(r['mlp_converged'] for r in rows)} of "
         f"{len(rows)}); train accuracy {acc:.3f}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
