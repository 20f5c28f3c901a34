// Symbolic analysis for the multifrontal LU: nested-dissection ordering by coordinate
// bisection with vertex separators, assembly tree, front index sets, and the maps the numeric
// kernels use (original-entry scatter, child contribution -> parent positions).
//
// The pattern of A = K - w^2 M is structurally symmetric (the coupling appears as -C in K and
// rho0 C^T in M), so one tree serves every expansion point; the analysis is done once per
// pattern and reused for all shifts, as the paper reuses its symbolic phase across frequencies.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>

#include "internal.h"

namespace cr {
namespace {

constexpr int kLeaf = 48;   // stop bisecting below this many vertices

struct Builder {
    int64_t n;
    const std::vector<int64_t>& rowptr;
    const std::vector<int32_t>& col;
    const std::vector<double>& xyz;
    std::vector<int32_t> order;             // elimination order (new -> old), appended in postorder
    std::vector<int32_t> sn_first, sn_npiv, sn_parent;
    std::vector<std::vector<int32_t>> sn_children;
    std::vector<char> side;                 // scratch marks

    Builder(int64_t n_, const std::vector<int64_t>& rp, const std::vector<int32_t>& c, const std::vector<double>& x)
        : n(n_), rowptr(rp), col(c), xyz(x), side(n_, 0) {}

    int add_supernode(const std::vector<int32_t>& verts, const std::vector<int>& kids) {
        int id = (int)sn_first.size();
        sn_first.push_back((int32_t)order.size());
        sn_npiv.push_back((int32_t)verts.size());
        sn_parent.push_back(-1);
        sn_children.push_back({});
        for (int k : kids) { sn_parent[k] = id; sn_children[id].push_back(k); }
        order.insert(order.end(), verts.begin(), verts.end());
        return id;
    }

    // returns the supernode id of the subtree root (or -1 when verts is empty)
    int dissect(std::vector<int32_t> verts) {
        if (verts.empty()) return -1;
        if ((int)verts.size() <= kLeaf || xyz.empty()) {
            if (xyz.empty() && (int)verts.size() > kLeaf) return dissect_bfs(std::move(verts));
            return add_supernode(verts, {});
        }
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int32_t v : verts)
            for (int d = 0; d < 3; ++d) { lo[d] = std::min(lo[d], xyz[3 * v + d]); hi[d] = std::max(hi[d], xyz[3 * v + d]); }
        int axes[3] = {0, 1, 2};
        std::sort(axes, axes + 3, [&](int a, int b) { return hi[a] - lo[a] > hi[b] - lo[b]; });
        for (int t = 0; t < 3; ++t) {
            int ax = axes[t];
            if (!(hi[ax] > lo[ax])) break;
            std::vector<double> cs(verts.size());
            for (size_t i = 0; i < verts.size(); ++i) cs[i] = xyz[3 * verts[i] + ax];
            std::vector<double> sorted = cs;
            std::nth_element(sorted.begin(), sorted.begin() + sorted.size() / 2, sorted.end());
            double med = sorted[sorted.size() / 2];
            double tol = 1e-9 * (hi[ax] - lo[ax]);
            // 1 = left (x < med), 2 = right (x > med), 3 = on the median plane
            for (size_t i = 0; i < verts.size(); ++i)
                side[verts[i]] = cs[i] < med - tol ? 1 : (cs[i] > med + tol ? 2 : 3);
            std::vector<int32_t> L, R, S;
            for (int32_t v : verts) {
                if (side[v] == 3) { S.push_back(v); continue; }
                if (side[v] == 2) { R.push_back(v); continue; }
                bool touches = false;   // left vertex adjacent to the right side joins the separator
                for (int64_t k = rowptr[v]; k < rowptr[v + 1] && !touches; ++k) touches = side[col[k]] == 2;
                if (touches) S.push_back(v); else L.push_back(v);
            }
            for (int32_t v : verts) side[v] = 0;
            if (L.empty() || R.empty() || S.size() * 2 > verts.size()) continue;
            int a = dissect(std::move(L));
            int b = dissect(std::move(R));
            std::vector<int> kids;
            if (a >= 0) kids.push_back(a);
            if (b >= 0) kids.push_back(b);
            return add_supernode(S, kids);
        }
        return add_supernode(verts, {});
    }

    // graph bisection by breadth-first level sets when no coordinates are known
    int dissect_bfs(std::vector<int32_t> verts) {
        for (int32_t v : verts) side[v] = 1;
        std::vector<int32_t> dist(0);
        std::vector<int32_t> lev(n, -1), q;
        auto bfs = [&](int32_t s) {
            for (int32_t v : verts) lev[v] = -1;
            q.assign(1, s);
            lev[s] = 0;
            for (size_t h = 0; h < q.size(); ++h) {
                int32_t v = q[h];
                for (int64_t k = rowptr[v]; k < rowptr[v + 1]; ++k) {
                    int32_t u = col[k];
                    if (side[u] == 1 && lev[u] < 0) { lev[u] = lev[v] + 1; q.push_back(u); }
                }
            }
            return q.back();
        };
        int32_t far = bfs(bfs(verts[0]));
        (void)far;
        int maxl = lev[q.back()];
        std::vector<int32_t> L, R, S, rest;
        if ((int)q.size() < (int)verts.size()) {   // disconnected: split off the reached part
            for (int32_t v : verts) (lev[v] >= 0 ? L : R).push_back(v);
            for (int32_t v : verts) side[v] = 0;
            int a = dissect(std::move(L)), b = dissect(std::move(R));
            std::vector<int> kids;
            if (a >= 0) kids.push_back(a);
            if (b >= 0) kids.push_back(b);
            return add_supernode({}, kids);
        }
        std::vector<int> cnt(maxl + 1, 0);
        for (int32_t v : verts) cnt[lev[v]]++;
        int half = (int)verts.size() / 2, acc = 0, mid = 0;
        for (int l = 0; l <= maxl; ++l) { acc += cnt[l]; if (acc >= half) { mid = l; break; } }
        for (int32_t v : verts) (lev[v] < mid ? L : (lev[v] == mid ? S : R)).push_back(v);
        for (int32_t v : verts) side[v] = 0;
        if (L.empty() || R.empty()) return add_supernode(verts, {});
        int a = dissect(std::move(L)), b = dissect(std::move(R));
        std::vector<int> kids;
        if (a >= 0) kids.push_back(a);
        if (b >= 0) kids.push_back(b);
        return add_supernode(S, kids);
    }
};

}  // namespace

std::unique_ptr<Symbolic> analyse_pattern(int64_t n, const std::vector<int64_t>& rowptr,
                                          const std::vector<int32_t>& col, const std::vector<double>& coords,
                                          const FrontClasses& fc) {
    auto t0 = std::chrono::steady_clock::now();
    CR_REQUIRE(n > 0 && (int64_t)rowptr.size() == n + 1, CR_E_INVALID, "analyse: bad pattern");
    Builder b(n, rowptr, col, coords);
    std::vector<int32_t> all(n);
    std::iota(all.begin(), all.end(), 0);
    int root = b.dissect(all);
    (void)root;
    CR_REQUIRE((int64_t)b.order.size() == n, CR_E_INVALID, "analyse: ordering lost vertices");

    auto sym = std::make_unique<Symbolic>();
    Symbolic& S = *sym;
    S.n = n;
    S.perm = b.order;
    S.iperm.assign(n, -1);
    for (int64_t i = 0; i < n; ++i) S.iperm[S.perm[i]] = (int32_t)i;
    const int nf = (int)b.sn_first.size();
    S.nfront = nf;
    S.first = b.sn_first;
    S.npiv = b.sn_npiv;
    S.parent = b.sn_parent;
    // supernodes are created in postorder (children before parents) by construction
    std::vector<int32_t> snode_of(n);
    for (int f = 0; f < nf; ++f)
        for (int k = 0; k < S.npiv[f]; ++k) snode_of[S.first[f] + k] = f;
    // contribution index sets
    std::vector<std::vector<int32_t>> cb(nf);
    std::vector<int32_t> mark(n, -1);
    for (int f = 0; f < nf; ++f) {
        int32_t end = S.first[f] + S.npiv[f];
        std::vector<int32_t>& out = cb[f];
        for (int k = 0; k < S.npiv[f]; ++k) {
            int32_t old = S.perm[S.first[f] + k];
            for (int64_t p = rowptr[old]; p < rowptr[old + 1]; ++p) {
                int32_t j = S.iperm[col[p]];
                if (j >= end && mark[j] != f) { mark[j] = f; out.push_back(j); }
            }
        }
        for (int c : b.sn_children[f])
            for (int32_t j : cb[c])
                if (j >= end && mark[j] != f) { mark[j] = f; out.push_back(j); }
        std::sort(out.begin(), out.end());
    }
    // children CSR, levels
    S.child_off.assign(nf + 1, 0);
    for (int f = 0; f < nf; ++f) S.child_off[f + 1] = S.child_off[f] + (int32_t)b.sn_children[f].size();
    S.child_list.reserve(S.child_off[nf]);
    for (int f = 0; f < nf; ++f)
        for (int c : b.sn_children[f]) S.child_list.push_back(c);
    S.level.assign(nf, 0);
    for (int f = 0; f < nf; ++f)
        for (int c : b.sn_children[f]) S.level[f] = std::max(S.level[f], S.level[c] + 1);
    S.nlevel = 0;
    for (int f = 0; f < nf; ++f) S.nlevel = std::max(S.nlevel, S.level[f] + 1);
    S.level_off.assign(S.nlevel + 1, 0);
    for (int f = 0; f < nf; ++f) S.level_off[S.level[f] + 1]++;
    for (int l = 0; l < S.nlevel; ++l) S.level_off[l + 1] += S.level_off[l];
    S.level_fronts.assign(nf, 0);
    {
        std::vector<int32_t> pos(S.level_off.begin(), S.level_off.end() - 1);
        for (int f = 0; f < nf; ++f) S.level_fronts[pos[S.level[f]]++] = f;
    }
    // front index lists, arena offsets, statistics
    S.fsize.resize(nf);
    S.idx_off.resize(nf + 1);
    S.front_off.resize(nf + 1);
    S.idx_off[0] = 0;
    S.front_off[0] = 0;
    S.factor_entries = 0;
    S.factor_flops = 0;
    for (int f = 0; f < nf; ++f) {
        int32_t p = S.npiv[f], c = (int32_t)cb[f].size(), m = p + c;
        S.fsize[f] = m;
        S.idx_off[f + 1] = S.idx_off[f] + m;
        S.front_off[f + 1] = S.front_off[f] + (int64_t)m * m;
        S.max_front = std::max(S.max_front, m);
        S.max_piv = std::max(S.max_piv, p);
        S.max_children = std::max(S.max_children, S.child_off[f + 1] - S.child_off[f]);
        S.factor_entries += (int64_t)m * m - (int64_t)c * c;
        for (int k = 0; k < p; ++k) {
            double r = m - k - 1;
            S.factor_flops += 8.0 * r * r + 8.0 * r;   // rank-1 update + column scaling (complex)
        }
        CR_REQUIRE((int64_t)m * m < (int64_t)INT32_MAX, CR_E_UNSUPPORTED, "front too large for 32-bit local indices");
    }
    S.arena = S.front_off[nf];
    S.idx.resize(S.idx_off[nf]);
    for (int f = 0; f < nf; ++f) {
        int32_t* dst = S.idx.data() + S.idx_off[f];
        for (int k = 0; k < S.npiv[f]; ++k) dst[k] = S.first[f] + k;
        std::copy(cb[f].begin(), cb[f].end(), dst + S.npiv[f]);
    }
    // local position of a global (new) index inside front f
    auto local = [&](int f, int32_t j) -> int32_t {
        if (j >= S.first[f] && j < S.first[f] + S.npiv[f]) return j - S.first[f];
        const std::vector<int32_t>& v = cb[f];
        auto it = std::lower_bound(v.begin(), v.end(), j);
        if (it == v.end() || *it != j) throw Error(CR_E_INVALID, "analyse: index missing from front");
        return S.npiv[f] + (int32_t)(it - v.begin());
    };
    // child contribution rows -> parent local positions
    S.cmap_off.assign(nf + 1, 0);
    for (int f = 0; f < nf; ++f) S.cmap_off[f + 1] = S.cmap_off[f] + (int64_t)cb[f].size();
    S.cmap.resize(S.cmap_off[nf]);
    for (int f = 0; f < nf; ++f) {
        int par = S.parent[f];
        if (par < 0) {
            CR_REQUIRE(cb[f].empty(), CR_E_INVALID, "analyse: root with contribution rows");
            continue;
        }
        for (size_t r = 0; r < cb[f].size(); ++r) S.cmap[S.cmap_off[f] + r] = local(par, cb[f][r]);
    }
    // original entries: (i, j) in new numbering belongs to the front of min(i, j)
    std::vector<int64_t> cnt(nf + 1, 0);
    const int64_t nnz = rowptr[n];
    for (int64_t r = 0; r < n; ++r)
        for (int64_t p = rowptr[r]; p < rowptr[r + 1]; ++p) {
            int32_t i = S.iperm[r], j = S.iperm[col[p]];
            cnt[snode_of[std::min(i, j)] + 1]++;
        }
    for (int f = 0; f < nf; ++f) cnt[f + 1] += cnt[f];
    S.ent_off = cnt;
    S.ent_src.resize(nnz);
    S.ent_dst.resize(nnz);
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t r = 0; r < n; ++r)
        for (int64_t p = rowptr[r]; p < rowptr[r + 1]; ++p) {
            int32_t i = S.iperm[r], j = S.iperm[col[p]];
            int f = snode_of[std::min(i, j)];
            int64_t k = pos[f]++;
            S.ent_src[k] = p;
            S.ent_dst[k] = local(f, i) + local(f, j) * S.fsize[f];
        }
    S.piv_off.assign(S.first.begin(), S.first.end());
    // large fronts: factored by 16-column panels with deferred 128-column trailing GEMMs spread
    // over many workgroups; per level the list of large fronts and the number of panel steps
    constexpr int kPanel = 16;
    S.big.assign(nf, 0);
    S.big_off.assign(S.nlevel + 1, 0);
    S.nsteps.assign(S.nlevel, 0);
    S.huge.assign(nf, 0);
    S.huge_off.assign(S.nlevel + 1, 0);
    S.huge_piv.assign(S.nlevel, 0);
    S.wide_solve.clear();
    for (int l = 0; l < S.nlevel; ++l) {
        int steps = 0;
        for (int q = S.level_off[l]; q < S.level_off[l + 1]; ++q) {
            const int f = S.level_fronts[q];
            if (S.fsize[f] >= fc.big_m && S.npiv[f] > 0) {
                S.big[f] = 1;
                S.big_list.push_back(f);
                steps = std::max(steps, (S.npiv[f] + kPanel - 1) / kPanel);
                // trailing GEMM after each 128-column block (kOB of the GEMM kernel): 8 (m - K1)^2 (K1 - K0) flops
                for (int K0 = 0; K0 < S.npiv[f]; K0 += 128) {
                    const double K1 = std::min(K0 + 128, S.npiv[f]), r = S.fsize[f] - K1;
                    S.gemm_flops += 8.0 * r * r * (K1 - K0);
                }
            }
            if (S.fsize[f] >= fc.huge_m && S.npiv[f] > 0) {
                S.huge[f] = 1;
                S.huge_list.push_back(f);
                S.huge_piv[l] = std::max(S.huge_piv[l], S.npiv[f]);
            }
        }
        S.big_off[l + 1] = (int32_t)S.big_list.size();
        S.huge_off[l + 1] = (int32_t)S.huge_list.size();
        S.nsteps[l] = steps;
        // levels whose one-workgroup solves carry large triangles get 1024-thread workgroups:
        // bit 0 for solves with several right-hand sides (m p >= 32768; below that the MFMA
        // kernels' register spills at 1024 threads cost more than the extra waves gain), bit 1
        // for single right-hand sides (m p >= 4096)
        double work = 0;
        for (int q = S.level_off[l]; q < S.level_off[l + 1]; ++q) {
            const int f = S.level_fronts[q];
            if (!S.huge[f]) work = std::max(work, (double)S.fsize[f] * S.npiv[f]);
        }
        S.wide_solve.push_back((work >= 32768.0 ? 1 : 0) | (work >= 4096.0 ? 2 : 0));
    }
    S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return sym;
}

}  // namespace cr
