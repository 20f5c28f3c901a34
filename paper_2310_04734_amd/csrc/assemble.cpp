// Host finite-element assembly of the coupled structural-acoustic system (paper Section 2,
// Eq. (1)-(3), two-domain subset; complex stiffness damping of Section 3.3) and upload of the
// Jacobi-scaled system to the device.
//
// Blocks: K = [K_s, -C; 0, K_f], M = [M_s, 0; rho0 C^T, M_f], with
//   K_f = int grad N . grad N,  M_f = int N N / (c^2 (1 + i eta_f)),
//   K_s: isotropic elasticity with E~ = E (1 + i eta_s), written per node pair as
//        K_(a,i)(b,j) = int lam d_i N_a d_j N_b + mu d_j N_a d_i N_b + mu delta_ij grad N_a . grad N_b,
//   M_s = rho_s int N_a N_b delta_ij,  C_(a,d) b = int_Gamma N_a n_d N_b (n out of the fluid).
// Trilinear hex8 with 2x2x2 Gauss points (+-1/sqrt 3, weight 1); bilinear quads with 2x2 points.
#include <algorithm>
#include <array>
#include <cmath>
#include <complex>

#include "internal.h"

namespace {

using cplx = std::complex<double>;

const double kG = 0.57735026918962576451;   // 1/sqrt(3)
const int kXi[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                       {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};
const int kXi2[4][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}};

struct HexPoint {
    double N[8];
    double dNdx[8][3];
    double detJ;
};

// shape values and physical gradients of a hex8 at natural point (r, s, t)
HexPoint hex_point(const double X[8][3], double r, double s, double t) {
    HexPoint hp;
    double dN[8][3];
    for (int a = 0; a < 8; ++a) {
        double fr = 1 + r * kXi[a][0], fs = 1 + s * kXi[a][1], ft = 1 + t * kXi[a][2];
        hp.N[a] = 0.125 * fr * fs * ft;
        dN[a][0] = 0.125 * kXi[a][0] * fs * ft;
        dN[a][1] = 0.125 * kXi[a][1] * fr * ft;
        dN[a][2] = 0.125 * kXi[a][2] * fr * fs;
    }
    double J[3][3] = {{0}};   // J[i][j] = d x_j / d xi_i
    for (int a = 0; a < 8; ++a)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) J[i][j] += dN[a][i] * X[a][j];
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                 J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    CR_REQUIRE(det > 0, CR_E_INVALID, "inverted or degenerate hex8 element");
    double inv[3][3];
    inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    for (int a = 0; a < 8; ++a)
        for (int i = 0; i < 3; ++i)
            hp.dNdx[a][i] = inv[i][0] * dN[a][0] + inv[i][1] * dN[a][1] + inv[i][2] * dN[a][2];
    hp.detJ = det;
    return hp;
}

// W[a][b][d] = int N_a N_b n_d dGamma over a bilinear quad (n scaled by the area element)
void quad_integrals(const double X[4][3], double W[4][4][3]) {
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            for (int d = 0; d < 3; ++d) W[a][b][d] = 0;
    for (int gt = 0; gt < 2; ++gt)
        for (int gs = 0; gs < 2; ++gs) {
            double s = gs ? kG : -kG, t = gt ? kG : -kG;
            double N[4], ts[3] = {0, 0, 0}, tt[3] = {0, 0, 0};
            for (int a = 0; a < 4; ++a) {
                double fs = 1 + s * kXi2[a][0], ft = 1 + t * kXi2[a][1];
                N[a] = 0.25 * fs * ft;
                for (int j = 0; j < 3; ++j) {
                    ts[j] += 0.25 * kXi2[a][0] * ft * X[a][j];
                    tt[j] += 0.25 * kXi2[a][1] * fs * X[a][j];
                }
            }
            double n[3] = {ts[1] * tt[2] - ts[2] * tt[1], ts[2] * tt[0] - ts[0] * tt[2],
                           ts[0] * tt[1] - ts[1] * tt[0]};
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b)
                    for (int d = 0; d < 3; ++d) W[a][b][d] += N[a] * N[b] * n[d];
        }
}

struct Pattern {
    int64_t n;
    std::vector<int64_t> rowptr;
    std::vector<int32_t> col;
    // position of (r, c) in CSR; binary search within the row
    int64_t find(int64_t r, int64_t c) const {
        auto b = col.begin() + rowptr[r], e = col.begin() + rowptr[r + 1];
        auto it = std::lower_bound(b, e, (int32_t)c);
        if (it == e || *it != c) throw cr::Error(CR_E_INVALID, "assembly pattern miss");
        return it - col.begin();
    }
};

// sorted unique neighbour lists of nodes from groups of k node ids
std::vector<std::vector<int64_t>> node_adjacency(int64_t n_nodes, const std::vector<const int64_t*>& groups, int k) {
    std::vector<std::vector<int64_t>> adj(n_nodes);
    for (const int64_t* g : groups)
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) adj[g[a]].push_back(g[b]);
    for (auto& v : adj) {
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
    }
    return adj;
}

}  // namespace

extern "C" cr_status cr_assemble(cr_ctx ctx, const cr_mesh* mesh, const cr_material* mats, int32_t nmat,
                                 const cr_load* loads, int32_t nload, const int64_t* recv_nodes,
                                 int32_t n_o, cr_sys* out) {
    if (!ctx) return CR_E_INVALID;
    return cr_guard(ctx, [&] {
        CR_REQUIRE(mesh && mats && out && nmat > 0 && nload >= 0 && n_o >= 0, CR_E_INVALID, "cr_assemble: bad arguments");
        CR_REQUIRE(mesh->n_nodes > 0 && mesh->n_el > 0 && mesh->coords && mesh->elems && mesh->elem_mat,
                   CR_E_INVALID, "cr_assemble: empty mesh");
        CR_REQUIRE(nload == 0 || loads, CR_E_INVALID, "cr_assemble: loads missing");
        CR_REQUIRE(n_o == 0 || recv_nodes, CR_E_INVALID, "cr_assemble: receivers missing");
        const int64_t nn = mesh->n_nodes, ne = mesh->n_el;
        int fluid_mat = -1;
        std::vector<int> term_of(nmat, -1);   // material -> frequency-dependent term
        int nterm = 0;
        for (int m = 0; m < nmat; ++m) {
            CR_REQUIRE(mats[m].kind == CR_FLUID || mats[m].kind == CR_SOLID, CR_E_INVALID, "bad material kind");
            CR_REQUIRE(mats[m].n_eta >= 0 && (mats[m].n_eta == 0 || (mats[m].eta_f_hz && mats[m].eta_val)),
                       CR_E_INVALID, "material loss-factor table missing");
            for (int k = 0; k < mats[m].n_eta; ++k)
                CR_REQUIRE(std::isfinite(mats[m].eta_val[k]) && std::isfinite(mats[m].eta_f_hz[k]) &&
                               (k == 0 || mats[m].eta_f_hz[k] > mats[m].eta_f_hz[k - 1]),
                           CR_E_INVALID, "loss-factor table frequencies must increase");
            if (mats[m].n_eta > 0) {
                CR_REQUIRE(nterm < cr::kMaxTerms, CR_E_UNSUPPORTED, "at most 4 materials with frequency-dependent loss");
                term_of[m] = nterm++;
            }
            if (mats[m].kind == CR_FLUID) {
                CR_REQUIRE(fluid_mat < 0, CR_E_UNSUPPORTED, "exactly one fluid material is supported");
                fluid_mat = m;
            }
        }
        std::vector<char> is_f(nn, 0), is_s(nn, 0), clamped(nn, 0);
        std::vector<const int64_t*> fl_el, so_el;
        for (int64_t e = 0; e < ne; ++e) {
            int m = mesh->elem_mat[e];
            CR_REQUIRE(m >= 0 && m < nmat, CR_E_INVALID, "element material out of range");
            const int64_t* c = mesh->elems + 8 * e;
            for (int a = 0; a < 8; ++a) CR_REQUIRE(c[a] >= 0 && c[a] < nn, CR_E_INVALID, "element node out of range");
            if (mats[m].kind == CR_FLUID) { fl_el.push_back(c); for (int a = 0; a < 8; ++a) is_f[c[a]] = 1; }
            else { so_el.push_back(c); for (int a = 0; a < 8; ++a) is_s[c[a]] = 1; }
        }
        for (int64_t i = 0; i < mesh->n_clamped; ++i) {
            int64_t v = mesh->clamped[i];
            CR_REQUIRE(v >= 0 && v < nn, CR_E_INVALID, "clamped node out of range");
            clamped[v] = 1;
        }
        CR_REQUIRE(mesh->n_iface == 0 || fluid_mat >= 0, CR_E_INVALID, "interface without a fluid");
        // DoF numbering: free solid displacements first, then fluid pressures
        std::vector<int64_t> udof(3 * nn, -1), pdof(nn, -1);
        int64_t nd = 0;
        for (int64_t v = 0; v < nn; ++v)
            if (is_s[v] && !clamped[v]) { for (int d = 0; d < 3; ++d) udof[3 * v + d] = nd++; }
        const int64_t n_u = nd;
        for (int64_t v = 0; v < nn; ++v)
            if (is_f[v]) pdof[v] = nd++;
        const int64_t n = nd;
        CR_REQUIRE(n > 0 && n < (int64_t)INT32_MAX, CR_E_UNSUPPORTED, "DoF count out of range");
        std::vector<const int64_t*> faces;
        for (int64_t f = 0; f < mesh->n_iface; ++f) {
            const int64_t* q = mesh->iface + 4 * f;
            for (int a = 0; a < 4; ++a)
                CR_REQUIRE(q[a] >= 0 && q[a] < nn && is_f[q[a]] && is_s[q[a]], CR_E_INVALID,
                           "interface node must belong to a fluid and a solid element");
            faces.push_back(q);
        }
        auto adj_s = node_adjacency(nn, so_el, 8);
        auto adj_f = node_adjacency(nn, fl_el, 8);
        auto adj_c = node_adjacency(nn, faces, 4);
        // DoF -> node map and the pattern rows
        std::vector<int64_t> dof_node(n);
        for (int64_t v = 0; v < nn; ++v) {
            for (int d = 0; d < 3; ++d) if (udof[3 * v + d] >= 0) dof_node[udof[3 * v + d]] = v;
            if (pdof[v] >= 0) dof_node[pdof[v]] = v;
        }
        Pattern P;
        P.n = n;
        P.rowptr.assign(n + 1, 0);
        std::vector<int32_t> rowbuf;
        std::vector<std::vector<int32_t>> rows(n);
        for (int64_t r = 0; r < n; ++r) {
            int64_t v = dof_node[r];
            bool is_p = r >= n_u;
            rowbuf.clear();
            if (!is_p) {
                for (int64_t b : adj_s[v]) for (int d = 0; d < 3; ++d) if (udof[3 * b + d] >= 0) rowbuf.push_back((int32_t)udof[3 * b + d]);
                for (int64_t b : adj_c[v]) if (b != -1 && pdof[b] >= 0) rowbuf.push_back((int32_t)pdof[b]);
            } else {
                for (int64_t b : adj_f[v]) rowbuf.push_back((int32_t)pdof[b]);
                for (int64_t b : adj_c[v]) for (int d = 0; d < 3; ++d) if (udof[3 * b + d] >= 0) rowbuf.push_back((int32_t)udof[3 * b + d]);
            }
            std::sort(rowbuf.begin(), rowbuf.end());
            rowbuf.erase(std::unique(rowbuf.begin(), rowbuf.end()), rowbuf.end());
            rows[r] = rowbuf;
            P.rowptr[r + 1] = P.rowptr[r] + (int64_t)rowbuf.size();
        }
        P.col.resize(P.rowptr[n]);
        for (int64_t r = 0; r < n; ++r) std::copy(rows[r].begin(), rows[r].end(), P.col.begin() + P.rowptr[r]);
        rows.clear();
        rows.shrink_to_fit();
        const int64_t nnz = P.rowptr[n];
        std::vector<cplx> Kv(nnz, 0.0), Mv(nnz, 0.0);
        std::vector<std::vector<cplx>> Tv(nterm, std::vector<cplx>(nnz, 0.0));

        double X[8][3];
        for (int64_t e = 0; e < ne; ++e) {
            const int64_t* c = mesh->elems + 8 * e;
            const cr_material& mt = mats[mesh->elem_mat[e]];
            for (int a = 0; a < 8; ++a)
                for (int j = 0; j < 3; ++j) X[a][j] = mesh->coords[3 * c[a] + j];
            if (mt.kind == CR_FLUID) {
                double Ke[8][8] = {{0}}, Me[8][8] = {{0}};
                for (int g = 0; g < 8; ++g) {
                    HexPoint hp = hex_point(X, (g & 1) ? kG : -kG, (g & 2) ? kG : -kG, (g & 4) ? kG : -kG);
                    for (int a = 0; a < 8; ++a)
                        for (int b = 0; b < 8; ++b) {
                            Ke[a][b] += hp.detJ * (hp.dNdx[a][0] * hp.dNdx[b][0] + hp.dNdx[a][1] * hp.dNdx[b][1] +
                                                   hp.dNdx[a][2] * hp.dNdx[b][2]);
                            Me[a][b] += hp.detJ * hp.N[a] * hp.N[b];
                        }
                }
                const int tm = term_of[mesh->elem_mat[e]];
                cplx inv_c2 = 1.0 / (mt.c * mt.c * cplx(1.0, mt.eta));
                for (int a = 0; a < 8; ++a)
                    for (int b = 0; b < 8; ++b) {
                        int64_t pos = P.find(pdof[c[a]], pdof[c[b]]);
                        Kv[pos] += Ke[a][b];
                        if (tm >= 0) Tv[tm][pos] += Me[a][b];   // int N^T N; 1 / c~^2(w) applied per frequency
                        else Mv[pos] += Me[a][b] * inv_c2;
                    }
            } else {
                const int tm = term_of[mesh->elem_mat[e]];
                // a frequency-dependent loss factor keeps the real-E stiffness as its own term
                cplx E = tm >= 0 ? cplx(mt.E, 0.0) : mt.E * cplx(1.0, mt.eta);
                cplx lam = E * mt.nu / ((1 + mt.nu) * (1 - 2 * mt.nu));
                cplx mu = E / (2 * (1 + mt.nu));
                double G1[8][8][3][3] = {{{{0}}}};   // int d_i N_a d_j N_b
                double Mn[8][8] = {{0}};
                for (int g = 0; g < 8; ++g) {
                    HexPoint hp = hex_point(X, (g & 1) ? kG : -kG, (g & 2) ? kG : -kG, (g & 4) ? kG : -kG);
                    for (int a = 0; a < 8; ++a)
                        for (int b = 0; b < 8; ++b) {
                            Mn[a][b] += hp.detJ * hp.N[a] * hp.N[b];
                            for (int i = 0; i < 3; ++i)
                                for (int j = 0; j < 3; ++j) G1[a][b][i][j] += hp.detJ * hp.dNdx[a][i] * hp.dNdx[b][j];
                        }
                }
                for (int a = 0; a < 8; ++a)
                    for (int b = 0; b < 8; ++b) {
                        double lap = G1[a][b][0][0] + G1[a][b][1][1] + G1[a][b][2][2];
                        for (int i = 0; i < 3; ++i) {
                            int64_t r = udof[3 * c[a] + i];
                            if (r < 0) continue;
                            for (int j = 0; j < 3; ++j) {
                                int64_t cc = udof[3 * c[b] + j];
                                if (cc < 0) continue;
                                cplx k = lam * G1[a][b][i][j] + mu * G1[a][b][j][i];
                                if (i == j) k += mu * lap;
                                int64_t pos = P.find(r, cc);
                                if (tm >= 0) Tv[tm][pos] += k;
                                else Kv[pos] += k;
                                if (i == j) Mv[pos] += mt.rho * Mn[a][b];
                            }
                        }
                    }
            }
        }
        const double rho0 = fluid_mat >= 0 ? mats[fluid_mat].rho : 0.0;
        double Xq[4][3], W[4][4][3];
        for (const int64_t* q : faces) {
            for (int a = 0; a < 4; ++a)
                for (int j = 0; j < 3; ++j) Xq[a][j] = mesh->coords[3 * q[a] + j];
            quad_integrals(Xq, W);
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b)
                    for (int d = 0; d < 3; ++d) {
                        int64_t u = udof[3 * q[a] + d], p = pdof[q[b]];
                        if (u < 0) continue;
                        Kv[P.find(u, p)] -= W[a][b][d];
                        Mv[P.find(p, u)] += rho0 * W[a][b][d];
                    }
        }
        // loads
        std::vector<cplx> F((size_t)n * nload, 0.0);
        std::vector<int32_t> flags(nload, 0);
        for (int l = 0; l < nload; ++l) {
            const cr_load& ld = loads[l];
            cplx val(ld.value.re, ld.value.im);
            if (ld.kind == CR_LOAD_VOLUME_VELOCITY) {
                CR_REQUIRE(ld.node >= 0 && ld.node < nn && pdof[ld.node] >= 0, CR_E_INVALID, "volume velocity at a node without pressure");
                F[(size_t)l * n + pdof[ld.node]] += rho0 * val;
                flags[l] = 1;
            } else if (ld.kind == CR_LOAD_POINT_FORCE) {
                CR_REQUIRE(ld.node >= 0 && ld.node < nn && ld.dir >= 0 && ld.dir < 3 && udof[3 * ld.node + ld.dir] >= 0,
                           CR_E_INVALID, "point force at a node without a free displacement");
                F[(size_t)l * n + udof[3 * ld.node + ld.dir]] += val;
            } else if (ld.kind == CR_LOAD_SKIN_PRESSURE) {
                CR_REQUIRE(ld.n_faces >= 0 && (ld.n_faces == 0 || (ld.faces && ld.amp)), CR_E_INVALID, "skin pressure arrays missing");
                for (int64_t f = 0; f < ld.n_faces; ++f) {
                    const int64_t* q = ld.faces + 4 * f;
                    for (int a = 0; a < 4; ++a) CR_REQUIRE(q[a] >= 0 && q[a] < nn, CR_E_INVALID, "skin face node out of range");
                    for (int a = 0; a < 4; ++a)
                        for (int j = 0; j < 3; ++j) Xq[a][j] = mesh->coords[3 * q[a] + j];
                    quad_integrals(Xq, W);
                    for (int a = 0; a < 4; ++a)
                        for (int d = 0; d < 3; ++d) {
                            int64_t u = udof[3 * q[a] + d];
                            if (u < 0) continue;
                            cplx acc = 0;
                            for (int b = 0; b < 4; ++b) acc += W[a][b][d] * cplx(ld.amp[q[b]].re, ld.amp[q[b]].im);
                            F[(size_t)l * n + u] -= acc;
                        }
                }
            } else {
                throw cr::Error(CR_E_INVALID, "unknown load kind");
            }
        }
        std::vector<int64_t> recv(n_o);
        for (int i = 0; i < n_o; ++i) {
            int64_t v = recv_nodes[i];
            CR_REQUIRE(v >= 0 && v < nn && pdof[v] >= 0, CR_E_INVALID, "receiver node without a pressure DoF");
            recv[i] = pdof[v];
        }

        auto sys = std::make_unique<cr_sys_s>();
        sys->ctx = ctx;
        sys->n = n;
        sys->n_u = n_u;
        sys->L = nload;
        sys->n_o = n_o;
        sys->rowptr = std::move(P.rowptr);
        sys->col = std::move(P.col);
        sys->K.resize(nnz);
        sys->M.resize(nnz);
        for (int64_t k = 0; k < nnz; ++k) {
            sys->K[k] = {Kv[k].real(), Kv[k].imag()};
            sys->M[k] = {Mv[k].real(), Mv[k].imag()};
        }
        for (int m = 0; m < nmat; ++m) {
            if (term_of[m] < 0) continue;
            cr::FreqTerm t;
            t.kind = mats[m].kind == CR_SOLID ? 0 : 1;
            t.c = mats[m].c;
            t.f_hz.assign(mats[m].eta_f_hz, mats[m].eta_f_hz + mats[m].n_eta);
            t.eta.assign(mats[m].eta_val, mats[m].eta_val + mats[m].n_eta);
            t.vals.resize(nnz);
            for (int64_t k = 0; k < nnz; ++k) t.vals[k] = {Tv[term_of[m]][k].real(), Tv[term_of[m]][k].imag()};
            sys->terms.push_back(std::move(t));
        }
        sys->F.resize(F.size());
        for (size_t k = 0; k < F.size(); ++k) sys->F[k] = {F[k].real(), F[k].imag()};
        sys->flags = flags;
        sys->recv = recv;
        sys->coords.resize(3 * n);
        for (int64_t r = 0; r < n; ++r)
            for (int j = 0; j < 3; ++j) sys->coords[3 * r + j] = mesh->coords[3 * dof_node[r] + j];
        cr::finalize_sys(sys.get());
        *out = sys.release();
    });
}
