// Faces of the structured curved mesh and the upwind face integrals.
//
// Numbering: for each reference axis a, faces lie on lattice planes
// P = 0..nx[a]; the element with index P-1 along a is the face's minus
// element, the one with index P its plus element (-1 on the boundary).  A face
// is parametrised by the remaining axes in ascending order (s, t); N is the
// area-scaled normal from minus to plus (2D axis 0: (t_y, -t_x), axis 1:
// (-t_y, t_x); 3D axes 0, 2: x_s x x_t, axis 1: x_t x x_s), so that
// (Omega . n) ds = (Omega . N) ds_ref and g = Omega . N.
//
// Face matrices of the upwind DG operator (eqs. localFDiagonalMatrix and
// localFOffDiagonalMatrix): P_plus[a][b] = int max(g,0) phi_a phi_b and
// P_minus[a][b] = int max(-g,0) phi_a phi_b over the reference face.  For a
// face without a sign change of g these are +-sum_k Omega_k B_k with the
// direction-independent moments B_k[a][b] = int N_k phi_a phi_b (exact Gauss
// rule).  Faces where g changes sign ("re-entrant faces", non-smooth
// integrand) are integrated
//   2D: exactly, splitting [0,1] at the real roots of the polynomial g(s)
//       (degree r-1 <= 2) and using ceil((r+2p)/2) Gauss points per piece;
//   3D: with a fixed composite rule of 4x4 sub-squares, (p+r)^2 Gauss points
//       each (the rule also decides whether a sign change is present).
// With SNSW_FACE_ROMBERG the sign-changing faces are integrated instead by
// adaptive Romberg (below) to the absolute tolerance face_tol * int |g|.
// Interior faces: a side whose measure int max(+-g,0) is at most 1e-12 of
// int |g| is dropped (matrix set to zero), so the operator and the graph
// agree.
#include <algorithm>
#include <cmath>
#include <functional>
#include <map>
#include <string>

#include "host.hpp"

namespace snsw {

namespace {
constexpr int kSub3 = 4;

// N = x_s x x_t of a triangular face from its control points X [nfc][3] and
// the basis derivatives at one point.
void tri_face_normal(const double* X, int nfc, const double* gs, const double* gt, double* N) {
    double t1[3] = {0, 0, 0}, t2[3] = {0, 0, 0};
    for (int m = 0; m < nfc; ++m)
        for (int c = 0; c < 3; ++c) {
            t1[c] += X[m * 3 + c] * gs[m];
            t2[c] += X[m * 3 + c] * gt[m];
        }
    N[0] = t1[1] * t2[2] - t1[2] * t2[1];
    N[1] = t1[2] * t2[0] - t1[0] * t2[2];
    N[2] = t1[0] * t2[1] - t1[1] * t2[0];
}
}  // namespace

void face_geometry(HostProblem& hp);

namespace {

// Element-local node numbers on slot s at per-axis order `order`, listed in
// the slot's own face order (remaining reference axes ascending, the first
// fastest).
std::vector<int32_t> slot_local_nodes(int dim, int order, int s) {
    const int a = s / 2, hi = s % 2, n1 = order + 1;
    const int cnt = dim == 2 ? n1 : n1 * n1;
    std::vector<int32_t> out(cnt);
    for (int l = 0; l < cnt; ++l) {
        int idx[3] = {0, 0, 0}, rem = l;
        for (int b = 0; b < dim; ++b) {
            if (b == a) continue;
            idx[b] = rem % n1;
            rem /= n1;
        }
        idx[a] = hi ? order : 0;
        int m = 0, st = 1;
        for (int b = 0; b < dim; ++b) { m += idx[b] * st; st *= n1; }
        out[l] = m;
    }
    return out;
}

// Kinds of reference faces: a segment (2D elements), a square (hexahedra),
// a triangle (tetrahedra).
enum FaceKind { FK_SEG = 2, FK_QUAD = 3, FK_TRI = 4 };
FaceKind face_kind(const HostProblem& hp) { return hp.dim == 2 ? FK_SEG : (hp.simplex ? FK_TRI : FK_QUAD); }

// The symmetries of the reference face as maps of face-local node indices at
// order k: segment (identity, reversal); square the eight maps
// (i, j) -> (x, y) or (y, x) with x in {i, k-i}, y in {j, k-j}; triangle the
// six permutations of its vertices acting on the barycentric lattice
// coordinates (k - a - b, a, b) of node (a, b).
int face_sym_count(FaceKind kind) { return kind == FK_SEG ? 2 : (kind == FK_QUAD ? 8 : 6); }
int face_sym(FaceKind kind, int t, int k, int l) {
    if (kind == FK_SEG) return t ? k - l : l;
    if (kind == FK_QUAD) {
        const int n1 = k + 1, i = l % n1, j = l / n1;
        const int x = (t & 1) ? k - i : i, y = (t & 2) ? k - j : j;
        return (t & 4) ? y + n1 * x : x + n1 * y;
    }
    static const int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int b = 0, rem = l;
    while (rem > k - b) rem -= k - b + 1, ++b;   // row b of the triangle lattice holds k - b + 1 nodes
    const int a = rem;
    const int c[3] = {k - a - b, a, b};
    int cp[3] = {0, 0, 0};
    for (int i = 0; i < 3; ++i) cp[kPerm[t][i]] = c[i];
    return tri_index(k, cp[1], cp[2]);
}

// Faces of an unstructured conforming mesh.  Two element slots are one face
// when their corner control points are the same (by index).  The face's
// minus element is the one with the smaller index (the only one on the
// boundary); the face is parametrised like the minus element's slot,
// mirrored (2D: reversed; 3D: its two axes exchanged) when that slot is a
// xi_a = 0 face, so that the normal of the axis formula is the minus
// element's outward normal.  The plus element's slot is matched to the face
// by the face symmetry that carries every control point onto its partner.
//
// Triangles: the three edge slots run counter-clockwise (v0 -> v1 -> v2), so
// the axis-0 normal of the slot's own order is already the outward normal:
// no slot is mirrored and every face has axis 0.  Tetrahedra: the four
// triangular face slots list their vertices in the outward order, so again
// no slot is mirrored; faces are matched by their three corners.
void unstructured_topology(HostProblem& hp) {
    const int dim = hp.dim, r = hp.r, p = hp.p, nf = hp.nf;
    const int ns = hp.simplex ? dim + 1 : 2 * dim;
    const FaceKind kind = face_kind(hp);
    const int64_t E = hp.E;
    const int Nv = hp.nv;
    const int nloc = kind == FK_SEG ? r + 1 : (kind == FK_QUAD ? (r + 1) * (r + 1) : (r + 1) * (r + 2) / 2);
    std::vector<std::vector<int32_t>> cl(ns), dl(ns);
    for (int s = 0; s < ns; ++s) {
        if (kind == FK_TRI) {
            cl[s] = tet_slot_nodes(r, s);
            dl[s] = tet_slot_nodes(p, s);
        } else if (hp.simplex) {
            cl[s] = tri_slot_nodes(r, s);
            dl[s] = tri_slot_nodes(p, s);
        } else {
            cl[s] = slot_local_nodes(dim, r, s);
            dl[s] = slot_local_nodes(dim, p, s);
        }
    }
    const int nc = kind == FK_SEG ? 2 : (kind == FK_QUAD ? 4 : 3);
    auto corner = [&](int k) {   // face-local index of corner k
        const int R = r;
        if (kind == FK_SEG) return k ? R : 0;
        if (kind == FK_TRI) return k == 0 ? 0 : (k == 1 ? R : nloc - 1);
        return (k & 1 ? R : 0) + (r + 1) * (k & 2 ? R : 0);
    };
    struct Key {
        int64_t c[4];
        bool operator<(const Key& o) const { return std::lexicographical_compare(c, c + 4, o.c, o.c + 4); }
    };
    std::map<Key, std::vector<std::pair<int64_t, int>>> table;
    for (int64_t e = 0; e < E; ++e)
        for (int s = 0; s < ns; ++s) {
            Key k{{-1, -1, -1, -1}};
            for (int c = 0; c < nc; ++c) k.c[c] = hp.elem_nodes[(size_t)e * Nv + cl[s][corner(c)]];
            std::sort(k.c, k.c + nc);
            table[k].push_back({e, s});
        }
    std::vector<std::vector<std::pair<int64_t, int>>> recs;
    recs.reserve(table.size());
    for (auto& kv : table) {
        std::sort(kv.second.begin(), kv.second.end());
        if (kv.second.size() > 2 || (kv.second.size() == 2 && kv.second[0].first == kv.second[1].first))
            throw Error(SNSW_E_SHAPE, "unstructured mesh: a face is shared by more than two element slots");
        recs.push_back(kv.second);
    }
    std::sort(recs.begin(), recs.end());
    hp.F = (int64_t)recs.size();
    hp.nslot = ns;
    hp.f_axis.assign(hp.F, 0);
    hp.f_minus.assign(hp.F, -1);
    hp.f_plus.assign(hp.F, -1);
    hp.f_ctrl.assign((size_t)hp.F * nloc * dim, 0.0);
    hp.f_slot_minus.assign(hp.F, -1);
    hp.f_slot_plus.assign(hp.F, -1);
    hp.slot_face.assign((size_t)E * ns, -1);
    hp.slot_nbr.assign((size_t)E * ns, -1);
    hp.hf_minus.assign((size_t)E * ns, 0);
    hp.hf_trace.assign((size_t)E * ns * nf, 0);
    hp.hf_up_trace.assign((size_t)E * ns * nf, 0);
    const int mirror = dim == 2 ? 1 : 4;   // face symmetry used to mirror a xi_a = 0 slot
    for (int64_t f = 0; f < hp.F; ++f) {
        const auto& rec = recs[f];
        const int64_t em = rec[0].first;
        const int sm = rec[0].second;
        const int tm = ((sm & 1) || hp.simplex) ? 0 : mirror;   // face index l <- slot index face_sym(tm, l)
        hp.f_axis[f] = hp.simplex ? 0 : sm / 2;
        hp.f_minus[f] = (int32_t)em;
        hp.f_slot_minus[f] = (int8_t)sm;
        std::vector<int64_t> ids(nloc);
        for (int l = 0; l < nloc; ++l) {
            ids[l] = hp.elem_nodes[(size_t)em * Nv + cl[sm][face_sym(kind, tm, r, l)]];
            for (int c = 0; c < dim; ++c) hp.f_ctrl[((size_t)f * nloc + l) * dim + c] = hp.nodes[(size_t)ids[l] * dim + c];
        }
        hp.slot_face[em * ns + sm] = (int32_t)f;
        hp.hf_minus[em * ns + sm] = 1;
        for (int l = 0; l < nf; ++l) hp.hf_trace[((size_t)em * ns + sm) * nf + l] = dl[sm][face_sym(kind, tm, p, l)];
        if (rec.size() == 1) continue;
        const int64_t ep = rec[1].first;
        const int sp = rec[1].second;
        int tp = -1;
        for (int t = 0; t < face_sym_count(kind) && tp < 0; ++t) {
            bool ok = true;
            for (int l = 0; l < nloc && ok; ++l)
                ok = hp.elem_nodes[(size_t)ep * Nv + cl[sp][face_sym(kind, t, r, l)]] == ids[l];
            if (ok) tp = t;
        }
        if (tp < 0) throw Error(SNSW_E_SHAPE, "unstructured mesh: non-conforming face between elements " +
                                                  std::to_string(em) + " and " + std::to_string(ep));
        hp.f_plus[f] = (int32_t)ep;
        hp.f_slot_plus[f] = (int8_t)sp;
        hp.slot_face[ep * ns + sp] = (int32_t)f;
        hp.slot_nbr[em * ns + sm] = (int32_t)ep;
        hp.slot_nbr[ep * ns + sp] = (int32_t)em;
        for (int l = 0; l < nf; ++l) hp.hf_trace[((size_t)ep * ns + sp) * nf + l] = dl[sp][face_sym(kind, tp, p, l)];
        for (int l = 0; l < nf; ++l) {
            hp.hf_up_trace[((size_t)em * ns + sm) * nf + l] = hp.hf_trace[((size_t)ep * ns + sp) * nf + l];
            hp.hf_up_trace[((size_t)ep * ns + sp) * nf + l] = hp.hf_trace[((size_t)em * ns + sm) * nf + l];
        }
    }
    for (int32_t v : hp.slot_face)
        if (v < 0) throw Error(SNSW_E_SHAPE, "unstructured mesh: an element slot has no face");
    hp.slot_nodes.assign((size_t)ns * nf, 0);
    for (int s = 0; s < ns; ++s)
        for (int l = 0; l < nf; ++l) hp.slot_nodes[(size_t)s * nf + l] = dl[s][l];
}

}  // namespace

void build_faces(HostProblem& hp) {
    const int dim = hp.dim, r = hp.r, p = hp.p;
    const int nf = hp.nf;
    if (hp.unstructured) {
        unstructured_topology(hp);
        face_geometry(hp);
        return;
    }
    int L[3] = {1, 1, 1};
    for (int a = 0; a < dim; ++a) L[a] = r * hp.nx[a] + 1;
    const int nloc = dim == 2 ? r + 1 : (r + 1) * (r + 1);
    hp.f_axis.clear(); hp.f_minus.clear(); hp.f_plus.clear(); hp.f_ctrl.clear();
    std::vector<int64_t> axis_off(dim);
    int64_t off = 0;
    for (int a = 0; a < dim; ++a) {
        axis_off[a] = off;
        int ext[3] = {1, 1, 1};
        for (int b = 0; b < dim; ++b) ext[b] = hp.nx[b] + (b == a ? 1 : 0);
        int64_t nfa = 1;
        for (int b = 0; b < dim; ++b) nfa *= ext[b];
        int others[2] = {0, 0}, no = 0;
        for (int b = 0; b < dim; ++b) if (b != a) others[no++] = b;
        for (int64_t fi = 0; fi < nfa; ++fi) {
            int idx[3] = {0, 0, 0};
            int64_t rem = fi;
            for (int b = 0; b < dim; ++b) { idx[b] = (int)(rem % ext[b]); rem /= ext[b]; }
            const int P = idx[a];
            auto elem = [&](int pa) -> int32_t {
                int64_t e = 0, s = 1;
                for (int b = 0; b < dim; ++b) { e += (b == a ? pa : idx[b]) * s; s *= hp.nx[b]; }
                return (int32_t)e;
            };
            hp.f_axis.push_back(a);
            hp.f_minus.push_back(P >= 1 ? elem(P - 1) : -1);
            hp.f_plus.push_back(P < hp.nx[a] ? elem(P) : -1);
            for (int l = 0; l < nloc; ++l) {
                int li[2] = {l % (r + 1), l / (r + 1)};
                int64_t lid = 0, stride = 1;
                for (int b = 0; b < dim; ++b) {
                    int coord;
                    if (b == a) coord = r * P;
                    else {
                        int k = (b == others[0]) ? 0 : 1;
                        coord = r * idx[b] + li[k];
                    }
                    lid += (int64_t)coord * stride;
                    stride *= L[b];
                }
                for (int c = 0; c < dim; ++c) hp.f_ctrl.push_back(hp.lattice[lid * dim + c]);
            }
        }
        off += nfa;
    }
    hp.F = off;
    // element slots: slot 2a is the xi_a = 0 face (element = plus side),
    // slot 2a+1 the xi_a = 1 face (element = minus side)
    hp.nslot = 2 * dim;
    hp.slot_face.assign((size_t)hp.E * hp.nslot, -1);
    hp.slot_nbr.assign((size_t)hp.E * hp.nslot, -1);
    for (int64_t e = 0; e < hp.E; ++e) {
        int ei[3] = {0, 0, 0};
        int64_t re = e;
        for (int b = 0; b < dim; ++b) { ei[b] = (int)(re % hp.nx[b]); re /= hp.nx[b]; }
        for (int s = 0; s < hp.nslot; ++s) {
            const int a = s / 2, hi = s % 2;
            int ext[3] = {1, 1, 1};
            for (int b = 0; b < dim; ++b) ext[b] = hp.nx[b] + (b == a ? 1 : 0);
            int64_t fid = 0, st = 1;
            for (int b = 0; b < dim; ++b) { fid += (ei[b] + (b == a ? hi : 0)) * st; st *= ext[b]; }
            fid += axis_off[a];
            hp.slot_face[e * hp.nslot + s] = (int32_t)fid;
            hp.slot_nbr[e * hp.nslot + s] = hi ? hp.f_plus[fid] : hp.f_minus[fid];
        }
    }
    hp.slot_nodes.assign((size_t)hp.nslot * nf, 0);
    for (int s = 0; s < hp.nslot; ++s) {
        const int a = s / 2, hi = s % 2;
        for (int l = 0; l < nf; ++l) {
            int idx[3] = {0, 0, 0}, rem = l;
            for (int b = 0; b < dim; ++b) {
                if (b == a) continue;
                idx[b] = rem % (p + 1);
                rem /= p + 1;
            }
            idx[a] = hi ? p : 0;
            int m = 0, st = 1;
            for (int b = 0; b < dim; ++b) { m += idx[b] * st; st *= p + 1; }
            hp.slot_nodes[s * nf + l] = m;
        }
    }

    face_geometry(hp);
}

// Triangular faces (tetrahedra): face map x(s, t) = sum_m X_m psi_m(s, t)
// over the P_r triangle basis of the face's control points, N = x_s x x_t
// (outward for the minus element by the slot's vertex order); B_k and int N
// with the collapsed Gauss rule of p + r points per direction (exact: N has
// degree 2(r-1), the traces' products 2p); the composite rule of 4 x 4
// sub-triangles for the classification of sign changes.
void face_geometry_tri(HostProblem& hp) {
    const int r = hp.r, p = hp.p, nf = hp.nf;
    const int nfc = (r + 1) * (r + 2) / 2;
    const TriBasis geo(tri_geometry_nodes(r), r), dg(tri_dg_nodes(p), p);
    std::vector<double> xs, ys, ws;
    tri_collapsed_rule(p + r, xs, ys, ws);
    const size_t Q = ws.size();
    std::vector<double> Gs(Q * nfc), Gt(Q * nfc), Ph(Q * nf);
    for (size_t q = 0; q < Q; ++q) {
        geo.eval(xs[q], ys[q], nullptr, &Gs[q * nfc], &Gt[q * nfc]);
        dg.eval(xs[q], ys[q], &Ph[q * nf], nullptr, nullptr);
    }
    FaceNormalData& nd = hp.fnd;
    nd = FaceNormalData();
    nd.nfc = nfc;
    std::vector<double> cs, ct;
    tri_composite_rule(kSub3, p + r, cs, ct, nd.cw);
    const size_t Qc = nd.cw.size();
    nd.tgs.resize(Qc * nfc);
    nd.tgt.resize(Qc * nfc);
    nd.cphi.resize(Qc * nf);
    for (size_t q = 0; q < Qc; ++q) {
        geo.eval(cs[q], ct[q], nullptr, &nd.tgs[q * nfc], &nd.tgt[q * nfc]);
        dg.eval(cs[q], ct[q], &nd.cphi[q * nf], nullptr, nullptr);
    }
    nd.Rf.assign(hp.F, 0.0);
    hp.B.assign((size_t)hp.F * 3 * nf * nf, 0.0);
    hp.Nint.assign((size_t)hp.F * 3, 0.0);
    parallel_for(hp.F, hp.nthreads, [&](int64_t f0, int64_t f1) {
        for (int64_t f = f0; f < f1; ++f) {
            const double* X = &hp.f_ctrl[(size_t)f * nfc * 3];
            double* Bf = &hp.B[(size_t)f * 3 * nf * nf];
            double* Nf = &hp.Nint[(size_t)f * 3];
            for (size_t q = 0; q < Q; ++q) {
                double N[3];
                tri_face_normal(X, nfc, &Gs[q * nfc], &Gt[q * nfc], N);
                const double* ph = &Ph[q * nf];
                for (int k = 0; k < 3; ++k) {
                    Nf[k] += ws[q] * N[k];
                    for (int i = 0; i < nf; ++i)
                        for (int j = 0; j < nf; ++j) Bf[(k * nf + i) * nf + j] += ws[q] * N[k] * ph[i] * ph[j];
                }
            }
            double R = 0.0;
            for (size_t q = 0; q < Qc; ++q) {
                double N[3];
                tri_face_normal(X, nfc, &nd.tgs[q * nfc], &nd.tgt[q * nfc], N);
                // the mean normal is 2 int N (the reference triangle has area 1/2)
                const double dx = N[0] - 2.0 * Nf[0], dy = N[1] - 2.0 * Nf[1], dz = N[2] - 2.0 * Nf[2];
                R = std::max(R, std::sqrt(dx * dx + dy * dy + dz * dz));
            }
            hp.fnd.Rf[f] = R;
        }
    });
}

// Normal moments B_k, int N_k and the 3D composite-rule tables of every face
// (from f_axis and f_ctrl).
void face_geometry(HostProblem& hp) {
    if (hp.simplex && hp.dim == 3) {
        face_geometry_tri(hp);
        return;
    }
    const int dim = hp.dim, r = hp.r, p = hp.p;
    const int nf = hp.nf;
    const int nloc = dim == 2 ? r + 1 : (r + 1) * (r + 1);
    // normal moments B_k and int N_k with an exact Gauss rule
    std::vector<double> geo_nodes(r + 1);
    for (int a = 0; a <= r; ++a) geo_nodes[a] = (double)a / r;
    const std::vector<double> dg = gll01(p);
    const int nq1 = dim == 2 ? (r + 2 * p + 1) / 2 : p + r;
    std::vector<double> x1, w1;
    gauss_legendre01(nq1, x1, w1);
    std::vector<double> gV(nq1 * (r + 1)), gD(nq1 * (r + 1)), uV(nq1 * (p + 1));
    for (int k = 0; k < nq1; ++k) {
        lagrange_eval(geo_nodes, x1[k], &gV[k * (r + 1)], &gD[k * (r + 1)]);
        lagrange_eval(dg, x1[k], &uV[k * (p + 1)], nullptr);
    }
    hp.B.assign((size_t)hp.F * dim * nf * nf, 0.0);
    hp.Nint.assign((size_t)hp.F * dim, 0.0);
    FaceNormalData& nd = hp.fnd;
    nd = FaceNormalData();
    if (dim == 2) nd.mono.assign((size_t)hp.F * 2 * r, 0.0);
    // 3D: w_q N(q) at the moments' Gauss points (the level sweeps of p = 2
    // lattices contract the inflow through them)
    hp.Nq.assign(dim == 3 ? (size_t)hp.F * nq1 * nq1 * 3 : 0, 0.0);
    // 3D composite rule tables
    if (dim == 3) {
        std::vector<double> xs, ws;
        gauss_legendre01(p + r, xs, ws);
        nd.nc1 = kSub3 * (p + r);
        std::vector<double> c1(nd.nc1), cw1(nd.nc1);
        for (int k = 0; k < kSub3; ++k)
            for (int j = 0; j < p + r; ++j) {
                c1[k * (p + r) + j] = (k + xs[j]) / kSub3;
                cw1[k * (p + r) + j] = ws[j] / kSub3;
            }
        nd.gV1.assign(nd.nc1 * (r + 1), 0.0);
        nd.gD1.assign(nd.nc1 * (r + 1), 0.0);
        std::vector<double> u1(nd.nc1 * (p + 1));
        for (int k = 0; k < nd.nc1; ++k) {
            lagrange_eval(geo_nodes, c1[k], &nd.gV1[k * (r + 1)], &nd.gD1[k * (r + 1)]);
            lagrange_eval(dg, c1[k], &u1[k * (p + 1)], nullptr);
        }
        for (int j = 0; j < nd.nc1; ++j)
            for (int i = 0; i < nd.nc1; ++i) {
                nd.ci.push_back(i);
                nd.cj.push_back(j);
                nd.cs.push_back(c1[i]);
                nd.ct.push_back(c1[j]);
                nd.cw.push_back(cw1[i] * cw1[j]);
                for (int bt = 0; bt <= p; ++bt)
                    for (int bs = 0; bs <= p; ++bs)
                        nd.cphi.push_back(u1[i * (p + 1) + bs] * u1[j * (p + 1) + bt]);
            }
        nd.Rf.assign(hp.F, 0.0);
    }
    auto dmono = lagrange_derivative_monomials(geo_nodes);

    parallel_for(hp.F, hp.nthreads, [&](int64_t f0, int64_t f1) {
        std::vector<double> phi(nf);
        for (int64_t f = f0; f < f1; ++f) {
            const double* X = &hp.f_ctrl[(size_t)f * nloc * dim];
            const int a = hp.f_axis[f];
            double* Bf = &hp.B[(size_t)f * dim * nf * nf];
            double* Nf = &hp.Nint[(size_t)f * dim];
            if (dim == 2) {
                const double sg = a == 0 ? 1.0 : -1.0;
                for (int q = 0; q < nq1; ++q) {
                    double tx = 0, ty = 0;
                    for (int b = 0; b <= r; ++b) {
                        tx += X[b * 2 + 0] * gD[q * (r + 1) + b];
                        ty += X[b * 2 + 1] * gD[q * (r + 1) + b];
                    }
                    const double N[2] = {sg * ty, -sg * tx};
                    for (int k = 0; k < 2; ++k) {
                        Nf[k] += w1[q] * N[k];
                        for (int i = 0; i < nf; ++i)
                            for (int j = 0; j < nf; ++j)
                                Bf[(k * nf + i) * nf + j] += w1[q] * N[k] * uV[q * (p + 1) + i] * uV[q * (p + 1) + j];
                    }
                }
                double* mo = &nd.mono[(size_t)f * 2 * r];
                for (int b = 0; b <= r; ++b)
                    for (int k = 0; k < r; ++k) {
                        double dk = k < (int)dmono[b].size() ? dmono[b][k] : 0.0;
                        mo[0 * r + k] += sg * X[b * 2 + 1] * dk;    // N_x = sg * t_y
                        mo[1 * r + k] += -sg * X[b * 2 + 0] * dk;   // N_y = -sg * t_x
                    }
            } else {
                auto normal_at = [&](const double* Vs, const double* Ds, const double* Vt,
                                     const double* Dt, double* N) {
                    double t1[3] = {0, 0, 0}, t2[3] = {0, 0, 0};
                    for (int bt = 0; bt <= r; ++bt)
                        for (int bs = 0; bs <= r; ++bs) {
                            const double* x = &X[(bt * (r + 1) + bs) * 3];
                            for (int c = 0; c < 3; ++c) {
                                t1[c] += x[c] * Ds[bs] * Vt[bt];
                                t2[c] += x[c] * Vs[bs] * Dt[bt];
                            }
                        }
                    double c0 = t1[1] * t2[2] - t1[2] * t2[1];
                    double c1 = t1[2] * t2[0] - t1[0] * t2[2];
                    double c2 = t1[0] * t2[1] - t1[1] * t2[0];
                    const double sgn = a == 1 ? -1.0 : 1.0;
                    N[0] = sgn * c0; N[1] = sgn * c1; N[2] = sgn * c2;
                };
                for (int qt = 0; qt < nq1; ++qt)
                    for (int qs = 0; qs < nq1; ++qs) {
                        double N[3];
                        normal_at(&gV[qs * (r + 1)], &gD[qs * (r + 1)], &gV[qt * (r + 1)], &gD[qt * (r + 1)], N);
                        const double wq = w1[qs] * w1[qt];
                        double* wn = &hp.Nq[(((size_t)f * nq1 + qt) * nq1 + qs) * 3];
                        for (int k = 0; k < 3; ++k) wn[k] = wq * N[k];
                        for (int bt = 0; bt <= p; ++bt)
                            for (int bs = 0; bs <= p; ++bs)
                                phi[bt * (p + 1) + bs] = uV[qs * (p + 1) + bs] * uV[qt * (p + 1) + bt];
                        for (int k = 0; k < 3; ++k) {
                            Nf[k] += wq * N[k];
                            for (int i = 0; i < nf; ++i)
                                for (int j = 0; j < nf; ++j) Bf[(k * nf + i) * nf + j] += wq * N[k] * phi[i] * phi[j];
                        }
                    }
                // bound of |N - Nbar| over the composite rule points
                double R = 0.0;
                const size_t Qc = nd.cw.size();
                for (size_t q = 0; q < Qc; ++q) {
                    double N[3];
                    const int i = nd.ci[q], j = nd.cj[q];
                    normal_at(&nd.gV1[i * (r + 1)], &nd.gD1[i * (r + 1)], &nd.gV1[j * (r + 1)],
                              &nd.gD1[j * (r + 1)], N);
                    double dx = N[0] - Nf[0], dy = N[1] - Nf[1], dz = N[2] - Nf[2];
                    R = std::max(R, std::sqrt(dx * dx + dy * dy + dz * dz));
                }
                nd.Rf[f] = R;
            }
        }
    });
}

// ---------------------------------------------------------------------------
// Adaptive Romberg integration of a sign-changing face (SNSW_FACE_ROMBERG;
// section 2 names Romberg for these piecewise smooth integrands without a
// tolerance or a refinement rule).  Reading: Romberg's table on [a, b]
// (trapezoid sums with 1, 2, 4, ... panels and Richardson's extrapolation)
// for up to 6 rows; the interval is accepted, from the third row on, when
// two successive diagonal entries differ by at most its tolerance in the
// max-norm over the components (or by 1e-14 times the largest component, the
// rounding level of the sums); otherwise it is halved, each half with half
// the tolerance, down to 30 halvings.  Hexahedron faces: iterated, the outer
// rule over t of the inner integral over s (inner tolerance a tenth of the
// outer).  The components are P_plus, P_minus (nf x nf each), m_plus,
// m_minus.

namespace {

constexpr int kRombergRows = 6;
constexpr int kRombergDepth = 30;

// f(s, k, out): the m components at the k points s, out[k][m]
using PointFn = std::function<void(const double*, int, double*)>;

void romberg(const PointFn& f, int m, double a, double b, double tol, int depth, double* result) {
    const double h = b - a;
    std::vector<double> prev((size_t)(kRombergRows + 1) * m), cur((size_t)(kRombergRows + 1) * m);
    std::vector<double> vals(2 * (size_t)m), pts;
    const double ends[2] = {a, b};
    f(ends, 2, vals.data());
    for (int c = 0; c < m; ++c) prev[c] = 0.5 * h * (vals[c] + vals[(size_t)m + c]);
    for (int k = 1; k <= kRombergRows; ++k) {
        const int n_new = 1 << (k - 1);
        const double hk = h / (double)(1 << k);
        pts.resize(n_new);
        for (int i = 0; i < n_new; ++i) pts[i] = a + hk * (2.0 * i + 1.0);
        vals.resize((size_t)n_new * m);
        f(pts.data(), n_new, vals.data());
        for (int c = 0; c < m; ++c) {
            double sum = 0.0;
            for (int i = 0; i < n_new; ++i) sum += vals[(size_t)i * m + c];
            cur[c] = 0.5 * prev[c] + hk * sum;
        }
        double p4 = 1.0;
        for (int j = 1; j <= k; ++j) {
            p4 *= 4.0;
            for (int c = 0; c < m; ++c) {
                const double t = cur[(size_t)(j - 1) * m + c];
                cur[(size_t)j * m + c] = t + (t - prev[(size_t)(j - 1) * m + c]) / (p4 - 1.0);
            }
        }
        if (k >= 2) {
            double diff = 0.0, big = 0.0;
            for (int c = 0; c < m; ++c) {
                diff = std::max(diff, std::fabs(cur[(size_t)k * m + c] - prev[(size_t)(k - 1) * m + c]));
                big = std::max(big, std::fabs(cur[(size_t)k * m + c]));
            }
            if (diff <= std::max(tol, 1e-14 * big)) {
                std::copy(&cur[(size_t)k * m], &cur[(size_t)k * m] + m, result);
                return;
            }
        }
        prev.swap(cur);
    }
    if (depth >= kRombergDepth) {
        std::copy(&prev[(size_t)kRombergRows * m], &prev[(size_t)kRombergRows * m] + m, result);
        return;
    }
    const double mid = 0.5 * (a + b);
    std::vector<double> left(m), right(m);
    romberg(f, m, a, mid, 0.5 * tol, depth + 1, left.data());
    romberg(f, m, mid, b, 0.5 * tol, depth + 1, right.data());
    for (int c = 0; c < m; ++c) result[c] = left[c] + right[c];
}

// Components at one face point from g = Omega . N and the trace values phi.
void face_components(double g, const double* phi, int nf, double* out) {
    const double gp = std::max(g, 0.0), gm = std::max(-g, 0.0);
    for (int i = 0; i < nf; ++i)
        for (int j = 0; j < nf; ++j) {
            out[i * nf + j] = gp * phi[i] * phi[j];
            out[nf * nf + i * nf + j] = gm * phi[i] * phi[j];
        }
    out[2 * nf * nf] = gp;
    out[2 * nf * nf + 1] = gm;
}

void romberg_face(const HostProblem& hp, int64_t f, const double* om, double tol, double& mp, double& mm,
                  double* Pp, double* Pm) {
    const int dim = hp.dim, r = hp.r, p = hp.p, nf = hp.nf, m = 2 * nf * nf + 2;
    std::vector<double> geo(r + 1);
    for (int a = 0; a <= r; ++a) geo[a] = (double)a / r;
    const std::vector<double> dg = gll01(p);
    std::vector<double> out(m);
    if (dim == 3 && hp.simplex) {
        // triangular face in collapsed coordinates: (s, t) = (u, v (1 - u)),
        // area element 1 - u; u outer, v inner
        const int nfc = (r + 1) * (r + 2) / 2;
        const double* X = &hp.f_ctrl[(size_t)f * nfc * 3];
        const TriBasis tg(tri_geometry_nodes(r), r), td(tri_dg_nodes(p), p);
        auto point = [&](double u, double v, double* w) {
            double gs[10], gt[10], phi[10], N[3];
            const double s = u, t = v * (1.0 - u);
            tg.eval(s, t, nullptr, gs, gt);
            td.eval(s, t, phi, nullptr, nullptr);
            tri_face_normal(X, nfc, gs, gt, N);
            face_components(om[0] * N[0] + om[1] * N[1] + om[2] * N[2], phi, nf, w);
            for (int c = 0; c < m; ++c) w[c] *= 1.0 - u;
        };
        PointFn outer = [&](const double* u, int k, double* v) {
            for (int q = 0; q < k; ++q) {
                const double uq = u[q];
                PointFn inner = [&](const double* vv, int kv, double* w) {
                    for (int i = 0; i < kv; ++i) point(uq, vv[i], w + (size_t)i * m);
                };
                romberg(inner, m, 0.0, 1.0, 0.1 * tol, 0, v + (size_t)q * m);
            }
        };
        romberg(outer, m, 0.0, 1.0, tol, 0, out.data());
    } else if (dim == 2) {
        const double* mo = &hp.fnd.mono[(size_t)f * 2 * r];
        PointFn fn = [&](const double* s, int k, double* v) {
            double phi[8];
            for (int q = 0; q < k; ++q) {
                double g = 0.0, sp = 1.0;
                for (int c = 0; c < r; ++c) {
                    g += (om[0] * mo[c] + om[1] * mo[r + c]) * sp;
                    sp *= s[q];
                }
                lagrange_eval(dg, s[q], phi, nullptr);
                face_components(g, phi, nf, v + (size_t)q * m);
            }
        };
        romberg(fn, m, 0.0, 1.0, tol, 0, out.data());
    } else {
        const double* X = &hp.f_ctrl[(size_t)f * (r + 1) * (r + 1) * 3];
        const double sgn = hp.f_axis[f] == 1 ? -1.0 : 1.0;
        auto point = [&](double s, double t, double* v) {
            double Vs[4], Ds[4], Vt[4], Dt[4], us[4], ut[4], phi[16];
            lagrange_eval(geo, s, Vs, Ds);
            lagrange_eval(geo, t, Vt, Dt);
            double t1[3] = {0, 0, 0}, t2[3] = {0, 0, 0};
            for (int bt = 0; bt <= r; ++bt)
                for (int bs = 0; bs <= r; ++bs) {
                    const double* x = &X[(bt * (r + 1) + bs) * 3];
                    for (int c = 0; c < 3; ++c) {
                        t1[c] += x[c] * Ds[bs] * Vt[bt];
                        t2[c] += x[c] * Vs[bs] * Dt[bt];
                    }
                }
            const double N0 = sgn * (t1[1] * t2[2] - t1[2] * t2[1]);
            const double N1 = sgn * (t1[2] * t2[0] - t1[0] * t2[2]);
            const double N2 = sgn * (t1[0] * t2[1] - t1[1] * t2[0]);
            lagrange_eval(dg, s, us, nullptr);
            lagrange_eval(dg, t, ut, nullptr);
            for (int bt = 0; bt <= p; ++bt)
                for (int bs = 0; bs <= p; ++bs) phi[bt * (p + 1) + bs] = us[bs] * ut[bt];
            face_components(om[0] * N0 + om[1] * N1 + om[2] * N2, phi, nf, v);
        };
        PointFn outer = [&](const double* t, int k, double* v) {
            for (int q = 0; q < k; ++q) {
                const double tq = t[q];
                PointFn inner = [&](const double* s, int ks, double* w) {
                    for (int i = 0; i < ks; ++i) point(s[i], tq, w + (size_t)i * m);
                };
                romberg(inner, m, 0.0, 1.0, 0.1 * tol, 0, v + (size_t)q * m);
            }
        };
        romberg(outer, m, 0.0, 1.0, tol, 0, out.data());
    }
    std::copy(out.begin(), out.begin() + nf * nf, Pp);
    std::copy(out.begin() + nf * nf, out.begin() + 2 * nf * nf, Pm);
    mp = out[2 * nf * nf];
    mm = out[2 * nf * nf + 1];
}

// Romberg replaces the fixed rule on a sign-changing face, except on a face
// along the direction (int |g| at most 1e-12 |int N|), which the graph drops.
void maybe_romberg(const HostProblem& hp, int64_t f, const double* om, double& mp, double& mm, double* Pp,
                   double* Pm) {
    if (hp.face_rule != SNSW_FACE_ROMBERG) return;
    double na = 0.0;
    for (int k = 0; k < hp.dim; ++k) na += hp.Nint[(size_t)f * hp.dim + k] * hp.Nint[(size_t)f * hp.dim + k];
    const bool interior = hp.f_minus[f] >= 0 && hp.f_plus[f] >= 0;
    if (interior && mp + mm <= 1e-12 * std::sqrt(na)) return;
    romberg_face(hp, f, om, hp.face_tol * (mp + mm), mp, mm, Pp, Pm);
}

}  // namespace

// Integrals of one face for direction om.  Returns the class; measures
// mp = int max(g,0), mm = int max(-g,0); for FC_KINK also Pp, Pm (nf x nf).
uint8_t face_integrals(const HostProblem& hp, int64_t f, const double* om, double& mp,
                       double& mm, double* Pp, double* Pm);

uint8_t face_integrals(const HostProblem& hp, int64_t f, const double* om, double& mp,
                       double& mm, double* Pp, double* Pm) {
    const int dim = hp.dim, r = hp.r, p = hp.p, nf = hp.nf;
    const FaceNormalData& nd = hp.fnd;
    const double* Nf = &hp.Nint[(size_t)f * dim];
    double gbar = 0.0;
    for (int k = 0; k < dim; ++k) gbar += om[k] * Nf[k];
    if (dim == 2) {
        const double* mo = &nd.mono[(size_t)f * 2 * r];
        double c[4] = {0, 0, 0, 0};
        for (int k = 0; k < r; ++k) c[k] = om[0] * mo[k] + om[1] * mo[r + k];
        double roots[2];
        int nr = 0;
        auto push = [&](double s) { if (s > 0.0 && s < 1.0) roots[nr++] = s; };
        if (r == 2) {
            if (c[1] != 0.0) push(-c[0] / c[1]);
        } else if (r == 3) {
            const double A = c[2], Bq = c[1], C = c[0];
            if (A == 0.0) {
                if (Bq != 0.0) push(-C / Bq);
            } else {
                const double disc = Bq * Bq - 4.0 * A * C;
                if (disc > 0.0) {
                    const double sq = std::sqrt(disc);
                    const double qq = -0.5 * (Bq + (Bq >= 0.0 ? sq : -sq));
                    push(qq / A);
                    if (qq != 0.0) push(C / qq);
                }
            }
        } else if (r > 3) {
            throw Error(SNSW_E_UNSUPPORTED, "2D geometry order r > 3 is not supported");
        }
        if (nr == 0) {
            // no sign change inside the face: sign of g at the midpoint
            double gm = 0.0, sp = 1.0;
            for (int k = 0; k < r; ++k) { gm += c[k] * sp; sp *= 0.5; }
            if (gm >= 0.0) { mp = gbar; mm = 0.0; return FC_POS; }
            mp = 0.0; mm = -gbar; return FC_NEG;
        }
        if (nr == 2 && roots[1] < roots[0]) std::swap(roots[0], roots[1]);
        double bp[4] = {0.0, 0, 0, 0};
        int nb = 1;
        for (int i = 0; i < nr; ++i) bp[nb++] = roots[i];
        bp[nb++] = 1.0;
        const int ng = (r + 2 * p + 1) / 2;
        std::vector<double> xg, wg;
        gauss_legendre01(ng, xg, wg);
        const std::vector<double> dg = gll01(p);
        std::fill(Pp, Pp + nf * nf, 0.0);
        std::fill(Pm, Pm + nf * nf, 0.0);
        mp = mm = 0.0;
        double phi[8];
        for (int piece = 0; piece + 1 < nb; ++piece) {
            const double s0 = bp[piece], h = bp[piece + 1] - bp[piece];
            for (int q = 0; q < ng; ++q) {
                const double s = s0 + h * xg[q], ww = h * wg[q];
                double g = 0.0, sp = 1.0;
                for (int k = 0; k < r; ++k) { g += c[k] * sp; sp *= s; }
                lagrange_eval(dg, s, phi, nullptr);
                const double wp = ww * std::max(g, 0.0), wm = ww * std::max(-g, 0.0);
                mp += wp;
                mm += wm;
                for (int i = 0; i < nf; ++i)
                    for (int j = 0; j < nf; ++j) {
                        Pp[i * nf + j] += wp * phi[i] * phi[j];
                        Pm[i * nf + j] += wm * phi[i] * phi[j];
                    }
            }
        }
        maybe_romberg(hp, f, om, mp, mm, Pp, Pm);
        return FC_KINK;
    }
    // 3D: cheap bound first (|Omega . N_mean| above the largest deviation of
    // N from its mean at the rule's points: no sign change there)
    const double R = nd.Rf[f];
    const double gmean = hp.simplex ? 2.0 * gbar : gbar;
    if (std::fabs(gmean) > R * (1.0 + 1e-9) + 1e-300) {
        if (gbar > 0.0) { mp = gbar; mm = 0.0; return FC_POS; }
        mp = 0.0; mm = -gbar; return FC_NEG;
    }
    if (hp.simplex) {
        // triangular faces: Omega . N at the points of the composite rule
        const int nfc = nd.nfc;
        const double* X = &hp.f_ctrl[(size_t)f * nfc * 3];
        const size_t Qc = nd.cw.size();
        std::vector<double> g(Qc);
        double gmin = 1e300, gmax = -1e300;
        for (size_t q = 0; q < Qc; ++q) {
            double N[3];
            tri_face_normal(X, nfc, &nd.tgs[q * nfc], &nd.tgt[q * nfc], N);
            g[q] = om[0] * N[0] + om[1] * N[1] + om[2] * N[2];
            gmin = std::min(gmin, g[q]);
            gmax = std::max(gmax, g[q]);
        }
        if (gmin >= 0.0) { mp = gbar; mm = 0.0; return FC_POS; }
        if (gmax <= 0.0) { mp = 0.0; mm = -gbar; return FC_NEG; }
        std::fill(Pp, Pp + nf * nf, 0.0);
        std::fill(Pm, Pm + nf * nf, 0.0);
        mp = mm = 0.0;
        for (size_t q = 0; q < Qc; ++q) {
            const double wp = nd.cw[q] * std::max(g[q], 0.0), wm = nd.cw[q] * std::max(-g[q], 0.0);
            mp += wp;
            mm += wm;
            const double* ph = &nd.cphi[q * nf];
            for (int i = 0; i < nf; ++i)
                for (int j = 0; j < nf; ++j) {
                    Pp[i * nf + j] += wp * ph[i] * ph[j];
                    Pm[i * nf + j] += wm * ph[i] * ph[j];
                }
        }
        maybe_romberg(hp, f, om, mp, mm, Pp, Pm);
        return FC_KINK;
    }
    const double* X = &hp.f_ctrl[(size_t)f * (r + 1) * (r + 1) * 3];
    const int a = hp.f_axis[f];
    const size_t Qc = nd.cw.size();
    std::vector<double> g(Qc);
    double gmin = 1e300, gmax = -1e300;
    for (size_t q = 0; q < Qc; ++q) {
        const int i = nd.ci[q], j = nd.cj[q];
        const double* Vs = &nd.gV1[i * (r + 1)];
        const double* Ds = &nd.gD1[i * (r + 1)];
        const double* Vt = &nd.gV1[j * (r + 1)];
        const double* Dt = &nd.gD1[j * (r + 1)];
        double t1[3] = {0, 0, 0}, t2[3] = {0, 0, 0};
        for (int bt = 0; bt <= r; ++bt)
            for (int bs = 0; bs <= r; ++bs) {
                const double* x = &X[(bt * (r + 1) + bs) * 3];
                for (int cc = 0; cc < 3; ++cc) {
                    t1[cc] += x[cc] * Ds[bs] * Vt[bt];
                    t2[cc] += x[cc] * Vs[bs] * Dt[bt];
                }
            }
        double N0 = t1[1] * t2[2] - t1[2] * t2[1];
        double N1 = t1[2] * t2[0] - t1[0] * t2[2];
        double N2 = t1[0] * t2[1] - t1[1] * t2[0];
        if (a == 1) { N0 = -N0; N1 = -N1; N2 = -N2; }
        g[q] = om[0] * N0 + om[1] * N1 + om[2] * N2;
        gmin = std::min(gmin, g[q]);
        gmax = std::max(gmax, g[q]);
    }
    if (gmin >= 0.0) { mp = gbar; mm = 0.0; return FC_POS; }
    if (gmax <= 0.0) { mp = 0.0; mm = -gbar; return FC_NEG; }
    std::fill(Pp, Pp + nf * nf, 0.0);
    std::fill(Pm, Pm + nf * nf, 0.0);
    mp = mm = 0.0;
    for (size_t q = 0; q < Qc; ++q) {
        const double wp = nd.cw[q] * std::max(g[q], 0.0), wm = nd.cw[q] * std::max(-g[q], 0.0);
        mp += wp;
        mm += wm;
        const double* ph = &nd.cphi[q * nf];
        for (int i = 0; i < nf; ++i)
            for (int j = 0; j < nf; ++j) {
                Pp[i * nf + j] += wp * ph[i] * ph[j];
                Pm[i * nf + j] += wm * ph[i] * ph[j];
            }
    }
    (void)p;
    maybe_romberg(hp, f, om, mp, mm, Pp, Pm);
    return FC_KINK;
}

}  // namespace snsw
