// Element geometry and direction-independent element matrices.
//
// Mesh map T_e(xi) = sum_m x_{e,m} v_m(xi), Q_r Lagrange at equispaced
// control points (eq. elementTransformation); Jacobian J = sum_m x_{e,m}
// grad v_m^T (eq. Jacobian).  With the Q_p Gauss-Lobatto nodal basis u_m:
//   M[m][n]    = int u_m u_n |J|                        (eq. localMtMatrix / sigma)
//   K_i[m][n]  = int (J^{-T} grad u_m)_i u_n |J|        (eq. localGMatrix:
//                                                         G = -sum_i Omega_i K_i)
// on a tensor Gauss-Legendre rule with p+r (2D) or p+ceil(3r/2) (3D) points
// per axis, exact for these polynomial integrands.
//
// Triangles (simplicial elements): P_r map at equispaced control points and
// P_p DG basis (Gauss-Lobatto points on the edges, equispaced inside), on
// the collapsed Gauss rule with p+r points per direction (exact for total
// degree 2(p+r)-2, the largest degree of these integrands).  Tetrahedra: the
// same with p + ceil(3r/2) points per direction (exact for 2p + 3r - 3).
#include <atomic>
#include <cmath>

#include "host.hpp"

namespace snsw {

namespace {

// Tensor-product tables: val[q][m] and grad[q][m][b], axis 0 fastest.
void tensor_tables(int dim, const std::vector<double>& nodes, const std::vector<double>& x1,
                   std::vector<double>& val, std::vector<double>& grad) {
    const int nn = (int)nodes.size(), nq1 = (int)x1.size();
    std::vector<double> V1(nq1 * nn), D1(nq1 * nn);
    for (int k = 0; k < nq1; ++k) lagrange_eval(nodes, x1[k], &V1[k * nn], &D1[k * nn]);
    int Q = 1, Nf = 1;
    for (int a = 0; a < dim; ++a) { Q *= nq1; Nf *= nn; }
    val.assign((size_t)Q * Nf, 0.0);
    grad.assign((size_t)Q * Nf * dim, 0.0);
    for (int q = 0; q < Q; ++q) {
        int qi[3] = {0, 0, 0}, rq = q;
        for (int a = 0; a < dim; ++a) { qi[a] = rq % nq1; rq /= nq1; }
        for (int m = 0; m < Nf; ++m) {
            int mi[3] = {0, 0, 0}, rm = m;
            for (int a = 0; a < dim; ++a) { mi[a] = rm % nn; rm /= nn; }
            double v = 1.0;
            for (int a = 0; a < dim; ++a) v *= V1[qi[a] * nn + mi[a]];
            val[(size_t)q * Nf + m] = v;
            for (int b = 0; b < dim; ++b) {
                double g = 1.0;
                for (int a = 0; a < dim; ++a) g *= (a == b ? D1 : V1)[qi[a] * nn + mi[a]];
                grad[((size_t)q * Nf + m) * dim + b] = g;
            }
        }
    }
}

// Reference tables of an element type: rule points' weights, the map's
// basis (values [Q][Nv], gradients [Q][Nv][dim]) and the DG basis (values
// [Q][n], gradients [Q][n][dim]) at the points.
struct RefTables {
    int Q = 0, Nv = 0;
    std::vector<double> w, Vg, Gg, U, GU;
};

int tensor_points_per_axis(const HostProblem& hp) {
    return hp.dim == 2 ? hp.p + hp.r : hp.p + (3 * hp.r + 1) / 2;
}

RefTables reference_tables(const HostProblem& hp, int extra) {
    const int dim = hp.dim, r = hp.r, p = hp.p;
    RefTables t;
    if (hp.simplex && dim == 3) {
        std::vector<double> x, y, z;
        tet_collapsed_rule(p + (3 * r + 1) / 2 + extra, x, y, z, t.w);
        t.Q = (int)t.w.size();
        const TetBasis geo(tet_geometry_nodes(r), r), dg(tet_dg_nodes(p), p);
        t.Nv = geo.n;
        t.Vg.resize((size_t)t.Q * geo.n);
        t.Gg.resize((size_t)t.Q * geo.n * 3);
        t.U.resize((size_t)t.Q * dg.n);
        t.GU.resize((size_t)t.Q * dg.n * 3);
        std::vector<double> dx(20), dy(20), dz(20);
        for (int q = 0; q < t.Q; ++q) {
            geo.eval(x[q], y[q], z[q], &t.Vg[(size_t)q * geo.n], dx.data(), dy.data(), dz.data());
            for (int m = 0; m < geo.n; ++m) {
                t.Gg[((size_t)q * geo.n + m) * 3 + 0] = dx[m];
                t.Gg[((size_t)q * geo.n + m) * 3 + 1] = dy[m];
                t.Gg[((size_t)q * geo.n + m) * 3 + 2] = dz[m];
            }
            dg.eval(x[q], y[q], z[q], &t.U[(size_t)q * dg.n], dx.data(), dy.data(), dz.data());
            for (int m = 0; m < dg.n; ++m) {
                t.GU[((size_t)q * dg.n + m) * 3 + 0] = dx[m];
                t.GU[((size_t)q * dg.n + m) * 3 + 1] = dy[m];
                t.GU[((size_t)q * dg.n + m) * 3 + 2] = dz[m];
            }
        }
        return t;
    }
    if (hp.simplex) {
        std::vector<double> x, y;
        tri_collapsed_rule(p + r + extra, x, y, t.w);
        t.Q = (int)t.w.size();
        const TriBasis geo(tri_geometry_nodes(r), r), dg(tri_dg_nodes(p), p);
        t.Nv = geo.n;
        t.Vg.resize((size_t)t.Q * geo.n);
        t.Gg.resize((size_t)t.Q * geo.n * 2);
        t.U.resize((size_t)t.Q * dg.n);
        t.GU.resize((size_t)t.Q * dg.n * 2);
        std::vector<double> dx(10), dy(10);
        for (int q = 0; q < t.Q; ++q) {
            geo.eval(x[q], y[q], &t.Vg[(size_t)q * geo.n], dx.data(), dy.data());
            for (int m = 0; m < geo.n; ++m) {
                t.Gg[((size_t)q * geo.n + m) * 2 + 0] = dx[m];
                t.Gg[((size_t)q * geo.n + m) * 2 + 1] = dy[m];
            }
            dg.eval(x[q], y[q], &t.U[(size_t)q * dg.n], dx.data(), dy.data());
            for (int m = 0; m < dg.n; ++m) {
                t.GU[((size_t)q * dg.n + m) * 2 + 0] = dx[m];
                t.GU[((size_t)q * dg.n + m) * 2 + 1] = dy[m];
            }
        }
        return t;
    }
    const int nq1 = tensor_points_per_axis(hp) + extra;
    std::vector<double> x1, w1;
    gauss_legendre01(nq1, x1, w1);
    std::vector<double> geo_nodes(r + 1);
    for (int a = 0; a <= r; ++a) geo_nodes[a] = (double)a / r;
    tensor_tables(dim, geo_nodes, x1, t.Vg, t.Gg);
    tensor_tables(dim, gll01(p), x1, t.U, t.GU);
    t.Q = 1;
    t.Nv = 1;
    for (int a = 0; a < dim; ++a) { t.Q *= nq1; t.Nv *= r + 1; }
    t.w.resize(t.Q);
    for (int q = 0; q < t.Q; ++q) {
        double ww = 1.0;
        int rq = q;
        for (int a = 0; a < dim; ++a) { ww *= w1[rq % nq1]; rq /= nq1; }
        t.w[q] = ww;
    }
    return t;
}

// Control points of element e, [nv][dim]: tensor elements in the local
// order a + (r+1) (b + (r+1) c), triangles in lattice order; from the
// structured lattice, or from the element's control-point list on
// unstructured meshes.
void element_ctrl(const HostProblem& hp, int64_t e, double* xe) {
    const int dim = hp.dim, r = hp.r;
    if (hp.unstructured) {
        const int Nv = hp.nv;
        for (int m = 0; m < Nv; ++m) {
            const int64_t id = hp.elem_nodes[(size_t)e * Nv + m];
            for (int c = 0; c < dim; ++c) xe[m * dim + c] = hp.nodes[(size_t)id * dim + c];
        }
        return;
    }
    int L[3] = {1, 1, 1};
    for (int a = 0; a < dim; ++a) L[a] = r * hp.nx[a] + 1;
    int ei[3] = {0, 0, 0};
    int64_t re = e;
    for (int ax = 0; ax < dim; ++ax) { ei[ax] = (int)(re % hp.nx[ax]); re /= hp.nx[ax]; }
    int Nv = 1;
    for (int a = 0; a < dim; ++a) Nv *= r + 1;
    for (int m = 0; m < Nv; ++m) {
        int mi[3] = {0, 0, 0}, rm = m;
        for (int ax = 0; ax < dim; ++ax) { mi[ax] = rm % (r + 1); rm /= r + 1; }
        int64_t lid = 0, stride = 1;
        for (int ax = 0; ax < dim; ++ax) { lid += (int64_t)(r * ei[ax] + mi[ax]) * stride; stride *= L[ax]; }
        for (int c = 0; c < dim; ++c) xe[m * dim + c] = hp.lattice[lid * dim + c];
    }
}

std::vector<double> equispaced(int r) {
    std::vector<double> g(r + 1);
    for (int a = 0; a <= r; ++a) g[a] = (double)a / r;
    return g;
}

}  // namespace

void node_coordinates(const HostProblem& hp, int64_t e0, int64_t count, double* xyz) {
    const int dim = hp.dim, n = hp.n;
    std::vector<double> Vg, Gg;
    if (hp.simplex && dim == 3) {
        const TetBasis geo(tet_geometry_nodes(hp.r), hp.r);
        const std::vector<double> xn = tet_dg_nodes(hp.p);
        Vg.resize((size_t)n * geo.n);
        for (int q = 0; q < n; ++q)
            geo.eval(xn[3 * q], xn[3 * q + 1], xn[3 * q + 2], &Vg[(size_t)q * geo.n], nullptr, nullptr, nullptr);
    } else if (hp.simplex) {
        const TriBasis geo(tri_geometry_nodes(hp.r), hp.r);
        const std::vector<double> xn = tri_dg_nodes(hp.p);
        Vg.resize((size_t)n * geo.n);
        for (int q = 0; q < n; ++q) geo.eval(xn[2 * q], xn[2 * q + 1], &Vg[(size_t)q * geo.n], nullptr, nullptr);
    } else {
        tensor_tables(dim, equispaced(hp.r), gll01(hp.p), Vg, Gg);
    }
    const int Nv = (int)(Vg.size() / n);
    std::vector<double> xe((size_t)Nv * dim);
    for (int64_t e = e0; e < e0 + count; ++e) {
        element_ctrl(hp, e, xe.data());
        for (int q = 0; q < n; ++q)
            for (int c = 0; c < dim; ++c) {
                double v = 0.0;
                for (int m = 0; m < Nv; ++m) v += xe[m * dim + c] * Vg[(size_t)q * Nv + m];
                xyz[((e - e0) * n + q) * dim + c] = v;
            }
    }
}

int volume_rule(const HostProblem& hp, int extra, int64_t e0, int64_t count, double* x, double* wdet,
                double* basis) {
    const int dim = hp.dim;
    if (!x) {
        if (hp.simplex && dim == 3) {
            const int nq = hp.p + (3 * hp.r + 1) / 2 + extra;
            return nq * nq * nq;
        }
        if (hp.simplex) return (hp.p + hp.r + extra) * (hp.p + hp.r + extra);
        int Q = 1;
        for (int a = 0; a < dim; ++a) Q *= tensor_points_per_axis(hp) + extra;
        return Q;
    }
    const RefTables t = reference_tables(hp, extra);
    const int Q = t.Q, Nv = t.Nv;
    if (basis) std::copy(t.U.begin(), t.U.end(), basis);
    std::vector<double> xe((size_t)Nv * dim);
    for (int64_t e = e0; e < e0 + count; ++e) {
        element_ctrl(hp, e, xe.data());
        for (int q = 0; q < Q; ++q) {
            double J[3][3] = {{0}}, X[3] = {0, 0, 0};
            for (int m = 0; m < Nv; ++m)
                for (int c = 0; c < dim; ++c) {
                    X[c] += xe[m * dim + c] * t.Vg[(size_t)q * Nv + m];
                    for (int b = 0; b < dim; ++b) J[c][b] += xe[m * dim + c] * t.Gg[((size_t)q * Nv + m) * dim + b];
                }
            double det;
            if (dim == 2) det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            else
                det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                      J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                      J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
            for (int c = 0; c < dim; ++c) x[((e - e0) * Q + q) * dim + c] = X[c];
            wdet[(e - e0) * Q + q] = t.w[q] * std::fabs(det);
        }
    }
    return Q;
}

void build_geometry(HostProblem& hp) {
    const int dim = hp.dim, n = hp.n;
    const RefTables t = reference_tables(hp, 0);
    const int Q = t.Q, Nv = t.Nv;
    const std::vector<double>&wq = t.w, &Gg = t.Gg, &U = t.U, &GU = t.GU;
    hp.M.assign((size_t)hp.E * n * n, 0.0);
    hp.K.assign((size_t)hp.E * dim * n * n, 0.0);
    std::atomic<bool> bad(false);

    parallel_for(hp.E, hp.nthreads, [&](int64_t e0, int64_t e1) {
        std::vector<double> xe(Nv * dim), a(n), gx(n * dim);
        double local_min = 1e300;
        for (int64_t e = e0; e < e1; ++e) {
            element_ctrl(hp, e, xe.data());
            double* Me = &hp.M[(size_t)e * n * n];
            double* Ke = &hp.K[(size_t)e * dim * n * n];
            for (int q = 0; q < Q; ++q) {
                double J[3][3] = {{0}};
                for (int m = 0; m < Nv; ++m)
                    for (int c = 0; c < dim; ++c)
                        for (int b = 0; b < dim; ++b) J[c][b] += xe[m * dim + c] * Gg[((size_t)q * Nv + m) * dim + b];
                double det, Ji[3][3];   // Ji = J^{-1}
                if (dim == 2) {
                    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
                    Ji[0][0] = J[1][1] / det; Ji[0][1] = -J[0][1] / det;
                    Ji[1][0] = -J[1][0] / det; Ji[1][1] = J[0][0] / det;
                } else {
                    double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
                    double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
                    double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
                    det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
                    Ji[0][0] = c00 / det;
                    Ji[1][0] = c01 / det;
                    Ji[2][0] = c02 / det;
                    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
                    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
                    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
                    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
                    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
                    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
                }
                if (det < local_min) local_min = det;
                const double wd = wq[q] * det;
                const double* Uq = &U[(size_t)q * n];
                for (int m = 0; m < n; ++m) {
                    a[m] = wd * Uq[m];
                    for (int i = 0; i < dim; ++i) {
                        double s = 0.0;
                        for (int b = 0; b < dim; ++b) s += Ji[b][i] * GU[((size_t)q * n + m) * dim + b];
                        gx[i * n + m] = wd * s;
                    }
                }
                for (int m = 0; m < n; ++m)
                    for (int nn2 = 0; nn2 < n; ++nn2) Me[m * n + nn2] += a[m] * Uq[nn2];
                for (int i = 0; i < dim; ++i)
                    for (int m = 0; m < n; ++m) {
                        const double gm = gx[i * n + m];
                        double* row = &Ke[((size_t)i * n + m) * n];
                        for (int nn2 = 0; nn2 < n; ++nn2) row[nn2] += gm * Uq[nn2];
                    }
            }
        }
        // per-chunk minimum is enough to detect an inverted element
        if (!(local_min > 0.0)) bad.store(true);
    });
    if (bad.load()) throw Error(SNSW_E_BAD_JACOBIAN, "non-positive Jacobian determinant in the mesh");
}

}  // namespace snsw
