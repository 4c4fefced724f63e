// 1D rules and Lagrange bases on [0, 1] for the host setup, and the
// reference triangle of the simplicial elements.
#include <algorithm>
#include <cmath>

#include "host.hpp"

namespace snsw {

// Legendre P_n and its derivative at z in [-1, 1] (three-term recurrence).
static void legendre(int n, double z, double& P, double& dP) {
    double p0 = 1.0, p1 = z;
    if (n == 0) { P = 1.0; dP = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
    }
    P = p1;
    dP = n * (z * p1 - p0) / (z * z - 1.0);
}

void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double P = 0, dP = 1;
        for (int it = 0; it < 100; ++it) {
            legendre(n, z, P, dP);
            double dz = P / dP;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        legendre(n, z, P, dP);
        // z descends with i: store ascending on [0, 1]
        x[n - 1 - i] = 0.5 * (z + 1.0);
        w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dP * dP);   // (2/((1-z^2)P'^2)) / 2
    }
}

std::vector<double> gll01(int p) {
    std::vector<double> z(p + 1);
    z[0] = -1.0;
    z[p] = 1.0;
    // interior points: roots of P_p'; Newton with P_p'' from Legendre's ODE
    for (int j = 1; j < p; ++j) {
        double t = -std::cos(M_PI * j / p);
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(p, t, P, dP);
            double d2P = (2.0 * t * dP - p * (p + 1.0) * P) / (1.0 - t * t);
            double dt = dP / d2P;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        z[j] = t;
    }
    std::sort(z.begin(), z.end());
    std::vector<double> x(p + 1);
    for (int j = 0; j <= p; ++j) x[j] = 0.5 * (z[j] + 1.0);
    x[0] = 0.0;
    x[p] = 1.0;
    return x;
}

void lagrange_eval(const std::vector<double>& nodes, double x, double* val, double* der) {
    const int nn = (int)nodes.size();
    for (int m = 0; m < nn; ++m) {
        double v = 1.0;
        for (int j = 0; j < nn; ++j)
            if (j != m) v *= (x - nodes[j]) / (nodes[m] - nodes[j]);
        if (val) val[m] = v;
        if (der) {
            double s = 0.0;
            for (int j = 0; j < nn; ++j) {
                if (j == m) continue;
                double t = 1.0 / (nodes[m] - nodes[j]);
                for (int k = 0; k < nn; ++k)
                    if (k != m && k != j) t *= (x - nodes[k]) / (nodes[m] - nodes[k]);
                s += t;
            }
            der[m] = s;
        }
    }
}

std::vector<std::vector<double>> lagrange_derivative_monomials(const std::vector<double>& nodes) {
    const int nn = (int)nodes.size();
    std::vector<std::vector<double>> out(nn);
    for (int m = 0; m < nn; ++m) {
        // expand prod_{j != m} (x - x_j) / (x_m - x_j) into ascending powers
        std::vector<double> c(1, 1.0);
        for (int j = 0; j < nn; ++j) {
            if (j == m) continue;
            double den = nodes[m] - nodes[j];
            std::vector<double> nc(c.size() + 1, 0.0);
            for (size_t k = 0; k < c.size(); ++k) {
                nc[k + 1] += c[k] / den;
                nc[k] -= c[k] * nodes[j] / den;
            }
            c.swap(nc);
        }
        std::vector<double> d(std::max(1, nn - 1), 0.0);
        for (int k = 1; k < (int)c.size(); ++k) d[k - 1] = k * c[k];
        out[m] = d;
    }
    return out;
}

// ------------------------------------------------------------- triangles
// Reference triangle {x, y >= 0, x + y <= 1}, vertices v0 = (0, 0),
// v1 = (1, 0), v2 = (0, 1).  Nodes of order k sit on the lattice pairs
// (i, j), i + j <= k, numbered row by row (j slowest).

int tri_index(int k, int i, int j) { return j * (k + 1) - j * (j - 1) / 2 + i; }

std::vector<int32_t> tri_slot_nodes(int k, int s) {
    std::vector<int32_t> out(k + 1);
    for (int b = 0; b <= k; ++b) {
        const int i = s == 0 ? b : (s == 1 ? k - b : 0);
        const int j = s == 0 ? 0 : (s == 1 ? b : k - b);
        out[b] = tri_index(k, i, j);
    }
    return out;
}

std::vector<double> tri_geometry_nodes(int r) {
    std::vector<double> x;
    for (int j = 0; j <= r; ++j)
        for (int i = 0; i + j <= r; ++i) {
            x.push_back((double)i / r);
            x.push_back((double)j / r);
        }
    return x;
}

std::vector<double> tri_dg_nodes(int p) {
    const std::vector<double> g = gll01(p);
    std::vector<double> x;
    for (int j = 0; j <= p; ++j)
        for (int i = 0; i + j <= p; ++i) {
            const bool edge = i == 0 || j == 0 || i + j == p;
            x.push_back(edge ? g[i] : (double)i / p);
            x.push_back(edge ? g[j] : (double)j / p);
        }
    return x;
}

TriBasis::TriBasis(const std::vector<double>& nodes, int k_) : k(k_), n((k_ + 1) * (k_ + 2) / 2) {
    for (int c = 0; c <= k; ++c)
        for (int a = 0; a + c <= k; ++a) mono.push_back({a, c});
    // C = V^{-1}, V[node][monomial]: Gauss-Jordan with partial pivoting
    std::vector<double> V((size_t)n * n), I((size_t)n * n, 0.0);
    for (int m = 0; m < n; ++m) {
        I[(size_t)m * n + m] = 1.0;
        for (int t = 0; t < n; ++t)
            V[(size_t)m * n + t] = std::pow(nodes[2 * m], mono[t].first) * std::pow(nodes[2 * m + 1], mono[t].second);
    }
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r2 = c + 1; r2 < n; ++r2)
            if (std::fabs(V[(size_t)r2 * n + c]) > std::fabs(V[(size_t)piv * n + c])) piv = r2;
        if (std::fabs(V[(size_t)piv * n + c]) < 1e-14) throw Error(SNSW_E_STATE, "triangle nodes are not unisolvent");
        for (int t = 0; t < n; ++t) {
            std::swap(V[(size_t)c * n + t], V[(size_t)piv * n + t]);
            std::swap(I[(size_t)c * n + t], I[(size_t)piv * n + t]);
        }
        const double d = 1.0 / V[(size_t)c * n + c];
        for (int t = 0; t < n; ++t) {
            V[(size_t)c * n + t] *= d;
            I[(size_t)c * n + t] *= d;
        }
        for (int r2 = 0; r2 < n; ++r2) {
            if (r2 == c) continue;
            const double f = V[(size_t)r2 * n + c];
            if (f == 0.0) continue;
            for (int t = 0; t < n; ++t) {
                V[(size_t)r2 * n + t] -= f * V[(size_t)c * n + t];
                I[(size_t)r2 * n + t] -= f * I[(size_t)c * n + t];
            }
        }
    }
    C = I;   // C[monomial][basis function]
}

void TriBasis::eval(double x, double y, double* val, double* dx, double* dy) const {
    auto pw = [](double t, int e) { return e < 0 ? 0.0 : std::pow(t, e); };
    for (int m = 0; m < n; ++m) {
        if (val) val[m] = 0.0;
        if (dx) dx[m] = 0.0;
        if (dy) dy[m] = 0.0;
    }
    for (int t = 0; t < n; ++t) {
        const int a = mono[t].first, c = mono[t].second;
        const double v = pw(x, a) * pw(y, c), vx = a * pw(x, a - 1) * pw(y, c), vy = c * pw(x, a) * pw(y, c - 1);
        const double* Ct = &C[(size_t)t * n];
        for (int m = 0; m < n; ++m) {
            if (val) val[m] += v * Ct[m];
            if (dx) dx[m] += vx * Ct[m];
            if (dy) dy[m] += vy * Ct[m];
        }
    }
}

void tri_collapsed_rule(int nq, std::vector<double>& x, std::vector<double>& y, std::vector<double>& w) {
    std::vector<double> g, gw;
    gauss_legendre01(nq, g, gw);
    x.clear();
    y.clear();
    w.clear();
    for (int a = 0; a < nq; ++a)
        for (int b = 0; b < nq; ++b) {
            x.push_back(g[a]);
            y.push_back(g[b] * (1.0 - g[a]));
            w.push_back(gw[a] * gw[b] * (1.0 - g[a]));
        }
}

// ----------------------------------------------------------- tetrahedra
// Reference tetrahedron with vertices V0 = (0,0,0), V1 = (1,0,0),
// V2 = (0,1,0), V3 = (0,0,1); nodes of order k on the lattice triples
// (i, j, l), i + j + l <= k, numbered with l slowest, then j, then i.

int tet_index(int k, int i, int j, int l) {
    int m = 0;
    for (int ll = 0; ll < l; ++ll) m += (k + 1 - ll) * (k + 2 - ll) / 2;
    const int kk = k - l;   // the layer l is a triangle of order k - l
    return m + j * (kk + 1) - j * (j - 1) / 2 + i;
}

// Vertices of face slot s (the face opposite V_s), in the order that makes
// x_s x x_t point out of the element.
static const int kTetFace[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};

std::vector<int32_t> tet_slot_nodes(int k, int s) {
    std::vector<int32_t> out;
    for (int b = 0; b <= k; ++b)
        for (int a = 0; a + b <= k; ++a) {
            int c[4] = {0, 0, 0, 0};
            c[kTetFace[s][0]] = k - a - b;
            c[kTetFace[s][1]] = a;
            c[kTetFace[s][2]] = b;
            out.push_back(tet_index(k, c[1], c[2], c[3]));
        }
    return out;
}

std::vector<double> tet_geometry_nodes(int r) {
    std::vector<double> x;
    for (int l = 0; l <= r; ++l)
        for (int j = 0; j + l <= r; ++j)
            for (int i = 0; i + j + l <= r; ++i) {
                x.push_back((double)i / r);
                x.push_back((double)j / r);
                x.push_back((double)l / r);
            }
    return x;
}

std::vector<double> tet_dg_nodes(int p) {
    const std::vector<double> g = gll01(p);
    std::vector<double> x;
    for (int l = 0; l <= p; ++l)
        for (int j = 0; j + l <= p; ++j)
            for (int i = 0; i + j + l <= p; ++i) {
                const int c[4] = {p - i - j - l, i, j, l};
                int nz = 0;
                for (int v = 0; v < 4; ++v) nz += c[v] > 0;
                // on an edge (two nonzero coordinates): Gauss-Lobatto; else equispaced
                for (int v = 1; v < 4; ++v) x.push_back(nz <= 2 ? g[c[v]] : (double)c[v] / p);
            }
    return x;
}

TetBasis::TetBasis(const std::vector<double>& nodes, int k_) : k(k_), n((k_ + 1) * (k_ + 2) * (k_ + 3) / 6) {
    for (int c = 0; c <= k; ++c)
        for (int b = 0; b + c <= k; ++b)
            for (int a = 0; a + b + c <= k; ++a) mono.push_back({a, b, c});
    std::vector<double> V((size_t)n * n), I((size_t)n * n, 0.0);
    for (int m = 0; m < n; ++m) {
        I[(size_t)m * n + m] = 1.0;
        for (int t = 0; t < n; ++t)
            V[(size_t)m * n + t] = std::pow(nodes[3 * m], mono[t][0]) * std::pow(nodes[3 * m + 1], mono[t][1]) *
                                   std::pow(nodes[3 * m + 2], mono[t][2]);
    }
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r2 = c + 1; r2 < n; ++r2)
            if (std::fabs(V[(size_t)r2 * n + c]) > std::fabs(V[(size_t)piv * n + c])) piv = r2;
        if (std::fabs(V[(size_t)piv * n + c]) < 1e-14) throw Error(SNSW_E_STATE, "tetrahedron nodes are not unisolvent");
        for (int t = 0; t < n; ++t) {
            std::swap(V[(size_t)c * n + t], V[(size_t)piv * n + t]);
            std::swap(I[(size_t)c * n + t], I[(size_t)piv * n + t]);
        }
        const double d = 1.0 / V[(size_t)c * n + c];
        for (int t = 0; t < n; ++t) {
            V[(size_t)c * n + t] *= d;
            I[(size_t)c * n + t] *= d;
        }
        for (int r2 = 0; r2 < n; ++r2) {
            if (r2 == c) continue;
            const double f = V[(size_t)r2 * n + c];
            if (f == 0.0) continue;
            for (int t = 0; t < n; ++t) {
                V[(size_t)r2 * n + t] -= f * V[(size_t)c * n + t];
                I[(size_t)r2 * n + t] -= f * I[(size_t)c * n + t];
            }
        }
    }
    C = I;
}

void TetBasis::eval(double x, double y, double z, double* val, double* dx, double* dy, double* dz) const {
    auto pw = [](double t, int e) { return e < 0 ? 0.0 : std::pow(t, e); };
    for (int m = 0; m < n; ++m) {
        if (val) val[m] = 0.0;
        if (dx) dx[m] = 0.0;
        if (dy) dy[m] = 0.0;
        if (dz) dz[m] = 0.0;
    }
    for (int t = 0; t < n; ++t) {
        const int a = mono[t][0], b = mono[t][1], c = mono[t][2];
        const double v = pw(x, a) * pw(y, b) * pw(z, c);
        const double vx = a * pw(x, a - 1) * pw(y, b) * pw(z, c);
        const double vy = b * pw(x, a) * pw(y, b - 1) * pw(z, c);
        const double vz = c * pw(x, a) * pw(y, b) * pw(z, c - 1);
        const double* Ct = &C[(size_t)t * n];
        for (int m = 0; m < n; ++m) {
            if (val) val[m] += v * Ct[m];
            if (dx) dx[m] += vx * Ct[m];
            if (dy) dy[m] += vy * Ct[m];
            if (dz) dz[m] += vz * Ct[m];
        }
    }
}

void tet_collapsed_rule(int nq, std::vector<double>& x, std::vector<double>& y, std::vector<double>& z,
                        std::vector<double>& w) {
    std::vector<double> g, gw;
    gauss_legendre01(nq, g, gw);
    x.clear();
    y.clear();
    z.clear();
    w.clear();
    for (int a = 0; a < nq; ++a)
        for (int b = 0; b < nq; ++b)
            for (int c = 0; c < nq; ++c) {
                x.push_back(g[a]);
                y.push_back(g[b] * (1.0 - g[a]));
                z.push_back(g[c] * (1.0 - g[a]) * (1.0 - g[b]));
                w.push_back(gw[a] * gw[b] * gw[c] * (1.0 - g[a]) * (1.0 - g[a]) * (1.0 - g[b]));
            }
}

void tri_composite_rule(int K, int nq, std::vector<double>& s, std::vector<double>& t, std::vector<double>& w) {
    std::vector<double> x, y, wq;
    tri_collapsed_rule(nq, x, y, wq);
    s.clear();
    t.clear();
    w.clear();
    for (int j = 0; j < K; ++j)
        for (int i = 0; i + j < K; ++i) {
            for (size_t q = 0; q < wq.size(); ++q) {   // upward sub-triangle at corner (i, j) / K
                s.push_back((i + x[q]) / K);
                t.push_back((j + y[q]) / K);
                w.push_back(wq[q] / (K * K));
            }
            if (i + j < K - 1)
                for (size_t q = 0; q < wq.size(); ++q) {   // downward one, corner (i+1, j+1) / K
                    s.push_back((i + 1 - x[q]) / K);
                    t.push_back((j + 1 - y[q]) / K);
                    w.push_back(wq[q] / (K * K));
                }
        }
}

}  // namespace snsw
