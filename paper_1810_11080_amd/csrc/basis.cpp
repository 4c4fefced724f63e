// 1D rules and Lagrange bases on [0, 1] for the host setup.
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

}  // namespace snsw
