// Level-symmetric S_N quadrature (section 2: positive weights summing to
// 4*pi; the paper's runs use S_2 and S_4 level-symmetric sets).
//
// Cosines: mu_i^2 = mu_1^2 + (i-1) * 2 (1 - 3 mu_1^2) / (N - 2), i = 1..N/2
// (S_2: mu_1 = 1/sqrt(3)); orders 2..12.  (S_16's moment system is rank
// deficient, so its weights are not fixed by it.)  Points of an octant are
// the triples (i, j, k) with i + j + k = N/2 + 2; points that are
// permutations of each other share a weight, fixed by the even moment
// conditions sum w mu_x^(2m) = 1/(2m+1), m < N/2 (solved in least squares
// with a Householder QR factorisation); mu_1 is fixed by the next even
// moment, m = N/2 (mu1_of).  Ordering: octant [x<0] + 2[y<0] + 4[z<0], then
// i, then j.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>

#include "host.hpp"

namespace snsw {

namespace {

struct OctantSet {
    int h = 0;                                // N/2 levels
    std::vector<std::array<int, 3>> pts;      // (i, j, k), i + j + k = h - 1
    std::vector<int> cls_of;                  // permutation class of each point
    int nc = 0;
};

OctantSet octant_set(int N) {
    OctantSet o;
    o.h = N / 2;
    for (int i = 0; i < o.h; ++i)
        for (int j = 0; j < o.h - i; ++j) o.pts.push_back({i, j, o.h - 1 - i - j});
    std::map<std::array<int, 3>, int> cls;
    for (auto key : o.pts) {
        std::sort(key.begin(), key.end());
        cls.emplace(key, 0);
    }
    for (auto& kv : cls) kv.second = o.nc++;
    for (auto key : o.pts) {
        std::sort(key.begin(), key.end());
        o.cls_of.push_back(cls[key]);
    }
    return o;
}

std::vector<double> level_cosines(int N, double mu1) {
    std::vector<double> mu(N / 2);
    for (int i = 0; i < N / 2; ++i)
        mu[i] = (N == 2) ? mu1 : std::sqrt(mu1 * mu1 + i * 2.0 * (1.0 - 3.0 * mu1 * mu1) / (N - 2));
    return mu;
}

// Class weights (octant sum 1) from the even moments m < N/2, in least
// squares by Householder QR (h equations, nc unknowns, h >= nc).
std::vector<double> class_weights(const OctantSet& o, const std::vector<double>& mu) {
    const int h = o.h, nc = o.nc;
    // A[m][c] = sum over points of class c of mu_x^(2m); b[m] = 1/(2m+1)
    std::vector<double> A(h * nc, 0.0), b(h);
    for (int m = 0; m < h; ++m) {
        b[m] = 1.0 / (2.0 * m + 1.0);
        for (size_t t = 0; t < o.pts.size(); ++t) A[m * nc + o.cls_of[t]] += std::pow(mu[o.pts[t][0]], 2.0 * m);
    }
    for (int k = 0; k < nc; ++k) {
        double norm = 0.0;
        for (int m = k; m < h; ++m) norm += A[m * nc + k] * A[m * nc + k];
        norm = std::sqrt(norm);
        if (norm == 0.0) continue;
        const double alpha = A[k * nc + k] > 0 ? -norm : norm;
        std::vector<double> v(h, 0.0);
        for (int m = k; m < h; ++m) v[m] = A[m * nc + k];
        v[k] -= alpha;
        double vv = 0.0;
        for (int m = k; m < h; ++m) vv += v[m] * v[m];
        if (vv == 0.0) continue;
        for (int j = k; j < nc; ++j) {
            double dot = 0.0;
            for (int m = k; m < h; ++m) dot += v[m] * A[m * nc + j];
            const double f = 2.0 * dot / vv;
            for (int m = k; m < h; ++m) A[m * nc + j] -= f * v[m];
        }
        double dot = 0.0;
        for (int m = k; m < h; ++m) dot += v[m] * b[m];
        const double f = 2.0 * dot / vv;
        for (int m = k; m < h; ++m) b[m] -= f * v[m];
    }
    std::vector<double> wc(nc);
    for (int k = nc - 1; k >= 0; --k) {
        double sum = b[k];
        for (int j = k + 1; j < nc; ++j) sum -= A[k * nc + j] * wc[j];
        wc[k] = sum / A[k * nc + k];
    }
    return wc;
}

// sum over the octant of w mu_x^N minus 1/(N+1): the first even moment the
// weights are not fitted to.
double next_moment_defect(const OctantSet& o, int N, double mu1, bool* positive = nullptr) {
    const std::vector<double> mu = level_cosines(N, mu1);
    const std::vector<double> wc = class_weights(o, mu);
    double s = 0.0;
    for (size_t t = 0; t < o.pts.size(); ++t) s += wc[o.cls_of[t]] * std::pow(mu[o.pts[t][0]], (double)N);
    if (positive) {
        *positive = true;
        for (double x : wc) *positive = *positive && x > 0.0;
    }
    return s - 1.0 / (N + 1);
}

// mu_1 of S_N: the level-symmetric sets leave mu_1 free after the weights
// are fitted to the moments below N, and are defined by the next one; the
// root of that condition in (0, 1/sqrt(3)) with all class weights positive
// (unique for S_4 .. S_12), bracketed on a grid and bisected.
double mu1_of(int N, const OctantSet& o) {
    if (N == 2) return 1.0 / std::sqrt(3.0);
    if (N < 2 || N > 12 || N % 2) throw Error(SNSW_E_INVALID_ARG, "unsupported level-symmetric order S" + std::to_string(N));
    const int steps = 1000;
    const double lo = 0.02, hi = 1.0 / std::sqrt(3.0) - 1e-4;
    double x0 = lo, f0 = next_moment_defect(o, N, lo);
    for (int k = 1; k <= steps; ++k) {
        const double x1 = lo + (hi - lo) * k / steps;
        const double f1 = next_moment_defect(o, N, x1);
        if (f0 == 0.0 || (f0 < 0.0) != (f1 < 0.0)) {
            double a = x0, b = x1, fa = f0;
            while (true) {
                const double m = 0.5 * (a + b);
                if (!(m > a && m < b)) break;
                const double fm = next_moment_defect(o, N, m);
                if (fm == 0.0) { a = b = m; break; }
                if ((fa < 0.0) == (fm < 0.0)) { a = m; fa = fm; } else b = m;
            }
            const double root = 0.5 * (a + b);
            bool pos = false;
            next_moment_defect(o, N, root, &pos);
            if (pos) return root;
        }
        x0 = x1;
        f0 = f1;
    }
    throw Error(SNSW_E_INVALID_ARG, "no positive level-symmetric set for S" + std::to_string(N));
}

}  // namespace

void level_symmetric(int N, int dim, std::vector<double>& omega, std::vector<double>& w) {
    if (N < 2 || N % 2) throw Error(SNSW_E_INVALID_ARG, "unsupported level-symmetric order S" + std::to_string(N));
    const OctantSet oct = octant_set(N);
    const std::vector<double> mu = level_cosines(N, mu1_of(N, oct));
    const std::vector<double> wc = class_weights(oct, mu);
    const auto& pts = oct.pts;
    const auto& cls_of = oct.cls_of;
    const int n_oct = dim == 3 ? 8 : 4;
    const double scale = 4.0 * M_PI / 8.0 * (dim == 2 ? 2.0 : 1.0);
    omega.clear();
    w.clear();
    for (int o = 0; o < n_oct; ++o) {
        double sx = (o & 1) ? -1.0 : 1.0, sy = (o & 2) ? -1.0 : 1.0, sz = (o & 4) ? -1.0 : 1.0;
        for (size_t t = 0; t < pts.size(); ++t) {
            omega.push_back(sx * mu[pts[t][0]]);
            omega.push_back(sy * mu[pts[t][1]]);
            omega.push_back(sz * mu[pts[t][2]]);
            w.push_back(wc[cls_of[t]] * scale);
        }
    }
}

}  // namespace snsw
