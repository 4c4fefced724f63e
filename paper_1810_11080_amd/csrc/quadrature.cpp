// Level-symmetric S_N quadrature (section 2: positive weights summing to
// 4*pi; the paper's runs use S_2 and S_4 level-symmetric sets).
//
// Cosines: mu_i^2 = mu_1^2 + (i-1) * 2 (1 - 3 mu_1^2) / (N - 2), i = 1..N/2,
// with the textbook mu_1 per order (S_2: 1/sqrt(3)); orders 2..12.  (S_16's
// moment system is rank deficient, so its weights are not fixed by it.)  Points of an octant are
// the triples (i, j, k) with i + j + k = N/2 + 2; points that are
// permutations of each other share a weight, fixed by the even moment
// conditions sum w mu_x^(2m) = 1/(2m+1), m < N/2 (solved in least squares
// with a Householder QR factorisation).  Ordering: octant [x<0] + 2[y<0] + 4[z<0],
// then i, then j.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>

#include "host.hpp"

namespace snsw {

static double mu1_of(int N) {
    switch (N) {
        case 2: return 1.0 / std::sqrt(3.0);
        case 4: return 0.3500212;
        case 6: return 0.2666355;
        case 8: return 0.2182179;
        case 10: return 0.1893213;
        case 12: return 0.1672126;
        default: throw Error(SNSW_E_INVALID_ARG, "unsupported level-symmetric order S" + std::to_string(N));
    }
}

void level_symmetric(int N, int dim, std::vector<double>& omega, std::vector<double>& w) {
    const int h = N / 2;
    const double mu1 = mu1_of(N);
    std::vector<double> mu(h);
    for (int i = 0; i < h; ++i)
        mu[i] = (N == 2) ? mu1 : std::sqrt(mu1 * mu1 + i * 2.0 * (1.0 - 3.0 * mu1 * mu1) / (N - 2));
    std::vector<std::array<int, 3>> pts;
    for (int i = 0; i < h; ++i)
        for (int j = 0; j < h - i; ++j) pts.push_back({i, j, h - 1 - i - j});
    // permutation classes
    std::map<std::array<int, 3>, int> cls;
    std::vector<int> cls_of(pts.size());
    for (size_t t = 0; t < pts.size(); ++t) {
        auto key = pts[t];
        std::sort(key.begin(), key.end());
        auto it = cls.find(key);
        if (it == cls.end()) it = cls.emplace(key, 0).first;
        (void)it;
    }
    int c = 0;
    for (auto& kv : cls) kv.second = c++;
    for (size_t t = 0; t < pts.size(); ++t) {
        auto key = pts[t];
        std::sort(key.begin(), key.end());
        cls_of[t] = cls[key];
    }
    const int nc = c;
    // A[m][c] = sum over points of class c of mu_x^(2m); b[m] = 1/(2m+1)
    std::vector<double> A(h * nc, 0.0), b(h);
    for (int m = 0; m < h; ++m) {
        b[m] = 1.0 / (2.0 * m + 1.0);
        for (size_t t = 0; t < pts.size(); ++t) A[m * nc + cls_of[t]] += std::pow(mu[pts[t][0]], 2.0 * m);
    }
    // least squares by Householder QR (A is h x nc, h >= nc)
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
