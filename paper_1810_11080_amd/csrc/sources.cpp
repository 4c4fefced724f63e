// Direction-dependent sources and tabulated boundary inflow.
//
// The load vector of eq. qVectorDef has two parts: the volume source,
// int q_d u_m over the element, and the inflow through the domain boundary,
// int_{inflow part of the boundary} |Omega . n| psi_inc u_m.  An isotropic
// source enters every direction alike and stays in the per-element source
// term of the sweep; a source that depends on the direction (e.g. a
// manufactured solution) and an incident flux tabulated per direction and
// boundary node are folded, once at setup, into a fixed right-hand side per
// (element, direction) pair:
//   rhs[d][e] = M_e q_d,e + sum over the boundary slots s of e of P_in(s, d) psi_inc,d,e|_s
// Both inputs are nodal values at the element's DG nodes (their DG
// interpolants are integrated exactly); P_in is the inflow face block the
// sweep kernels use for that slot (normal moments for a face without a sign
// change of Omega . n, the split table for a re-entrant face).
#include <algorithm>
#include <cmath>

#include "host.hpp"

namespace snsw {

void build_fixed_rhs(HostProblem& hp) {
    hp.rhs_fixed.clear();
    const bool have_q = !hp.q_dir.empty(), have_tab = !hp.psi_tab.empty();
    if (!have_q && !have_tab) return;
    const int64_t E = hp.E;
    const int n = hp.n, nf = hp.nf, ns = hp.nslot, dim = hp.dim, D = hp.D;
    hp.rhs_fixed.assign((size_t)D * E * n, 0.0);
    parallel_for(D, hp.nthreads, [&](int64_t d0, int64_t d1) {
        std::vector<double> pin((size_t)nf * nf);
        for (int64_t d = d0; d < d1; ++d) {
            const DirGraph& g = hp.graphs[d];
            const double* om = &hp.omega[(size_t)d * 3];
            for (int64_t e = 0; e < E; ++e) {
                double* r = &hp.rhs_fixed[((size_t)d * E + e) * n];
                if (have_q) {
                    const double* Me = &hp.M[(size_t)e * n * n];
                    const double* qe = &hp.q_dir[((size_t)d * E + e) * n];
                    for (int i = 0; i < n; ++i) {
                        double s = 0.0;
                        for (int j = 0; j < n; ++j) s += Me[i * n + j] * qe[j];
                        r[i] += s;
                    }
                }
                if (!have_tab) continue;
                const double* pe = &hp.psi_tab[((size_t)d * E + e) * n];
                for (int s = 0; s < ns; ++s) {
                    if (hp.slot_nbr[(size_t)e * ns + s] >= 0) continue;   // interior face
                    const int32_t f = hp.slot_face[(size_t)e * ns + s];
                    const bool minus_side = slot_is_minus(hp, e, s);
                    const uint8_t fc = g.face_class[f];
                    if (fc == FC_KINK) {
                        const auto it = std::lower_bound(g.kink_face.begin(), g.kink_face.end(), f);
                        const double* T = &g.kink_tab[(size_t)(it - g.kink_face.begin()) * 2 * nf * nf];
                        std::copy(T + (minus_side ? nf * nf : 0), T + (minus_side ? 2 : 1) * nf * nf, pin.begin());
                    } else if ((fc == FC_POS) == minus_side) {
                        continue;   // outflow face
                    } else {
                        // P_in = -(outward normal) moments; outward = N on the minus side
                        const double sgn = minus_side ? -1.0 : 1.0;
                        const double* Bf = &hp.B[(size_t)f * dim * nf * nf];
                        for (int k = 0; k < nf * nf; ++k) {
                            double v = 0.0;
                            for (int a = 0; a < dim; ++a) v += om[a] * Bf[(size_t)a * nf * nf + k];
                            pin[k] = sgn * v;
                        }
                    }
                    const int32_t* tn = slot_trace(hp, e, s);
                    for (int la = 0; la < nf; ++la) {
                        double v = 0.0;
                        for (int b = 0; b < nf; ++b) v += pin[(size_t)la * nf + b] * pe[tn[b]];
                        r[tn[la]] += v;
                    }
                }
            }
        }
    });
}

}  // namespace snsw
