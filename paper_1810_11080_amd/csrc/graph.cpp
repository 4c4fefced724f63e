// Per-direction dependency graph, cycle cutting and levels (section 3), and
// the combined (element, direction) schedule of the device sweep.
//
// Graph: vertices are elements; edge up -> down when the downwind element
// receives inflow through a shared face (its coupling block F_{down,up} is
// nonzero).  Weights (section 3, eq. graphWeight; ||.|| the max-entry norm):
// Unity 1, Face ||F||, SigInvFace ||M_{t,down}^{-1} F||, made integer as
// w = clamp(rint(z / z_max * 2^20), 1, 2^20) (ties to even; Unity: 1) so that
// everything after this point is exact integer work.
//
// Cycle cutting: Tarjan SCCs; in each component an order minimising the
// total weight of couplings whose upwind element is ordered after the
// downwind one (those are lagged).  Components of at most exact_max vertices:
// exact subset dynamic programme (vertices by ascending element id; the last
// vertex v of a subset T costs sum_{u in T\v} w(v->u); smallest v wins ties).
// Larger ones: weighted Eades-Lin-Smyth (peel the smallest-id sink / source
// repeatedly, else the vertex of largest w_out - w_in, smallest id on ties).
// Levels: ASAP levels of the graph without the lagged edges.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>

#include "host.hpp"

namespace snsw {

namespace {

constexpr double kTau = 1e-12;
constexpr double kQuant = 1048576.0;   // 2^20

struct Edge {
    int32_t down, up;
    double z;
};

// inverse of a small dense matrix (Gauss-Jordan, partial pivoting)
void invert(int n, const double* A, double* Ainv) {
    std::vector<double> a(A, A + n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ainv[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(a[i * n + k]) > std::fabs(a[piv * n + k])) piv = i;
        if (piv != k)
            for (int j = 0; j < n; ++j) {
                std::swap(a[k * n + j], a[piv * n + j]);
                std::swap(Ainv[k * n + j], Ainv[piv * n + j]);
            }
        const double d = 1.0 / a[k * n + k];
        for (int j = 0; j < n; ++j) { a[k * n + j] *= d; Ainv[k * n + j] *= d; }
        for (int i = 0; i < n; ++i) {
            if (i == k) continue;
            const double l = a[i * n + k];
            if (l == 0.0) continue;
            for (int j = 0; j < n; ++j) { a[i * n + j] -= l * a[k * n + j]; Ainv[i * n + j] -= l * Ainv[k * n + j]; }
        }
    }
}

// Tarjan's algorithm, iterative.  adj in CSR form.
std::vector<int32_t> tarjan(int64_t V, const std::vector<int64_t>& off, const std::vector<int32_t>& adj) {
    std::vector<int32_t> index(V, -1), low(V, 0), comp(V, -1);
    std::vector<char> on(V, 0);
    std::vector<int32_t> stack;
    std::vector<std::pair<int32_t, int64_t>> work;
    int32_t counter = 0, ncomp = 0;
    for (int64_t v0 = 0; v0 < V; ++v0) {
        if (index[v0] != -1) continue;
        index[v0] = low[v0] = counter++;
        stack.push_back((int32_t)v0);
        on[v0] = 1;
        work.emplace_back((int32_t)v0, off[v0]);
        while (!work.empty()) {
            auto& top = work.back();
            const int32_t v = top.first;
            if (top.second < off[v + 1]) {
                const int32_t u = adj[top.second++];
                if (index[u] == -1) {
                    index[u] = low[u] = counter++;
                    stack.push_back(u);
                    on[u] = 1;
                    work.emplace_back(u, off[u]);
                } else if (on[u]) {
                    low[v] = std::min(low[v], index[u]);
                }
            } else {
                work.pop_back();
                if (!work.empty()) {
                    const int32_t parent = work.back().first;
                    low[parent] = std::min(low[parent], low[v]);
                }
                if (low[v] == index[v]) {
                    while (true) {
                        const int32_t u = stack.back();
                        stack.pop_back();
                        on[u] = 0;
                        comp[u] = ncomp;
                        if (u == v) break;
                    }
                    ++ncomp;
                }
            }
        }
    }
    return comp;
}

// exact minimum-lagged-weight order of a small component (local indices)
std::vector<int> exact_order(int s, const std::vector<int64_t>& W) {
    const uint32_t full = (1u << s) - 1u;
    std::vector<int64_t> f(full + 1, 0);
    std::vector<int8_t> best(full + 1, -1);
    for (uint32_t T = 1; T <= full; ++T) {
        int64_t bc = 0;
        int bv = -1;
        for (int v = 0; v < s; ++v) {
            if (!((T >> v) & 1u)) continue;
            const uint32_t rest = T & ~(1u << v);
            int64_t c = f[rest];
            for (int u = 0; u < s; ++u)
                if ((rest >> u) & 1u) c += W[v * s + u];
            if (bv < 0 || c < bc) { bc = c; bv = v; }
        }
        f[T] = bc;
        best[T] = (int8_t)bv;
    }
    std::vector<int> rev;
    uint32_t T = full;
    while (T) {
        const int v = best[T];
        rev.push_back(v);
        T &= ~(1u << v);
    }
    std::reverse(rev.begin(), rev.end());
    return rev;
}

// weighted Eades-Lin-Smyth order of a component (local indices)
std::vector<int> eades_order(int s, const std::vector<std::vector<std::pair<int, int64_t>>>& out,
                             const std::vector<std::vector<std::pair<int, int64_t>>>& in) {
    std::vector<char> alive(s, 1);
    std::vector<int64_t> outdeg(s), indeg(s), wout(s, 0), win(s, 0);
    for (int v = 0; v < s; ++v) {
        outdeg[v] = (int64_t)out[v].size();
        indeg[v] = (int64_t)in[v].size();
        for (auto& e : out[v]) wout[v] += e.second;
        for (auto& e : in[v]) win[v] += e.second;
    }
    std::vector<int> head, tail_rev;
    int left = s;
    auto remove = [&](int v) {
        alive[v] = 0;
        --left;
        for (auto& e : out[v])
            if (alive[e.first]) { --indeg[e.first]; win[e.first] -= e.second; }
        for (auto& e : in[v])
            if (alive[e.first]) { --outdeg[e.first]; wout[e.first] -= e.second; }
    };
    while (left) {
        while (true) {
            int v = -1;
            for (int u = 0; u < s; ++u)
                if (alive[u] && outdeg[u] == 0) { v = u; break; }
            if (v < 0) break;
            remove(v);
            tail_rev.push_back(v);   // prepended to the tail sequence
        }
        while (true) {
            int v = -1;
            for (int u = 0; u < s; ++u)
                if (alive[u] && indeg[u] == 0) { v = u; break; }
            if (v < 0) break;
            remove(v);
            head.push_back(v);
        }
        if (left) {
            int bv = -1;
            int64_t bd = 0;
            for (int u = 0; u < s; ++u) {
                if (!alive[u]) continue;
                const int64_t dl = wout[u] - win[u];
                if (bv < 0 || dl > bd) { bd = dl; bv = u; }
            }
            remove(bv);
            head.push_back(bv);
        }
    }
    std::vector<int> order = head;
    for (auto it = tail_rev.rbegin(); it != tail_rev.rend(); ++it) order.push_back(*it);
    return order;
}

void build_direction(const HostProblem& hp, int d, const std::vector<double>& Minv, DirGraph& g) {
    const int nf = hp.nf, dim = hp.dim;
    const double* om = &hp.omega[(size_t)d * 3];
    g.face_class.assign(hp.F, FC_POS);
    g.face_drop.assign(hp.F, 0);
    g.kink_face.clear();
    g.kink_tab.clear();
    std::vector<Edge> edges;
    std::vector<double> Pp(nf * nf), Pm(nf * nf), Pin(nf * nf);
    for (int64_t f = 0; f < hp.F; ++f) {
        double mp = 0, mm = 0;
        const uint8_t cls = face_integrals(hp, f, om, mp, mm, Pp.data(), Pm.data());
        g.face_class[f] = cls;
        const bool interior = hp.f_minus[f] >= 0 && hp.f_plus[f] >= 0;
        uint8_t drop = 0;
        if (interior) {
            // a face along the direction (int |g| at most tau |int N|) couples
            // nothing; otherwise a side whose measure is at most tau int |g|
            // is dropped
            const double mabs = mp + mm;
            double na = 0.0;
            for (int k = 0; k < dim; ++k) na += hp.Nint[(size_t)f * dim + k] * hp.Nint[(size_t)f * dim + k];
            const bool tangential = mabs <= kTau * std::sqrt(na);
            if (tangential || mm <= kTau * mabs) { drop |= 1; mm = 0.0; }
            if (tangential || mp <= kTau * mabs) { drop |= 2; mp = 0.0; }
        }
        g.face_drop[f] = drop;
        if (cls == FC_KINK) {
            if (drop & 1) std::fill(Pm.begin(), Pm.end(), 0.0);
            if (drop & 2) std::fill(Pp.begin(), Pp.end(), 0.0);
            g.kink_face.push_back((int32_t)f);
            g.kink_tab.insert(g.kink_tab.end(), Pp.begin(), Pp.end());
            g.kink_tab.insert(g.kink_tab.end(), Pm.begin(), Pm.end());
        }
        if (!interior) continue;
        // two possible edges: plus -> minus (inflow P_minus), minus -> plus (P_plus)
        for (int side = 0; side < 2; ++side) {
            const double meas = side == 0 ? mm : mp;
            if (!(meas > 0.0)) continue;
            const int32_t down = side == 0 ? hp.f_minus[f] : hp.f_plus[f];
            const int32_t up = side == 0 ? hp.f_plus[f] : hp.f_minus[f];
            double z = 1.0;
            if (hp.weighting != SNSW_WEIGHT_UNITY) {
                if (cls == FC_KINK) {
                    std::memcpy(Pin.data(), side == 0 ? Pm.data() : Pp.data(), sizeof(double) * nf * nf);
                } else {
                    // non-kink: P_in = -(sum_k om_k B_k) for the minus side (g <= 0),
                    // +(sum_k om_k B_k) for the plus side (g >= 0)
                    const double sg = side == 0 ? -1.0 : 1.0;
                    const double* Bf = &hp.B[(size_t)f * dim * nf * nf];
                    for (int i = 0; i < nf * nf; ++i) {
                        double v = 0.0;
                        for (int k = 0; k < dim; ++k) v += om[k] * Bf[k * nf * nf + i];
                        Pin[i] = sg * v;
                    }
                }
                z = 0.0;
                if (hp.weighting == SNSW_WEIGHT_FACE) {
                    for (int i = 0; i < nf * nf; ++i) z = std::max(z, std::fabs(Pin[i]));
                } else {
                    const int32_t* tn = slot_trace(hp, down, face_slot(hp, f, side));
                    const int n = hp.n;
                    const double* Mi = &Minv[(size_t)down * n * n];
                    const double st = hp.sigma_t[down];
                    for (int m = 0; m < n; ++m)
                        for (int b = 0; b < nf; ++b) {
                            double v = 0.0;
                            for (int aa = 0; aa < nf; ++aa) v += Mi[m * n + tn[aa]] * Pin[aa * nf + b];
                            z = std::max(z, std::fabs(v / st));
                        }
                }
            }
            edges.push_back({down, up, z});
        }
    }
    // quantised weights
    double zmax = 0.0;
    for (auto& e : edges) zmax = std::max(zmax, e.z);
    std::sort(edges.begin(), edges.end(), [](const Edge& a, const Edge& b) {
        return a.down != b.down ? a.down < b.down : a.up < b.up;
    });
    const size_t m = edges.size();
    g.up.resize(m);
    g.down.resize(m);
    g.weight.resize(m);
    for (size_t i = 0; i < m; ++i) {
        g.up[i] = edges[i].up;
        g.down[i] = edges[i].down;
        int64_t w = 1;
        if (hp.weighting != SNSW_WEIGHT_UNITY) {
            double t = std::nearbyint(edges[i].z / zmax * kQuant);
            t = std::min(std::max(t, 1.0), kQuant);
            w = (int64_t)t;
        }
        g.weight[i] = w;
    }
    // CSR of out-edges (up -> down)
    const int64_t E = hp.E;
    std::vector<int64_t> off(E + 1, 0);
    for (size_t i = 0; i < m; ++i) ++off[g.up[i] + 1];
    for (int64_t v = 0; v < E; ++v) off[v + 1] += off[v];
    std::vector<int32_t> adj(m);
    std::vector<int64_t> adjw(m);
    {
        std::vector<int64_t> pos(off.begin(), off.end() - 1);
        for (size_t i = 0; i < m; ++i) {
            adj[pos[g.up[i]]] = g.down[i];
            adjw[pos[g.up[i]]++] = g.weight[i];
        }
    }
    std::vector<int32_t> comp = tarjan(E, off, adj);
    int32_t ncomp = 0;
    for (int64_t v = 0; v < E; ++v) ncomp = std::max(ncomp, comp[v] + 1);
    std::vector<int32_t> csize(ncomp, 0);
    for (int64_t v = 0; v < E; ++v) ++csize[comp[v]];
    std::vector<int64_t> coff(ncomp + 1, 0);
    for (int c = 0; c < ncomp; ++c) coff[c + 1] = coff[c] + csize[c];
    std::vector<int32_t> members(E);
    {
        std::vector<int64_t> pos(coff.begin(), coff.end() - 1);
        for (int64_t v = 0; v < E; ++v) members[pos[comp[v]]++] = (int32_t)v;   // ascending ids
    }
    std::vector<std::pair<int32_t, int32_t>> removed;   // (down, up)
    snsw_graph_stats st{};
    st.n_edges = (int64_t)m;
    std::vector<int> loc(E, -1);
    for (int c = 0; c < ncomp; ++c) {
        const int s = csize[c];
        if (s < 2) continue;
        st.max_scc = std::max<int64_t>(st.max_scc, s);
        if (s == 2) ++st.n_scc_simple;
        else { ++st.n_scc_large; st.n_elements_in_large += s; }
        const int32_t* vs = &members[coff[c]];
        for (int i = 0; i < s; ++i) loc[vs[i]] = i;
        std::vector<int> order;
        if (s <= hp.exact_max) {
            std::vector<int64_t> W((size_t)s * s, 0);
            for (int i = 0; i < s; ++i)
                for (int64_t k = off[vs[i]]; k < off[vs[i] + 1]; ++k)
                    if (comp[adj[k]] == c) W[(size_t)i * s + loc[adj[k]]] = adjw[k];
            order = exact_order(s, W);
        } else {
            std::vector<std::vector<std::pair<int, int64_t>>> out(s), in(s);
            for (int i = 0; i < s; ++i)
                for (int64_t k = off[vs[i]]; k < off[vs[i] + 1]; ++k)
                    if (comp[adj[k]] == c) {
                        out[i].emplace_back(loc[adj[k]], adjw[k]);
                        in[loc[adj[k]]].emplace_back(i, adjw[k]);
                    }
            order = eades_order(s, out, in);
        }
        std::vector<int> pos(s);
        for (int k = 0; k < s; ++k) pos[order[k]] = k;
        for (int i = 0; i < s; ++i)
            for (int64_t k = off[vs[i]]; k < off[vs[i] + 1]; ++k) {
                const int32_t u = adj[k];
                if (comp[u] == c && pos[i] > pos[loc[u]]) {
                    removed.emplace_back(u, vs[i]);
                    st.removed_weight += adjw[k];
                }
            }
        for (int i = 0; i < s; ++i) loc[vs[i]] = -1;
    }
    std::sort(removed.begin(), removed.end());
    g.rem_down.resize(removed.size());
    g.rem_up.resize(removed.size());
    for (size_t i = 0; i < removed.size(); ++i) {
        g.rem_down[i] = removed[i].first;
        g.rem_up[i] = removed[i].second;
    }
    st.n_removed = (int64_t)removed.size();
    // ASAP levels of the cut graph (Kahn)
    std::vector<int32_t> indeg(E, 0);
    auto is_removed = [&](int32_t up, int32_t down) {
        return std::binary_search(removed.begin(), removed.end(), std::make_pair(down, up));
    };
    std::vector<char> kept(m, 1);
    for (int64_t v = 0; v < E; ++v)
        for (int64_t k = off[v]; k < off[v + 1]; ++k)
            if (is_removed((int32_t)v, adj[k])) kept[k] = 0;
            else ++indeg[adj[k]];
    g.level.assign(E, 0);
    std::vector<int32_t> frontier, next;
    for (int64_t v = 0; v < E; ++v)
        if (indeg[v] == 0) frontier.push_back((int32_t)v);
    int64_t seen = 0;
    while (!frontier.empty()) {
        next.clear();
        for (int32_t u : frontier) {
            ++seen;
            for (int64_t k = off[u]; k < off[u + 1]; ++k) {
                if (!kept[k]) continue;
                const int32_t v = adj[k];
                g.level[v] = std::max(g.level[v], g.level[u] + 1);
                if (--indeg[v] == 0) next.push_back(v);
            }
        }
        frontier.swap(next);
    }
    if (seen != E) throw Error(SNSW_E_STATE, "cut graph is not acyclic (internal error)");
    int32_t lmax = 0;
    for (int64_t v = 0; v < E; ++v) lmax = std::max(lmax, g.level[v]);
    st.n_levels = E ? lmax + 1 : 0;
    g.stats = st;
}

}  // namespace

void build_graphs(HostProblem& hp) {
    std::vector<double> Minv;
    if (hp.weighting == SNSW_WEIGHT_SIGINVFACE) {
        const int n = hp.n;
        Minv.assign((size_t)hp.E * n * n, 0.0);
        parallel_for(hp.E, hp.nthreads, [&](int64_t e0, int64_t e1) {
            for (int64_t e = e0; e < e1; ++e) invert(n, &hp.M[(size_t)e * n * n], &Minv[(size_t)e * n * n]);
        });
    }
    hp.graphs.assign(hp.D, DirGraph());
    parallel_for(hp.D, hp.nthreads, [&](int64_t d0, int64_t d1) {
        for (int64_t d = d0; d < d1; ++d) build_direction(hp, (int)d, Minv, hp.graphs[d]);
    });
}

void build_schedule(HostProblem& hp) {
    const int64_t E = hp.E;
    const int D = hp.D, ns = hp.nslot;
    int32_t L = 0;
    for (int d = 0; d < D; ++d) L = std::max<int32_t>(L, (int32_t)hp.graphs[d].stats.n_levels);
    // global kink rows: per-direction tables concatenated
    std::vector<int64_t> kink_base(D + 1, 0);
    for (int d = 0; d < D; ++d) kink_base[d + 1] = kink_base[d] + (int64_t)hp.graphs[d].kink_face.size();
    hp.n_kinks = kink_base[D];
    const int nf2 = 2 * hp.nf * hp.nf;
    hp.kink_tab.assign((size_t)hp.n_kinks * nf2, 0.0);
    for (int d = 0; d < D; ++d)
        std::copy(hp.graphs[d].kink_tab.begin(), hp.graphs[d].kink_tab.end(),
                  hp.kink_tab.begin() + kink_base[d] * nf2);
    // lag flags per (direction, element): bit s set when slot s is lagged
    std::vector<std::vector<uint8_t>> lag(D);
    parallel_for(D, hp.nthreads, [&](int64_t d0, int64_t d1) {
        for (int64_t d = d0; d < d1; ++d) {
            lag[d].assign(E, 0);
            const DirGraph& g = hp.graphs[d];
            for (size_t i = 0; i < g.rem_down.size(); ++i) {
                const int32_t dn = g.rem_down[i], up = g.rem_up[i];
                for (int s = 0; s < ns; ++s)
                    if (hp.slot_nbr[(size_t)dn * ns + s] == up) lag[d][dn] |= (uint8_t)(1u << s);
            }
        }
    });
    std::vector<int64_t> count(L + 1, 0);
    for (int d = 0; d < D; ++d)
        for (int64_t e = 0; e < E; ++e) ++count[hp.graphs[d].level[e] + 1];
    // Levels are padded to a multiple of G = 64/n pairs (the pairs one
    // wavefront claims at once), so that a wavefront never holds a pair
    // together with one of its upwind pairs.  Padding entries have e = -1.
    const int64_t G = std::max(1, 64 / hp.n);
    hp.level_off.assign(L + 1, 0);
    for (int k = 0; k < L; ++k) hp.level_off[k + 1] = hp.level_off[k] + (count[k + 1] + G - 1) / G * G;
    const int64_t P = hp.level_off[L];
    hp.pairs.assign((size_t)P * 4, 0);
    for (int64_t t = 0; t < P; ++t) hp.pairs[(size_t)t * 4] = -1;
    hp.kink_idx.clear();
    std::vector<int64_t> pos(hp.level_off.begin(), hp.level_off.end() - 1);
    for (int64_t e = 0; e < E; ++e) {
        for (int d = 0; d < D; ++d) {
            const DirGraph& g = hp.graphs[d];
            const int64_t slot_pos = pos[g.level[e]]++;
            uint32_t packed = (uint32_t)d;
            const int32_t kb = (int32_t)hp.kink_idx.size();
            for (int s = 0; s < ns; ++s) {
                const int32_t f = hp.slot_face[(size_t)e * ns + s];
                const uint8_t fc = g.face_class[f];
                const bool minus_side = slot_is_minus(hp, e, s);
                // drop bits: 1 = P_minus side, 2 = P_plus side
                const bool in_dropped = (g.face_drop[f] & (minus_side ? 1 : 2)) != 0;
                const bool out_dropped = (g.face_drop[f] & (minus_side ? 2 : 1)) != 0;
                bool lagged = (lag[d][e] >> s) & 1u;
                uint32_t cls;
                if (fc == FC_KINK) {
                    cls = SC_KINK;
                    auto it = std::lower_bound(g.kink_face.begin(), g.kink_face.end(), f);
                    hp.kink_idx.push_back((int32_t)(kink_base[d] + (it - g.kink_face.begin())));
                    if (in_dropped) lagged = true;
                } else {
                    cls = ((fc == FC_POS) == minus_side) ? SC_OUT : SC_IN;
                    if ((cls == SC_IN && in_dropped) || (cls == SC_OUT && out_dropped)) cls = SC_NONE;
                }
                packed |= pack_slot(cls, lagged, s);
            }
            int32_t* pr = &hp.pairs[(size_t)slot_pos * 4];
            pr[0] = (int32_t)e;
            pr[1] = (int32_t)packed;
            pr[2] = kb;
            pr[3] = 0;
        }
    }
    // Every pair that a pair waits for (kept inflow) must lie in an earlier
    // batch of G pairs: the persistent kernel claims batches in schedule
    // order, so each awaited pair is owned by another, running wavefront.
    std::vector<int64_t> where((size_t)D * E, -1);
    for (int64_t t = 0; t < P; ++t) {
        const int32_t* pr = &hp.pairs[(size_t)t * 4];
        if (pr[0] < 0) continue;
        where[(size_t)((uint32_t)pr[1] & ((1u << kDirBits) - 1)) * E + pr[0]] = t;
    }
    for (size_t i = 0; i < where.size(); ++i)
        if (where[i] < 0) throw Error(SNSW_E_STATE, "schedule: a pair is missing");
    for (int64_t t = 0; t < P; ++t) {
        const int32_t* pr = &hp.pairs[(size_t)t * 4];
        if (pr[0] < 0) continue;
        const int64_t batch0 = t - t % G;
        const uint32_t packed = (uint32_t)pr[1];
        const int d = (int)(packed & ((1u << kDirBits) - 1));
        for (int s = 0; s < ns; ++s) {
            const uint32_t bits = packed >> (kDirBits + 3 * s);
            const uint32_t cls = bits & 3u;
            const bool lagged = (bits >> 2) & 1u;
            const int32_t nb = hp.slot_nbr[(size_t)pr[0] * ns + s];
            if ((cls == SC_IN || cls == SC_KINK) && !lagged && nb >= 0 && where[(size_t)d * E + nb] >= batch0)
                throw Error(SNSW_E_STATE, "schedule: a kept upwind pair does not precede its dependant");
        }
    }
}


void arrange_levels_for_cache(HostProblem& hp, int Dc) {
    const int D = hp.D;
    if (Dc <= 0) return;                          // all assembled: element-major, as built
    const bool split = Dc < D;
    const bool dir_major = hp.dim == 3;
    if (!split && !dir_major) return;
    const int64_t L = (int64_t)hp.level_off.size() - 1;
    const int64_t G = std::max(1, 64 / hp.n);
    const uint32_t dmask = (1u << kDirBits) - 1;
    std::vector<int32_t> pairs;
    std::vector<int64_t> off(L + 1, 0), cut(L, 0);
    pairs.reserve(hp.pairs.size());
    std::vector<std::array<int32_t, 4>> part;
    auto emit = [&](bool by_dir) {
        if (by_dir)
            std::stable_sort(part.begin(), part.end(), [&](const auto& a, const auto& b) {
                return ((uint32_t)a[1] & dmask) < ((uint32_t)b[1] & dmask);
            });
        for (const auto& r : part) pairs.insert(pairs.end(), r.begin(), r.end());
        while ((pairs.size() / 4) % G) {
            pairs.push_back(-1);
            pairs.push_back(0);
            pairs.push_back(0);
            pairs.push_back(0);
        }
        part.clear();
    };
    for (int64_t k = 0; k < L; ++k) {
        // entries of a level come element-major; the cached ones go
        // direction-major in 3D, the assembled ones stay element-major (they
        // share the element matrices across directions)
        for (int cached = 1; cached >= 0; --cached) {
            for (int64_t t = hp.level_off[k]; t < hp.level_off[k + 1]; ++t) {
                const int32_t* pr = &hp.pairs[(size_t)t * 4];
                if (pr[0] < 0) continue;
                if (((int)((uint32_t)pr[1] & dmask) < Dc) != (cached == 1)) continue;
                part.push_back({pr[0], pr[1], pr[2], pr[3]});
            }
            if (cached == 1) {
                emit(dir_major);
                cut[k] = (int64_t)pairs.size() / 4;
            } else {
                emit(false);
            }
        }
        off[k + 1] = (int64_t)pairs.size() / 4;
    }
    hp.pairs.swap(pairs);
    hp.level_off.swap(off);
    if (split) hp.level_split.swap(cut);
    else hp.level_split.clear();
}


bool build_tiled_schedule(HostProblem& hp, int T) {
    hp.tile = 0;
    hp.tlevel_off.clear();
    hp.tpairs.clear();
    hp.tintra.clear();
    if (hp.dim != 2 || T < 1 || T * T != std::max(1, 64 / hp.n)) return false;
    const int64_t E = hp.E;
    const int D = hp.D, ns = hp.nslot;
    const int nx = hp.nx[0];
    const int tx = (nx + T - 1) / T, ty = (hp.nx[1] + T - 1) / T;
    const int64_t NT = (int64_t)tx * ty;   // tile ids: [0, NT) T x T tiles, NT + e singleton of e
    const int G = T * T;
    auto base_tile = [&](int64_t e) { return (int64_t)((e % nx) / T) + (int64_t)tx * ((e / nx) / T); };
    auto group_of = [&](int64_t e) { return (int)((e % nx) % T) + T * (int)((e / nx) % T); };
    // entry of every (d, e) in the level schedule
    std::vector<int64_t> where((size_t)D * E, -1);
    const int64_t P = hp.level_off.back();
    for (int64_t t = 0; t < P; ++t) {
        const int32_t* pr = &hp.pairs[(size_t)t * 4];
        if (pr[0] >= 0) where[(size_t)((uint32_t)pr[1] & ((1u << kDirBits) - 1)) * E + pr[0]] = t;
    }
    auto kept_up = [&](const int32_t* pr, int s) -> int32_t {
        const uint32_t bits = (uint32_t)pr[1] >> (kDirBits + 3 * s);
        const uint32_t cls = bits & 3u;
        const bool lagged = (bits >> 2) & 1u;
        if ((cls != SC_IN && cls != SC_KINK) || lagged) return -1;
        return hp.slot_nbr[(size_t)pr[0] * ns + s];
    };
    // Per direction: tiles of the kept graph, contracted; tiles in a cycle
    // of the contracted graph are split into single elements (repeated
    // until it is acyclic, which single elements always are); then ASAP
    // levels of the tiles.
    const int64_t NI = NT + E;
    std::vector<std::vector<int64_t>> tile_id(D);
    std::vector<std::vector<int32_t>> tlev(D);   // [NI], -1 for unused ids
    parallel_for(D, hp.nthreads, [&](int64_t d0, int64_t d1) {
        for (int64_t d = d0; d < d1; ++d) {
            std::vector<int64_t>& tid = tile_id[d];
            tid.resize(E);
            for (int64_t e = 0; e < E; ++e) tid[e] = base_tile(e);
            std::vector<std::pair<int32_t, int32_t>> edges;   // element edges up -> down
            for (int64_t e = 0; e < E; ++e) {
                const int32_t* pr = &hp.pairs[(size_t)where[(size_t)d * E + e] * 4];
                for (int s = 0; s < ns; ++s) {
                    const int32_t up = kept_up(pr, s);
                    if (up >= 0) edges.emplace_back(up, (int32_t)e);
                }
            }
            while (true) {
                std::vector<std::pair<int32_t, int32_t>> tedges;
                for (auto& ed : edges) {
                    const int64_t a = tid[ed.first], b = tid[ed.second];
                    if (a != b) tedges.emplace_back((int32_t)a, (int32_t)b);
                }
                std::sort(tedges.begin(), tedges.end());
                tedges.erase(std::unique(tedges.begin(), tedges.end()), tedges.end());
                std::vector<int64_t> off(NI + 1, 0);
                for (auto& te : tedges) ++off[te.first + 1];
                for (int64_t i = 0; i < NI; ++i) off[i + 1] += off[i];
                std::vector<int32_t> adj(tedges.size());
                {
                    std::vector<int64_t> fill(off.begin(), off.end() - 1);
                    for (auto& te : tedges) adj[fill[te.first]++] = te.second;
                }
                const std::vector<int32_t> comp = tarjan(NI, off, adj);
                std::vector<int32_t> csize(NI, 0);
                for (int64_t i = 0; i < NI; ++i) ++csize[comp[i]];
                bool split = false;
                for (int64_t e = 0; e < E; ++e)
                    if (csize[comp[tid[e]]] > 1) {
                        tid[e] = NT + e;
                        split = true;
                    }
                if (split) continue;
                // ASAP levels (Kahn) of the used tile ids
                std::vector<int32_t> indeg(NI, 0);
                for (int32_t v : adj) ++indeg[v];
                std::vector<char> used(NI, 0);
                for (int64_t e = 0; e < E; ++e) used[tid[e]] = 1;
                std::vector<int32_t>& lev = tlev[d];
                lev.assign(NI, -1);
                std::vector<int32_t> queue;
                for (int64_t i = 0; i < NI; ++i)
                    if (used[i] && indeg[i] == 0) {
                        queue.push_back((int32_t)i);
                        lev[i] = 0;
                    }
                for (size_t h = 0; h < queue.size(); ++h) {
                    const int32_t t = queue[h];
                    for (int64_t k = off[t]; k < off[t + 1]; ++k) {
                        const int32_t b = adj[k];
                        lev[b] = std::max(lev[b], lev[t] + 1);
                        if (--indeg[b] == 0) queue.push_back(b);
                    }
                }
                break;
            }
        }
    });
    int32_t Lt = 0;
    for (int d = 0; d < D; ++d)
        for (int32_t l : tlev[d]) Lt = std::max(Lt, l + 1);
    std::vector<int64_t> count(Lt + 1, 0);
    for (int d = 0; d < D; ++d)
        for (int32_t l : tlev[d])
            if (l >= 0) ++count[l + 1];
    hp.tlevel_off.assign(Lt + 1, 0);
    for (int32_t l = 0; l < Lt; ++l) hp.tlevel_off[l + 1] = hp.tlevel_off[l] + count[l + 1] * G;
    const int64_t PT = hp.tlevel_off[Lt];
    hp.tpairs.assign((size_t)PT * 4, 0);
    hp.tintra.assign((size_t)PT, 0);
    for (int64_t t = 0; t < PT; ++t) hp.tpairs[(size_t)t * 4] = -1;
    // batches: level by level, direction by direction, tile id by tile id
    std::vector<int64_t> pos(hp.tlevel_off.begin(), hp.tlevel_off.end() - 1);
    std::vector<std::vector<int64_t>> batch_of(D);
    for (int d = 0; d < D; ++d) {
        batch_of[d].assign(NI, -1);
        for (int64_t i = 0; i < NI; ++i) {
            const int32_t l = tlev[d][i];
            if (l < 0) continue;
            batch_of[d][i] = pos[l];
            pos[l] += G;
        }
    }
    for (int d = 0; d < D; ++d)
        for (int64_t e = 0; e < E; ++e) {
            const int64_t src = where[(size_t)d * E + e];
            const int64_t tt = tile_id[d][e];
            const int64_t dst = batch_of[d][tt] + group_of(e);
            const int32_t* pr = &hp.pairs[(size_t)src * 4];
            int32_t* out = &hp.tpairs[(size_t)dst * 4];
            out[0] = pr[0];
            out[1] = pr[1];
            out[2] = pr[2];
            out[3] = 0;
            uint32_t intra = 0;
            for (int s = 0; s < ns; ++s) {
                const int32_t up = kept_up(pr, s);
                if (up < 0) continue;
                const int64_t tu = tile_id[d][up];
                if (tu == tt)
                    intra |= (1u << s) | ((uint32_t)group_of(up) << (kIntraGroupShift + 4 * s));
                else if (batch_of[d][tu] >= batch_of[d][tt])
                    throw Error(SNSW_E_STATE, "tiled schedule: an upwind tile does not precede its dependant");
            }
            hp.tintra[(size_t)dst] = (int32_t)intra;
        }
    hp.tile = T;
    return true;
}

}  // namespace snsw
