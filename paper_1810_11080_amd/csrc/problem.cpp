// C-ABI: errors, contexts, problem setup and host-side introspection.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <memory>
#include <cmath>
#include <cstring>
#include <thread>

#include "internal.hpp"

namespace snsw {

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }

void parallel_for(int64_t n, int nthreads, const std::function<void(int64_t, int64_t)>& fn) {
    if (n <= 0) return;
    int nt = nthreads > 0 ? nthreads : (int)std::max(1u, std::thread::hardware_concurrency());
    nt = (int)std::min<int64_t>(nt, n);
    if (nt <= 1) { fn(0, n); return; }
    std::vector<std::thread> th;
    std::vector<std::exception_ptr> errs(nt);
    // interleaved small chunks balance uneven work (e.g. kink faces)
    const int64_t chunk = std::max<int64_t>(1, n / (nt * 16));
    std::atomic<int64_t> next(0);
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
            try {
                while (true) {
                    const int64_t b = next.fetch_add(chunk);
                    if (b >= n) break;
                    fn(b, std::min(n, b + chunk));
                }
            } catch (...) {
                errs[t] = std::current_exception();
            }
        });
    for (auto& x : th) x.join();
    for (auto& e : errs)
        if (e) std::rethrow_exception(e);
}

}  // namespace snsw

using namespace snsw;

extern "C" {

const char* snsw_last_error(void) { return g_last_error.c_str(); }

const char* snsw_version(void) { return "snsweep 0.1 (gfx950)"; }

int snsw_ctx_create(int device, void* hip_stream, snsw_ctx** out) {
    return snsw_guard([&] {
        if (!out) throw Error(SNSW_E_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (device < -1) throw Error(SNSW_E_INVALID_ARG, "device must be >= -1");
        auto* c = new snsw_ctx();
        c->device = device;
        c->stream = hip_stream;
        if (device >= 0) {
            try {
                device_check_ctx(c);
            } catch (...) {
                delete c;
                throw;
            }
        }
        *out = c;
    });
}

void snsw_ctx_destroy(snsw_ctx* ctx) { delete ctx; }

static void check_finite(const double* a, size_t n, const char* name) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) throw Error(SNSW_E_NONFINITE, std::string("non-finite value in ") + name);
}

// Validates and stores the volume source and the boundary condition (the
// fixed right-hand side is rebuilt separately, once the discretisation
// exists).
static void set_host_source(HostProblem& hp, int q_kind, const double* q, int bc, double psi_inc,
                            const double* psi_tab) {
    if (!q) throw Error(SNSW_E_INVALID_ARG, "source q is NULL");
    if (bc != SNSW_BC_VACUUM && bc != SNSW_BC_ISO_CONST && bc != SNSW_BC_TABULATED)
        throw Error(SNSW_E_INVALID_ARG, "bc_kind");
    if (q_kind != SNSW_Q_PER_ELEMENT && q_kind != SNSW_Q_PER_DOF && q_kind != SNSW_Q_PER_DIRECTION)
        throw Error(SNSW_E_INVALID_ARG, "q_per_dof must be 0, 1 or 2");
    if (bc == SNSW_BC_TABULATED && !psi_tab) throw Error(SNSW_E_INVALID_ARG, "psi_inc_tab is NULL");
    const size_t en = (size_t)hp.E * hp.n, den = (size_t)hp.D * en;
    std::vector<double> qn(en, 0.0), qd, pt;
    if (q_kind == SNSW_Q_PER_DOF) std::copy(q, q + en, qn.begin());
    else if (q_kind == SNSW_Q_PER_ELEMENT)
        for (int64_t e = 0; e < hp.E; ++e)
            for (int i = 0; i < hp.n; ++i) qn[(size_t)e * hp.n + i] = q[e];
    else qd.assign(q, q + den);
    check_finite(qn.data(), qn.size(), "q");
    check_finite(qd.data(), qd.size(), "q");
    if (bc == SNSW_BC_TABULATED) {
        pt.assign(psi_tab, psi_tab + den);
        check_finite(pt.data(), pt.size(), "psi_inc_tab");
    }
    const double pin = bc == SNSW_BC_ISO_CONST ? psi_inc : 0.0;
    if (!std::isfinite(pin)) throw Error(SNSW_E_NONFINITE, "psi_inc");
    hp.bc = bc;
    hp.psi_inc = pin;
    hp.q.swap(qn);
    hp.q_dir.swap(qd);
    hp.psi_tab.swap(pt);
}

int snsw_problem_create(snsw_ctx* ctx, const snsw_problem_desc* desc, snsw_problem** out) {
    return snsw_guard([&] {
        if (!ctx || !desc || !out) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        *out = nullptr;
        const auto t0 = std::chrono::steady_clock::now();
        auto prob = std::make_unique<snsw_problem>();
        prob->ctx = ctx;
        HostProblem& hp = prob->hp;
        hp.dim = desc->dim;
        if (hp.dim != 2 && hp.dim != 3) throw Error(SNSW_E_INVALID_ARG, "dim must be 2 or 3");
        hp.r = desc->geom_order;
        hp.p = desc->dg_order;
        if (hp.r < 1 || hp.r > 3) throw Error(SNSW_E_UNSUPPORTED, "geom_order must be 1..3");
        if (hp.p < 1 || hp.p > 3) throw Error(SNSW_E_UNSUPPORTED, "dg_order must be 1..3");
        hp.E = 1;
        for (int a = 0; a < hp.dim; ++a) {
            hp.nx[a] = desc->nx[a];
            if (hp.nx[a] < 1) throw Error(SNSW_E_SHAPE, "nx must be >= 1");
            hp.E *= hp.nx[a];
        }
        if (hp.E > (int64_t)1 << 30) throw Error(SNSW_E_SHAPE, "too many elements");
        if (desc->element != SNSW_ELEM_TENSOR && desc->element != SNSW_ELEM_SIMPLEX)
            throw Error(SNSW_E_INVALID_ARG, "element must be TENSOR or SIMPLEX");
        hp.simplex = desc->element == SNSW_ELEM_SIMPLEX;
        if (desc->face_rule != SNSW_FACE_EXACT && desc->face_rule != SNSW_FACE_ROMBERG)
            throw Error(SNSW_E_INVALID_ARG, "face_rule must be EXACT or ROMBERG");
        hp.face_rule = desc->face_rule;
        if (!std::isfinite(desc->face_tol)) throw Error(SNSW_E_NONFINITE, "face_tol");
        hp.face_tol = desc->face_tol > 0.0 ? desc->face_tol : 1e-10;
        if (hp.simplex && !desc->elem_nodes)
            throw Error(SNSW_E_INVALID_ARG, "simplicial elements need an element list (elem_nodes)");
        hp.n = 1;
        hp.nf = 1;
        hp.nv = 1;
        for (int a = 0; a < hp.dim; ++a) hp.n *= hp.p + 1;
        for (int a = 0; a + 1 < hp.dim; ++a) hp.nf *= hp.p + 1;
        for (int a = 0; a < hp.dim; ++a) hp.nv *= hp.r + 1;
        if (hp.simplex && hp.dim == 2) {
            hp.n = (hp.p + 1) * (hp.p + 2) / 2;
            hp.nv = (hp.r + 1) * (hp.r + 2) / 2;
        } else if (hp.simplex) {
            hp.n = (hp.p + 1) * (hp.p + 2) * (hp.p + 3) / 6;
            hp.nf = (hp.p + 1) * (hp.p + 2) / 2;
            hp.nv = (hp.r + 1) * (hp.r + 2) * (hp.r + 3) / 6;
        }
        hp.nthreads = desc->n_threads > 0 ? desc->n_threads
                                          : (int)std::max(1u, std::thread::hardware_concurrency());
        hp.weighting = desc->weighting;
        if (hp.weighting < 0 || hp.weighting > 2) throw Error(SNSW_E_INVALID_ARG, "weighting must be 0..2");
        hp.exact_max = desc->exact_scc_max;
        if (hp.exact_max < 1 || hp.exact_max > 20) throw Error(SNSW_E_INVALID_ARG, "exact_scc_max must be 1..20");
        hp.precision = desc->precision;
        if (hp.precision != SNSW_PREC_FP64 && hp.precision != SNSW_PREC_MIXED)
            throw Error(SNSW_E_INVALID_ARG, "precision must be FP64 or MIXED");
        hp.schedule = desc->schedule;
        if (hp.schedule != SNSW_SCHED_AUTO && hp.schedule != SNSW_SCHED_PERSISTENT &&
            hp.schedule != SNSW_SCHED_LEVELS)
            throw Error(SNSW_E_INVALID_ARG, "schedule must be AUTO, PERSISTENT or LEVELS");
        hp.cache_inverse = desc->cache_inverse;
        if (!std::isfinite(desc->cache_budget)) throw Error(SNSW_E_NONFINITE, "cache_budget");
        hp.cache_budget = desc->cache_budget;
        // mixed precision sweeps persistently where a persistent kernel reads
        // the FP32 inverses: 2D lattices, inverses not switched off
        const bool mixed_persistent = hp.dim == 2 && !desc->elem_nodes && hp.cache_inverse != SNSW_CACHE_OFF;
        if (hp.schedule == SNSW_SCHED_AUTO) {
            // 2D sweeps are latency-bound: persistent (FP64: p = 2 only with
            // cached inverses; its assembled persistent kernel is slower than
            // the level schedule)
            const bool ok = desc->precision == SNSW_PREC_MIXED
                                ? mixed_persistent
                                : hp.dim == 2 && (hp.p != 2 || hp.cache_inverse != SNSW_CACHE_OFF);
            hp.schedule = ok ? SNSW_SCHED_PERSISTENT : SNSW_SCHED_LEVELS;
        }
        if (hp.cache_inverse != SNSW_CACHE_AUTO && hp.cache_inverse != SNSW_CACHE_ON &&
            hp.cache_inverse != SNSW_CACHE_OFF)
            throw Error(SNSW_E_INVALID_ARG, "cache_inverse must be AUTO, ON or OFF");
        if (hp.cache_inverse == SNSW_CACHE_ON && desc->precision == SNSW_PREC_MIXED && hp.n > 32)
            throw Error(SNSW_E_UNSUPPORTED, "cached FP32 inverses need elements of at most 32 nodes");

        if (desc->precision == SNSW_PREC_MIXED && hp.schedule == SNSW_SCHED_PERSISTENT && !mixed_persistent)
            throw Error(SNSW_E_UNSUPPORTED,
                        "mixed precision runs on the LEVELS schedule (persistent: 2D lattices with cached "
                        "inverses)");

        // mesh: structured lattice or element control-point lists
        if (desc->elem_nodes) {
            hp.unstructured = true;
            for (int a = 1; a < hp.dim; ++a)
                if (hp.nx[a] != 1) throw Error(SNSW_E_SHAPE, "unstructured mesh: nx[1] (and nx[2]) must be 1");
            if (!desc->nodes || desc->n_nodes < 1) throw Error(SNSW_E_INVALID_ARG, "unstructured mesh: no nodes");
            // element lists: the generic persistent kernels on request, else levels
            hp.schedule = desc->schedule == SNSW_SCHED_PERSISTENT ? SNSW_SCHED_PERSISTENT : SNSW_SCHED_LEVELS;
            const int64_t Nv = hp.nv;
            hp.nodes.assign(desc->nodes, desc->nodes + desc->n_nodes * hp.dim);
            check_finite(hp.nodes.data(), hp.nodes.size(), "nodes");
            hp.elem_nodes.assign(desc->elem_nodes, desc->elem_nodes + hp.E * Nv);
            for (int64_t id : hp.elem_nodes)
                if (id < 0 || id >= desc->n_nodes) throw Error(SNSW_E_INVALID_ARG, "elem_nodes index out of range");
        } else {
            if (!desc->lattice) throw Error(SNSW_E_INVALID_ARG, "lattice is NULL");
            int64_t Lp = 1;
            for (int a = 0; a < hp.dim; ++a) Lp *= (int64_t)hp.r * hp.nx[a] + 1;
            hp.lattice.assign(desc->lattice, desc->lattice + Lp * hp.dim);
            check_finite(hp.lattice.data(), hp.lattice.size(), "lattice");
        }
        // quadrature
        if (desc->sn_order > 0) {
            if (desc->sn_order % 2) throw Error(SNSW_E_INVALID_ARG, "sn_order must be even");
            level_symmetric(desc->sn_order, hp.dim, hp.omega, hp.w);
        } else {
            if (desc->n_dirs < 1 || !desc->omega || !desc->w) throw Error(SNSW_E_INVALID_ARG, "quadrature");
            hp.omega.assign(desc->omega, desc->omega + 3 * desc->n_dirs);
            hp.w.assign(desc->w, desc->w + desc->n_dirs);
            check_finite(hp.omega.data(), hp.omega.size(), "omega");
            check_finite(hp.w.data(), hp.w.size(), "w");
        }
        hp.D = (int)hp.w.size();
        if (hp.D >= (1 << kDirBits)) throw Error(SNSW_E_SHAPE, "too many directions (max 1023)");
        // materials and source
        if (!desc->sigma_t || !desc->sigma_s) throw Error(SNSW_E_INVALID_ARG, "materials NULL");
        hp.sigma_t.assign(desc->sigma_t, desc->sigma_t + hp.E);
        hp.sigma_s.assign(desc->sigma_s, desc->sigma_s + hp.E);
        check_finite(hp.sigma_t.data(), hp.E, "sigma_t");
        check_finite(hp.sigma_s.data(), hp.E, "sigma_s");
        for (int64_t e = 0; e < hp.E; ++e) {
            if (!(hp.sigma_t[e] > 0.0)) throw Error(SNSW_E_INVALID_ARG, "sigma_t must be > 0");
            if (hp.sigma_s[e] < 0.0) throw Error(SNSW_E_INVALID_ARG, "sigma_s must be >= 0");
        }
        set_host_source(hp, desc->q_per_dof, desc->q, desc->bc_kind, desc->psi_inc, desc->psi_inc_tab);

        build_geometry(hp);
        build_faces(hp);
        build_graphs(hp);
        build_schedule(hp);
        build_fixed_rhs(hp);
        // tiles of T x T elements per persistent batch for the DPP shapes
        if (hp.dim == 2 && (hp.n == 16 || hp.n == 4) && !hp.unstructured)
            build_tiled_schedule(hp, hp.n == 16 ? 2 : 4);
        hp.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (ctx->device >= 0) {
            try {
                device_upload(prob.get());
            } catch (...) {
                device_release(prob.get());
                throw;
            }
        }
        *out = prob.release();
    });
}

void snsw_problem_destroy(snsw_problem* prob) {
    if (!prob) return;
    device_release(prob);
    delete prob;
}

int snsw_problem_get_info(const snsw_problem* prob, snsw_problem_info* info) {
    return snsw_guard([&] {
        if (!prob || !info) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        const HostProblem& hp = prob->hp;
        info->n_elements = hp.E;
        info->n_dofs_per_element = hp.n;
        info->n_dirs = hp.D;
        info->n_levels_total = (int64_t)hp.level_off.size() - 1;
        info->n_pairs = hp.E * hp.D;
        info->n_edges_total = 0;
        info->n_removed_total = 0;
        for (auto& g : hp.graphs) {
            info->n_edges_total += g.stats.n_edges;
            info->n_removed_total += g.stats.n_removed;
        }
        info->n_kink_faces_total = hp.n_kinks;
        info->setup_seconds = hp.setup_seconds;
        info->cached_inverse = hp.inverse_cached;
        info->cached_dirs = hp.cached_dirs;
        info->inverse_block_bytes = ainv_block_bytes(hp.dim, hp.p, hp.simplex, hp.precision == SNSW_PREC_MIXED);
        info->tile = hp.tile;
        info->schedule = hp.schedule;
    });
}

int snsw_get_quadrature(const snsw_problem* prob, double* omega, double* w) {
    return snsw_guard([&] {
        if (!prob || !omega || !w) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        std::copy(prob->hp.omega.begin(), prob->hp.omega.end(), omega);
        std::copy(prob->hp.w.begin(), prob->hp.w.end(), w);
    });
}

int snsw_problem_set_source(snsw_problem* prob, int32_t q_per_dof, const double* q, int32_t bc_kind, double psi_inc,
                            const double* psi_inc_tab) {
    return snsw_guard([&] {
        if (!prob) throw Error(SNSW_E_INVALID_ARG, "NULL problem");
        HostProblem& hp = prob->hp;
        set_host_source(hp, q_per_dof, q, bc_kind, psi_inc, psi_inc_tab);
        build_fixed_rhs(hp);
        if (prob->dev) device_update_source(prob);
    });
}

int snsw_get_node_coordinates(const snsw_problem* prob, int64_t e0, int64_t count, double* xyz) {
    return snsw_guard([&] {
        if (!prob || !xyz) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        if (e0 < 0 || count < 0 || e0 + count > prob->hp.E) throw Error(SNSW_E_SHAPE, "element range");
        node_coordinates(prob->hp, e0, count, xyz);
    });
}

int snsw_get_volume_rule(const snsw_problem* prob, int32_t extra, int64_t e0, int64_t count, int32_t* n_points,
                         double* x, double* wdet, double* basis) {
    return snsw_guard([&] {
        if (!prob || !n_points) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        if (extra < 0 || extra > 8) throw Error(SNSW_E_INVALID_ARG, "extra must be 0..8");
        if (e0 < 0 || count < 0 || e0 + count > prob->hp.E) throw Error(SNSW_E_SHAPE, "element range");
        if (x && !wdet) throw Error(SNSW_E_INVALID_ARG, "wdet is NULL");
        *n_points = volume_rule(prob->hp, extra, e0, count, x, wdet, basis);
    });
}

int snsw_get_element_matrices(const snsw_problem* prob, int64_t e0, int64_t count, double* M, double* K) {
    return snsw_guard([&] {
        if (!prob) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        const HostProblem& hp = prob->hp;
        if (e0 < 0 || count < 0 || e0 + count > hp.E) throw Error(SNSW_E_SHAPE, "element range");
        const size_t nn = (size_t)hp.n * hp.n;
        if (M) std::copy(hp.M.begin() + e0 * nn, hp.M.begin() + (e0 + count) * nn, M);
        if (K) std::copy(hp.K.begin() + e0 * nn * hp.dim, hp.K.begin() + (e0 + count) * nn * hp.dim, K);
    });
}

static const DirGraph& graph_of(const snsw_problem* prob, int d) {
    if (!prob) throw Error(SNSW_E_INVALID_ARG, "NULL problem");
    if (d < 0 || d >= prob->hp.D) throw Error(SNSW_E_INVALID_ARG, "direction out of range");
    return prob->hp.graphs[d];
}

int snsw_graph_stats_get(const snsw_problem* prob, int d, snsw_graph_stats* st) {
    return snsw_guard([&] {
        const DirGraph& g = graph_of(prob, d);
        if (!st) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        *st = g.stats;
    });
}

int snsw_get_edges(const snsw_problem* prob, int d, int32_t* up, int32_t* down, int64_t* weight,
                   int64_t cap, int64_t* count) {
    return snsw_guard([&] {
        const DirGraph& g = graph_of(prob, d);
        const int64_t m = (int64_t)g.up.size();
        if (count) *count = m;
        const int64_t k = std::min(cap, m);
        for (int64_t i = 0; i < k; ++i) {
            if (up) up[i] = g.up[i];
            if (down) down[i] = g.down[i];
            if (weight) weight[i] = g.weight[i];
        }
    });
}

int snsw_get_removed_edges(const snsw_problem* prob, int d, int32_t* down, int32_t* up, int64_t cap,
                           int64_t* count) {
    return snsw_guard([&] {
        const DirGraph& g = graph_of(prob, d);
        const int64_t m = (int64_t)g.rem_down.size();
        if (count) *count = m;
        const int64_t k = std::min(cap, m);
        for (int64_t i = 0; i < k; ++i) {
            if (down) down[i] = g.rem_down[i];
            if (up) up[i] = g.rem_up[i];
        }
    });
}

int snsw_get_face_integrals(const snsw_problem* prob, int d, int64_t f, int32_t* cls, double* mp, double* mm,
                            double* Pp, double* Pm) {
    return snsw_guard([&] {
        if (!prob) throw Error(SNSW_E_INVALID_ARG, "NULL problem");
        const HostProblem& hp = prob->hp;
        if (d < 0 || d >= hp.D) throw Error(SNSW_E_INVALID_ARG, "direction out of range");
        if (f < 0 || f >= hp.F) throw Error(SNSW_E_INVALID_ARG, "face out of range");
        const int nf = hp.nf;
        std::vector<double> pp((size_t)nf * nf, 0.0), pm((size_t)nf * nf, 0.0);
        double a = 0.0, b = 0.0;
        const uint8_t c = face_integrals(hp, f, &hp.omega[(size_t)d * 3], a, b, pp.data(), pm.data());
        if (c != FC_KINK) {
            std::fill(pp.begin(), pp.end(), 0.0);
            std::fill(pm.begin(), pm.end(), 0.0);
        }
        if (cls) *cls = c;
        if (mp) *mp = a;
        if (mm) *mm = b;
        if (Pp) std::copy(pp.begin(), pp.end(), Pp);
        if (Pm) std::copy(pm.begin(), pm.end(), Pm);
    });
}

int snsw_get_levels(const snsw_problem* prob, int d, int32_t* level) {
    return snsw_guard([&] {
        const DirGraph& g = graph_of(prob, d);
        if (!level) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        std::copy(g.level.begin(), g.level.end(), level);
    });
}

}  // extern "C"
