// Batches of independent problems: merged per-class schedules, autotuned
// schedule choice, one captured hipGraph per set of flux pointers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <set>
#include <tuple>

#include "device.hpp"

namespace snsw {

struct BatchGraph {
    std::vector<const double*> in;
    std::vector<double*> out;
    const double** d_in = nullptr;    // device copies of the pointer lists
    double** d_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};

struct BatchClass {
    SweepClass cls;
    bool has_inv = false;              // every member keeps cached inverses
    bool levels_only = false;          // unstructured meshes, mixed precision without a persistent FP32 kernel
    int4* d_pairs = nullptr;           // level schedule
    std::vector<int64_t> level_off;
    bool tiled = false;                // every member has a tiled schedule
    int4* d_tpairs = nullptr;          // tiled schedule (persistent kernels)
    int32_t* d_tintra = nullptr;
    std::vector<int64_t> tlevel_off;
    int full_blocks = 0;
    double tuned_ms[4] = {0.0, 0.0, 0.0, 0.0};
};

}  // namespace snsw

struct snsw_batch {
    snsw_ctx* ctx = nullptr;
    std::vector<snsw_problem*> probs;
    std::vector<int> entry_cur;            // buffer index in each entry's psi_cur
    std::vector<int> entry_class;
    snsw::SweepArgs* table = nullptr;
    std::vector<snsw::BatchClass> classes;
    unsigned int* tickets = nullptr;
    int32_t* error = nullptr;
    int64_t max_En = 0, max_DEn = 0;
    bool use_graph = true;
    hipStream_t capture = nullptr;         // private stream for graph capture
    std::vector<snsw::BatchGraph> graphs;
    uint64_t clock = 0;
};

namespace snsw {

namespace {

constexpr size_t kMaxGraphs = 4;

void release_graph(BatchGraph& g) noexcept {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    if (g.d_in) (void)hipFree(g.d_in);
    if (g.d_out) (void)hipFree(g.d_out);
    g = BatchGraph();
}

void release_batch(snsw_batch* b) noexcept {
    if (!b) return;
    hipStream_t s = static_cast<hipStream_t>(b->ctx->stream);
    (void)hipStreamSynchronize(s);
    for (BatchGraph& g : b->graphs) release_graph(g);
    for (BatchClass& c : b->classes) {
        if (c.d_pairs) (void)hipFree(c.d_pairs);
        if (c.d_tpairs) (void)hipFree(c.d_tpairs);
        if (c.d_tintra) (void)hipFree(c.d_tintra);
    }
    if (b->table) (void)hipFree(b->table);
    if (b->tickets) (void)hipFree(b->tickets);
    if (b->error) (void)hipFree(b->error);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    delete b;
}

std::vector<SweepClass> active_classes(const snsw_batch* b) {
    std::vector<SweepClass> out;
    for (const BatchClass& c : b->classes) out.push_back(c.cls);
    return out;
}

SweepLaunch base_launch(const snsw_batch* b) {
    SweepLaunch L;
    L.table = b->table;
    L.count = (int)b->probs.size();
    L.max_En = b->max_En;
    L.max_DEn = b->max_DEn;
    L.any_persistent = false;
    for (const BatchClass& c : b->classes) L.any_persistent |= c.cls.persistent;
    L.tickets = b->tickets;
    L.n_tickets = (int)b->classes.size();
    L.error = b->error;
    return L;
}

// Uploads the whole table from the host mirror (synchronous).  `all_fill`
// marks every entry persistent (sentinel fill for all, used while tuning).
void upload_table(snsw_batch* b, bool all_fill) {
    hipStream_t s = static_cast<hipStream_t>(b->ctx->stream);
    std::vector<SweepArgs> host(b->probs.size());
    for (size_t k = 0; k < b->probs.size(); ++k) {
        host[k] = make_args(b->probs[k], b->entry_cur[k]);
        host[k].persistent = (all_fill || b->classes[b->entry_class[k]].cls.persistent) ? 1 : 0;
    }
    HIP_OK(hipMemcpyAsync(b->table, host.data(), host.size() * sizeof(SweepArgs), hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
}

void sync_entries(snsw_batch* b, hipStream_t s) {
    for (size_t k = 0; k < b->probs.size(); ++k) sync_entry(b->table, (int)k, b->probs[k], &b->entry_cur[k], s);
}

// Every problem has swept once: flip the host mirrors.
void advance_mirrors(snsw_batch* b) {
    for (size_t k = 0; k < b->probs.size(); ++k) {
        DeviceProblem* dp = b->probs[k]->dev;
        dp->cur = 1 - dp->cur;
        b->entry_cur[k] = dp->cur;
    }
}

void reset_members(snsw_batch* b) {
    hipStream_t s = static_cast<hipStream_t>(b->ctx->stream);
    for (snsw_problem* p : b->probs) {
        const HostProblem& hp = p->hp;
        for (int k = 0; k < 2; ++k)
            HIP_OK(hipMemsetAsync(p->dev->psi[k], 0, sizeof(double) * hp.D * hp.E * hp.n, s));
    }
    HIP_OK(hipStreamSynchronize(s));
}

// Merged schedule of one class: level k lists, problem by problem, every
// member's level-k segment (each a multiple of G entries); the problem field
// of each entry is its table index.  `tiled` merges the members' tiled
// schedules instead (levels of tiles; intra-tile dependency words kept).
// Checks that every kept upwind pair lies in an earlier batch of G entries
// than its dependant, or in the same tile when the intra word says so.
void build_class_schedule(const std::vector<snsw_problem*>& probs, const std::vector<int>& members, bool tiled,
                          std::vector<int64_t>& level_off, std::vector<int32_t>& pairs, std::vector<int32_t>& intra) {
    auto lo_of = [&](const HostProblem& hp) -> const std::vector<int64_t>& { return tiled ? hp.tlevel_off : hp.level_off; };
    auto pr_of = [&](const HostProblem& hp) -> const std::vector<int32_t>& { return tiled ? hp.tpairs : hp.pairs; };
    int64_t L = 0;
    for (int k : members) L = std::max<int64_t>(L, (int64_t)lo_of(probs[k]->hp).size() - 1);
    const int n = probs[members[0]]->hp.n;
    const int64_t G = std::max(1, 64 / n);
    level_off.assign(L + 1, 0);
    for (int64_t l = 0; l < L; ++l) {
        int64_t cnt = 0;
        for (int k : members) {
            const auto& lo = lo_of(probs[k]->hp);
            if (l + 1 < (int64_t)lo.size()) cnt += lo[l + 1] - lo[l];
        }
        level_off[l + 1] = level_off[l] + cnt;
    }
    const int64_t total = level_off[L];
    pairs.assign((size_t)total * 4, 0);
    intra.assign(tiled ? (size_t)total : 0, 0);
    std::vector<std::vector<int64_t>> where(members.size());
    for (size_t m = 0; m < members.size(); ++m) {
        const HostProblem& hp = probs[members[m]]->hp;
        where[m].assign((size_t)hp.D * hp.E, -1);
    }
    for (int64_t l = 0; l < L; ++l) {
        int64_t pos = level_off[l];
        for (size_t m = 0; m < members.size(); ++m) {
            const int k = members[m];
            const HostProblem& hp = probs[k]->hp;
            const auto& lo = lo_of(hp);
            const auto& hpairs = pr_of(hp);
            if (l + 1 >= (int64_t)lo.size()) continue;
            if ((pos % G) != 0 || ((lo[l + 1] - lo[l]) % G) != 0)
                throw Error(SNSW_E_STATE, "batch schedule: level segment not a multiple of G");
            for (int64_t t = lo[l]; t < lo[l + 1]; ++t, ++pos) {
                const int32_t* src = &hpairs[(size_t)t * 4];
                int32_t* dst = &pairs[(size_t)pos * 4];
                dst[0] = src[0];
                dst[1] = src[1];
                dst[2] = src[2];
                dst[3] = k;
                if (tiled) intra[(size_t)pos] = hp.tintra[(size_t)t];
                if (src[0] >= 0)
                    where[m][(size_t)((uint32_t)src[1] & ((1u << kDirBits) - 1)) * hp.E + src[0]] = pos;
            }
        }
    }
    for (size_t m = 0; m < members.size(); ++m) {
        const HostProblem& hp = probs[members[m]]->hp;
        const int ns = hp.nslot;
        for (size_t i = 0; i < where[m].size(); ++i)
            if (where[m][i] < 0) throw Error(SNSW_E_STATE, "batch schedule: a pair is missing");
        for (int64_t d = 0; d < hp.D; ++d)
            for (int64_t e = 0; e < hp.E; ++e) {
                const int64_t t = where[m][(size_t)d * hp.E + e];
                const uint32_t packed = (uint32_t)pairs[(size_t)t * 4 + 1];
                const uint32_t iw = tiled ? (uint32_t)intra[(size_t)t] : 0u;
                for (int s = 0; s < ns; ++s) {
                    const uint32_t bits = packed >> (kDirBits + 3 * s);
                    const uint32_t cls = bits & 3u;
                    const bool lagged = (bits >> 2) & 1u;
                    const int32_t nb = hp.slot_nbr[(size_t)e * ns + s];
                    if (!((cls == SC_IN || cls == SC_KINK) && !lagged && nb >= 0)) continue;
                    const int64_t tu = where[m][(size_t)d * hp.E + nb];
                    if ((iw >> s) & 1u) {
                        const int64_t g_up = (iw >> (kIntraGroupShift + 4 * s)) & 15u;
                        if (tu != t - t % G + g_up)
                            throw Error(SNSW_E_STATE, "batch schedule: an intra-tile dependency is misplaced");
                    } else if (tu >= t - t % G) {
                        throw Error(SNSW_E_STATE, "batch schedule: a kept upwind pair does not precede its dependant");
                    }
                }
            }
    }
}

// Active schedule of a class for a schedule choice (tiles: use the tiled
// schedule when the class has one).
void choose(BatchClass& bc, bool persistent, int blocks, bool tiles = true) {
    SweepClass& c = bc.cls;
    c.persistent = persistent;
    c.blocks = persistent ? blocks : 0;
    c.inv = bc.has_inv && (!persistent || persistent_uses_inverse(c.dim, c.p));
    tiles = tiles && persistent && bc.tiled;
    c.pairs = tiles ? bc.d_tpairs : bc.d_pairs;
    c.level_off = tiles ? bc.tlevel_off : bc.level_off;
    c.intra = tiles ? bc.d_tintra : nullptr;
}

// Times `reps` sweeps of one class with the given schedule (ms per sweep,
// class kernels only).
double time_class(snsw_batch* b, size_t ci, bool persistent, int blocks, bool tiles, int reps, double* phi_in,
                  double* phi_out) {
    hipStream_t s = static_cast<hipStream_t>(b->ctx->stream);
    BatchClass tmp = b->classes[ci];
    choose(tmp, persistent, blocks, tiles);
    const SweepClass c = tmp.cls;
    SweepLaunch L = base_launch(b);
    L.any_persistent = true;
    L.phi_in_one = phi_in;
    L.phi_out_one = phi_out;
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    double best = 1e300;
    for (int r = 0; r <= reps; ++r) {   // the first sweep warms up
        launch_source(L.table, L.count, L.max_En, nullptr, phi_in, L.tickets, L.n_tickets, s);
        launch_fill_sentinel(L.table, L.count, L.max_DEn, s);
        HIP_OK(hipEventRecord(e0, s));
        enqueue_sweep_class(L, c, s);
        HIP_OK(hipEventRecord(e1, s));
        HIP_OK(hipStreamSynchronize(s));
        advance_mirrors(b);
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, e0, e1));
        if (r > 0) best = std::min(best, (double)ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    check_error_flag(b->error, s);
    return best;
}

BatchGraph& graph_for(snsw_batch* b, const double* const* in, double* const* out) {
    const size_t n = b->probs.size();
    for (BatchGraph& g : b->graphs)
        if (std::equal(g.in.begin(), g.in.end(), in) && std::equal(g.out.begin(), g.out.end(), out)) {
            g.last_use = ++b->clock;
            return g;
        }
    hipStream_t s = static_cast<hipStream_t>(b->ctx->stream);
    if (b->graphs.size() >= kMaxGraphs) {
        auto it = std::min_element(b->graphs.begin(), b->graphs.end(),
                                   [](const BatchGraph& x, const BatchGraph& y) { return x.last_use < y.last_use; });
        HIP_OK(hipStreamSynchronize(s));   // a replay in flight may still read its pointer lists
        release_graph(*it);
        b->graphs.erase(it);
    }
    BatchGraph g;
    g.in.assign(in, in + n);
    g.out.assign(out, out + n);
    try {
        HIP_OK(hipMalloc(&g.d_in, n * sizeof(double*)));
        HIP_OK(hipMalloc(&g.d_out, n * sizeof(double*)));
        HIP_OK(hipMemcpy(g.d_in, g.in.data(), n * sizeof(double*), hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(g.d_out, g.out.data(), n * sizeof(double*), hipMemcpyHostToDevice));
        SweepLaunch L = base_launch(b);
        L.phi_in_list = g.d_in;
        L.phi_out_list = g.d_out;
        HIP_OK(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
        try {
            enqueue_sweep(L, active_classes(b), b->capture, nullptr);
        } catch (...) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(b->capture, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            throw;
        }
        HIP_OK(hipStreamEndCapture(b->capture, &g.graph));
        HIP_OK(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
    } catch (...) {
        release_graph(g);
        throw;
    }
    g.last_use = ++b->clock;
    b->graphs.push_back(g);
    return b->graphs.back();
}

}  // namespace

void enqueue_sweep_class(const SweepLaunch& L, const SweepClass& c, hipStream_t s) {
    if (c.persistent) {
        PersistArgs pa{};
        pa.table = L.table;
        pa.pairs = c.pairs;
        pa.ticket = L.tickets + (size_t)c.ticket * kTicketWords;
        pa.error = L.error;
        pa.total = c.level_off.back();
        pa.spin_limit = L.spin_limit;
        pa.intra = c.intra;
        pa.problem = class_problem(c);
        pa.slots = c.slots;
        pa.nt = 0;
        if (!launch_sweep_persistent(c.dim, c.p, c.simplex, c.unstructured, c.inv, pa, c.blocks, s, c.mixed && c.inv))
            throw Error(SNSW_E_STATE, "batch class without a persistent kernel");
    } else {
        for (size_t k = 0; k + 1 < c.level_off.size(); ++k) {
            const int64_t b = c.level_off[k], n = c.level_off[k + 1] - b;
            launch_sweep_level(c.dim, c.p, c.simplex, c.mixed, c.inv, c.unstructured, L.table, c.pairs, b, n,
                                   class_problem(c), s, c.face_points);
        }
    }
    HIP_OK(hipGetLastError());
}

}  // namespace snsw

using namespace snsw;

extern "C" {

int snsw_batch_create(snsw_ctx* ctx, snsw_problem* const* probs, int32_t count, const snsw_batch_opts* opts,
                      snsw_batch** out) {
    snsw_batch* b = nullptr;
    const int rc = snsw_guard([&] {
        if (!ctx || !probs || !out) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        *out = nullptr;
        if (count < 1) throw Error(SNSW_E_INVALID_ARG, "a batch needs at least one problem");
        if (ctx->device < 0) throw Error(SNSW_E_UNSUPPORTED, "host-only context: no device work");
        snsw_batch_opts o{};
        if (opts) o = *opts;
        if (o.schedule != SNSW_SCHED_AUTO && o.schedule != SNSW_SCHED_PERSISTENT && o.schedule != SNSW_SCHED_LEVELS)
            throw Error(SNSW_E_INVALID_ARG, "schedule must be AUTO, PERSISTENT or LEVELS");
        if (o.tune_reps < 0) throw Error(SNSW_E_INVALID_ARG, "tune_reps must be >= 0");
        const int reps = o.tune_reps > 0 ? o.tune_reps : 3;
        std::set<const snsw_problem*> seen;
        for (int32_t k = 0; k < count; ++k) {
            if (!probs[k]) throw Error(SNSW_E_INVALID_ARG, "NULL problem in batch");
            if (probs[k]->ctx != ctx || !probs[k]->dev)
                throw Error(SNSW_E_INVALID_ARG, "every problem must be device-backed and belong to this context");
            if (!seen.insert(probs[k]).second) throw Error(SNSW_E_INVALID_ARG, "a problem appears twice in the batch");
        }
        DeviceGuard guard(ctx->device);
        hipStream_t s = static_cast<hipStream_t>(ctx->stream);
        b = new snsw_batch();
        b->ctx = ctx;
        b->probs.assign(probs, probs + count);
        b->use_graph = o.use_graph != 0;
        // classes by (dim, p, precision, cached inverse), in order of first appearance
        std::map<std::tuple<int, int, int, int, int>, int> key;
        b->entry_class.resize(count);
        for (int32_t k = 0; k < count; ++k) {
            const HostProblem& hp = probs[k]->hp;
            // members with a partial inverse cache sweep assembled here
            const int has_inv =
                (probs[k]->dev->ainv != nullptr || probs[k]->dev->ainv32 != nullptr) && hp.cached_dirs == hp.D ? 1 : 0;
            const auto kk = std::make_tuple(hp.dim, hp.p, hp.precision, has_inv, (hp.unstructured ? 1 : 0) + (hp.simplex ? 2 : 0));
            auto it = key.find(kk);
            if (it == key.end()) {
                it = key.emplace(kk, (int)b->classes.size()).first;
                BatchClass bc;
                bc.cls.dim = hp.dim;
                bc.cls.p = hp.p;
                bc.cls.mixed = hp.precision == SNSW_PREC_MIXED;
                // unstructured meshes sweep level by level, and so does mixed
                // precision except on 2D lattices with FP32 inverses
                bc.levels_only = hp.unstructured ||
                                 (bc.cls.mixed && !(has_inv && persistent_f32(hp.dim, hp.p, hp.simplex, hp.unstructured)));
                bc.cls.unstructured = hp.unstructured;
                bc.cls.simplex = hp.simplex;
                bc.cls.face_points = true;
                bc.has_inv = has_inv != 0;
                bc.cls.ticket = (int)b->classes.size();
                b->classes.push_back(bc);
            }
            b->entry_class[k] = it->second;
            b->classes[it->second].cls.members.push_back(k);
            b->classes[it->second].cls.face_points &= probs[k]->dev->Nq != nullptr;
            b->max_En = std::max<int64_t>(b->max_En, hp.E * hp.n);
            b->max_DEn = std::max<int64_t>(b->max_DEn, hp.D * hp.E * hp.n);
        }
        for (BatchClass& bc : b->classes) {
            std::vector<int32_t> pairs, intra;
            build_class_schedule(b->probs, bc.cls.members, false, bc.level_off, pairs, intra);
            HIP_OK(hipMalloc(&bc.d_pairs, std::max<size_t>(1, pairs.size()) * sizeof(int32_t)));
            HIP_OK(hipMemcpyAsync(bc.d_pairs, pairs.data(), pairs.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
            bc.tiled = !bc.levels_only;
            for (int k : bc.cls.members) bc.tiled = bc.tiled && b->probs[k]->hp.tile > 0;
            if (bc.tiled) {
                build_class_schedule(b->probs, bc.cls.members, true, bc.tlevel_off, pairs, intra);
                HIP_OK(hipMalloc(&bc.d_tpairs, std::max<size_t>(1, pairs.size()) * sizeof(int32_t)));
                HIP_OK(hipMemcpyAsync(bc.d_tpairs, pairs.data(), pairs.size() * sizeof(int32_t),
                                      hipMemcpyHostToDevice, s));
                HIP_OK(hipMalloc(&bc.d_tintra, std::max<size_t>(1, intra.size()) * sizeof(int32_t)));
                HIP_OK(hipMemcpyAsync(bc.d_tintra, intra.data(), intra.size() * sizeof(int32_t),
                                      hipMemcpyHostToDevice, s));
            }
            HIP_OK(hipStreamSynchronize(s));
            const bool pinv = bc.has_inv && persistent_uses_inverse(bc.cls.dim, bc.cls.p);
            const int64_t ptotal = bc.tiled ? bc.tlevel_off.back() : bc.level_off.back();
            bc.full_blocks = persistent_grid(bc.cls.dim, bc.cls.p, bc.cls.simplex, bc.cls.unstructured, pinv, ptotal,
                                             ctx->device, 1.0, bc.cls.mixed && pinv);
            choose(bc, !bc.levels_only && o.schedule == SNSW_SCHED_PERSISTENT, bc.full_blocks);
        }
        HIP_OK(hipMalloc(&b->table, count * sizeof(SweepArgs)));
        HIP_OK(hipMalloc(&b->tickets, b->classes.size() * kTicketWords * sizeof(unsigned int)));
        HIP_OK(hipMemsetAsync(b->tickets, 0, b->classes.size() * kTicketWords * sizeof(unsigned int), s));
        HIP_OK(hipMalloc(&b->error, sizeof(int32_t)));
        HIP_OK(hipMemsetAsync(b->error, 0, sizeof(int32_t), s));
        HIP_OK(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
        b->entry_cur.resize(count);
        for (int32_t k = 0; k < count; ++k) b->entry_cur[k] = probs[k]->dev->cur;

        if (o.schedule == SNSW_SCHED_AUTO) {
            // autotuner: levels vs persistent (full and half grid) per class
            upload_table(b, true);
            double* phi_in = nullptr;
            double* phi_out = nullptr;
            HIP_OK(hipMalloc(&phi_in, b->max_En * sizeof(double)));
            HIP_OK(hipMalloc(&phi_out, b->max_En * sizeof(double)));
            try {
                HIP_OK(hipMemsetAsync(phi_in, 0, b->max_En * sizeof(double), s));
                for (size_t ci = 0; ci < b->classes.size(); ++ci) {
                    BatchClass& bc = b->classes[ci];
                    if (bc.levels_only) continue;
                    const int half = std::max(1, bc.full_blocks / 2);
                    bc.tuned_ms[0] = time_class(b, ci, false, 0, true, reps, phi_in, phi_out);
                    bc.tuned_ms[1] = time_class(b, ci, true, bc.full_blocks, true, reps, phi_in, phi_out);
                    bc.tuned_ms[2] = time_class(b, ci, true, half, true, reps, phi_in, phi_out);
                    const int cands = bc.tiled ? 4 : 3;
                    if (bc.tiled) bc.tuned_ms[3] = time_class(b, ci, true, bc.full_blocks, false, reps, phi_in, phi_out);
                    const int best = (int)(std::min_element(bc.tuned_ms, bc.tuned_ms + cands) - bc.tuned_ms);
                    choose(bc, best != 0, best == 2 ? half : bc.full_blocks, best != 3);
                }
            } catch (...) {
                (void)hipFree(phi_in);
                (void)hipFree(phi_out);
                throw;
            }
            HIP_OK(hipFree(phi_in));
            HIP_OK(hipFree(phi_out));
            reset_members(b);
        }
        upload_table(b, false);
        *out = b;
    });
    if (rc != SNSW_OK && b) release_batch(b);
    return rc;
}

void snsw_batch_destroy(snsw_batch* batch) {
    if (!batch) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(batch->ctx->device);
    release_batch(batch);
    if (prev >= 0) (void)hipSetDevice(prev);
}

int snsw_batch_sweep(snsw_batch* b, const double* const* d_phi_in, double* const* d_phi_out) {
    return snsw_guard([&] {
        if (!b || !d_phi_in || !d_phi_out) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        const size_t n = b->probs.size();
        for (size_t k = 0; k < n; ++k) {
            if (!d_phi_in[k] || !d_phi_out[k]) throw Error(SNSW_E_INVALID_ARG, "NULL flux pointer");
            if (d_phi_in[k] == d_phi_out[k]) throw Error(SNSW_E_INVALID_ARG, "phi_in and phi_out alias");
        }
        DeviceGuard guard(b->ctx->device);
        hipStream_t s = static_cast<hipStream_t>(b->ctx->stream);
        sync_entries(b, s);
        if (b->use_graph) {
            BatchGraph& g = graph_for(b, d_phi_in, d_phi_out);
            HIP_OK(hipGraphLaunch(g.exec, s));
        } else {
            // pointer lists for the eager path live in the graph cache too:
            // reuse a cached copy when one exists, else upload a new one
            BatchGraph* hit = nullptr;
            for (BatchGraph& g : b->graphs)
                if (std::equal(g.in.begin(), g.in.end(), d_phi_in) && std::equal(g.out.begin(), g.out.end(), d_phi_out))
                    hit = &g;
            if (!hit) {
                if (b->graphs.size() >= kMaxGraphs) {
                    HIP_OK(hipStreamSynchronize(s));
                    release_graph(b->graphs.front());
                    b->graphs.erase(b->graphs.begin());
                }
                BatchGraph g;
                g.in.assign(d_phi_in, d_phi_in + n);
                g.out.assign(d_phi_out, d_phi_out + n);
                try {
                    HIP_OK(hipMalloc(&g.d_in, n * sizeof(double*)));
                    HIP_OK(hipMalloc(&g.d_out, n * sizeof(double*)));
                    HIP_OK(hipMemcpy(g.d_in, g.in.data(), n * sizeof(double*), hipMemcpyHostToDevice));
                    HIP_OK(hipMemcpy(g.d_out, g.out.data(), n * sizeof(double*), hipMemcpyHostToDevice));
                } catch (...) {
                    release_graph(g);
                    throw;
                }
                b->graphs.push_back(g);
                hit = &b->graphs.back();
            }
            SweepLaunch L = base_launch(b);
            L.phi_in_list = hit->d_in;
            L.phi_out_list = hit->d_out;
            enqueue_sweep(L, active_classes(b), s, nullptr);
        }
        advance_mirrors(b);
    });
}

int snsw_batch_synchronize(snsw_batch* b) {
    return snsw_guard([&] {
        if (!b) throw Error(SNSW_E_INVALID_ARG, "NULL batch");
        DeviceGuard guard(b->ctx->device);
        check_error_flag(b->error, static_cast<hipStream_t>(b->ctx->stream));
    });
}

int snsw_batch_n_classes(const snsw_batch* b, int32_t* n) {
    return snsw_guard([&] {
        if (!b || !n) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        *n = (int32_t)b->classes.size();
    });
}

int snsw_batch_class_get(const snsw_batch* b, int32_t c, snsw_batch_class_info* info) {
    return snsw_guard([&] {
        if (!b || !info) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        if (c < 0 || c >= (int32_t)b->classes.size()) throw Error(SNSW_E_INVALID_ARG, "class index out of range");
        const BatchClass& bc = b->classes[c];
        info->dim = bc.cls.dim;
        info->dg_order = bc.cls.p;
        info->precision = bc.cls.mixed ? SNSW_PREC_MIXED : SNSW_PREC_FP64;
        info->persistent = bc.cls.persistent ? 1 : 0;
        info->blocks = bc.cls.persistent ? bc.cls.blocks : 0;
        info->n_problems = (int32_t)bc.cls.members.size();
        info->n_levels = (int64_t)bc.cls.level_off.size() - 1;
        info->n_entries = bc.cls.level_off.back();
        for (int i = 0; i < 4; ++i) info->tuned_ms[i] = bc.tuned_ms[i];
        info->tiled = (bc.cls.persistent && bc.cls.intra) ? 1 : 0;
    });
}

}  // extern "C"
