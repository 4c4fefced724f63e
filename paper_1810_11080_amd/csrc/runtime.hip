// Device side of a problem: uploads, one sweep, source iteration, state.
#include <hip/hip_runtime.h>

#include <cstddef>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstdint>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <string>

#include "device.hpp"
#include "net.hpp"

namespace snsw {

namespace {

template <class T>
T* dalloc(DeviceProblem* dp, size_t count) {
    if (count == 0) count = 1;
    void* p = nullptr;
    HIP_OK(hipMalloc(&p, count * sizeof(T)));
    dp->bytes += count * sizeof(T);
    return static_cast<T*>(p);
}

template <class T>
T* dupload(DeviceProblem* dp, const std::vector<T>& v, hipStream_t s) {
    T* p = dalloc<T>(dp, v.size());
    if (!v.empty()) HIP_OK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return p;
}

__global__ void set_entry_kernel(SweepArgs* table, int k, double* cur, double* prev) {
    table[k].psi_cur = cur;
    table[k].psi_prev = prev;
}

void do_sweep(snsw_problem* prob, const double* phi_in, double* phi_out, double* psi_out) {
    DeviceProblem* dp = need_device(prob);
    const HostProblem& hp = prob->hp;
    const hipStream_t s = dp->stream;
    sync_entry(dp->table, 0, prob, &dp->table_cur, s);
    SweepLaunch L;
    L.table = dp->table;
    L.count = 1;
    L.max_En = hp.E * hp.n;
    L.max_DEn = hp.D * hp.E * hp.n;
    L.any_persistent = dp->cls.persistent;
    L.spin_limit = dp->spin_limit;
    L.tickets = dp->ticket;
    L.n_tickets = 1;
    L.error = dp->error;
    L.phi_in_one = phi_in;
    L.phi_out_one = phi_out;
    enqueue_sweep(L, std::vector<SweepClass>{dp->cls}, s, &dp->prof);
    dp->cur = 1 - dp->cur;
    dp->table_cur = dp->cur;
    if (psi_out)
        HIP_OK(hipMemcpyAsync(psi_out, dp->psi[dp->cur], sizeof(double) * hp.D * hp.E * hp.n,
                              hipMemcpyDeviceToDevice, s));
}

double do_residual(DeviceProblem* dp, int64_t len, const double* a, const double* b) {
    HIP_OK(hipMemsetAsync(dp->red, 0, 2 * sizeof(unsigned long long), dp->stream));
    launch_residual(len, a, b, dp->red, dp->stream);
    HIP_OK(hipGetLastError());
    unsigned long long h[2] = {0, 0};
    HIP_OK(hipMemcpyAsync(h, dp->red, sizeof(h), hipMemcpyDeviceToHost, dp->stream));
    HIP_OK(hipStreamSynchronize(dp->stream));
    check_error_flag(dp->error, dp->stream);
    double num, den;
    std::memcpy(&num, &h[0], 8);
    std::memcpy(&den, &h[1], 8);
    if (!(den > 0.0)) return num > 0.0 || num != num ? INFINITY : 0.0;
    return num / den;
}

}  // namespace

DeviceProblem* need_device(snsw_problem* prob) {
    if (!prob) throw Error(SNSW_E_INVALID_ARG, "NULL problem");
    if (!prob->dev) throw Error(SNSW_E_UNSUPPORTED, "host-only context: no device work");
    return prob->dev;
}

void LaunchProfiler::begin(hipStream_t s) {
    if (!on) return;
    while (used + 2 > events.size()) {
        hipEvent_t ev;
        HIP_OK(hipEventCreate(&ev));
        events.push_back(ev);
    }
    HIP_OK(hipEventRecord(events[used++], s));
}

void LaunchProfiler::end(hipStream_t s) {
    if (!on) return;
    HIP_OK(hipEventRecord(events[used++], s));
}

void LaunchProfiler::read(int64_t* launches, double* ms) {
    double total = 0.0;
    for (size_t i = 0; i + 1 < used; i += 2) {
        float t = 0.0f;
        HIP_OK(hipEventElapsedTime(&t, events[i], events[i + 1]));
        total += t;
    }
    if (launches) *launches = (int64_t)(used / 2);
    if (ms) *ms = total;
    used = 0;
}

void LaunchProfiler::release() noexcept {
    for (hipEvent_t ev : events) (void)hipEventDestroy(ev);
    events.clear();
    used = 0;
}

SweepArgs make_args(const snsw_problem* prob, int cur) {
    const DeviceProblem* dp = prob->dev;
    const HostProblem& hp = prob->hp;
    SweepArgs a{};
    a.geo = dp->geo;
    a.B = dp->B;
    a.kink_tab = dp->kink_tab;
    a.kink_idx = dp->kink_idx;
    a.slot_face = dp->slot_face;
    a.slot_nbr = dp->slot_nbr;
    a.sigma_t = dp->sigma_t;
    a.sigma_s = dp->sigma_s;
    a.q = dp->q;
    a.omega = dp->omega;
    a.w = dp->w;
    a.src = dp->src;
    a.psi_cur = dp->psi[cur];
    a.psi_prev = dp->psi[1 - cur];
    a.psi_inc = hp.psi_inc;
    a.E = hp.E;
    a.n = hp.n;
    a.D = hp.D;
    a.dim = hp.dim;
    a.persistent = 0;
    a.ainv = dp->ainv;
    a.Bsym = dp->Bsym;
    a.rhs_dir = hp.rhs_fixed.empty() ? nullptr : dp->rhs_dir;
    a.nbr_nodes = dp->nbr_nodes;
    a.ainv32 = dp->ainv32;
    a.Nq = dp->Nq;
    return a;
}

// Face data of an unstructured mesh in the layout the sweep kernels read on
// a lattice, one entry per element slot, in the element's own slot order
// (local index la of slot s = remaining reference axes ascending):
//  * B [E*nslot][dim][nf][nf]: the face's normal moments, rows and columns
//    permuted from the face's node order to the slot's, times the sign that
//    makes (s odd ? 1 : -1) B the moments of the element's outward normal
//    (the kernels' convention, where odd slots are the minus side);
//  * slot_face[e][s] = e*nslot + s;
//  * kink rows: every row of a (face, direction) with a sign change becomes
//    two rows, 2R + [element is the minus side], each holding its element's
//    inflow block in half (s & 1) and its outflow block in the other half
//    (the halves the kernels read for a slot of that parity), and the
//    schedule's kink indices are remapped to them;
//  * nbr_nodes [E*nslot][nf]: the neighbour's DG node on the same point as
//    local index la of the slot.
void unstructured_face_view(const HostProblem& hp, std::vector<double>& B, std::vector<int32_t>& slot_face,
                            std::vector<double>& kink, std::vector<int32_t>& kink_idx, std::vector<int32_t>& nbr) {
    const int ns = hp.nslot, nf = hp.nf, dim = hp.dim;
    const int64_t E = hp.E;
    // face-order index of each local index of every element slot
    std::vector<int32_t> pos((size_t)E * ns * nf);
    for (int64_t e = 0; e < E; ++e)
        for (int s = 0; s < ns; ++s) {
            const int32_t* tr = slot_trace(hp, e, s);
            for (int la = 0; la < nf; ++la) {
                int l = -1;
                for (int k = 0; k < nf; ++k)
                    if (tr[k] == hp.slot_nodes[(size_t)s * nf + la]) l = k;
                if (l < 0) throw Error(SNSW_E_STATE, "unstructured mesh: slot node map");
                pos[((size_t)e * ns + s) * nf + la] = l;
            }
        }
    B.assign((size_t)E * ns * dim * nf * nf, 0.0);
    slot_face.assign((size_t)E * ns, 0);
    nbr.assign((size_t)E * ns * nf, 0);
    for (int64_t e = 0; e < E; ++e)
        for (int s = 0; s < ns; ++s) {
            const size_t hs = (size_t)e * ns + s;
            slot_face[hs] = (int32_t)hs;
            const int32_t f = hp.slot_face[hs];
            const double sg = ((s & 1) ? 1.0 : -1.0) * (slot_is_minus(hp, e, s) ? 1.0 : -1.0);
            const int32_t* P = &pos[hs * nf];
            for (int a = 0; a < dim; ++a)
                for (int i = 0; i < nf; ++i)
                    for (int j = 0; j < nf; ++j)
                        B[((hs * dim + a) * nf + i) * nf + j] =
                            sg * hp.B[(((size_t)f * dim + a) * nf + P[i]) * nf + P[j]];
            if (hp.slot_nbr[hs] >= 0)
                for (int la = 0; la < nf; ++la) nbr[hs * nf + la] = hp.hf_up_trace[hs * nf + P[la]];
        }
    // kink rows per element slot
    const size_t K = hp.kink_tab.size() / (2 * (size_t)nf * nf);
    kink.assign(2 * K * 2 * nf * nf, 0.0);
    kink_idx.assign(hp.kink_idx.size(), 0);
    std::vector<uint8_t> done(2 * K, 0);
    const size_t P4 = hp.pairs.size() / 4;
    for (size_t t = 0; t < P4; ++t) {
        const int32_t e = hp.pairs[4 * t], packed = hp.pairs[4 * t + 1], kb = hp.pairs[4 * t + 2];
        if (e < 0) continue;
        int kc = 0;
        for (int s = 0; s < ns; ++s) {
            const uint32_t cls = ((uint32_t)packed >> (kDirBits + 3 * s)) & 3u;
            if (cls != SC_KINK) continue;
            const size_t hs = (size_t)e * ns + s;
            const bool minus = slot_is_minus(hp, e, s);
            const int32_t R = hp.kink_idx[(size_t)kb + kc];
            const size_t row = 2 * (size_t)R + (minus ? 1 : 0);
            kink_idx[(size_t)kb + kc] = (int32_t)row;
            ++kc;
            if (done[row]) continue;
            done[row] = 1;
            const double* Pp = &hp.kink_tab[(size_t)R * 2 * nf * nf];
            const double* Pm = Pp + (size_t)nf * nf;
            const double* Pin = minus ? Pm : Pp;
            const double* Pout = minus ? Pp : Pm;
            double* dst = &kink[row * 2 * nf * nf];
            double* din = dst + ((s & 1) ? nf * nf : 0);
            double* dout = dst + ((s & 1) ? 0 : nf * nf);
            const int32_t* P = &pos[hs * nf];
            for (int i = 0; i < nf; ++i)
                for (int j = 0; j < nf; ++j) {
                    din[i * nf + j] = Pin[P[i] * nf + P[j]];
                    dout[i * nf + j] = Pout[P[i] * nf + P[j]];
                }
        }
    }
}

void sync_entry(SweepArgs* table, int k, const snsw_problem* prob, int* entry_cur, hipStream_t s) {
    const DeviceProblem* dp = prob->dev;
    if (*entry_cur == dp->cur) return;
    hipLaunchKernelGGL(set_entry_kernel, dim3(1), dim3(1), 0, s, table, k, dp->psi[dp->cur], dp->psi[1 - dp->cur]);
    HIP_OK(hipGetLastError());
    *entry_cur = dp->cur;
}

void enqueue_sweep(const SweepLaunch& L, const std::vector<SweepClass>& classes, hipStream_t s,
                   LaunchProfiler* prof) {
    launch_source(L.table, L.count, L.max_En, L.phi_in_list, L.phi_in_one, L.tickets, L.n_tickets, s);
    HIP_OK(hipGetLastError());
    if (L.any_persistent) {
        launch_fill_sentinel(L.table, L.count, L.max_DEn, s);
        HIP_OK(hipGetLastError());
    }
    for (const SweepClass& c : classes) {
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
            // streaming loads of A^{-1} paid off on tiled single-problem
            // sweeps (2D 128^2 p = 3 S8: 4 %) and lost on batches
            pa.nt = c.intra != nullptr ? 1 : 0;
            if (prof) prof->begin(s);
            if (!launch_sweep_persistent(c.dim, c.p, c.simplex, c.unstructured, c.inv, pa, c.blocks, s,
                                         c.mixed && c.inv))
                throw Error(SNSW_E_UNSUPPORTED, "no persistent kernel reads FP32 inverses for this element");
            if (prof) prof->end(s);
        } else {
            for (size_t k = 0; k + 1 < c.level_off.size(); ++k) {
                // with a partial inverse cache: the cached pairs of the
                // level, then its assembled ones
                const int64_t b = c.level_off[k], end = c.level_off[k + 1];
                const int64_t m = c.level_split.empty() ? end : c.level_split[k];
                if (prof) prof->begin(s);
                launch_sweep_level(c.dim, c.p, c.simplex, c.mixed, c.inv, c.unstructured, L.table, c.pairs, b, m - b,
                                   class_problem(c), s, c.face_points);
                if (prof) prof->end(s);
                if (end > m) {
                    if (prof) prof->begin(s);
                    launch_sweep_level(c.dim, c.p, c.simplex, c.mixed, false, c.unstructured, L.table, c.pairs, m,
                                       end - m, class_problem(c), s, c.face_points);
                    if (prof) prof->end(s);
                }
            }
        }
        HIP_OK(hipGetLastError());
    }
    launch_scalar_flux(L.table, L.count, L.max_En, L.phi_out_list, L.phi_out_one, s);
    HIP_OK(hipGetLastError());
}

void check_error_flag(int32_t* flag, hipStream_t s) {
    int32_t err = 0;
    HIP_OK(hipMemcpyAsync(&err, flag, sizeof(err), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (err) {
        HIP_OK(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
        HIP_OK(hipStreamSynchronize(s));
        throw Error(SNSW_E_STATE, "a dependency wait of the persistent sweep timed out; results are invalid");
    }
}

int persistent_grid(int dim, int p, bool simplex, bool unstructured, bool inv, int64_t total, int device,
                    double fraction, bool f32) {
    int cus = 0;
    HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    const int per_cu = persistent_blocks_per_cu(dim, p, simplex, unstructured, inv, f32);
    const int n = simplex ? (p + 1) * (p + 2) / 2 : dim == 2 ? (p + 1) * (p + 1) : (p + 1) * (p + 1) * (p + 1);
    const int64_t per_block = 4 * (64 / n);
    const int64_t need = (total + per_block - 1) / per_block;
    const int64_t cap = std::max<int64_t>(1, (int64_t)(fraction * per_cu * cus));
    return (int)std::max<int64_t>(1, std::min<int64_t>(need, cap));
}

void device_check_ctx(snsw_ctx* ctx) {
    int n = 0;
    HIP_OK(hipGetDeviceCount(&n));
    if (ctx->device >= n) throw Error(SNSW_E_INVALID_ARG, "device id out of range");
}

void device_upload(snsw_problem* prob) {
    HostProblem& hp = prob->hp;
    DeviceGuard g(prob->ctx->device);
    auto* dp = new DeviceProblem();
    prob->dev = dp;
    dp->device = prob->ctx->device;
    dp->stream = static_cast<hipStream_t>(prob->ctx->stream);
    const hipStream_t s = dp->stream;
    const int n = hp.n, dim = hp.dim;
    // cached inverses, decided before anything is allocated: D*E blocks of
    // about n^2 doubles (FP64), or of n^2 floats in mixed precision
    // (elements of at most 32 nodes).  AUTO: all of them within the budget,
    // else (level schedule) the first directions that fit, whose pairs each
    // level then sweeps apart from the assembled ones
    const bool mixed = hp.precision == SNSW_PREC_MIXED;
    const int64_t blk = ainv_block_bytes(hp.dim, hp.p, hp.simplex, mixed);
    int cache_dirs = 0;
    if (hp.cache_inverse != SNSW_CACHE_OFF && blk > 0) {
        if (hp.cache_inverse == SNSW_CACHE_ON) {
            cache_dirs = hp.D;
        } else {
            size_t free_b = 0, total_b = 0;
            HIP_OK(hipMemGetInfo(&free_b, &total_b));
            const double budget = hp.cache_budget > 0.0 ? hp.cache_budget : 0.5 * (double)free_b;
            const double fit = std::floor(budget / ((double)hp.E * (double)blk));
            if (fit >= (double)hp.D) cache_dirs = hp.D;
            else if (hp.schedule == SNSW_SCHED_LEVELS && fit >= 1.0) cache_dirs = (int)fit;
        }
    }
    if (hp.schedule == SNSW_SCHED_LEVELS) arrange_levels_for_cache(hp, cache_dirs);
    // geometry: matrix k of element e stored column-major at [e][k][j][i]
    {
        std::vector<double> geo((size_t)hp.E * (dim + 1) * n * n);
        for (int64_t e = 0; e < hp.E; ++e) {
            double* G = &geo[(size_t)e * (dim + 1) * n * n];
            const double* Me = &hp.M[(size_t)e * n * n];
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) G[j * n + i] = Me[i * n + j];
            for (int k = 0; k < dim; ++k) {
                const double* Kk = &hp.K[((size_t)e * dim + k) * n * n];
                double* Gk = G + (size_t)(k + 1) * n * n;
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j) Gk[j * n + i] = Kk[i * n + j];
            }
        }
        dp->geo = dupload(dp, geo, s);
        HIP_OK(hipStreamSynchronize(s));
    }
    // face data as the kernels read it: per face in the face's node order on
    // a lattice; per element slot in the element's own slot order on an
    // unstructured mesh (see unstructured_face_view)
    std::vector<double> uB, ukink;
    std::vector<int32_t> uslot_face, ukink_idx, unbr;
    if (hp.unstructured) unstructured_face_view(hp, uB, uslot_face, ukink, ukink_idx, unbr);
    const std::vector<double>& Bdev = hp.unstructured ? uB : hp.B;
    const int64_t Fdev = hp.unstructured ? hp.E * hp.nslot : hp.F;
    dp->B = dupload(dp, Bdev, s);
    if (hp.unstructured) dp->nbr_nodes = dupload(dp, unbr, s);
    if (hp.dim == 3) {
        // B_a[i][j] = int N_a phi_i phi_j is symmetric in the two face nodes:
        // the level sweeps read its packed upper triangle
        const int nf = hp.nf, nt = nf * (nf + 1) / 2, fs = bsym_face_stride(nf);
        // the kernels index the packed moments with 32-bit offsets
        if ((double)Fdev * fs >= 2147483647.0) throw Error(SNSW_E_UNSUPPORTED, "too many faces for the 3D sweep");
        std::vector<double> bs((size_t)Fdev * fs, 0.0);
        for (int64_t f = 0; f < Fdev; ++f)
            for (int a = 0; a < 3; ++a) {
                const double* Bm = &Bdev[((size_t)f * 3 + a) * nf * nf];
                double* dst = &bs[(size_t)f * fs + a * nt];
                for (int i = 0; i < nf; ++i)
                    for (int j = i; j < nf; ++j)
                        dst[i * nf - (i * (i - 1)) / 2 + (j - i)] = 0.5 * (Bm[i * nf + j] + Bm[j * nf + i]);
            }
        dp->Bsym = dupload(dp, bs, s);
        HIP_OK(hipStreamSynchronize(s));
        // p = 2 lattices with 4 x 4 face Gauss points (r = 2): the level
        // sweep contracts the inflow through w_q N(q) instead of the moments
        if (!hp.unstructured && hp.p == 2 && hp.r == 2) dp->Nq = dupload(dp, hp.Nq, s);
    }
    dp->kink_tab = dupload(dp, hp.unstructured ? ukink : hp.kink_tab, s);
    dp->kink_idx = dupload(dp, hp.unstructured ? ukink_idx : hp.kink_idx, s);
    {
        int4* pp = dalloc<int4>(dp, hp.pairs.size() / 4);
        HIP_OK(hipMemcpyAsync(pp, hp.pairs.data(), hp.pairs.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        dp->pairs = pp;
    }
    if (hp.tile > 0) {
        dp->tpairs = dalloc<int4>(dp, hp.tpairs.size() / 4);
        HIP_OK(hipMemcpyAsync(dp->tpairs, hp.tpairs.data(), hp.tpairs.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, s));
        dp->tintra = dupload(dp, hp.tintra, s);
        if (hp.dim == 2) {
            // slot records of every tiled entry, read together with the entry
            // (one round trip less before the element's inflow can be formed)
            const int NS = 4;
            const size_t Pt = hp.tpairs.size() / 4;
            std::vector<int32_t> rec(Pt * 3 * NS, 0);
            for (size_t t = 0; t < Pt; ++t) {
                const int32_t e = hp.tpairs[4 * t], packed = hp.tpairs[4 * t + 1], kb = hp.tpairs[4 * t + 2];
                if (e < 0) continue;
                int kc = 0;
                for (int sl = 0; sl < NS; ++sl) {
                    rec[(3 * t + 0) * NS + sl] = hp.slot_nbr[(size_t)e * NS + sl];
                    rec[(3 * t + 1) * NS + sl] = hp.slot_face[(size_t)e * NS + sl];
                    const uint32_t cls = ((uint32_t)packed >> (kDirBits + 3 * sl)) & 3u;
                    if (cls == SC_KINK) rec[(3 * t + 2) * NS + sl] = hp.kink_idx[(size_t)kb + kc++];
                }
            }
            dp->tslots = dalloc<int4>(dp, Pt * 3);
            HIP_OK(hipMemcpyAsync(dp->tslots, rec.data(), rec.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
            HIP_OK(hipStreamSynchronize(s));
        }
    }
    dp->slot_face = dupload(dp, hp.unstructured ? uslot_face : hp.slot_face, s);
    dp->slot_nbr = dupload(dp, hp.slot_nbr, s);
    dp->sigma_t = dupload(dp, hp.sigma_t, s);
    dp->sigma_s = dupload(dp, hp.sigma_s, s);
    dp->q = dupload(dp, hp.q, s);
    if (!hp.rhs_fixed.empty()) dp->rhs_dir = dupload(dp, hp.rhs_fixed, s);
    dp->omega = dupload(dp, hp.omega, s);
    dp->w = dupload(dp, hp.w, s);
    dp->src = dalloc<double>(dp, (size_t)hp.E * n);
    dp->phi_tmp = dalloc<double>(dp, (size_t)hp.E * n);
    for (int b = 0; b < 2; ++b) {
        dp->psi[b] = dalloc<double>(dp, (size_t)hp.D * hp.E * n);
        HIP_OK(hipMemsetAsync(dp->psi[b], 0, sizeof(double) * hp.D * hp.E * n, s));
    }
    dp->red = dalloc<unsigned long long>(dp, 2);
    dp->ticket = dalloc<unsigned int>(dp, kTicketWords);
    HIP_OK(hipMemsetAsync(dp->ticket, 0, sizeof(unsigned int) * kTicketWords, s));
    dp->error = dalloc<int32_t>(dp, 1);
    HIP_OK(hipMemsetAsync(dp->error, 0, sizeof(int32_t), s));
    {
        const size_t need = (size_t)cache_dirs * hp.E * (size_t)blk;
        if (cache_dirs > 0 && mixed) dp->ainv32 = dalloc<float>(dp, need / sizeof(float));
        else if (cache_dirs > 0) dp->ainv = dalloc<double>(dp, need / sizeof(double));
        hp.inverse_cached = cache_dirs > 0 ? (mixed ? 2 : 1) : 0;
        hp.cached_dirs = cache_dirs;
    }
    SweepClass& c = dp->cls;
    c.dim = hp.dim;
    c.p = hp.p;
    c.mixed = hp.precision == SNSW_PREC_MIXED;
    c.unstructured = hp.unstructured;
    c.simplex = hp.simplex;
    c.face_points = dp->Nq != nullptr;
    // mixed precision without cached inverses (AUTO found too little
    // memory) sweeps level by level: no persistent kernel assembles in FP32
    if (c.mixed && hp.schedule == SNSW_SCHED_PERSISTENT && !dp->ainv32) hp.schedule = SNSW_SCHED_LEVELS;
    c.persistent = hp.schedule == SNSW_SCHED_PERSISTENT;
    c.inv = (dp->ainv != nullptr || dp->ainv32 != nullptr) && (!c.persistent || persistent_uses_inverse(hp.dim, hp.p));
    c.ticket = 0;
    c.pairs = dp->pairs;
    c.level_off = hp.level_off;
    if (!c.persistent) c.level_split = hp.level_split;
    if (c.persistent && hp.tile > 0) {
        c.pairs = dp->tpairs;
        c.level_off = hp.tlevel_off;
        c.intra = dp->tintra;
        c.slots = dp->tslots;
    }
    c.members = {0};
    c.blocks = c.persistent ? persistent_grid(hp.dim, hp.p, hp.simplex, hp.unstructured, c.inv,
                                              hp.level_off.back(), dp->device, 1.0, c.mixed && c.inv)
                            : 0;
    {
        dp->cur = 0;
        dp->table_cur = 0;
        SweepArgs a = make_args(prob, 0);
        a.persistent = c.persistent ? 1 : 0;
        dp->table = dalloc<SweepArgs>(dp, 1);
        HIP_OK(hipMemcpyAsync(dp->table, &a, sizeof(a), hipMemcpyHostToDevice, s));
    }
    if (dp->ainv || dp->ainv32) {
        // a partial cache factors the cached part of every level only
        const int4* fpairs = dp->pairs;
        int64_t fcount = hp.level_off.back();
        std::vector<int32_t> cp;
        int4* tmp = nullptr;
        if (!hp.level_split.empty()) {
            for (size_t k = 0; k < hp.level_split.size(); ++k)
                cp.insert(cp.end(), hp.pairs.begin() + hp.level_off[k] * 4, hp.pairs.begin() + hp.level_split[k] * 4);
            fcount = (int64_t)cp.size() / 4;
            if (fcount > 0) {
                HIP_OK(hipMalloc(&tmp, cp.size() * sizeof(int32_t)));
                HIP_OK(hipMemcpyAsync(tmp, cp.data(), cp.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
            }
            fpairs = tmp;
        }
        if (fcount > 0)
            launch_factor(hp.dim, hp.p, hp.simplex, dp->ainv32 != nullptr, hp.unstructured, dp->table, fpairs, fcount,
                          dp->ainv32 ? (void*)dp->ainv32 : (void*)dp->ainv, s);
        const hipError_t launch_rc = hipGetLastError();
        const hipError_t sync_rc = hipStreamSynchronize(s);
        if (tmp) HIP_OK(hipFree(tmp));
        HIP_OK(launch_rc);
        HIP_OK(sync_rc);
    }
    HIP_OK(hipStreamSynchronize(s));
}

void device_update_source(snsw_problem* prob) {
    DeviceProblem* dp = prob->dev;
    const HostProblem& hp = prob->hp;
    DeviceGuard g(dp->device);
    hipStream_t s = dp->stream;
    HIP_OK(hipStreamSynchronize(s));
    HIP_OK(hipMemcpy(dp->q, hp.q.data(), sizeof(double) * hp.q.size(), hipMemcpyHostToDevice));
    if (!hp.rhs_fixed.empty()) {
        if (!dp->rhs_dir) dp->rhs_dir = dalloc<double>(dp, hp.rhs_fixed.size());
        HIP_OK(hipMemcpy(dp->rhs_dir, hp.rhs_fixed.data(), sizeof(double) * hp.rhs_fixed.size(),
                         hipMemcpyHostToDevice));
    }
    // patch the problem's table entry (its flux buffers stay as they are)
    const double* rd = hp.rhs_fixed.empty() ? nullptr : dp->rhs_dir;
    HIP_OK(hipMemcpy(reinterpret_cast<char*>(dp->table) + offsetof(SweepArgs, rhs_dir), &rd, sizeof(rd),
                     hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(reinterpret_cast<char*>(dp->table) + offsetof(SweepArgs, psi_inc), &hp.psi_inc,
                     sizeof(double), hipMemcpyHostToDevice));
}

void device_release(snsw_problem* prob) noexcept {
    DeviceProblem* dp = prob->dev;
    if (!dp) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(dp->device);
    (void)hipStreamSynchronize(dp->stream);
    dp->prof.release();
    void* ptrs[] = {dp->geo, dp->B, dp->Bsym, dp->nbr_nodes, dp->kink_tab, dp->kink_idx, dp->pairs, dp->tpairs,
                    dp->tintra, dp->tslots,
                    dp->slot_face, dp->slot_nbr,
                    dp->sigma_t, dp->sigma_s, dp->q, dp->rhs_dir, dp->omega, dp->w, dp->src, dp->psi[0], dp->psi[1],
                    dp->phi_tmp, dp->red, dp->ticket, dp->error, dp->table, dp->ainv, dp->ainv32, dp->Nq};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete dp;
    prob->dev = nullptr;
}

}  // namespace snsw

using namespace snsw;

extern "C" {

int snsw_sweep(snsw_problem* prob, const double* d_phi_in, double* d_phi_out, double* d_psi_out) {
    return snsw_guard([&] {
        if (!d_phi_in || !d_phi_out) throw Error(SNSW_E_INVALID_ARG, "NULL flux pointer");
        DeviceProblem* dp = need_device(prob);
        DeviceGuard g(dp->device);
        do_sweep(prob, d_phi_in, d_phi_out, d_psi_out);
    });
}

int snsw_reset(snsw_problem* prob) {
    return snsw_guard([&] {
        DeviceProblem* dp = need_device(prob);
        DeviceGuard g(dp->device);
        const HostProblem& hp = prob->hp;
        for (int b = 0; b < 2; ++b)
            HIP_OK(hipMemsetAsync(dp->psi[b], 0, sizeof(double) * hp.D * hp.E * hp.n, dp->stream));
        dp->cur = 0;
    });
}

int snsw_synchronize(snsw_problem* prob) {
    return snsw_guard([&] {
        DeviceProblem* dp = need_device(prob);
        DeviceGuard g(dp->device);
        check_error_flag(dp->error, dp->stream);
    });
}

int snsw_set_wait_limit(snsw_problem* prob, int32_t polls) {
    return snsw_guard([&] {
        if (polls < 0) throw Error(SNSW_E_INVALID_ARG, "wait limit must be >= 0");
        need_device(prob)->spin_limit = polls;
    });
}

int snsw_residual(snsw_problem* prob, const double* d_a, const double* d_b, double* out) {
    return snsw_guard([&] {
        if (!d_a || !d_b || !out) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        DeviceProblem* dp = need_device(prob);
        DeviceGuard g(dp->device);
        *out = do_residual(dp, prob->hp.E * prob->hp.n, d_a, d_b);
    });
}

int snsw_solve(snsw_problem* prob, const snsw_solve_opts* opts, double* d_phi, double* d_psi,
               snsw_solve_report* report) {
    int status = SNSW_OK;
    const int rc = snsw_guard([&] {
        if (!opts || !d_phi) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        if (opts->max_iters < 1 || opts->check_every < 1 || !(opts->tol >= 0.0))
            throw Error(SNSW_E_INVALID_ARG, "bad solve options");
        DeviceProblem* dp = need_device(prob);
        DeviceGuard g(dp->device);
        const HostProblem& hp = prob->hp;
        const int64_t len = hp.E * hp.n;
        const auto t0 = std::chrono::steady_clock::now();
        double* cur = d_phi;
        double* nxt = dp->phi_tmp;
        double res = INFINITY;
        int it = 0, nh = 0;
        bool done = false;
        // learned correction and its safeguard
        snsw_net* net = opts->precond;
        bool enabled = net != nullptr, pending = false, have_start = false;
        int start_it = 1;
        double start_res = 0.0, plain_rate = INFINITY;
        int rejections = 0, n_corr = 0, n_rej = 0;
        const int check_every = net ? 1 : opts->check_every;
        if (opts->precond_every < 0) throw Error(SNSW_E_INVALID_ARG, "precond_every must be >= 0");
        const int every = opts->precond_every > 1 ? opts->precond_every : 1;
        for (it = 1; it <= opts->max_iters; ++it) {
            do_sweep(prob, cur, nxt, nullptr);
            if (it % check_every == 0 || it == opts->max_iters) {
                res = do_residual(dp, len, nxt, cur);
                if (report && report->history && nh < report->history_cap) report->history[nh++] = res;
                if (std::isnan(res) || res > 1e300) {
                    status = SNSW_E_DIVERGED;
                    done = true;
                } else if (res <= opts->tol) {
                    done = true;
                }
            }
            if (!done && net && !have_start) {
                start_res = res;
                have_start = true;
            }
            if (!done && net && enabled && it % every == 0 && it > start_it) {
                // per-sweep residual reduction over the window now ending
                // (at least one sweep long: with every = 1 the first
                // correction follows sweep 2); a window that followed a
                // correction must beat the latest plain window
                const double rate = std::pow(res / start_res, 1.0 / std::max(1, it - start_it));
                bool apply = true;
                if (pending) {
                    if (rate >= plain_rate) {
                        ++rejections;
                        ++n_rej;
                        apply = false;
                        if (rejections >= 3) enabled = false;
                    }
                } else {
                    plain_rate = rate;
                }
                pending = apply;
                start_it = it;
                start_res = res;
                if (apply) {
                    net_apply_correction(net, prob, cur, nxt);
                    ++n_corr;
                }
            }
            std::swap(cur, nxt);
            if (done) break;
        }
        if (it > opts->max_iters) it = opts->max_iters;
        if (cur != d_phi) HIP_OK(hipMemcpyAsync(d_phi, cur, sizeof(double) * len, hipMemcpyDeviceToDevice, dp->stream));
        if (d_psi)
            HIP_OK(hipMemcpyAsync(d_psi, dp->psi[dp->cur], sizeof(double) * hp.D * len, hipMemcpyDeviceToDevice,
                                  dp->stream));
        HIP_OK(hipStreamSynchronize(dp->stream));
        if (report) {
            report->iterations = it;
            report->residual = res;
            report->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            report->n_corrected = n_corr;
            report->n_rejected = n_rej;
        }
        if (status == SNSW_OK && !(res <= opts->tol)) status = SNSW_E_NOT_CONVERGED;
        if (status == SNSW_E_DIVERGED) throw Error(SNSW_E_DIVERGED, "source iteration diverged");
        if (status == SNSW_E_NOT_CONVERGED) throw Error(SNSW_E_NOT_CONVERGED, "max_iters reached");
    });
    return rc;
}

int snsw_profile_enable(snsw_problem* prob, int enable) {
    return snsw_guard([&] {
        DeviceProblem* dp = need_device(prob);
        dp->prof.on = enable != 0;
    });
}

int snsw_profile_read(snsw_problem* prob, int64_t* launches, double* kernel_ms) {
    return snsw_guard([&] {
        DeviceProblem* dp = need_device(prob);
        DeviceGuard g(dp->device);
        HIP_OK(hipStreamSynchronize(dp->stream));
        dp->prof.read(launches, kernel_ms);
        check_error_flag(dp->error, dp->stream);
    });
}

int snsw_state_size(const snsw_problem* prob, size_t* bytes) {
    return snsw_guard([&] {
        if (!prob || !bytes) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        *bytes = 64 + sizeof(double) * (size_t)prob->hp.D * prob->hp.E * prob->hp.n;
    });
}

// Layout: 8 int64 header {magic, dim, E, n, D, 0, 0, 0} then psi [D][E][n].
int snsw_state_save(const snsw_problem* prob, void* host_buf, size_t cap) {
    return snsw_guard([&] {
        if (!prob || !host_buf) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        DeviceProblem* dp = need_device(const_cast<snsw_problem*>(prob));
        DeviceGuard g(dp->device);
        const HostProblem& hp = prob->hp;
        const size_t body = sizeof(double) * (size_t)hp.D * hp.E * hp.n;
        if (cap < 64 + body) throw Error(SNSW_E_SHAPE, "state buffer too small");
        int64_t hdr[8] = {0x534e535745455031LL, hp.dim, hp.E, hp.n, hp.D, 0, 0, 0};
        std::memcpy(host_buf, hdr, 64);
        HIP_OK(hipMemcpyAsync(static_cast<char*>(host_buf) + 64, dp->psi[dp->cur], body, hipMemcpyDeviceToHost,
                              dp->stream));
        HIP_OK(hipStreamSynchronize(dp->stream));
    });
}

int snsw_state_load(snsw_problem* prob, const void* host_buf, size_t size) {
    return snsw_guard([&] {
        if (!prob || !host_buf) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        DeviceProblem* dp = need_device(prob);
        DeviceGuard g(dp->device);
        const HostProblem& hp = prob->hp;
        const size_t body = sizeof(double) * (size_t)hp.D * hp.E * hp.n;
        int64_t hdr[8];
        if (size < 64 + body) throw Error(SNSW_E_STATE, "state buffer too small");
        std::memcpy(hdr, host_buf, 64);
        if (hdr[0] != 0x534e535745455031LL || hdr[1] != hp.dim || hdr[2] != hp.E || hdr[3] != hp.n || hdr[4] != hp.D)
            throw Error(SNSW_E_STATE, "state does not match this problem");
        HIP_OK(hipMemcpyAsync(dp->psi[dp->cur], static_cast<const char*>(host_buf) + 64, body,
                              hipMemcpyHostToDevice, dp->stream));
        HIP_OK(hipStreamSynchronize(dp->stream));
    });
}

}  // extern "C"
