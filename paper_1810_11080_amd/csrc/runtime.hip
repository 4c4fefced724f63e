// Device side of a problem: uploads, one sweep, source iteration, state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstdint>
#include <cmath>
#include <cstring>
#include <string>

#include "internal.hpp"
#include "kernels.hpp"

namespace snsw {

#define HIP_OK(expr)                                                                          \
    do {                                                                                      \
        hipError_t _e = (expr);                                                               \
        if (_e != hipSuccess)                                                                 \
            throw Error(_e == hipErrorOutOfMemory ? SNSW_E_OOM : SNSW_E_HIP,                  \
                        std::string(#expr) + ": " + hipGetErrorString(_e));                  \
    } while (0)

struct DeviceProblem {
    int device = 0;
    hipStream_t stream = nullptr;
    double* geo = nullptr;        // [E][dim+1][n][n] column-major matrices
    double* B = nullptr;          // [F][dim][nf][nf]
    double* kink_tab = nullptr;   // [K][2][nf][nf]
    int32_t* kink_idx = nullptr;
    int4* pairs = nullptr;
    int32_t* slot_face = nullptr;
    int32_t* slot_nbr = nullptr;
    double* sigma_t = nullptr;
    double* sigma_s = nullptr;
    double* q = nullptr;
    double* omega = nullptr;
    double* w = nullptr;
    double* src = nullptr;        // [E][n]
    double* psi[2] = {nullptr, nullptr};
    double* phi_tmp = nullptr;    // [E][n]
    unsigned long long* red = nullptr;   // residual scratch [2]
    unsigned int* ticket = nullptr;
    int32_t* error = nullptr;     // device-side wait failure flag
    int32_t epoch = 0;
    int blocks = 0;               // persistent grid size
    int cur = 0;                  // psi[cur] holds the previous sweep
    std::vector<int64_t> level_off;
    size_t bytes = 0;
    // profiling: event pairs around level launches
    bool profiling = false;
    std::vector<hipEvent_t> events;
    size_t n_events = 0;
};

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

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (dev >= 0 && dev != prev) HIP_OK(hipSetDevice(dev));
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

DeviceProblem* need_device(snsw_problem* prob) {
    if (!prob) throw Error(SNSW_E_INVALID_ARG, "NULL problem");
    if (!prob->dev) throw Error(SNSW_E_UNSUPPORTED, "host-only context: no device work");
    return prob->dev;
}

void do_sweep(snsw_problem* prob, const double* phi_in, double* phi_out, double* psi_out) {
    DeviceProblem* dp = need_device(prob);
    const HostProblem& hp = prob->hp;
    const hipStream_t s = dp->stream;
    const bool persistent = hp.schedule == SNSW_SCHED_PERSISTENT;
    launch_source(hp.dim, hp.n, hp.E, dp->geo, dp->q, dp->sigma_s, phi_in, dp->src,
                  persistent ? dp->ticket : nullptr, s);
    HIP_OK(hipGetLastError());
    SweepArgs a;
    a.pairs = dp->pairs;
    a.geo = dp->geo;
    a.B = dp->B;
    a.kink_tab = dp->kink_tab;
    a.kink_idx = dp->kink_idx;
    a.slot_face = dp->slot_face;
    a.slot_nbr = dp->slot_nbr;
    a.sigma_t = dp->sigma_t;
    a.omega = dp->omega;
    a.src = dp->src;
    a.psi_prev = dp->psi[dp->cur];
    a.psi_cur = dp->psi[1 - dp->cur];
    a.psi_inc = hp.psi_inc;
    a.E = hp.E;
    const bool mixed = hp.precision == SNSW_PREC_MIXED;
    if (persistent) {
        if (dp->epoch == INT32_MAX) dp->epoch = 0;   // sentinel payloads only need to differ from 0
        PersistArgs pa;
        pa.s = a;
        pa.ticket = dp->ticket;
        pa.error = dp->error;
        pa.total = dp->level_off.back();
        pa.epoch = ++dp->epoch;
        pa.spin_limit = 1 << 20;
        launch_fill_sentinel(a.psi_cur, (int64_t)hp.D * hp.E * hp.n, pa.epoch, s);
        if (dp->profiling) {
            while (dp->n_events + 2 > dp->events.size()) {
                hipEvent_t ev;
                HIP_OK(hipEventCreate(&ev));
                dp->events.push_back(ev);
            }
            HIP_OK(hipEventRecord(dp->events[dp->n_events++], s));
        }
        launch_sweep_persistent(hp.dim, hp.p, mixed, pa, dp->blocks, s);
        if (dp->profiling) HIP_OK(hipEventRecord(dp->events[dp->n_events++], s));
    }
    for (size_t k = 0; !persistent && k + 1 < dp->level_off.size(); ++k) {
        const int64_t b = dp->level_off[k], c = dp->level_off[k + 1] - b;
        if (dp->profiling) {
            while (dp->n_events + 2 > dp->events.size()) {
                hipEvent_t ev;
                HIP_OK(hipEventCreate(&ev));
                dp->events.push_back(ev);
            }
            HIP_OK(hipEventRecord(dp->events[dp->n_events++], s));
            launch_sweep_level(hp.dim, hp.p, mixed, a, b, c, s);
            HIP_OK(hipEventRecord(dp->events[dp->n_events++], s));
        } else {
            launch_sweep_level(hp.dim, hp.p, mixed, a, b, c, s);
        }
    }
    HIP_OK(hipGetLastError());
    launch_scalar_flux(hp.D, hp.E * hp.n, dp->w, a.psi_cur, phi_out, s);
    HIP_OK(hipGetLastError());
    if (psi_out)
        HIP_OK(hipMemcpyAsync(psi_out, a.psi_cur, sizeof(double) * hp.D * hp.E * hp.n, hipMemcpyDeviceToDevice, s));
    dp->cur = 1 - dp->cur;
}

void check_device_error(DeviceProblem* dp) {
    int32_t err = 0;
    HIP_OK(hipMemcpyAsync(&err, dp->error, sizeof(err), hipMemcpyDeviceToHost, dp->stream));
    HIP_OK(hipStreamSynchronize(dp->stream));
    if (err) {
        HIP_OK(hipMemsetAsync(dp->error, 0, sizeof(int32_t), dp->stream));
        HIP_OK(hipStreamSynchronize(dp->stream));
        throw Error(SNSW_E_STATE, "a dependency wait of the persistent sweep timed out; results are invalid");
    }
}

double do_residual(DeviceProblem* dp, int64_t len, const double* a, const double* b) {
    HIP_OK(hipMemsetAsync(dp->red, 0, 2 * sizeof(unsigned long long), dp->stream));
    launch_residual(len, a, b, dp->red, dp->stream);
    HIP_OK(hipGetLastError());
    unsigned long long h[2] = {0, 0};
    HIP_OK(hipMemcpyAsync(h, dp->red, sizeof(h), hipMemcpyDeviceToHost, dp->stream));
    HIP_OK(hipStreamSynchronize(dp->stream));
    check_device_error(dp);
    double num, den;
    std::memcpy(&num, &h[0], 8);
    std::memcpy(&den, &h[1], 8);
    if (!(den > 0.0)) return num > 0.0 || num != num ? INFINITY : 0.0;
    return num / den;
}

}  // namespace

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
    dp->B = dupload(dp, hp.B, s);
    dp->kink_tab = dupload(dp, hp.kink_tab, s);
    dp->kink_idx = dupload(dp, hp.kink_idx, s);
    {
        int4* pp = dalloc<int4>(dp, hp.pairs.size() / 4);
        HIP_OK(hipMemcpyAsync(pp, hp.pairs.data(), hp.pairs.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        dp->pairs = pp;
    }
    dp->slot_face = dupload(dp, hp.slot_face, s);
    dp->slot_nbr = dupload(dp, hp.slot_nbr, s);
    dp->sigma_t = dupload(dp, hp.sigma_t, s);
    dp->sigma_s = dupload(dp, hp.sigma_s, s);
    dp->q = dupload(dp, hp.q, s);
    dp->omega = dupload(dp, hp.omega, s);
    dp->w = dupload(dp, hp.w, s);
    dp->src = dalloc<double>(dp, (size_t)hp.E * n);
    dp->phi_tmp = dalloc<double>(dp, (size_t)hp.E * n);
    for (int b = 0; b < 2; ++b) {
        dp->psi[b] = dalloc<double>(dp, (size_t)hp.D * hp.E * n);
        HIP_OK(hipMemsetAsync(dp->psi[b], 0, sizeof(double) * hp.D * hp.E * n, s));
    }
    dp->red = dalloc<unsigned long long>(dp, 2);
    dp->ticket = dalloc<unsigned int>(dp, 1);
    HIP_OK(hipMemsetAsync(dp->ticket, 0, sizeof(unsigned int), s));
    dp->error = dalloc<int32_t>(dp, 1);
    HIP_OK(hipMemsetAsync(dp->error, 0, sizeof(int32_t), s));
    dp->level_off = hp.level_off;
    {
        int cus = 0;
        HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dp->device));
        const int per_cu = persistent_blocks_per_cu(hp.dim, hp.p, hp.precision == SNSW_PREC_MIXED);
        const int64_t total = hp.level_off.back();
        const int64_t per_block = 4 * (64 / hp.n);
        const int64_t need = (total + per_block - 1) / per_block;
        dp->blocks = (int)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)per_cu * cus));
    }
    HIP_OK(hipStreamSynchronize(s));
}

void device_release(snsw_problem* prob) noexcept {
    DeviceProblem* dp = prob->dev;
    if (!dp) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(dp->device);
    (void)hipStreamSynchronize(dp->stream);
    for (hipEvent_t ev : dp->events) (void)hipEventDestroy(ev);
    void* ptrs[] = {dp->geo, dp->B, dp->kink_tab, dp->kink_idx, dp->pairs, dp->slot_face, dp->slot_nbr,
                    dp->sigma_t, dp->sigma_s, dp->q, dp->omega, dp->w, dp->src, dp->psi[0], dp->psi[1],
                    dp->phi_tmp, dp->red, dp->ticket, dp->error};
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
        check_device_error(dp);
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
        for (it = 1; it <= opts->max_iters; ++it) {
            do_sweep(prob, cur, nxt, nullptr);
            if (it % opts->check_every == 0 || it == opts->max_iters) {
                res = do_residual(dp, len, nxt, cur);
                if (report && report->history && nh < report->history_cap) report->history[nh++] = res;
                if (std::isnan(res) || res > 1e300) {
                    status = SNSW_E_DIVERGED;
                    done = true;
                } else if (res <= opts->tol) {
                    done = true;
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
        dp->profiling = enable != 0;
    });
}

int snsw_profile_read(snsw_problem* prob, int64_t* launches, double* kernel_ms) {
    return snsw_guard([&] {
        DeviceProblem* dp = need_device(prob);
        DeviceGuard g(dp->device);
        HIP_OK(hipStreamSynchronize(dp->stream));
        double total = 0.0;
        for (size_t i = 0; i + 1 < dp->n_events; i += 2) {
            float ms = 0.0f;
            HIP_OK(hipEventElapsedTime(&ms, dp->events[i], dp->events[i + 1]));
            total += ms;
        }
        if (launches) *launches = (int64_t)(dp->n_events / 2);
        if (kernel_ms) *kernel_ms = total;
        dp->n_events = 0;
        check_device_error(dp);
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
