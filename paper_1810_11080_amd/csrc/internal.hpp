// Handles behind the C-ABI (internal).
#pragma once

#include "host.hpp"

struct snsw_ctx {
    int device = -1;          // -1: host-only
    void* stream = nullptr;   // hipStream_t
};

namespace snsw {
struct DeviceProblem;
}
struct snsw_net;

struct snsw_problem {
    snsw_ctx* ctx = nullptr;
    snsw::HostProblem hp;
    snsw::DeviceProblem* dev = nullptr;
};

namespace snsw {
// runtime.hip
void device_check_ctx(snsw_ctx* ctx);           // validates the device id
void device_upload(snsw_problem* prob);         // allocates and copies
void device_release(snsw_problem* prob) noexcept;
void device_update_source(snsw_problem* prob);  // re-uploads q and the fixed right-hand side
}  // namespace snsw

// Wraps a C-ABI body: maps snsw::Error / std::bad_alloc / others to codes.
template <class F>
int snsw_guard(F&& body) {
    try {
        body();
        snsw::set_last_error("");
        return SNSW_OK;
    } catch (const snsw::Error& e) {
        snsw::set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        snsw::set_last_error("host allocation failed");
        return SNSW_E_OOM;
    } catch (const std::exception& e) {
        snsw::set_last_error(e.what());
        return SNSW_E_STATE;
    } catch (...) {
        snsw::set_last_error("unknown error");
        return SNSW_E_STATE;
    }
}
