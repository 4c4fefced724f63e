// Device-side state shared by single-problem sweeps and batches.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

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

// One group of problems swept by the same kernel: same dim, p and
// precision.  Its schedule concatenates, level by level, the level segments
// of its problems (each a multiple of G entries, so a batch of G entries
// never spans two problems).
struct SweepClass {
    int dim = 2, p = 1;
    bool mixed = false;
    bool persistent = false;
    bool inv = false;                  // cached inverses (every member has them)
    bool unstructured = false;         // members are unstructured meshes (upwind nodes from a table)
    bool simplex = false;              // members are simplex meshes
    bool face_points = false;          // every member carries face Gauss-point normals (DeviceProblem::Nq)
    int blocks = 0;                    // persistent grid
    int ticket = 0;                    // index into the ticket array
    const int4* pairs = nullptr;       // device schedule
    const int32_t* intra = nullptr;    // tiled schedule: intra-tile dependency words
    const int4* slots = nullptr;       // per entry slot records (2D; else null: element tables)
    std::vector<int64_t> level_off;    // [L+1] offsets into pairs
    std::vector<int64_t> level_split;  // [L] partial inverse cache: end of each level's cached pairs (else empty)
    std::vector<int> members;          // table indices of its problems
};

// The table index shared by every entry of a one-problem class, else -1.
inline int class_problem(const SweepClass& c) { return c.members.size() == 1 ? c.members[0] : -1; }

// Optional HIP events around the sweep kernels of eager sweeps.
struct LaunchProfiler {
    bool on = false;
    std::vector<hipEvent_t> events;
    size_t used = 0;
    void begin(hipStream_t s);
    void end(hipStream_t s);
    void read(int64_t* launches, double* ms);
    void release() noexcept;
};

struct DeviceProblem {
    int device = 0;
    hipStream_t stream = nullptr;
    double* geo = nullptr;        // [E][dim+1][n][n] column-major matrices
    double* B = nullptr;          // [F][dim][nf][nf]
    double* Bsym = nullptr;       // 3D: [F][bsym_face_stride(nf)] packed upper triangles of B
    double* Nq = nullptr;         // 3D p = 2 lattices (r = 2): [F][16][3] w_q N(q) at the face Gauss points
    int32_t* nbr_nodes = nullptr; // unstructured meshes: [E][nslot][nf] neighbour node of each slot node
    double* kink_tab = nullptr;   // [K][2][nf][nf]
    int32_t* kink_idx = nullptr;
    int4* pairs = nullptr;
    int4* tpairs = nullptr;       // tiled schedule (or null)
    int32_t* tintra = nullptr;
    int4* tslots = nullptr;       // tiled schedule: per entry neighbours, faces, kink rows of its slots
    int32_t* slot_face = nullptr;
    int32_t* slot_nbr = nullptr;
    double* sigma_t = nullptr;
    double* sigma_s = nullptr;
    double* q = nullptr;
    double* rhs_dir = nullptr;    // [D][E][n] fixed right-hand side per pair, or null
    double* omega = nullptr;
    double* w = nullptr;
    double* src = nullptr;        // [E][n]
    double* psi[2] = {nullptr, nullptr};
    double* phi_tmp = nullptr;    // [E][n]
    unsigned long long* red = nullptr;   // residual scratch [2]
    unsigned int* ticket = nullptr;
    int32_t* error = nullptr;     // device-side wait failure flag
    int32_t spin_limit = 1 << 20; // polls per dependency wait of persistent sweeps
    double* ainv = nullptr;       // [D][E] cached A^{-1} blocks (InvLayout) or null
    float* ainv32 = nullptr;      // mixed precision: [D][E] FP32 A^{-1} blocks (InvLayout32) or null
    SweepArgs* table = nullptr;   // this problem as a table of one
    int table_cur = 0;            // buffer index in table->psi_cur
    int cur = 0;                  // psi[cur] holds the latest sweep
    SweepClass cls;
    size_t bytes = 0;
    LaunchProfiler prof;
};

// Table entry of a problem whose psi_cur is psi[cur] (the next sweep swaps).
SweepArgs make_args(const snsw_problem* prob, int cur);
// Makes entry k of a device table agree with the problem's latest buffer.
void sync_entry(SweepArgs* table, int k, const snsw_problem* prob, int* entry_cur, hipStream_t s);

// Enqueues one sweep of every problem of a table on stream s: source (and
// buffer swap), sentinel fill, the classes' sweep kernels, scalar flux.
struct SweepLaunch {
    SweepArgs* table = nullptr;
    int count = 0;
    int64_t max_En = 0, max_DEn = 0;
    bool any_persistent = false;
    unsigned int* tickets = nullptr;
    int n_tickets = 0;
    int32_t* error = nullptr;
    int32_t spin_limit = 1 << 20;      // polls per dependency wait of persistent sweeps
    const double* const* phi_in_list = nullptr;
    const double* phi_in_one = nullptr;
    double* const* phi_out_list = nullptr;
    double* phi_out_one = nullptr;
};
void enqueue_sweep(const SweepLaunch& L, const std::vector<SweepClass>& classes, hipStream_t s,
                   LaunchProfiler* prof);

// Enqueues the sweep kernels of one class (no source, fill or scalar flux).
void enqueue_sweep_class(const SweepLaunch& L, const SweepClass& c, hipStream_t s);

// Reads and clears a device wait-failure flag (synchronises s).
void check_error_flag(int32_t* flag, hipStream_t s);

DeviceProblem* need_device(snsw_problem* prob);
int persistent_grid(int dim, int p, bool simplex, bool unstructured, bool inv, int64_t total, int device,
                    double fraction = 1.0, bool f32 = false);

}  // namespace snsw
