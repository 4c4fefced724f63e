// Device kernels of the sweep (declarations shared by the HIP sources).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace snsw {

// Per-problem arguments, kept in a device table indexed by the problem
// field of each schedule entry (a single problem is a table of one).  Every
// batch of G = 64/n consecutive schedule entries belongs to one problem, so a
// wavefront reads its entry with scalar loads.
struct SweepArgs {
    const double* geo;        // [E][dim+1][n][n], matrix k stored column-major
    const double* B;          // [F][dim][nf][nf] face normal moments
    const double* kink_tab;   // [K][2][nf][nf] P_plus, P_minus
    const int32_t* kink_idx;  // per-pair kink rows
    const int32_t* slot_face; // [E][2 dim]
    const int32_t* slot_nbr;  // [E][2 dim]
    const double* sigma_t;    // [E]
    const double* sigma_s;    // [E]
    const double* q;          // [E][n]
    const double* omega;      // [D][3]
    const double* w;          // [D]
    double* src;              // [E][n] volume source incl. scattering
    double* psi_cur;          // [D][E][n] written by the current sweep
    double* psi_prev;         // [D][E][n] the previous sweep (lagged couplings)
    double psi_inc;           // incident flux on inflow boundary faces
    int64_t E;
    int32_t n, D, dim;
    int32_t persistent;       // swept by a persistent kernel (needs the sentinel fill)
    const double* ainv;       // [D][E] blocks of cached A^{-1} (kernels.hip InvLayout; null: not cached)
    const double* Bsym;       // 3D: [F][bsym_face_stride(nf)]: per face the dim moment matrices
                              // (symmetric in the two face nodes), each as its upper triangle row by
                              // row, nf (nf + 1) / 2 entries (null in 2D)
    const double* rhs_dir;    // [D][E][n] fixed right-hand side per pair: M q_d (direction-dependent
                              // source) + tabulated boundary inflow; null when the problem has neither
    const int32_t* nbr_nodes; // unstructured meshes: [E][2 dim][nf] the upwind neighbour's node on the
                              // point of each slot node (slot order); null on a lattice, where it is
                              // the opposite slot's node of the same local index
    const float* ainv32;      // mixed precision: [D][E] blocks of A^{-1} rounded to FP32 (kernels.hip
                              // InvLayout32), or null
    const double* Nq;         // 3D lattices, p = 2, 4 x 4 face Gauss points: [F][16][3] w_q N(q) at the
                              // points q = 4 q_t + q_s (face order), or null (moments instead)
};

// Doubles per face in the packed face-moment array Bsym: dim packed upper
// triangles of nf (nf + 1) / 2 entries, padded to an even count so that every
// face starts on a 16-byte boundary.
__host__ __device__ constexpr int bsym_face_stride(int nf) { return (3 * nf * (nf + 1) / 2 + 1) & ~1; }

// Persistent sweeps take batches from kStreams counters per schedule, each
// kTicketStride words apart (separate cache lines).
constexpr unsigned kTicketStride = 64;
constexpr unsigned kMaxStreams = 64;
constexpr unsigned kTicketWords = kMaxStreams * kTicketStride;   // per schedule

// Schedule entry (int4): {element (-1 = padding), packed word, kink base,
// problem index}.

// Arguments of the persistent sweep: pairs are claimed in schedule order from
// an atomic ticket; a pair waits only for the upwind face values it reads
// (the current buffer holds the sentinel until they are written).
struct PersistArgs {
    const SweepArgs* table;
    const int4* pairs;
    unsigned int* ticket;     // kMaxStreams counters, kTicketStride apart; zeroed by the source kernel
    int32_t* error;           // set to 1 when a dependency wait times out
    int64_t total;            // entries in the schedule
    int32_t spin_limit;       // polls per dependency wait before giving up
    const int32_t* intra;     // tiled schedules: intra-tile dependency word per entry (else null)
    int32_t problem;          // table index of every entry, or -1 when entries name their problem
    const int4* slots;        // 2D: per entry {neighbour[4]}, {face[4]}, {kink row[4]} of its slots, or null
    int32_t nt;               // DPP kernels: read the cached inverses with non-temporal loads
};

// Launches the persistent sweep kernel (all levels in one launch); inv: read
// the cached inverses (f32: their FP32 copy); simplex / unstructured: element
// lists (triangles, or quads / hexes), swept by the generic persistent
// kernels with the upwind node table.  Returns false, launching nothing, for
// a combination without a kernel (f32 outside persistent_f32).
bool launch_sweep_persistent(int dim, int p, bool simplex, bool unstructured, bool inv, const PersistArgs& a,
                             int blocks, hipStream_t stream, bool f32 = false);
// Blocks per CU that the persistent kernel can keep resident.
int persistent_blocks_per_cu(int dim, int p, bool simplex, bool unstructured, bool inv, bool f32 = false);
// Whether the persistent kernel of this shape reads FP32 cached inverses
// (2D lattices: the DPP and LDS kernels).
bool persistent_f32(int dim, int p, bool simplex, bool unstructured);
// Whether the persistent kernel of this shape has a cached-inverse variant.
bool persistent_uses_inverse(int dim, int p);
// Launches the level-sweep kernel over schedule entries [begin, begin+count)
// (begin and count multiples of G); simplex: order-p triangles (2D, always
// with the upwind node table); inv: x = A^{-1} b with cached inverses (FP32
// copies when mixed, else FP64);
// unstructured: upwind nodes from SweepArgs::nbr_nodes; problem: table index
// of every entry, or -1 when entries name their problem.
// face_points: every problem of the launch carries SweepArgs::Nq (3D p = 2
// lattices), and the cached-inverse kernel contracts the inflow through it.
void launch_sweep_level(int dim, int p, bool simplex, bool mixed, bool inv, bool unstructured,
                        const SweepArgs* table, const int4* pairs, int64_t begin, int64_t count, int problem,
                        hipStream_t stream, bool face_points = false);
// Bytes per pair of the cached A^{-1}: FP64 (n^2 doubles, n^2 + 1 where blocks
// are padded to a 16-byte multiple) or, f32, rounded to FP32 in groups of four
// columns (0: no FP32 copy for this shape, n > 32).
int64_t ainv_block_bytes(int dim, int p, bool simplex, bool f32);
// Computes A^{-1} of schedule entries [0, count) of one problem in FP64 and
// stores it (f32: rounded to FP32).
void launch_factor(int dim, int p, bool simplex, bool f32, bool unstructured, const SweepArgs* table,
                   const int4* pairs, int64_t count, void* ainv, hipStream_t stream);

// Start of a sweep, for problems [0, count) of the table: swaps psi_cur and
// psi_prev of each entry, zeroes the ticket counters of n_tickets schedules
// (kTicketWords words each), and computes
// src[e][i] = sum_j M_e[i][j] (q[e][j] + sigma_s[e]/(4 pi) phi_in[e][j]).
// phi_in of problem k is phi_list[k], or phi_one when phi_list is null.
void launch_source(SweepArgs* table, int count, int64_t max_En, const double* const* phi_list,
                   const double* phi_one, unsigned int* tickets, int n_tickets, hipStream_t stream);
// Fills psi_cur of every persistent problem with the sentinel.
void launch_fill_sentinel(const SweepArgs* table, int count, int64_t max_DEn, hipStream_t stream);
// phi_out[e][i] = sum_d w[d] psi_cur[d][e][i] (ascending d) for every problem
void launch_scalar_flux(const SweepArgs* table, int count, int64_t max_En, double* const* phi_list,
                        double* phi_one, hipStream_t stream);
// out[0] = max|a-b|, out[1] = max|a| as the bit patterns of nonnegative
// doubles (out must be zeroed first)
void launch_residual(int64_t len, const double* a, const double* b, unsigned long long* out,
                     hipStream_t stream);

}  // namespace snsw
