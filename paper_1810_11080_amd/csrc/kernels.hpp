// Device kernels of the sweep (declarations shared by the HIP sources).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace snsw {

// Arguments of one level launch (all device pointers).
struct SweepArgs {
    const int4* pairs;        // [P] {element, packed word, kink base, 0}
    const double* geo;        // [E][dim+1][n][n], matrix k stored column-major
    const double* B;          // [F][dim][nf][nf] face normal moments
    const double* kink_tab;   // [K][2][nf][nf] P_plus, P_minus
    const int32_t* kink_idx;  // per-pair kink rows
    const int32_t* slot_face; // [E][2 dim]
    const int32_t* slot_nbr;  // [E][2 dim]
    const double* sigma_t;    // [E]
    const double* omega;      // [D][3]
    const double* src;        // [E][n] volume source incl. scattering
    const double* psi_prev;   // [D][E][n] previous sweep (lagged couplings)
    double* psi_cur;          // [D][E][n] this sweep
    double psi_inc;           // incident flux on inflow boundary faces
    int64_t E;
};

// Arguments of the persistent sweep: pairs are claimed in schedule order from
// an atomic ticket; a pair waits only for the upwind face values it reads
// (psi_cur holds the epoch's sentinel until they are written).
struct PersistArgs {
    SweepArgs s;
    unsigned int* ticket;     // zeroed by the source kernel before each sweep
    int32_t* error;           // set to 1 when a dependency wait times out
    int64_t total;            // pairs in the schedule
    int32_t epoch;            // >= 1; tags the sentinel of this sweep
    int32_t spin_limit;       // polls per dependency wait before giving up
};

// Launches the persistent sweep kernel (all levels in one launch).
void launch_sweep_persistent(int dim, int p, bool mixed, const PersistArgs& a, int blocks, hipStream_t stream);
// Fills psi (count doubles) with the "not written" sentinel of `epoch`.
void launch_fill_sentinel(double* psi, int64_t count, int epoch, hipStream_t stream);
// Blocks per CU that the persistent kernel can keep resident.
int persistent_blocks_per_cu(int dim, int p, bool mixed);

// Launches the level-sweep kernel over pairs [begin, begin+count).
void launch_sweep_level(int dim, int p, bool mixed, const SweepArgs& a, int64_t begin, int64_t count,
                        hipStream_t stream);
// src[e][i] = sum_j M_e[i][j] (q[e][j] + sigma_s[e]/(4 pi) phi[e][j]);
// also resets the persistent kernel's ticket (if not NULL)
void launch_source(int dim, int n, int64_t E, const double* geo, const double* q,
                   const double* sigma_s, const double* phi, double* src, unsigned int* ticket,
                   hipStream_t stream);
// phi[e][i] = sum_d w[d] psi[d][e][i], ascending d
void launch_scalar_flux(int D, int64_t En, const double* w, const double* psi, double* phi,
                        hipStream_t stream);
// out[0] = max|a-b|, out[1] = max|a| as the bit patterns of nonnegative
// doubles (out must be zeroed first)
void launch_residual(int64_t len, const double* a, const double* b, unsigned long long* out,
                     hipStream_t stream);

}  // namespace snsw
