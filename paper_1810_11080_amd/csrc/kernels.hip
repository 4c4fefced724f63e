// HIP kernels of the lagged transport sweep for gfx950.
//
// One launch processes every (element, direction) pair of one level of the
// combined schedule: their upwind inputs were produced by earlier levels
// (kept couplings) or by the previous sweep (lagged couplings), so all pairs
// of a level are independent.  Per pair the local system of eq.
// laggedSourceIteration is assembled and solved in registers:
//
//   A = sigma_t M - sum_i Omega_i K_i + sum_{outflow faces} P_out
//   b = M (q + sigma_s/(4 pi) phi) + sum_{inflow faces} P_in psi_upwind
//
// Mapping: a wavefront holds G = 64 / n pairs, lane `row` of a group owns row
// `row` of A and b.  Elimination without pivoting (the symmetric part of A is
// positive definite: A + A^T = 2 sigma_t M + int |Omega.n| u u over the
// element boundary) broadcasts the pivot row through LDS.  Matrices are read
// column-major so that the n lanes of a group load consecutive addresses.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <utility>

#include "kernels.hpp"

namespace snsw {

namespace {

constexpr int kWaves = 4;              // wavefronts per block
#ifndef SNSW_LEVEL_WAVES
#define SNSW_LEVEL_WAVES 1
#endif
// wavefronts per block of the level sweeps (smaller blocks refill the CUs
// sooner as a level drains: 48^3 S12 with cached inverses 32.3 / 31.6 /
// 31.5 ms FP64 and 24.4 / 23.7 / 23.6 ms mixed with 4 / 2 / 1, 8 slower;
// assembled 145.3 -> 127.2 ms with 1)
constexpr int kLevelWaves = SNSW_LEVEL_WAVES;
constexpr int kDirMask = 1023;         // packed word: direction bits
constexpr int kSlotShift = 10;         // then 3 bits per slot
constexpr unsigned kOut = 0, kIn = 1, kKink = 2, kNone = 3;
constexpr int kIntraGroupShiftDev = 8;   // intra word: group of slot s at bits 8 + 4 s
#ifndef SNSW_LEVEL_CHUNK_MIN
#define SNSW_LEVEL_CHUNK_MIN 16   // level sweeps stream A^{-1} in chunks for n above this
#endif
#ifndef SNSW_LEVEL_CHUNK
#define SNSW_LEVEL_CHUNK 0        // level sweeps, n > 16: A^{-1} columns per chunk (0: automatic)
#endif
#ifndef SNSW_LEVEL_LDS_GROUP
#define SNSW_LEVEL_LDS_GROUP 4    // level sweeps, n > 16: entries of b read from LDS per group
#endif
#ifndef SNSW_POLL_SLEEP
#define SNSW_POLL_SLEEP 1   // s_sleep units (64 clocks) between dependency polls
#endif

template <int DIM, int P>
struct TensorShape {
    static constexpr int Q = P + 1;
    static constexpr int N = DIM == 2 ? Q * Q : Q * Q * Q;
    static constexpr int NF = DIM == 2 ? Q : Q * Q;
    static constexpr int NS = 2 * DIM;
    static constexpr int G = 64 / N;
    __host__ __device__ static constexpr int coord(int i, int a) {
        return a == 0 ? i % Q : (a == 1 ? (i / Q) % Q : i / (Q * Q));
    }
    // element node of face-local index b on slot s (remaining axes ascending)
    __host__ __device__ static constexpr int tn(int s, int b) {
        int idx[3] = {0, 0, 0};
        int rem = b;
        for (int x = 0; x < DIM; ++x) {
            if (x == s / 2) continue;
            idx[x] = rem % Q;
            rem /= Q;
        }
        idx[s / 2] = (s & 1) ? P : 0;
        return idx[0] + Q * (idx[1] + Q * idx[2]);
    }
    // face-local index of node i on slot s
    __host__ __device__ static constexpr int local(int i, int s) {
        int l = 0, mul = 1;
        for (int x = 0; x < DIM; ++x) {
            if (x == s / 2) continue;
            l += coord(i, x) * mul;
            mul *= Q;
        }
        return l;
    }
    // whether node i lies on slot s (the xi_a = 0 face for s = 2a, xi_a = 1 for s = 2a + 1)
    __host__ __device__ static constexpr bool on(int i, int s) { return coord(i, s / 2) == ((s & 1) ? P : 0); }
};

// Triangle of order P (simplicial element): nodes on the lattice pairs
// (i, j), i + j <= P, numbered row by row (j slowest); slots are the edges
// v0 -> v1 (j = 0), v1 -> v2 (i + j = P), v2 -> v0 (i = 0), each listed from
// its first vertex.
template <int P>
struct TriShape {
    static constexpr int N = (P + 1) * (P + 2) / 2;
    static constexpr int NF = P + 1;
    static constexpr int NS = 3;
    static constexpr int G = 64 / N;
    __host__ __device__ static constexpr int index(int i, int j) { return j * (P + 1) - j * (j - 1) / 2 + i; }
    __host__ __device__ static constexpr int row_of(int m) {
        int j = 0;
        while (j < P && m >= index(0, j + 1)) ++j;
        return j;
    }
    __host__ __device__ static constexpr int tn(int s, int b) {
        return s == 0 ? index(b, 0) : (s == 1 ? index(P - b, b) : index(0, P - b));
    }
    __host__ __device__ static constexpr bool on(int m, int s) {
        const int j = row_of(m), i = m - index(0, j);
        return s == 0 ? j == 0 : (s == 1 ? i + j == P : i == 0);
    }
    __host__ __device__ static constexpr int local(int m, int s) {
        const int j = row_of(m), i = m - index(0, j);
        return s == 0 ? i : (s == 1 ? j : P - j);
    }
};

// Tetrahedron of order P: nodes on the lattice triples (i, j, l),
// i + j + l <= P, numbered with l slowest, then j; barycentric lattice
// coordinates c = (P - i - j - l, i, j, l).  Slot s is the face opposite
// vertex s, its nodes listed in the face's triangle lattice order over the
// face's vertices in the outward order (1,2,3), (0,3,2), (0,1,3), (0,2,1).
template <int P>
struct TetShape {
    static constexpr int N = (P + 1) * (P + 2) * (P + 3) / 6;
    static constexpr int NF = (P + 1) * (P + 2) / 2;
    static constexpr int NS = 4;
    static constexpr int G = 64 / N;
    __host__ __device__ static constexpr int face_vertex(int s, int v) {
        return s == 0 ? v + 1 : (s == 1 ? (v == 0 ? 0 : 4 - v) : (s == 2 ? (v == 0 ? 0 : (v == 1 ? 1 : 3)) : (v == 0 ? 0 : 3 - v)));
    }
    __host__ __device__ static constexpr int index(int i, int j, int l) {
        int m = 0;
        for (int ll = 0; ll < l; ++ll) m += (P + 1 - ll) * (P + 2 - ll) / 2;
        return m + j * (P - l + 1) - j * (j - 1) / 2 + i;
    }
    // barycentric lattice coordinate v of node m
    __host__ __device__ static constexpr int bary(int m, int v) {
        int l = 0;
        while (l < P && m >= index(0, 0, l + 1)) ++l;
        int r = m - index(0, 0, l), j = 0;
        while (r > P - l - j) r -= P - l - j + 1, ++j;
        const int i = r;
        return v == 0 ? P - i - j - l : (v == 1 ? i : (v == 2 ? j : l));
    }
    __host__ __device__ static constexpr int tn(int s, int b) {
        int bb = 0, r = b;
        while (r > P - bb) r -= P - bb + 1, ++bb;   // face node (a, bb)
        const int a = r;
        int c[4] = {0, 0, 0, 0};
        c[face_vertex(s, 0)] = P - a - bb;
        c[face_vertex(s, 1)] = a;
        c[face_vertex(s, 2)] = bb;
        return index(c[1], c[2], c[3]);
    }
    __host__ __device__ static constexpr bool on(int m, int s) { return bary(m, s) == 0; }
    __host__ __device__ static constexpr int local(int m, int s) {
        const int a = bary(m, face_vertex(s, 1)), bb = bary(m, face_vertex(s, 2));
        return bb * (P + 1) - bb * (bb - 1) / 2 + a;
    }
};

// Element shapes: Shape<DIM, P> is the Q_P tensor element; for P >= kTri
// the triangle of order P - kTri (2D) and for P >= kTet the tetrahedron of
// order P - kTet (3D).
constexpr int kTri = 16;
constexpr int kTet = 32;
template <int DIM, int P>
using Shape = std::conditional_t<(P >= kTet), TetShape<P - kTet>,
                                 std::conditional_t<(P >= kTri), TriShape<P - kTri>, TensorShape<DIM, P>>>;

template <int P>
constexpr bool tri_tables_ok() {
    using S = TriShape<P>;
    for (int s = 0; s < S::NS; ++s)
        for (int b = 0; b < S::NF; ++b) {
            const int m = S::tn(s, b);
            if (m < 0 || m >= S::N || !S::on(m, s) || S::local(m, s) != b) return false;
        }
    for (int m = 0; m < S::N; ++m)
        for (int s = 0; s < S::NS; ++s)
            if (S::on(m, s) && S::tn(s, S::local(m, s)) != m) return false;
    return true;
}
static_assert(tri_tables_ok<1>() && tri_tables_ok<2>() && tri_tables_ok<3>(), "triangle slot tables");

template <int P>
constexpr bool tet_tables_ok() {
    using S = TetShape<P>;
    for (int s = 0; s < S::NS; ++s) {
        int on_count = 0;
        for (int m = 0; m < S::N; ++m) on_count += S::on(m, s) ? 1 : 0;
        if (on_count != S::NF) return false;
        for (int b = 0; b < S::NF; ++b) {
            const int m = S::tn(s, b);
            if (m < 0 || m >= S::N || !S::on(m, s) || S::local(m, s) != b) return false;
        }
    }
    return true;
}
static_assert(tet_tables_ok<1>() && tet_tables_ok<2>() && tet_tables_ok<3>(), "tetrahedron slot tables");

// Layout of one pair's cached A^{-1} block.  Column-major (entry (i, j) at
// j n + i), except for 3D p = 2 (n = 27): there columns 2c and 2c + 1 are
// interleaved row by row (entry (i, j) at 2 (c n + i) + (j & 1)), the odd
// last column follows plainly, and blocks are padded to an even length, so
// that a lane reads two entries of its row with one aligned 16-byte load
// (14 loads per row instead of 27).
template <int DIM, int P>
struct InvLayout {
    static constexpr int N = Shape<DIM, P>::N;
    static constexpr bool kPaired = DIM == 3 && P == 2;
    static constexpr int kStride = kPaired ? N * N + (N * N & 1) : N * N;
    __host__ __device__ static constexpr int at(int i, int j) {
        return !kPaired ? j * N + i : (j < (N & ~1) ? ((j >> 1) * N + i) * 2 + (j & 1) : (N & ~1) * N + i);
    }
};
typedef double dbl2 __attribute__((ext_vector_type(2)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// Layout of one pair's A^{-1} rounded to FP32 (mixed precision): groups of 4
// columns, entry (i, j) at ((j / 4) n + i) 4 + j mod 4, the last group padded,
// so that a lane reads four entries of its row with one 16-byte load.
template <int DIM, int P>
struct InvLayout32 {
    static constexpr int N = Shape<DIM, P>::N;
    static constexpr int kGroups = (N + 3) / 4;
    static constexpr int kStride = kGroups * N * 4;
    __host__ __device__ static constexpr int at(int i, int j) { return ((j >> 2) * N + i) * 4 + (j & 3); }
};
// FP32 inverses are kept for elements with at most this many nodes (their
// row of A^{-1} stays in registers); larger ones use the assembled path.
constexpr int kMaxInv32 = 32;

// Every block layout is a permutation of [0, n^2) inside its stride, and the
// paired columns sit at even offsets next to each other (16-byte loads).
template <int DIM, int P>
constexpr bool inv_layout_ok() {
    using IL = InvLayout<DIM, P>;
    constexpr int N = IL::N;
    bool seen[IL::kStride] = {};
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            const int k = IL::at(i, j);
            if (k < 0 || k >= IL::kStride || seen[k]) return false;
            seen[k] = true;
            if (IL::kPaired && j + 1 < (N & ~1) && !(j & 1) && (k % 2 != 0 || IL::at(i, j + 1) != k + 1))
                return false;
        }
    return IL::kStride % 2 == 0 || !IL::kPaired;
}
static_assert(inv_layout_ok<2, 1>() && inv_layout_ok<2, 2>() && inv_layout_ok<2, 3>() && inv_layout_ok<3, 1>() &&
                  inv_layout_ok<3, 2>() && inv_layout_ok<3, 3>() && inv_layout_ok<2, kTri + 1>() &&
                  inv_layout_ok<2, kTri + 2>() && inv_layout_ok<2, kTri + 3>() && inv_layout_ok<3, kTet + 1>() &&
                  inv_layout_ok<3, kTet + 2>() && inv_layout_ok<3, kTet + 3>(),
              "A^{-1} block layouts");

// Table entry and problem index read through the constant address space, so
// that a wavefront-uniform index gives scalar loads (neither is written while
// a sweep kernel runs).
// Table index of the problem owning schedule entry t: `fixed` when the
// schedule belongs to one problem (no load on the wavefront's critical path),
// else read from the entry.
__device__ __forceinline__ int batch_problem(const int4* pairs, int64_t t, int fixed) {
    typedef const __attribute__((address_space(4))) int* cint_ptr;
    return fixed >= 0 ? fixed : ((cint_ptr)(const int*)(pairs + t))[3];
}

__device__ __forceinline__ SweepArgs load_args(const SweepArgs* table, int k) {
    typedef const __attribute__((address_space(4))) SweepArgs* cargs_ptr;
    const cargs_ptr c = (cargs_ptr)(table + k);
    SweepArgs a;
    a.geo = c->geo;
    a.B = c->B;
    a.kink_tab = c->kink_tab;
    a.kink_idx = c->kink_idx;
    a.slot_face = c->slot_face;
    a.slot_nbr = c->slot_nbr;
    a.sigma_t = c->sigma_t;
    a.sigma_s = c->sigma_s;
    a.q = c->q;
    a.omega = c->omega;
    a.w = c->w;
    a.src = c->src;
    a.psi_cur = c->psi_cur;
    a.psi_prev = c->psi_prev;
    a.psi_inc = c->psi_inc;
    a.E = c->E;
    a.n = c->n;
    a.D = c->D;
    a.dim = c->dim;
    a.persistent = c->persistent;
    a.ainv = c->ainv;
    a.Bsym = c->Bsym;
    a.rhs_dir = c->rhs_dir;
    a.Nq = c->Nq;
    a.nbr_nodes = c->nbr_nodes;
    a.ainv32 = c->ainv32;
    return a;
}

// Node of the upwind neighbour that lies on the point of local node b of
// slot s of element e: on a lattice the opposite slot's node of the same
// local index; on an unstructured mesh read from the table (its faces meet
// in any orientation).
template <int DIM, int P, bool U>
__device__ __forceinline__ int up_node(const SweepArgs& args, int e, int s, int b) {
    using S = Shape<DIM, P>;
    static_assert(U || P < kTri, "triangles read the upwind node table");
    if constexpr (U) return args.nbr_nodes[((size_t)e * S::NS + s) * S::NF + b];
    else return S::tn(s ^ 1, b);
}

// Volume source of row `row` of pair (e, d): the direction-independent
// src = M (q + sigma_s phi / (4 pi)), plus the optional per-pair fixed term
// (direction-dependent source and tabulated boundary inflow, assembled at
// setup; null when the problem has neither).
__device__ __forceinline__ double source_row(const SweepArgs& args, int e, int d, int row, int N) {
    double v = args.src[(size_t)e * N + row];
    if (args.rhs_dir) v += args.rhs_dir[((size_t)d * args.E + e) * N + row];
    return v;
}

// Assembles row `row` of A and b for pair (e, d).  With DEFER, inflow through
// kept couplings (read from this sweep's flux) is left out of b and the slots
// that need it are returned in *kept; lagged and boundary inflow are added.
template <int DIM, int P, bool DEFER, bool KEEP_PIN = false, bool U = false>
__device__ __forceinline__ void assemble_row(const SweepArgs& args, int4 pr, int row, double (&a)[Shape<DIM, P>::N],
                                             double& rhs, unsigned& kept, int (&krow)[2 * DIM],
                                             double (*pk)[Shape<DIM, P>::NF] = nullptr) {
    using S = Shape<DIM, P>;
    constexpr int N = S::N, NF = S::NF, NS = S::NS;
    const int e = pr.x;
    const unsigned packed = (unsigned)pr.y;
    const int kb = pr.z;
    const int d = (int)(packed & kDirMask);
    const double* Ge = args.geo + (size_t)e * (DIM + 1) * N * N;
    const double st = args.sigma_t[e];
    const double o0 = args.omega[3 * d + 0], o1 = args.omega[3 * d + 1], o2 = args.omega[3 * d + 2];
    // large rows are assembled in chunks of 9 columns so that the loads in
    // flight do not dictate the register budget
    constexpr int CH = N > 16 ? 9 : N;
#pragma unroll
    for (int j0 = 0; j0 < N; j0 += CH) {
#pragma unroll
        for (int j = j0; j < j0 + CH && j < N; ++j) {
            double v = st * Ge[j * N + row];
            v -= o0 * Ge[1 * N * N + j * N + row];
            v -= o1 * Ge[2 * N * N + j * N + row];
            if (DIM == 3) v -= o2 * Ge[3 * N * N + j * N + row];
            a[j] = v;
        }
        if (N > 16) __builtin_amdgcn_sched_barrier(0);
    }
    rhs = source_row(args, e, d, row, N);
    kept = 0;
    int kc = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const unsigned cls = (packed >> (kSlotShift + 3 * s)) & 3u;
        const bool lagged = (packed >> (kSlotShift + 3 * s + 2)) & 1u;
        krow[s] = 0;
        if (cls == kKink) krow[s] = args.kink_idx[kb + kc++];
        if (cls == kNone) continue;
        const int nb = args.slot_nbr[(size_t)e * NS + s];
        const bool defer = DEFER && cls != kOut && nb >= 0 && !lagged;
        if (defer) kept |= 1u << s;
        const bool on = S::on(row, s);
        if (!on) continue;
        const int la = S::local(row, s);
        double pout[NF], pin[NF];
        if (cls == kKink) {
            // element is the face's minus side on odd slots: out = P_plus
            const double* T = args.kink_tab + (size_t)krow[s] * 2 * NF * NF;
            const double* To = T + ((s & 1) ? 0 : NF * NF);
            const double* Ti = T + ((s & 1) ? NF * NF : 0);
#pragma unroll
            for (int b = 0; b < NF; ++b) {
                pout[b] = To[la * NF + b];
                pin[b] = Ti[la * NF + b];
            }
        } else {
            const int f = args.slot_face[(size_t)e * NS + s];
            const double* Bf = args.B + (size_t)f * DIM * NF * NF + la * NF;
            const double sgn = (s & 1) ? 1.0 : -1.0;   // outward normal = sgn * N
#pragma unroll
            for (int b = 0; b < NF; ++b) {
                double v = o0 * Bf[b] + o1 * Bf[NF * NF + b];
                if (DIM == 3) v += o2 * Bf[2 * NF * NF + b];
                v *= sgn;                               // int (Omega . n_out) phi phi
                pout[b] = cls == kOut ? v : 0.0;
                pin[b] = cls == kOut ? 0.0 : -v;
            }
        }
#pragma unroll
        for (int b = 0; b < NF; ++b) a[S::tn(s, b)] += pout[b];
        if constexpr (KEEP_PIN) {
            if (defer) {
#pragma unroll
                for (int b = 0; b < NF; ++b) pk[s][b] = pin[b];
            }
        }
        if (cls != kOut && !defer) {
            if (nb >= 0) {
                const double* up = (lagged ? args.psi_prev : args.psi_cur) + ((size_t)d * args.E + nb) * N;
#pragma unroll
                for (int b = 0; b < NF; ++b) rhs += pin[b] * up[up_node<DIM, P, U>(args, e, s, b)];
            } else {
#pragma unroll
                for (int b = 0; b < NF; ++b) rhs += pin[b] * args.psi_inc;
            }
        }
    }
}

// Orders LDS traffic of one wavefront (no hardware barrier needed: a
// wavefront's LDS instructions execute in order).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One launch per level.  FP64: Gaussian elimination of [A | b] and back
// substitution, pivot rows broadcast through LDS.  MIXED: the assembled FP64
// row is rounded to FP32, factored A32 = L U in FP32, x0 = (LU)^{-1} b in
// FP32; then one correction with the FP64 operator, r = b - A x0 (FP64),
// x = x0 + (LU)^{-1} r.
template <int DIM, int P, bool MIXED, bool U = false>
__global__ void __launch_bounds__(64 * kLevelWaves) sweep_level_fp64(const SweepArgs* table, const int4* pairs,
                                                                 int64_t begin, int64_t count, int problem) {
    using S = Shape<DIM, P>;
    constexpr int N = S::N, G = S::G;
    __shared__ double lds[kLevelWaves][G][N + 1];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int grp = lane / N, row = lane - grp * N;
    const bool in_group = grp < G;
    // this wavefront's batch of G entries (one problem; count is a multiple of G)
    const int64_t wbase = begin + ((int64_t)blockIdx.x * kLevelWaves + wave) * G;
    if (wbase >= begin + count) return;   // LDS is per wavefront: no block barrier follows
    const SweepArgs args = load_args(table, batch_problem(pairs, wbase, problem));
    int4 pr = make_int4(-1, 0, 0, 0);
    if (in_group) pr = pairs[wbase + grp];
    const bool active = pr.x >= 0;    // padding entries have e = -1

    double a[N];
    double rhs = 0.0;
    int e = 0, d = 0;
    if (active) {
        e = pr.x;
        d = (int)((unsigned)pr.y & kDirMask);
        unsigned kept;
        int krow[2 * DIM];
        assemble_row<DIM, P, false, false, U>(args, pr, row, a, rhs, kept, krow);
    } else {
#pragma unroll
        for (int j = 0; j < N; ++j) a[j] = (j == row) ? 1.0 : 0.0;
    }

    double x = 0.0;
    if constexpr (!MIXED) {
        // Gaussian elimination, pivot row broadcast through LDS
#pragma unroll
        for (int k = 0; k < N; ++k) {
            if (in_group && row == k) {
#pragma unroll
                for (int j = k; j < N; ++j) lds[wave][grp][j] = a[j];
                lds[wave][grp][N] = rhs;
            }
            wave_sync();
            if (in_group && row > k) {
                const double l = a[k] / lds[wave][grp][k];
#pragma unroll
                for (int j = k + 1; j < N; ++j) a[j] -= l * lds[wave][grp][j];
                rhs -= l * lds[wave][grp][N];
            }
            wave_sync();
        }
        // back substitution
#pragma unroll
        for (int k = N - 1; k >= 0; --k) {
            if (in_group && row == k) {
                x = rhs / a[k];
                lds[wave][grp][0] = x;
            }
            wave_sync();
            if (in_group && row < k) rhs -= a[k] * lds[wave][grp][0];
            wave_sync();
        }
    } else {
        float* F = reinterpret_cast<float*>(&lds[wave][grp][0]);
        float f[N];
#pragma unroll
        for (int j = 0; j < N; ++j) f[j] = (float)a[j];
        // LU in FP32, multipliers below the diagonal
#pragma unroll
        for (int k = 0; k < N - 1; ++k) {
            if (in_group && row == k) {
#pragma unroll
                for (int j = k; j < N; ++j) F[j] = f[j];
            }
            wave_sync();
            if (in_group && row > k) {
                const float l = f[k] / F[k];
                f[k] = l;
#pragma unroll
                for (int j = k + 1; j < N; ++j) f[j] -= l * F[j];
            }
            wave_sync();
        }
        // solves (LU) y = c in FP32 for this lane's entry c of the column
        auto lu_solve = [&](float c) -> float {
#pragma unroll
            for (int k = 0; k < N - 1; ++k) {
                if (in_group && row == k) F[0] = c;
                wave_sync();
                if (in_group && row > k) c -= f[k] * F[0];
                wave_sync();
            }
            float y = 0.0f;
#pragma unroll
            for (int k = N - 1; k >= 0; --k) {
                if (in_group && row == k) {
                    y = c / f[k];
                    F[0] = y;
                }
                wave_sync();
                if (in_group && row < k) c -= f[k] * F[0];
                wave_sync();
            }
            return y;
        };
        const double x0 = (double)lu_solve((float)rhs);
        // r = b - A x0 with the FP64 row and x0 shared through LDS
        if (in_group) lds[wave][grp][row] = x0;
        wave_sync();
        double r = rhs;
#pragma unroll
        for (int j = 0; j < N; ++j) r -= a[j] * lds[wave][grp][j];
        wave_sync();
        x = x0 + (double)lu_solve((float)r);
    }
    if (active) args.psi_cur[((size_t)d * args.E + e) * N + row] = x;
}


// Striped tickets.  One global counter handing out one batch per atomic cost
// about 12 ns per batch (the atomics on one address serialise) and bounded
// the persistent sweeps.  Instead block b belongs to stream s = b mod
// kStreams and takes batches s, s + kStreams, s + 2 kStreams, ... in
// increasing order from the stream's own counter.  Deadlock-free: the
// smallest unfinished batch depends only on smaller (earlier-level) batches,
// which are finished; and it is either held by a wavefront of its stream
// (which processes its batches in increasing order) or not yet handed out,
// in which case every batch its stream has handed out is smaller, finished,
// and the stream's wavefronts go on to take it.  This needs a resident block
// in every stream: the grid is sized to what stays resident, and workgroups
// are dispatched in increasing id order, so blocks 0 .. S-1 start first.
// (Assigning streams in arrival order instead measured 5 % slower.)
#ifndef SNSW_STREAMS
#define SNSW_STREAMS 16
#endif
constexpr unsigned kStreams = SNSW_STREAMS;

static_assert(kStreams >= 1 && kStreams <= kMaxStreams, "stream count");

// Next batch index of this block's stream (one lane per wavefront).  A grid
// smaller than kStreams uses one stream per block, so that every stream has
// resident wavefronts.
__device__ __forceinline__ unsigned take_batch(unsigned* counters) {
    const unsigned S = gridDim.x < kStreams ? gridDim.x : kStreams;
    const unsigned s = blockIdx.x % S;
    return atomicAdd(counters + s * kTicketStride, 1u) * S + s;
}

// Bit pattern marking "not yet written in this sweep": a signalling NaN.
// Arithmetic never produces a signalling NaN (IEEE quiets them), so no
// computed flux can carry this pattern; only the fill kernel writes it.
constexpr unsigned long long kSentinel = 0x7FF4000000005EEDull;

// Persistent sweep with LDS broadcasts (groups of 8, 9, 27 or 64 lanes):
// each wavefront repeatedly claims G consecutive pairs of the level-ordered
// schedule, assembles A and b0 (lagged and boundary inflow included) and
// factors A = LU (no pivoting; multipliers kept below the diagonal) before
// it waits.  Then the lane on the first node of each kept face polls the
// upwind flux until it no longer holds this sweep's sentinel, the face lanes
// add their inflow rows P_in psi_up straight into b, and the two triangular
// solves finish the pair.  Fluxes are stored and polled with device-scope
// accesses (coherent across the XCD L2 caches).  Pairs are claimed in
// increasing schedule order, levels are padded to whole batches and every
// kept upwind pair sits on an earlier level, so each awaited pair belongs to
// another running wavefront (or to a ticket held by a wavefront that is
// finishing a smaller one): the waits end.  A wait that exceeds spin_limit
// polls sets *error and gives up (the result is then wrong but the kernel
// still terminates).
template <int DIM, int P, bool U = false>
__global__ void __launch_bounds__(64 * kWaves) sweep_persistent_fp64(PersistArgs pa) {
    using S = Shape<DIM, P>;
    constexpr int N = S::N, NF = S::NF, NS = S::NS, G = S::G;
    __shared__ double lds[kWaves][G][N + 1];   // odd stride: groups hit different banks
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane / N, row = lane - grp * N;
    const bool in_group = grp < G;
    const int g0 = in_group ? grp : 0;
    double* L = &lds[wave][g0][0];
    const unsigned long long sent = kSentinel;

    // The next batch is claimed while the current one is processed, which
    // hides the atomic's latency.
    unsigned t_next = 0;
    if (lane == 0) t_next = take_batch(pa.ticket) * (unsigned)G;
    t_next = __shfl(t_next, 0);
    while (true) {
        const unsigned t0 = __builtin_amdgcn_readfirstlane(t_next);
        if ((int64_t)t0 >= pa.total) break;
        unsigned t_pre = 0;
        if (lane == 0) t_pre = take_batch(pa.ticket) * (unsigned)G;
        const SweepArgs args = load_args(pa.table, batch_problem(pa.pairs, t0, pa.problem));
        const int64_t pidx = (int64_t)t0 + grp;
        int4 pr = make_int4(-1, 0, 0, 0);
        if (in_group && pidx < pa.total) pr = pa.pairs[pidx];
        const bool active = pr.x >= 0;    // padding entries have e = -1

        // Branch-free: padding lanes assemble element 0 with every face an
        // outflow face (packed = 0) and never publish (a divergent branch
        // here would keep two copies of the row alive).
        double a[N];
        double rhs = 0.0;
        unsigned kept = 0;
        int krow[2 * DIM];
        const int4 prs = active ? pr : make_int4(0, 0, 0, 0);
        assemble_row<DIM, P, true, false, U>(args, prs, row, a, rhs, kept, krow);
        const int e = prs.x;
        const unsigned packed = (unsigned)pr.y;
        const int d = (int)(packed & kDirMask);

        // LU factorisation; row `row` keeps its multipliers in a[0..row-1]
#pragma unroll
        for (int k = 0; k < N - 1; ++k) {
            if (in_group && row == k) {
#pragma unroll
                for (int j = k; j < N; ++j) L[j] = a[j];
            }
            wave_sync();
            if (in_group && row > k) {
                const double l = a[k] / L[k];
                a[k] = l;
#pragma unroll
                for (int j = k + 1; j < N; ++j) a[j] -= l * L[j];
            }
            wave_sync();
        }

        // wait: the lane on the first node of each kept face polls the
        // upwind value there; then every face lane reads its face's values
        bool need[NS];
        bool ok = true;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            need[s] = active && row == S::tn(s, 0) && ((kept >> s) & 1u);
            if (need[s]) ok = false;
        }
        int polls = 0;
        while (true) {
            if (!ok) {
                bool all = true;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (!need[s]) continue;
                    const int nb = args.slot_nbr[(size_t)e * NS + s];
                    double* ad = args.psi_cur + ((size_t)d * args.E + nb) * N + up_node<DIM, P, U>(args, e, s, 0);
                    const double val = __hip_atomic_load(ad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if ((unsigned long long)__double_as_longlong(val) == sent) all = false;
                    else need[s] = false;
                }
                ok = all;
            }
            if (__all(ok)) break;
            if (++polls > pa.spin_limit) {
                if (!ok) atomicExch(pa.error, 1);
                break;
            }
            if ((polls & 255) == 0) {
                // another wait already failed: stop waiting so the grid drains
                int err = 0;
                if (lane == 0) err = __hip_atomic_load(pa.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (__shfl(err, 0)) break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        // kept inflow straight into this lane's entry of b; values written
        // by other lanes of the upwind wavefront may lag the first node, so
        // any that still holds the sentinel is re-read (bounded likewise)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const bool on = S::on(row, s);
            if (!(active && on && ((kept >> s) & 1u))) continue;
            const int la = S::local(row, s);
            const unsigned cls = (packed >> (kSlotShift + 3 * s)) & 3u;
            const int nb = args.slot_nbr[(size_t)e * NS + s];
            double* up = args.psi_cur + ((size_t)d * args.E + nb) * N;
            const double* prow;
            double scale = 1.0;
            double o[3] = {args.omega[3 * d + 0], args.omega[3 * d + 1], args.omega[3 * d + 2]};
            if (cls == kKink) {
                prow = args.kink_tab + (size_t)krow[s] * 2 * NF * NF + ((s & 1) ? NF * NF : 0) + la * NF;
            } else {
                prow = args.B + (size_t)args.slot_face[(size_t)e * NS + s] * DIM * NF * NF + la * NF;
                scale = (s & 1) ? -1.0 : 1.0;   // P_in = -(outward) normal moments
            }
            double vals[NF];
#pragma unroll
            for (int b = 0; b < NF; ++b)
                vals[b] = __hip_atomic_load(up + up_node<DIM, P, U>(args, e, s, b), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
            for (int b = 0; b < NF; ++b) {
                for (int spin = 0;
                     (unsigned long long)__double_as_longlong(vals[b]) == sent && spin < pa.spin_limit; ++spin) {
                    __builtin_amdgcn_s_sleep(1);
                    vals[b] = __hip_atomic_load(up + up_node<DIM, P, U>(args, e, s, b), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                // a value still unwritten after the bound is a failed wait
                if ((unsigned long long)__double_as_longlong(vals[b]) == sent) atomicExch(pa.error, 1);
            }
#pragma unroll
            for (int b = 0; b < NF; ++b) {
                const double val = vals[b];
                double pv;
                if (cls == kKink) {
                    pv = prow[b];
                } else {
                    pv = o[0] * prow[b] + o[1] * prow[NF * NF + b];
                    if (DIM == 3) pv += o[2] * prow[2 * NF * NF + b];
                    pv *= scale;
                }
                rhs += pv * val;
            }
        }
        // forward substitution (unit lower), then back substitution
#pragma unroll
        for (int k = 0; k < N - 1; ++k) {
            if (in_group && row == k) L[0] = rhs;
            wave_sync();
            if (in_group && row > k) rhs -= a[k] * L[0];
            wave_sync();
        }
        double x = 0.0;
#pragma unroll
        for (int k = N - 1; k >= 0; --k) {
            if (in_group && row == k) {
                x = rhs / a[k];
                L[0] = x;
            }
            wave_sync();
            if (in_group && row < k) rhs -= a[k] * L[0];
            wave_sync();
        }
        // publish with device-scope (write-through) stores
        if (active)
            __hip_atomic_store(args.psi_cur + ((size_t)d * args.E + e) * N + row, x, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        t_next = __shfl(t_pre, 0);
    }
}

// Value of v on lane src of the wavefront (any lane; the source lane must be
// active).

// Component s (0..3) of an int4.
__device__ __forceinline__ int int4_get(const int4& v, int s) {
    return s == 0 ? v.x : s == 1 ? v.y : s == 2 ? v.z : v.w;
}

// A double in the global address space: loads through such pointers are
// global (not flat) memory instructions.
typedef __attribute__((address_space(1))) double gdouble;

__device__ __forceinline__ double lane_read(double v, int src) {
    const int addr = src << 2;
    const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Broadcast of lane K of each group of N lanes to the whole group, register
// to register: DPP row broadcast for 16-lane groups, quad permutation for
// 4-lane groups.
// Every lane has a valid source lane under both controls, so the old value
// is never used; the 16-lane form is one 64-bit DPP move (v_mov_b64_dpp).
template <int N, int K>
__device__ __forceinline__ double group_bcast(double x) {
    static_assert(N == 16 || N == 4, "DPP broadcast needs 4- or 16-lane groups");
    constexpr int ctrl = N == 16 ? 0x150 + K : (K | (K << 2) | (K << 4) | (K << 6));
    return __builtin_amdgcn_update_dpp(x, x, ctrl, 0xF, 0xF, true);
}

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Persistent sweep for 4- and 16-lane groups (2D, p = 1 and p = 3): the same
// schedule and protocol as sweep_persistent_fp64, with every intra-group
// exchange done by DPP broadcasts.  Register economy decides occupancy here:
// the assembly is branch-free, the inflow rows of the deferred slots are
// parked in LDS (each face lane writes its own row), the wait state is kept
// per axis, and after the wait the face lanes form c = P_in psi_up, which is
// broadcast into x += A^{-1}[:, tn_s] c.  NT: the rows of A^{-1} are read
// with non-temporal loads.  F32 (mixed precision): the cached A^{-1} is the
// FP32 copy, held in registers as FP32, with products and sums in FP64.
template <int DIM, int P, bool INV, bool NT = false, bool F32 = false>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(3, 8))) sweep_persistent_dpp(PersistArgs pa) {
    using S = Shape<DIM, P>;
    constexpr int N = S::N, NF = S::NF, NS = S::NS, G = S::G;
    static_assert(G * N == 64, "groups must tile the wavefront");
    static_assert(INV || !F32, "FP32 rows come from the cached inverses");
    __shared__ double pin_lds[kWaves][G][NS][NF][NF + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane / N, row = lane - grp * N;
    const unsigned long long sent = kSentinel;

    // The next batch is claimed while the current one is processed, which
    // hides the atomic's latency.  Deadlock-free: the smallest unfinished
    // ticket is always being processed (a held-but-unstarted ticket implies
    // a smaller unfinished one in progress), and its upwind pairs are in
    // smaller, finished tickets.
    unsigned t_next = 0;
    if (lane == 0) t_next = take_batch(pa.ticket) * (unsigned)G;
    t_next = __shfl(t_next, 0);
    while (true) {
        const unsigned t0 = __builtin_amdgcn_readfirstlane(t_next);
        if ((int64_t)t0 >= pa.total) break;
        unsigned t_pre = 0;
        if (lane == 0) t_pre = take_batch(pa.ticket) * (unsigned)G;
        const SweepArgs args = load_args(pa.table, batch_problem(pa.pairs, t0, pa.problem));
        const int64_t pidx = (int64_t)t0 + grp;
        int4 pr = make_int4(-1, 0, 0, 0);
        if (pidx < pa.total) pr = pa.pairs[pidx];
        // the entry's slot records, loaded together with the entry
        int4 rec[3] = {make_int4(0, 0, 0, 0), make_int4(0, 0, 0, 0), make_int4(0, 0, 0, 0)};
        if (pa.slots && pidx < pa.total) {
#pragma unroll
            for (int k = 0; k < 3; ++k) rec[k] = pa.slots[3 * pidx + k];
        }
        const bool active = pr.x >= 0;    // padding entries have e = -1
        const int e = active ? pr.x : 0;
        const unsigned packed = (unsigned)pr.y;
        const int d = (int)(packed & kDirMask);

        // ---- assembly of row `row`, branch-free: padding lanes assemble
        // element 0 and are masked (divergent branches here would keep two
        // copies of the row alive).
        std::conditional_t<F32, float, double> m[N];
        if constexpr (F32) {
            // row `row` of the FP32 copy, four entries per 16-byte load
            using IL32 = InvLayout32<DIM, P>;
            static_assert(IL32::kGroups * 4 == N, "whole groups of four columns");
            const float* Af = args.ainv32 + ((size_t)d * args.E + e) * IL32::kStride;
#pragma unroll
            for (int g = 0; g < IL32::kGroups; ++g) {
                const flt4* src = reinterpret_cast<const flt4*>(Af + IL32::at(row, 4 * g));
                const flt4 v = NT ? __builtin_nontemporal_load(src) : *src;
                m[4 * g] = v.x;
                m[4 * g + 1] = v.y;
                m[4 * g + 2] = v.z;
                m[4 * g + 3] = v.w;
            }
        } else if constexpr (INV) {
            // row `row` of the cached A^{-1} (stored column-major; a column
            // of n = 4 or 16 doubles lies in one 128 B line).  NT: read as
            // streaming (non-temporal) data, once per sweep, so that it does
            // not push the reused face data out of the caches
            static_assert(!InvLayout<DIM, P>::kPaired, "column-major blocks only");
            const double* Ai = args.ainv + ((size_t)d * args.E + e) * N * N + row;
            if constexpr (NT) {
#pragma unroll
                for (int j = 0; j < N; ++j) m[j] = __builtin_nontemporal_load(Ai + j * N);
            } else {
#pragma unroll
                for (int j = 0; j < N; ++j) m[j] = Ai[j * N];
            }
        } else {
            const double* Ge = args.geo + (size_t)e * (DIM + 1) * N * N + row;
            const double st = args.sigma_t[e];
            const double o0 = args.omega[3 * d + 0], o1 = args.omega[3 * d + 1];
#pragma unroll
            for (int j = 0; j < N; ++j) m[j] = st * Ge[j * N] - o0 * Ge[N * N + j * N] - o1 * Ge[2 * N * N + j * N];
        }
        // ---- faces.  All index loads first (one round trip together with
        // the volume loads), then all face data (a second one).
        int nbs[NS], fcs[NS], krows[NS];
        static_assert(NS == 4, "slot records hold four slots");
        if (pa.slots) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                nbs[s] = int4_get(rec[0], s);
                fcs[s] = int4_get(rec[1], s);
                krows[s] = active ? int4_get(rec[2], s) : 0;
            }
        } else {
            int kc = 0;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                nbs[s] = args.slot_nbr[(size_t)e * NS + s];
                fcs[s] = args.slot_face[(size_t)e * NS + s];
                const unsigned cls = (packed >> (kSlotShift + 3 * s)) & 3u;
                krows[s] = (active && cls == kKink) ? args.kink_idx[pr.z + kc] : 0;
                kc += (cls == kKink) ? 1 : 0;
            }
        }
        double rhs = source_row(args, e, d, row, N);
        unsigned kept = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const unsigned cls = active ? (packed >> (kSlotShift + 3 * s)) & 3u : kNone;
            const bool lagged = (packed >> (kSlotShift + 3 * s + 2)) & 1u;
            if (cls == kNone) continue;
            const int nb = nbs[s];
            const bool defer = cls != kOut && nb >= 0 && !lagged;
            if (defer) kept |= 1u << s;
            const bool on = S::on(row, s);
            if (!on) continue;
            const int la = S::local(row, s);
            double pout[NF], pin[NF];
            if (cls == kKink) {
                const double* T = args.kink_tab + (size_t)krows[s] * 2 * NF * NF;
                const double* To = T + ((s & 1) ? 0 : NF * NF);
                const double* Ti = T + ((s & 1) ? NF * NF : 0);
#pragma unroll
                for (int b = 0; b < NF; ++b) {
                    pout[b] = To[la * NF + b];
                    pin[b] = Ti[la * NF + b];
                }
            } else {
                const double* Bf = args.B + (size_t)fcs[s] * DIM * NF * NF + la * NF;
                const double o0 = args.omega[3 * d + 0], o1 = args.omega[3 * d + 1];
                const double sgn = (s & 1) ? 1.0 : -1.0;
#pragma unroll
                for (int b = 0; b < NF; ++b) {
                    const double vv = sgn * (o0 * Bf[b] + o1 * Bf[NF * NF + b]);
                    pout[b] = cls == kOut ? vv : 0.0;
                    pin[b] = cls == kOut ? 0.0 : -vv;
                }
            }
            if constexpr (!INV) {
#pragma unroll
                for (int b = 0; b < NF; ++b) m[S::tn(s, b)] += pout[b];
            }
            if (cls == kOut) continue;
            if (defer) {
#pragma unroll
                for (int b = 0; b < NF; ++b) pin_lds[wave][grp][s][la][b] = pin[b];
            } else if (nb >= 0) {
                const double* up = args.psi_prev + ((size_t)d * args.E + nb) * N;
#pragma unroll
                for (int b = 0; b < NF; ++b) rhs += pin[b] * up[S::tn(s ^ 1, b)];
            } else {
#pragma unroll
                for (int b = 0; b < NF; ++b) rhs += pin[b] * args.psi_inc;
            }
        }

        // ---- in-place Gauss-Jordan: m ends as row `row` of A^{-1}
        if constexpr (!INV) static_for<0, N>([&](auto kc2) {
            constexpr int k = decltype(kc2)::value;
            const bool piv = row == k;
            const double r = 1.0 / m[k];
            const double f = piv ? 0.0 : m[k];
#pragma unroll
            for (int j = 0; j < N; ++j) {
                if (j == k) m[j] = piv ? r : 0.0;
                else m[j] = piv ? m[j] * r : m[j];
            }
            static_for<0, N>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                m[j] -= f * group_bcast<N, k>(m[j]);
            });
        });
        // x0 = A^{-1} b0
        double x = 0.0;
        static_for<0, N>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            x += (double)m[j] * group_bcast<N, j>(rhs);
        });

        // ---- wait and finish: the lane on face-local node la of a kept slot
        // polls the upwind element's value at the matching node; each group
        // finishes its pair as soon as all of its values are there, so the
        // pairs of one wavefront do not wait for each other.
        // With a tiled schedule the groups of a wavefront are the pairs of
        // one tile of elements for one direction: a kept upwind pair in the
        // same tile (intra bit s) is read from its group's registers once
        // that group is done, not from memory.
        const unsigned intra = (active && pa.intra) ? (unsigned)pa.intra[pidx] : 0u;
        // Wait state per axis: in 2D a face lane lies on at most one face of
        // each axis (slot 2a or 2a + 1), so its polled value, address and
        // intra-tile source are kept per axis, not per slot.
        static_assert(DIM == 2, "per-axis wait state");
        const gdouble* addr[DIM];
        bool need[DIM];
        double own[DIM];
        int src_lane[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int ca = S::coord(row, a);
            const bool on = ca == 0 || ca == P;
            const int s = 2 * a + (ca == P ? 1 : 0);
            const bool internal = (intra >> s) & 1u;
            need[a] = active && on && ((kept >> s) & 1u) && !internal;
            addr[a] = (const gdouble*)args.psi_cur;
            own[a] = 0.0;
            src_lane[a] = lane;
            const int la = S::local(row, s);
            if (need[a]) {
                const int nb = ca == P ? nbs[2 * a + 1] : nbs[2 * a];
                addr[a] = (const gdouble*)(args.psi_cur + ((size_t)d * args.E + nb) * N + S::tn(s ^ 1, la));
            }
            if (internal && on) {
                const int g_up = (int)((intra >> (kIntraGroupShiftDev + 4 * s)) & 15u);
                src_lane[a] = g_up * N + S::tn(s ^ 1, la);
            }
        }
        constexpr unsigned long long gmask = N == 64 ? ~0ull : ((1ull << N) - 1ull);
        bool done = !active;
        int polls = 0;
        while (true) {
            // every face lane of a kept face polls its own upwind value, one
            // per axis, both loads issued before the first compare (one
            // round trip per poll; the polling traffic is small)
            double val[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a)
                val[a] = need[a] ? __hip_atomic_load(addr[a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0.0;
            bool have = true;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                if (need[a] && (unsigned long long)__double_as_longlong(val[a]) != sent) {
                    own[a] = val[a];
                    need[a] = false;
                }
                if (need[a]) have = false;
            }
            // Finish every ready group.  With a tiled schedule a finished
            // group can make groups of the same tile ready; they are finished
            // in further passes without new polls (at most G passes).
            for (int pass = 0; pass < G; ++pass) {
                const unsigned long long done_mask = __ballot(done);
                bool ready_lane = have;
                // intra-tile upwind values from the upwind group's lanes (all
                // lanes execute the permutes; only finished sources are used)
                double perm[DIM];
#pragma unroll
                for (int a = 0; a < DIM; ++a) perm[a] = pa.intra ? lane_read(x, src_lane[a]) : 0.0;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if ((intra >> s) & 1u) {
                        const int g_up = (int)((intra >> (kIntraGroupShiftDev + 4 * s)) & 15u);
                        if (!((done_mask >> (g_up * N)) & 1ull)) ready_lane = false;
                    }
                }
                const unsigned long long ready = __ballot(ready_lane);
                const bool gready = ((ready >> (grp * N)) & gmask) == gmask;
                const bool fin = gready && !done;
                if (fin) {
                    // c_s[la] = sum_b P_in,s[la][b] psi_up,s[b] on the face
                    // lanes (psi_up,s[b] sits on lane tn_s(b)); then
                    // x += sum_a A^{-1}[row][tn_s(a)] c_s[a].  The whole group
                    // takes this branch together, so the DPP sources are active.
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    static_for<0, NS>([&](auto sc) {
                        constexpr int s = decltype(sc)::value;
                        constexpr int a = s / 2;
                        const bool on = S::coord(row, a) == ((s & 1) ? P : 0);
                        if (((intra >> s) & 1u) && on) own[a] = perm[a];
                        if ((kept >> s) & 1u) {
                            const int la = on ? S::local(row, s) : 0;
                            double c = 0.0;
                            static_for<0, NF>([&](auto bc) {
                                constexpr int b = decltype(bc)::value;
                                c += pin_lds[wave][grp][s][la][b] * group_bcast<N, S::tn(s, b)>(own[a]);
                            });
                            static_for<0, NF>([&](auto ac) {
                                constexpr int aa = decltype(ac)::value;
                                x += (double)m[S::tn(s, aa)] * group_bcast<N, S::tn(s, aa)>(c);
                            });
                        }
                    });
                    __hip_atomic_store(args.psi_cur + ((size_t)d * args.E + e) * N + row, x, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    done = true;
                }
                if (!pa.intra || !__any(fin) || __all(done)) break;
            }
            if (__all(done)) break;
            if (++polls > pa.spin_limit) {
                atomicExch(pa.error, 1);
                break;
            }
            if ((polls & 255) == 0) {
                // another wait already failed: stop waiting so the grid drains
                int err = 0;
                if (lane == 0) err = __hip_atomic_load(pa.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (__shfl(err, 0)) break;
            }
            __builtin_amdgcn_s_sleep(SNSW_POLL_SLEEP);
        }
        t_next = __shfl(t_pre, 0);
    }
}


// Persistent sweep with cached inverses for 2D groups that DPP cannot
// broadcast within (p = 2, n = 9 lanes): the protocol of
// sweep_persistent_dpp with LDS exchanges.  Before the wait each face lane
// parks its inflow row P_in,s[la] of every kept slot in LDS and the lagged
// and boundary inflow go into b; every face lane of a kept face then polls
// all nf upwind values of the face (all loads of a poll issued together),
// and each group finishes as soon as its lanes hold them: b += P_in psi_up
// on the face lanes, b through LDS, x = A^{-1} b, device-scope store.  The
// groups of a wavefront do not wait for each other.  F32 (mixed precision):
// the FP32 copy of A^{-1}, FP64 products and sums.
template <int P, bool F32 = false>
__global__ void __launch_bounds__(64 * kWaves) sweep_persistent_lds2d(PersistArgs pa) {
    constexpr int DIM = 2;
    using S = Shape<DIM, P>;
    constexpr int N = S::N, NF = S::NF, NS = S::NS, G = S::G;
    __shared__ double lds[kWaves][G][N + 1];
    __shared__ double pin_lds[kWaves][G][NS][NF][NF + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane / N, row = lane - grp * N;
    const bool in_group = grp < G;
    const int g0 = in_group ? grp : 0;
    double* L = &lds[wave][g0][0];
    const unsigned long long sent = kSentinel;
    constexpr unsigned long long gmask = (1ull << N) - 1ull;

    unsigned t_next = 0;
    if (lane == 0) t_next = take_batch(pa.ticket) * (unsigned)G;
    t_next = __shfl(t_next, 0);
    while (true) {
        const unsigned t0 = __builtin_amdgcn_readfirstlane(t_next);
        if ((int64_t)t0 >= pa.total) break;
        unsigned t_pre = 0;
        if (lane == 0) t_pre = take_batch(pa.ticket) * (unsigned)G;
        const SweepArgs args = load_args(pa.table, batch_problem(pa.pairs, t0, pa.problem));
        const int64_t pidx = (int64_t)t0 + grp;
        int4 pr = make_int4(-1, 0, 0, 0);
        if (in_group && pidx < pa.total) pr = pa.pairs[pidx];
        const bool active = pr.x >= 0;    // padding entries have e = -1
        const int4 prs = active ? pr : make_int4(0, 0, 0, 0);
        const int e = prs.x;
        const unsigned packed = (unsigned)prs.y;
        const int d = (int)(packed & kDirMask);
        static_assert(!InvLayout<DIM, P>::kPaired, "column-major blocks only");
        using IL32 = InvLayout32<DIM, P>;
        std::conditional_t<F32, float, double> m[F32 ? IL32::kGroups * 4 : N];
        if constexpr (F32) {
            // four entries of the FP32 row per 16-byte load
            const float* Af = args.ainv32 + ((size_t)d * args.E + e) * IL32::kStride;
#pragma unroll
            for (int g = 0; g < IL32::kGroups; ++g) {
                const flt4 v = *reinterpret_cast<const flt4*>(Af + IL32::at(row, 4 * g));
                m[4 * g] = v.x;
                m[4 * g + 1] = v.y;
                m[4 * g + 2] = v.z;
                m[4 * g + 3] = v.w;
            }
        } else {
            const double* Ai = args.ainv + ((size_t)d * args.E + e) * N * N + row;
#pragma unroll
            for (int j = 0; j < N; ++j) m[j] = Ai[j * N];
        }

        // ---- faces: index loads first, then face data
        int nbs[NS], fcs[NS], krows[NS];
        {
            int kc = 0;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                nbs[s] = args.slot_nbr[(size_t)e * NS + s];
                fcs[s] = args.slot_face[(size_t)e * NS + s];
                const unsigned cls = (packed >> (kSlotShift + 3 * s)) & 3u;
                krows[s] = (active && cls == kKink) ? args.kink_idx[prs.z + kc] : 0;
                kc += (cls == kKink) ? 1 : 0;
            }
        }
        double rhs = source_row(args, e, d, row, N);
        const double o0 = args.omega[3 * d + 0], o1 = args.omega[3 * d + 1];
        unsigned kept = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const unsigned cls = active ? (packed >> (kSlotShift + 3 * s)) & 3u : kNone;
            const bool lagged = (packed >> (kSlotShift + 3 * s + 2)) & 1u;
            if (cls == kNone || cls == kOut) continue;
            const int nb = nbs[s];
            const bool defer = nb >= 0 && !lagged;
            if (defer) kept |= 1u << s;
            const bool on = S::on(row, s);
            if (!on) continue;
            const int la = S::local(row, s);
            double pin[NF];
            if (cls == kKink) {
                const double* Ti = args.kink_tab + (size_t)krows[s] * 2 * NF * NF + ((s & 1) ? NF * NF : 0) + la * NF;
#pragma unroll
                for (int b = 0; b < NF; ++b) pin[b] = Ti[b];
            } else {
                const double* Bf = args.B + (size_t)fcs[s] * DIM * NF * NF + la * NF;
                const double sgn = (s & 1) ? -1.0 : 1.0;   // P_in = -(outward normal) moments
#pragma unroll
                for (int b = 0; b < NF; ++b) pin[b] = sgn * (o0 * Bf[b] + o1 * Bf[NF * NF + b]);
            }
            if (defer) {
#pragma unroll
                for (int b = 0; b < NF; ++b) pin_lds[wave][grp][s][la][b] = pin[b];
            } else if (nb >= 0) {
                const double* up = args.psi_prev + ((size_t)d * args.E + nb) * N;
#pragma unroll
                for (int b = 0; b < NF; ++b) rhs += pin[b] * up[S::tn(s ^ 1, b)];
            } else {
#pragma unroll
                for (int b = 0; b < NF; ++b) rhs += pin[b] * args.psi_inc;
            }
        }

        // ---- wait and finish
        const gdouble* up[NS];
        bool need[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const bool on = S::on(row, s);
            need[s] = active && on && ((kept >> s) & 1u);
            up[s] = (const gdouble*)(args.psi_cur + ((size_t)d * args.E + (need[s] ? nbs[s] : 0)) * N);
        }
        double vals[NS][NF];
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int b = 0; b < NF; ++b) vals[s][b] = 0.0;
        bool done = !active;
        int polls = 0;
        while (true) {
            double v[NS][NF];
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int b = 0; b < NF; ++b)
                    v[s][b] = need[s] ? __hip_atomic_load(up[s] + S::tn(s ^ 1, b), __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT)
                                      : 0.0;
            bool have = true;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (!need[s]) continue;
                bool all = true;
#pragma unroll
                for (int b = 0; b < NF; ++b) all = all && (unsigned long long)__double_as_longlong(v[s][b]) != sent;
                if (all) {
#pragma unroll
                    for (int b = 0; b < NF; ++b) vals[s][b] = v[s][b];
                    need[s] = false;
                } else {
                    have = false;
                }
            }
            const unsigned long long ready = __ballot(have);
            const bool fin = in_group && !done && ((ready >> (grp * N)) & gmask) == gmask;
            if (fin) {
                // the whole group takes this branch together
                double b = rhs;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const bool on = S::on(row, s);
                    if (!(on && ((kept >> s) & 1u))) continue;
                    const int la = S::local(row, s);
#pragma unroll
                    for (int bb = 0; bb < NF; ++bb) b += pin_lds[wave][grp][s][la][bb] * vals[s][bb];
                }
                L[row] = b;
                wave_sync();
                double x = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) x += (double)m[j] * L[j];
                __hip_atomic_store(args.psi_cur + ((size_t)d * args.E + e) * N + row, x, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                done = true;
            }
            if (__all(done)) break;
            if (++polls > pa.spin_limit) {
                atomicExch(pa.error, 1);
                break;
            }
            if ((polls & 255) == 0) {
                // another wait already failed: stop waiting so the grid drains
                int err = 0;
                if (lane == 0) err = __hip_atomic_load(pa.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (__shfl(err, 0)) break;
            }
            __builtin_amdgcn_s_sleep(SNSW_POLL_SLEEP);
        }
        t_next = __shfl(t_pre, 0);
    }
}


// ---- cached element inverses ------------------------------------------
//
// The element operator A = sigma_t M - sum_i Omega_i K_i + outflow blocks of
// a pair does not change between source iterations, so it can be inverted
// once and kept in HBM; a sweep then only assembles b and forms A^{-1} b.

// Setup: for schedule entries [0, count) of one problem, assemble A and
// invert it in place by Gauss-Jordan without pivoting (A + A^T is positive
// definite), pivot rows broadcast through LDS; A^{-1} is stored at
// ainv[(d E + e) stride + InvLayout::at(i, j)].
template <int DIM, int P, bool U = false, bool F32 = false>
__global__ void __launch_bounds__(64 * kWaves) factor_kernel(const SweepArgs* table, const int4* pairs, int64_t count,
                                                            void* ainv) {
    using S = Shape<DIM, P>;
    constexpr int N = S::N, G = S::G;
    __shared__ double lds[kWaves][G][N + 1];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int grp = lane / N, row = lane - grp * N;
    const bool in_group = grp < G;
    const int64_t wbase = ((int64_t)blockIdx.x * kWaves + wave) * G;
    if (wbase >= count) return;   // LDS is per wavefront: no block barrier follows
    const SweepArgs args = load_args(table, batch_problem(pairs, wbase, -1));
    int4 pr = make_int4(-1, 0, 0, 0);
    if (in_group) pr = pairs[wbase + grp];
    const bool active = pr.x >= 0;
    const int4 prs = active ? pr : make_int4(0, 0, 0, 0);
    double m[N];
    double rhs;
    unsigned kept;
    int krow[2 * DIM];
    assemble_row<DIM, P, true, false, U>(args, prs, row, m, rhs, kept, krow);
    double* L = &lds[wave][in_group ? grp : 0][0];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        if (in_group && row == k) {
            const double r = 1.0 / m[k];
#pragma unroll
            for (int j = 0; j < N; ++j) L[j] = (j == k) ? r : m[j] * r;
        }
        wave_sync();
        if (in_group) {
            if (row == k) {
#pragma unroll
                for (int j = 0; j < N; ++j) m[j] = L[j];
            } else {
                const double f = m[k];
                m[k] = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) m[j] -= f * L[j];
            }
        }
        wave_sync();
    }
    if (active) {
        const int d = (int)((unsigned)pr.y & kDirMask);
        if constexpr (F32) {
            using IL = InvLayout32<DIM, P>;
            float* dst = static_cast<float*>(ainv) + ((size_t)d * args.E + pr.x) * IL::kStride;
#pragma unroll
            for (int j = 0; j < N; ++j) dst[IL::at(row, j)] = (float)m[j];
        } else {
            using IL = InvLayout<DIM, P>;
            double* dst = static_cast<double*>(ainv) + ((size_t)d * args.E + pr.x) * IL::kStride;
#pragma unroll
            for (int j = 0; j < N; ++j) dst[IL::at(row, j)] = m[j];
        }
    }
}

// b of row `row` of pair pr: source plus every inflow term (kept couplings
// read this sweep's flux, lagged ones the previous sweep's, boundary faces
// psi_inc).
template <int DIM, int P, bool DEFER = false, bool U = false>
__device__ __forceinline__ double inflow_rhs(const SweepArgs& args, int4 pr, int row, unsigned* kept_out = nullptr) {
    using S = Shape<DIM, P>;
    constexpr int N = S::N, NF = S::NF, NS = S::NS;
    const int e = pr.x;
    const unsigned packed = (unsigned)pr.y;
    const int d = (int)(packed & kDirMask);
    double rhs = source_row(args, e, d, row, N);
    const double o0 = args.omega[3 * d + 0], o1 = args.omega[3 * d + 1], o2 = args.omega[3 * d + 2];
    int kc = 0;
    unsigned kept = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const unsigned cls = (packed >> (kSlotShift + 3 * s)) & 3u;
        const bool lagged = (packed >> (kSlotShift + 3 * s + 2)) & 1u;
        int kr = 0;
        if (cls == kKink) kr = args.kink_idx[pr.z + kc++];
        if (cls == kOut || cls == kNone) continue;
        if (DEFER && !lagged && args.slot_nbr[(size_t)e * NS + s] >= 0) {
            kept |= 1u << s;   // read from this sweep's flux after the wait
            continue;
        }
        const bool on = S::on(row, s);
        if (!on) continue;
        const int la = S::local(row, s);
        double pin[NF];
        if (cls == kKink) {
            const double* Ti = args.kink_tab + (size_t)kr * 2 * NF * NF + ((s & 1) ? NF * NF : 0) + la * NF;
#pragma unroll
            for (int b = 0; b < NF; ++b) pin[b] = Ti[b];
        } else {
            const double* Bf = args.B + (size_t)args.slot_face[(size_t)e * NS + s] * DIM * NF * NF + la * NF;
            const double sgn = (s & 1) ? -1.0 : 1.0;   // P_in = -(outward normal) moments
#pragma unroll
            for (int b = 0; b < NF; ++b) {
                double v = o0 * Bf[b] + o1 * Bf[NF * NF + b];
                if (DIM == 3) v += o2 * Bf[2 * NF * NF + b];
                pin[b] = sgn * v;
            }
        }
        const int nb = args.slot_nbr[(size_t)e * NS + s];
        if (nb >= 0) {
            const double* up = (lagged ? args.psi_prev : args.psi_cur) + ((size_t)d * args.E + nb) * N;
#pragma unroll
            for (int b = 0; b < NF; ++b) rhs += pin[b] * up[up_node<DIM, P, U>(args, e, s, b)];
        } else {
#pragma unroll
            for (int b = 0; b < NF; ++b) rhs += pin[b] * args.psi_inc;
        }
    }
    if (kept_out) *kept_out = kept;
    return rhs;
}

// Inflow of one pair assembled cooperatively (3D, n >= dim * nf): lane
// (a, la) = (row / nf, row mod nf) contracts component a of the face moments
// with the upwind trace, t = sum_b B_a[la][b] psi_up[b], so each lane loads
// nf contiguous moments instead of a face lane loading dim * nf of them; the
// dim partial sums of face-local row la meet in LDS (cf, [NS][dim * nf] per
// pair) and are added to the rows on the face.  Same sums as inflow_rhs up to
// their order.
template <int DIM, int P, bool U = false>
__device__ __forceinline__ double inflow_rhs_coop(const SweepArgs& args, int4 pr, int row, bool in_group,
                                                  double (*cf)[DIM * Shape<DIM, P>::NF]) {
    using S = Shape<DIM, P>;
    constexpr int N = S::N, NF = S::NF, NS = S::NS;
    static_assert(DIM * NF <= N, "one lane per moment row and component");
    const int e = pr.x;
    const unsigned packed = (unsigned)pr.y;
    const int d = (int)(packed & kDirMask);
    const int a = row / NF, la = row - a * NF;
    const bool worker = in_group && a < DIM;
    const double oa = args.omega[3 * d + (a < DIM ? a : 0)];
    int kc = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const unsigned cls = (packed >> (kSlotShift + 3 * s)) & 3u;
        const bool lagged = (packed >> (kSlotShift + 3 * s + 2)) & 1u;
        int kr = 0;
        if (cls == kKink) kr = args.kink_idx[pr.z + kc++];
        if (cls == kOut || cls == kNone || !worker) continue;
        const int nb = args.slot_nbr[(size_t)e * NS + s];
        const double* up = (lagged ? args.psi_prev : args.psi_cur) + ((size_t)d * args.E + (nb >= 0 ? nb : 0)) * N;
        double t = 0.0;
        if (cls == kKink) {
            // the tabulated inflow block is the whole moment: component 0 only
            if (a == 0) {
                const double* Ti = args.kink_tab + (size_t)kr * 2 * NF * NF + ((s & 1) ? NF * NF : 0) + la * NF;
#pragma unroll
                for (int b = 0; b < NF; ++b) t += Ti[b] * (nb >= 0 ? up[up_node<DIM, P, U>(args, e, s, b)] : args.psi_inc);
            }
        } else {
            const int fc = args.slot_face[(size_t)e * NS + s];
            if (args.Bsym) {
                // row la of the symmetric moment matrix from its packed upper
                // triangle (44 % fewer bytes than the full matrix)
                constexpr int NT = NF * (NF + 1) / 2;
                const double* Bs = args.Bsym + (size_t)(fc * bsym_face_stride(NF) + a * NT);
#pragma unroll
                for (int b = 0; b < NF; ++b) {
                    const int i = la < b ? la : b, j = la < b ? b : la;
                    t += Bs[i * NF - (i * (i - 1)) / 2 + (j - i)] *
                         (nb >= 0 ? up[up_node<DIM, P, U>(args, e, s, b)] : args.psi_inc);
                }
            } else {
                const double* Bf = args.B + ((size_t)fc * DIM + a) * NF * NF + la * NF;
#pragma unroll
                for (int b = 0; b < NF; ++b) t += Bf[b] * (nb >= 0 ? up[up_node<DIM, P, U>(args, e, s, b)] : args.psi_inc);
            }
            t *= (s & 1) ? -oa : oa;   // P_in = -(outward normal) moments
        }
        cf[s][row] = t;
    }
    wave_sync();
    double rhs = in_group ? source_row(args, e, d, row, N) : 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const unsigned cls = (packed >> (kSlotShift + 3 * s)) & 3u;
        if (cls == kOut || cls == kNone) continue;
        if (!S::on(row, s)) continue;
        const int l = S::local(row, s);
#pragma unroll
        for (int c = 0; c < DIM; ++c) rhs += cf[s][c * NF + l];
    }
    return rhs;
}

// inflow_rhs_coop with the upwind traces staged: first the lanes of component
// 0 park the trace of each inflow slot in LDS (uf, [NS][nf] per pair), one
// load per face lane instead of nf broadcast loads in every lane (p = 2: 24
// fewer vector memory instructions per wavefront of two pairs, about a tenth
// of the 3D level sweep); then the contraction reads the trace from LDS.  The
// same sums in the same order as inflow_rhs_coop.  Not used for nf = 16,
// where holding the staged slots costs more registers than it saves.
template <int DIM, int P, bool U = false>
__device__ __forceinline__ double inflow_rhs_staged(const SweepArgs& args, int4 pr, int row, bool in_group,
                                                  double (*cf)[DIM * Shape<DIM, P>::NF],
                                                  double (*uf)[Shape<DIM, P>::NF]) {
    using S = Shape<DIM, P>;
    constexpr int N = S::N, NF = S::NF, NS = S::NS;
    static_assert(DIM * NF <= N, "one lane per moment row and component");
    const int e = pr.x;
    const unsigned packed = (unsigned)pr.y;
    const int d = (int)(packed & kDirMask);
    const int a = row / NF, la = row - a * NF;
    const bool worker = in_group && a < DIM;
    const double oa = args.omega[3 * d + (a < DIM ? a : 0)];
    int fcs[NS], krs[NS];
    int kc = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const unsigned cls = (packed >> (kSlotShift + 3 * s)) & 3u;
        const bool lagged = (packed >> (kSlotShift + 3 * s + 2)) & 1u;
        krs[s] = 0;
        fcs[s] = 0;
        if (cls == kKink) krs[s] = args.kink_idx[pr.z + kc++];
        if (cls == kOut || cls == kNone || !worker) continue;
        if (cls != kKink) fcs[s] = args.slot_face[(size_t)e * NS + s];
        if (a == 0) {
            const int nb = args.slot_nbr[(size_t)e * NS + s];
            const double* up = (lagged ? args.psi_prev : args.psi_cur) + ((size_t)d * args.E + (nb >= 0 ? nb : 0)) * N;
            uf[s][la] = nb >= 0 ? up[up_node<DIM, P, U>(args, e, s, la)] : args.psi_inc;
        }
    }
    wave_sync();
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const unsigned cls = (packed >> (kSlotShift + 3 * s)) & 3u;
        if (cls == kOut || cls == kNone || !worker) continue;
        double t = 0.0;
        if (cls == kKink) {
            if (a == 0) {
                const double* Ti = args.kink_tab + (size_t)krs[s] * 2 * NF * NF + ((s & 1) ? NF * NF : 0) + la * NF;
#pragma unroll
                for (int b = 0; b < NF; ++b) t += Ti[b] * uf[s][b];
            }
        } else {
            if (args.Bsym) {
                constexpr int NT = NF * (NF + 1) / 2;
                const double* Bs = args.Bsym + (size_t)(fcs[s] * bsym_face_stride(NF) + a * NT);
#pragma unroll
                for (int b = 0; b < NF; ++b) {
                    const int i = la < b ? la : b, j = la < b ? b : la;
                    t += Bs[i * NF - (i * (i - 1)) / 2 + (j - i)] * uf[s][b];
                }
            } else {
                const double* Bf = args.B + ((size_t)fcs[s] * DIM + a) * NF * NF + la * NF;
#pragma unroll
                for (int b = 0; b < NF; ++b) t += Bf[b] * uf[s][b];
            }
            t *= (s & 1) ? -oa : oa;
        }
        cf[s][row] = t;
    }
    wave_sync();
    double rhs = in_group ? source_row(args, e, d, row, N) : 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const unsigned cls = (packed >> (kSlotShift + 3 * s)) & 3u;
        if (cls == kOut || cls == kNone) continue;
        if (!S::on(row, s)) continue;
        const int l = S::local(row, s);
#pragma unroll
        for (int c = 0; c < DIM; ++c) rhs += cf[s][c * NF + l];
    }
    return rhs;
}

// Inflow of one pair through the face normals at Gauss points (3D lattices,
// p = 2, faces with 4 x 4 Gauss points: SweepArgs::Nq).  The inflow block of
// an inflow slot applied to the upwind trace u is
//   (P_in u)_i = -sgn sum_q phi_i(q) (Omega . w_q N(q)) u(q),  u(q) = sum_b phi_b(q) u_b,
// the same sums as the moments B_a = sum_q w_q N_a(q) phi_i(q) phi_j(q) (the
// rule is exact for them) in another order, reading 48 doubles per face
// instead of 135 packed moments.  Traces staged in LDS as in
// inflow_rhs_staged; lanes 0..15 of a pair form the point values
// t_q = (Omega . w_q N(q)) u(q) of each inflow face in cf[s][q], then every
// row sums phi_l(q) t_q over the faces it lies on.  phi at the points is the
// product of the 1D Lagrange polynomials of the Gauss-Lobatto nodes
// {0, 1/2, 1} at the 4 Gauss points.
__device__ __forceinline__ void lagrange3(double x, double* l) {
    l[0] = 2.0 * (x - 0.5) * (x - 1.0);
    l[1] = -4.0 * x * (x - 1.0);
    l[2] = 2.0 * x * (x - 0.5);
}
// the i-th of them at x (i in 0..2, not known at compile time)
__device__ __forceinline__ double lagrange3_at(int i, double x) {
    return i == 0 ? 2.0 * (x - 0.5) * (x - 1.0) : (i == 1 ? -4.0 * x * (x - 1.0) : 2.0 * x * (x - 0.5));
}
// The k-th point of the 4-point Gauss-Legendre rule on [0, 1], ascending
// (1/2 -+ x/2 with x^2 = 3/7 +- (2/7) sqrt(6/5)); a select, not a table, so
// that a runtime k costs no memory access.
__device__ __forceinline__ double gauss4(int k) {
    constexpr double a = 0.86113631159405257522, b = 0.33998104358485626480;
    return k == 0 ? 0.5 - 0.5 * a : (k == 1 ? 0.5 - 0.5 * b : (k == 2 ? 0.5 + 0.5 * b : 0.5 + 0.5 * a));
}

template <int DIM, int P>
__device__ __forceinline__ double inflow_rhs_quad(const SweepArgs& args, int4 pr, int row, bool in_group,
                                                 double (*cf)[DIM * Shape<DIM, P>::NF],
                                                 double (*uf)[Shape<DIM, P>::NF]) {
    using S = Shape<DIM, P>;
    constexpr int NF = S::NF, NS = S::NS;
    static_assert(DIM == 3 && P == 2 && NF == 9, "3D p = 2 lattices");
    const int e = pr.x;
    const unsigned packed = (unsigned)pr.y;
    const int d = (int)(packed & kDirMask);
    const int a = row / NF, la = row - a * NF;
    const bool worker = in_group && a < DIM;
    const double o0 = args.omega[3 * d], o1 = args.omega[3 * d + 1], o2 = args.omega[3 * d + 2];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const unsigned cls = (packed >> (kSlotShift + 3 * s)) & 3u;
        const bool lagged = (packed >> (kSlotShift + 3 * s + 2)) & 1u;
        if (cls == kOut || cls == kNone || !worker) continue;
        if (a == 0) {
            const int nb = args.slot_nbr[(size_t)e * NS + s];
            const double* up = (lagged ? args.psi_prev : args.psi_cur) + ((size_t)d * args.E + (nb >= 0 ? nb : 0)) * S::N;
            uf[s][la] = nb >= 0 ? up[S::tn(s ^ 1, la)] : args.psi_inc;
        }
    }
    wave_sync();
    // point values t_q (lanes row < 16) and kink contractions (lanes a == 0)
    const int q0 = row & 3, q1 = (row >> 2) & 3;
    int kc = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const unsigned cls = (packed >> (kSlotShift + 3 * s)) & 3u;
        int kr = 0;
        if (cls == kKink) kr = args.kink_idx[pr.z + kc++];
        if (cls == kOut || cls == kNone || !worker) continue;
        if (cls == kKink) {
            if (a == 0) {
                const double* Ti = args.kink_tab + (size_t)kr * 2 * NF * NF + ((s & 1) ? NF * NF : 0) + la * NF;
                double t = 0.0;
#pragma unroll
                for (int b = 0; b < NF; ++b) t += Ti[b] * uf[s][b];
                cf[s][la] = t;
            }
        } else if (row < 16) {
            // phi_b at this lane's point (recomputed per face: fewer live registers)
            double lq0[3], lq1[3];
            lagrange3(gauss4(q0), lq0);
            lagrange3(gauss4(q1), lq1);
            double u = 0.0;
#pragma unroll
            for (int b1 = 0; b1 < 3; ++b1) {
                double v = 0.0;
#pragma unroll
                for (int b0 = 0; b0 < 3; ++b0) v += lq0[b0] * uf[s][b1 * 3 + b0];
                u += lq1[b1] * v;
            }
            const double* wn = args.Nq + ((size_t)args.slot_face[(size_t)e * NS + s] * 16 + row) * 3;
            cf[s][row] = (o0 * wn[0] + o1 * wn[1] + o2 * wn[2]) * u;
        }
    }
    wave_sync();
    double rhs = in_group ? source_row(args, e, d, row, S::N) : 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const unsigned cls = (packed >> (kSlotShift + 3 * s)) & 3u;
        if (cls == kOut || cls == kNone) continue;
        if (!S::on(row, s)) continue;
        const int l = S::local(row, s);
        if (cls == kKink) {
            rhs += cf[s][l];
            continue;
        }
        const int i0 = l % 3, i1 = l / 3;
        double e0[4], c = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) e0[j] = lagrange3_at(i0, gauss4(j));
#pragma unroll
        for (int j1 = 0; j1 < 4; ++j1) {
            double v = 0.0;
#pragma unroll
            for (int j0 = 0; j0 < 4; ++j0) v += e0[j0] * cf[s][j1 * 4 + j0];
            c += lagrange3_at(i1, gauss4(j1)) * v;
        }
        rhs += (s & 1) ? -c : c;   // P_in = -(outward normal) moments
    }
    return rhs;
}

// One launch per level with cached inverses: b assembled per row, shared
// through the wavefront's LDS, x = A^{-1} b.
template <int DIM, int P, bool U = false, bool F32 = false, bool QUAD = false>
__global__ void __launch_bounds__(64 * kLevelWaves) sweep_level_inv(const SweepArgs* table, const int4* pairs,
                                                              int64_t begin, int64_t count, int problem) {
    using S = Shape<DIM, P>;
    constexpr int N = S::N, G = S::G;
    constexpr bool kCoop = DIM == 3 && DIM * S::NF <= N;
    __shared__ double lds[kLevelWaves][G][N + 1];
    __shared__ double cfl[kLevelWaves][kCoop ? G : 1][kCoop ? S::NS : 1][DIM * S::NF];
    constexpr bool kStage = kCoop && S::NF <= 9;
    __shared__ double ufl[kLevelWaves][kStage ? G : 1][kStage ? S::NS : 1][kStage ? S::NF : 1];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int grp = lane / N, row = lane - grp * N;
    const bool in_group = grp < G;
    const int64_t wbase = begin + ((int64_t)blockIdx.x * kLevelWaves + wave) * G;
    if (wbase >= begin + count) return;   // LDS is per wavefront: no block barrier follows
    const SweepArgs args = load_args(table, batch_problem(pairs, wbase, problem));
    int4 pr = make_int4(-1, 0, 0, 0);
    if (in_group) pr = pairs[wbase + grp];
    const bool active = pr.x >= 0;
    const int4 prs = active ? pr : make_int4(0, 0, 0, 0);
    const int e = prs.x;
    const int d = (int)((unsigned)prs.y & kDirMask);
    using IL = InvLayout<DIM, P>;
    const double* Ab = F32 ? nullptr : args.ainv + ((size_t)d * args.E + e) * IL::kStride;
    auto rhs_of = [&]() {
        const int g = in_group ? grp : 0;
        if constexpr (QUAD) {
            static_assert(kStage && !U && DIM == 3 && P == 2, "face points: 3D p = 2 lattices");
            return inflow_rhs_quad<DIM, P>(args, prs, row, in_group, cfl[wave][g], ufl[wave][g]);
        } else if constexpr (kStage) return inflow_rhs_staged<DIM, P, U>(args, prs, row, in_group, cfl[wave][g], ufl[wave][g]);
        else if constexpr (kCoop) return inflow_rhs_coop<DIM, P, U>(args, prs, row, in_group, cfl[wave][g]);
        else return inflow_rhs<DIM, P, false, U>(args, prs, row);
    };
    double* L = &lds[wave][in_group ? grp : 0][0];
    double x = 0.0;
    if constexpr (F32) {
        // mixed precision: the row of A^{-1} rounded to FP32, four entries
        // per 16-byte load, products and sum in FP64
        static_assert(N <= kMaxInv32, "FP32 inverse rows are held in registers");
        using IL32 = InvLayout32<DIM, P>;
        const float* Af = args.ainv32 + ((size_t)d * args.E + e) * IL32::kStride;
        const double b = rhs_of();
        if (in_group) L[row] = b;
        wave_sync();
        __builtin_amdgcn_sched_barrier(0);
        float m[IL32::kGroups * 4];
#pragma unroll
        for (int g = 0; g < IL32::kGroups; ++g) {
            const flt4 v = __builtin_nontemporal_load(reinterpret_cast<const flt4*>(Af + IL32::at(row, 4 * g)));
            m[4 * g] = v.x;
            m[4 * g + 1] = v.y;
            m[4 * g + 2] = v.z;
            m[4 * g + 3] = v.w;
        }
        // b read back from LDS a few entries at a time (fewer live registers)
        constexpr int LG = SNSW_LEVEL_LDS_GROUP;
#pragma unroll
        for (int g0 = 0; g0 < N; g0 += LG) {
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = g0; j < g0 + LG && j < N; ++j) x += (double)m[j] * L[j];
        }
        __builtin_amdgcn_sched_barrier(0);
        __asm__ volatile("" : "+v"(x));
    } else if constexpr (N > SNSW_LEVEL_CHUNK_MIN) {
        // large elements: b first; then the row of A^{-1} is loaded a chunk
        // of columns at a time (all of it for n <= 32) while b is read back
        // from LDS a few entries at a time.  The scheduling barriers keep
        // the LDS values from all being live together (fewer registers, more
        // wavefronts in flight); the empty asm keeps the products out of the
        // store branch, where they would lose the barriers.  In 3D the rows
        // are read as streaming data (each is read once per sweep), which
        // leaves the L2 to the face moments and traces that pairs share.
        const double b = rhs_of();
        if (in_group) L[row] = b;
        wave_sync();
        __builtin_amdgcn_sched_barrier(0);
        constexpr int CH = SNSW_LEVEL_CHUNK > 0 ? SNSW_LEVEL_CHUNK : (N <= 32 ? N : 16);
        constexpr int LG = SNSW_LEVEL_LDS_GROUP;
#pragma unroll
        for (int j0 = 0; j0 < N; j0 += CH) {
            double a[CH];
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                if constexpr (IL::kPaired) {
                    static_assert(CH == N, "paired columns are read in one chunk");
                    if (j + 1 < (N & ~1) && !(j & 1)) {
                        const dbl2 v = __builtin_nontemporal_load(
                            reinterpret_cast<const dbl2*>(Ab + IL::at(row, j)));
                        a[j] = v.x;
                        a[j + 1] = v.y;
                    } else if (j >= (N & ~1)) {
                        a[j] = __builtin_nontemporal_load(Ab + IL::at(row, j));
                    }
                } else if constexpr (DIM == 3) {
                    a[j] = j0 + j < N ? __builtin_nontemporal_load(Ab + IL::at(row, j0 + j)) : 0.0;
                } else {
                    a[j] = j0 + j < N ? Ab[IL::at(row, j0 + j)] : 0.0;
                }
            }
#pragma unroll
            for (int g0 = 0; g0 < CH; g0 += LG) {
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int j = g0; j < g0 + LG && j < CH && j0 + j < N; ++j) x += a[j] * L[j0 + j];
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        __asm__ volatile("" : "+v"(x));
    } else {
        // the row of A^{-1} is loaded while b is assembled
        double m[N];
#pragma unroll
        for (int j = 0; j < N; ++j) m[j] = Ab[IL::at(row, j)];
        const double b = rhs_of();
        if (in_group) L[row] = b;
        wave_sync();
#pragma unroll
        for (int j = 0; j < N; ++j) x += m[j] * L[j];
    }
    if (active) args.psi_cur[((size_t)d * args.E + e) * N + row] = x;
}


// Persistent sweep with cached inverses for the 3D LDS shapes (n = 8, 27,
// 64): the ticket and wait protocol of sweep_persistent_fp64; per pair the
// row of A^{-1} is loaded and b assembled without the kept inflow before the
// wait; after it the face lanes add the kept inflow and x = A^{-1} b is one
// LDS exchange of b.
template <int DIM, int P, bool U = false>
__global__ void __launch_bounds__(64 * kWaves) sweep_persistent_inv(PersistArgs pa) {
    using S = Shape<DIM, P>;
    constexpr int N = S::N, NF = S::NF, NS = S::NS, G = S::G;
    __shared__ double lds[kWaves][G][N + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane / N, row = lane - grp * N;
    const bool in_group = grp < G;
    double* L = &lds[wave][in_group ? grp : 0][0];
    const unsigned long long sent = kSentinel;

    unsigned t_next = 0;
    if (lane == 0) t_next = take_batch(pa.ticket) * (unsigned)G;
    t_next = __shfl(t_next, 0);
    while (true) {
        const unsigned t0 = __builtin_amdgcn_readfirstlane(t_next);
        if ((int64_t)t0 >= pa.total) break;
        unsigned t_pre = 0;
        if (lane == 0) t_pre = take_batch(pa.ticket) * (unsigned)G;
        const SweepArgs args = load_args(pa.table, batch_problem(pa.pairs, t0, pa.problem));
        const int64_t pidx = (int64_t)t0 + grp;
        int4 pr = make_int4(-1, 0, 0, 0);
        if (in_group && pidx < pa.total) pr = pa.pairs[pidx];
        const bool active = pr.x >= 0;    // padding entries have e = -1
        const int4 prs = active ? pr : make_int4(0, 0, 0, 0);
        const int e = prs.x;
        const unsigned packed = (unsigned)prs.y;
        const int d = (int)(packed & kDirMask);
        using IL = InvLayout<DIM, P>;
        const double* Ai = args.ainv + ((size_t)d * args.E + e) * IL::kStride;
        double m[N];
#pragma unroll
        for (int j = 0; j < N; ++j) m[j] = Ai[IL::at(row, j)];
        unsigned kept = 0;
        double rhs = inflow_rhs<DIM, P, true, U>(args, prs, row, &kept);
        if (!active) kept = 0;

        // wait: the lane on the first node of each kept face polls the
        // upwind value there (bounded, as in sweep_persistent_fp64)
        bool need[NS];
        bool ok = true;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            need[s] = row == S::tn(s, 0) && ((kept >> s) & 1u);
            if (need[s]) ok = false;
        }
        int polls = 0;
        while (true) {
            if (!ok) {
                bool all = true;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (!need[s]) continue;
                    const int nb = args.slot_nbr[(size_t)e * NS + s];
                    double* ad = args.psi_cur + ((size_t)d * args.E + nb) * N + up_node<DIM, P, U>(args, e, s, 0);
                    const double val = __hip_atomic_load(ad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if ((unsigned long long)__double_as_longlong(val) == sent) all = false;
                    else need[s] = false;
                }
                ok = all;
            }
            if (__all(ok)) break;
            if (++polls > pa.spin_limit) {
                if (!ok) atomicExch(pa.error, 1);
                break;
            }
            if ((polls & 255) == 0) {
                int err = 0;
                if (lane == 0) err = __hip_atomic_load(pa.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (__shfl(err, 0)) break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        // kept inflow into this lane's entry of b
        {
            const double o0 = args.omega[3 * d + 0], o1 = args.omega[3 * d + 1], o2 = args.omega[3 * d + 2];
            int kc = 0;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const unsigned cls = (packed >> (kSlotShift + 3 * s)) & 3u;
                int kr = 0;
                if (cls == kKink) kr = args.kink_idx[prs.z + kc++];
                const bool on = S::on(row, s);
                if (!(on && ((kept >> s) & 1u))) continue;
                const int la = S::local(row, s);
                const int nb = args.slot_nbr[(size_t)e * NS + s];
                double* up = args.psi_cur + ((size_t)d * args.E + nb) * N;
                // all values of the face in flight together, then re-read
                // any that still hold the sentinel
                double val[NF];
#pragma unroll
                for (int b = 0; b < NF; ++b)
                    val[b] = __hip_atomic_load(up + up_node<DIM, P, U>(args, e, s, b), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                for (int b = 0; b < NF; ++b) {
                    for (int spin = 0;
                         (unsigned long long)__double_as_longlong(val[b]) == sent && spin < pa.spin_limit; ++spin) {
                        __builtin_amdgcn_s_sleep(1);
                        val[b] = __hip_atomic_load(up + up_node<DIM, P, U>(args, e, s, b), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    // a value still unwritten after the bound is a failed wait
                    if ((unsigned long long)__double_as_longlong(val[b]) == sent) atomicExch(pa.error, 1);
                }
#pragma unroll
                for (int b = 0; b < NF; ++b) {
                    double pv;
                    if (cls == kKink) {
                        pv = args.kink_tab[(size_t)kr * 2 * NF * NF + ((s & 1) ? NF * NF : 0) + la * NF + b];
                    } else {
                        const double* Bf =
                            args.B + (size_t)args.slot_face[(size_t)e * NS + s] * DIM * NF * NF + la * NF;
                        pv = o0 * Bf[b] + o1 * Bf[NF * NF + b];
                        if (DIM == 3) pv += o2 * Bf[2 * NF * NF + b];
                        pv *= (s & 1) ? -1.0 : 1.0;
                    }
                    rhs += pv * val[b];
                }
            }
        }
        // x = A^{-1} b
        if (in_group) L[row] = rhs;
        wave_sync();
        double x = 0.0;
#pragma unroll
        for (int j = 0; j < N; ++j) x += m[j] * L[j];
        wave_sync();
        if (active)
            __hip_atomic_store(args.psi_cur + ((size_t)d * args.E + e) * N + row, x, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        t_next = __shfl(t_pre, 0);
    }
}

// Persistent form of the 3D staged level sweep (n >= dim nf with nf <= 9:
// p = 2): the per-pair structure of sweep_level_inv (upwind traces staged in
// LDS, face moments contracted cooperatively, the row of A^{-1} in 16-byte
// column pairs) with the level barriers replaced by per-value waits.  A
// wavefront claims kChunk consecutive batches of G pairs at a time from its
// stream's ticket and processes them in order; the lanes that stage a kept
// upwind trace poll that value until it no longer holds this sweep's
// sentinel (each flux value is its own ready flag: it is stored once, with a
// device-scope store, after the pair is solved).  Deadlock freedom is the
// argument of sweep_persistent_fp64 with chunks in place of batches: the
// smallest unfinished batch depends only on smaller ones, and its chunk is
// either held by a wavefront that has finished the chunk's smaller batches
// or not yet handed out, in which case its stream's earlier chunks are all
// finished and the stream's wavefronts go on to claim it.
constexpr unsigned kChunk = 4;
#ifndef SNSW_STAGED_MIN_WAVES
#define SNSW_STAGED_MIN_WAVES 5   // wavefronts per SIMD the register allocation must allow
#endif

template <int DIM, int P>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(SNSW_STAGED_MIN_WAVES, 8)))
sweep_persistent_staged(PersistArgs pa) {
    using S = Shape<DIM, P>;
    constexpr int N = S::N, NF = S::NF, NS = S::NS, G = S::G;
    static_assert(DIM == 3 && DIM * NF <= N && NF <= 9, "staged 3D shapes");
    using IL = InvLayout<DIM, P>;
    static_assert(IL::kPaired, "paired A^{-1} columns");
    __shared__ double lds[kWaves][G][N + 1];
    __shared__ double cfl[kWaves][G][NS][DIM * NF];
    __shared__ double ufl[kWaves][G][NS][NF];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned long long sent = kSentinel;
    const int64_t nbatch = pa.total / G;

    unsigned chunk = 0;
    if (lane == 0) chunk = take_batch(pa.ticket);
    chunk = __builtin_amdgcn_readfirstlane(__shfl(chunk, 0));
    while ((int64_t)chunk * kChunk < nbatch) {
        unsigned next = 0;
        if (lane == 0) next = take_batch(pa.ticket);
        for (unsigned j = 0; j < kChunk; ++j) {
            const int64_t bt = (int64_t)chunk * kChunk + j;
            if (bt >= nbatch) break;
            const int64_t t0 = bt * G;
            // lane-derived indices are recomputed in every batch instead of
            // being kept live across the loop (registers for wavefronts)
            int lane_b = lane;
            __asm__ volatile("" : "+v"(lane_b));
            const int grp = lane_b / N, row = lane_b - grp * N;
            const bool in_group = grp < G;
            const int g = in_group ? grp : 0;
            double* L = &lds[wave][g][0];
            const SweepArgs args = load_args(pa.table, batch_problem(pa.pairs, t0, pa.problem));
            int4 pr = make_int4(-1, 0, 0, 0);
            if (in_group) pr = pa.pairs[t0 + grp];
            const bool active = pr.x >= 0;   // padding entries have e = -1
            const int4 prs = active ? pr : make_int4(0, 0, 0, 0);
            const int e = prs.x;
            const unsigned packed = (unsigned)prs.y;
            const int d = (int)(packed & kDirMask);
            const int a = row / NF, la = row - a * NF;
            const bool worker = in_group && a < DIM && active;
            const double oa = args.omega[3 * d + (a < DIM ? a : 0)];

            // 1. traces: lane (0, la) of each inflow slot loads the upwind
            // value on face node la (kept couplings from this sweep's flux,
            // polled until written; lagged ones from the previous sweep;
            // boundary faces the incident flux)
            int fcs[NS], krs[NS];
            double tv[NS];
            bool wait[NS];
            int kc = 0;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const unsigned cls = (packed >> (kSlotShift + 3 * s)) & 3u;
                const bool lagged = (packed >> (kSlotShift + 3 * s + 2)) & 1u;
                krs[s] = 0;
                fcs[s] = 0;
                tv[s] = 0.0;
                wait[s] = false;
                if (cls == kKink) krs[s] = args.kink_idx[prs.z + kc++];
                if (cls == kOut || cls == kNone || !worker) continue;
                if (cls != kKink) fcs[s] = args.slot_face[(size_t)e * NS + s];
                if (a == 0) {
                    const int nb = args.slot_nbr[(size_t)e * NS + s];
                    if (nb < 0) {
                        tv[s] = args.psi_inc;
                    } else if (lagged) {
                        tv[s] = args.psi_prev[((size_t)d * args.E + nb) * N + S::tn(s ^ 1, la)];
                    } else {
                        tv[s] = __hip_atomic_load(args.psi_cur + ((size_t)d * args.E + nb) * N + S::tn(s ^ 1, la),
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        wait[s] = true;
                    }
                }
            }
            int polls = 0;
            while (true) {
                bool pending = false;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (!wait[s]) continue;
                    if ((unsigned long long)__double_as_longlong(tv[s]) == sent) pending = true;
                    else wait[s] = false;
                }
                if (!__any(pending)) break;
                if (++polls > pa.spin_limit) {
                    if (pending) atomicExch(pa.error, 1);   // a failed wait: reported, the kernel drains
                    break;
                }
                if ((polls & 255) == 0) {
                    int err = 0;
                    if (lane == 0) err = __hip_atomic_load(pa.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (__shfl(err, 0)) break;
                }
                __builtin_amdgcn_s_sleep(SNSW_POLL_SLEEP);
                const int nbr_base = e * NS;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (!wait[s]) continue;
                    const int nb = args.slot_nbr[(size_t)nbr_base + s];
                    tv[s] = __hip_atomic_load(args.psi_cur + ((size_t)d * args.E + nb) * N + S::tn(s ^ 1, la),
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            if (worker && a == 0) {
#pragma unroll
                for (int s = 0; s < NS; ++s) ufl[wave][g][s][la] = tv[s];
            }
            wave_sync();

            // 2. inflow contraction: lane (a, la), component a of row la of
            // each inflow face's moments, partial sums through LDS
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const unsigned cls = (packed >> (kSlotShift + 3 * s)) & 3u;
                if (cls == kOut || cls == kNone || !worker) continue;
                double t = 0.0;
                if (cls == kKink) {
                    if (a == 0) {
                        const double* Ti =
                            args.kink_tab + (size_t)krs[s] * 2 * NF * NF + ((s & 1) ? NF * NF : 0) + la * NF;
#pragma unroll
                        for (int b = 0; b < NF; ++b) t += Ti[b] * ufl[wave][g][s][b];
                    }
                } else {
                    constexpr int NT = NF * (NF + 1) / 2;
                    const double* Bs = args.Bsym + (size_t)(fcs[s] * bsym_face_stride(NF) + a * NT);
#pragma unroll
                    for (int b = 0; b < NF; ++b) {
                        const int i = la < b ? la : b, jj = la < b ? b : la;
                        t += Bs[i * NF - (i * (i - 1)) / 2 + (jj - i)] * ufl[wave][g][s][b];
                    }
                    t *= (s & 1) ? -oa : oa;   // P_in = -(outward normal) moments
                }
                cfl[wave][g][s][row] = t;
            }
            wave_sync();
            double rhs = (in_group && active) ? source_row(args, e, d, row, N) : 0.0;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const unsigned cls = (packed >> (kSlotShift + 3 * s)) & 3u;
                if (cls == kOut || cls == kNone || !active) continue;
                if (!S::on(row, s)) continue;
                const int l = S::local(row, s);
#pragma unroll
                for (int c = 0; c < DIM; ++c) rhs += cfl[wave][g][s][c * NF + l];
            }

            // 3. x = A^{-1} b: b through LDS, the row of A^{-1} streamed in
            // 16-byte column pairs while b is read back a few entries at a time
            if (in_group) L[row] = rhs;
            wave_sync();
            __builtin_amdgcn_sched_barrier(0);
            const double* Ab = args.ainv + ((size_t)d * args.E + e) * IL::kStride;
            double m[N];
#pragma unroll
            for (int jj = 0; jj < N; ++jj) {
                if (jj + 1 < (N & ~1) && !(jj & 1)) {
                    const dbl2 v = __builtin_nontemporal_load(reinterpret_cast<const dbl2*>(Ab + IL::at(row, jj)));
                    m[jj] = v.x;
                    m[jj + 1] = v.y;
                } else if (jj >= (N & ~1)) {
                    m[jj] = __builtin_nontemporal_load(Ab + IL::at(row, jj));
                }
            }
            constexpr int LG = SNSW_LEVEL_LDS_GROUP;
            double x = 0.0;
#pragma unroll
            for (int g0 = 0; g0 < N; g0 += LG) {
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int jj = g0; jj < g0 + LG && jj < N; ++jj) x += m[jj] * L[jj];
            }
            __builtin_amdgcn_sched_barrier(0);
            __asm__ volatile("" : "+v"(x));
            wave_sync();   // L, cfl and ufl are reused by the next batch
            if (in_group && active)
                __hip_atomic_store(args.psi_cur + ((size_t)d * args.E + e) * N + row, x, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        chunk = __builtin_amdgcn_readfirstlane(__shfl(next, 0));
    }
}

__global__ void fill_sentinel_kernel(const SweepArgs* table) {
    const SweepArgs& a = table[blockIdx.y];
    if (!a.persistent) return;
    const int64_t count = (int64_t)a.D * a.E * a.n;
    unsigned long long* p = reinterpret_cast<unsigned long long*>(a.psi_cur);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = kSentinel;
}

template <int DIM, int P, bool U>
void launch_tpl_u(const SweepArgs* table, const int4* pairs, int64_t begin, int64_t count, int problem, bool mixed,
                  bool inv, hipStream_t stream, bool quad = false) {
    // level kernels take blocks of kLevelWaves wavefronts
    constexpr int per_iblock = kLevelWaves * Shape<DIM, P>::G;
    const int64_t blocks = (count + per_iblock - 1) / per_iblock;
    if (blocks == 0) return;
    const dim3 igrid((unsigned)blocks), iblock(64 * kLevelWaves);
    if constexpr (DIM == 3 && P == 2 && !U) {
        // lattices with face Gauss-point normals: inflow contracted through them
        if (inv && quad) {
            if (mixed)
                hipLaunchKernelGGL((sweep_level_inv<DIM, P, U, true, true>), igrid, iblock, 0, stream, table, pairs,
                                   begin, count, problem);
            else
                hipLaunchKernelGGL((sweep_level_inv<DIM, P, U, false, true>), igrid, iblock, 0, stream, table, pairs,
                                   begin, count, problem);
            return;
        }
    }
    if (inv && mixed) {
        // mixed precision with cached inverses: the FP32 copy
        if constexpr (Shape<DIM, P>::N <= kMaxInv32)
            hipLaunchKernelGGL((sweep_level_inv<DIM, P, U, true>), igrid, iblock, 0, stream, table, pairs, begin, count,
                               problem);
    } else if (inv)
        hipLaunchKernelGGL((sweep_level_inv<DIM, P, U>), igrid, iblock, 0, stream, table,
                           pairs, begin, count, problem);
    else if (mixed)
        hipLaunchKernelGGL((sweep_level_fp64<DIM, P, true, U>), igrid, iblock, 0, stream,
                           table, pairs, begin, count, problem);
    else
        hipLaunchKernelGGL((sweep_level_fp64<DIM, P, false, U>), igrid, iblock, 0,
                           stream, table, pairs, begin, count, problem);
}

// unstructured: the upwind neighbour's nodes come from the table (the
// kernels of lattice meshes compute them)
template <int DIM, int P>
void launch_tpl(const SweepArgs* table, const int4* pairs, int64_t begin, int64_t count, int problem, bool mixed,
                bool inv, bool unstructured, hipStream_t stream, bool quad = false) {
    if (unstructured) launch_tpl_u<DIM, P, true>(table, pairs, begin, count, problem, mixed, inv, stream);
    else launch_tpl_u<DIM, P, false>(table, pairs, begin, count, problem, mixed, inv, stream, quad);
}

// groups of 4 or 16 lanes exchange values by DPP, the others through LDS
template <int DIM, int P>
constexpr bool use_dpp() {
    return Shape<DIM, P>::N == 16 || Shape<DIM, P>::N == 4;
}

// 3D shapes with the staged persistent kernel (cached inverses)
template <int DIM, int P>
constexpr bool use_staged() {
    return DIM == 3 && P == 2;
}

template <int DIM, int P>
bool launch_persist_tpl(const PersistArgs& a, int blocks, bool inv, bool f32, hipStream_t stream) {
    const dim3 grid((unsigned)blocks), block(64 * kWaves);
    if constexpr (use_dpp<DIM, P>()) {
        if (inv && f32 && a.nt)
            hipLaunchKernelGGL((sweep_persistent_dpp<DIM, P, true, true, true>), grid, block, 0, stream, a);
        else if (inv && f32)
            hipLaunchKernelGGL((sweep_persistent_dpp<DIM, P, true, false, true>), grid, block, 0, stream, a);
        else if (inv && a.nt)
            hipLaunchKernelGGL((sweep_persistent_dpp<DIM, P, true, true>), grid, block, 0, stream, a);
        else if (inv)
            hipLaunchKernelGGL((sweep_persistent_dpp<DIM, P, true>), grid, block, 0, stream, a);
        else
            hipLaunchKernelGGL((sweep_persistent_dpp<DIM, P, false>), grid, block, 0, stream, a);
        return true;
    } else {
        if (f32 && !(inv && DIM == 2)) return false;   // FP32 inverses: the 2D lattice kernels only
        if constexpr (DIM == 2) {
            if (inv && f32) hipLaunchKernelGGL((sweep_persistent_lds2d<P, true>), grid, block, 0, stream, a);
            else if (inv) hipLaunchKernelGGL((sweep_persistent_lds2d<P>), grid, block, 0, stream, a);
            else hipLaunchKernelGGL((sweep_persistent_fp64<DIM, P>), grid, block, 0, stream, a);
        } else if constexpr (use_staged<DIM, P>()) {
            if (inv) hipLaunchKernelGGL((sweep_persistent_staged<DIM, P>), grid, block, 0, stream, a);
            else hipLaunchKernelGGL((sweep_persistent_fp64<DIM, P>), grid, block, 0, stream, a);
        } else {
            if (inv) hipLaunchKernelGGL((sweep_persistent_inv<DIM, P>), grid, block, 0, stream, a);
            else hipLaunchKernelGGL((sweep_persistent_fp64<DIM, P>), grid, block, 0, stream, a);
        }
        return true;
    }
}

// Element lists (lattices given as element lists, triangles): the generic
// persistent kernels with the per-slot upwind node table.
template <int DIM, int P>
void launch_persist_u(const PersistArgs& a, int blocks, bool inv, hipStream_t stream) {
    if (inv)
        hipLaunchKernelGGL((sweep_persistent_inv<DIM, P, true>), dim3((unsigned)blocks), dim3(64 * kWaves), 0, stream,
                           a);
    else
        hipLaunchKernelGGL((sweep_persistent_fp64<DIM, P, true>), dim3((unsigned)blocks), dim3(64 * kWaves), 0,
                           stream, a);
}

template <int DIM, int P>
int occupancy_u(bool inv) {
    int nb = 0;
    const hipError_t rc =
        inv ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep_persistent_inv<DIM, P, true>, 64 * kWaves, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep_persistent_fp64<DIM, P, true>, 64 * kWaves, 0);
    return rc == hipSuccess && nb > 0 ? nb : 1;
}

template <int DIM, int P, bool F32>
void launch_factor_f(const SweepArgs* table, const int4* pairs, int64_t count, void* ainv, bool unstructured,
                     hipStream_t stream) {
    constexpr int per_block = kWaves * Shape<DIM, P>::G;
    const int64_t blocks = (count + per_block - 1) / per_block;
    if (blocks == 0) return;
    if constexpr (P >= kTri) {
        // triangles always come with the upwind node table
        hipLaunchKernelGGL((factor_kernel<DIM, P, true, F32>), dim3((unsigned)blocks), dim3(64 * kWaves), 0, stream,
                           table, pairs, count, ainv);
    } else {
        if (unstructured)
            hipLaunchKernelGGL((factor_kernel<DIM, P, true, F32>), dim3((unsigned)blocks), dim3(64 * kWaves), 0,
                               stream, table, pairs, count, ainv);
        else
            hipLaunchKernelGGL((factor_kernel<DIM, P, false, F32>), dim3((unsigned)blocks), dim3(64 * kWaves), 0,
                               stream, table, pairs, count, ainv);
    }
}

template <int DIM, int P>
void launch_factor_tpl(const SweepArgs* table, const int4* pairs, int64_t count, void* ainv, bool f32,
                       bool unstructured, hipStream_t stream) {
    if (!f32) launch_factor_f<DIM, P, false>(table, pairs, count, ainv, unstructured, stream);
    else if constexpr (Shape<DIM, P>::N <= kMaxInv32)
        launch_factor_f<DIM, P, true>(table, pairs, count, ainv, unstructured, stream);
}

template <int DIM, int P>
int occupancy_tpl(bool inv, bool f32) {
    int nb = 0;
    hipError_t rc;
    if constexpr (use_dpp<DIM, P>())
        rc = inv && f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                              &nb, sweep_persistent_dpp<DIM, P, true, false, true>, 64 * kWaves, 0)
             : inv ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep_persistent_dpp<DIM, P, true>, 64 * kWaves, 0)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep_persistent_dpp<DIM, P, false>, 64 * kWaves, 0);
    else if constexpr (DIM == 2)
        rc = inv && f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep_persistent_lds2d<P, true>, 64 * kWaves, 0)
             : inv ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep_persistent_lds2d<P>, 64 * kWaves, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep_persistent_fp64<DIM, P>, 64 * kWaves, 0);
    else if constexpr (use_staged<DIM, P>())
        rc = inv ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep_persistent_staged<DIM, P>, 64 * kWaves, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep_persistent_fp64<DIM, P>, 64 * kWaves, 0);
    else
        rc = inv ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep_persistent_inv<DIM, P>, 64 * kWaves, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep_persistent_fp64<DIM, P>, 64 * kWaves, 0);
    if (rc != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

// blockIdx.y = problem.  Block (0, k) starts problem k's sweep: it swaps the
// two angular-flux buffers; block (0, 0) also zeroes the tickets.  No other
// block reads the buffer pointers.
__global__ void source_kernel(SweepArgs* table, const double* const* phi_list, const double* phi_one,
                              unsigned int* tickets, int n_tickets) {
    SweepArgs& a = table[blockIdx.y];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double* t = a.psi_cur;
        a.psi_cur = a.psi_prev;
        a.psi_prev = t;
    }
    if (blockIdx.x == 0 && blockIdx.y == 0)
        for (int k = threadIdx.x; k < n_tickets * (int)kMaxStreams; k += blockDim.x) tickets[k * kTicketStride] = 0u;
    const int n = a.n;
    const int64_t E = a.E;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= E * n) return;
    const double* __restrict__ phi = phi_list ? phi_list[blockIdx.y] : phi_one;
    const int64_t e = t / n;
    const int i = (int)(t - e * n);
    const double c = a.sigma_s[e] * (0.25 / M_PI);
    // global (not flat) loads, eight columns of M in flight
    const gdouble* M = (const gdouble*)(a.geo + (size_t)e * (a.dim + 1) * n * n);
    const gdouble* qe = (const gdouble*)(a.q + e * n);
    const gdouble* pe = (const gdouble*)(phi + e * n);
    double s = 0.0;
#pragma unroll 8
    for (int j = 0; j < n; ++j) s += M[(size_t)j * n + i] * (qe[j] + c * pe[j]);
    a.src[t] = s;
}

__global__ void scalar_flux_kernel(const SweepArgs* table, double* const* phi_list, double* phi_one) {
    const SweepArgs& a = table[blockIdx.y];
    const int64_t En = a.E * a.n;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= En) return;
    double* __restrict__ phi = phi_list ? phi_list[blockIdx.y] : phi_one;
    // global (not flat) loads, eight directions in flight
    const gdouble* __restrict__ psi = (const gdouble*)a.psi_cur;
    const gdouble* __restrict__ w = (const gdouble*)a.w;
    double s = 0.0;
#pragma unroll 8
    for (int d = 0; d < a.D; ++d) s += w[d] * psi[(size_t)d * En + t];
    phi[t] = s;
}

__global__ void residual_kernel(int64_t len, const double* __restrict__ a, const double* __restrict__ b,
                                unsigned long long* out) {
    __shared__ double s0[256], s1[256];
    double m0 = 0.0, m1 = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < len; t += (int64_t)gridDim.x * blockDim.x) {
        const double x = a[t], y = b[t];
        const double dd = fabs(x - y), ax = fabs(x);
        m0 = (dd > m0 || dd != dd) ? dd : m0;   // keeps a NaN
        m1 = (ax > m1 || ax != ax) ? ax : m1;
    }
    s0[threadIdx.x] = m0;
    s1[threadIdx.x] = m1;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            const double u0 = s0[threadIdx.x + st], u1 = s1[threadIdx.x + st];
            if (u0 > s0[threadIdx.x] || u0 != u0) s0[threadIdx.x] = u0;
            if (u1 > s1[threadIdx.x] || u1 != u1) s1[threadIdx.x] = u1;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // nonnegative doubles order like their bit patterns; NaN sorts last
        atomicMax(&out[0], (unsigned long long)__double_as_longlong(s0[0]));
        atomicMax(&out[1], (unsigned long long)__double_as_longlong(s1[0]));
    }
}

}  // namespace

void launch_sweep_level(int dim, int p, bool simplex, bool mixed, bool inv, bool unstructured,
                        const SweepArgs* table, const int4* pairs, int64_t begin, int64_t count, int problem,
                        hipStream_t stream, bool face_points) {
    const bool u = unstructured;
    if (simplex && dim == 3) {
        if (p == 1) launch_tpl_u<3, kTet + 1, true>(table, pairs, begin, count, problem, mixed, inv, stream);
        else if (p == 2) launch_tpl_u<3, kTet + 2, true>(table, pairs, begin, count, problem, mixed, inv, stream);
        else launch_tpl_u<3, kTet + 3, true>(table, pairs, begin, count, problem, mixed, inv, stream);
    } else if (simplex) {
        // triangles come as element lists: always the table of upwind nodes
        if (p == 1) launch_tpl_u<2, kTri + 1, true>(table, pairs, begin, count, problem, mixed, inv, stream);
        else if (p == 2) launch_tpl_u<2, kTri + 2, true>(table, pairs, begin, count, problem, mixed, inv, stream);
        else launch_tpl_u<2, kTri + 3, true>(table, pairs, begin, count, problem, mixed, inv, stream);
    } else if (dim == 2) {
        if (p == 1) launch_tpl<2, 1>(table, pairs, begin, count, problem, mixed, inv, u, stream);
        else if (p == 2) launch_tpl<2, 2>(table, pairs, begin, count, problem, mixed, inv, u, stream);
        else launch_tpl<2, 3>(table, pairs, begin, count, problem, mixed, inv, u, stream);
    } else {
        if (p == 1) launch_tpl<3, 1>(table, pairs, begin, count, problem, mixed, inv, u, stream);
        else if (p == 2) launch_tpl<3, 2>(table, pairs, begin, count, problem, mixed, inv, u, stream, face_points);
        else launch_tpl<3, 3>(table, pairs, begin, count, problem, mixed, inv, u, stream);
    }
}

template <int DIM, int P>
int64_t inv_bytes_tpl(bool f32) {
    if (f32) return Shape<DIM, P>::N <= kMaxInv32 ? (int64_t)sizeof(float) * InvLayout32<DIM, P>::kStride : 0;
    return (int64_t)sizeof(double) * InvLayout<DIM, P>::kStride;
}

int64_t ainv_block_bytes(int dim, int p, bool simplex, bool f32) {
    if (simplex && dim == 3)
        return p == 1 ? inv_bytes_tpl<3, kTet + 1>(f32) : p == 2 ? inv_bytes_tpl<3, kTet + 2>(f32)
                                                                 : inv_bytes_tpl<3, kTet + 3>(f32);
    if (simplex)
        return p == 1 ? inv_bytes_tpl<2, kTri + 1>(f32) : p == 2 ? inv_bytes_tpl<2, kTri + 2>(f32)
                                                                 : inv_bytes_tpl<2, kTri + 3>(f32);
    if (dim == 2)
        return p == 1 ? inv_bytes_tpl<2, 1>(f32) : p == 2 ? inv_bytes_tpl<2, 2>(f32) : inv_bytes_tpl<2, 3>(f32);
    return p == 1 ? inv_bytes_tpl<3, 1>(f32) : p == 2 ? inv_bytes_tpl<3, 2>(f32) : inv_bytes_tpl<3, 3>(f32);
}

void launch_factor(int dim, int p, bool simplex, bool f32, bool unstructured, const SweepArgs* table,
                   const int4* pairs, int64_t count, void* ainv, hipStream_t stream) {
    const bool u = unstructured;
    if (simplex && dim == 3) {
        if (p == 1) launch_factor_tpl<3, kTet + 1>(table, pairs, count, ainv, f32, true, stream);
        else if (p == 2) launch_factor_tpl<3, kTet + 2>(table, pairs, count, ainv, f32, true, stream);
        else launch_factor_tpl<3, kTet + 3>(table, pairs, count, ainv, f32, true, stream);
    } else if (simplex) {
        if (p == 1) launch_factor_tpl<2, kTri + 1>(table, pairs, count, ainv, f32, true, stream);
        else if (p == 2) launch_factor_tpl<2, kTri + 2>(table, pairs, count, ainv, f32, true, stream);
        else launch_factor_tpl<2, kTri + 3>(table, pairs, count, ainv, f32, true, stream);
    } else if (dim == 2) {
        if (p == 1) launch_factor_tpl<2, 1>(table, pairs, count, ainv, f32, u, stream);
        else if (p == 2) launch_factor_tpl<2, 2>(table, pairs, count, ainv, f32, u, stream);
        else launch_factor_tpl<2, 3>(table, pairs, count, ainv, f32, u, stream);
    } else {
        if (p == 1) launch_factor_tpl<3, 1>(table, pairs, count, ainv, f32, u, stream);
        else if (p == 2) launch_factor_tpl<3, 2>(table, pairs, count, ainv, f32, u, stream);
        else launch_factor_tpl<3, 3>(table, pairs, count, ainv, f32, u, stream);
    }
}

void launch_source(SweepArgs* table, int count, int64_t max_En, const double* const* phi_list,
                   const double* phi_one, unsigned int* tickets, int n_tickets, hipStream_t stream) {
    const int64_t blocks = std::max<int64_t>(1, (max_En + 255) / 256);
    hipLaunchKernelGGL(source_kernel, dim3((unsigned)blocks, (unsigned)count), dim3(256), 0, stream, table,
                       phi_list, phi_one, tickets, n_tickets);
}

void launch_fill_sentinel(const SweepArgs* table, int count, int64_t max_DEn, hipStream_t stream) {
    int64_t blocks = (max_DEn + 255) / 256;
    blocks = std::max<int64_t>(1, std::min<int64_t>(blocks, std::max<int64_t>(1, 8192 / count)));
    hipLaunchKernelGGL(fill_sentinel_kernel, dim3((unsigned)blocks, (unsigned)count), dim3(256), 0, stream, table);
}

bool launch_sweep_persistent(int dim, int p, bool simplex, bool unstructured, bool inv, const PersistArgs& a,
                             int blocks, hipStream_t stream, bool f32) {
    if (simplex || unstructured) {
        if (f32) return false;
        if (simplex && dim == 3) {
            if (p == 1) launch_persist_u<3, kTet + 1>(a, blocks, inv, stream);
            else if (p == 2) launch_persist_u<3, kTet + 2>(a, blocks, inv, stream);
            else launch_persist_u<3, kTet + 3>(a, blocks, inv, stream);
        } else if (simplex) {
            if (p == 1) launch_persist_u<2, kTri + 1>(a, blocks, inv, stream);
            else if (p == 2) launch_persist_u<2, kTri + 2>(a, blocks, inv, stream);
            else launch_persist_u<2, kTri + 3>(a, blocks, inv, stream);
        } else if (dim == 2) {
            if (p == 1) launch_persist_u<2, 1>(a, blocks, inv, stream);
            else if (p == 2) launch_persist_u<2, 2>(a, blocks, inv, stream);
            else launch_persist_u<2, 3>(a, blocks, inv, stream);
        } else {
            if (p == 1) launch_persist_u<3, 1>(a, blocks, inv, stream);
            else if (p == 2) launch_persist_u<3, 2>(a, blocks, inv, stream);
            else launch_persist_u<3, 3>(a, blocks, inv, stream);
        }
        return true;
    }
    if (dim == 2) {
        if (p == 1) return launch_persist_tpl<2, 1>(a, blocks, inv, f32, stream);
        if (p == 2) return launch_persist_tpl<2, 2>(a, blocks, inv, f32, stream);
        return launch_persist_tpl<2, 3>(a, blocks, inv, f32, stream);
    }
    if (p == 1) return launch_persist_tpl<3, 1>(a, blocks, inv, f32, stream);
    if (p == 2) return launch_persist_tpl<3, 2>(a, blocks, inv, f32, stream);
    return launch_persist_tpl<3, 3>(a, blocks, inv, f32, stream);
}

int persistent_blocks_per_cu(int dim, int p, bool simplex, bool unstructured, bool inv, bool f32) {
    if (simplex && dim == 3)
        return p == 1 ? occupancy_u<3, kTet + 1>(inv) : p == 2 ? occupancy_u<3, kTet + 2>(inv)
                                                             : occupancy_u<3, kTet + 3>(inv);
    if (simplex)
        return p == 1 ? occupancy_u<2, kTri + 1>(inv) : p == 2 ? occupancy_u<2, kTri + 2>(inv)
                                                             : occupancy_u<2, kTri + 3>(inv);
    if (unstructured) {
        if (dim == 2) return p == 1 ? occupancy_u<2, 1>(inv) : p == 2 ? occupancy_u<2, 2>(inv) : occupancy_u<2, 3>(inv);
        return p == 1 ? occupancy_u<3, 1>(inv) : p == 2 ? occupancy_u<3, 2>(inv) : occupancy_u<3, 3>(inv);
    }
    if (dim == 2)
        return p == 1 ? occupancy_tpl<2, 1>(inv, f32) : p == 2 ? occupancy_tpl<2, 2>(inv, f32)
                                                             : occupancy_tpl<2, 3>(inv, f32);
    return p == 1 ? occupancy_tpl<3, 1>(inv, f32) : p == 2 ? occupancy_tpl<3, 2>(inv, f32)
                                                         : occupancy_tpl<3, 3>(inv, f32);
}

bool persistent_f32(int dim, int p, bool simplex, bool unstructured) {
    (void)p;
    return dim == 2 && !simplex && !unstructured;
}

bool persistent_uses_inverse(int dim, int p) {
    (void)dim;
    (void)p;
    return true;
}

void launch_scalar_flux(const SweepArgs* table, int count, int64_t max_En, double* const* phi_list,
                        double* phi_one, hipStream_t stream) {
    const int64_t blocks = std::max<int64_t>(1, (max_En + 255) / 256);
    hipLaunchKernelGGL(scalar_flux_kernel, dim3((unsigned)blocks, (unsigned)count), dim3(256), 0, stream, table,
                       phi_list, phi_one);
}

void launch_residual(int64_t len, const double* a, const double* b, unsigned long long* out, hipStream_t stream) {
    int64_t blocks = (len + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(residual_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, len, a, b, out);
}

}  // namespace snsw
