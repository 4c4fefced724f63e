// Internal host-side structures of the snsweep library (not part of the ABI).
#pragma once

#include <array>
#include <cstdint>
#include <functional>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "snsweep.h"

namespace snsw {

// Error carried from deep inside setup to the C boundary.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

// Runs fn(i) for i in [0, n) on up to nthreads host threads (static chunks).
void parallel_for(int64_t n, int nthreads, const std::function<void(int64_t, int64_t)>& fn);

// ----------------------------------------------------------------- basis.cpp
// n-point Gauss-Legendre rule on [0, 1], ascending points.
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w);
// p+1 Gauss-Lobatto-Legendre points on [0, 1], ascending.
std::vector<double> gll01(int p);
// Values and derivatives of the Lagrange polynomials of `nodes` at x.
void lagrange_eval(const std::vector<double>& nodes, double x, double* val, double* der);
// Monomial coefficients (ascending powers) of the derivative of each Lagrange
// polynomial of `nodes`: out[m][k], k = 0..nn-2.
std::vector<std::vector<double>> lagrange_derivative_monomials(const std::vector<double>& nodes);

// Triangles (simplicial elements): reference triangle {x, y >= 0, x + y <= 1}
// with vertices v0 = (0,0), v1 = (1,0), v2 = (0,1); nodes of order k on the
// lattice pairs (i, j), i + j <= k, numbered row by row (j slowest).
int tri_index(int k, int i, int j);
// Element-local nodes of edge slot s in slot order (slot 0: v0 -> v1,
// slot 1: v1 -> v2, slot 2: v2 -> v0, counter-clockwise).
std::vector<int32_t> tri_slot_nodes(int k, int s);
// Node positions [n][2]: control points at (i/r, j/r); DG nodes at the
// Gauss-Lobatto points (g_i, g_j) on the edges and at (i/p, j/p) inside.
std::vector<double> tri_geometry_nodes(int r);
std::vector<double> tri_dg_nodes(int p);
// Nodal P_k basis of the given nodes (monomial Vandermonde inverse).
struct TriBasis {
    int k = 0, n = 0;
    std::vector<std::pair<int, int>> mono;   // exponents (a, c) of x^a y^c
    std::vector<double> C;                   // [monomial][basis function]
    TriBasis(const std::vector<double>& nodes, int k);
    // values and x / y derivatives of the n basis functions (nullable outputs)
    void eval(double x, double y, double* val, double* dx, double* dy) const;
};
// Collapsed Gauss rule on the triangle: nq x nq points (x = u, y = v (1 - u),
// weight w_u w_v (1 - u)), exact for total degree 2 nq - 2.
void tri_collapsed_rule(int nq, std::vector<double>& x, std::vector<double>& y, std::vector<double>& w);

// Tetrahedra: reference tetrahedron with vertices V0 = (0,0,0), V1 = (1,0,0),
// V2 = (0,1,0), V3 = (0,0,1); nodes of order k on the lattice triples
// (i, j, l), i + j + l <= k, numbered with l slowest, then j, then i.
int tet_index(int k, int i, int j, int l);
// Element nodes of face slot s (the face opposite V_s, its vertices in the
// outward order (V1,V2,V3), (V0,V3,V2), (V0,V1,V3), (V0,V2,V1)), in the
// face's triangle lattice order: face node (a, b) has barycentric
// coordinates k - a - b, a, b on the face's vertices.
std::vector<int32_t> tet_slot_nodes(int k, int s);
// Node positions [n][3]: control points at (i, j, l) / r; DG nodes at the
// Gauss-Lobatto points of the edges on the edges, equispaced elsewhere.
std::vector<double> tet_geometry_nodes(int r);
std::vector<double> tet_dg_nodes(int p);
// Nodal P_k basis of the given nodes on the tetrahedron.
struct TetBasis {
    int k = 0, n = 0;
    std::vector<std::array<int, 3>> mono;    // exponents of x^a y^b z^c
    std::vector<double> C;                   // [monomial][basis function]
    TetBasis(const std::vector<double>& nodes, int k);
    void eval(double x, double y, double z, double* val, double* dx, double* dy, double* dz) const;
};
// Collapsed Gauss rule on the tetrahedron, nq^3 points, exact for total
// degree 2 nq - 3.
void tet_collapsed_rule(int nq, std::vector<double>& x, std::vector<double>& y, std::vector<double>& z,
                        std::vector<double>& w);
// The reference triangle cut into K^2 congruent sub-triangles with the
// collapsed Gauss rule (nq per direction) on each.
void tri_composite_rule(int K, int nq, std::vector<double>& s, std::vector<double>& t, std::vector<double>& w);

// ------------------------------------------------------------ quadrature.cpp
// Level-symmetric S_N set: omega [D][3], w [D] (2D: z > 0 half, doubled).
void level_symmetric(int N, int dim, std::vector<double>& omega, std::vector<double>& w);

// ------------------------------------------------------------------ mesh data
// Face classes relative to the face normal N (minus -> plus element).
enum FaceClass : uint8_t { FC_POS = 0, FC_NEG = 1, FC_KINK = 2 };
// Slot classes from the element's point of view (packed in the schedule).
// SC_NONE: the face carries no flux for this direction (both sides dropped).
enum SlotClass : uint32_t { SC_OUT = 0, SC_IN = 1, SC_KINK = 2, SC_NONE = 3 };

struct DirGraph {
    std::vector<int32_t> up, down;       // edges sorted by (down, up)
    std::vector<int64_t> weight;
    std::vector<int32_t> rem_down, rem_up;  // lagged edges sorted by (down, up)
    std::vector<int32_t> level;          // [E]
    snsw_graph_stats stats{};
    std::vector<uint8_t> face_class;     // [F]
    std::vector<uint8_t> face_drop;      // [F] bit0: minus side dropped, bit1: plus side
    std::vector<int32_t> kink_face;      // faces with FC_KINK
    std::vector<double> kink_tab;        // [nk][2][nf][nf]: P_plus, P_minus
};

// Per-face normal data used to classify (face, direction) pairs.
struct FaceNormalData {
    std::vector<double> mono;        // 2D: monomials of N_x(s), N_y(s) [F][2][r]
    std::vector<double> cs, ct, cw;  // 3D composite rule points and weights
    std::vector<double> cphi;        // 3D trace values at the points [Qc][nf]
    std::vector<double> gV1, gD1;    // geometry 1D tables at the abscissae
    std::vector<int> ci, cj;         // abscissa index of each point
    int nc1 = 0;
    std::vector<double> Rf;          // 3D: max |N_q - mean N| over the points
    std::vector<double> tgs, tgt;    // triangular faces: map basis derivatives at the points [Qc][nfc]
    int nfc = 0;                     // triangular faces: control points per face
};

struct HostProblem {
    int dim = 2, nx[3] = {1, 1, 1}, r = 1, p = 1;
    int n = 0, nf = 0, nslot = 0;
    int64_t E = 0, F = 0;
    int D = 0;
    int weighting = 1, exact_max = 10, precision = 0, bc = 0, nthreads = 1, schedule = 0, cache_inverse = 0;
    int inverse_cached = 0;   // set by the device upload
    int cached_dirs = 0;      // directions whose inverses are cached (set by the device upload)
    double cache_budget = 0.0;  // bytes the inverses may take under CACHE_AUTO (<= 0: half the free memory)
    double psi_inc = 0.0;
    std::vector<double> lattice;              // [L][dim] (structured meshes)
    bool unstructured = false;                // mesh given as element control-point lists
    bool simplex = false;                     // P_r triangles with a P_p DG basis (unstructured, 2D)
    int nv = 0;                               // control points per element
    int face_rule = 0;                        // SNSW_FACE_*: sign-changing faces exact/fixed or Romberg
    double face_tol = 1e-10;                  // relative tolerance of the Romberg face rule
    std::vector<double> nodes;                // [n_nodes][dim] (unstructured)
    std::vector<int64_t> elem_nodes;          // [E][nv] (unstructured)
    std::vector<double> omega, w;             // [D][3], [D]
    std::vector<double> sigma_t, sigma_s, q;  // [E], [E], [E][n] (isotropic source)
    std::vector<double> q_dir;                // [D][E][n] direction-dependent source, or empty
    std::vector<double> psi_tab;              // [D][E][n] tabulated incident flux, or empty
    std::vector<double> rhs_fixed;            // [D][E][n] M q_dir + tabulated inflow, or empty
    // element matrices, row-major (m, n)
    std::vector<double> M, K;                 // [E][n][n], [E][dim][n][n]
    // faces
    std::vector<int32_t> f_axis, f_minus, f_plus;
    std::vector<double> f_ctrl;               // [F][(r+1)^(dim-1)][dim]
    std::vector<double> B;                    // [F][dim][nf][nf] int N_k phi_a phi_b
    std::vector<double> Nint;                 // [F][dim] int N_k
    std::vector<double> Nq;                   // 3D tensor faces: [F][nq][nq][3] w_q N(q) at the Gauss points of B
    FaceNormalData fnd;
    std::vector<int32_t> slot_face, slot_nbr; // [E][nslot]
    std::vector<int32_t> slot_nodes;          // [nslot][nf]
    // unstructured meshes: per element slot whether the element is its
    // face's minus side, and the element's / the neighbour's DG nodes listed
    // in the face's (s, t) order ([E][nslot][nf]); per face the slot of its
    // minus and plus element
    std::vector<uint8_t> hf_minus;
    std::vector<int32_t> hf_trace, hf_up_trace;
    std::vector<int8_t> f_slot_minus, f_slot_plus;
    std::vector<DirGraph> graphs;             // [D]
    // combined schedule
    std::vector<int64_t> level_off;           // [L+1]
    // partial inverse cache: level k holds the cached pairs in
    // [level_off[k], level_split[k]) and the others up to level_off[k+1],
    // both padded to whole batches; empty when every pair is alike
    std::vector<int64_t> level_split;         // [L]
    std::vector<int32_t> pairs;               // [P][4]: e, packed, kink_base, 0
    std::vector<int32_t> kink_idx;            // per pair kink slots -> kink rows
    // tiled schedule (2D, persistent kernels with G = T*T groups): a batch is
    // one T x T tile of elements for one direction; empty when not built
    int tile = 0;                             // T, 0 = no tiled schedule
    std::vector<int64_t> tlevel_off;          // [Lt+1]
    std::vector<int32_t> tpairs;              // [Pt][4] as pairs
    std::vector<int32_t> tintra;              // [Pt] intra-tile dependency word
    std::vector<double> kink_tab;             // [K][2][nf][nf]
    int64_t n_kinks = 0;
    double setup_seconds = 0.0;
};

// Whether element e is the minus side of the face on its slot s.
inline bool slot_is_minus(const HostProblem& hp, int64_t e, int s) {
    return hp.unstructured ? hp.hf_minus[(size_t)e * hp.nslot + s] != 0 : (s & 1) != 0;
}
// Element e's DG nodes on slot s, in the face's (s, t) order.
inline const int32_t* slot_trace(const HostProblem& hp, int64_t e, int s) {
    return hp.unstructured ? &hp.hf_trace[((size_t)e * hp.nslot + s) * hp.nf] : &hp.slot_nodes[(size_t)s * hp.nf];
}
// Slot of face f on its minus (side 0) or plus (side 1) element.
inline int face_slot(const HostProblem& hp, int64_t f, int side) {
    if (hp.unstructured) return side == 0 ? hp.f_slot_minus[f] : hp.f_slot_plus[f];
    return 2 * hp.f_axis[f] + (side == 0 ? 1 : 0);
}

// geometry.cpp: element matrices; throws Error(SNSW_E_BAD_JACOBIAN)
void build_geometry(HostProblem& hp);
// faces.cpp: face enumeration, normal moments, per-direction classification
void build_faces(HostProblem& hp);
// Class of face f for direction om with measures mp = int max(g,0),
// mm = int max(-g,0); for FC_KINK also the matrices Pp, Pm (nf x nf).
uint8_t face_integrals(const HostProblem& hp, int64_t f, const double* om, double& mp,
                       double& mm, double* Pp, double* Pm);
// sources.cpp: fixed right-hand side per pair from q_dir and psi_tab
// (needs the element matrices, faces and graphs)
void build_fixed_rhs(HostProblem& hp);
// Physical coordinates of the DG nodes of elements [e0, e0+count): [count][n][dim].
void node_coordinates(const HostProblem& hp, int64_t e0, int64_t count, double* xyz);
// Volume rule with `extra` Gauss points per axis beyond the element-matrix
// rule: points per element (returned), and if x is not null the physical
// points [count][Q][dim], weights times |det J| [count][Q] and, if basis is
// not null, the DG basis at the reference points [Q][n].
int volume_rule(const HostProblem& hp, int extra, int64_t e0, int64_t count, double* x, double* wdet,
                double* basis);
// graph.cpp: per-direction graph, FAS and levels; combined schedule
void build_graphs(HostProblem& hp);
void build_schedule(HostProblem& hp);
// Arranges every level of the combined schedule for an inverse cache of the
// first Dc directions: their pairs first (direction-major in 3D), then the
// others (element-major), each part padded to whole batches; fills
// level_split when 0 < Dc < D.  Dc = 0 keeps the schedule as built.
void arrange_levels_for_cache(HostProblem& hp, int Dc);
// Device bytes of one pair's cached A^{-1} (FP64, or the FP32 copy when f32;
// 0 when that element has no cached form), as the kernels lay it out.
int64_t ainv_block_bytes(int dim, int p, bool simplex, bool f32);
// Tiled schedule with T x T tiles (T*T = 64/n); returns false (and leaves it
// empty) when the contracted tile graph of some direction has a cycle.
bool build_tiled_schedule(HostProblem& hp, int T);

// Intra-tile dependency word of a tiled schedule entry: bit s set when slot
// s reads a kept upwind pair of the same tile, whose group index is in bits
// [8 + 4s, 12 + 4s).
constexpr int kIntraGroupShift = 8;

// Packed pair word: bits 0..9 direction, then per slot s 3 bits at 10+3s:
// class (2 bits, SlotClass) and lag flag (bit 2).  The lag flag is also set
// when the slot's inflow side was dropped (its matrix is zero): such a slot
// never waits for the upwind element.
constexpr int kDirBits = 10;
inline uint32_t pack_slot(uint32_t cls, bool lag, int s) {
    return (cls | (lag ? 4u : 0u)) << (kDirBits + 3 * s);
}

}  // namespace snsw
