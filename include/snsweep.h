/*
 * snsweep -- graph-based upwind DG transport sweeps for the steady,
 * mono-energetic S_N equations on curved high-order quad/hex (and
 * triangle) meshes, on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Haut, Maginot, Tomov, Southworth, Brunner, Bailey, "An Efficient
 * Sweep-based Solver for the S_N Equations on High-Order Meshes".
 *   - problem and quadrature: section 2, eqs. linearSnTransport, snScalarFlux;
 *   - DG operators: eqs. matrixFormLinearTransport .. localFOffDiagonalMatrix;
 *   - source iteration and lagged sweep: section 3, eqs. sourceIteration,
 *     fSplitting, laggedSourceIteration;
 *   - dependency graph, edge weights, SCC + feedback arc set: section 3,
 *     eq. graphWeight and the text after it.
 *
 * Conventions used by every call:
 *   - All functions return 0 (SNSW_OK) or a negative SNSW_E_* status; the
 *     message of the last failure on the calling thread is returned by
 *     snsw_last_error().  No C++ exception crosses this boundary.
 *   - Host arrays passed to *_create are copied before the call returns; the
 *     caller keeps ownership and may free them afterwards.
 *   - Pointers named d_* are device pointers on the context's device, owned
 *     by the caller (the library never frees them), contiguous, of the stated
 *     element type.  Work on them is enqueued on the context's stream and is
 *     complete once that stream is synchronised, unless stated otherwise.
 *   - Library device memory is allocated by *_create and freed by *_destroy.
 *   - Handles are not thread-safe: one thread at a time per handle.
 *
 * Array layouts (C order, last index fastest):
 *   lattice  [L_z][L_y][L_x][dim]   control points of the Q_r mesh map,
 *                                   L_a = r*nx[a] + 1 (x fastest);
 *   element  e = i + nx*(j + ny*k);
 *   DOFs     [E][n],   n = (p+1)^dim nodal values at the Gauss-Lobatto
 *            points of the element, local node m = a + (p+1)*(b + (p+1)*c);
 *   psi      [D][E][n] angular flux of direction d;
 *   phi      [E][n]    scalar flux, phi = sum_d w_d psi_d.
 */
#ifndef SNSWEEP_H
#define SNSWEEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define SNSW_OK                0
#define SNSW_E_INVALID_ARG    -1  /* null pointer, out-of-range value       */
#define SNSW_E_SHAPE          -2  /* sizes inconsistent with each other      */
#define SNSW_E_NONFINITE      -3  /* NaN/Inf in an input array               */
#define SNSW_E_BAD_JACOBIAN   -4  /* det J <= 0 at a quadrature point        */
#define SNSW_E_NOT_CONVERGED  -5  /* max_iters reached (last iterate kept)   */
#define SNSW_E_DIVERGED       -6  /* residual became NaN or grew past 1e300  */
#define SNSW_E_HIP            -7  /* HIP runtime error                       */
#define SNSW_E_OOM            -8  /* host or device allocation failed        */
#define SNSW_E_UNSUPPORTED    -9  /* option not supported (e.g. host-only)   */
#define SNSW_E_STATE         -10  /* call out of order / bad checkpoint      */

/* ------------------------------------------------------------ enumerations */
#define SNSW_BC_VACUUM     0      /* psi_inc = 0                             */
#define SNSW_BC_ISO_CONST  1      /* psi_inc = constant on all inflow faces  */
#define SNSW_BC_TABULATED  2      /* psi_inc per direction and boundary node
                                     (psi_inc_tab)                           */

/* Layout of the volume source q (snsw_problem_desc.q_per_dof).              */
#define SNSW_Q_PER_ELEMENT    0   /* [E]: isotropic, constant per element    */
#define SNSW_Q_PER_DOF        1   /* [E][n]: isotropic, nodal values         */
#define SNSW_Q_PER_DIRECTION  2   /* [D][E][n]: nodal values per direction   */

#define SNSW_WEIGHT_UNITY       0 /* z = 1                                   */
#define SNSW_WEIGHT_FACE        1 /* z = max |F_{e,e'}|                      */
#define SNSW_WEIGHT_SIGINVFACE  2 /* z = max |M_{t,e}^{-1} F_{e,e'}|          */

#define SNSW_PREC_FP64   0        /* assembly, LU and solve in FP64          */
#define SNSW_PREC_MIXED  1        /* assembled: FP32 LU + one FP64 residual
                                     correction; cached: A^{-1} rounded to
                                     FP32 (SNSW_CACHE_*)                     */

/* Device schedule of one sweep.  PERSISTENT: one launch; wavefronts claim
 * (element, direction) pairs in level order and wait only for the upwind
 * values they read (latency-bound sweeps: 2D).  LEVELS: one launch per level
 * (throughput-bound sweeps: 3D).  AUTO picks PERSISTENT for 2D FP64
 * problems (for p = 2 unless cache_inverse is SNSW_CACHE_OFF) and for 2D
 * SNSW_PREC_MIXED lattices whose inverses are not switched off, and LEVELS
 * otherwise.  SNSW_PREC_MIXED takes PERSISTENT only there
 * (SNSW_E_UNSUPPORTED elsewhere); if AUTO then finds too little memory for
 * the FP32 inverses the problem sweeps on LEVELS (info reports it).      */
#define SNSW_SCHED_AUTO        0
#define SNSW_SCHED_PERSISTENT  1
#define SNSW_SCHED_LEVELS      2

/* The element operator of a pair, A = sigma_t M - sum_i Omega_i K_i + its
 * outflow face blocks, is the same in every source iteration.  With a cached
 * inverse it is factored once (Gauss-Jordan on the device, at create) and a
 * sweep only assembles b and forms A^{-1} b: D*E*n^2 doubles of device
 * memory, one more double per pair for 3D p = 2 (e.g. 15 GB for 32^3
 * elements, p = 2, S8).  With SNSW_PREC_MIXED the inverse (computed in
 * FP64) is kept rounded to FP32, D*E*n*4*ceil(n/4) floats, and the sweep
 * forms A^{-1} b with FP64 products and sums (elements of at most 32 nodes;
 * larger ones take the assembled path).  AUTO caches when that takes at
 * most cache_budget bytes (default: half of the free device memory); on
 * the LEVELS schedule, when all of them would take more, it caches the
 * inverses of as many whole directions as fit (the first ones) and
 * assembles the pairs of the others in every sweep: each level then runs
 * as two launches, cached pairs and assembled pairs.  Persistent schedules
 * cache all or nothing.                                                    */
#define SNSW_CACHE_AUTO    0
#define SNSW_CACHE_ON      1
#define SNSW_CACHE_OFF     2

/* Element type of an unstructured mesh (snsw_problem_desc.element).
 * SIMPLEX: the simplicial elements that section 2 allows next to the
 * tensor-product ones (after eq. elementTransformation: P_r map and P_s
 * DG basis): triangles (dim 2) and tetrahedra (dim 3).
 * Triangles: reference {x, y >= 0, x + y <= 1}, vertices v0 = (0,0),
 * v1 = (1,0), v2 = (0,1).  Nodes of order k sit on the lattice pairs
 * (i, j), i + j <= k, numbered row by row (j slowest): node (i, j) is local
 * index j (k+1) - j (j-1)/2 + i.
 *   control points (k = r): at (i/r, j/r), elem_nodes [E][(r+1)(r+2)/2];
 *   DOFs (k = p): n = (p+1)(p+2)/2, on the edges at the Gauss-Lobatto
 *     points (g_i, g_j) of [0, 1], inside (p = 3: the centroid) at (i/p, j/p).
 * Element slots are the edges v0->v1, v1->v2, v2->v0 (counter-clockwise).
 * Tetrahedra: vertices V0 = (0,0,0), V1 = (1,0,0), V2 = (0,1,0),
 * V3 = (0,0,1); nodes of order k on the lattice triples (i, j, l),
 * i + j + l <= k, numbered with l slowest, then j, then i; barycentric
 * lattice coordinates c = (k-i-j-l, i, j, l).
 *   control points (k = r): at (i, j, l)/r, elem_nodes [E][(r+1)(r+2)(r+3)/6];
 *   DOFs (k = p): n = (p+1)(p+2)(p+3)/6, at sum_v lambda_v V_v with
 *     lambda_v = g_{c_v} on the edges (Gauss-Lobatto) and c_v/p elsewhere
 *     (p = 3: the centroid of each face).
 * Element slot s is the face opposite V_s.  Every element map must keep
 * the orientation of its reference element (det J > 0).                   */
#define SNSW_ELEM_TENSOR   0
#define SNSW_ELEM_SIMPLEX  1

/* Integration of the face matrices (eqs. localFDiagonalMatrix,
 * localFOffDiagonalMatrix) on faces where Omega . n changes sign, whose
 * integrands are only piecewise smooth (section 2, end):
 *   EXACT   2D: split at the real roots of the polynomial Omega . N(s),
 *           Gauss on each piece (exact); 3D: fixed composite Gauss rule on
 *           4 x 4 sub-squares of the face (exact without a sign change);
 *   ROMBERG adaptive Romberg, the paper's choice: Romberg's table (up to 6
 *           rows) on an interval, halved with half the tolerance until two
 *           successive diagonal entries agree to the tolerance (or to 1e-14
 *           of the largest entry); faces of hexahedra iterated (t outer,
 *           inner tolerance a tenth).  Absolute tolerance face_tol times
 *           int |Omega . N| over the face (face_tol <= 0: 1e-10).
 * Which faces change sign is decided as for EXACT, and faces without a sign
 * change keep their exact Gauss rule under both.                           */
#define SNSW_FACE_EXACT    0
#define SNSW_FACE_ROMBERG  1

typedef struct snsw_ctx snsw_ctx;
typedef struct snsw_problem snsw_problem;

/* Message of the last failed call on this thread ("" if none). */
const char* snsw_last_error(void);

/* Library version string. */
const char* snsw_version(void);

/* ---------------------------------------------------------------- context
 * Binds a device and a HIP stream.  device = -1 makes a host-only context:
 * problems built on it run the whole host setup (quadrature, geometry,
 * faces, graph, levels) and support every introspection call, but no device
 * work (sweep/solve return SNSW_E_UNSUPPORTED).  hip_stream may be NULL (the
 * default stream) or a hipStream_t on `device` (e.g. the value of
 * torch.cuda.current_stream().cuda_stream).                                  */
int  snsw_ctx_create(int device, void* hip_stream, snsw_ctx** out);
void snsw_ctx_destroy(snsw_ctx* ctx);

/* ---------------------------------------------------------------- problem */
typedef struct {
    int32_t dim;             /* 2 or 3                                        */
    int32_t nx[3];           /* elements per axis (nx[2] ignored in 2D)       */
    int32_t geom_order;      /* r >= 1: Q_r mesh map (equispaced control pts) */
    int32_t dg_order;        /* p >= 1: Q_p DG basis at Gauss-Lobatto points  */
    const double* lattice;   /* control points, layout above                  */
    int32_t sn_order;        /* level-symmetric S_N order (2,4,..,12), or 0  
                                to use n_dirs/omega/w below                   */
    int32_t n_dirs;          /* user quadrature size (sn_order == 0)          */
    const double* omega;     /* [n_dirs][3] unit directions (sn_order == 0)   */
    const double* w;         /* [n_dirs] weights, sum 4*pi (sn_order == 0)    */
    const double* sigma_t;   /* [E] total cross section, > 0                  */
    const double* sigma_s;   /* [E] scattering cross section, >= 0            */
    const double* q;         /* volume source per steradian, layout by
                                q_per_dof (SNSW_Q_*): [E], [E][n] nodal, or
                                [D][E][n] nodal per direction                 */
    int32_t q_per_dof;
    int32_t bc_kind;         /* SNSW_BC_*                                     */
    double  psi_inc;         /* incident flux for SNSW_BC_ISO_CONST           */
    int32_t weighting;       /* SNSW_WEIGHT_*                                 */
    int32_t exact_scc_max;   /* components up to this size get an exact
                                minimum feedback arc set (<= 20; paper: 10)   */
    int32_t precision;       /* SNSW_PREC_*                                   */
    int32_t n_threads;       /* host threads for setup (0 = hardware count)   */
    int32_t schedule;        /* SNSW_SCHED_*                                  */
    int32_t cache_inverse;   /* SNSW_CACHE_*: keep A^{-1} of every (element,
                                direction) pair in device memory            */
    const double* psi_inc_tab; /* SNSW_BC_TABULATED: [D][E][n] incident flux
                                of direction d at the DG nodes of element e;
                                only nodes on boundary faces through which d
                                flows in are read (others are ignored)      */
    /* Unstructured conforming mesh (section 2: each element's map is given
     * by its own control points, taken from a global list; shared faces
     * share their control points).  elem_nodes == NULL: the structured
     * lattice above.  Otherwise lattice is ignored, E = nx[0] (nx[1] and
     * nx[2] must be 1), nodes [n_nodes][dim] are the control points and
     * elem_nodes [E][(r+1)^dim] the indices of each element's control
     * points in its local lexicographic order (x fastest).  Two element
     * faces are the same face when their corner control points coincide (by
     * index); they may meet in any orientation.  Every element map must be
     * orientation preserving (det J > 0).  Such problems sweep on the LEVELS
     * schedule unless SNSW_SCHED_PERSISTENT is asked for (FP64 only: the
     * generic persistent kernels with a per-slot upwind node table).       */
    int64_t n_nodes;
    const double* nodes;
    const int64_t* elem_nodes;
    int32_t element;         /* SNSW_ELEM_*: element type of an unstructured
                                mesh (SIMPLEX needs elem_nodes)             */
    int32_t face_rule;       /* SNSW_FACE_*                                   */
    double  face_tol;        /* relative tolerance of SNSW_FACE_ROMBERG       */
    double  cache_budget;    /* bytes of device memory the cached inverses
                                may take under SNSW_CACHE_AUTO (<= 0: half
                                the free memory); see SNSW_CACHE_*            */
} snsw_problem_desc;

/* Builds the discretisation and the sweep schedule (section 3): quadrature,
 * geometry and element matrices, upwind face integrals, per-direction
 * dependency graph, cycle cutting and levels; then uploads to the device.
 * Errors: SNSW_E_INVALID_ARG/SHAPE/NONFINITE for bad inputs,
 * SNSW_E_BAD_JACOBIAN for an inverted element, SNSW_E_OOM, SNSW_E_HIP.     */
int  snsw_problem_create(snsw_ctx* ctx, const snsw_problem_desc* desc,
                         snsw_problem** out);
void snsw_problem_destroy(snsw_problem* prob);

typedef struct {
    int64_t n_elements, n_dofs_per_element, n_dirs;
    int64_t n_levels_total;      /* levels of the combined schedule          */
    int64_t n_pairs;             /* (element, direction) pairs = E*D         */
    int64_t n_edges_total;       /* dependency edges over all directions     */
    int64_t n_removed_total;     /* lagged edges over all directions         */
    int64_t n_kink_faces_total;  /* (face, direction) with a sign change     */
    double  setup_seconds;       /* host setup wall time                     */
    int32_t cached_inverse;      /* A^{-1} per pair kept on device: 0 no,
                                    1 FP64, 2 FP32 (mixed precision)        */
    int32_t schedule;            /* resolved SNSW_SCHED_PERSISTENT / LEVELS  */
    int32_t tile;                /* T > 0: the persistent sweep takes T x T
                                    tiles of elements of one direction per
                                    wavefront (2D, p = 1 or 3); 0: single
                                    pairs                                    */
    int32_t cached_dirs;         /* directions whose inverses are cached: D
                                    (all), 0 (none) or, partially, the first
                                    cached_dirs of them                      */
    int64_t inverse_block_bytes; /* device bytes of one pair's cached A^{-1}
                                    in the problem's precision (0: none
                                    possible)                                 */
} snsw_problem_info;
int snsw_problem_get_info(const snsw_problem* prob, snsw_problem_info* info);

/* Quadrature actually used: omega [D][3], w [D] (host, caller-allocated). */
int snsw_get_quadrature(const snsw_problem* prob, double* omega, double* w);

/* Load vector of eq. qVectorDef for sources and incident fluxes given as
 * nodal values (the DG interpolant is integrated exactly): the source term
 * is M_e q (per direction with SNSW_Q_PER_DIRECTION); the boundary term of
 * a slot through which direction d flows in is P_in psi_inc, with P_in the
 * same inflow face block the sweep applies to an upwind neighbour (normal
 * moments of the face, or the split integrals of a face where Omega . n
 * changes sign).  Direction-dependent parts are assembled once into a fixed
 * right-hand side per (element, direction) pair: D*E*n doubles of device
 * memory while a SNSW_Q_PER_DIRECTION source or SNSW_BC_TABULATED inflow is
 * set.
 *
 * Replaces the volume source and the boundary condition of an existing
 * problem (arguments as the fields of the same names in snsw_problem_desc;
 * host arrays, copied).  The graph, schedule and cached inverses do not
 * depend on them and are kept, as is the stored angular flux.  Synchronous.
 * Batches created earlier keep the old source: set sources before creating a
 * batch that includes the problem.  Errors: SNSW_E_INVALID_ARG,
 * SNSW_E_NONFINITE, SNSW_E_OOM, SNSW_E_HIP.                                  */
int snsw_problem_set_source(snsw_problem* prob, int32_t q_per_dof, const double* q, int32_t bc_kind,
                            double psi_inc, const double* psi_inc_tab);

/* Physical coordinates of the DG nodes of elements [e0, e0+count): the mesh
 * map of eq. elementTransformation at the Gauss-Lobatto nodes, host
 * [count][n][dim] (caller-allocated).  For evaluating sources and incident
 * fluxes at the nodes.                                                      */
int snsw_get_node_coordinates(const snsw_problem* prob, int64_t e0, int64_t count, double* xyz);

/* Tensor Gauss-Legendre rule on elements [e0, e0+count) with `extra` points
 * per axis beyond the rule of the element matrices (extra in [0, 8]; on
 * triangles the collapsed Gauss rule, (p + r + extra)^2 points):
 * *n_points receives Q, the points per element; if x is not NULL, x
 * [count][Q][dim] receives the physical points, wdet [count][Q] the weights
 * times |det J|, and basis (nullable) [Q][n] the DG basis at the reference
 * points (the same for every element).  For error norms of nodal fields:
 * int f over element e = sum_q wdet[e][q] f(x[e][q]).  Host arrays.          */
int snsw_get_volume_rule(const snsw_problem* prob, int32_t extra, int64_t e0, int64_t count,
                         int32_t* n_points, double* x, double* wdet, double* basis);

/* Direction-independent element matrices of elements [e0, e0+count) (host,
 * caller-allocated): M [count][n][n] = int u_m u_n, K [count][dim][n][n] =
 * int (d u_m/d x_i) u_n (row m, column n).                                   */
int snsw_get_element_matrices(const snsw_problem* prob, int64_t e0,
                              int64_t count, double* M, double* K);

/* ------------------------------------------------------ graph introspection
 * Per direction d (host arrays, caller-allocated).                          */
typedef struct {
    int64_t n_edges;             /* dependency edges                         */
    int64_t n_scc_simple;        /* strongly connected components of size 2  */
    int64_t n_scc_large;         /* components of size >= 3                  */
    int64_t n_elements_in_large; /* elements in components of size >= 3      */
    int64_t max_scc;             /* largest component                        */
    int64_t n_removed;           /* lagged (removed) edges                   */
    int64_t n_levels;            /* ASAP levels of the cut graph             */
    int64_t removed_weight;      /* total quantised weight of removed edges  */
} snsw_graph_stats;
int snsw_graph_stats_get(const snsw_problem* prob, int d, snsw_graph_stats* st);

/* Edges up -> down (down receives inflow from up) with quantised weights,
 * sorted by (down, up).  *count receives the number of edges; at most cap
 * are written.                                                               */
int snsw_get_edges(const snsw_problem* prob, int d, int32_t* up,
                   int32_t* down, int64_t* weight, int64_t cap,
                   int64_t* count);
/* Lagged edges, sorted by (down, up).                                        */
int snsw_get_removed_edges(const snsw_problem* prob, int d, int32_t* down,
                           int32_t* up, int64_t cap, int64_t* count);
/* ASAP level of every element in the cut graph of direction d, [E].         */
int snsw_get_levels(const snsw_problem* prob, int d, int32_t* level);

/* Upwind integrals of face f (0 <= f < n_faces) for direction d as the setup
 * computes them with the problem's face rule, before near-empty sides are
 * dropped (eqs. localFDiagonalMatrix, localFOffDiagonalMatrix): *cls = 0 when
 * Omega . N >= 0 on the whole face, 1 when <= 0, 2 when it changes sign;
 * *mp = int max(Omega . N, 0), *mm = int max(-Omega . N, 0) over the
 * reference face; for class 2, Pp / Pm [nf][nf] = the same integrals
 * weighted by the products of the face's trace basis functions (zero for
 * the other classes).  N is the area-scaled normal from the face's minus
 * to its plus element.  Faces: on a lattice numbered per axis a (faces on
 * the planes xi_a = const, x fastest), offset by the counts of the earlier
 * axes; on element lists ordered by the (element, slot) of their minus
 * side.  Every output is nullable; host arrays.  Introspection for tests.  */
int snsw_get_face_integrals(const snsw_problem* prob, int d, int64_t f, int32_t* cls, double* mp,
                            double* mm, double* Pp, double* Pm);

/* ------------------------------------------------------------------- sweep
 * One lagged transport sweep over all directions (eq. laggedSourceIteration):
 * reads d_phi_in [E][n], writes d_phi_out [E][n] and, if d_psi_out is not
 * NULL, the new angular flux [D][E][n].  Lagged couplings read the angular
 * flux of the previous sweep kept inside the problem (zero after create or
 * snsw_reset); the new flux replaces it.  Asynchronous on the ctx stream.   */
int snsw_sweep(snsw_problem* prob, const double* d_phi_in, double* d_phi_out,
               double* d_psi_out);

/* Clears the stored angular flux used by lagged couplings.                  */
int snsw_reset(snsw_problem* prob);

/* Waits for the ctx stream and reports device-side failures of earlier
 * sweeps: SNSW_E_STATE if a dependency wait of the persistent schedule timed
 * out (the affected sweep's output is invalid).                              */
int snsw_synchronize(snsw_problem* prob);

/* Bound of every dependency wait of this problem's persistent sweeps: polls
 * before the wait gives up, flags the failure (reported by
 * snsw_synchronize as SNSW_E_STATE) and lets the grid drain.  polls >= 0;
 * default 2^20 (far above any wait of a valid schedule).  A small bound
 * forces the failure path from the host, for tests of it; the sweeps of a
 * batch keep the default.  SNSW_E_INVALID_ARG for polls < 0.                */
int snsw_set_wait_limit(snsw_problem* prob, int32_t polls);

/* ------------------------------------------------------------------- solve
 * Source iteration (eq. sourceIteration) from the guess in d_phi until
 * max|phi_{l+1}-phi_l| / max|phi_{l+1}| <= tol (checked every check_every
 * iterations; only then does the host wait for the device).  d_phi [E][n]
 * receives the last iterate; d_psi (nullable) its angular flux.  The
 * residual history is written to report->history if non-NULL (capacity
 * history_cap).  Returns SNSW_E_NOT_CONVERGED after max_iters (result
 * kept), SNSW_E_DIVERGED on NaN/overflow.  Synchronous.
 *
 * With opts->precond, after the plain sweeps phi~ = S(phi_l) numbered
 * k, 2k, 3k, ... (k = precond_every) the element means of the residual,
 * rbar_e = mean over element e of (phi~ - phi_l), scaled by s = max|rbar|,
 * together with log(sigma_t)/5 and c = sigma_s/sigma_t, form the network
 * input on the element grid; the network output y gives
 * phi_{l+1} = phi~ + s*y_e on every node of element e.  Convergence is
 * judged by the plain-sweep residual only, so the fixed point is unchanged.
 * Safeguard: over the k sweeps after a correction the mean residual
 * reduction per sweep must beat the one of the latest window without a
 * correction (sweeps 1..k are plain; a window must span at least one sweep,
 * so with k = 1 the first correction follows sweep 2); otherwise the
 * correction counts as rejected and the next window is plain.  After 3 rejections the network is
 * not used again in this solve.                                             */
typedef struct snsw_net snsw_net;
typedef struct {
    double  tol;
    int32_t max_iters;
    int32_t check_every;         /* >= 1 (ignored with precond: every step) */
    snsw_net* precond;           /* learned correction (see above) or NULL  */
    int32_t precond_every;       /* correct after every k-th sweep (0 = 1)  */
} snsw_solve_opts;
typedef struct {
    int32_t iterations;
    double  residual;
    double  seconds;
    double* history;             /* caller buffer or NULL                    */
    int32_t history_cap;
    int32_t n_corrected;         /* steps the learned correction was applied */
    int32_t n_rejected;          /* steps it was skipped by the safeguard    */
} snsw_solve_report;
int snsw_solve(snsw_problem* prob, const snsw_solve_opts* opts, double* d_phi,
               double* d_psi, snsw_solve_report* report);

/* Relative L-infinity residual of two device scalar-flux vectors:
 * max|a-b| / max|a| in FP64 (synchronous).                                  */
int snsw_residual(snsw_problem* prob, const double* d_a, const double* d_b,
                  double* out);

/* --------------------------------------------------------------- profiling
 * While enabled, every level-sweep kernel launch is bracketed by two HIP
 * events on the ctx stream.  snsw_profile_read waits for the stream and
 * returns the number of level launches and their summed kernel time (ms)
 * since the last read, then clears the counters.                            */
int snsw_profile_enable(snsw_problem* prob, int enable);
int snsw_profile_read(snsw_problem* prob, int64_t* launches, double* kernel_ms);

/* ---------------------------------------------------------- checkpointing
 * Source-iteration state = the stored angular flux of the previous sweep.
 * snsw_state_size gives the bytes; save copies it to host memory, load
 * restores it (same problem shape; SNSW_E_STATE otherwise).  Synchronous.   */
int snsw_state_size(const snsw_problem* prob, size_t* bytes);
int snsw_state_save(const snsw_problem* prob, void* host_buf, size_t cap);
int snsw_state_load(snsw_problem* prob, const void* host_buf, size_t size);

/* ------------------------------------------------------ learned correction
 * A 3D U-Net over the element grid (nz, ny, nx) (nz = 1 for 2D problems):
 * 3x3x3 convolutions with zero padding and bias, leaky ReLU (slope 0.1),
 * widths (c0, c1, c2) at full, half and quarter resolution (stride-2
 * convolutions down, nearest-neighbour upsampling plus skip connections
 * up), 3 input channels (scaled residual mean, log(sigma_t)/5, c), one
 * output channel.  Parameters: FP32 masters, in layer order weights
 * [cout][cin][3][3][3] then bias [cout]; the convolutions use a BF16 copy of
 * the weights and accumulate in FP32.  The paper has no learned component
 * (it leaves the strongly scattering regime open); this is the project's.   */
typedef struct {
    int32_t  widths[3];          /* (c0, c1, c2), each in [1, 64]             */
    uint64_t seed;               /* initial weights: He-uniform from seed     */
} snsw_net_desc;
typedef struct {
    float lr, beta1, beta2, eps; /* Adam (bias-corrected)                      */
} snsw_adam;

int  snsw_net_create(snsw_ctx* ctx, const snsw_net_desc* desc, snsw_net** out);
void snsw_net_destroy(snsw_net* net);
int  snsw_net_n_params(const snsw_net* net, int64_t* n);
/* host float[n_params]; set also clears the Adam moments (synchronous)     */
int  snsw_net_get_params(const snsw_net* net, float* host);
int  snsw_net_set_params(snsw_net* net, const float* host);
/* gradient of the last backward pass, host float[n_params] (synchronous)   */
int  snsw_net_get_grads(const snsw_net* net, float* host);

/* d_x float [batch][3][nz][ny][nx] -> d_y float [batch][1][nz][ny][nx].
 * Keeps the activations for snsw_net_backward; d_x must stay unchanged
 * until then.                                                               */
int snsw_net_forward(snsw_net* net, const float* d_x, float* d_y, int32_t batch,
                     int32_t nz, int32_t ny, int32_t nx);
/* loss = mean((y - t)^2) over count values (FP64 accumulation) and
 * d_dy = 2 (y - t) / count (synchronous for the loss value).                */
int snsw_net_loss(snsw_net* net, const float* d_y, const float* d_t, int64_t count,
                  float* d_dy, double* loss);
/* Gradient of sum(d_dy * y) for the last forward pass: replaces the
 * parameter gradient; d_dx (nullable) receives the input gradient.          */
int snsw_net_backward(snsw_net* net, const float* d_dy, float* d_dx);
/* One Adam step on the masters with the current gradient; refreshes the
 * BF16 weights.                                                              */
int snsw_net_step(snsw_net* net, const snsw_adam* opt);

/* Training pair of one plain iteration phi_prev -> phi_swept of a problem
 * converged to phi_star: d_x float [3][E] network input (as in the solve),
 * d_t float [E] target mean(phi_star - phi_swept)_e / s (d_phi_star and d_t
 * nullable: input only).  Synchronous.                                      */
int snsw_learn_pair(snsw_problem* prob, const double* d_phi_prev, const double* d_phi_swept,
                    const double* d_phi_star, float* d_x, float* d_t);

/* snsw_learn_pair for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving or training loops, harnesses that
 * forbid hipMalloc): same arguments and results, but its element-mean
 * scratch lives in a static device array of the library instead of a
 * per-call allocation, and it is only enqueued on the problem's stream (not
 * synchronous; results are valid after the stream is synchronised).
 * Limit: E <= 2^20 elements (SNSW_E_SHAPE beyond).  The array is allocated
 * once per GPU when the library is loaded (16 MiB) and held until the
 * process ends; the call itself allocates nothing.  Every call on a GPU
 * shares that GPU's array, so calls on one GPU that overlap in time (on
 * different streams) race; calls on one stream are ordered.                 */
int snsw_learn_pair_noalloc(snsw_problem* prob, const double* d_phi_prev, const double* d_phi_swept,
                            const double* d_phi_star, float* d_x, float* d_t);

/* ------------------------------------------------------------------ batch
 * Many independent problems swept together (same context, device-backed,
 * each at most once per batch).  Problems with equal (dim, p, precision)
 * form a class: its schedule concatenates, level by level, the level
 * segments of its problems, so one persistent launch (or one launch per
 * level) sweeps all of them.  Each sweep of the batch is one captured
 * hipGraph replay (one graph per distinct set of flux pointers, at most 4
 * kept) or, with use_graph = 0, an eager launch sequence.
 *
 * opts (nullable: all fields 0):
 *   schedule   SNSW_SCHED_AUTO: the autotuner times, per class, the
 *              level schedule and the persistent one at full and half grid,
 *              and with single pairs instead of tiles per wavefront where
 *              the class has tiles (tune_reps sweeps each, default 3), and
 *              keeps the fastest;
 *              SNSW_SCHED_PERSISTENT / SNSW_SCHED_LEVELS force one for every
 *              class.  Classes of unstructured meshes, and mixed-precision
 *              classes other than 2D lattices with FP32 inverses, always
 *              use LEVELS.
 *   use_graph  0: eager launches; otherwise hipGraph replay.
 * Autotuning sweeps the member problems, so create leaves their stored
 * angular flux zero (as snsw_reset).  A batch refers to its problems'
 * device data: destroy the batch before any of its problems.  A problem may
 * also be swept on its own or through other batches between batch sweeps;
 * its lagged angular flux stays consistent.                                 */
typedef struct snsw_batch snsw_batch;
typedef struct {
    int32_t schedule;
    int32_t use_graph;
    int32_t tune_reps;
} snsw_batch_opts;

int  snsw_batch_create(snsw_ctx* ctx, snsw_problem* const* probs, int32_t count,
                       const snsw_batch_opts* opts, snsw_batch** out);
void snsw_batch_destroy(snsw_batch* batch);

/* One lagged sweep of every problem: d_phi_in[k] / d_phi_out[k] are device
 * scalar-flux vectors [E_k][n_k] of problem k (host arrays of count device
 * pointers; in and out must not alias).  Asynchronous on the ctx stream.    */
int snsw_batch_sweep(snsw_batch* batch, const double* const* d_phi_in,
                     double* const* d_phi_out);

/* Waits for the ctx stream; SNSW_E_STATE if a persistent dependency wait of
 * an earlier batch sweep timed out.                                         */
int snsw_batch_synchronize(snsw_batch* batch);

typedef struct {
    int32_t dim, dg_order, precision;
    int32_t persistent;          /* chosen schedule: 1 persistent, 0 levels   */
    int32_t blocks;              /* persistent grid (0 for levels)            */
    int32_t n_problems;
    int64_t n_levels;            /* levels of the merged schedule            */
    int64_t n_entries;           /* schedule entries incl. padding           */
    double  tuned_ms[4];         /* autotuner: levels, persistent full grid,
                                    persistent half grid, persistent full grid
                                    without tiles (ms per sweep; 0 if not
                                    timed)                                   */
    int32_t tiled;               /* chosen schedule takes tiles per wavefront */
} snsw_batch_class_info;
int snsw_batch_n_classes(const snsw_batch* batch, int32_t* n);
int snsw_batch_class_get(const snsw_batch* batch, int32_t c, snsw_batch_class_info* info);

#ifdef __cplusplus
}
#endif
#endif /* SNSWEEP_H */
