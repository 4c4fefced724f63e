"""Seeded synthetic workloads for the S_N sweep (inputs only).

This module produces the *inputs* of a problem: the control-point lattice of a
curved structured quad/hex mesh on the unit square/cube, per-element cross
sections and sources, and the angular-quadrature order.  It holds none of the
method's arithmetic (no basis functions, quadrature rules, operators or graph
work), so that both the CPU oracle and the GPU library can consume it without
sharing any code with each other.

Mesh recipe.  The domain is [0,1]^dim, split into nx[0] x nx[1] (x nx[2])
elements of geometric order r.  Control points sit on a global lattice of
(r*nx[a]+1) points per axis, equispaced in the reference coordinate
X_a = I_a / (r*nx[a]); each point is displaced by the warp
    W(X) = X + amp * prod_j sin(2*pi*freq*X_j) * (1, ..., 1),
which vanishes on the boundary of the unit box, so the domain stays [0,1]^dim.
Lattice points are ordered x fastest (then y, then z); element e = i + nx*(j +
ny*k) uses lattice points (r*i + a, r*j + b, r*k + c), a/b/c = 0..r.  Shared
faces therefore use bit-identical control points (mesh continuity, section 2,
"Discrete representation of the HO mesh").

Synthetic problems stand in for the paper's meshes (annulus, triple point,
Rayleigh-Taylor), which are not available: the configurations below follow the
sizes, orders, quadratures and material layouts of the workloads the
performance targets are quoted on.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

VACUUM = 0
ISO_CONST = 1
TABULATED = 2


@dataclass
class Problem:
    """Inputs of one steady mono-energetic S_N problem on a curved mesh."""
    name: str
    dim: int
    nx: tuple
    r: int                 # geometric order of the mesh map (Q_r)
    p: int                 # DG order (Q_p)
    sn_order: int          # level-symmetric S_N order (even)
    lattice: np.ndarray    # (n_lattice, dim) float64 control points
    sigma_t: np.ndarray    # (E,) float64
    sigma_s: np.ndarray    # (E,) float64
    q: np.ndarray          # (E,) float64 isotropic source per steradian
    bc_kind: int = VACUUM
    psi_inc: float = 0.0   # constant isotropic inflow for ISO_CONST
    tol: float = 1e-10
    weighting: int = 1     # 0 unity, 1 face, 2 sigma-inverse face
    exact_scc_max: int = 10
    meta: dict = field(default_factory=dict)
    # optional direction-dependent data, nodal values at the DG nodes:
    q_dir: Optional[np.ndarray] = None        # (D, E, n) source per direction (replaces q)
    psi_inc_tab: Optional[np.ndarray] = None  # (D, E, n) incident flux (bc_kind TABULATED)
    # optional unstructured conforming mesh (then `lattice` is unused and nx
    # is (E, 1[, 1])): global control points and, per element, the indices of
    # its (r+1)^dim control points in local lexicographic order (x fastest);
    # elements sharing a face share its control points (in any orientation)
    nodes: Optional[np.ndarray] = None        # (n_nodes, dim) float64
    elem_nodes: Optional[np.ndarray] = None   # (E, (r+1)^dim) int64
    # "tensor" (quadrilaterals / hexahedra) or "simplex" (P_r triangles /
    # tetrahedra: then elem_nodes lists the element's control points in the
    # lattice order of tri_lattice / tet_lattice, and n = (p+1)(p+2)/2 /
    # (p+1)(p+2)(p+3)/6)
    element: str = "tensor"
    # integration of the face matrices on faces where Omega . n changes sign:
    # "exact" (2D: split at the roots; 3D: fixed composite rule) or
    # "romberg" (adaptive Romberg to the relative tolerance face_tol)
    face_rule: str = "exact"
    face_tol: float = 1e-10

    @property
    def n_elements(self) -> int:
        return int(np.prod(self.nx))

    @property
    def n_dof(self) -> int:
        if self.element == "simplex":
            k = self.p
            return (k + 1) * (k + 2) // 2 if self.dim == 2 else (k + 1) * (k + 2) * (k + 3) // 6
        return (self.p + 1) ** self.dim

    @property
    def n_dirs(self) -> int:
        n = self.sn_order
        return n * (n + 2) // 2 if self.dim == 2 else n * (n + 2)


def lattice_shape(dim: int, nx, r: int) -> tuple:
    return tuple(r * int(nx[a]) + 1 for a in range(dim))


def make_lattice(dim: int, nx, r: int, amp: float, freq: int) -> np.ndarray:
    """Warped control-point lattice, x fastest.  See the module docstring."""
    shape = lattice_shape(dim, nx, r)
    axes = [np.arange(shape[a], dtype=np.float64) / (r * nx[a]) for a in range(dim)]
    # meshgrid with 'ij' then transpose so that x is the fastest index
    grids = np.meshgrid(*axes[::-1], indexing="ij")[::-1]
    X = np.stack([g.reshape(-1) for g in grids], axis=1)
    bump = np.ones(X.shape[0])
    for a in range(dim):
        bump = bump * np.sin(2.0 * math.pi * freq * X[:, a])
    return X + amp * bump[:, None]


def element_ijk(dim: int, nx) -> np.ndarray:
    """(E, dim) integer element indices, e = i + nx*(j + ny*k)."""
    E = int(np.prod(nx))
    e = np.arange(E)
    out = np.zeros((E, dim), dtype=np.int64)
    rem = e.copy()
    for a in range(dim):
        out[:, a] = rem % nx[a]
        rem //= nx[a]
    return out


def make_problem(name: str, dim: int, nx, r: int, p: int, sn_order: int,
                 amp: float, freq: int, sigma_t, c, q, *, bc_kind=VACUUM,
                 psi_inc=0.0, tol=1e-10, weighting=1, exact_scc_max=10,
                 meta: Optional[dict] = None) -> Problem:
    nx = tuple(int(v) for v in nx)
    E = int(np.prod(nx))
    st = np.broadcast_to(np.asarray(sigma_t, dtype=np.float64), (E,)).copy()
    cc = np.broadcast_to(np.asarray(c, dtype=np.float64), (E,)).copy()
    qq = np.broadcast_to(np.asarray(q, dtype=np.float64), (E,)).copy()
    return Problem(name=name, dim=dim, nx=nx, r=r, p=p, sn_order=sn_order,
                   lattice=make_lattice(dim, nx, r, amp, freq),
                   sigma_t=st, sigma_s=cc * st, q=qq, bc_kind=bc_kind,
                   psi_inc=float(psi_inc), tol=tol, weighting=weighting,
                   exact_scc_max=exact_scc_max,
                   meta=dict(meta or {}, amp=amp, freq=freq))


# --------------------------------------------------------------------------
# Named configurations
# --------------------------------------------------------------------------

def c1() -> Problem:
    """2D 8x8 Q2 mesh, warp 0.05, p=1, S4, sigma_t=1, c=0.5, q=1, vacuum."""
    return make_problem("c1_2d_8x8_q2_p1_s4", 2, (8, 8), 2, 1, 4, 0.05, 1,
                        1.0, 0.5, 1.0, tol=1e-10)


def c2() -> Problem:
    """2D 128x128 Q3 mesh warped by 0.3 element widths with a 4-element
    wavelength (cycles in the sweep graph), p=3, S8, sigma_t=1, c=0.8, q=1."""
    return make_problem("c2_2d_128x128_q3_p3_s8", 2, (128, 128), 3, 3, 8,
                        0.3 / 128, 32, 1.0, 0.8, 1.0, tol=1e-8)


def c3() -> Problem:
    """3D 32^3 Q2 mesh, p=2, S8, checkerboard sigma_t in {1,10} (8^3 blocks),
    c=0.9, q=1 in the central 8^3 block, vacuum."""
    nx = (32, 32, 32)
    ijk = element_ijk(3, nx)
    odd = ((ijk[:, 0] // 8 + ijk[:, 1] // 8 + ijk[:, 2] // 8) % 2) == 1
    st = np.where(odd, 10.0, 1.0)
    inside = np.all((ijk >= 12) & (ijk <= 19), axis=1)
    q = np.where(inside, 1.0, 0.0)
    return make_problem("c3_3d_32cube_q2_p2_s8", 3, nx, 2, 2, 8, 0.05, 1,
                        st, 0.9, q, tol=1e-8)


def c4(seed: int = 0, count: int = 64) -> List[Problem]:
    """Batch of independent 2D problems drawn from a seed."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        m = int(rng.integers(16, 97))
        p = int(rng.integers(1, 4))
        N = 2 * int(rng.integers(2, 7))
        st = float(10.0 ** rng.uniform(-1.0, 1.0))
        c = float(rng.uniform(0.0, 0.95))
        out.append(make_problem(f"c4_{b}_2d_{m}x{m}_q2_p{p}_s{N}", 2, (m, m), 2,
                                p, N, 0.05, 1, st, c, 1.0, tol=1e-8))
    return out


def c5(seed: int = 100, nx: int = 48, sn_order: int = 12) -> Problem:
    """3D 48^3 Q2 mesh, p=2, S12, c=0.99, random two-material layout with
    sigma_t in {1,100}, q=1 everywhere, vacuum."""
    dims = (nx, nx, nx)
    E = nx ** 3
    rng = np.random.default_rng(seed)
    st = np.where(rng.random(E) < 0.5, 100.0, 1.0)
    return make_problem(f"c5_3d_{nx}cube_q2_p2_s{sn_order}_seed{seed}", 3, dims,
                        2, 2, sn_order, 0.05, 1, st, 0.99, 1.0, tol=1e-8)


def c5_reduced(seed: int = 100, nx: int = 12, p: int = 1, sn_order: int = 4) -> Problem:
    """The 48^3 two-material c = 0.99 family at a size where plain source
    iteration converges in seconds: nx^3 Q2 mesh (warp 0.05), sigma_t = 100
    where default_rng(seed).random(E) < 0.5 else 1, c = 0.99, q = 1, vacuum."""
    dims = (nx, nx, nx)
    E = nx ** 3
    rng = np.random.default_rng(seed)
    st = np.where(rng.random(E) < 0.5, 100.0, 1.0)
    return make_problem(f"c5r_3d_{nx}cube_q2_p{p}_s{sn_order}_seed{seed}", 3, dims,
                        2, p, sn_order, 0.05, 1, st, 0.99, 1.0, tol=1e-8)


def element_centres(dim: int, nx, r: int, lattice: np.ndarray) -> np.ndarray:
    """(E, dim) mean of each element's control points (used to place
    analytic sources on elements)."""
    shape = lattice_shape(dim, nx, r)
    grid = lattice.reshape(tuple(reversed(shape)) + (dim,))
    ijk = element_ijk(dim, nx)
    out = np.zeros((len(ijk), dim))
    for e, idx in enumerate(ijk):
        sl = tuple(slice(r * idx[a], r * idx[a] + r + 1) for a in reversed(range(dim)))
        out[e] = grid[sl].reshape(-1, dim).mean(axis=0)
    return out


def strong_warp_amp(dim: int, slope: float, freq: int) -> float:
    """Warp amplitude whose largest slope amp*2*pi*freq is `slope`.  The
    Jacobian determinant of the warp is 1 + sum_a dW/dX_a >= 1 - slope in 2D
    and >= 1 - 1.155 slope in 3D (the largest of sum_a of the partial
    derivatives of prod_j sin), so slope < 1 (2D) / < 0.866 (3D) keeps the
    map invertible."""
    return slope / (2.0 * math.pi * freq)


def cyclic_2d(n: int = 32, freq: int = 8, slope: float = 0.9, p: int = 2, sn_order: int = 8,
              c: float = 0.9) -> Problem:
    """Strongly warped 2D n x n Q3 mesh: faces tilt past the directions of
    the quadrature, so the sweep graphs have cycles (at n = 32, S8: up to 4
    elements per cycle with freq 8, up to 16 with freq 4); p, S_N,
    sigma_t = 1, scattering ratio c, q = 1, vacuum."""
    return make_problem(f"cyc_2d_{n}x{n}_q3_f{freq}_s{slope}_p{p}_s{sn_order}", 2, (n, n), 3, p, sn_order,
                        strong_warp_amp(2, slope, freq), freq, 1.0, c, 1.0, tol=1e-8)


def standin_2d(nx: int = 16, ny: int = 21, slope: float = 0.9, p: int = 2) -> Problem:
    """Stand-in shaped like the paper's 2D weighting tests (336 or 1344 Q3
    elements, S2, sigma_s = 1, sigma_t = 2, q = 1 + sin^2(2x + y), isotropic
    inflow 1) on a strongly warped unit square (warp frequency nx/4) instead
    of the paper's meshes, which are not available; q is evaluated at
    element centres."""
    freq = max(1, nx // 4)
    lat = make_lattice(2, (nx, ny), 3, strong_warp_amp(2, slope, freq), freq)
    xc = element_centres(2, (nx, ny), 3, lat)
    q = 1.0 + np.sin(2.0 * xc[:, 0] + xc[:, 1]) ** 2
    wp = make_problem(f"standin_2d_{nx}x{ny}_q3_p{p}_s2", 2, (nx, ny), 3, p, 2,
                      strong_warp_amp(2, slope, freq), freq, 2.0, 0.5, q, bc_kind=ISO_CONST,
                      psi_inc=1.0, tol=1e-8)
    return wp


def standin_3d(slope: float = 0.8, p: int = 2) -> Problem:
    """Stand-in shaped like the paper's 3D weighting test (8 x 8 x 4 Q3
    elements, S2, sigma_s = 1, sigma_t = 2, q = 1 + sin^2(4x + 2yz + 2y),
    isotropic inflow 1) on a strongly warped unit cube (warp frequency 2)."""
    nx = (8, 8, 4)
    freq = 2
    lat = make_lattice(3, nx, 3, strong_warp_amp(3, slope, freq), freq)
    xc = element_centres(3, nx, 3, lat)
    q = 1.0 + np.sin(4.0 * xc[:, 0] + 2.0 * xc[:, 1] * xc[:, 2] + 2.0 * xc[:, 1]) ** 2
    return make_problem(f"standin_3d_8x8x4_q3_p{p}_s2", 3, nx, 3, p, 2,
                        strong_warp_amp(3, slope, freq), freq, 2.0, 0.5, q, bc_kind=ISO_CONST,
                        psi_inc=1.0, tol=1e-8)


def annulus_quarter(nr: int = 9, nt: int = 15, p: int = 3, sn_order: int = 4, r_in: float = 1.0,
                    r_out: float = 2.0) -> Problem:
    """Quarter annulus r in [r_in, r_out], theta in [0, pi/2], nr x nt Q3
    elements (radial index fastest), control points on circles, so the arcs
    are curved boundaries and curved interior faces; three nested rings of
    equal width with sigma_t = 2.0, 2.2, 2.4 and sigma_s = 1 (the material
    table of the paper's nested-annuli problem, whose dimensions are not
    given), q = 1, vacuum.  A quarter of the paper's coarse and refined HO
    element counts (540, 2160) is 9 x 15 and 18 x 30."""
    r = 3
    unit = make_lattice(2, (nr, nt), r, 0.0, 1)
    rad = r_in + (r_out - r_in) * unit[:, 0]
    th = 0.5 * math.pi * unit[:, 1]
    lattice = np.stack([rad * np.cos(th), rad * np.sin(th)], axis=1)
    ring = np.minimum(element_ijk(2, (nr, nt))[:, 0] * 3 // nr, 2)
    st = np.array([2.0, 2.2, 2.4])[ring]
    E = nr * nt
    return Problem(name=f"annulus_quarter_{nr}x{nt}_q3_p{p}_s{sn_order}", dim=2, nx=(nr, nt), r=r, p=p,
                   sn_order=sn_order, lattice=lattice, sigma_t=st, sigma_s=np.ones(E), q=np.ones(E),
                   tol=1e-8, meta=dict(r_in=r_in, r_out=r_out))


def small(dim=2, n=4, r=2, p=1, N=4, amp=0.05, freq=1, sigma_t=1.0, c=0.5,
          q=1.0, **kw) -> Problem:
    nx = (n,) * dim if np.isscalar(n) else tuple(n)
    return make_problem(f"small_{dim}d_{'x'.join(map(str, nx))}_q{r}_p{p}_s{N}",
                        dim, nx, r, p, N, amp, freq, sigma_t, c, q, **kw)


def random_problem(seed: int, dim: int = 2) -> Problem:
    """A small random problem for parity sweeps (ragged sizes, mixed media)."""
    rng = np.random.default_rng(seed)
    # the warp's maximum slope amp*2*pi*freq is drawn directly; the Jacobian
    # determinant of the warp stays >= 1 - dim*slope > 0
    if dim == 2:
        nx = (int(rng.integers(3, 13)), int(rng.integers(3, 13)))
        r = int(rng.integers(1, 4))
        p = int(rng.integers(1, 4))
        N = int(2 * rng.integers(1, 5))
        freq = int(rng.integers(1, max(2, min(nx) // 2 + 1)))
        slope = float(rng.uniform(0.0, 0.45))
    else:
        nx = tuple(int(v) for v in rng.integers(2, 6, size=3))
        r = int(rng.integers(1, 3))
        p = int(rng.integers(1, 3))
        N = int(2 * rng.integers(1, 4))
        freq = int(rng.integers(1, 3))
        slope = float(rng.uniform(0.0, 0.25))
    amp = slope / (2.0 * math.pi * freq)
    E = int(np.prod(nx))
    st = 10.0 ** rng.uniform(-1, 1, size=E)
    c = rng.uniform(0.0, 0.9, size=E)
    q = rng.uniform(0.0, 2.0, size=E)
    bc = int(rng.integers(0, 2))
    return make_problem(f"rand{seed}_{dim}d", dim, nx, r, p, N, amp, freq, st, c,
                        q, bc_kind=bc, psi_inc=float(rng.uniform(0, 1)) * bc,
                        weighting=int(rng.integers(0, 3)))


CONFIGS = {"c1": c1, "c2": c2, "c3": c3, "c5": c5}


def sweep_inputs(prob: Problem, seed: int, directions) -> tuple:
    """Seeded inputs of one lagged sweep: scalar flux phi0 (E, n) uniform in
    [0, 2], and for each listed direction d its lagged angular flux (E, n)
    uniform in [0, 0.2] from its own stream default_rng([seed, d]), so that
    the rows of any subset of directions are the same whichever subset is
    drawn.  Returns (phi0, {d: psi0_d})."""
    E, n = prob.n_elements, prob.n_dof
    phi0 = np.random.default_rng([seed, 1 << 20]).uniform(0.0, 2.0, (E, n))
    psi0 = {int(d): np.random.default_rng([seed, int(d)]).uniform(0.0, 0.2, (E, n)) for d in directions}
    return phi0, psi0


def sample_elements(prob: Problem, seed: int, count: int) -> np.ndarray:
    """Sorted distinct element ids drawn from default_rng(seed), plus the
    first and last element (the corners a sweep starts or ends at)."""
    E = prob.n_elements
    rng = np.random.default_rng(seed)
    pick = rng.choice(E, size=min(count, E), replace=False)
    return np.unique(np.concatenate([pick, [0, E - 1]])).astype(np.int64)


def corner_block(prob: Problem, m: int) -> Problem:
    """The m x m (x m) corner block of elements 0 <= i, j (, k) < m of a
    structured problem, as a problem of its own: the same control points,
    materials and source on those elements (a bounded sample of a large
    workload; its outer faces become vacuum boundaries)."""
    dim, r = prob.dim, prob.r
    nx = tuple(int(v) for v in prob.nx)
    m = min(m, min(nx))
    shape = lattice_shape(dim, nx, r)
    grid = prob.lattice.reshape(tuple(reversed(shape)) + (dim,))
    sl = tuple(slice(0, r * m + 1) for _ in range(dim))
    lat = np.ascontiguousarray(grid[sl]).reshape(-1, dim)
    ijk = element_ijk(dim, nx)
    keep = np.all(ijk < m, axis=1)
    sub = tuple([m] * dim)
    return replace(prob, name=f"{prob.name}_corner{m}", nx=sub, lattice=lat,
                   sigma_t=prob.sigma_t[keep].copy(), sigma_s=prob.sigma_s[keep].copy(),
                   q=prob.q[keep].copy(), meta=dict(prob.meta, corner_of=prob.name, corner=m))


def random_direction_data(prob: Problem, n_dirs: int, seed: int) -> tuple:
    """Seeded nodal data per direction: a source q_dir uniform in [0, 2] and
    an incident flux uniform in [0.5, 1.5], both (D, E, n)."""
    rng = np.random.default_rng(seed)
    shape = (n_dirs, prob.n_elements, prob.n_dof)
    return rng.uniform(0.0, 2.0, shape), rng.uniform(0.5, 1.5, shape)


def mms_annular(xyz: np.ndarray, omega: np.ndarray, w: np.ndarray, sigma_t, sigma_s) -> tuple:
    """The manufactured solution of the paper's annulus test (eq.
    psiAnnularMMS), psi_d(x, y) = f(x, y) (mu_d^2 + eta_d) with
    f = (1 + x^2 + y^2)/2 + cos(3x + 3y/2), evaluated at given points xyz
    (..., dim) for every direction: returns (q, psi, phi) with
      q_d   = Omega_d . grad psi_d + sigma_t psi_d - sigma_s/(4 pi) phi,
      psi_d the solution, phi = sum_d w_d psi_d (with the quadrature given,
    so that the discrete problem has psi as its exact solution up to the
    discretisation error); sigma_t, sigma_s broadcast against xyz[..., 0].
    Shapes (D,) + xyz.shape[:-1]."""
    x, y = xyz[..., 0], xyz[..., 1]
    f = 0.5 * (1.0 + x * x + y * y) + np.cos(3.0 * x + 1.5 * y)
    sn = np.sin(3.0 * x + 1.5 * y)
    fx, fy = x - 3.0 * sn, y - 1.5 * sn
    a = omega[:, 0] ** 2 + omega[:, 1]                       # (D,)
    aw = float(np.dot(w, a))
    st = np.broadcast_to(np.asarray(sigma_t, dtype=np.float64), x.shape)
    ss = np.broadcast_to(np.asarray(sigma_s, dtype=np.float64), x.shape)
    psi = a[:, None] * f.reshape(1, -1)
    grad = omega[:, 0:1] * fx.reshape(1, -1) + omega[:, 1:2] * fy.reshape(1, -1)
    q = a[:, None] * grad + st.reshape(1, -1) * psi - ss.reshape(1, -1) / (4.0 * np.pi) * aw * f.reshape(1, -1)
    shp = (len(a),) + x.shape
    return q.reshape(shp), psi.reshape(shp), (aw * f)


def straightened(prob: Problem, p: int = 1) -> Problem:
    """The low-order mesh of a Q_r problem refined r times per axis: every
    element is split into r^dim sub-elements whose vertices are its control
    points (equispaced in the reference element, so they lie on the curved
    element: the straightening of the paper's high-order vs low-order
    comparison with N_ref = r), as a Q_1 problem on the same lattice with DG
    order p; each sub-element keeps its parent's materials and source."""
    r, dim = prob.r, prob.dim
    nx = tuple(int(v) for v in prob.nx)
    sub = tuple(r * v for v in nx)
    ijk = element_ijk(dim, sub)
    parent = np.zeros(len(ijk), dtype=np.int64)
    stride = 1
    for a in range(dim):
        parent += (ijk[:, a] // r) * stride
        stride *= nx[a]
    return replace(prob, name=f"{prob.name}_straightened", nx=sub, r=1, p=p, lattice=prob.lattice.copy(),
                   sigma_t=prob.sigma_t[parent].copy(), sigma_s=prob.sigma_s[parent].copy(),
                   q=prob.q[parent].copy(), q_dir=None, psi_inc_tab=None,
                   meta=dict(prob.meta, straightened_from=prob.name, n_ref=r))


# --------------------------------------------------------------------------
# Unstructured conforming meshes (explicit element -> control point lists)
# --------------------------------------------------------------------------

def rotations(dim: int) -> List[np.ndarray]:
    """The orientation-preserving symmetries of the reference square (4) or
    cube (24) as signed permutation matrices with determinant +1."""
    import itertools
    out = []
    for perm in itertools.permutations(range(dim)):
        for signs in itertools.product((1, -1), repeat=dim):
            R = np.zeros((dim, dim), dtype=np.int64)
            for i, j in enumerate(perm):
                R[i, j] = signs[i]
            if round(np.linalg.det(R)) == 1:
                out.append(R)
    return out


def local_index_map(dim: int, n1: int, R: np.ndarray) -> np.ndarray:
    """For a local grid of n1 points per axis (lexicographic, x fastest) and a
    rotation R of the reference element about its centre: old[m] = index of
    the point that moves to new index m, so new_values = old_values[old]."""
    m = np.arange(n1 ** dim)
    idx = np.stack([(m // n1 ** a) % n1 for a in range(dim)], axis=1)   # new positions
    c = 2 * idx - (n1 - 1)                                             # centred, doubled
    old_c = c @ R          # new = R old  ->  old = R^T new  (rows: c_new @ R = (R^T c_new)^T)
    old_idx = (old_c + (n1 - 1)) // 2
    return sum(old_idx[:, a] * n1 ** a for a in range(dim))


def unstructured_from_elements(name: str, dim: int, r: int, p: int, sn_order: int, nodes: np.ndarray,
                               elem_nodes: np.ndarray, sigma_t, sigma_s, q, seed: Optional[int] = None,
                               **kw) -> Problem:
    """An unstructured problem from element control-point lists; with a seed
    the elements are renumbered at random and each element's local frame is
    turned by a random rotation (so neighbours meet through arbitrary slot
    pairs and face orientations).  The applied permutation and rotations are
    kept in meta ('perm': new element k is old element perm[k]; 'rot': index
    of the rotation in rotations(dim) for new element k)."""
    E = len(elem_nodes)
    st = np.broadcast_to(np.asarray(sigma_t, dtype=np.float64), (E,)).copy()
    ss = np.broadcast_to(np.asarray(sigma_s, dtype=np.float64), (E,)).copy()
    qq = np.broadcast_to(np.asarray(q, dtype=np.float64), (E,)).copy()
    en = np.asarray(elem_nodes, dtype=np.int64).copy()
    perm = np.arange(E)
    rot = np.zeros(E, dtype=np.int64)
    if seed is not None:
        rng = np.random.default_rng(seed)
        perm = rng.permutation(E)
        rots = rotations(dim)
        rot = rng.integers(0, len(rots), size=E)
        maps = [local_index_map(dim, r + 1, R) for R in rots]
        en = np.stack([en[perm[k]][maps[rot[k]]] for k in range(E)])
        st, ss, qq = st[perm], ss[perm], qq[perm]
    meta = dict(kw.pop("meta", {}), perm=perm, rot=rot, unstructured=True)
    nx = (E,) + (1,) * (dim - 1)
    return Problem(name=name, dim=dim, nx=nx, r=r, p=p, sn_order=sn_order, lattice=np.zeros((0, dim)),
                   sigma_t=st, sigma_s=ss, q=qq, nodes=np.asarray(nodes, dtype=np.float64),
                   elem_nodes=en, meta=meta, **kw)


def structured_element_nodes(dim: int, nx, r: int) -> np.ndarray:
    """(E, (r+1)^dim) lattice indices of the control points of each element
    of a structured lattice (the lattice layout of the module docstring)."""
    L = lattice_shape(dim, nx, r)
    ijk = element_ijk(dim, nx)
    n1 = r + 1
    m = np.arange(n1 ** dim)
    loc = np.stack([(m // n1 ** a) % n1 for a in range(dim)], axis=1)
    flat = np.zeros((len(ijk), len(m)), dtype=np.int64)
    stride = 1
    for a in range(dim):
        flat += (r * ijk[:, a][:, None] + loc[:, a][None, :]) * stride
        stride *= L[a]
    return flat


def as_unstructured(prob: Problem, seed: int = 0) -> Problem:
    """The same mesh and materials given as an unstructured element list,
    renumbered and locally rotated at random (seeded)."""
    en = structured_element_nodes(prob.dim, prob.nx, prob.r)
    return unstructured_from_elements(f"{prob.name}_unstructured{seed}", prob.dim, prob.r, prob.p,
                                      prob.sn_order, prob.lattice, en, prob.sigma_t, prob.sigma_s, prob.q,
                                      seed=seed, bc_kind=prob.bc_kind, psi_inc=prob.psi_inc, tol=prob.tol,
                                      weighting=prob.weighting, exact_scc_max=prob.exact_scc_max,
                                      meta=dict(prob.meta, structured_from=prob.name))


def _merge_nodes(points: np.ndarray, ndigits: int = 9):
    """Unique control points (by coordinates rounded to ndigits) and the index
    of each input point among them."""
    keys = np.round(points, ndigits)
    _, first, inv = np.unique(keys, axis=0, return_index=True, return_inverse=True)
    return points[first], inv.reshape(-1)


def annulus_full(nr: int = 4, nt: int = 16, p: int = 2, sn_order: int = 4, r: int = 3, r_in: float = 1.0,
                 r_out: float = 2.0, seed: Optional[int] = 1) -> Problem:
    """Full annulus r in [r_in, r_out] (theta periodic: the mesh closes on
    itself, which no structured lattice can express), nr x nt elements of
    order r with control points on circles, three nested material rings
    (sigma_t = 2.0, 2.2, 2.4, sigma_s = 1), q = 1, vacuum; renumbered and
    locally rotated at random (seed)."""
    n1 = r + 1
    m = np.arange(n1 * n1)
    a, b = m % n1, m // n1
    i, j = np.meshgrid(np.arange(nr), np.arange(nt), indexing="ij")
    i, j = i.reshape(-1), j.reshape(-1)
    ri = r * i[:, None] + a[None, :]                    # radial node index
    tj = (r * j[:, None] + b[None, :]) % (r * nt)       # angular node index (periodic)
    elem = ri * (r * nt) + tj
    rr = r_in + (r_out - r_in) * np.arange(r * nr + 1) / (r * nr)
    th = 2.0 * math.pi * np.arange(r * nt) / (r * nt)
    R, T = np.meshgrid(rr, th, indexing="ij")
    nodes = np.stack([(R * np.cos(T)).reshape(-1), (R * np.sin(T)).reshape(-1)], axis=1)
    ring = np.minimum(i * 3 // nr, 2)
    st = np.array([2.0, 2.2, 2.4])[ring]
    return unstructured_from_elements(f"annulus_{nr}x{nt}_q{r}_p{p}_s{sn_order}", 2, r, p, sn_order, nodes, elem,
                                      st, 1.0, 1.0, seed=seed, tol=1e-8,
                                      meta=dict(r_in=r_in, r_out=r_out))


def disk_ogrid(n: int = 3, m: int = 2, p: int = 2, sn_order: int = 4, r: int = 2, seed: Optional[int] = 2) -> Problem:
    """Unit disk as a five-block O-grid: a central square [-h, h]^2 of n x n
    elements and four blocks of m x n elements joining its sides to the
    circle (the square's corners are vertices of three elements, so the mesh
    is not a lattice).  Order-r elements; the outer blocks blend the square
    side into the circular arc.  sigma_t = 1 inside the square, 2 outside,
    c = 0.5, q = 1, vacuum; renumbered and locally rotated at random."""
    h = 0.45
    n1 = r + 1
    loc = np.arange(n1 * n1)
    la, lb = (loc % n1) / r, (loc // n1) / r
    pts, mats = [], []
    # central square, element (i, j): x = -h + 2h (i + a)/n
    for jj in range(n):
        for ii in range(n):
            x = -h + 2 * h * (ii + la) / n
            y = -h + 2 * h * (jj + lb) / n
            pts.append(np.stack([x, y], axis=1))
            mats.append(1.0)
    # outer blocks: side k of the square (counter-clockwise), xi along the
    # side, eta outward; the inner edge is the square side, the outer the arc
    for k in range(4):
        ang0 = -0.25 * math.pi + 0.5 * math.pi * k
        c0, s0 = math.cos(0.5 * math.pi * k), math.sin(0.5 * math.pi * k)
        # local axes (outward, counter-clockwise along the side): right-handed
        for ii in range(n):
            for jj in range(m):
                eta = (jj + la) / m
                xi = (ii + lb) / n
                # square side point (rotated copy of the right side x = h)
                sx, sy = h, -h + 2 * h * xi
                ix, iy = c0 * sx - s0 * sy, s0 * sx + c0 * sy
                phi = ang0 + 0.5 * math.pi * xi
                ox, oy = np.cos(phi), np.sin(phi)
                pts.append(np.stack([(1 - eta) * ix + eta * ox, (1 - eta) * iy + eta * oy], axis=1))
                mats.append(2.0)
    allp = np.concatenate(pts)
    nodes, inv = _merge_nodes(allp)
    elem = inv.reshape(len(pts), n1 * n1)
    st = np.array(mats)
    return unstructured_from_elements(f"disk_ogrid_{n}x{m}_q{r}_p{p}_s{sn_order}", 2, r, p, sn_order, nodes, elem,
                                      st, 0.5 * st, 1.0, seed=seed, tol=1e-8)


def annulus_shell_3d(nr: int = 2, nt: int = 8, nz: int = 2, p: int = 2, sn_order: int = 4, r: int = 2,
                     r_in: float = 1.0, r_out: float = 2.0, height: float = 1.0,
                     seed: Optional[int] = 3) -> Problem:
    """Cylindrical shell r in [r_in, r_out], theta periodic, z in [0, height],
    nr x nt x nz elements of order r (control points on circles), sigma_t = 1
    in the inner half of the radius and 3 in the outer, c = 0.5, q = 1,
    vacuum; renumbered and locally rotated at random (any of the 24 rotations
    of the reference cube, so faces meet in all eight orientations)."""
    n1 = r + 1
    m = np.arange(n1 ** 3)
    a, b, c = m % n1, (m // n1) % n1, m // (n1 * n1)
    i, j, k = np.meshgrid(np.arange(nr), np.arange(nt), np.arange(nz), indexing="ij")
    i, j, k = i.reshape(-1), j.reshape(-1), k.reshape(-1)
    NR, NT, NZ = r * nr + 1, r * nt, r * nz + 1
    ri = r * i[:, None] + a[None, :]
    tj = (r * j[:, None] + b[None, :]) % NT
    zk = r * k[:, None] + c[None, :]
    elem = (ri * NT + tj) * NZ + zk
    rr = r_in + (r_out - r_in) * np.arange(NR) / (NR - 1)
    th = 2.0 * math.pi * np.arange(NT) / NT
    zz = height * np.arange(NZ) / (NZ - 1)
    R, T, Z = np.meshgrid(rr, th, zz, indexing="ij")
    nodes = np.stack([(R * np.cos(T)).reshape(-1), (R * np.sin(T)).reshape(-1), Z.reshape(-1)], axis=1)
    st = np.where(i * 2 < nr, 1.0, 3.0)
    return unstructured_from_elements(f"shell3d_{nr}x{nt}x{nz}_q{r}_p{p}_s{sn_order}", 3, r, p, sn_order, nodes,
                                      elem, st, 0.5 * st, 1.0, seed=seed, tol=1e-8)


# ---------------------------------------------------------------- triangles
def tri_lattice(k: int) -> np.ndarray:
    """(n, 2) lattice pairs (i, j), i + j <= k, of the nodes of order k on a
    triangle, row by row (j slowest): the local order of a simplex element's
    control points (reference position (i / k, j / k) for vertices v0 = (0, 0),
    v1 = (1, 0), v2 = (0, 1))."""
    return np.array([(i, j) for j in range(k + 1) for i in range(k + 1 - j)], dtype=np.int64)


def tri_rotation_map(r: int, turns: int) -> np.ndarray:
    """Local index map of a triangle whose vertex order is turned `turns`
    times (v0, v1, v2) -> (v1, v2, v0): new local node k is old node map[k]."""
    L = tri_lattice(r)
    idx = {(int(i), int(j)): k for k, (i, j) in enumerate(L)}
    out = np.arange(len(L))
    for _ in range(turns % 3):
        # new (i', j') is the old node with barycentrics lambda_v1 = 1 - (i'+j')/r, lambda_v2 = i'/r
        out = np.array([out[idx[(r - int(i) - int(j), int(i))]] for i, j in L])
    return out


def triangulated(name: str, r: int, p: int, sn_order: int, nx: int, ny: int, x_of, sigma_t, sigma_s, q,
                 periodic_v: bool = False, seed: Optional[int] = None, **kw) -> Problem:
    """Triangles from an nx x ny grid of cells on the parameter square
    [0, 1]^2, each cell cut along one diagonal (alternating), counter-clockwise
    in parameter space, mapped by x_of(u, v) -> (x, y) (orientation
    preserving): each triangle's control points are the map at its order-r
    lattice points, so triangles are curved wherever the map is not affine.
    periodic_v: v = 1 is glued to v = 0 (a closed ring).  sigma_t, sigma_s, q:
    per element or callables of the cell centre (u, v).  With a seed the
    elements are renumbered and each element's vertex order turned at
    random (meta 'perm', 'turns')."""
    fu, fv = r * nx + 1, r * ny + (0 if periodic_v else 1)
    U, V = np.meshgrid(np.arange(fu) / (r * nx), np.arange(fv) / (r * ny), indexing="xy")   # u fastest
    X = x_of(U.reshape(-1), V.reshape(-1))
    nodes = np.stack([np.asarray(X[0], dtype=np.float64), np.asarray(X[1], dtype=np.float64)], axis=1)
    L = tri_lattice(r)
    elems, centres = [], []
    for cj in range(ny):
        for ci in range(nx):
            P00, P10, P01, P11 = (r * ci, r * cj), (r * (ci + 1), r * cj), (r * ci, r * (cj + 1)), \
                (r * (ci + 1), r * (cj + 1))
            tris = [(P00, P10, P11), (P00, P11, P01)] if (ci + cj) % 2 == 0 else \
                [(P00, P10, P01), (P10, P11, P01)]
            for A, B, C in tris:
                ids = []
                for i, j in L:
                    fi = A[0] + i * (B[0] - A[0]) // r + j * (C[0] - A[0]) // r
                    fj = A[1] + i * (B[1] - A[1]) // r + j * (C[1] - A[1]) // r
                    ids.append(fi + fu * (fj % fv if periodic_v else fj))
                elems.append(ids)
                centres.append(((A[0] + B[0] + C[0]) / (3.0 * r * nx), (A[1] + B[1] + C[1]) / (3.0 * r * ny)))
    en = np.array(elems, dtype=np.int64)
    cu, cv = np.array(centres).T
    E = len(en)

    def per_elem(v):
        return np.asarray(v(cu, cv) if callable(v) else np.broadcast_to(v, (E,)), dtype=np.float64).copy()

    st, ss, qq = per_elem(sigma_t), per_elem(sigma_s), per_elem(q)
    perm = np.arange(E)
    turns = np.zeros(E, dtype=np.int64)
    if seed is not None:
        rng = np.random.default_rng(seed)
        perm = rng.permutation(E)
        turns = rng.integers(0, 3, size=E)
        maps = [tri_rotation_map(r, t) for t in range(3)]
        en = np.stack([en[perm[k]][maps[turns[k]]] for k in range(E)])
        st, ss, qq = st[perm], ss[perm], qq[perm]
    meta = dict(kw.pop("meta", {}), perm=perm, turns=turns, unstructured=True)
    return Problem(name=name, dim=2, nx=(E, 1), r=r, p=p, sn_order=sn_order, lattice=np.zeros((0, 2)),
                   sigma_t=st, sigma_s=ss, q=qq, nodes=nodes, elem_nodes=en, element="simplex", meta=meta, **kw)


def tri_square(n: int = 4, r: int = 2, p: int = 2, sn_order: int = 4, amp: float = 0.05,
               seed: Optional[int] = 3) -> Problem:
    """Warped unit square, x = u + amp sin(2 pi u) sin(2 pi v),
    y = v + amp sin(2 pi u) sin(pi v), n x n cells cut into 2 n^2 curved
    order-r triangles; checkerboard sigma_t in {1, 4} by cell, sigma_s = 0.5,
    q = 1, vacuum."""
    def x_of(u, v):
        return (u + amp * np.sin(2 * math.pi * u) * np.sin(2 * math.pi * v),
                v + amp * np.sin(2 * math.pi * u) * np.sin(math.pi * v))

    def sig(cu, cv):
        return np.where((np.floor(cu * n) + np.floor(cv * n)) % 2 == 0, 1.0, 4.0)

    return triangulated(f"tri_square_{n}_q{r}_p{p}_s{sn_order}", r, p, sn_order, n, n, x_of, sig, 0.5, 1.0,
                        seed=seed, tol=1e-10, meta=dict(amp=amp))


def tri_annulus(nr: int = 3, nt: int = 12, r: int = 3, p: int = 2, sn_order: int = 4, r_in: float = 1.0,
                r_out: float = 2.0, seed: Optional[int] = 1) -> Problem:
    """Full annulus (closed in theta) of 2 nr nt curved order-r triangles with
    control points on circles; curved faces on which Omega . n changes sign
    and cyclic dependencies; sigma_t rings 2.0 / 2.2 / 2.4, sigma_s = 1,
    q = 1, vacuum."""
    def x_of(u, v):
        rho = r_in + (r_out - r_in) * u
        return rho * np.cos(2 * math.pi * v), rho * np.sin(2 * math.pi * v)

    def sig(cu, cv):
        return np.array([2.0, 2.2, 2.4])[np.minimum((cu * 3).astype(int), 2)]

    return triangulated(f"tri_annulus_{nr}x{nt}_q{r}_p{p}_s{sn_order}", r, p, sn_order, nr, nt, x_of, sig, 1.0,
                        1.0, periodic_v=True, seed=seed, tol=1e-8, meta=dict(r_in=r_in, r_out=r_out))


# --------------------------------------------------------------- tetrahedra
def tet_lattice(k: int) -> np.ndarray:
    """(n, 3) lattice triples (i, j, l), i + j + l <= k, of the nodes of order
    k on a tetrahedron, l slowest then j: the local order of a tetrahedron's
    control points (reference position (i, j, l) / k for vertices (0,0,0),
    (1,0,0), (0,1,0), (0,0,1))."""
    return np.array([(i, j, l) for l in range(k + 1) for j in range(k + 1 - l) for i in range(k + 1 - j - l)],
                    dtype=np.int64)


def tet_even_permutations() -> List[tuple]:
    import itertools
    out = []
    for perm in itertools.permutations(range(4)):
        inv = sum(1 for a in range(4) for b in range(a + 1, 4) if perm[a] > perm[b])
        if inv % 2 == 0:
            out.append(perm)
    return out


def tet_rotation_map(r: int, perm) -> np.ndarray:
    """Local index map of a tetrahedron whose vertex t becomes old vertex
    perm[t] (an even permutation keeps the orientation): new local node k is
    old node map[k]."""
    L = tet_lattice(r)
    idx = {tuple(int(v) for v in t): k for k, t in enumerate(L)}
    out = []
    for i, j, l in L:
        cn = [r - i - j - l, i, j, l]
        co = [0, 0, 0, 0]
        for t in range(4):
            co[perm[t]] = cn[t]
        out.append(idx[(co[1], co[2], co[3])])
    return np.array(out, dtype=np.int64)


def tetrahedralized(name: str, r: int, p: int, sn_order: int, n: tuple, x_of, sigma_t, sigma_s, q,
                    periodic_v: bool = False, seed: Optional[int] = None, **kw) -> Problem:
    """Tetrahedra from an n[0] x n[1] x n[2] grid of cells on the parameter
    cube [0, 1]^3, each cell cut into the six tetrahedra along its main
    diagonal (the same cut in every cell, so the mesh is conforming), with
    the vertex order chosen to keep the orientation, mapped by
    x_of(u, v, w) -> (x, y, z) (orientation preserving): control points are
    the map at each tetrahedron's order-r lattice points.  periodic_v: v = 1
    is glued to v = 0.  sigma_t, sigma_s, q: per element or callables of the
    cell centre.  With a seed the elements are renumbered and each one's
    vertex order permuted by a random even permutation (meta 'perm',
    'rot')."""
    import itertools
    fu, fv, fw = r * n[0] + 1, r * n[1] + (0 if periodic_v else 1), r * n[2] + 1
    W_, V, U = np.meshgrid(np.arange(fw) / (r * n[2]), np.arange(fv) / (r * n[1]), np.arange(fu) / (r * n[0]),
                           indexing="ij")
    X = x_of(U.reshape(-1), V.reshape(-1), W_.reshape(-1))                 # u fastest, then v, then w
    nodes = np.stack([np.asarray(c, dtype=np.float64) for c in X], axis=1)
    L = tet_lattice(r)
    elems, centres = [], []
    for ck in range(n[2]):
        for cj in range(n[1]):
            for ci in range(n[0]):
                base = np.array([ci, cj, ck]) * r
                for perm in itertools.permutations(range(3)):
                    e = [np.zeros(3, dtype=np.int64)]
                    for a in perm:
                        v = e[-1].copy()
                        v[a] += 1
                        e.append(v)
                    verts = [e[0], e[1], e[2], e[3]]
                    if np.linalg.det(np.stack([verts[1], verts[2], verts[3]]).astype(float)) < 0:
                        verts = [verts[0], verts[2], verts[1], verts[3]]
                    ids = []
                    for i, j, l in L:
                        pt = base + i * verts[1] + j * verts[2] + l * verts[3]
                        ids.append(int(pt[0] + fu * ((pt[1] % fv) if periodic_v else pt[1]) + fu * fv * pt[2]))
                    elems.append(ids)
                    centres.append(((ci + 0.5) / n[0], (cj + 0.5) / n[1], (ck + 0.5) / n[2]))
    en = np.array(elems, dtype=np.int64)
    cu, cv, cw = np.array(centres).T
    E = len(en)

    def per_elem(v):
        return np.asarray(v(cu, cv, cw) if callable(v) else np.broadcast_to(v, (E,)), dtype=np.float64).copy()

    st, ss, qq = per_elem(sigma_t), per_elem(sigma_s), per_elem(q)
    perm_e = np.arange(E)
    rot = np.zeros(E, dtype=np.int64)
    if seed is not None:
        rng = np.random.default_rng(seed)
        perm_e = rng.permutation(E)
        evens = tet_even_permutations()
        rot = rng.integers(0, len(evens), size=E)
        maps = [tet_rotation_map(r, P_) for P_ in evens]
        en = np.stack([en[perm_e[k]][maps[rot[k]]] for k in range(E)])
        st, ss, qq = st[perm_e], ss[perm_e], qq[perm_e]
    meta = dict(kw.pop("meta", {}), perm=perm_e, rot=rot, unstructured=True)
    return Problem(name=name, dim=3, nx=(E, 1, 1), r=r, p=p, sn_order=sn_order, lattice=np.zeros((0, 3)),
                   sigma_t=st, sigma_s=ss, q=qq, nodes=nodes, elem_nodes=en, element="simplex", meta=meta, **kw)


def tet_cube(n: int = 2, r: int = 2, p: int = 2, sn_order: int = 4, amp: float = 0.04,
             seed: Optional[int] = 3) -> Problem:
    """Warped unit cube, x = u + amp sin(2 pi u) sin(2 pi v) sin(2 pi w) and
    likewise for y, z with the factors shifted (the warp fixes the boundary),
    n^3 cells cut into 6 n^3 curved order-r tetrahedra; checkerboard
    sigma_t in {1, 4} by cell, sigma_s = 0.5, q = 1, vacuum."""
    def x_of(u, v, w):
        s = np.sin(2 * math.pi * u) * np.sin(2 * math.pi * v) * np.sin(2 * math.pi * w)
        return u + amp * s, v + 0.7 * amp * s, w - 0.5 * amp * s

    def sig(cu, cv, cw):
        return np.where((np.floor(cu * n) + np.floor(cv * n) + np.floor(cw * n)) % 2 == 0, 1.0, 4.0)

    return tetrahedralized(f"tet_cube_{n}_q{r}_p{p}_s{sn_order}", r, p, sn_order, (n, n, n), x_of, sig, 0.5, 1.0,
                           seed=seed, tol=1e-10, meta=dict(amp=amp))


def tet_shell(nr: int = 2, nt: int = 8, nz: int = 1, r: int = 2, p: int = 2, sn_order: int = 4,
              r_in: float = 1.0, r_out: float = 2.0, height: float = 1.0, seed: Optional[int] = 1) -> Problem:
    """Cylindrical shell r in [r_in, r_out], theta closed, z in [0, height],
    of 6 nr nt nz curved order-r tetrahedra with control points on circles:
    faces on which Omega . n changes sign and cyclic dependencies around the
    hole; sigma_t 2.0 / 2.4 by radial half, sigma_s = 1, q = 1, vacuum."""
    def x_of(u, v, w):
        rho = r_in + (r_out - r_in) * u
        return rho * np.cos(2 * math.pi * v), rho * np.sin(2 * math.pi * v), height * w

    def sig(cu, cv, cw):
        return np.where(cu < 0.5, 2.0, 2.4)

    return tetrahedralized(f"tet_shell_{nr}x{nt}x{nz}_q{r}_p{p}_s{sn_order}", r, p, sn_order, (nr, nt, nz), x_of,
                           sig, 1.0, 1.0, periodic_v=True, seed=seed, tol=1e-8,
                           meta=dict(r_in=r_in, r_out=r_out, height=height))
