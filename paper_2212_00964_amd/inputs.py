"""Seeded synthetic inputs for the HEX8 finite-element path.

This module generates problem *data* only: box meshes (optionally distorted or
relabelled), per-element parameter fields, Dirichlet masks and values, lists of
loaded boundary faces, nodal source values and observation fields.  It contains
no finite-element arithmetic (no shape functions, quadrature, constitutive laws
or assembly), so that the GPU path and the CPU oracle can both consume it while
sharing no method code.

Conventions (both sides rely on them):

* node id  = ix + (nx+1) * (iy + (ny+1) * iz), coordinates ``ix*Lx/nx`` etc.;
* element id = ex + nx * (ey + ny * ez);
* HEX8 local node order: 0:(0,0,0) 1:(1,0,0) 2:(1,1,0) 3:(0,1,0)
  4:(0,0,1) 5:(1,0,1) 6:(1,1,1) 7:(0,1,1) (bottom face counter-clockwise,
  then the top face);
* degree of freedom ``dof = ndpn * node + component``;
* a boundary face is the pair (element, local face) with
  local face = 2*axis + side, i.e. the element face on which the reference
  coordinate ``xi_axis`` equals -1 (side 0) or +1 (side 1).

Every random draw uses ``numpy.random.default_rng(seed)`` (PCG64), in element-id
order, and the same arrays are handed to both implementations.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

# model / parameter-map codes shared by both implementations' interfaces
POISSON, LINEAR_ELASTIC, NEO_HOOKEAN, J2_PLASTIC = 0, 1, 2, 3
THETA_IDENTITY, THETA_SIMP = 0, 1
CG, BICGSTAB = 0, 1

_LOCAL = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                   [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], dtype=np.int64)


@dataclasses.dataclass
class Problem:
    """A complete synthetic problem definition (host arrays only)."""
    name: str
    coords: np.ndarray            # [Nn, 3] float64
    conn: np.ndarray              # [Ne, 8] int32
    ndpn: int                     # 1 (Poisson) or 3
    model: int
    theta: np.ndarray             # [Ne] float64 per-element parameter
    dirichlet_mask: np.ndarray    # [N] uint8
    dirichlet_values: np.ndarray  # [N] float64, values at the final load step
    pmap: int = THETA_IDENTITY
    nu: float = 0.3
    bulk_ratio: float = 10.0
    simp_p: float = 3.0
    simp_emin: float = 1e-3
    simp_e0: float = 1.0
    yield_stress: float = 0.0                     # J2 plasticity
    traction_faces: Optional[np.ndarray] = None   # [nf, 2] int32 (element, local face)
    traction: Optional[np.ndarray] = None         # [nf, ndpn] float64
    source_nodal: Optional[np.ndarray] = None     # [Nn*ndpn] float64 nodal source values
    f_nodal: Optional[np.ndarray] = None          # [N] float64 nodal point loads
    n_load_steps: int = 1
    krylov: int = CG
    shape: tuple = ()                             # (nx, ny, nz) when structured
    lengths: tuple = ()                           # (Lx, Ly, Lz)

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.conn.shape[0])

    @property
    def n_dofs(self) -> int:
        return self.n_nodes * self.ndpn


# ----------------------------------------------------------------------------- meshes

def box_mesh(nx: int, ny: int, nz: int, Lx: float = 1.0, Ly: float = 1.0, Lz: float = 1.0):
    """Structured HEX8 mesh of the box [0,Lx]x[0,Ly]x[0,Lz]."""
    ix = np.arange(nx + 1, dtype=np.float64)
    iy = np.arange(ny + 1, dtype=np.float64)
    iz = np.arange(nz + 1, dtype=np.float64)
    Z, Y, X = np.meshgrid(iz * Lz / nz, iy * Ly / ny, ix * Lx / nx, indexing="ij")
    coords = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    ex, ey, ez = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ex, ey, ez = (a.transpose(2, 1, 0).ravel() for a in (ex, ey, ez))
    conn = np.empty((nx * ny * nz, 8), dtype=np.int64)
    for a, (dx, dy, dz) in enumerate(_LOCAL):
        conn[:, a] = (ex + dx) + (nx + 1) * ((ey + dy) + (ny + 1) * (ez + dz))
    return coords, conn.astype(np.int32)


def distort(coords: np.ndarray, shape, lengths, seed: int, amp: float = 0.2) -> np.ndarray:
    """Move every interior node by U(-amp*h_i, amp*h_i) along each axis i."""
    nx, ny, nz = shape
    h = np.array([lengths[0] / nx, lengths[1] / ny, lengths[2] / nz])
    rng = np.random.default_rng(seed)
    out = coords.copy()
    d = rng.uniform(-amp, amp, size=coords.shape) * h
    eps = 1e-12 * np.array(lengths)
    interior = np.all((coords > eps) & (coords < np.array(lengths) - eps), axis=1)
    out[interior] += d[interior]
    return out


def relabel(prob: Problem, seed: int) -> tuple[Problem, np.ndarray, np.ndarray]:
    """Randomly renumber nodes and elements (returns problem, node perm, elem perm).

    ``new_node_of[old] = new`` and ``new_elem_of[old] = new``.  The structure of
    the mesh is unchanged, so any result must be the same field, relabelled.
    """
    rng = np.random.default_rng(seed)
    Nn, Ne, nd = prob.n_nodes, prob.n_elems, prob.ndpn
    new_node_of = rng.permutation(Nn)
    new_elem_of = rng.permutation(Ne)
    coords = np.empty_like(prob.coords)
    coords[new_node_of] = prob.coords
    conn = np.empty_like(prob.conn)
    conn[new_elem_of] = new_node_of[prob.conn]
    theta = np.empty_like(prob.theta)
    theta[new_elem_of] = prob.theta

    def dof_perm(v):
        if v is None:
            return None
        w = np.empty_like(v)
        w.reshape(Nn, nd)[new_node_of] = v.reshape(Nn, nd)
        return w

    faces = None
    if prob.traction_faces is not None:
        faces = prob.traction_faces.copy()
        faces[:, 0] = new_elem_of[faces[:, 0]]
    q = dataclasses.replace(
        prob, name=prob.name + "-relabelled", coords=coords, conn=conn.astype(np.int32), theta=theta,
        dirichlet_mask=dof_perm(prob.dirichlet_mask), dirichlet_values=dof_perm(prob.dirichlet_values),
        traction_faces=faces, source_nodal=dof_perm(prob.source_nodal), f_nodal=dof_perm(prob.f_nodal),
        shape=(), lengths=prob.lengths)
    return q, new_node_of, new_elem_of


def box_face_list(shape, axis: int, side: int) -> np.ndarray:
    """(element, local face) pairs of the elements touching one face of a structured box."""
    nx, ny, nz = shape
    ex, ey, ez = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ex, ey, ez = (a.transpose(2, 1, 0).ravel() for a in (ex, ey, ez))
    idx = (ex, ey, ez)[axis]
    sel = idx == (0 if side == 0 else shape[axis] - 1)
    elems = (ex + nx * (ey + ny * ez))[sel]
    return np.stack([elems, np.full_like(elems, 2 * axis + side)], axis=1).astype(np.int32)


def _on_plane(coords, axis, value, length):
    return np.abs(coords[:, axis] - value) <= 1e-9 * max(length, 1.0)


def _dof_mask(nodes_sel: np.ndarray, ndpn: int, comps) -> np.ndarray:
    m = np.zeros((nodes_sel.shape[0], ndpn), dtype=np.uint8)
    for c in comps:
        m[nodes_sel, c] = 1
    return m.ravel()


# ----------------------------------------------------------------------------- fields

def lognormal_field(n: int, mu: float, sigma: float, seed: int) -> np.ndarray:
    """exp(mu + sigma z), z ~ N(0,1) i.i.d., drawn in element-id order."""
    rng = np.random.default_rng(seed)
    return np.exp(mu + sigma * rng.standard_normal(n))


def uniform_field(n: int, lo: float, hi: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=n)


def element_centroids(coords: np.ndarray, conn: np.ndarray) -> np.ndarray:
    return coords[conn].mean(axis=1)


def smooth_field(points: np.ndarray, lengths, seed: int, n_modes: int = 8, kmax: int = 2) -> np.ndarray:
    """Sum of ``n_modes`` random low-wavenumber sine/cosine modes, scaled to max |psi| = 1."""
    rng = np.random.default_rng(seed)
    L = np.asarray(lengths, dtype=np.float64)
    psi = np.zeros(points.shape[0])
    for _ in range(n_modes):
        k = rng.integers(0, kmax + 1, size=3)
        if not k.any():
            k[rng.integers(0, 3)] = 1
        amp = rng.uniform(-1.0, 1.0)
        phase = rng.uniform(0.0, 2.0 * np.pi)
        psi += amp * np.cos(np.pi * (points / L) @ k + phase)
    m = np.max(np.abs(psi))
    return psi / m if m > 0 else psi


# ----------------------------------------------------------------------------- workloads

def poisson_sine(n: int = 8, distort_seed: Optional[int] = None) -> Problem:
    """-Laplace(u) = f on the unit cube, u = 0 on the boundary, manufactured
    u = sin(pi x) sin(pi y) sin(pi z), so f = 3 pi^2 u (given at the nodes)."""
    coords, conn = box_mesh(n, n, n)
    if distort_seed is not None:
        coords = distort(coords, (n, n, n), (1.0, 1.0, 1.0), distort_seed)
    bnd = np.zeros(coords.shape[0], dtype=bool)
    for ax in range(3):
        bnd |= _on_plane(coords, ax, 0.0, 1.0) | _on_plane(coords, ax, 1.0, 1.0)
    u_exact = np.sin(np.pi * coords[:, 0]) * np.sin(np.pi * coords[:, 1]) * np.sin(np.pi * coords[:, 2])
    return Problem(
        name=f"poisson-sine-{n}", coords=coords, conn=conn, ndpn=1, model=POISSON,
        theta=np.ones(conn.shape[0]), dirichlet_mask=bnd.astype(np.uint8),
        dirichlet_values=np.zeros(coords.shape[0]), source_nodal=3.0 * np.pi ** 2 * u_exact,
        krylov=CG, shape=(n, n, n), lengths=(1.0, 1.0, 1.0))


def cantilever(nx: int = 64, ny: int = 32, nz: int = 32, L=(2.0, 1.0, 1.0), E: float = 70e3, nu: float = 0.3,
               traction=(0.0, 0.0, -1.0), distort_seed: Optional[int] = None) -> Problem:
    """Linear-elastic cantilever: x=0 clamped, uniform traction on the face x=Lx."""
    coords, conn = box_mesh(nx, ny, nz, *L)
    if distort_seed is not None:
        coords = distort(coords, (nx, ny, nz), L, distort_seed)
    left = _on_plane(coords, 0, 0.0, L[0])
    faces = box_face_list((nx, ny, nz), 0, 1)
    return Problem(
        name=f"cantilever-{nx}x{ny}x{nz}", coords=coords, conn=conn, ndpn=3, model=LINEAR_ELASTIC,
        theta=np.full(conn.shape[0], E), dirichlet_mask=_dof_mask(left, 3, (0, 1, 2)),
        dirichlet_values=np.zeros(coords.shape[0] * 3), nu=nu, traction_faces=faces,
        traction=np.tile(np.asarray(traction, dtype=np.float64), (faces.shape[0], 1)),
        krylov=CG, shape=(nx, ny, nz), lengths=tuple(L))


def nh_tensile(nx: int = 100, ny: int = 100, nz: int = 100, L=(1.0, 1.0, 1.0), stretch: float = 1.2,
               n_load_steps: int = 5, seed: int = 0, sigma: float = 0.3, mu: float = float(np.log(10.0)),
               bulk_ratio: float = 10.0, distort_seed: Optional[int] = None, theta: Optional[np.ndarray] = None,
               krylov: int = BICGSTAB) -> Problem:
    """Compressible neo-Hookean block pulled along x: x=0 fixed (u=0), x=Lx moved by
    (stretch-1)*Lx along x with u_y = u_z = 0; per-element shear modulus lognormal."""
    coords, conn = box_mesh(nx, ny, nz, *L)
    if distort_seed is not None:
        coords = distort(coords, (nx, ny, nz), L, distort_seed)
    left = _on_plane(coords, 0, 0.0, L[0])
    right = _on_plane(coords, 0, L[0], L[0])
    mask = _dof_mask(left | right, 3, (0, 1, 2))
    vals = np.zeros((coords.shape[0], 3))
    vals[right, 0] = (stretch - 1.0) * L[0]
    if theta is None:
        theta = lognormal_field(conn.shape[0], mu, sigma, seed)
    return Problem(
        name=f"nh-tensile-{nx}x{ny}x{nz}", coords=coords, conn=conn, ndpn=3, model=NEO_HOOKEAN,
        theta=theta, dirichlet_mask=mask, dirichlet_values=vals.ravel(), bulk_ratio=bulk_ratio,
        n_load_steps=n_load_steps, krylov=krylov, shape=(nx, ny, nz), lengths=tuple(L))


def nh_roller_uniaxial(nx: int, ny: int, nz: int, stretch: float = 1.2, G: float = 10.0, bulk_ratio: float = 10.0,
                       n_load_steps: int = 4, distort_seed: Optional[int] = None) -> Problem:
    """Unit cube with symmetry rollers (u_x=0 on x=0, u_y=0 on y=0, u_z=0 on z=0) and
    u_x = stretch-1 on x=1; constant modulus.  The exact discrete solution is a
    homogeneous stretch, which makes this a closed-form check."""
    coords, conn = box_mesh(nx, ny, nz)
    if distort_seed is not None:
        coords = distort(coords, (nx, ny, nz), (1.0, 1.0, 1.0), distort_seed)
    Nn = coords.shape[0]
    m = np.zeros((Nn, 3), dtype=np.uint8)
    m[_on_plane(coords, 0, 0.0, 1.0), 0] = 1
    m[_on_plane(coords, 1, 0.0, 1.0), 1] = 1
    m[_on_plane(coords, 2, 0.0, 1.0), 2] = 1
    right = _on_plane(coords, 0, 1.0, 1.0)
    m[right, 0] = 1
    vals = np.zeros((Nn, 3))
    vals[right, 0] = stretch - 1.0
    return Problem(
        name=f"nh-roller-{nx}x{ny}x{nz}", coords=coords, conn=conn, ndpn=3, model=NEO_HOOKEAN,
        theta=np.full(conn.shape[0], G), dirichlet_mask=m.ravel(), dirichlet_values=vals.ravel(),
        bulk_ratio=bulk_ratio, n_load_steps=n_load_steps, krylov=BICGSTAB, shape=(nx, ny, nz),
        lengths=(1.0, 1.0, 1.0))


def simp_cantilever(nx: int = 120, ny: int = 60, nz: int = 30, L=(2.0, 1.0, 0.5), seed: int = 0,
                    traction=(0.0, 0.0, -1.0), distort_seed: Optional[int] = None) -> Problem:
    """SIMP compliance gradient workload: density theta ~ U(0.4, 0.6) per element,
    E(theta) = 1e-3 + theta^3 (1 - 1e-3), nu = 0.3, x=0 clamped, traction on x=Lx."""
    p = cantilever(nx, ny, nz, L=L, E=1.0, nu=0.3, traction=traction, distort_seed=distort_seed)
    p.name = f"simp-{nx}x{ny}x{nz}"
    p.theta = uniform_field(p.n_elems, 0.4, 0.6, seed)
    p.pmap = THETA_SIMP
    p.simp_p, p.simp_emin, p.simp_e0 = 3.0, 1e-3, 1.0
    return p


def nh_inverse(nx: int = 200, ny: int = 100, nz: int = 100, L=(2.0, 1.0, 1.0), stretch: float = 1.2,
               n_load_steps: int = 5, field_seed: int = 2, theta0: float = 10.0, distort_seed: Optional[int] = None):
    """Inverse modulus identification: returns (problem at theta = theta0 uniform,
    theta_true = theta0 * exp(0.3 psi(x_e)) with psi a seeded smooth field)."""
    p = nh_tensile(nx, ny, nz, L=L, stretch=stretch, n_load_steps=n_load_steps,
                   theta=np.full(nx * ny * nz, theta0), distort_seed=distort_seed)
    p.name = f"nh-inverse-{nx}x{ny}x{nz}"
    psi = smooth_field(element_centroids(p.coords, p.conn), L, field_seed)
    theta_true = theta0 * np.exp(0.3 * psi)
    return p, theta_true


def cylinder_mesh(n: int, nz: int, R: float = 5.0, H: float = 10.0):
    """HEX8 mesh of the cylinder x^2 + y^2 <= R^2, 0 <= z <= H: the structured n x n x nz
    grid of [-1, 1]^2 x [0, H], its cross-section mapped onto the disk by
    (x, y) -> R (x sqrt(1 - y^2 / 2), y sqrt(1 - x^2 / 2)) (a smooth map of the square
    onto the disk; boundary nodes land on the circle)."""
    coords, conn = box_mesh(n, n, nz, 2.0, 2.0, H)
    x, y = coords[:, 0] - 1.0, coords[:, 1] - 1.0
    out = coords.copy()
    out[:, 0] = R * x * np.sqrt(1.0 - 0.5 * y * y)
    out[:, 1] = R * y * np.sqrt(1.0 - 0.5 * x * x)
    return out, conn


def fan_mesh(k: int = 8, layers: int = 4, R: float = 1.0, H: float = 1.0):
    """HEX8 prism over the regular k-gon of circumradius R: the polygon is split into k
    kites (centre, midpoint of edge i, corner i+1, midpoint of edge i+1) and extruded in
    `layers` layers to height H.  The nodes on the axis are shared by 2k elements and
    have 3 (2k + 1) neighbours (51 for k = 8): a mesh outside the structured-grid
    degrees (at most 8 elements and 27 neighbours per node)."""
    a = 2.0 * np.pi * np.arange(k) / k
    v = R * np.stack([np.cos(a), np.sin(a)], axis=1)
    m = 0.5 * (v + np.roll(v, -1, axis=0))  # m[i] halves the edge from corner i to i+1
    pts = np.vstack([np.zeros((1, 2)), m, v])  # 0: centre, 1..k: midpoints, k+1..2k: corners
    quads = np.array([[0, 1 + i, k + 1 + (i + 1) % k, 1 + (i + 1) % k] for i in range(k)])
    npl = 2 * k + 1
    coords = np.vstack([np.column_stack([pts, np.full(npl, H * l / layers)]) for l in range(layers + 1)])
    conn = np.vstack([np.hstack([quads + l * npl, quads + (l + 1) * npl]) for l in range(layers)])
    return coords, conn.astype(np.int32)


def nh_fan(k: int = 8, layers: int = 4, stretch: float = 1.1, n_load_steps: int = 2, seed: int = 0,
           sigma: float = 0.3, mu: float = float(np.log(10.0)), bulk_ratio: float = 10.0) -> Problem:
    """Compressible neo-Hookean fan prism (fan_mesh) stretched along its axis: the bottom
    face fixed, the top face moved by (stretch-1) H along z with u_x = u_y = 0;
    per-element shear modulus lognormal."""
    H = 1.0
    coords, conn = fan_mesh(k, layers, 1.0, H)
    bottom = np.isclose(coords[:, 2], 0.0)
    top = np.isclose(coords[:, 2], H)
    mask = _dof_mask(bottom | top, 3, (0, 1, 2))
    vals = np.zeros((coords.shape[0], 3))
    vals[top, 2] = (stretch - 1.0) * H
    return Problem(
        name=f"nh-fan-{k}x{layers}", coords=coords, conn=conn, ndpn=3, model=NEO_HOOKEAN,
        theta=lognormal_field(conn.shape[0], mu, sigma, seed), dirichlet_mask=mask, dirichlet_values=vals.ravel(),
        bulk_ratio=bulk_ratio, n_load_steps=n_load_steps, krylov=CG, lengths=(2.0, 2.0, H))


def j2_cylinder(n: int = 8, nz: int = 16, R: float = 5.0, H: float = 10.0, E: float = 70e3, nu: float = 0.3,
                yield_stress: float = 250.0, disp: float = 0.1, n_load_steps: int = 10) -> Problem:
    """Perfect J2 plasticity in uniaxial tension of a cylinder (radius R, height H): bottom
    face fixed, top face moved by (0, 0, disp); dirichlet_values hold the fully loaded
    state, reached in n_load_steps (unloading is a second solve back to zero)."""
    coords, conn = cylinder_mesh(n, nz, R, H)
    bottom = _on_plane(coords, 2, 0.0, H)
    top = _on_plane(coords, 2, H, H)
    vals = np.zeros((coords.shape[0], 3))
    vals[top, 2] = disp
    return Problem(
        name=f"j2-cylinder-{n}x{n}x{nz}", coords=coords, conn=conn, ndpn=3, model=J2_PLASTIC,
        theta=np.full(conn.shape[0], E), dirichlet_mask=_dof_mask(bottom | top, 3, (0, 1, 2)),
        dirichlet_values=vals.ravel(), nu=nu, yield_stress=yield_stress, n_load_steps=n_load_steps, krylov=CG,
        shape=(n, n, nz), lengths=(2.0 * R, 2.0 * R, H))


def j2_roller_uniaxial(nx: int, ny: int, nz: int, strain: float = 0.01, E: float = 70e3, nu: float = 0.3,
                       yield_stress: float = 250.0, n_load_steps: int = 5,
                       distort_seed: Optional[int] = None) -> Problem:
    """Unit cube of J2 material on symmetry rollers (u_x=0 on x=0, u_y=0 on y=0, u_z=0
    on z=0) with u_z = strain on z=1: the exact discrete solution is homogeneous
    uniaxial stress, sigma_zz following the one-dimensional elastic-perfectly-plastic
    recursion (a closed-form check)."""
    coords, conn = box_mesh(nx, ny, nz)
    if distort_seed is not None:
        coords = distort(coords, (nx, ny, nz), (1.0, 1.0, 1.0), distort_seed)
    Nn = coords.shape[0]
    m = np.zeros((Nn, 3), dtype=np.uint8)
    m[_on_plane(coords, 0, 0.0, 1.0), 0] = 1
    m[_on_plane(coords, 1, 0.0, 1.0), 1] = 1
    m[_on_plane(coords, 2, 0.0, 1.0), 2] = 1
    top = _on_plane(coords, 2, 1.0, 1.0)
    m[top, 2] = 1
    vals = np.zeros((Nn, 3))
    vals[top, 2] = strain
    return Problem(
        name=f"j2-roller-{nx}x{ny}x{nz}", coords=coords, conn=conn, ndpn=3, model=J2_PLASTIC,
        theta=np.full(conn.shape[0], E), dirichlet_mask=m.ravel(), dirichlet_values=vals.ravel(), nu=nu,
        yield_stress=yield_stress, n_load_steps=n_load_steps, krylov=CG, shape=(nx, ny, nz),
        lengths=(1.0, 1.0, 1.0))


def sample_elements(n_elems: int, k: int = 20, seed: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_elems, size=min(k, n_elems), replace=False))


# The five named workloads, full size.
def poisson_inference(nx: int = 50, ny: int = 50, nz: int = 10, L=(1.0, 1.0, 0.2), alpha: float = 1.0,
                      n_obs: int = 250, seed: int = 1, distort_seed: Optional[int] = None):
    """Full-field inference workload: -alpha Lap u = b on the box, u = 0 on the boundary,
    b a bimodal source of two Gaussian bumps centred at (0.25, 0.25, 0.1) and
    (0.75, 0.75, 0.1) of the box (b = 10 exp(-1000 |x - c|^2) each), observations at
    n_obs distinct interior nodes drawn from `seed`.  Returns (problem carrying the true
    source as source_nodal, observed node indices)."""
    coords, conn = box_mesh(nx, ny, nz, *L)
    if distort_seed is not None:
        coords = distort(coords, (nx, ny, nz), L, distort_seed)
    bnd = np.zeros(coords.shape[0], dtype=bool)
    for ax in range(3):
        bnd |= _on_plane(coords, ax, 0.0, L[ax]) | _on_plane(coords, ax, L[ax], L[ax])
    b = np.zeros(coords.shape[0])
    for c in ((0.25 * L[0], 0.25 * L[1], 0.5 * L[2]), (0.75 * L[0], 0.75 * L[1], 0.5 * L[2])):
        b += 10.0 * np.exp(-1000.0 * np.sum((coords - np.asarray(c)) ** 2, axis=1))
    interior = np.flatnonzero(~bnd)
    obs = np.sort(np.random.default_rng(seed).choice(interior, size=min(n_obs, interior.size), replace=False))
    p = Problem(name=f"poisson-inference-{nx}x{ny}x{nz}", coords=coords, conn=conn, ndpn=1, model=POISSON,
                theta=np.full(conn.shape[0], float(alpha)), dirichlet_mask=bnd.astype(np.uint8),
                dirichlet_values=np.zeros(coords.shape[0]), source_nodal=b, krylov=CG, shape=(nx, ny, nz),
                lengths=tuple(L))
    return p, obs


def workload(idx: int):
    if idx == 1:
        return poisson_sine(8)
    if idx == 2:
        return cantilever(64, 32, 32)
    if idx == 3:
        return nh_tensile(100, 100, 100)
    if idx == 4:
        return simp_cantilever(120, 60, 30)
    if idx == 5:
        return nh_inverse(200, 100, 100)[0]
    raise ValueError(idx)
