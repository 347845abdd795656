"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module builds *inputs only*: macro meshes (Kuhn-split boxes), boundary
tags, per-macro viscosities, nodal forcing fields and random initial guesses.
It contains none of the solver's arithmetic (no element matrices, no
stencils, no smoothing); both the CPU oracle and the GPU path consume exactly
the arrays produced here, and neither regenerates them.

Nodal fields are given on the vertices of the R-times refined box in lattice
order: the node with integer lattice coordinates (X, Y, Z), 0 <= X <= a*2^R,
0 <= Y, Z <= 2^R, has index X + nx*(Y + ny*Z) with nx = a*2^R + 1 and
ny = 2^R + 1.

Workloads (the paper's serial problems are the unit cube split into 6 macro
tetrahedra, Section 4 and Table "iteration numbers and time-to-solution"):

  1  unit cube, 6 macros, R=4 (17^3 lattice), manufactured forcing, nu=1, fp64
  2  unit cube, 6 macros, R=7 (129^3), manufactured forcing + N(0, 0.01) nodal
     noise (seed 2), fp64
  3  unit cube, 6 macros, R=8 (257^3), manufactured forcing, mixed precision
  4  box [0,2]x[0,1]^2, 12 macros, R=6, nu_e log-uniform in [0.1, 10] (seed 4),
     8-mode Fourier forcing (seed 41), observation viscosity nu_e*exp(0.1 xi_e)
     (seed 42), fp64 forward + adjoint
  5  channel [0,4]x[0,1]^2, 24 macros, R=7, parabolic inflow at x=0, natural
     outflow at x=4, no-slip walls, f=0, nu_e log-uniform in [0.5, 2] (seed 5),
     observation viscosity seed 52, mixed precision forward + adjoint
  6  unit cube, 6 macros, R=7, the analytic solution of the efficiency study
     (Section 5) with its forcing and Dirichlet data, fp64 full multigrid
  7  spherical shell 0.55 < |x| < 1 (Section 4.4), 156 macros (the hollow cube
     [0,3]^3 minus its central cell, its vertices put on the two spheres by the
     equiangular cubed-sphere map), R=5, f=0, homogeneous Dirichlet data on
     both spheres, the paper's random start (u in [0,1], p in [0, 1/h_min]), fp64
  8  the same shell, R=4, the analytic solution of the efficiency study as
     forcing and Dirichlet data (a manufactured solution on the shell)
  9  the same shell, R=5, free-slip on the inner sphere (Section 6.1: u . n = 0
     with the mass-conservative normals; the obstacle of the paper's sphere-bed
     application) and no-slip on the outer one, the forcing of workload 8;
     with_slip("both") puts free-slip on both spheres

For the shell the nodal arrays live on the lattice of the bounding box of the
hollow cube; lattice points in the removed central cell are not vertices
(NaN coordinates; their values are ignored).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

# boundary tags of macro faces (face f is the face opposite local vertex f)
FACE_INTERIOR = 0
FACE_DIRICHLET = 1
FACE_NATURAL = 2
FACE_SLIP = 3


def box_mesh(a: int):
    """Macro mesh of the box [0,a]x[0,1]x[0,1]: each unit cube is split into the
    6 Kuhn tetrahedra {c, c+e_s0, c+e_s0+e_s1, c+(1,1,1)} over the permutations
    s of the three axes.  Vertices are listed in this path order, which is the
    order the refinement and the tests rely on.

    Returns (xyz [nv,3] float64, tet [nt,4] int32)."""
    nx, ny, nz = a + 1, 2, 2
    pts = np.array([(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx)],
                   dtype=np.float64)

    def vid(x, y, z):
        return x + nx * (y + ny * z)

    tets = []
    for cx in range(a):
        for perm in itertools.permutations((0, 1, 2)):
            v = np.array([cx, 0, 0])
            path = [vid(*v)]
            for ax in perm:
                v = v.copy()
                v[ax] += 1
                path.append(vid(*v))
            tets.append(path)
    return pts, np.asarray(tets, dtype=np.int32)


def face_tags(xyz, tet, a: int, natural_x: float | None = None):
    """Boundary tag per (macro, face): a face lying in a plane of the box
    boundary is Dirichlet, except the face(s) in the plane x = natural_x, which
    are natural (do-nothing) faces.  Interior faces are 0."""
    nt = tet.shape[0]
    tags = np.zeros((nt, 4), dtype=np.int8)
    planes = [(0, 0.0), (0, float(a)), (1, 0.0), (1, 1.0), (2, 0.0), (2, 1.0)]
    for t in range(nt):
        for f in range(4):
            fv = xyz[np.delete(tet[t], f)]
            for ax, val in planes:
                if np.all(fv[:, ax] == val):
                    if natural_x is not None and ax == 0 and val == natural_x:
                        tags[t, f] = FACE_NATURAL
                    else:
                        tags[t, f] = FACE_DIRICHLET
    return tags


def hollow_cube_mesh(m: int = 3):
    """Macro mesh of the hollow cube [0,m]^3 minus its central unit cell (m odd):
    every other unit cell is split into the 6 Kuhn tetrahedra of box_mesh, in
    the same path order.  These are the lattice (topological) coordinates of
    the spherical shell; shell_coordinates gives the physical ones.

    Returns (xyz [nv,3] float64 integer-valued, tet [nt,4] int32)."""
    c0 = m // 2
    nx = m + 1
    pts = np.array([(x, y, z) for z in range(nx) for y in range(nx) for x in range(nx)],
                   dtype=np.float64)

    def vid(x, y, z):
        return x + nx * (y + nx * z)

    tets = []
    for cz in range(m):
        for cy in range(m):
            for cx in range(m):
                if (cx, cy, cz) == (c0, c0, c0):
                    continue
                for perm in itertools.permutations((0, 1, 2)):
                    v = np.array([cx, cy, cz])
                    path = [vid(*v)]
                    for ax in perm:
                        v = v.copy()
                        v[ax] += 1
                        path.append(vid(*v))
                    tets.append(path)
    tet = np.asarray(tets, dtype=np.int32)
    used = np.unique(tet)
    remap = -np.ones(pts.shape[0], dtype=np.int64)
    remap[used] = np.arange(used.shape[0])
    return pts[used], remap[tet].astype(np.int32)


def shell_coordinates(xyz, m: int = 3, r_in: float = 0.55, r_out: float = 1.0):
    """Physical coordinates of the hollow-cube macro vertices on the spherical
    shell r_in < |x| < r_out (Section 4.4 uses 0.55 < |x| < 1): a vertex on the
    surface of the removed central cell goes to |x| = r_in, a vertex on the
    outer surface to |x| = r_out (every macro vertex lies on one of the two,
    for m = 3).  Directions follow the equiangular cubed-sphere map (Ronchi,
    Iacono and Paolucci, J. Comput. Phys. 124, 1996): a point a of a cube face
    (|a|_inf = 1) goes to the direction of tan(pi a / 4), which spaces the face
    lines at equal angles; its macros are less skewed than under the central
    projection a / |a| (the shell's multigrid contracts faster on them)."""
    c = xyz - m / 2.0
    mx = np.abs(c).max(axis=1)
    r = np.where(np.isclose(mx, 0.5), r_in, r_out)
    if not np.all(np.isclose(mx, 0.5) | np.isclose(mx, m / 2.0)):
        raise ValueError("every macro vertex must lie on the inner or the outer surface")
    d = np.tan(0.25 * np.pi * c / mx[:, None])
    return d / np.linalg.norm(d, axis=1, keepdims=True) * r[:, None]


def perturbed_coordinates(xyz, amp: float, seed: int):
    """Physical coordinates xyz + amp * U[-1,1]^3 per vertex (seeded): every
    macro of a box mesh becomes a different general tetrahedron."""
    rng = np.random.default_rng(seed)
    return xyz + amp * rng.uniform(-1.0, 1.0, size=xyz.shape)


def boundary_face_tags(tet, tag=FACE_DIRICHLET):
    """`tag` (Dirichlet by default) on every face that belongs to one
    tetrahedron only, 0 on faces shared by two."""
    nt = tet.shape[0]
    count = {}
    for t in range(nt):
        for f in range(4):
            key = tuple(sorted(np.delete(tet[t], f).tolist()))
            count[key] = count.get(key, 0) + 1
    tags = np.zeros((nt, 4), dtype=np.int8)
    for t in range(nt):
        for f in range(4):
            key = tuple(sorted(np.delete(tet[t], f).tolist()))
            if count[key] == 1:
                tags[t, f] = tag
    return tags


def refined_points(xyz, tet, phys, R: int):
    """Physical coordinates [N,3] of the vertices of the R times uniformly
    refined macro mesh, on the lattice of the bounding box of xyz (index X +
    nx (Y + ny Z) at spacing 2^-R); lattice points outside every macro are NaN.
    Each macro carries its vertices affinely: a refined vertex with barycentric
    coordinates l in macro t sits at sum_q l_q phys[tet[t, q]]."""
    n = 1 << R
    lo = xyz.min(axis=0)
    ext = ((xyz.max(axis=0) - lo) * n + 1).astype(np.int64)
    out = np.full((int(ext[0] * ext[1] * ext[2]), 3), np.nan)
    # barycentric coordinates of the refined vertices of one macro, (i, j, k, l)/n
    ijk = np.array([(a, b, c) for a in range(n + 1) for b in range(n + 1 - a)
                    for c in range(n + 1 - a - b)], dtype=np.int64)
    lam = np.concatenate([n - ijk.sum(axis=1, keepdims=True), ijk], axis=1) / n    # [nv,4]
    for t in range(tet.shape[0]):
        L = xyz[tet[t]]                                    # [4,3]
        X = np.rint((lam @ L - lo) * n).astype(np.int64)   # lattice coordinates
        idx = X[:, 0] + ext[0] * (X[:, 1] + ext[1] * X[:, 2])
        out[idx] = lam @ phys[tet[t]]
    return out


def lattice_shape(a: int, R: int):
    n = 1 << R
    return a * n + 1, n + 1, n + 1


def lattice_points(a: int, R: int):
    """Physical coordinates [N,3] of the refined box vertices in lattice order."""
    nx, ny, nz = lattice_shape(a, R)
    h = 1.0 / (1 << R)
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([X.ravel() * h, Y.ravel() * h, Z.ravel() * h], axis=1)


# ---------------------------------------------------------------------------
# manufactured solution of configs 1-3:
#   u = curl(psi*(1,1,1)), psi = (sin(pi x) sin(pi y) sin(pi z))^2,
#   p = x + y + z - 3/2,  f = -nu*Lap(u) + grad(p)
# written with S(t) = sin^2(pi t) and its derivatives D1 = S', D2 = S'', D3 = S'''
# ---------------------------------------------------------------------------
def _S(t):
    return np.sin(np.pi * t) ** 2


def _D1(t):
    return np.pi * np.sin(2 * np.pi * t)


def _D2(t):
    return 2 * np.pi ** 2 * np.cos(2 * np.pi * t)


def _D3(t):
    return -4 * np.pi ** 3 * np.sin(2 * np.pi * t)


def manufactured_velocity(x):
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    px = _D1(X) * _S(Y) * _S(Z)
    py = _S(X) * _D1(Y) * _S(Z)
    pz = _S(X) * _S(Y) * _D1(Z)
    return np.stack([py - pz, pz - px, px - py], axis=0)


def manufactured_pressure(x):
    return x[:, 0] + x[:, 1] + x[:, 2] - 1.5


def manufactured_forcing(x, nu: float = 1.0):
    """[3,N] nodal values of f = -nu*Lap(u) + grad(p) for the manufactured pair."""
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    # derivatives of Lap(psi) along each axis
    lx = _D3(X) * _S(Y) * _S(Z) + _D1(X) * _D2(Y) * _S(Z) + _D1(X) * _S(Y) * _D2(Z)
    ly = _D2(X) * _D1(Y) * _S(Z) + _S(X) * _D3(Y) * _S(Z) + _S(X) * _D1(Y) * _D2(Z)
    lz = _D2(X) * _S(Y) * _D1(Z) + _S(X) * _D2(Y) * _D1(Z) + _S(X) * _S(Y) * _D3(Z)
    lap_u = np.stack([ly - lz, lz - lx, lx - ly], axis=0)
    return -nu * lap_u + 1.0


def tme_velocity(x):
    """[3,N] analytic velocity of the efficiency study (Section 5):
    u = (-4 cos 4z, 8 cos 8x, -2 cos 2y), divergence free."""
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    return np.stack([-4.0 * np.cos(4.0 * Z), 8.0 * np.cos(8.0 * X), -2.0 * np.cos(2.0 * Y)])


def tme_pressure(x):
    """[N] analytic pressure of the efficiency study: sin 4x sin 8y sin 2z minus
    its mean over the unit cube."""
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    mean = ((1.0 - np.cos(4.0)) / 4.0) * ((1.0 - np.cos(8.0)) / 8.0) * ((1.0 - np.cos(2.0)) / 2.0)
    return np.sin(4.0 * X) * np.sin(8.0 * Y) * np.sin(2.0 * Z) - mean


def tme_forcing(x):
    """[3,N] f = -Laplace(u) + grad(p) (nu = 1) of the efficiency study."""
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    s4x, c4x = np.sin(4.0 * X), np.cos(4.0 * X)
    s8y, c8y = np.sin(8.0 * Y), np.cos(8.0 * Y)
    s2z, c2z = np.sin(2.0 * Z), np.cos(2.0 * Z)
    return np.stack([-64.0 * np.cos(4.0 * Z) + 4.0 * c4x * s8y * s2z,
                     512.0 * np.cos(8.0 * X) + 8.0 * s4x * c8y * s2z,
                     -8.0 * np.cos(2.0 * Y) + 2.0 * s4x * s8y * c2z])


def fourier_forcing(x, seed: int, modes: int = 8):
    """f = sum_m d_m sin(pi k_m . x + phi_m): k_m in {1,2,3}^3, phi_m ~ U[0, 2 pi),
    d_m a random unit vector (amplitude 1).  Returns [3,N]."""
    rng = np.random.default_rng(seed)
    k = rng.integers(1, 4, size=(modes, 3))
    phi = rng.uniform(0.0, 2 * np.pi, size=modes)
    d = rng.normal(size=(modes, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    f = np.zeros((3, x.shape[0]))
    for m in range(modes):
        s = np.sin(np.pi * (x @ k[m]) + phi[m])
        f += d[m][:, None] * s[None, :]
    return f


def nodal_noise(N: int, seed: int, sigma: float):
    """i.i.d. N(0, sigma^2) per node and component, [3,N]."""
    return np.random.default_rng(seed).normal(0.0, sigma, size=(3, N))


def log_uniform_viscosity(nt: int, lo: float, hi: float, seed: int):
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=nt))


def perturbed_viscosity(nu, seed: int, scale: float = 0.1):
    """Viscosity of the synthetic observation: nu_e * exp(scale * xi_e), xi ~ N(0,1)."""
    xi = np.random.default_rng(seed).normal(size=nu.shape[0])
    return nu * np.exp(scale * xi)


def inflow_profile(x):
    """[3,N] Dirichlet data of the channel: u_x = 16 y(1-y) z(1-z) on the inflow
    plane x = 0; zero elsewhere (walls).  Values off the Dirichlet set are
    ignored by both solvers."""
    g = np.zeros((3, x.shape[0]))
    on = x[:, 0] == 0.0
    y, z = x[on, 1], x[on, 2]
    g[0, on] = 16.0 * y * (1 - y) * z * (1 - z)
    return g


def random_initial_guess(N: int, pmax: float, seed: int = 0):
    """Random start of the paper's serial runs: u in U[0,1], p in U[0, pmax]
    (the paper uses pmax = 1/h_min).  Returns [4,N]."""
    rng = np.random.default_rng(seed)
    x = np.empty((4, N))
    x[:3] = rng.uniform(0.0, 1.0, size=(3, N))
    x[3] = rng.uniform(0.0, pmax, size=N)
    return x


# ---------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    a: int                      # box length in x (unit cubes)
    R: int                      # refinements of the macro mesh
    precision: str              # "fp64" | "mixed"
    natural_x: float | None = None
    nu_range: tuple | None = None
    nu_seed: int | None = None
    nu_obs_seed: int | None = None
    forcing: str = "manufactured"   # manufactured | manufactured+noise | fourier | zero
    forcing_seed: int | None = None
    noise_sigma: float = 0.0
    inflow: bool = False
    solution: str | None = None     # "tme": the analytic solution of the efficiency study
    kind: str = "box"               # "box" | "shell" (the spherical shell of Section 4.4)
    slip: str | None = None         # shell: free-slip on the inner sphere ("inner") or on both
                                    # ("both"); no-slip elsewhere
    extra: dict = field(default_factory=dict)

    # -- inputs ----------------------------------------------------------
    def mesh(self):
        if self.kind == "shell":
            xyz, tet = hollow_cube_mesh(3)
            tags = boundary_face_tags(tet, FACE_DIRICHLET)
            if self.slip is not None:
                # the inner sphere holds the vertices of the removed central cell
                inner = np.isclose(np.abs(xyz - 1.5).max(axis=1), 0.5)
                for t, f in zip(*np.nonzero(tags)):
                    if self.slip == "both" or np.all(inner[np.delete(tet[t], f)]):
                        tags[t, f] = FACE_SLIP
            return xyz, tet, np.ones(tet.shape[0]), tags
        xyz, tet = box_mesh(self.a)
        tags = face_tags(xyz, tet, self.a, self.natural_x)
        if self.nu_range is None:
            nu = np.ones(tet.shape[0])
        else:
            nu = log_uniform_viscosity(tet.shape[0], self.nu_range[0], self.nu_range[1],
                                       self.nu_seed)
        return xyz, tet, nu, tags

    def with_R(self, R: int) -> "Workload":
        d = dict(self.__dict__)
        d["R"] = R
        return Workload(**d)

    def with_slip(self, slip: str | None) -> "Workload":
        d = dict(self.__dict__)
        d["slip"] = slip
        return Workload(**d)

    def h_min(self) -> float:
        """min_T h_T = min_T |T|^(1/3) over the finest tetrahedra: uniform
        refinement splits a tetrahedron into 8 of equal volume, so a macro's
        children at R refinements have volume |T_macro| / 8^R."""
        xyz, tet, _, _ = self.mesh()
        P = self.physical()
        P = xyz if P is None else P
        e = np.stack([P[tet[:, q + 1]] - P[tet[:, 0]] for q in range(3)], axis=1)
        vol = np.abs(np.linalg.det(e)) / 6.0
        return float((vol.min() / 8.0 ** self.R) ** (1.0 / 3.0))

    def physical(self):
        """Physical coordinates of the macro vertices (None: the lattice ones)."""
        if self.kind == "shell":
            xyz, _ = hollow_cube_mesh(3)
            return shell_coordinates(xyz, 3)
        return None

    def points(self):
        if self.kind == "shell":
            xyz, tet, _, _ = self.mesh()
            return refined_points(xyz, tet, self.physical(), self.R)
        return lattice_points(self.a, self.R)

    def forcing_field(self):
        x = self.points()
        if self.forcing == "manufactured":
            return manufactured_forcing(x)
        if self.forcing == "manufactured+noise":
            return manufactured_forcing(x) + nodal_noise(x.shape[0], self.forcing_seed,
                                                         self.noise_sigma)
        if self.forcing == "fourier":
            return fourier_forcing(x, self.forcing_seed)
        if self.forcing == "zero":
            return np.zeros((3, x.shape[0]))
        if self.forcing == "tme":
            return np.nan_to_num(tme_forcing(x))
        raise ValueError(self.forcing)

    def dirichlet_field(self):
        """[3,N] Dirichlet velocity values (inflow profile, the analytic
        velocity, or zero)."""
        x = self.points()
        if self.inflow:
            return inflow_profile(x)
        if self.solution == "tme":
            return np.nan_to_num(tme_velocity(x))
        return np.zeros((3, x.shape[0]))

    def exact_solution(self):
        """[4,N] nodal values of the analytic solution, if the workload has one."""
        x = self.points()
        if self.solution == "tme":
            return np.concatenate([tme_velocity(x), tme_pressure(x)[None, :]])
        raise ValueError("workload has no analytic solution")

    def observation_viscosity(self):
        _, _, nu, _ = self.mesh()
        return perturbed_viscosity(nu, self.nu_obs_seed)


WORKLOADS = {
    1: Workload("unit-cube-R4-fp64", a=1, R=4, precision="fp64"),
    2: Workload("unit-cube-R7-fp64", a=1, R=7, precision="fp64",
                forcing="manufactured+noise", forcing_seed=2, noise_sigma=0.1),
    3: Workload("unit-cube-R8-mixed", a=1, R=8, precision="mixed"),
    4: Workload("box2-R6-adjoint-fp64", a=2, R=6, precision="fp64", nu_range=(0.1, 10.0),
                nu_seed=4, nu_obs_seed=42, forcing="fourier", forcing_seed=41),
    5: Workload("channel4-R7-adjoint-mixed", a=4, R=7, precision="mixed", natural_x=4.0,
                nu_range=(0.5, 2.0), nu_seed=5, nu_obs_seed=52, forcing="zero", inflow=True),
    6: Workload("unit-cube-tme-R7-fp64", a=1, R=7, precision="fp64", forcing="tme", solution="tme"),
    7: Workload("shell-R5-fp64", a=3, R=5, precision="fp64", forcing="zero", kind="shell"),
    8: Workload("shell-tme-R4-fp64", a=3, R=4, precision="fp64", forcing="tme", solution="tme",
                kind="shell"),
    9: Workload("shell-slip-R5-fp64", a=3, R=5, precision="fp64", forcing="tme", kind="shell",
                slip="inner"),
}
