"""Mesh hierarchy and P1-P1 PSPG finite element matrices (oracle, FP64).

Follows Section 2 of the paper:
  * Section 2.1: the hierarchy T_l is built from the unstructured macro mesh
    T_{-2} by successive uniform refinement, each tetrahedron split into 8;
    T_0 is the twice refined macro mesh (Section 4: "the coarse grid T_0 is a
    two times refined initial grid").
  * eq. (varform) and the forms below it: a_1(u,v) = <nu grad u, grad v>,
    b(u,q) = -<div u, q>, f(v) = <f, v>, and the level dependent PSPG terms
    c_l(q,p) = sum_T delta_T h_T^2 <grad p, grad q>_T,
    g_l(q) = -sum_T delta_T h_T^2 <f, grad q>_T with h_T = |T|^(1/3) and
    delta_T = 1/12.
  * eq. (linear-system): K = [[A, B^T], [B, -C]], right-hand side (f, g).
  * the D form a_2(u,v) = 2 <nu D(u), D(v)> with D(u) = (grad u + grad u^T)/2
    (eq. cauchystress and the forms below eq. varform): for P1 functions
    2 D(phi_b e_l) : D(phi_a e_k) = delta_kl grad phi_a . grad phi_b
    + d_l phi_a d_k phi_b, so A_2 = diag(A_1, A_1, A_1) + E with the coupling
    blocks E^{kl}[a, b] = sum_T nu_T |T| d_l phi_a d_k phi_b (row a and
    component k test, column b and component l trial).

Everything is assembled element by element on the global mesh with generic P1
formulas (gradients of the barycentric coordinates from the inverse of the
element Jacobian); nothing here assumes the lattice structure of the meshes.

Readings taken where the paper is silent:
  * uniform refinement is the standard 1->8 red refinement with the interior
    octahedron cut along the diagonal joining the midpoints of edges (0,2) and
    (1,3) (Bey's rule); on Kuhn macro tetrahedra this keeps every child a Kuhn
    tetrahedron of the finer lattice;
  * the forcing enters as its nodal P1 interpolant I_h f, so both f(v) and
    g_l(q) are integrated exactly for that interpolant;
  * per-macro viscosity nu_e multiplies a_1 element-wise (Laplace form) and
    divides the PSPG weight, delta_T h_T^2 / nu_T in both c_l and g_l.  At
    nu = 1 (all of the paper's runs) this is the paper's form; for nu != 1 it
    is the scaling under which the discrete system is invariant under
    p -> nu p (the Schur complement B A^-1 B^T scales like 1/nu, and so does
    C, which keeps the pressure smoother on C matched to it).  Without the
    1/nu the Uzawa iteration diverges for macro viscosities around 0.1;
  * velocity Dirichlet nodes are the nodes on closed macro faces tagged
    Dirichlet; pressure is an unknown at every node.
  * free-slip faces (tag 3; Section 6.1): their nodes, unless also on a
    Dirichlet face, carry the point-wise constraint u . n = 0 with the
    mass-conservative normal n_i = <grad phi_i, 1> / |.|, the velocity
    column sum of b at the constant pressure, n_i = -(B^T 1)_i / |.|.  The
    tangential stress condition is the natural one of the weak form.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

DELTA = 1.0 / 12.0          # PSPG parameter delta_T (Section 2.1)
FACE_DIRICHLET = 1
FACE_SLIP = 3


# --------------------------------------------------------------------------
# uniform refinement (Section 2.1)
# --------------------------------------------------------------------------
_EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def refine(P):
    """One uniform refinement of tetrahedra given by integer vertex coordinates
    P [nt,4,3] at lattice scale s; returns children [8nt,4,3] at scale 2s."""
    Q = 2 * P
    x = [Q[:, i] for i in range(4)]
    mid = {e: (x[e[0]] + x[e[1]]) // 2 for e in _EDGES}
    x01, x02, x03, x12, x13, x23 = (mid[e] for e in _EDGES)
    children = [
        (x[0], x01, x02, x03),
        (x01, x[1], x12, x13),
        (x02, x12, x[2], x23),
        (x03, x13, x23, x[3]),
        # interior octahedron, cut along x02 -- x13
        (x01, x02, x03, x13),
        (x01, x02, x12, x13),
        (x02, x03, x13, x23),
        (x02, x12, x13, x23),
    ]
    C = np.stack([np.stack(c, axis=1) for c in children], axis=1)
    return C.reshape(-1, 4, 3)


def p1_geometry(Pphys):
    """Volumes [nt] and gradients of the barycentric coordinates [nt,4,3] of P1
    tetrahedra with physical vertex coordinates Pphys [nt,4,3]."""
    J = Pphys[:, 1:, :] - Pphys[:, :1, :]          # rows: edge vectors x_i - x_0
    Jinv = np.linalg.inv(J)
    G = np.empty(Pphys.shape)
    G[:, 1:, :] = np.transpose(Jinv, (0, 2, 1))    # grad(lambda_i) = column i of J^-1
    G[:, 0, :] = -G[:, 1:, :].sum(axis=1)
    vol = np.abs(np.linalg.det(J)) / 6.0
    return vol, G


# --------------------------------------------------------------------------
@dataclass
class Level:
    R: int
    n: int
    shape: tuple
    lat: np.ndarray            # [N] lattice index of every node (sorted: lattice order)
    X: np.ndarray              # [N,3] integer lattice coordinates
    tets: np.ndarray           # [nt,4] node indices
    tet_macro: np.ndarray      # [nt] macro id of every element
    vol: np.ndarray            # [nt]
    G: np.ndarray              # [nt,4,3] gradients of barycentric coordinates
    dirichlet: np.ndarray      # [N] bool, velocity Dirichlet node
    A: sp.csr_matrix = None    # a_1 (scalar block; the velocity block is diag(A,A,A))
    C: sp.csr_matrix = None    # c_l
    M: sp.csr_matrix = None    # consistent mass
    B: list = field(default_factory=list)    # B_k[q, v] = b(phi_v e_k, phi_q)
    Gf: list = field(default_factory=list)   # g_l as a map of nodal f_k: g = sum_k Gf_k f_k
    colour: np.ndarray = None  # [N] (X+Y+Z) mod 4
    mass: np.ndarray = None    # [N] int phi_i (row sums of M)
    Xphys: np.ndarray = None   # [N,3] physical coordinates
    E: list = None             # D form only: E[k][l] coupling blocks (N x N)
    A2: sp.csr_matrix = None   # D form only: the 3N x 3N velocity block (component major)
    slip: np.ndarray = None    # [N] bool, free-slip node (velocity tangential)
    normal: np.ndarray = None  # [N,3] mass-conservative unit normal at slip nodes, 0 elsewhere

    @property
    def N(self):
        return self.lat.shape[0]

    @property
    def free(self):
        return ~self.dirichlet

    def ndofs(self):
        """3 * free velocity nodes + all pressure nodes (Section 4: 206 on T_0)."""
        return 3 * int(self.free.sum()) + self.N


def _assemble(rows, cols, vals, N):
    return sp.coo_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=(N, N)).tocsr()


def assemble_level(lv: Level, nu_macro, chunk=1 << 21, op="laplace"):
    """Element-by-element assembly of A (a_1), C (c_l), M, B_k and the g_l map;
    for op == "D" also the coupling blocks E of a_2 and the velocity block A_2."""
    N = lv.N
    keys = ["A", "C", "M", "B0", "B1", "B2", "G0", "G1", "G2"]
    if op == "D":
        keys += [f"E{k}{l}" for k in range(3) for l in range(3)]
    mats = {k: None for k in keys}
    nt = lv.tets.shape[0]
    eye = np.eye(4)
    for s in range(0, nt, chunk):
        e = slice(s, min(nt, s + chunk))
        T = lv.tets[e]
        vol, G = lv.vol[e], lv.G[e]
        nu = nu_macro[lv.tet_macro[e]]
        hT2 = vol ** (2.0 / 3.0)                       # h_T^2 with h_T = |T|^(1/3)
        rows = np.repeat(T[:, :, None], 4, axis=2)     # local a (test / row)
        cols = np.repeat(T[:, None, :], 4, axis=1)     # local b (trial / column)
        GG = np.einsum("tak,tbk->tab", G, G)
        part = {
            "A": (nu * vol)[:, None, None] * GG,
            "C": (DELTA * hT2 * vol / nu)[:, None, None] * GG,
            "M": (vol / 20.0)[:, None, None] * (1.0 + eye)[None],
        }
        for k in range(3):
            # b(phi_b e_k, phi_a) = -int div(phi_b e_k) phi_a = -(|T|/4) d_k phi_b
            part[f"B{k}"] = np.broadcast_to((-vol / 4.0)[:, None, None] * G[:, None, :, k],
                                            (T.shape[0], 4, 4))
            # g_l(phi_a) for f = phi_b e_k: -delta h_T^2 (|T|/4) d_k phi_a
            part[f"G{k}"] = np.broadcast_to((-DELTA * hT2 * vol / (4.0 * nu))[:, None, None]
                                            * G[:, :, None, k], (T.shape[0], 4, 4))
        if op == "D":
            for k in range(3):
                for l in range(3):
                    # nu |T| d_l phi_a d_k phi_b, a the row (test) node
                    part[f"E{k}{l}"] = (nu * vol)[:, None, None] * (G[:, :, None, l]
                                                                   * G[:, None, :, k])
        for key, val in part.items():
            m = _assemble(rows, cols, np.ascontiguousarray(val), N)
            mats[key] = m if mats[key] is None else mats[key] + m
    lv.A, lv.C, lv.M = mats["A"], mats["C"], mats["M"]
    lv.B = [mats[f"B{k}"] for k in range(3)]
    lv.Gf = [mats[f"G{k}"] for k in range(3)]
    lv.mass = np.asarray(lv.M.sum(axis=1)).ravel()
    if op == "D":
        lv.E = [[mats[f"E{k}{l}"] for l in range(3)] for k in range(3)]
        lv.A2 = sp.bmat([[lv.E[k][l] + (lv.A if k == l else 0) for l in range(3)]
                         for k in range(3)], format="csr")


def _dirichlet_nodes(X, n, macro_int, tet, face_bc, tag=FACE_DIRICHLET):
    """Nodes (integer coords X at scale n) on a closed macro face tagged `tag`
    (Dirichlet by default)."""
    mask = np.zeros(X.shape[0], dtype=bool)
    Xl = X.astype(np.int64)
    for t in range(tet.shape[0]):
        for f in range(4):
            if face_bc[t, f] != tag:
                continue
            a, b, c = (macro_int[v].astype(np.int64) * n for v in np.delete(tet[t], f))
            nrm = np.cross(b - a, c - a)
            on = (Xl - a) @ nrm == 0
            Y = Xl[on]
            inside = np.ones(Y.shape[0], dtype=bool)
            for p, q in ((a, b), (b, c), (c, a)):
                inside &= np.cross(q - p, Y - p) @ nrm >= 0
            idx = np.nonzero(on)[0][inside]
            mask[idx] = True
    return mask


def macro_maps(macro_int, tet, phys):
    """Affine maps of the macro tetrahedra from the integer lattice to physical
    space: x_phys = o_m + (x - L0_m) F_m, with F_m [3,3] (row vectors) taking
    the lattice edge vectors L_q - L0 of macro m to P_q - P0.  Uniform
    refinement is affine on every macro (Section 2.1: each tetrahedron is split
    into 8 by its edge midpoints), so a refined vertex with lattice
    coordinates x sits at that image."""
    L = macro_int[tet].astype(np.float64)                 # [nt,4,3]
    Pp = np.asarray(phys, dtype=np.float64)[tet]          # [nt,4,3]
    EL = L[:, 1:] - L[:, :1]
    EP = Pp[:, 1:] - Pp[:, :1]
    F = np.linalg.solve(EL, EP)                           # EL F = EP
    return L[:, 0], Pp[:, 0], F


def _make_level(Pint, tet_macro, R, macro_int, tet, face_bc, nu, op="laplace", maps=None):
    n = 1 << R
    ext = macro_int.max(axis=0).astype(np.int64) * n + 1
    shape = (int(ext[0]), int(ext[1]), int(ext[2]))
    Pl = Pint.astype(np.int64)
    latv = Pl[..., 0] + shape[0] * (Pl[..., 1] + shape[1] * Pl[..., 2])
    lat, inv = np.unique(latv.ravel(), return_inverse=True)
    tets = inv.reshape(-1, 4).astype(np.int64)
    X = np.stack([lat % shape[0], (lat // shape[0]) % shape[1], lat // (shape[0] * shape[1])],
                 axis=1)
    if maps is None:
        Pphys = Pint.astype(np.float64) / n
    else:
        L0, O, F = maps
        m = tet_macro
        Pphys = O[m][:, None, :] + np.einsum("tqd,tde->tqe",
                                             Pint.astype(np.float64) / n - L0[m][:, None, :], F[m])
    vol, G = p1_geometry(Pphys)
    lv = Level(R=R, n=n, shape=shape, lat=lat, X=X, tets=tets, tet_macro=tet_macro,
               vol=vol, G=G, dirichlet=_dirichlet_nodes(X, n, macro_int, tet, face_bc))
    # physical coordinates of the nodes (from the first element holding each)
    first = np.full(lat.shape[0], -1, dtype=np.int64)
    flat = tets.ravel()
    order = np.arange(flat.shape[0])
    first[flat[::-1]] = order[::-1]
    lv.Xphys = Pphys.reshape(-1, 3)[first]
    lv.colour = (X.sum(axis=1) % 4).astype(np.int64)
    assemble_level(lv, nu, op=op)
    lv.slip = _dirichlet_nodes(X, n, macro_int, tet, face_bc, FACE_SLIP) & ~lv.dirichlet
    lv.normal = np.zeros((lv.N, 3))
    if lv.slip.any():
        one = np.ones(lv.N)
        g = -np.stack([lv.B[k].T @ one for k in range(3)], axis=1)     # <grad phi_i, 1>
        gs = g[lv.slip]
        lv.normal[lv.slip] = gs / np.linalg.norm(gs, axis=1, keepdims=True)
    return lv


def project_slip(lv, v):
    """Removes the normal component of the velocity rows v[:3] at the
    free-slip nodes (in place): v_i <- (I - n_i n_i^T) v_i."""
    if lv.slip is not None and lv.slip.any():
        n = lv.normal[lv.slip]
        vs = v[:3, lv.slip]
        v[:3, lv.slip] = vs - n.T * np.sum(n.T * vs, axis=0)
    return v


def tangential_basis(lv):
    """Sparse T [3 nf, m]: the velocity unknowns of the constrained space in
    Cartesian components (component-major over the free nodes): one column
    per component at nodes without the constraint, two tangent vectors
    (orthonormal, perpendicular to n_i) at free-slip nodes."""
    fr = np.nonzero(lv.free)[0]
    nf = fr.shape[0]
    rows, cols, vals = [], [], []
    col = 0
    pos = {int(i): q for q, i in enumerate(fr)}
    for i in fr:
        q = pos[int(i)]
        if lv.slip is not None and lv.slip[i]:
            nrm = lv.normal[i]
            a = np.zeros(3)
            a[np.argmin(np.abs(nrm))] = 1.0
            t1 = a - np.dot(a, nrm) * nrm
            t1 /= np.linalg.norm(t1)
            t2 = np.cross(nrm, t1)
            for t in (t1, t2):
                for k in range(3):
                    rows.append(k * nf + q)
                    cols.append(col)
                    vals.append(t[k])
                col += 1
        else:
            for k in range(3):
                rows.append(k * nf + q)
                cols.append(col)
                vals.append(1.0)
                col += 1
    return sp.csr_matrix((vals, (rows, cols)), shape=(3 * nf, col))


def _prolongation(coarse: Level, Pc_int, fine: Level):
    """P1 interpolation T_{l-1} -> T_l: fine nodes that are coarse nodes take the
    coarse value; every other fine node is the midpoint of a coarse edge and
    takes the mean of the two end values."""
    Nf, Nc = fine.N, coarse.N
    sf0, sf1 = fine.shape[0], fine.shape[0] * fine.shape[1]

    def fine_index(Xf):
        return np.searchsorted(fine.lat, Xf[..., 0] + sf0 * Xf[..., 1] + sf1 * Xf[..., 2])

    rows, cols, vals = [], [], []
    # coarse vertices
    rows.append(fine_index(2 * coarse.X))
    cols.append(np.arange(Nc))
    vals.append(np.ones(Nc))
    # edge midpoints of the coarse elements
    e = np.array(_EDGES)
    ea = coarse.tets[:, e[:, 0]].ravel()
    eb = coarse.tets[:, e[:, 1]].ravel()
    mid = fine_index(coarse.X[ea] + coarse.X[eb])
    mid, first = np.unique(mid, return_index=True)
    for parent in (ea[first], eb[first]):
        rows.append(mid)
        cols.append(parent)
        vals.append(np.full(mid.shape[0], 0.5))
    P = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(Nf, Nc)).tocsr()
    return P


@dataclass
class Hierarchy:
    levels: list               # Level objects, coarsest (R0) first
    P: list                    # P[l] maps level l-1 -> level l (P[0] is None)
    nu: np.ndarray
    project: bool              # pressure determined up to a constant (no natural face)
    op: str = "laplace"        # velocity form: "laplace" (a_1) or "D" (a_2)
    macro_int: np.ndarray = None   # [nv,3] integer lattice coordinates of the macro vertices
    tet: np.ndarray = None         # [nt,4] macro tetrahedra

    @property
    def finest(self):
        return self.levels[-1]


def build_hierarchy(xyz, tet, nu, face_bc, R, R0=2, op="laplace", phys=None):
    """Levels R0..R of the uniformly refined macro mesh; op selects the velocity
    form, "laplace" (a_1) or "D" (a_2).  xyz are integer lattice coordinates of
    the macro vertices (the topology: refinement, node numbering, colours);
    phys, if given, their physical coordinates, which every macro carries
    affinely into its refinement (general macro geometry); otherwise the
    lattice coordinates are physical.  Lattice points outside every macro
    (a hole in the bounding box) are not nodes."""
    if op not in ("laplace", "D"):
        raise ValueError(op)
    macro_int = np.rint(xyz).astype(np.int64)
    if not np.array_equal(macro_int, xyz):
        raise ValueError("oracle expects macro vertices on the integer lattice")
    maps = None if phys is None else macro_maps(macro_int, tet, phys)
    nu = np.asarray(nu, dtype=np.float64)
    P = macro_int[tet]                                  # [nt,4,3] at scale 1
    tet_macro = np.arange(tet.shape[0])
    for _ in range(R0):
        P = refine(P)
        tet_macro = np.repeat(tet_macro, 8)
    levels = [_make_level(P, tet_macro, R0, macro_int, tet, face_bc, nu, op, maps)]
    prol = [None]
    for r in range(R0 + 1, R + 1):
        P = refine(P)
        tet_macro = np.repeat(tet_macro, 8)
        lv = _make_level(P, tet_macro, r, macro_int, tet, face_bc, nu, op, maps)
        prol.append(_prolongation(levels[-1], None, lv))
        levels.append(lv)
    project = not np.any(face_bc == 2)
    return Hierarchy(levels=levels, P=prol, nu=nu, project=project, op=op, macro_int=macro_int,
                     tet=np.asarray(tet))


def primitives(lv, macro_int, tet):
    """HHG primitive of every node (Section 3.4): the macro vertex, edge, face or
    volume whose relative interior holds it, i.e. the sub-simplex spanned by
    the macro vertices with positive barycentric coordinate.  Returns
    (cls [N], prim [N]): cls 0 vertex, 1 edge, 2 face, 3 volume; prim numbers
    the primitives (equal for nodes of one primitive)."""
    n = lv.n
    N = lv.N
    key = np.full((N, 4), -1, dtype=np.int64)
    for t in range(tet.shape[0]):
        L = macro_int[tet[t]].astype(np.int64)
        E = (L[1:] - L[0]).T                          # columns: edge vectors
        Einv = np.rint(np.linalg.inv(E)).astype(np.int64)   # unimodular (Kuhn macros)
        mu = (lv.X - n * L[0]) @ Einv.T               # n * (lambda_1..3)
        lam = np.concatenate([n - mu.sum(axis=1, keepdims=True), mu], axis=1)
        inside = np.all(lam >= 0, axis=1)
        ids = np.where(lam[inside] > 0, tet[t][None, :], -1)
        key[inside] = np.sort(ids, axis=1)
    if np.any(key[:, 3] < 0):
        raise ValueError("a node lies in no macro")
    cls = (key >= 0).sum(axis=1) - 1
    _, prim = np.unique(key, axis=0, return_inverse=True)
    return cls.astype(np.int64), prim.ravel().astype(np.int64)
