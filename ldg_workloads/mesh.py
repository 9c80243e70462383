"""Seeded synthetic meshes for the line-DG workloads.

This module only produces *inputs*: node coordinates of curved quad/hex
elements, face connectivity, the coinciding-node map across faces and the
switch signs.  It contains none of the discretisation's arithmetic; both the
CPU oracle and the GPU library consume its arrays unchanged.

Layout conventions (shared by every consumer):

* element ``e`` owns ``Np = (p+1)**D`` nodes on a tensor grid, local node index
  ``i + (p+1)*j + (p+1)**2*k`` (``i`` fastest, Section 2.1 of the paper);
* ``xyz[e, a, node]`` is physical coordinate ``a`` of that node;
* face ``2*n + s`` of an element is the face ``xi_n = s`` (``s`` in {0, 1});
* ``face_nbr[e, f]`` is the neighbouring element across face ``f`` or
  ``-(tag+1)`` for a boundary face (tag 0 = Dirichlet);
* the ``(p+1)**(D-1)`` nodes of a face are numbered by the reference lines of
  direction ``n`` that end on it: the remaining coordinates in increasing
  dimension order, the lowest dimension fastest;
* ``nbr_node[e, f, l]`` is the local node index, inside ``face_nbr[e, f]``, of
  the node that coincides with face node ``l`` (``-1`` on boundary faces);
* ``switch_plus[e, n]`` is the switch ``S^+_n`` at ``xi_n = 1`` (the switch at
  ``xi_n = 0`` is ``-S^+_n``); across a shared face the two elements carry
  opposite signs (Section 3 of the paper).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


def gll_points(p: int) -> np.ndarray:
    """Gauss-Lobatto-Legendre points mapped to [0, 1] (mesh node placement).

    Interior points are the roots of P_p'; they are found by Newton's method on
    the Legendre recurrence.  Used here only to place the high-order nodes of
    the synthetic meshes.
    """
    if p < 1:
        raise ValueError("p >= 1 required")
    x = -np.cos(np.pi * np.arange(p + 1) / p)
    for _ in range(100):
        # P_p and P_{p-1} by the three-term recurrence
        p0 = np.ones_like(x)
        p1 = x.copy()
        for k in range(2, p + 1):
            p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
        if p == 1:
            break
        xi = x[1:-1]
        pp = p1[1:-1]
        pm = p0[1:-1]
        d1 = p * (pm - xi * pp) / (1.0 - xi * xi)              # P_p'
        d2 = (2.0 * xi * d1 - p * (p + 1) * pp) / (1.0 - xi * xi)  # P_p''
        step = d1 / d2
        x[1:-1] = xi - step
        if np.max(np.abs(step)) < 1e-16:
            break
    x[0], x[-1] = -1.0, 1.0
    s = 0.5 * (x + 1.0)
    # enforce exact symmetry
    s = 0.5 * (s + (1.0 - s[::-1]))
    s[0], s[-1] = 0.0, 1.0
    return s


@dataclasses.dataclass
class Mesh:
    dim: int
    p: int
    xyz: np.ndarray          # [E, D, Np] float64
    face_nbr: np.ndarray     # [E, 2D] int64
    nbr_node: np.ndarray     # [E, 2D, Nf] int32
    switch_plus: np.ndarray  # [E, D] int8
    name: str = ""

    @property
    def n_elem(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n1(self) -> int:
        return self.p + 1

    @property
    def np_(self) -> int:
        return self.n1 ** self.dim

    @property
    def nf(self) -> int:
        return self.n1 ** (self.dim - 1)

    def arrays(self):
        return dict(xyz=self.xyz, face_nbr=self.face_nbr, nbr_node=self.nbr_node,
                    switch_plus=self.switch_plus)


def line_end_node(dim: int, p: int, n: int, line: int, t: int) -> int:
    """Local node index of position ``t`` on line ``line`` of direction ``n``."""
    n1 = p + 1
    others = [d for d in range(dim) if d != n]
    idx = [0] * dim
    rem = line
    for d in others:
        idx[d] = rem % n1
        rem //= n1
    idx[n] = t
    node = 0
    for d in reversed(range(dim)):
        node = node * n1 + idx[d]
    return node


def _structured_connectivity(shape, p, periodic):
    """Connectivity of a structured grid of elements with aligned local axes."""
    dim = len(shape)
    n1 = p + 1
    nf = n1 ** (dim - 1)
    n_elem = int(np.prod(shape))
    face_nbr = np.empty((n_elem, 2 * dim), dtype=np.int64)
    nbr_node = np.full((n_elem, 2 * dim, nf), -1, dtype=np.int32)
    strides = [int(np.prod(shape[:d])) for d in range(dim)]
    end0 = np.array([[line_end_node(dim, p, n, l, 0) for l in range(nf)] for n in range(dim)],
                    dtype=np.int32)
    endp = np.array([[line_end_node(dim, p, n, l, p) for l in range(nf)] for n in range(dim)],
                    dtype=np.int32)
    for e in range(n_elem):
        coords = [(e // strides[d]) % shape[d] for d in range(dim)]
        for n in range(dim):
            for s in (0, 1):
                c = list(coords)
                c[n] += 1 if s == 1 else -1
                if 0 <= c[n] < shape[n] or periodic[n]:
                    c[n] %= shape[n]
                    nb = sum(c[d] * strides[d] for d in range(dim))
                    face_nbr[e, 2 * n + s] = nb
                    nbr_node[e, 2 * n + s] = end0[n] if s == 1 else endp[n]
                else:
                    face_nbr[e, 2 * n + s] = -1  # tag 0: Dirichlet
    switch_plus = np.ones((n_elem, dim), dtype=np.int8)
    return face_nbr, nbr_node, switch_plus


def quad_mesh(nx: int, ny: int, p: int, box=((0.0, 1.0), (0.0, 1.0)), periodic=(False, False),
              perturb: float = 0.0, seed: int = 0, curve=None, name: str = "") -> Mesh:
    """Structured quadrilateral mesh, optionally with perturbed interior vertices.

    Vertices of an ``(nx+1) x (ny+1)`` grid on ``box``; if ``perturb > 0`` every
    interior vertex moves by ``U[-perturb*h, perturb*h]`` per coordinate drawn
    from ``numpy.random.default_rng(seed)`` (boundary vertices stay, so periodic
    faces keep matching).  Elements are bilinear; their high-order nodes are the
    bilinear image of the GLL tensor grid.  ``curve(x, y) -> (x', y')`` is then
    applied to every high-order node (an isoparametric curved mesh).
    """
    (x0, x1), (y0, y1) = box
    hx, hy = (x1 - x0) / nx, (y1 - y0) / ny
    vx, vy = np.meshgrid(np.linspace(x0, x1, nx + 1), np.linspace(y0, y1, ny + 1), indexing="xy")
    if perturb > 0:
        rng = np.random.default_rng(seed)
        dx = rng.uniform(-perturb * hx, perturb * hx, size=(ny - 1, nx - 1))
        dy = rng.uniform(-perturb * hy, perturb * hy, size=(ny - 1, nx - 1))
        vx[1:-1, 1:-1] += dx
        vy[1:-1, 1:-1] += dy
    s = gll_points(p)
    n1 = p + 1
    xi, eta = np.meshgrid(s, s, indexing="xy")  # [j, i]
    xi = xi.reshape(-1)
    eta = eta.reshape(-1)  # node = i + n1*j
    n_elem = nx * ny
    xyz = np.empty((n_elem, 2, n1 * n1))
    for ey in range(ny):
        for ex in range(nx):
            e = ex + nx * ey
            c00 = (vx[ey, ex], vy[ey, ex])
            c10 = (vx[ey, ex + 1], vy[ey, ex + 1])
            c01 = (vx[ey + 1, ex], vy[ey + 1, ex])
            c11 = (vx[ey + 1, ex + 1], vy[ey + 1, ex + 1])
            for a in range(2):
                xyz[e, a] = ((1 - xi) * (1 - eta) * c00[a] + xi * (1 - eta) * c10[a]
                             + (1 - xi) * eta * c01[a] + xi * eta * c11[a])
    if curve is not None:
        cx, cy = curve(xyz[:, 0], xyz[:, 1])
        xyz[:, 0], xyz[:, 1] = cx, cy
    face_nbr, nbr_node, sw = _structured_connectivity((nx, ny), p, periodic)
    return Mesh(2, p, xyz, face_nbr, nbr_node, sw, name=name)


def hex_mesh(n: int, p: int, length: float = 2 * math.pi, periodic: bool = True,
             amp: float = 0.1, name: str = "", curve=None) -> Mesh:
    """Structured ``n^3`` hex mesh of ``[0, L]^3`` curved by a sine map.

    Straight-sided GLL nodes are moved by ``X -> X + amp*sin(X)sin(Y)sin(Z)``
    applied to each coordinate (with the arguments scaled by ``2*pi/L``).  The
    map is the identity on the box faces, so periodic faces still match.
    ``curve(X, Y, Z) -> (x, y, z)`` replaces the sine map when given.
    """
    s = gll_points(p)
    n1 = p + 1
    h = length / n
    k3, j3, i3 = np.meshgrid(s, s, s, indexing="ij")  # node = i + n1*j + n1^2*k
    li, lj, lk = i3.reshape(-1), j3.reshape(-1), k3.reshape(-1)
    ez, ey, ex = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ex, ey, ez = ex.reshape(-1), ey.reshape(-1), ez.reshape(-1)  # e = ex + n*(ey + n*ez)
    X = (ex[:, None] + li[None, :]) * h
    Y = (ey[:, None] + lj[None, :]) * h
    Z = (ez[:, None] + lk[None, :]) * h
    w = 2 * math.pi / length
    bump = amp * np.sin(w * X) * np.sin(w * Y) * np.sin(w * Z) / w
    if curve is None:
        xyz = np.stack([X + bump, Y + bump, Z + bump], axis=1)
    else:
        xyz = np.stack(curve(X, Y, Z), axis=1)
    face_nbr, nbr_node, sw = _structured_connectivity((n, n, n), p, (periodic,) * 3)
    return Mesh(3, p, np.ascontiguousarray(xyz), face_nbr, nbr_node, sw, name=name)


def reorient_elements(mesh: Mesh, flips: np.ndarray, perm: np.ndarray | None = None,
                      axes: np.ndarray | None = None) -> Mesh:
    """Relabel a mesh: rotate the local frames of some elements and renumber elements.

    New local axis ``n`` of element ``e`` is old axis ``axes[e, n]`` (identity
    when ``axes`` is None), reversed when ``flips[e, n]``; so new face ``2n + s``
    is old face ``2 axes[e, n] + s`` (or ``+ 1 - s`` when flipped).  The map must
    keep a positive Jacobian determinant: the permutation's sign times
    (-1)^(number of flips) is +1 (in 3-D these are the 24 rotations of the cube).
    ``perm`` renumbers elements (new index ``perm[old]``).  Coordinates,
    connectivity, the coinciding-node map and the switch signs are all updated
    consistently, so the discrete operator is only relabelled.  Returns the new mesh.
    """
    dim, p = mesh.dim, mesh.p
    n1 = p + 1
    E = mesh.n_elem
    Np = n1 ** dim
    nf = n1 ** (dim - 1)
    if perm is None:
        perm = np.arange(E)
    if axes is None:
        axes = np.tile(np.arange(dim), (E, 1))
    axes = np.asarray(axes)
    for e in range(E):
        if sorted(axes[e].tolist()) != list(range(dim)):
            raise ValueError("axes[e] must be a permutation")
        # sign of the permutation by counting inversions
        inv = sum(1 for i in range(dim) for j in range(i + 1, dim) if axes[e, i] > axes[e, j])
        if (inv + int(np.sum(flips[e]))) % 2:
            raise ValueError("the relabelling would make det(G) negative")
    # node relabelling per element: new local node -> old local node
    idx = np.stack(np.meshgrid(*([np.arange(n1)] * dim), indexing="ij"), axis=0)
    idx = idx[::-1].reshape(dim, -1)  # idx[d, node] = coordinate d of node (i fastest)
    def node_of(coords):
        node = np.zeros(coords.shape[1:], dtype=np.int64)
        for d in reversed(range(dim)):
            node = node * n1 + coords[d]
        return node
    new_to_old = np.empty((E, Np), dtype=np.int64)
    old_to_new = np.empty((E, Np), dtype=np.int64)
    for e in range(E):
        c = np.empty_like(idx)
        for d in range(dim):
            c[axes[e, d]] = p - idx[d] if flips[e, d] else idx[d]
        old = node_of(c)  # new node k corresponds to old node old[k]
        new_to_old[e] = old
        old_to_new[e, old] = np.arange(Np)
    xyz = np.empty_like(mesh.xyz)
    face_nbr = np.empty_like(mesh.face_nbr)
    nbr_node = np.full_like(mesh.nbr_node, -1)
    sw = np.empty_like(mesh.switch_plus)
    for e in range(E):
        ne = perm[e]
        xyz[ne] = mesh.xyz[e][:, new_to_old[e]]
        for n in range(dim):
            no = int(axes[e, n])
            sw[ne, n] = -mesh.switch_plus[e, no] if flips[e, n] else mesh.switch_plus[e, no]
            for s in (0, 1):
                so = (1 - s) if flips[e, n] else s          # old side for new side s
                fo, fn = 2 * no + so, 2 * n + s
                nb = mesh.face_nbr[e, fo]
                face_nbr[ne, fn] = perm[nb] if nb >= 0 else nb
                for l in range(nf):
                    # new face node l -> new node -> old node -> old face line index
                    new_node = line_end_node(dim, p, n, l, p if s == 1 else 0)
                    old_node = new_to_old[e, new_node]
                    lo = None
                    for cand in range(nf):
                        if line_end_node(dim, p, no, cand, p if so == 1 else 0) == old_node:
                            lo = cand
                            break
                    if nb >= 0:
                        old_nb_node = mesh.nbr_node[e, fo, lo]
                        nbr_node[ne, fn, l] = old_to_new[nb, old_nb_node]
    return Mesh(dim, p, xyz, face_nbr, nbr_node, sw, name=mesh.name + "+relabelled")


def random_rotations(dim: int, E: int, seed: int, frac: float = 1.0):
    """Seeded orientation-preserving local frames for ``reorient_elements``: for a
    fraction ``frac`` of the elements a uniformly drawn rotation of the square / cube
    (axis permutation with flips of matching parity), the identity for the rest.
    Returns (axes, flips)."""
    import itertools
    rng = np.random.default_rng(seed)
    rots = []
    for pa in itertools.permutations(range(dim)):
        inv = sum(1 for i in range(dim) for j in range(i + 1, dim) if pa[i] > pa[j])
        for fl in itertools.product((False, True), repeat=dim):
            if (inv + sum(fl)) % 2 == 0:
                rots.append((pa, fl))
    axes = np.tile(np.arange(dim), (E, 1))
    flips = np.zeros((E, dim), dtype=bool)
    for e in range(E):
        if rng.random() < frac:
            pa, fl = rots[rng.integers(len(rots))]
            axes[e] = pa
            flips[e] = fl
    return axes, flips


# boundary kinds of a face: face_nbr = -(kind + 1)
BC_DIRICHLET, BC_NEUMANN, BC_SLIP = 0, 1, 2


def with_boundary_kinds(mesh: Mesh, kinds: dict) -> Mesh:
    """Copy of a structured mesh whose boundary faces carry the kind ``kinds[f]`` by local face
    index f = 2n + s (the side xi_n = s of the box for meshes built here); faces not listed
    stay Dirichlet."""
    fn = mesh.face_nbr.copy()
    for f, k in kinds.items():
        col = fn[:, f]
        col[col < 0] = -(int(k) + 1)
    return Mesh(mesh.dim, mesh.p, mesh.xyz, fn, mesh.nbr_node, mesh.switch_plus, name=mesh.name)
