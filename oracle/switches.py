"""Switch function along chords of elements (Section 3, figure switchplt) -- oracle.

TEST INFRASTRUCTURE ONLY: part of the plain CPU oracle.

Each element carries S^+_n on its face xi_n = 1 and -S^+_n on xi_n = 0, and the
two elements that share a face carry opposite signs on it.  A chord is the
sequence of elements met by leaving an element through one face of a
direction and entering the neighbour, which is then left through its opposite
face (of whatever local direction that face has there).  The paper gives an
arbitrary face a sign and propagates the alternating pattern along the chord in
both directions, repeating until every face has been processed.

Order used here (any order gives a valid switch function; a fixed one makes
the result unique): elements by index, then local directions; the first
(element, direction) not yet reached gets S^+ = +1.
"""
from __future__ import annotations

import numpy as np


def _face_node(dim, p, n, line, s):
    """Local node at the end xi_n = s of line ``line`` of direction n (lowest other
    dimension fastest, as in the mesh arrays)."""
    n1 = p + 1
    idx = [0] * dim
    rem = line
    for d in range(dim):
        if d == n:
            continue
        idx[d] = rem % n1
        rem //= n1
    idx[n] = p if s else 0
    node = 0
    for d in reversed(range(dim)):
        node = node * n1 + idx[d]
    return node


def _line_of(dim, p, node, n):
    """(line index, position) of a local node on its direction-n line."""
    n1 = p + 1
    coords = [(node // n1 ** d) % n1 for d in range(dim)]
    line, mul = 0, 1
    for d in range(dim):
        if d == n:
            continue
        line += coords[d] * mul
        mul *= n1
    return line, coords[n]


def shared_face(dim, p, face_nbr, nbr_node, e, f):
    """Face of the neighbour across face f of element e that is that same face,
    identified through the coinciding-node maps (an element may touch the same
    neighbour through two faces on a periodic mesh)."""
    nb = int(face_nbr[e, f])
    n, s = divmod(f, 2)
    mine = _face_node(dim, p, n, 0, s)
    theirs = int(nbr_node[e, f, 0])
    for f2 in range(2 * dim):
        if int(face_nbr[nb, f2]) != e:
            continue
        n2, s2 = divmod(f2, 2)
        l2, t2 = _line_of(dim, p, theirs, n2)
        if t2 != (p if s2 else 0):
            continue
        if int(nbr_node[nb, f2, l2]) == mine:
            return f2
    raise ValueError(f"face {f} of element {e} has no matching face on element {nb}")


def assign_switches(dim: int, p: int, face_nbr: np.ndarray, nbr_node: np.ndarray) -> np.ndarray:
    """S^+[e, n] in {-1, +1} for every element and local direction (int8)."""
    E = face_nbr.shape[0]
    S = np.zeros((E, dim), dtype=np.int8)
    for e in range(E):
        for n in range(dim):
            if S[e, n] != 0:
                continue
            S[e, n] = 1
            for start in (1, 0):  # along xi_n = 1, then back through xi_n = 0
                ce, cn, side = e, n, start
                while True:
                    f = 2 * cn + side
                    nb = int(face_nbr[ce, f])
                    if nb < 0:
                        break
                    f2 = shared_face(dim, p, face_nbr, nbr_node, ce, f)
                    n2, s2 = divmod(f2, 2)
                    mine = S[ce, cn] if side == 1 else -S[ce, cn]   # sign on the shared face, this side
                    want = -mine if s2 == 1 else mine               # S^+ that puts -mine on face f2
                    if S[nb, n2] != 0:
                        if S[nb, n2] != want:
                            raise ValueError("inconsistent chord")
                        break
                    S[nb, n2] = want
                    ce, cn, side = nb, n2, 1 - s2
    return S


def chords(dim, p, face_nbr, nbr_node):
    """Chord id of every (element, direction), following the same walk."""
    E = face_nbr.shape[0]
    cid = -np.ones((E, dim), dtype=np.int64)
    nxt = 0
    for e in range(E):
        for n in range(dim):
            if cid[e, n] >= 0:
                continue
            cid[e, n] = nxt
            for start in (1, 0):
                ce, cn, side = e, n, start
                while True:
                    nb = int(face_nbr[ce, 2 * cn + side])
                    if nb < 0:
                        break
                    f2 = shared_face(dim, p, face_nbr, nbr_node, ce, 2 * cn + side)
                    n2, s2 = divmod(f2, 2)
                    if cid[nb, n2] >= 0:
                        break
                    cid[nb, n2] = nxt
                    ce, cn, side = nb, n2, 1 - s2
            nxt += 1
    return cid
