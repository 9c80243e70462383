"""Pins of the oracle's switch function (Section 3, figure switchplt) and of the general
element relabelling (rotations of the reference square / cube) the GPU tests run on."""
import numpy as np
import pytest

from ldg_workloads import fields, hex_mesh, quad_mesh, random_rotations, reorient_elements
from ldg_workloads.configs import EQ_EULER, EQ_NS
from oracle.switches import assign_switches, chords, shared_face
from tests.gpu_cases import relabel_nodal, rotate_mesh


def signs_on_shared_faces(mesh, S):
    """(sign seen from e, sign seen from the neighbour) for every interior face."""
    out = []
    for e in range(mesh.n_elem):
        for f in range(2 * mesh.dim):
            nb = int(mesh.face_nbr[e, f])
            if nb < 0:
                continue
            f2 = shared_face(mesh.dim, mesh.p, mesh.face_nbr, mesh.nbr_node, e, f)
            n, s = divmod(f, 2)
            n2, s2 = divmod(f2, 2)
            out.append((S[e, n] if s else -S[e, n], S[nb, n2] if s2 else -S[nb, n2]))
    return np.array(out)


def meshes():
    return [quad_mesh(4, 3, 2, box=((0, 4), (0, 3)), periodic=(True, False), perturb=0.1, seed=1),
            quad_mesh(3, 3, 3, box=((0, 3), (0, 3)), periodic=(True, True), perturb=0.15, seed=2),
            hex_mesh(3, 2, length=3.0, periodic=True, amp=0.05),
            hex_mesh(2, 1, length=2.0, periodic=False, amp=0.0)]


@pytest.mark.parametrize("k", range(4))
def test_aligned_mesh_gives_all_plus(k):
    """Elements that all share one orientation: every chord starts with +1 and keeps the
    orientation, so the function is S^+ = +1 everywhere (the generator's own choice)."""
    m = meshes()[k]
    S = assign_switches(m.dim, m.p, m.face_nbr, m.nbr_node)
    assert np.all(S == 1)
    assert np.array_equal(S, m.switch_plus)


@pytest.mark.parametrize("k", range(4))
def test_rotated_mesh_switches_valid_and_canonical(k):
    base = meshes()[k]
    axes, flips = random_rotations(base.dim, base.n_elem, 5 + k)
    perm = np.random.default_rng(k).permutation(base.n_elem)
    m = reorient_elements(base, flips, perm, axes)
    assert np.any(axes != np.arange(base.dim))  # some frames are permuted, not only flipped
    # the relabelling keeps the (valid) switches of the aligned mesh valid
    pairs = signs_on_shared_faces(m, m.switch_plus)
    assert np.all(pairs[:, 0] == -pairs[:, 1])
    S = assign_switches(m.dim, m.p, m.face_nbr, m.nbr_node)
    assert set(np.unique(S)) <= {-1, 1}
    pairs = signs_on_shared_faces(m, S)
    assert len(pairs) > 0 and np.all(pairs[:, 0] == -pairs[:, 1])
    # one free sign per chord: the first (element, direction) of each chord has +1, and the
    # function differs from the relabelled one by one sign per chord
    cid = chords(m.dim, m.p, m.face_nbr, m.nbr_node)
    seen = set()
    for e in range(m.n_elem):
        for n in range(m.dim):
            if cid[e, n] not in seen:
                seen.add(cid[e, n])
                assert S[e, n] == 1
    for c in np.unique(cid):
        ratio = (S * m.switch_plus)[cid == c]
        assert np.all(ratio == ratio[0])
    # chords of a structured box: one per line of elements in each direction
    n_exp = {0: 3 + 4, 1: 3 + 3, 2: 3 * 9, 3: 3 * 4}[k]
    assert len(np.unique(cid)) == n_exp


@pytest.mark.parametrize("eq", [EQ_EULER, EQ_NS])
@pytest.mark.parametrize("dim", [2, 3])
def test_rotation_relabelling_invariance(eq, dim):
    """Rotating element frames (with axis permutations) only relabels the discrete operator
    when the switches are carried along; with the chord switches of the rotated mesh, the
    residual equals the one of the aligned mesh carrying the corresponding switches."""
    from oracle import LineDG
    from oracle.physics import Physics
    if dim == 2:
        base = quad_mesh(3, 3, 2, box=((0, 3), (0, 3)), periodic=(True, True), perturb=0.15, seed=4)
        st = [1.0, 0.3, -0.2, 2.6]
    else:
        base = hex_mesh(2, 2, length=2.0, periodic=True, amp=0.05)
        st = [1.0, 0.3, -0.2, 0.1, 2.6]
    m = dim + 2
    U = fields.random_smooth_state(base, m, seed=7, base=st, amp=0.1)
    rot, flips, perm, axes = rotate_mesh(base, seed=9)
    # the aligned mesh with the switch function carried back: S_old[e, axes[e, n]] from the
    # rotated element's S[perm[e], n] (negated where the axis was reversed)
    sw = np.empty_like(base.switch_plus)
    for e in range(base.n_elem):
        for n in range(dim):
            v = rot.switch_plus[perm[e], n]
            sw[e, axes[e, n]] = -v if flips[e, n] else v
    from ldg_workloads.mesh import Mesh
    base_sw = Mesh(base.dim, base.p, base.xyz, base.face_nbr, base.nbr_node, sw)
    ph = Physics(eq, dim, mu=0.05 if eq == EQ_NS else 0.0)
    d0 = LineDG(dim, base.p, base_sw.xyz, base_sw.face_nbr, base_sw.nbr_node, base_sw.switch_plus, ph)
    d1 = LineDG(dim, rot.p, rot.xyz, rot.face_nbr, rot.nbr_node, rot.switch_plus, ph)
    R0 = d0.residual(U).numpy()
    R1 = d1.residual(relabel_nodal(U, base, flips, perm, axes)).numpy()
    assert np.abs(relabel_nodal(R0, base, flips, perm, axes) - R1).max() <= 1e-12 * np.abs(R0).max()
    assert np.any(rot.switch_plus < 0)
