"""Host-side checks of the C ABI: the library loads, exports every declared entry point,
and rejects bad descriptions before any device work (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from ldg_workloads import quad_mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1204_1533_amd", "libldg.so")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ldg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(ldg_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libldg.so not built")
    from paper_1204_1533_amd import ldg
    return ldg.load_library()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "ldg_residual" in names and "ldg_newton_step" in names
    for n in names:
        assert hasattr(lib, n), n
    from paper_1204_1533_amd import ldg
    assert set(names) <= set(ldg.exported_symbols()) | set(names)


def _desc(mesh, **kw):
    from paper_1204_1533_amd import ldg
    keep = dict(xyz=np.ascontiguousarray(mesh.xyz), fn=np.ascontiguousarray(mesh.face_nbr),
                nn=np.ascontiguousarray(mesh.nbr_node), sw=np.ascontiguousarray(mesh.switch_plus))
    d = ldg.ldg_problem_desc()
    d.dim, d.p, d.equation, d.node_family = mesh.dim, mesh.p, kw.get("equation", 1), 0
    d.gamma, d.mu, d.prandtl, d.c11_interior, d.c11_dirichlet = 1.4, 0.0, 0.72, 0.0, 10.0
    d.n_elem = mesh.n_elem
    for k, v in kw.items():
        setattr(d, k, v)
    d.node_xyz_host = keep["xyz"].ctypes.data
    d.face_nbr_host = keep["fn"].ctypes.data
    d.nbr_node_host = keep["nn"].ctypes.data
    d.switch_plus_host = keep["sw"].ctypes.data
    return d, keep


def _create(lib, d):
    h = ctypes.c_void_p()
    return lib.ldg_create(ctypes.byref(d), None, ctypes.byref(h))


def test_create_rejects_bad_descriptions(lib):
    from paper_1204_1533_amd import ldg
    mesh = quad_mesh(3, 3, 2, periodic=(True, True))
    d, keep = _desc(mesh, p=7)
    assert _create(lib, d) == ldg.LDG_E_UNSUPPORTED
    assert lib.ldg_last_error(None) == b"ldg_create: p must be in 1..4"
    d, keep = _desc(mesh, dim=4)
    assert _create(lib, d) == ldg.LDG_E_UNSUPPORTED
    d, keep = _desc(mesh, gamma=0.5)
    assert _create(lib, d) == ldg.LDG_E_INVALID
    d, keep = _desc(mesh)
    d.face_nbr_host = None
    assert _create(lib, d) == ldg.LDG_E_INVALID
    # broken reciprocity
    bad = mesh.nbr_node.copy()
    bad[0, 1, 0] = (bad[0, 1, 0] + 1) % mesh.np_
    mesh2 = type(mesh)(mesh.dim, mesh.p, mesh.xyz, mesh.face_nbr, bad, mesh.switch_plus)
    d, keep = _desc(mesh2)
    assert _create(lib, d) == ldg.LDG_E_SHAPE
    assert b"not reciprocal" in lib.ldg_last_error(None)
    # switch signs not opposite across a face
    sw = mesh.switch_plus.copy()
    sw[4, 0] = -1
    mesh3 = type(mesh)(mesh.dim, mesh.p, mesh.xyz, mesh.face_nbr, mesh.nbr_node, sw)
    d, keep = _desc(mesh3)
    assert _create(lib, d) == ldg.LDG_E_SHAPE
    # switch values must be +-1
    sw = mesh.switch_plus.copy()
    sw[0, 0] = 0
    mesh4 = type(mesh)(mesh.dim, mesh.p, mesh.xyz, mesh.face_nbr, mesh.nbr_node, sw)
    d, keep = _desc(mesh4)
    assert _create(lib, d) == ldg.LDG_E_INVALID
    assert b"switch_plus must be +-1 (element 0)" in lib.ldg_last_error(None)
    # Dirichlet faces need a positive penalty (Poisson)
    m5 = quad_mesh(2, 2, 2)
    d, keep = _desc(m5, equation=0, c11_dirichlet=0.0)
    assert _create(lib, d) == ldg.LDG_E_INVALID


def test_null_context_calls(lib):
    from paper_1204_1533_amd import ldg
    assert lib.ldg_residual(None, None, None, None) == ldg.LDG_E_INVALID
    assert lib.ldg_num_dofs(None) == -1
    assert lib.ldg_status_string(ldg.LDG_E_NOT_ASSEMBLED) == b"operators not assembled"


def test_learned_entry_points_validate_before_device_work(lib):
    """Network and learned-correction calls reject bad arguments without touching a GPU."""
    from paper_1204_1533_amd import ldg
    h = ctypes.c_void_p()
    assert lib.ldg_net_create(4, 3, 5, 256, 0, None, ctypes.byref(h)) == ldg.LDG_E_INVALID
    assert lib.ldg_net_create(3, 3, 4, 256, 0, None, ctypes.byref(h)) == ldg.LDG_E_INVALID  # m must be 1 or dim+2
    assert lib.ldg_net_create(3, 0, 5, 256, 0, None, ctypes.byref(h)) == ldg.LDG_E_INVALID
    assert lib.ldg_net_create(3, 3, 5, 0, 0, None, ctypes.byref(h)) == ldg.LDG_E_INVALID
    assert not h.value
    assert lib.ldg_net_num_params(None) == -1
    assert lib.ldg_net_set_params(None, None) == ldg.LDG_E_INVALID
    assert lib.ldg_net_adam_step(None, 1e-3) == ldg.LDG_E_INVALID
    assert lib.ldg_learned_attach(None, None, ldg.LDG_BF16) == ldg.LDG_E_INVALID
    assert lib.ldg_learned_collect(None, 1) == ldg.LDG_E_INVALID
    assert lib.ldg_learned_active(None) == 0
    el = (ctypes.c_int64 * 1)(0)
    assert lib.ldg_learned_samples(None, el, 1, None, 1, None, None, None, None) == ldg.LDG_E_INVALID
    lib.ldg_net_destroy(None)


def test_time_step_and_newton_validate_before_device_work(lib):
    from paper_1204_1533_amd import ldg
    so = ldg.ldg_step_opts(ldg.LDG_DIRK3, 10, 1e-8, 0.0, 0, 1, 15)
    lo = ldg.ldg_solver_opts(50, 100, 10, 0, 1e-8, 1e-3, 0, 0)
    rep = ldg.ldg_step_report()
    assert lib.ldg_implicit_step(None, None, None, 0.1, ctypes.byref(so), ctypes.byref(lo),
                                 ctypes.byref(rep)) == ldg.LDG_E_INVALID
    assert lib.ldg_newton_step(None, None, None, 1.0, 0.1, ctypes.byref(lo), None) == ldg.LDG_E_INVALID


@pytest.mark.parametrize("dim", [2, 3])
def test_assign_switches_matches_oracle(lib, dim):
    """The library's chord switch function (host code, no device) equals the oracle's
    element for element on meshes with rotated and renumbered elements."""
    from ldg_workloads import hex_mesh, random_rotations, reorient_elements
    from oracle.switches import assign_switches
    from paper_1204_1533_amd.ldg import ldg_assign_switches
    if dim == 2:
        base = quad_mesh(5, 4, 3, box=((0, 5), (0, 4)), periodic=(True, False), perturb=0.1, seed=3)
    else:
        base = hex_mesh(3, 2, length=3.0, periodic=True, amp=0.05)
    axes, flips = random_rotations(dim, base.n_elem, 21, frac=0.7)
    perm = np.random.default_rng(22).permutation(base.n_elem)
    m = reorient_elements(base, flips, perm, axes)
    S_lib = ldg_assign_switches(dim, m.p, m.face_nbr, m.nbr_node)
    S_orc = assign_switches(dim, m.p, m.face_nbr, m.nbr_node)
    assert np.array_equal(S_lib, S_orc)
    assert np.any(S_lib < 0)
    # aligned mesh: all +1
    assert np.all(ldg_assign_switches(dim, base.p, base.face_nbr, base.nbr_node) == 1)


def test_assign_switches_rejects_broken_connectivity(lib):
    from paper_1204_1533_amd.ldg import LDGError, ldg_assign_switches
    m = quad_mesh(3, 3, 2, box=((0, 3), (0, 3)), periodic=(True, True))
    nn = m.nbr_node.copy()
    nn[4, 1, :] = nn[4, 1, ::-1]  # face 1 of element 4 no longer maps back
    with pytest.raises(LDGError) as ei:
        ldg_assign_switches(2, m.p, m.face_nbr, nn)
    assert ei.value.status == -2 and "not reciprocal" in str(ei.value)
    with pytest.raises(LDGError) as ei:
        ldg_assign_switches(4, m.p, m.face_nbr, m.nbr_node)
    assert ei.value.status == -1
