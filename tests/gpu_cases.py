"""Shared construction of workloads for the GPU parity tests (oracle and GPU sides)."""
import numpy as np
import torch

from ldg_workloads import configs, fields, hex_mesh, quad_mesh
from oracle import LineDG, Physics


def oracle_of(pr):
    me = pr.mesh
    ph = Physics(pr.equation, me.dim, gamma=pr.gamma, mu=pr.mu, prandtl=pr.prandtl)
    return LineDG(me.dim, me.p, me.xyz, me.face_nbr, me.nbr_node, me.switch_plus, ph,
                  pr.c11_interior, pr.c11_dirichlet, pr.source, pr.gD, gN=pr.gN)


def gpu_of(pr):
    from paper_1204_1533_amd import Context
    stream = torch.cuda.current_stream().cuda_stream
    ctx = Context(pr.mesh, pr.equation, gamma=pr.gamma, mu=pr.mu, prandtl=pr.prandtl,
                  c11_interior=pr.c11_interior, c11_dirichlet=pr.c11_dirichlet, stream=stream)
    dev = {}
    if pr.source is not None:
        dev["S"] = torch.as_tensor(pr.source, device="cuda").contiguous()
        ctx.ldg_set_source(dev["S"])
    if pr.gD is not None:
        dev["gD"] = torch.as_tensor(pr.gD, device="cuda").contiguous()
        ctx.ldg_set_dirichlet(dev["gD"])
    if pr.gN is not None:
        dev["gN"] = torch.as_tensor(pr.gN, device="cuda").contiguous()
        ctx.ldg_set_neumann(dev["gN"])
    ctx._dev = dev
    return ctx


def small_ns_2d(p=3, n=4, mu=0.05, seed=0):
    mesh = quad_mesh(n, n, p, box=((0, 4), (0, 4)), periodic=(True, True), perturb=0.2, seed=seed)
    U = fields.random_smooth_state(mesh, 4, seed=seed + 1, base=[1.0, 0.3, -0.2, 2.6], amp=0.1)
    return configs.Problem(f"ns2d_n{n}p{p}", mesh, configs.EQ_NS, 4, U, mu=mu)


def small_euler_3d(p=2, n=3, seed=0):
    mesh = hex_mesh(n, p)
    U = fields.random_smooth_state(mesh, 5, seed=seed + 1, base=[1.0, 0.3, -0.2, 0.1, 2.6], amp=0.1)
    return configs.Problem(f"euler3d_n{n}p{p}", mesh, configs.EQ_EULER, 5, U)


def small_poisson_3d(p=2, n=2):
    mesh = hex_mesh(n, p, length=1.0, periodic=False, amp=0.05)
    u, f, g = fields.poisson_polynomial_3d(mesh, degs=(2, 1, 2))
    return configs.Problem(f"poisson3d_n{n}p{p}", mesh, configs.EQ_POISSON, 1, u, source=f,
                           gD=fields.face_values(mesh, u), c11_dirichlet=10.0)


def flip_mesh(mesh, seed, frac=0.5):
    """Reverse two local axes of a seeded random subset of elements (a rotation by 180 degrees
    in the plane of those axes) and renumber the elements, so that switch signs S = -1 and
    reversed face-node maps occur.  Returns (mesh, flips, perm)."""
    from ldg_workloads import reorient_elements
    rng = np.random.default_rng(seed)
    E, D = mesh.n_elem, mesh.dim
    flips = np.zeros((E, D), dtype=bool)
    for e in np.nonzero(rng.random(E) < frac)[0]:
        flips[e, rng.choice(D, size=2, replace=False)] = True
    perm = rng.permutation(E)
    return reorient_elements(mesh, flips, perm), flips, perm


def rotate_mesh(mesh, seed, frac=1.0):
    """Rotate the local frames of a seeded random subset of elements by any rotation of the
    square / cube (axis permutations with flips), renumber the elements, and give the result
    the switch function of the chord algorithm.  Returns (mesh, flips, perm, axes)."""
    from ldg_workloads import random_rotations, reorient_elements
    from ldg_workloads.mesh import Mesh
    from oracle.switches import assign_switches
    rng = np.random.default_rng(seed)
    axes, flips = random_rotations(mesh.dim, mesh.n_elem, seed + 1, frac)
    perm = rng.permutation(mesh.n_elem)
    m2 = reorient_elements(mesh, flips, perm, axes)
    sw = assign_switches(m2.dim, m2.p, m2.face_nbr, m2.nbr_node)
    m3 = Mesh(m2.dim, m2.p, m2.xyz, m2.face_nbr, m2.nbr_node, sw, name=m2.name + "+chords")
    return m3, flips, perm, axes


def relabel_nodal(V, mesh, flips, perm, axes=None):
    """A nodal field [E][C][Np] of the original mesh in the numbering of the relabelled mesh
    (new local axis d = old axis axes[e, d], reversed where flips[e, d])."""
    n1, D = mesh.p + 1, mesh.dim
    idx = np.arange(mesh.np_)
    coords = [(idx // n1 ** d) % n1 for d in range(D)]
    out = np.empty_like(V)
    for e in range(mesh.n_elem):
        ax = range(D) if axes is None else axes[e]
        c_old = [None] * D
        for d, a in enumerate(ax):
            c_old[a] = mesh.p - coords[d] if flips[e, d] else coords[d]
        old = np.zeros_like(idx)
        for a in reversed(range(D)):
            old = old * n1 + c_old[a]
        out[perm[e]] = V[e][:, old]
    return out


def poisson_mixed(p=3, n=3, dim=2):
    """Poisson with Dirichlet faces xi_n = 0 and Neumann faces xi_n = 1 of the box (rectangular
    elements), u in Q_p with its Dirichlet values and Neumann data -grad u . nhat."""
    from ldg_workloads import BC_NEUMANN, with_boundary_kinds
    if dim == 2:
        base = quad_mesh(n, n, p, box=((0.2, 1.4), (-0.3, 0.9)))
        u, f, g = fields.poisson_polynomial(base, degs=(p, p - 1))
    else:
        base = hex_mesh(n, p, length=1.0, periodic=False, amp=0.0)
        u, f, g = fields.poisson_polynomial_3d(base, degs=(p, 1, p))
    mesh = with_boundary_kinds(base, {2 * k + 1: BC_NEUMANN for k in range(dim)})
    pr = configs.Problem(f"poisson{dim}d_mixed_n{n}p{p}", mesh, configs.EQ_POISSON, 1,
                         u + 0.05 * np.sin(3.0 * mesh.xyz[:, 0:1]), source=f, gD=fields.face_values(mesh, u),
                         gN=-fields.axis_normal_face_values(mesh, g), c11_dirichlet=10.0)
    pr.extra["u_exact"] = u
    return pr


def channel_case(eq, p=3, seed=0):
    """Periodic in x, slip walls at y = 0 and y = 2 on a perturbed mesh; a smooth random state."""
    from ldg_workloads import BC_SLIP, with_boundary_kinds
    base = quad_mesh(4, 3, p, box=((0, 4), (0, 2)), periodic=(True, False), perturb=0.2, seed=3)
    mesh = with_boundary_kinds(base, {2: BC_SLIP, 3: BC_SLIP})
    U = fields.random_smooth_state(mesh, 4, seed=seed + 1, base=[1.0, 0.3, -0.2, 2.6], amp=0.1)
    return configs.Problem(f"channel_{'ns' if eq == configs.EQ_NS else 'euler'}_p{p}", mesh, eq, 4, U,
                           mu=0.05 if eq == configs.EQ_NS else 0.0)


def box_mixed_ns(p=2, seed=0):
    """3-D Navier-Stokes on a non-periodic 2^3 box: Dirichlet faces x = 0, 1, slip walls y = 0, 1,
    Neumann faces z = 0, 1 (data: a smooth field's face values, small)."""
    from ldg_workloads import BC_NEUMANN, BC_SLIP, with_boundary_kinds
    base = hex_mesh(2, p, length=1.0, periodic=False, amp=0.05)
    mesh = with_boundary_kinds(base, {2: BC_SLIP, 3: BC_SLIP, 4: BC_NEUMANN, 5: BC_NEUMANN})
    st = [1.0, 0.3, -0.2, 0.1, 2.6]
    U = fields.random_smooth_state(mesh, 5, seed=seed + 1, base=st, amp=0.05)
    gD = fields.face_values(mesh, fields.random_smooth_state(mesh, 5, seed=seed + 2, base=st, amp=0.05))
    gN = 0.05 * fields.face_values(mesh, fields.random_smooth_state(mesh, 5, seed=seed + 3, base=None, amp=1.0))
    return configs.Problem(f"box_mixed_ns_p{p}", mesh, configs.EQ_NS, 5, U, mu=0.05, gD=gD, gN=gN)


def case(name):
    if name == "poisson2d_mixed":
        return poisson_mixed(3, 3, 2)
    if name == "poisson3d_mixed":
        return poisson_mixed(2, 2, 3)
    if name == "channel_euler":
        return channel_case(configs.EQ_EULER)
    if name == "channel_ns":
        return channel_case(configs.EQ_NS)
    if name == "box_mixed_ns":
        return box_mixed_ns()
    if name.endswith("_flip"):
        # the same workload on a mesh whose elements have reversed axes (S = -1 faces)
        pr = case(name[:-len("_flip")])
        assert pr.source is None and pr.gD is None
        mesh2, flips, perm = flip_mesh(pr.mesh, seed=17)
        U2 = relabel_nodal(pr.U0, pr.mesh, flips, perm)
        return configs.Problem(pr.name + "_flip", mesh2, pr.equation, pr.m, U2, gamma=pr.gamma, mu=pr.mu,
                               prandtl=pr.prandtl, c11_interior=pr.c11_interior,
                               c11_dirichlet=pr.c11_dirichlet, dt=pr.dt, extra=dict(pr.extra))
    if name.endswith("_rot"):
        # the same workload on a mesh whose element frames are rotated (axis permutations and
        # reversals), renumbered, with the switch function of the chord algorithm
        pr = case(name[:-len("_rot")])
        assert pr.source is None and pr.gD is None
        mesh2, flips, perm, axes = rotate_mesh(pr.mesh, seed=23)
        U2 = relabel_nodal(pr.U0, pr.mesh, flips, perm, axes)
        return configs.Problem(pr.name + "_rot", mesh2, pr.equation, pr.m, U2, gamma=pr.gamma, mu=pr.mu,
                               prandtl=pr.prandtl, c11_interior=pr.c11_interior,
                               c11_dirichlet=pr.c11_dirichlet, dt=pr.dt, extra=dict(pr.extra))
    if name == "C1":
        pr = configs.config1()
        pr.U0 = pr.extra["u_exact"] + 0.01 * np.sin(7 * pr.mesh.xyz[:, 0:1])  # a non-trivial state
        return pr
    if name == "C2":
        return configs.config2()
    if name == "C3":
        return configs.config3()
    if name == "C4":
        return configs.config4()
    if name.startswith("ns2d"):
        return small_ns_2d(p=int(name[-1]))
    if name.startswith("euler3d"):
        return small_euler_3d(p=int(name[-1]))
    if name.startswith("poisson3d"):
        return small_poisson_3d(p=int(name[-1]))
    if name.startswith("tgv"):  # tgv<n>p<p>
        n, p = name[3:].split("p")
        return configs.taylor_green(int(n), int(p), 400.0)
    raise KeyError(name)


def rounding_sensitivity(orc, pr, elems=None, seed=0, per_component=False):
    """Largest change of the oracle residual under random one-ulp perturbations of its
    inputs (node coordinates, then state): the scale of rounding differences that two
    correct FP64 evaluations of the same residual can show (per component if asked)."""
    from oracle import LineDG
    rng = np.random.default_rng(seed)
    base = orc.residual(pr.U0, elems=elems)
    x = pr.mesh.xyz * (1 + 2.0 ** -52 * rng.standard_normal(pr.mesh.xyz.shape))
    o2 = LineDG(pr.mesh.dim, pr.mesh.p, x, pr.mesh.face_nbr, pr.mesh.nbr_node, pr.mesh.switch_plus, orc.ph,
                pr.c11_interior, pr.c11_dirichlet, pr.source, pr.gD)
    d1 = (o2.residual(pr.U0, elems=elems) - base).abs()
    U1 = pr.U0 * (1 + 2.0 ** -52 * rng.standard_normal(pr.U0.shape))
    d2 = (orc.residual(U1, elems=elems) - base).abs()
    if per_component:
        return np.maximum(d1.amax(dim=(0, 2)).numpy(), d2.amax(dim=(0, 2)).numpy())
    return max(float(d1.max()), float(d2.max()))


def record(case_name, quantity, err, bound):
    """Append a measured parity error and its bound to the file named by LDG_PARITY_LOG (if set)."""
    import json
    import os
    path = os.environ.get("LDG_PARITY_LOG")
    print(f"  [{case_name}] {quantity}: error {err:.3e}, bound {bound:.3e}, ratio {err / bound if bound else 0:.2e}",
          flush=True)
    if path:
        with open(path, "a") as f:
            f.write(json.dumps({"case": case_name, "quantity": quantity, "err": float(err), "bound": float(bound)}) + "\n")
