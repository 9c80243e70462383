"""Shared construction of workloads for the GPU parity tests (oracle and GPU sides)."""
import numpy as np
import torch

from ldg_workloads import configs, fields, hex_mesh, quad_mesh
from oracle import LineDG, Physics


def oracle_of(pr):
    me = pr.mesh
    ph = Physics(pr.equation, me.dim, gamma=pr.gamma, mu=pr.mu, prandtl=pr.prandtl)
    return LineDG(me.dim, me.p, me.xyz, me.face_nbr, me.nbr_node, me.switch_plus, ph,
                  pr.c11_interior, pr.c11_dirichlet, pr.source, pr.gD)


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


def case(name):
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


def rounding_sensitivity(orc, pr, elems=None, seed=0):
    """Largest change of the oracle residual under random one-ulp perturbations of its
    inputs (node coordinates, then state): the scale of rounding differences that two
    correct FP64 evaluations of the same residual can show."""
    from oracle import LineDG
    rng = np.random.default_rng(seed)
    base = orc.residual(pr.U0, elems=elems)
    x = pr.mesh.xyz * (1 + 2.0 ** -52 * rng.standard_normal(pr.mesh.xyz.shape))
    o2 = LineDG(pr.mesh.dim, pr.mesh.p, x, pr.mesh.face_nbr, pr.mesh.nbr_node, pr.mesh.switch_plus, orc.ph,
                pr.c11_interior, pr.c11_dirichlet, pr.source, pr.gD)
    s1 = float((o2.residual(pr.U0, elems=elems) - base).abs().max())
    U1 = pr.U0 * (1 + 2.0 ** -52 * rng.standard_normal(pr.U0.shape))
    s2 = float((orc.residual(U1, elems=elems) - base).abs().max())
    return max(s1, s2)
