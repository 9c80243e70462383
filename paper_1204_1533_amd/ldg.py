"""Thin ctypes binding of libldg.so (argument marshalling only).

Every function mirrors an entry point of ``include/ldg.h`` with the same name;
device arrays are passed as raw pointers (``tensor.data_ptr()``).  The library
must have been built (``paper_1204_1533_amd/build.py``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libldg.so")

LDG_OK = 0
LDG_PRECOND_BILU0, LDG_PRECOND_BLOCK_LU = 0, 1
LDG_E_INVALID, LDG_E_SHAPE, LDG_E_UNSUPPORTED, LDG_E_HIP = -1, -2, -3, -4
LDG_E_NOMEM, LDG_E_NOT_ASSEMBLED, LDG_E_NOT_CONVERGED, LDG_E_NONFINITE = -5, -6, -7, -8
LDG_POISSON, LDG_EULER, LDG_NS = 0, 1, 2
LDG_F64, LDG_F32, LDG_BF16 = 0, 1, 2


class ldg_problem_desc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("p", ctypes.c_int32), ("equation", ctypes.c_int32),
        ("node_family", ctypes.c_int32),
        ("gamma", ctypes.c_double), ("mu", ctypes.c_double), ("prandtl", ctypes.c_double),
        ("c11_interior", ctypes.c_double), ("c11_dirichlet", ctypes.c_double),
        ("n_elem", ctypes.c_int64),
        ("node_xyz_host", ctypes.c_void_p), ("face_nbr_host", ctypes.c_void_p),
        ("nbr_node_host", ctypes.c_void_p), ("switch_plus_host", ctypes.c_void_p),
    ]


class ldg_solver_opts(ctypes.Structure):
    _fields_ = [
        ("restart", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("max_refine", ctypes.c_int32),
        ("storage_prec", ctypes.c_int32), ("rtol", ctypes.c_double), ("inner_rtol", ctypes.c_double),
        ("use_learned", ctypes.c_int32), ("reassemble", ctypes.c_int32),
    ]


class ldg_solver_report(ctypes.Structure):
    _fields_ = [
        ("gmres_iters", ctypes.c_int32), ("refine_steps", ctypes.c_int32), ("fallback_used", ctypes.c_int32),
        ("converged", ctypes.c_int32), ("lin_relres", ctypes.c_double),
        ("newton_res_before", ctypes.c_double), ("newton_res_after", ctypes.c_double),
        ("t_resid_ms", ctypes.c_double), ("t_assemble_ms", ctypes.c_double), ("t_solve_ms", ctypes.c_double),
        ("t_total_ms", ctypes.c_double),
        ("t_jacvec_ms", ctypes.c_double), ("t_k21_ms", ctypes.c_double), ("t_precond_ms", ctypes.c_double),
        ("n_jacvec", ctypes.c_int32), ("n_k21", ctypes.c_int32), ("n_precond", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


LDG_BDF2, LDG_DIRK3, LDG_BACKWARD_EULER = 0, 1, 2


class ldg_step_opts(ctypes.Structure):
    _fields_ = [
        ("scheme", ctypes.c_int32), ("max_newton", ctypes.c_int32), ("newton_rtol", ctypes.c_double),
        ("newton_atol", ctypes.c_double), ("gmres_per_newton", ctypes.c_int32), ("reuse", ctypes.c_int32),
        ("reassemble_after", ctypes.c_int32),
    ]


class ldg_step_report(ctypes.Structure):
    _fields_ = [
        ("stages", ctypes.c_int32), ("newton_iters", ctypes.c_int32), ("max_stage_newton", ctypes.c_int32),
        ("assemblies", ctypes.c_int32), ("gmres_iters", ctypes.c_int32), ("converged", ctypes.c_int32),
        ("fallback_used", ctypes.c_int32), ("newton_res_first", ctypes.c_double),
        ("newton_res_final", ctypes.c_double), ("lin_relres_max", ctypes.c_double),
        ("t_assemble_ms", ctypes.c_double), ("t_solve_ms", ctypes.c_double), ("t_ms", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ldg_sample_batch(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_probe", ctypes.c_int32), ("X_dev", ctypes.c_void_p),
                ("A_dev", ctypes.c_void_p), ("S_dev", ctypes.c_void_p), ("T_dev", ctypes.c_void_p)]


_P = ctypes.c_void_p
_SIGS = {
    "ldg_create": (ctypes.c_int, [ctypes.POINTER(ldg_problem_desc), _P, ctypes.POINTER(_P)]),
    "ldg_destroy": (None, [_P]),
    "ldg_set_preconditioner": (ctypes.c_int, [_P, ctypes.c_int32]),
    "ldg_assign_switches": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _P, _P, _P]),
    "ldg_set_source": (ctypes.c_int, [_P, _P]),
    "ldg_set_dirichlet": (ctypes.c_int, [_P, _P]),
    "ldg_set_neumann": (ctypes.c_int, [_P, _P]),
    "ldg_set_c22": (ctypes.c_int, [_P, ctypes.c_double]),
    "ldg_coupled_solve": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "ldg_gradient": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32]),
    "ldg_residual": (ctypes.c_int, [_P, _P, _P, _P]),
    "ldg_jacobian_assemble": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_int32]),
    "ldg_jacvec": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32]),
    "ldg_jacvec_noalloc": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32]),
    "ldg_precond_apply": (ctypes.c_int, [_P, _P, _P]),
    "ldg_export_operators": (ctypes.c_int, [_P, _P, _P, _P]),
    "ldg_newton_step": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.c_double,
                                       ctypes.POINTER(ldg_solver_opts), ctypes.POINTER(ldg_solver_report)]),
    "ldg_implicit_step": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.POINTER(ldg_step_opts),
                                         ctypes.POINTER(ldg_solver_opts), ctypes.POINTER(ldg_step_report)]),
    "ldg_rk4": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_int32]),
    "ldg_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ldg_last_error": (ctypes.c_char_p, [_P]),
    "ldg_num_dofs": (ctypes.c_int64, [_P]),
    "ldg_net_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                      _P, ctypes.POINTER(_P)]),
    "ldg_net_destroy": (None, [_P]),
    "ldg_net_num_params": (ctypes.c_int64, [_P]),
    "ldg_net_set_params": (ctypes.c_int, [_P, _P]),
    "ldg_net_get_params": (ctypes.c_int, [_P, _P]),
    "ldg_net_forward": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int32, _P]),
    "ldg_net_loss_grad": (ctypes.c_int, [_P, ctypes.POINTER(ldg_sample_batch), ctypes.c_int32, _P,
                                         ctypes.POINTER(ctypes.c_double)]),
    "ldg_net_adam_step": (ctypes.c_int, [_P, ctypes.c_double]),
    "ldg_net_last_error": (ctypes.c_char_p, [_P]),
    "ldg_learned_attach": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "ldg_learned_collect": (ctypes.c_int, [_P, ctypes.c_int32]),
    "ldg_learned_active": (ctypes.c_int32, [_P]),
    "ldg_learned_samples": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, ctypes.c_int32, _P, _P, _P, _P]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libldg.so; raises if it has not been built (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1204_1533_amd/build.py")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGS)


class LDGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status}: {msg}")
        self.status = status


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def ldg_assign_switches(dim, p, face_nbr, nbr_node):
    """Switch function S^+ [E][D] (int8) for the given connectivity (host arrays)."""
    lib = load_library()
    fn = np.ascontiguousarray(face_nbr, dtype=np.int64)
    nn = np.ascontiguousarray(nbr_node, dtype=np.int32)
    out = np.zeros((fn.shape[0], dim), dtype=np.int8)
    st = lib.ldg_assign_switches(int(dim), int(p), int(fn.shape[0]), fn.ctypes.data, nn.ctypes.data,
                                 out.ctypes.data)
    if st != LDG_OK:
        raise LDGError(st, lib.ldg_last_error(None).decode())
    return out


class Context:
    """Owns one ldg_ctx.  Device arrays are torch tensors on the GPU (float64)."""

    def __init__(self, mesh, equation, gamma=1.4, mu=0.0, prandtl=0.72, c11_interior=0.0, c11_dirichlet=10.0,
                 node_family=0, stream=None):
        lib = load_library()
        self.lib = lib
        self.mesh = mesh
        self._keep = dict(
            xyz=np.ascontiguousarray(mesh.xyz, dtype=np.float64),
            fn=np.ascontiguousarray(mesh.face_nbr, dtype=np.int64),
            nn=np.ascontiguousarray(mesh.nbr_node, dtype=np.int32),
            sw=np.ascontiguousarray(mesh.switch_plus, dtype=np.int8),
        )
        d = ldg_problem_desc()
        d.dim, d.p, d.equation, d.node_family = mesh.dim, mesh.p, equation, node_family
        d.gamma, d.mu, d.prandtl = gamma, mu, prandtl
        d.c11_interior, d.c11_dirichlet = c11_interior, c11_dirichlet
        d.n_elem = mesh.n_elem
        d.node_xyz_host = self._keep["xyz"].ctypes.data
        d.face_nbr_host = self._keep["fn"].ctypes.data
        d.nbr_node_host = self._keep["nn"].ctypes.data
        d.switch_plus_host = self._keep["sw"].ctypes.data
        self.desc = d
        h = _P()
        st = lib.ldg_create(ctypes.byref(d), stream, ctypes.byref(h))
        if st != LDG_OK:
            raise LDGError(st, lib.ldg_last_error(None).decode())
        self.h = h
        self.dim, self.p = mesh.dim, mesh.p
        self.m = 1 if equation == LDG_POISSON else mesh.dim + 2
        self.n1 = mesh.p + 1
        self.Np = self.n1 ** mesh.dim
        self.E = mesh.n_elem

    def _check(self, st):
        if st != LDG_OK:
            raise LDGError(st, self.lib.ldg_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.ldg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # thin wrappers with the ABI names
    def ldg_set_source(self, S):
        self._check(self.lib.ldg_set_source(self.h, _ptr(S)))

    def ldg_set_dirichlet(self, gD):
        self._check(self.lib.ldg_set_dirichlet(self.h, _ptr(gD)))

    def ldg_set_neumann(self, gN):
        self._check(self.lib.ldg_set_neumann(self.h, _ptr(gN)))

    def ldg_set_c22(self, c22):
        self._check(self.lib.ldg_set_c22(self.h, float(c22)))

    def ldg_coupled_solve(self, U, Q, rtol=1e-10, inner_rtol=1e-2, restart=60, max_iters=500, raise_on_error=True):
        its = ctypes.c_int32(0)
        inner = ctypes.c_int32(0)
        rr = ctypes.c_double(0.0)
        st = self.lib.ldg_coupled_solve(self.h, _ptr(U), _ptr(Q), float(rtol), float(inner_rtol), int(restart),
                                        int(max_iters), ctypes.byref(its), ctypes.byref(inner), ctypes.byref(rr))
        if raise_on_error:
            self._check(st)
        return {"status": st, "iters": int(its.value), "inner_iters": int(inner.value), "relres": float(rr.value)}

    def ldg_gradient(self, U, Q, homogeneous=False):
        self._check(self.lib.ldg_gradient(self.h, _ptr(U), _ptr(Q), int(homogeneous)))

    def ldg_residual(self, U, R, Q=None):
        self._check(self.lib.ldg_residual(self.h, _ptr(U), _ptr(R), _ptr(Q)))

    def ldg_jacobian_assemble(self, U, alpha, gamma, storage_prec=LDG_F64):
        self._check(self.lib.ldg_jacobian_assemble(self.h, _ptr(U), float(alpha), float(gamma), int(storage_prec)))

    def ldg_jacvec(self, x, y, exact_fp64=False):
        self._check(self.lib.ldg_jacvec(self.h, _ptr(x), _ptr(y), int(exact_fp64)))

    def ldg_jacvec_noalloc(self, x, y, exact_fp64=False):
        self._check(self.lib.ldg_jacvec_noalloc(self.h, _ptr(x), _ptr(y), int(exact_fp64)))

    def ldg_set_preconditioner(self, kind):
        self._check(self.lib.ldg_set_preconditioner(self.h, int(kind)))

    def ldg_precond_apply(self, r, z):
        self._check(self.lib.ldg_precond_apply(self.h, _ptr(r), _ptr(z)))

    def ldg_export_operators(self, K11=None, K12=None, F=None):
        self._check(self.lib.ldg_export_operators(self.h, _ptr(K11), _ptr(K12), _ptr(F)))

    def ldg_newton_step(self, U, Ucomb, alpha, gamma, restart=50, max_iters=2000, max_refine=20,
                        storage_prec=LDG_F64, rtol=1e-8, inner_rtol=1e-3, use_learned=0, reassemble=1,
                        raise_on_error=True):
        o = ldg_solver_opts(restart, max_iters, max_refine, storage_prec, rtol, inner_rtol, use_learned, reassemble)
        rep = ldg_solver_report()
        st = self.lib.ldg_newton_step(self.h, _ptr(U), _ptr(Ucomb), float(alpha), float(gamma), ctypes.byref(o),
                                      ctypes.byref(rep))
        if raise_on_error:
            self._check(st)
        out = rep.as_dict()
        out["status"] = st
        return out

    def ldg_implicit_step(self, U, Uprev, dt, scheme=LDG_DIRK3, max_newton=30, newton_rtol=1e-8, newton_atol=0.0,
                          gmres_per_newton=0, reuse=1, reassemble_after=15, restart=50, max_iters=2000,
                          max_refine=20, storage_prec=LDG_F64, rtol=1e-8, inner_rtol=1e-3, use_learned=0,
                          raise_on_error=True):
        so = ldg_step_opts(scheme, max_newton, newton_rtol, newton_atol, gmres_per_newton, reuse, reassemble_after)
        lo = ldg_solver_opts(restart, max_iters, max_refine, storage_prec, rtol, inner_rtol, use_learned, 0)
        rep = ldg_step_report()
        st = self.lib.ldg_implicit_step(self.h, _ptr(U), _ptr(Uprev), float(dt), ctypes.byref(so), ctypes.byref(lo),
                                        ctypes.byref(rep))
        if raise_on_error:
            self._check(st)
        out = rep.as_dict()
        out["status"] = st
        return out

    def ldg_rk4(self, U, dt, n_steps):
        self._check(self.lib.ldg_rk4(self.h, _ptr(U), float(dt), int(n_steps)))

    def ldg_num_dofs(self):
        return int(self.lib.ldg_num_dofs(self.h))

    def ldg_learned_attach(self, net, infer_prec=LDG_BF16):
        self._net = net
        self._check(self.lib.ldg_learned_attach(self.h, net.h if net is not None else None, int(infer_prec)))

    def ldg_learned_collect(self, on=True):
        self._check(self.lib.ldg_learned_collect(self.h, int(on)))

    def ldg_learned_active(self):
        return int(self.lib.ldg_learned_active(self.h))

    def ldg_learned_samples(self, elems, V, K, X, A, S, T):
        el = np.ascontiguousarray(elems, dtype=np.int64)
        self._check(self.lib.ldg_learned_samples(self.h, el.ctypes.data, len(el), _ptr(V), int(K), _ptr(X), _ptr(A),
                                                 _ptr(S), _ptr(T)))

    # sizes of the exchange layouts
    def nslots(self):
        D, p = self.dim, self.p
        return D * p + 1 + 2 * D, D * p + 1 + D, D * p + 1


class Net:
    """Owns one ldg_net (the learned preconditioner correction's network)."""

    def __init__(self, dim, p, m, hidden=256, seed=0, stream=None):
        lib = load_library()
        self.lib = lib
        h = _P()
        st = lib.ldg_net_create(int(dim), int(p), int(m), int(hidden), int(seed), stream, ctypes.byref(h))
        if st != LDG_OK:
            raise LDGError(st, lib.ldg_status_string(st).decode())
        self.h = h
        self.dim, self.p, self.m, self.hidden = dim, p, m, hidden
        self.np_ = (p + 1) ** dim
        self.n_in = self.np_ * m * m + self.np_ * m
        self.n_out = self.np_ * m * m

    def _check(self, st):
        if st != LDG_OK:
            raise LDGError(st, self.lib.ldg_net_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.ldg_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def ldg_net_num_params(self):
        return int(self.lib.ldg_net_num_params(self.h))

    def ldg_net_set_params(self, params):
        self._check(self.lib.ldg_net_set_params(self.h, _ptr(params)))

    def ldg_net_get_params(self, params):
        self._check(self.lib.ldg_net_get_params(self.h, _ptr(params)))

    def ldg_net_forward(self, X, n, prec, Y):
        self._check(self.lib.ldg_net_forward(self.h, _ptr(X), int(n), int(prec), _ptr(Y)))

    def ldg_net_loss_grad(self, X, A, S, T, n, n_probe, prec=LDG_BF16, grad=None):
        b = ldg_sample_batch(int(n), int(n_probe), _ptr(X), _ptr(A), _ptr(S), _ptr(T))
        loss = ctypes.c_double()
        self._check(self.lib.ldg_net_loss_grad(self.h, ctypes.byref(b), int(prec), _ptr(grad), ctypes.byref(loss)))
        return loss.value

    def ldg_net_adam_step(self, lr):
        self._check(self.lib.ldg_net_adam_step(self.h, float(lr)))
