"""Data generation, training and evaluation of the learned preconditioner correction.

Orchestration only: every arithmetic step runs in libldg's kernels through the
C ABI (Newton steps, sample extraction, network forward / backward / Adam);
torch provides device buffers, seeded random probes and batch gathers.

Recipe (3-D Navier-Stokes Taylor-Green runs, p = 3): for each seed s the
Reynolds number is uniform in [200, 2000] and the Mach number uniform in
[0.1, 0.4] (numpy default_rng(s)), with a seeded low-mode velocity
perturbation of amplitude 0.05.  Each run takes BDF2 steps (dt = 0.05, one
Newton step each, FP32 storage); after each step's assembly `n_elem` random
elements are sampled with `n_probe` Gaussian probes.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from .ldg import LDG_BDF2, LDG_BF16, LDG_F32, Context, Net


def _log(msg, log):
    if log:
        print(msg, flush=True)


def problem(seed, n, p=3):
    from ldg_workloads import configs
    return configs.config5_sample(seed, n=n, p=p)


def context_for(pr, stream):
    return Context(pr.mesh, pr.equation, gamma=pr.gamma, mu=pr.mu, prandtl=pr.prandtl,
                   c11_interior=pr.c11_interior, c11_dirichlet=pr.c11_dirichlet, stream=stream)


class SampleSet:
    """Training samples on the device (FP32), rows appended in order."""

    def __init__(self, capacity, n_in, np_, nsl, m, n_probe):
        dev = "cuda"
        self.X = torch.empty(capacity, n_in, device=dev)
        self.A = torch.empty(capacity, np_, nsl, m, m, device=dev)
        self.S = torch.empty(capacity, n_probe, np_, m, device=dev)
        self.T = torch.empty(capacity, n_probe, np_, m, device=dev)
        self.n = 0
        self.n_probe = n_probe

    def view(self, sl):
        return self.X[sl], self.A[sl], self.S[sl], self.T[sl]


def generate(seeds, n=24, p=3, steps=10, n_elem=256, n_probe=4, rtol=1e-6, seed_probes=0, log=True):
    """Run the solver on each seed and collect samples after every Newton step's assembly."""
    stream = torch.cuda.current_stream().cuda_stream
    data = None
    g = torch.Generator(device="cuda").manual_seed(seed_probes)
    t0 = time.perf_counter()
    for s in seeds:
        pr = problem(s, n, p)
        ctx = context_for(pr, stream)
        ctx.ldg_learned_collect(True)
        E, m, Np = pr.mesh.n_elem, pr.m, pr.mesh.np_
        D = pr.mesh.dim
        nsl = D * p + 1
        if data is None:
            data = SampleSet(len(seeds) * steps * n_elem, Np * m * m + Np * m, Np, nsl, m, n_probe)
        rng = np.random.default_rng(10_000 + s)
        U = torch.as_tensor(pr.U0, device="cuda").contiguous()
        Uprev = U.clone()
        V = torch.empty(n_probe, E, m, Np, dtype=torch.float64, device="cuda")
        for k in range(steps):
            # one Newton iteration per BDF2 step (the library forms (4 U^n - U^{n-1}) / 3 and keeps the history)
            rep = ctx.ldg_implicit_step(U, Uprev, pr.dt, scheme=LDG_BDF2, max_newton=1, newton_rtol=0.0,
                                        newton_atol=0.0, reuse=0, storage_prec=LDG_F32, rtol=rtol, inner_rtol=1e-2,
                                        max_iters=3000)
            el = np.sort(rng.choice(E, size=min(n_elem, E), replace=False))
            V.normal_(generator=g)
            i0 = data.n
            i1 = i0 + len(el)
            X, A, S, T = data.view(slice(i0, i1))
            ctx.ldg_learned_samples(el, V, n_probe, X, A, S, T)
            data.n = i1
            _log(f"[learned] seed {s} step {k}: gmres {rep['gmres_iters']}, samples {data.n}, "
                 f"{time.perf_counter() - t0:.1f} s", log)
        ctx.close()
    return data


def train(net, data, iters=2000, batch=512, lr=1e-3, prec=LDG_BF16, seed=0, log_every=100, log=True):
    """Adam on random batches; returns the loss history (one value per iteration)."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    hist = []
    t0 = time.perf_counter()
    for it in range(iters):
        idx = torch.randint(0, data.n, (batch,), device="cuda", generator=g)
        X, A, S, T = data.X[idx], data.A[idx], data.S[idx], data.T[idx]
        loss = net.ldg_net_loss_grad(X, A, S, T, batch, data.n_probe, prec=prec)
        net.ldg_net_adam_step(lr)
        hist.append(loss)
        if log and (it % log_every == 0 or it == iters - 1):
            _log(f"[learned] iter {it}: loss {loss:.5f} ({time.perf_counter() - t0:.1f} s)", log)
    return hist


def evaluate(net, seeds, n=24, p=3, steps=1, storage_prec=LDG_F32, infer_prec=LDG_BF16, rtol=1e-8,
             inner_rtol=1e-3, log=True):
    """Newton steps with and without the correction; GMRES iterations and residuals per seed."""
    stream = torch.cuda.current_stream().cuda_stream
    out = []
    for s in seeds:
        pr = problem(s, n, p)
        ctx = context_for(pr, stream)
        ctx.ldg_learned_attach(net, infer_prec)
        U0 = torch.as_tensor(pr.U0, device="cuda").contiguous()
        row = {"seed": s, "re": pr.extra["re"], "mach": pr.extra["mach"]}
        for use in (0, 1):
            U = U0.clone()
            reps = []
            Uprev = U0.clone()
            for k in range(steps):
                r = ctx.ldg_implicit_step(U, Uprev, pr.dt, scheme=LDG_BDF2, max_newton=1, newton_rtol=0.0,
                                          newton_atol=0.0, reuse=0, storage_prec=storage_prec, rtol=rtol,
                                          inner_rtol=inner_rtol, use_learned=use, max_iters=4000)
                reps.append(r)
            key = "learned" if use else "ilu0"
            row[key] = {"gmres_iters": int(sum(r["gmres_iters"] for r in reps)),
                        "lin_relres": max(r["lin_relres_max"] for r in reps),
                        "newton_res_after": reps[-1]["newton_res_final"],
                        "t_solve_ms": float(sum(r["t_solve_ms"] for r in reps)),
                        "fallback_used": int(max(r["fallback_used"] for r in reps))}
            row[key + "_U"] = U
        _log(f"[learned] eval seed {s}: ilu0 {row['ilu0']['gmres_iters']} its, learned "
             f"{row['learned']['gmres_iters']} its", log)
        ctx.close()
        out.append(row)
    return out


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="generate samples, train the correction network, evaluate it")
    ap.add_argument("--n", type=int, default=24)
    ap.add_argument("--train-seeds", type=int, default=200)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--elems", type=int, default=256)
    ap.add_argument("--probes", type=int, default=4)
    ap.add_argument("--iters", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-seeds", type=int, default=20)
    ap.add_argument("--save", default="")
    a = ap.parse_args()
    torch.cuda.set_device(0)
    data = generate(list(range(a.train_seeds)), n=a.n, steps=a.steps, n_elem=a.elems, n_probe=a.probes)
    stream = torch.cuda.current_stream().cuda_stream
    net = Net(3, 3, 5, hidden=256, seed=1, stream=stream)
    hist = train(net, data, iters=a.iters, batch=a.batch, lr=a.lr)
    res = evaluate(net, list(range(1000, 1000 + a.eval_seeds)), n=a.n)
    summary = [{k: v for k, v in r.items() if not k.endswith("_U")} for r in res]
    print(json.dumps({"loss_first": hist[0], "loss_last": float(np.mean(hist[-50:])), "eval": summary}))
    if a.save:
        w = torch.empty(net.ldg_net_num_params(), device="cuda")
        net.ldg_net_get_params(w)
        torch.save(w.cpu(), a.save)


if __name__ == "__main__":
    main()
