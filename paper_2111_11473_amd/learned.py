"""Learned starting guess: training data from converged solves, training, and evaluation.

Orchestration only.  Every computation runs in the library: the features of the MP2 guess
(thc_guess_features), the solves (thc_iterate), the least-squares targets (thc_guess_targets),
the network's standardization, training steps and BF16 inference (thc_mlp_*), and applying a
prediction (thc_guess_apply).  Python moves arrays between those calls and shuffles row order.

Protocol.  A system is solved from the plain MP2 guess; its per-rank-index features phi_P and
targets (c*_P, delta*_P) become training rows.  A held-out system is solved twice: plainly, and
from the predicted start diag(1 + c) T^0 diag(1 + c) with denominators shifted by delta; if the
learned attempt does not converge it is rerun from the plain guess (fallback) and its iterations
are counted in full.  Both solves use the same convergence test, so the converged residual
decides whether a start was good.

Run:  python -m paper_2111_11473_amd.learned --train 200 --heldout 56 --o-min 10 --o-max 24
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import synth


COUPLING = 0.2


def system_config(s: int, o_min: int, o_max: int, coupling: float | None = None) -> synth.Config:
    """System s of the learned-guess set with o in [o_min, o_max] and the set's ratios
    (v = 9o, nL = 30o, nP = 20o, nQ = 50o); o_min = 30, o_max = 80 is the full-size set.
    `coupling` sets the Cholesky scale (fraction of the smallest pair gap; 0.2 by default)."""
    o = o_min + int(synth.bits(7, 0, np.array([s]))[0] % np.uint64(o_max - o_min + 1))
    c = COUPLING if coupling is None else coupling
    return synth.Config(f"learn{s}", o, 9 * o, 30 * o, 20 * o, 50 * o, 30.0, 2000 + s, coupling=c)


def _context(thc, cfg, singles, tol_energy):
    import torch
    s = synth.make_system(cfg)
    ctx = thc.THC(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ, singles=singles, diis_max=8, tol_energy=tol_energy)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    Z0 = ctx.build_factors(d(s["L"]), d(s["eps"]), d(s["Xo"]), d(s["Xv"]), d(s["xo"]), d(s["xv"]))
    return ctx, Z0


def generate(systems, o_min, o_max, tol=1e-7, tol_energy=1e-8, maxit=100, singles=True, log=print):
    """Training rows (features, targets) from converged plain solves of the given systems."""
    from . import thc
    X, T, info = [], [], []
    for sidx in systems:
        cfg = system_config(sidx, o_min, o_max)
        t0 = time.perf_counter()
        ctx, Z0 = _context(thc, cfg, singles, tol_energy)
        phi = ctx.guess_features()
        Th0, sig0 = ctx.working(residual=True)
        it, rn, ok = ctx.iterate(tol=tol, maxit=maxit, raise_on_notconv=False)
        if not ok:
            log(f"  system {sidx} (o={cfg.o}) did not converge in {maxit}; skipped")
            ctx.close()
            continue
        Ts, _ = ctx.working()
        c, d = ctx.guess_targets(Th0, Ts, sig0)
        X.append(phi.cpu().numpy())
        T.append(np.stack([c.cpu().numpy(), d.cpu().numpy()], axis=1).astype(np.float32))
        info.append({"system": sidx, "o": cfg.o, "nP": cfg.nP, "iterations": it, "energy": ctx.energy(),
                     "seconds": time.perf_counter() - t0})
        ctx.close()
        log(f"  system {sidx}: o={cfg.o} nP={cfg.nP} plain iterations {it} ({info[-1]['seconds']:.1f} s)")
    return np.concatenate(X), np.concatenate(T), info


def train(X, T, epochs=60, batch=4096, lr=2e-3, seed=1, log=print):
    """A fresh network (10 -> 256 -> 256 -> 2, SiLU) trained with Adam on standardized rows."""
    import torch
    from . import thc
    net = thc.MLP(X.shape[1], 256, T.shape[1], seed=seed)
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to("cuda")
    Td = torch.from_numpy(np.ascontiguousarray(T, dtype=np.float32)).to("cuda")
    net.fit_norm(Xd, Td)
    rng = np.random.default_rng(seed)
    losses = []
    first, _ = net.loss_grad(Xd, Td)
    for ep in range(epochs):
        perm = rng.permutation(X.shape[0])
        Xp = torch.from_numpy(np.ascontiguousarray(X[perm], dtype=np.float32)).to("cuda")
        Tp = torch.from_numpy(np.ascontiguousarray(T[perm], dtype=np.float32)).to("cuda")
        step_lr = lr * (0.5 * (1.0 + np.cos(np.pi * ep / epochs)))  # cosine decay
        for b0 in range(0, X.shape[0], batch):
            net.train_step(Xp[b0:b0 + batch], Tp[b0:b0 + batch], max(step_lr, 1e-5))
        loss, _ = net.loss_grad(Xd, Td)
        losses.append(loss)
        if ep % 10 == 0 or ep == epochs - 1:
            log(f"  epoch {ep}: loss {loss:.4f} (initial {first:.4f})")
    return net, first, losses


def solve_pair(net, cfg, tol=1e-7, tol_energy=1e-8, maxit=100, singles=True):
    """Iterations of the plain solve and of the learned-guess solve (with fallback)."""
    from . import thc
    ctx, Z0 = _context(thc, cfg, singles, tol_energy)
    it_p, _, ok_p = ctx.iterate(tol=tol, maxit=maxit, raise_on_notconv=False)
    e_p = ctx.energy()
    ctx.set_state(Z0)
    ctx.set_shift(None)
    phi = ctx.guess_features()
    pred = net.infer(phi)
    ctx.guess_apply(pred)
    fallback = False
    try:
        it_l, _, ok_l = ctx.iterate(tol=tol, maxit=maxit, raise_on_notconv=False)
    except thc.ThcError:  # non-finite residual: the prediction diverged
        it_l, ok_l = maxit, False
    if not ok_l:
        fallback = True
        ctx.set_state(Z0)
        ctx.set_shift(None)
        it2, _, ok_l = ctx.iterate(tol=tol, maxit=maxit, raise_on_notconv=False)
        it_l += it2
    e_l = ctx.energy()
    ctx.close()
    return {"o": cfg.o, "nP": cfg.nP, "plain_iterations": it_p, "learned_iterations": it_l, "plain_converged": ok_p,
            "learned_converged": ok_l, "fallback": fallback, "energy_plain": e_p, "energy_learned": e_l,
            "energy_difference": abs(e_l - e_p)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=200)
    ap.add_argument("--heldout", type=int, default=56)
    ap.add_argument("--o-min", type=int, default=30)
    ap.add_argument("--o-max", type=int, default=80)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--coupling", type=float, default=0.2)
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    global COUPLING
    COUPLING = args.coupling
    log = lambda *a: print(*a, flush=True)
    t0 = time.perf_counter()
    log(f"generating training data from {args.train} systems (o in [{args.o_min}, {args.o_max}])")
    X, T, info = generate(range(args.train), args.o_min, args.o_max, tol=args.tol, log=log)
    log(f"{X.shape[0]} rows; training")
    net, first, losses = train(X, T, epochs=args.epochs, log=log)
    log(f"evaluating on {args.heldout} held-out systems")
    res = []
    for s in range(200, 200 + args.heldout):
        r = solve_pair(net, system_config(s, args.o_min, args.o_max), tol=args.tol)
        r["system"] = s
        res.append(r)
        log(f"  system {s}: o={r['o']} plain {r['plain_iterations']} learned {r['learned_iterations']}"
            f"{' (fallback)' if r['fallback'] else ''} |dE| {r['energy_difference']:.1e}")
    ip = np.array([r["plain_iterations"] for r in res], dtype=float)
    il = np.array([r["learned_iterations"] for r in res], dtype=float)
    report = {"systems_train": args.train, "systems_heldout": args.heldout, "o_range": [args.o_min, args.o_max],
              "coupling": args.coupling, "tol": args.tol,
              "rows": int(X.shape[0]), "loss_initial": first, "loss_final": losses[-1],
              "mean_iterations_plain": float(ip.mean()), "mean_iterations_learned": float(il.mean()),
              "median_iterations_plain": float(np.median(ip)), "median_iterations_learned": float(np.median(il)),
              "mean_reduction": float(1.0 - il.mean() / ip.mean()), "fallbacks": int(sum(r["fallback"] for r in res)),
              "max_energy_difference": float(max(r["energy_difference"] for r in res)),
              "seconds": time.perf_counter() - t0, "heldout": res}
    log(json.dumps({k: v for k, v in report.items() if k != "heldout"}))
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(report, fh, indent=1)


if __name__ == "__main__":
    main()
