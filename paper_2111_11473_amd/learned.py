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


def _context(thc, cfg, singles, tol_energy, precision=0):
    """A context for system cfg with its inputs generated on the GPU by the library (the same
    values as synth.make_system) and the factors built; returns (context, MP2-guess core Z0)."""
    ctx = thc.THC(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ, singles=singles, diis_max=8, tol_energy=tol_energy,
                  precision=precision)
    ctx.set_synthetic(cfg.seed, cfg.decay, cfg.coupling, 0.0 if cfg.gamma is None else cfg.gamma)
    return ctx, ctx.build_synthetic()


def _to_target(energies, seconds, e_ref, thresh=1e-6):
    """(iterations, seconds) until the energy is within thresh of e_ref and stays there."""
    k = len(energies)
    while k > 0 and abs(energies[k - 1] - e_ref) < thresh:
        k -= 1
    if k == len(energies):
        return None, None
    return k + 1, seconds[k]


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


def _learned_solve(ctx, Z0, net, tol, maxit):
    """Solve from the network's prediction with fallback to the plain guess; returns
    (iterations, converged, fallback, energies, seconds) with the fallback's record appended."""
    from . import thc
    ctx.set_state(Z0)
    ctx.set_shift(None)
    ctx.guess_apply(net.infer(ctx.guess_features()))
    fallback = False
    try:
        it, _, ok = ctx.iterate(tol=tol, maxit=maxit, raise_on_notconv=False)
        e, _, t = ctx.history()
    except thc.ThcError:  # the prediction diverged past the solver's own restart
        it, ok, e, t = maxit, False, [], []
    if not ok:
        fallback = True
        t_used = t[-1] if t else 0.0
        ctx.set_state(Z0)
        ctx.set_shift(None)
        it2, _, ok = ctx.iterate(tol=tol, maxit=maxit, raise_on_notconv=False)
        e2, _, t2 = ctx.history()
        it, e, t = it + it2, e + e2, t + [t_used + x for x in t2]
    return it, ok, fallback, e, t


def solve_pair(net, cfg, tol=1e-7, tol_energy=1e-8, maxit=100, singles=True, mixed=False):
    """Iterations of the plain FP64 solve and of the learned-guess FP64 solve (with fallback);
    with mixed=True also the learned-guess solve in mixed precision.  Each solve also reports the
    iterations and seconds (iteration time only, set-up excluded) until its energy is within
    1e-6 Eh of the plain solve's converged energy and stays there."""
    from . import thc
    ctx, Z0 = _context(thc, cfg, singles, tol_energy)
    it_p, _, ok_p = ctx.iterate(tol=tol, maxit=maxit, raise_on_notconv=False)
    e_p = ctx.energy()
    hp, _, tp = ctx.history()
    it_l, ok_l, fallback, hl, tl = _learned_solve(ctx, Z0, net, tol, maxit)
    e_l = ctx.energy()
    ctx.close()
    r = {"o": cfg.o, "nP": cfg.nP, "plain_iterations": it_p, "learned_iterations": it_l, "plain_converged": ok_p,
         "learned_converged": ok_l, "fallback": fallback, "energy_plain": e_p, "energy_learned": e_l,
         "energy_difference": abs(e_l - e_p), "plain_seconds": tp[-1] if tp else None,
         "learned_seconds": tl[-1] if tl else None}
    r["plain_to_1e-6"] = _to_target(hp, tp, e_p)
    r["learned_to_1e-6"] = _to_target(hl, tl, e_p)
    if mixed:
        ctx, Z0 = _context(thc, cfg, singles, tol_energy, precision=1)
        it_m, ok_m, fb_m, hm, tm = _learned_solve(ctx, Z0, net, tol, maxit)
        e_m = ctx.energy()
        ctx.close()
        r.update({"mixed_learned_iterations": it_m, "mixed_learned_converged": ok_m, "mixed_fallback": fb_m,
                  "energy_mixed_learned": e_m, "mixed_energy_difference": abs(e_m - e_p),
                  "mixed_learned_seconds": tm[-1] if tm else None, "mixed_learned_to_1e-6": _to_target(hm, tm, e_p)})
    return r


def save_net(net, path):
    mu_in, sd_in, mu_out, sd_out = net.get_norm()
    np.savez(path, params=net.get_params().cpu().numpy(), mu_in=mu_in, sd_in=sd_in, mu_out=mu_out, sd_out=sd_out,
             shape=np.array([net.n_in, net.width, net.n_out]))


def load_net(path):
    import torch
    from . import thc
    d = np.load(path)
    n_in, width, n_out = (int(x) for x in d["shape"])
    net = thc.MLP(n_in, width, n_out)
    net.set_norm(d["mu_in"], d["sd_in"], d["mu_out"], d["sd_out"])
    net.set_params(torch.from_numpy(np.ascontiguousarray(d["params"], dtype=np.float32)).to("cuda"))
    return net


def _summary(res, args, extra):
    ip = np.array([r["plain_iterations"] for r in res], dtype=float)
    il = np.array([r["learned_iterations"] for r in res], dtype=float)
    out = {"systems_heldout": len(res), "o_range": [args.o_min, args.o_max], "coupling": args.coupling,
           "tol": args.tol, **extra,
           "mean_iterations_plain": float(ip.mean()), "mean_iterations_learned": float(il.mean()),
           "median_iterations_plain": float(np.median(ip)), "median_iterations_learned": float(np.median(il)),
           "mean_reduction": float(1.0 - il.mean() / ip.mean()), "fallbacks": int(sum(r["fallback"] for r in res)),
           "max_energy_difference": float(max(r["energy_difference"] for r in res))}
    for key in ("plain_to_1e-6", "learned_to_1e-6", "mixed_learned_to_1e-6"):
        v = [r[key] for r in res if key in r]
        if v and all(x[0] is not None for x in v):
            out[key + "_mean_iterations"] = float(np.mean([x[0] for x in v]))
            out[key + "_total_seconds"] = float(np.sum([x[1] for x in v]))
    if any("mixed_learned_iterations" in r for r in res):
        im = np.array([r["mixed_learned_iterations"] for r in res], dtype=float)
        out["mean_iterations_mixed_learned"] = float(im.mean())
        out["mixed_fallbacks"] = int(sum(r["mixed_fallback"] for r in res))
        out["max_mixed_energy_difference"] = float(max(r["mixed_energy_difference"] for r in res))
    return out


def main():
    ap = argparse.ArgumentParser(description="Learned-guess experiment. Without --gen/--eval: generate, train "
                                 "and evaluate in one run. --gen A B --save rows.npz: training rows of systems "
                                 "A..B-1 only. --rows f1.npz,... --save-net net.npz: train on saved rows. "
                                 "--net net.npz --eval A B: evaluate held-out systems A..B-1.")
    ap.add_argument("--train", type=int, default=200)
    ap.add_argument("--heldout", type=int, default=56)
    ap.add_argument("--o-min", type=int, default=30)
    ap.add_argument("--o-max", type=int, default=80)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--coupling", type=float, default=0.2)
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--mixed", action="store_true", help="also solve each held-out system in mixed precision "
                    "from the learned start")
    ap.add_argument("--gen", type=int, nargs=2, default=None)
    ap.add_argument("--rows", default=None)
    ap.add_argument("--net", default=None)
    ap.add_argument("--save-net", default=None)
    ap.add_argument("--eval", type=int, nargs=2, default=None)
    ap.add_argument("--save", default=None)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    global COUPLING
    COUPLING = args.coupling
    log = lambda *a: print(*a, flush=True)
    t0 = time.perf_counter()
    if args.gen:  # saved after every system, so a run cut short keeps what it made
        Xs, Ts, infos = [], [], []
        for sidx in range(*args.gen):
            X, T, info = generate([sidx], args.o_min, args.o_max, tol=args.tol, log=log)
            Xs.append(X), Ts.append(T), infos.extend(info)
            np.savez(args.save, X=np.concatenate(Xs), T=np.concatenate(Ts), info=json.dumps(infos))
        log(f"{sum(x.shape[0] for x in Xs)} rows from systems {args.gen[0]}..{args.gen[1] - 1} "
            f"in {time.perf_counter() - t0:.0f} s")
        return
    extra = {}
    if args.net:
        net = load_net(args.net)
    else:
        if args.rows:
            parts = [np.load(f) for f in args.rows.split(",")]
            X = np.concatenate([d["X"] for d in parts])
            T = np.concatenate([d["T"] for d in parts])
            info = sum((json.loads(str(d["info"])) for d in parts), [])
        else:
            log(f"generating training data from {args.train} systems (o in [{args.o_min}, {args.o_max}])")
            X, T, info = generate(range(args.train), args.o_min, args.o_max, tol=args.tol, log=log)
        log(f"{X.shape[0]} rows from {len(info)} systems; training")
        net, first, losses = train(X, T, epochs=args.epochs, log=log)
        extra = {"systems_train": len(info), "rows": int(X.shape[0]), "loss_initial": first,
                 "loss_final": losses[-1]}
        if args.save_net:
            save_net(net, args.save_net)
    heldout = range(*args.eval) if args.eval else range(200, 200 + args.heldout)
    log(f"evaluating on held-out systems {heldout.start}..{heldout.stop - 1}")
    res = []
    for s in heldout:
        r = solve_pair(net, system_config(s, args.o_min, args.o_max), tol=args.tol, mixed=args.mixed)
        r["system"] = s
        res.append(r)
        log(f"  system {s}: o={r['o']} plain {r['plain_iterations']} learned {r['learned_iterations']}"
            f"{' (fallback)' if r['fallback'] else ''} |dE| {r['energy_difference']:.1e}; to 1e-6 Eh: plain "
            f"{r['plain_to_1e-6']} learned {r['learned_to_1e-6']}"
            + (f" mixed+learned {r['mixed_learned_to_1e-6']} ({r['mixed_learned_iterations']} it)" if args.mixed
               else ""))
        if args.out:  # after every system, so a run cut short keeps what it measured
            with open(args.out, "w") as fh:
                json.dump({**_summary(res, args, extra), "seconds": time.perf_counter() - t0, "heldout": res}, fh,
                          indent=1)
    report = {**_summary(res, args, extra), "seconds": time.perf_counter() - t0, "heldout": res}
    log(json.dumps({k: v for k, v in report.items() if k != "heldout"}))
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(report, fh, indent=1)


if __name__ == "__main__":
    main()
