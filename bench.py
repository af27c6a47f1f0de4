#!/usr/bin/env python
"""Benchmark of the THC-CCSD hot path on one MI355X.

A step is one iteration of the solver: the full projected doubles + singles residual of the
current amplitudes (paper Alg. 1-10), the correlation energy, the Jacobi update in the working
basis and DIIS.  The workload is the FP64 configuration o=50, v=450, N_L=1500, N_P=1000,
N_Q=2500 with seeded synthetic inputs (all resident in HBM before the timed region).

Prints one JSON line: FP64 residual evaluations per second (the value), the roofline of the
dominant kernel (the VALU H-kernel of Alg. 6, timed with HIP events on the library's stream
during the timed steps), the MFMA rates of the GEMMs and of the fused exchange kernel, the
fraction of the ideal residual time, the time to converge to 1e-6 Eh of the final energy, the
same for the mixed-precision path (its energy against the FP64 solve), and the FP64 CPU oracle
timed on a bounded sample on the host cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VALU_TFLOPS = 78.6   # MI355X FP64 vector peak (256 CUs, 2.4 GHz)
PEAK_FP32_MFMA_TFLOPS = 157.3  # MI355X dense FP32 matrix peak
PEAK_FP32_VALU_TFLOPS = 157.3  # MI355X FP32 vector peak (counts packed FP32 FMAs)
PEAK_BF16_MFMA_TFLOPS = 2500.0  # MI355X dense BF16 matrix peak
PEAK_HBM_GBS = 8000.0


def _kernel_hash():
    """Hash of the H-kernel source code with comments and blank lines removed."""
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2111_11473_amd", "csrc", "kernels_h.hip")) as fh:
        for line in fh:
            code = line.split("//")[0].strip()
            if code:
                h.update(code.encode())
    return h.hexdigest()[:16]


def _traffic(config_name, launches_per_residual):
    """HBM bytes per H-kernel launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source with the same launches per residual (grid points per
    launch); else None."""
    p = os.path.join(ROOT, "profiles", f"h_kernel_{config_name}_traffic.json")
    try:
        with open(p) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_sha256_16") != _kernel_hash() or d.get("launches_per_residual") != launches_per_residual:
        return None
    return d.get("bytes_per_launch")


def _dense_oracle_cost(c):
    """Leading operation count of the dense oracle residual (integral build + contractions)."""
    o, v, nL = c.o, c.v, c.nL
    return nL * v ** 4 + o * o * v ** 4 + 6 * o ** 3 * v ** 3 + nL * (o + v) ** 2 * o * v


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(target_cfg, sample_name="wide", budget_s=20.0):
    """The FP64 oracle as it is, timed on the host cores: dense residual evaluations of the
    largest parity system it holds comfortably (it materializes (ac|bd), v^4 values, so the
    benchmark workload itself, 328 GB at v = 450, is out of its reach), repeated for about
    budget_s.  The measured rate is the value; the rate scaled to the benchmark workload by the
    oracle's dense cost is reported separately and labelled an estimate."""
    import numpy as np
    import oracle
    from paper_2111_11473_amd import synth
    try:
        from threadpoolctl import threadpool_info
        blas = [{k: i.get(k) for k in ("internal_api", "num_threads", "version")} for i in threadpool_info()]
    except Exception:
        blas = []
    sc = synth.CONFIGS[sample_name]
    s = synth.make_system(sc)
    z, _ = oracle.eri_fit(s["L"], sc.o, s["xo"], s["xv"])
    V = oracle.eri_thc_dense(s["xo"], s["xv"], z)
    Z0 = oracle.mp2_guess(s["eps"], s["L"], s["Xo"], s["Xv"])
    t1 = np.zeros((sc.o, sc.v))
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.thc_residual(s["eps"], s["L"], s["Xo"], s["Xv"], Z0, t1, V)
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    rate = n / dt
    scale = _dense_oracle_cost(sc) / _dense_oracle_cost(target_cfg)
    return {
        "value": rate,
        "unit": "residual_evals/s",
        "cores": len(os.sched_getaffinity(0)),
        "kind": "oracle",
        "sample": (f"dense FP64 oracle residual (numpy/scipy, as written) of the '{sc.name}' system o={sc.o} "
                   f"v={sc.v} nL={sc.nL} nP={sc.nP} nQ={sc.nQ}: {n} evaluations in {dt:.1f} s; the benchmark "
                   f"workload itself does not fit the oracle (its (ac|bd) block alone is "
                   f"{8 * target_cfg.v ** 4 / 1e9:.0f} GB)"),
        "sample_config": {"o": sc.o, "v": sc.v, "nL": sc.nL, "nP": sc.nP, "nQ": sc.nQ},
        "cpu_model": _cpu_model(),
        "blas": blas,
        "estimate_at_workload": {"value": rate * scale, "unit": "residual_evals/s", "kind": "estimate",
                                 "how": "measured rate x dense-cost ratio (nL v^4 + o^2 v^4 + 6 o^3 v^3 + "
                                        f"nL n^2 o v) = {scale:.3e}"},
    }


def gpu_rate_on(sample_name, n_eval=10):
    """GPU residual evaluations per second (FP64) on the same sample system as the CPU oracle."""
    import numpy as np
    import torch
    from paper_2111_11473_amd import synth, thc
    cfg = synth.CONFIGS[sample_name]
    s = synth.make_system(cfg)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    ctx = thc.THC(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ, singles=True)
    Z0 = ctx.build_factors(dev(s["L"]), dev(s["eps"]), *(dev(s[k]) for k in ("Xo", "Xv", "xo", "xv")))
    t1 = torch.zeros((cfg.o, cfg.v), dtype=torch.float64, device="cuda")
    ctx.residual(Z0, t1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_eval):
        ctx.residual(Z0, t1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    return n_eval / dt


LEG_PRECISION = {"fp64": 0, "mixed": 1, "mixed_split_bf16": 2}


def counter_summary(csv_dir, top=14):
    """Per-kernel table from a rocprofv3 --pmc run of this script (--output-format csv) with the
    counters SQ_VALU_MFMA_BUSY_CYCLES, SQ_INSTS_VALU_MFMA_MOPS_F64/F32, SQ_INSTS_VALU_FLOPS_FP64,
    SQ_INSTS_VALU, SQ_INSTS_LDS, SQ_LDS_BANK_CONFLICT and GRBM_GUI_ACTIVE: fractions of the
    kernel's active cycles (clock independent) and the work counted by the hardware."""
    import collections
    import csv
    import glob
    import re
    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    for f in glob.glob(os.path.join(csv_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                m = re.search(r"(\w+_kernel)(<[^>]*>)?", row["Kernel_Name"])
                k = (m.group(1) + (m.group(2) or "")) if m else row["Kernel_Name"][:40]
                agg[k][row["Counter_Name"]] += float(row["Counter_Value"])
                disp[k].add(row.get("Dispatch_Id", ""))
    simds, xcc = 1024, 8  # MI355X: 256 CUs x 4 SIMDs; GRBM_GUI_ACTIVE is reported per XCD
    rows = sorted(agg.items(), key=lambda kv: -kv[1]["GRBM_GUI_ACTIVE"])
    total = sum(v["GRBM_GUI_ACTIVE"] for _, v in rows)
    lines = ["| kernel | dispatches | share of active cycles | MFMA busy | MFMA flops (MOPS x 512) | "
             "FP64 VALU flops issued | VALU issue busy | LDS bank-conflict cycles per LDS instruction |",
             "|---|---|---|---|---|---|---|---|"]
    for k, v in rows[:top]:
        cyc = v["GRBM_GUI_ACTIVE"] / xcc
        mf = 512.0 * (v.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) + v.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0))
        lds = v.get("SQ_INSTS_LDS", 0.0)
        lines.append(f"| {k} | {len(disp[k])} | {100 * v['GRBM_GUI_ACTIVE'] / total:.1f}% | "
                     f"{v.get('SQ_VALU_MFMA_BUSY_CYCLES', 0.0) / (simds * cyc):.2f} | {mf:.3e} | "
                     f"{64 * v.get('SQ_INSTS_VALU_FLOPS_FP64', 0.0):.3e} | "
                     f"{4 * v.get('SQ_INSTS_VALU', 0.0) / (simds * cyc):.2f} | "
                     f"{(v.get('SQ_LDS_BANK_CONFLICT', 0.0) / lds) if lds else 0.0:.2f} |")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="fp64")
    ap.add_argument("--legs", default=None,
                    help="comma list of fp64, mixed, mixed_split_bf16 (default: all three on the fp64 workload, "
                         "mixed alone on the larger ones); the first is the headline")
    ap.add_argument("--energy-iters", type=int, default=0,
                    help="instead of a converge run, the energies of this many iterations from the MP2 guess")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-converge", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision legs")
    ap.add_argument("--no-next", action="store_true", help="skip the Alg. 4/5 and MP2-density timings")
    ap.add_argument("--converge-maxit", type=int, default=40)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device-to-device copy first (a known-traffic kernel for counter scaling)")
    ap.add_argument("--counter-summary", metavar="DIR",
                    help="print the per-kernel table of a rocprofv3 --pmc CSV output directory and exit")
    args = ap.parse_args()
    if args.counter_summary:
        print(counter_summary(args.counter_summary))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        sys.exit("bench.py: the THC-CCSD hot path runs on one GPU; multi-GPU runs are not "
                 "implemented (use --gpus 1)")

    import torch
    from paper_2111_11473_amd import synth, thc

    cfg = synth.CONFIGS[args.config]
    large = cfg.name != "fp64"
    legs = args.legs.split(",") if args.legs else (["mixed"] if large else ["fp64", "mixed", "mixed_split_bf16"])
    if args.no_mixed:
        legs = [g for g in legs if g == "fp64"]
    if not legs or any(g not in LEG_PRECISION for g in legs):
        sys.exit(f"bench.py: --legs must name some of {list(LEG_PRECISION)}")
    cpu = None
    if not args.no_cpu_baseline and not large:
        cpu = cpu_baseline(cfg)
        print(f"bench: cpu baseline done ({cpu['value']:.3f} residual evals/s on '{cpu['sample_config']}')",
              file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    if args.copy_calibration:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if cpu is not None:
        g = gpu_rate_on("wide")
        cpu["gpu_same_sample"] = {"value": g, "unit": "residual_evals/s", "gpu_over_cpu": g / cpu["value"]}
    P, Q, o = cfg.nP, cfg.nQ, cfg.o
    flags = thc.FLAG_PROGRESS if large else 0

    def leg(precision):
        """Timed solver steps (one residual + update each) and the converge (or energy) run of one
        precision, on inputs generated on the device by the library (bit-identical to the Python
        generator's)."""
        ctx = thc.THC(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ, singles=True, diis_max=8, tol_energy=1e-8,
                      precision=precision, flags=flags)
        ctx.set_synthetic(cfg.seed, cfg.decay, cfg.coupling)
        tb = time.perf_counter()
        Z0 = ctx.build_synthetic()
        torch.cuda.synchronize()
        build_s = time.perf_counter() - tb
        print(f"bench: leg precision {precision} built in {build_s:.1f} s", file=sys.stderr, flush=True)
        for _ in range(args.warmup):
            ctx.iterate(tol=0.0, maxit=1, raise_on_notconv=False)
        torch.cuda.synchronize()
        ctx.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step_e, step_t, step_r = [], [], []  # per timed step: energy evaluated, wall time, residual norm
        for _ in range(args.steps):
            ctx.iterate(tol=0.0, maxit=1, raise_on_notconv=False)
            if large:
                E_, R_, _ = ctx.history()
                step_e.append(E_[-1])
                step_r.append(R_[-1])
                step_t.append(time.perf_counter() - t0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(f"bench: leg precision {precision}: {args.steps} timed steps in {dt:.1f} s", file=sys.stderr, flush=True)
        prof = {name: ctx.profile_get(name) for name in ("h_kernel", "residual", "gemm", "misc", "exch")}
        flops64, flops32, flops16 = ctx.profile_flops()
        ctx.profile(False)
        conv = None
        if args.energy_iters > 0:
            ctx.set_state(Z0)
            tc = time.perf_counter()
            it, rn, ok = ctx.iterate(tol=0.0, maxit=args.energy_iters, raise_on_notconv=False)
            E, R, T = ctx.history()
            conv = {"iterations": it, "energies": E, "rnorms": R, "seconds": T,
                    "wall_s": time.perf_counter() - tc, "mixed_iterations": sum(ctx.history_precision()),
                    "guess": "MP2 least-squares fit", "solver": "Jacobi (pseudo-canonical) + DIIS(8)"}
        elif not args.no_converge and large and args.warmup == 0:
            # the timed steps were the solve's first iterations (from the MP2 guess, warmup 0):
            # continue from there (DIIS history kept) instead of evaluating them again
            tc = time.perf_counter()
            it, rn, ok = ctx.iterate(tol=1e-7, maxit=max(1, args.converge_maxit - args.steps), raise_on_notconv=False)
            wall = time.perf_counter() - tc
            E, R, T = ctx.history()
            E, T, it = step_e + E, step_t + [dt + t for t in T], args.steps + it
            Ef = E[-1]
            conv = {"converged": bool(ok), "iterations": it, "final_energy": Ef, "final_rnorm": rn,
                    "solve_seconds": dt + wall, "energies": E, "seconds": T, "rnorms": step_r + R,
                    "mixed_iterations": sum(ctx.history_precision()) + (args.steps if precision else 0),
                    "guess": "MP2 least-squares fit", "solver": "Jacobi (pseudo-canonical) + DIIS(8)",
                    "note": "the timed steps are the first iterations of this solve"}
        elif not args.no_converge:
            ctx.set_state(Z0)
            tc = time.perf_counter()
            it, rn, ok = ctx.iterate(tol=1e-7, maxit=args.converge_maxit, raise_on_notconv=False)
            wall = time.perf_counter() - tc
            E, R, T = ctx.history()
            Ef = E[-1]
            conv = {"converged": bool(ok), "iterations": it, "final_energy": Ef, "final_rnorm": rn,
                    "solve_seconds": wall, "energies": E, "seconds": T,
                    "mixed_iterations": sum(ctx.history_precision()),
                    "guess": "MP2 least-squares fit", "solver": "Jacobi (pseudo-canonical) + DIIS(8)"}
        plan = ctx.plan()
        plan["build_seconds"] = build_s
        if step_e:
            plan["step_energies"] = step_e
        plan["gamma"] = ctx.synth_gamma()
        ctx.close()
        torch.cuda.synchronize()
        return dt, prof, flops64 / args.steps, (flops32 + flops16) / args.steps, conv, plan

    def to_target(conv, e_ref):
        """Iterations and seconds until the energy stays within 1e-6 Eh of e_ref."""
        if conv is None or "final_energy" not in conv:
            return conv
        E, T = conv.pop("energies"), conv.pop("seconds")
        k = len(E) - 1
        while k > 0 and abs(E[k - 1] - e_ref) < 1e-6:
            k -= 1
        if abs(E[k] - e_ref) >= 1e-6:
            return conv
        conv["iterations_to_1e-6"] = k + 1
        conv["seconds_to_1e-6"] = T[k]
        return conv

    # algorithmic count of the three-way accumulation H^XYZ += (E^XY F^XZ + E^XZ F^XY) G^YZ as the
    # paper writes it: 5 flops per (X, Y, Z, I) -- two products, a sum, a product and the
    # accumulation.  The kernel issues 3.5 per (X, Y, Z, I): for Y != Z one bracket (3 flops)
    # serves both H^XYZ and H^XZY (one FMA each).
    h_flops_per_residual = 5.0 * Q * P ** 3
    h_flops_issued = 3.5 * Q * P ** 3
    exch_flops = 2 * 4.0 * P * o * Q * Q  # two exchange passes, two products of 2 o Q^2 each per X

    results = {}
    for name in legs:
        results[name] = leg(LEG_PRECISION[name])

    def next_rows():
        """The two further paths on the same workload (FP64): Eq. 32 + 33 by Alg. 4 and 5 (O(N^5),
        matrix products only) against Alg. 6 (the H-kernel path), and the MP2 one-particle density
        of the guess amplitudes (App. II, O(N^4))."""
        res = {}
        for key, flag in (("alg6_eq32_33_ms", thc.FLAG_QUARTIC), ("alg45_eq32_33_ms", thc.FLAG_QUINTIC)):
            ctx = thc.THC(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ, flags=flag | flags)
            ctx.set_synthetic(cfg.seed, cfg.decay, cfg.coupling)
            Z0 = ctx.build_synthetic()
            ctx.residual(Z0, None, mask=thc.TERM_EQ32)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(2):
                ctx.residual(Z0, None, mask=thc.TERM_EQ32)
            torch.cuda.synchronize()
            res[key] = 1e3 * (time.perf_counter() - t0) / 2
            if flag == thc.FLAG_QUARTIC:
                ctx.mp2_density()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(5):
                    ctx.mp2_density()
                torch.cuda.synchronize()
                res["mp2_density_ms"] = 1e3 * (time.perf_counter() - t0) / 5
            ctx.close()
            torch.cuda.synchronize()
        res["cost_model_choice"] = "alg45" if thc.plan_query(cfg.o, cfg.v, cfg.nL, cfg.nP, cfg.nQ, 270e9, synthetic=True)["quintic"] else "alg6"
        print(f"bench: next rows {res}", file=sys.stderr, flush=True)
        return res

    extra = next_rows() if (not large and "fp64" in legs and not args.no_next) else None
    head = legs[0]
    dt, prof, gf64, gfm, conv_head, plan_head = results[head]
    h_ms, h_n = prof["h_kernel"]
    r_ms, r_n = prof["residual"]
    g_ms, _ = prof["gemm"]
    m_ms, _ = prof["misc"]
    x_ms, _ = prof["exch"]
    launches_per_residual = max(1, h_n // max(1, r_n))
    h_peak = PEAK_FP64_VALU_TFLOPS if LEG_PRECISION[head] == 0 else PEAK_FP32_VALU_TFLOPS
    flops_per_launch = h_flops_per_residual / launches_per_residual
    avg_launch_s = (h_ms / 1e3) / max(1, h_n)
    achieved = flops_per_launch / avg_launch_s / 1e12
    achieved_issued = h_flops_issued / launches_per_residual / avg_launch_s / 1e12
    g_per = g_ms / args.steps / 1e3
    x_per = x_ms / args.steps / 1e3
    t_res = r_ms / max(1, r_n) / 1e3
    e_ref = None
    if "fp64" in results and results["fp64"][4] is not None and "final_energy" in results["fp64"][4]:
        e_ref = results["fp64"][4]["final_energy"]

    def ideal_seconds(precision, gf64_, gfm_):
        """Every part at its peak: the H-kernel at the vector peak of its arithmetic type, the
        exchange and contractions at the matrix peak of theirs (a split-BF16 product is six BF16
        products), the products kept in FP64 at the FP64 peak."""
        if precision == 0:
            return (h_flops_per_residual + gf64_ + exch_flops) / (PEAK_FP64_VALU_TFLOPS * 1e12)
        peak = PEAK_FP32_MFMA_TFLOPS if precision == 1 else PEAK_BF16_MFMA_TFLOPS / 6.0
        return (h_flops_per_residual / (PEAK_FP32_VALU_TFLOPS * 1e12) + exch_flops / (PEAK_FP32_MFMA_TFLOPS * 1e12)
                + gfm_ / (peak * 1e12) + gf64_ / (PEAK_FP64_VALU_TFLOPS * 1e12))

    def mixed_summary(name):
        precision = LEG_PRECISION[name]
        dtm, profm, gf64m, gfm_, convm, planm = results[name]
        rm_ms, rm_n = profm["residual"]
        gm_s = profm["gemm"][0] / args.steps / 1e3
        t_res_m = rm_ms / max(1, rm_n) / 1e3
        if convm is not None and e_ref is not None and "final_energy" in convm:
            convm["energy_minus_fp64"] = convm["final_energy"] - e_ref
            convm = to_target(convm, e_ref)
        rate = gfm_ / max(gm_s, 1e-12) / 1e12
        return {"residual_evals_per_s": args.steps / dtm, "ms_per_step": 1e3 * dtm / args.steps,
                "residual_ms": 1e3 * t_res_m, "h_kernel_ms": profm["h_kernel"][0] / args.steps,
                "gemm_ms": profm["gemm"][0] / args.steps, "exchange_ms": profm["exch"][0] / args.steps,
                ("gemm_fp32_mfma" if precision == 1 else "gemm_split_bf16_mfma"):
                    {"achieved": rate if precision == 1 else 6.0 * rate,
                     "peak": PEAK_FP32_MFMA_TFLOPS if precision == 1 else PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "note": "product flops" if precision == 1 else "six BF16 products per split product"},
                "residual_roofline_frac": ideal_seconds(precision, gf64m, gfm_) / t_res_m,
                "precision": ("FP32 MFMA contractions" if precision == 1 else
                              "compensated split-BF16 contractions (three bf16 pieces per operand, six products, "
                              "FP32 accumulation)") +
                             " and the H accumulation in FP32 per grid-point chunk, FP64 energy, denominators, fit, DIIS; "
                             "FP64 finishing iterations",
                "plan": planm, "converge": convm}

    head_prec = LEG_PRECISION[head]
    conv64 = results["fp64"][4] if "fp64" in results else None
    if conv64 is not None and "final_energy" in conv64:
        conv64 = to_target(conv64, conv64["final_energy"])
    out = {
        "metric": "residual_evals_per_s",
        "value": args.steps / dt,
        "unit": "residual_evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head_prec == 0 else ("f32+f64" if head_prec == 1 else "bf16x6+f32+f64"),
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: THC-CCSD residual + energy + Jacobi/DIIS step, o={cfg.o} v={cfg.v} "
                               f"nL={cfg.nL} nP={cfg.nP} nQ={cfg.nQ}, seeded synthetic inputs generated on the device",
                   "o": cfg.o, "v": cfg.v, "nL": cfg.nL, "nP": cfg.nP, "nQ": cfg.nQ, "precision": head,
                   "parallelism": "single GPU"},
        "roofline": {"kernel": "h_kernel (three-way accumulation of Alg. 6, Y<->Z symmetric, "
                               + ("FP64 VALU arithmetic" if head_prec == 0 else
                                  "FP32 VALU arithmetic and operands, FP64 H across grid-point chunks") + ")",
                     "bound": "alu",
                     "achieved": achieved, "peak": h_peak, "unit": "TFLOP/s",
                     "frac": achieved / h_peak,
                     "traffic": _traffic(cfg.name, launches_per_residual) if head_prec == 0 else None,
                     "launches": h_n,
                     "avg_launch_ms": 1e3 * avg_launch_s, "algorithmic_flops_per_launch": flops_per_launch,
                     "flop_count": "5 N_Q N_P^3 per residual (the accumulation as written)",
                     "issued": {"achieved": achieved_issued, "frac": achieved_issued / h_peak,
                                "flop_count": "3.5 N_Q N_P^3 (one bracket for both H^XYZ and H^XZY)"},
                     **({} if head_prec == 0 else {
                         "without_packed_fp32": {"peak": PEAK_FP64_VALU_TFLOPS, "frac": achieved / PEAK_FP64_VALU_TFLOPS,
                                                 "note": "the FP32 issue rate with packed FP32 instructions "
                                                         "disabled (one FMA per lane per instruction)"}})},
        "mfma": {("gemm_fp64" if head_prec == 0 else "gemm_reduced"):
                     {"achieved": (gf64 if head_prec == 0 else gfm) / max(g_per, 1e-12) / 1e12,
                      "peak": PEAK_FP64_VALU_TFLOPS if head_prec == 0 else PEAK_FP32_MFMA_TFLOPS,
                      "unit": "TFLOP/s", "flops_per_residual": gf64 if head_prec == 0 else gfm},
                 "exchange": {"achieved": exch_flops / max(x_per, 1e-12) / 1e12,
                              "peak": PEAK_FP64_VALU_TFLOPS if head_prec == 0 else PEAK_FP32_MFMA_TFLOPS,
                              "unit": "TFLOP/s", "flops_per_residual": exch_flops}},
        "residual_roofline_frac": ideal_seconds(head_prec, gf64, gfm) / t_res,
        "breakdown_ms_per_step": {"residual": 1e3 * t_res, "h_kernel": h_ms / args.steps, "gemm": g_ms / args.steps,
                                  "exchange": x_ms / args.steps, "misc": m_ms / args.steps},
        "plan": plan_head,
        "converge": conv64 if head == "fp64" else results[head][4],
        "cpu_baseline": cpu,
        "next_rows": extra,
    }
    for name in legs:
        if name != "fp64":
            out[name] = mixed_summary(name)
    if "fp64" in legs and head != "fp64":
        out["fp64"] = {"residual_evals_per_s": args.steps / results["fp64"][0], "converge": conv64,
                       "plan": results["fp64"][5]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
