"""Benchmark: smoothed-kernel pair interactions/s of a full mixed-precision ddm_solve.

One step = one coupled Stokes-Darcy solve (Dirichlet-Neumann interface
equation by GMRES) of the porous unit sphere at h = 1/64 (N = 68166
quadrature nodes, delta = 3h) in the stream U = e_z, mu = 1, K = 1e-2,
alpha = 1, with the library's default solver settings: local GMRES tolerance
1e-10, interface tolerance 1e-8, float-pair kernel sums with double
accumulation inside relaxed local GMRES (double-pair products until the
residual reaches 1e-4, double-pair true residuals), and inexact interface
products (local solves loosened as the interface residual falls, full-accuracy
final solves).  Every layer-sum pass evaluates N^2 (target, source) pairs;
`value` is the total pair count of the timed steps divided by their wall time
(inputs resident on the GPU).

Also reported: the all-FP64 GPU path with the same settings and with strict
interface products (every local solve to 1e-10), each the median of 3 solves
and the faster of with and without the recycled deflation space, their drag,
the drag of each against the closed-form solution, the staging time of the
surface (once per surface, outside the solve), the roofline of the dominant
kernel (HIP-event durations recorded by the library around every pair-sum
kernel during the timed region), and the CPU oracle on a bounded sample of
target rows of the same surface: its pair rate, and the residual of the mixed
solve's (p, u) in both coupled equations that its pair sums give (the error
of the GPU solution against the FP64 oracle).

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--workload sphere-h64|perturbed-h128]
    python bench.py --passes          (per-pass kernel times only)

The second workload is the large surface (N = 351866); one solve takes minutes,
so run it with --steps 1 --warmup 0 --no-fp64 (SDBIE_DEBUG=1 prints the
interface steps as they complete).  --passes times every single layer pass of
the workload's surface, float and double pairs, one-direction and symmetric.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published vector peaks.  FP32: 256 CU x 128 lanes x 2 flop x 2.4 GHz = 157.3
# TFLOP/s, reached without packed instructions (the library is compiled without them):
# an FP32 VALU instruction whose operands are all VGPRs issues every 2 cycles
# per wave64 (probe: 2.05-2.5), one that reads an SGPR every 4 cycles.
# FP64: 78.6 TFLOP/s (probe: 4.3 cycles per wave64 FMA).
PEAK_FP32 = 157.3
PEAK_FP64 = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")

# Algorithmic flops per (target, source) pair of the layer kernels (FMA 2, add or
# multiply 1, the rsqrt 1; far-field form, smoothing not counted): Laplace single
# layer 10, Laplace double layer 20, Stokeslet 28, stresslet 33.  A pass that
# evaluates a double and a single layer of one family counts the sum of the two
# (the Stokes matvec with slip: stresslet of u plus Stokeslet of beta P_tau u,
# 61), whatever the pass shares between them; the library's own count of the
# fused form as evaluated is reported beside it.
KERNEL_FLOPS = {("laplace", False, True): 10, ("laplace", True, False): 20, ("laplace", True, True): 30,
                ("stokes", False, True): 28, ("stokes", True, False): 33, ("stokes", True, True): 61}


def kernel_flops(name: str):
    """Flops per pair of a pass kernel's timing name (None for other kernels)."""
    fam = name.split("_", 1)[0]
    if "<" not in name or ("pass<" not in name and "sympass<" not in name) or "_T_" in name:
        return None
    flags = name[name.index("<") + 1:-1].split(",")
    return KERNEL_FLOPS.get((fam, "DL" in flags, "SL" in flags))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(S, delta, prm, U, p, u, budget_s: float = 15.0):
    """Oracle (plain FP64 C loops, OpenMP over targets) on sampled target rows.

    The sample is the residual of the GPU's solution (p, u) in both coupled
    equations, evaluated by the oracle: the Laplace subtracted double layer
    of p and single layer of u.n, the Stokes subtracted double layer of u and
    single layers of -p n and of the slip traction, each on M target rows
    against all N sources; M is sized for ~budget_s of CPU time.
    Pairs/s = 5 M N / time (4 without slip).
    The same evaluation is the stated error of the GPU solve against the
    FP64 oracle: the relative root-mean-square residuals on the M rows
    (Darcy rows up to the constant that the completion fixes).
    """
    import numpy as np

    from oracle import oracle as O

    geo = O.Geometry(S.x, S.n, S.w, delta)
    oprm = O.Params(*prm)

    def run(M):
        t = np.unique(np.linspace(0, S.N - 1, M).astype(np.int64))
        t0 = time.perf_counter()
        res = O.coupled_residual(geo, oprm, U, p, u, t)
        return time.perf_counter() - t0, t, res

    # size the sample from probes until it takes at least half the budget
    M = 64
    dt, t, res = run(M)
    for _ in range(4):
        if dt >= 0.5 * budget_s or M >= S.N:
            break
        M = int(max(M + 1, min(S.N, M * budget_s / max(dt, 1e-6))))
        dt, t, res = run(M)
    r1, b1, r2, b2 = res
    rms = lambda a: float(np.sqrt(np.mean(np.asarray(a) ** 2)))
    resid = {"darcy": rms(r1 - r1.mean()) / rms(b1), "stokes": rms(r2) / rms(b2),
             "rows": int(len(t)),
             "definition": "RMS over the sampled rows of A_D p - (mu/K) S_L[u.n] (minus its mean) relative to that "
                           "of (mu/K) S_L[u.n], and of A_S u + (w.n.u/|S|) n + V[beta P_tau u] - (U - V[-p n]) "
                           "relative to that of U - V[-p n]; FP64 oracle pair loops"}
    napply = 5 if oprm.beta != 0.0 else 4
    base = {"value": napply * len(t) * S.N / dt, "unit": "pair-interactions/s", "cores": O.num_threads(),
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": f"residual of the GPU solution in both coupled equations: {napply} layer applies (Laplace "
                      f"DL-subtracted, Laplace SL, Stokes DL-subtracted, Stokes SL of -p n and of the slip traction) "
                      f"on {len(t)} of {S.N} target "
                      f"rows x all {S.N} sources, FP64, {dt:.1f} s"}
    return base, resid


def kernel_source_digest() -> str:
    """Digest of the pair-kernel sources (traffic counters are only valid for them)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("pair_kernels.hip", "smoothing_coeffs.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_2110_10749_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_name: str, n: int):
    """HBM bytes per launch of the dominant pass from rocprofv3 --pmc FETCH_SIZE /
    WRITE_SIZE runs (profiles/traffic.json), scaled by the same counters on a plain
    copy of known size; null when absent or when the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_digest") != kernel_source_digest() or t.get("N") != n:
        return None
    ent = t.get("kernels", {}).get(kernel_name)
    return None if ent is None else ent.get("bytes_per_launch")


def time_passes(sd, plan, S, dev) -> int:
    """Per-pass kernel times (HIP events of the library) of every layer kind,
    precision and symmetric-family setting, one JSON line each."""
    import torch
    from workloads import fields
    q = dev(fields.random_scalar(S.N, 1))
    u = dev(fields.random_vector(S.N, 2))
    for prec in ("mixed", "fp64"):
        for mask in (0, sd.SYM_ALL):
            plan.set_symmetric(mask)
            for fam, layer in (("laplace", "sl"), ("laplace", "dl_sub"), ("stokes", "sl"), ("stokes", "dl_sub")):
                if fam == "laplace":
                    f = lambda: sd.laplace_layer_apply(plan, layer, q, prec=prec)
                else:
                    f = lambda: sd.stokes_layer_apply(plan, 1.0, layer, u, prec=prec)
                f()
                torch.cuda.synchronize()
                sd.profile_enable(True)
                for _ in range(5):
                    f()
                torch.cuda.synchronize()
                st = sd.profile_read()
                sd.profile_enable(False)
                k = max((x for x in st if x["pairs"] > 0), key=lambda x: x["ms"])
                print(json.dumps({"pass": f"{fam} {layer}", "prec": prec, "symmetric": bool(mask),
                                  "kernel": k["name"], "ms_per_launch": k["ms"] / k["launches"]}), flush=True)
    plan.set_symmetric(sd.SYM_DEFAULT)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["sphere-h64", "perturbed-h128"], default="sphere-h64",
                    help="sphere-h64: the porous unit sphere at h=1/64 (N=68166), K=1e-2, U=e_z (closed-form "
                         "drag); perturbed-h128: a sphere perturbed by degree<=8 harmonics (seeded, sigma 0.05) "
                         "at h=1/128 (N=351866), K=1e-3, U seeded on the unit sphere")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--passes", action="store_true",
                    help="only time the single layer passes of the workload's surface (Laplace and Stokes single "
                         "and subtracted double layers of seeded densities, float and double pairs, one-direction "
                         "and target-source symmetric far field), 5 launches each, and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (calibrates the HBM "
                         "byte counters of a profiler) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the multi-GPU sharding is a design only).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": 8 * n, "launches": 3}), flush=True)
        return 0

    import paper_2110_10749_amd as sd
    from workloads import exact, surfaces

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        return 1
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")

    from workloads import fields
    mu, alpha = 1.0, 1.0
    if args.workload == "sphere-h64":
        h, K = 1.0 / 64, 1e-2
        E = [0.0, 0.0, 1.0]
        S = surfaces.sphere(h)
        D_exact = exact.bjs_drag(K=K, beta=alpha * mu / math.sqrt(K))
        wl = (f"porous unit sphere, h=1/64 (N={S.N}), delta=3h, U=e_z, mu=1, K=1e-2, alpha=1")
    else:
        h, K = 1.0 / 128, 1e-3
        E = [float(v) for v in fields.unit_vector(53)]
        S = surfaces.perturbed_sphere(h, lmax=8, sigma=0.05, seed=0)
        D_exact = None
        wl = (f"sphere perturbed by degree<=8 real harmonics (N(0,0.05^2) coefficients, seed 0), h=1/128 "
              f"(N={S.N}), delta=3h, U={np.round(E, 4).tolist()}, mu=1, K=1e-3, alpha=1")
    delta = 3 * h
    xd, nd, wd = dev(S.x), dev(S.n), dev(S.w)
    # step a1 (staging: Morton sort, padded copies, tile boxes, near masks) runs
    # once per surface, outside the solve; timed here on its own (median of 3)
    stage_ms = []
    for _ in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = sd.Plan(xd, nd, wd, delta)
        torch.cuda.synchronize()
        stage_ms.append(1e3 * (time.perf_counter() - t0))
        plan.close()
    plan = sd.Plan(xd, nd, wd, delta)
    if args.passes:
        return time_passes(sd, plan, S, dev)
    opts_mixed = dict(prec="mixed", outer="gmres", tol_gmres=1e-10, tol_ddm=1e-8)
    opts_fp64 = dict(prec="fp64", outer="gmres", tol_gmres=1e-10, tol_ddm=1e-8)
    flow = lambda D: float(np.dot(D, E))

    for _ in range(args.warmup):
        sd.ddm_solve(plan, mu, K, alpha, E, None, opts=opts_mixed)
    torch.cuda.synchronize()

    sd.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pairs = 0.0
    infos = []
    for k in range(args.steps):
        p, u, D, info = sd.ddm_solve(plan, mu, K, alpha, E, None, opts=opts_mixed)
        pairs += info["pairs"]
        infos.append(info)
        log(f"step {k}: drag {flow(D):.12f} info {info}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = sd.profile_read()
    sd.profile_enable(False)
    wall = t1 - t0
    D_mixed = flow(D)

    # dominant kernel over the timed region
    dom = max(stats, key=lambda s: s["ms"])
    avg_ms = dom["ms"] / dom["launches"]
    pairs_per_launch = dom["pairs"] / dom["launches"]
    fpp = kernel_flops(dom["name"]) or dom["flops_per_pair"]
    achieved = fpp * pairs_per_launch / (avg_ms * 1e-3) / 1e12
    achieved_eval = dom["flops_per_pair"] * pairs_per_launch / (avg_ms * 1e-3) / 1e12
    is32 = "f32" in dom["name"]
    peak = PEAK_FP32 if is32 else PEAK_FP64
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": measured_traffic(dom["name"], S.N),
                "kernel": dom["name"], "avg_ms": avg_ms, "launches_per_step": dom["launches"] / args.steps,
                "flops_per_pair": fpp, "pairs_per_launch": pairs_per_launch,
                "flops_convention": "algorithmic work per pair of the layer kernels (Laplace SL 10, DL 20; "
                                    "Stokeslet 28, stresslet 33; a fused double+single layer pass counts both)",
                "flops_per_pair_as_evaluated": dom["flops_per_pair"],
                "achieved_as_evaluated": achieved_eval, "frac_as_evaluated": achieved_eval / peak,
                "peak_basis": ("published fp32 vector peak (VGPR-operand VALU at 2 cycles per wave64 "
                               "instruction, no packed instructions)" if is32 else "published fp64 vector peak")}
    kernel_ms_total = sum(s["ms"] for s in stats)

    result = {
        "metric": "smoothed-kernel pair interactions/s (mixed-precision ddm_solve)",
        "value": pairs / wall,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-pairs+f64",
        "data": "synthetic",
        "config": {"workload": wl + "; ddm_solve with interface GMRES (tol 1e-8, inexact products), local "
                               "GMRES tol 1e-10 (float pairs below residual 1e-4; final solves end on double-pair residuals)",
                   "N": S.N, "pairs_per_step": pairs / args.steps},
        "roofline": roofline,
        "kernels": stats,
        "kernel_time_frac": kernel_ms_total * 1e-3 / wall,
        "drag_mixed": D_mixed,
        "drag_exact": D_exact,
        "drag_rel_err_mixed": None if D_exact is None else abs(D_mixed - D_exact) / D_exact,
        "mixed_info": infos[-1],
        "stage_ms": float(np.median(stage_ms[1:])),
    }

    if not args.no_fp64:
        # the FP64 baselines at their best: with and without the recycled
        # deflation space, each the median of 3 timed solves after a warm-up,
        # the faster of the two
        def best_fp64(extra):
            best = None
            for rc in (1, 0):
                o = dict(opts_fp64, recycle=rc, **extra)
                sd.ddm_solve(plan, mu, K, alpha, E, None, opts=o)
                torch.cuda.synchronize()
                times = []
                for _ in range(3):
                    t0 = time.perf_counter()
                    out = sd.ddm_solve(plan, mu, K, alpha, E, None, opts=o)
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t0)
                t = float(np.median(times))
                if best is None or t < best[0]:
                    best = (t, out, rc, times)
            return best
        t64, (p64, u64, D64, info64), rc64, times64 = best_fp64({})
        t64s, (_, _, D64s, info64s), rc64s, times64s = best_fp64({"relax_outer": 0})
        result.update({
            "fp64_recycle": rc64,
            "fp64_strict_recycle": rc64s,
            "fp64_strict_ms_per_solve": 1e3 * t64s,
            "fp64_strict_ms_samples": [1e3 * v for v in times64s],
            "speedup_mixed_vs_fp64_strict": t64s / (wall / args.steps),
            "drag_fp64_strict": flow(D64s),
            "fp64_strict_info": info64s,
        })
        result.update({
            "fp64_ms_per_solve": 1e3 * t64,
            "fp64_ms_samples": [1e3 * v for v in times64],
            "fp64_pairs_per_s": info64["pairs"] / t64,
            "speedup_mixed_vs_fp64": t64 / (wall / args.steps),
            "drag_fp64": flow(D64),
            "drag_rel_err_fp64": None if D_exact is None else abs(flow(D64) - D_exact) / D_exact,
            "drag_rel_diff_mixed_vs_fp64": abs(D_mixed - flow(D64)) / abs(flow(D64)),
            "u_max_rel_diff_mixed_vs_fp64": float((u - u64).abs().max() / u64.abs().max()),
            "p_max_rel_diff_mixed_vs_fp64": float((p - p64).abs().max() / p64.abs().max()),
            "fp64_info": info64,
        })

    if not args.no_cpu_baseline:
        base, resid = cpu_baseline(S, delta, (mu, K, alpha), np.asarray(E), p.cpu().numpy(), u.cpu().numpy())
        result["cpu_baseline"] = base
        result["oracle_residual_mixed"] = resid
    plan.close()
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
