"""Benchmark: multigrid solve time to a 1e-10 relative residual on a 513^3 grid.

Workload: 3D Poisson, 7-point finite differences, 513^3 nodes (zero Dirichlet data),
f = U[-1,1] on interior nodes (numpy default_rng(3)), V(2,2) red-black Gauss-Seidel,
9 levels.  One step = one complete solve from u = 0 to ||f - A u|| <= 1e-10 ||f|| with
FP32 V-cycles inside FP64 iterative refinement (the headline form); the plain FP64 solve
of the same system is timed beside it.  Inputs are resident on the GPU before timing.

Also reported:
  - fine-level smoother throughput (GLUP/s) from 20 sweeps timed alone, and the roofline
    of the fine-level FP64 smoother kernel: algorithmic bytes per launch (24 B per interior
    node: read u, read f, write u, for the 2 sweeps one launch fuses) / average launch
    duration from HIP events on the library's stream;
  - HBM traffic per launch from rocprofv3 counters committed under profiles/ (null if
    absent or taken on different kernel source);
  - the CPU oracle on the same workload: full FP64 solves to 1e-10 on all host threads
    (median of 3 after a warm-up; about 20 s of host time);
  - the paper's own benchmark solver (Sect. 5-6) on a uniform cell-centred grid of 512^3
    cells ("fv_benchmark"): the fine-level damped-Jacobi sweep in GLUP/s against the
    paper's light-speed model (24 B per cell update: load u, load f, store u), the average
    time of a V(3,3) cycle over 100 cycles with 256 coarsest iterations (Sect. 6), and the
    L2 error of the harmonic problem (Eq. 1-2) at 256^3 and 512^3 cells with its
    grid-convergence ratio kappa (Eq. 3).  --no-fv skips it;
  - the differentiable variable-coefficient solve ("gradient") on workloads 4 (257^3, FP64)
    and 5 (513^3, FP32-refined): forward solve, adjoint solve, the fused gradient pass (and its
    bandwidth at 32 B per node) and one torch.autograd step.  --no-gradient skips it;
  - Galerkin coarse operators ("galerkin") against the rediscretised hierarchy on the
    lognormal-coefficient workloads at 257^3 and 513^3: setup, cycles and time of an FP64
    solve to 1e-10.  --no-galerkin skips it;
  - the 2:1 refined block layout of Sect. 5 ("refined_blocks", 56 + 64 blocks): time of the
    ghost exchange (Sect. 3: same-level, F2C, quadratic C2F), of a composite Jacobi sweep and
    of a V(3,3) cycle of Sect. 5's multigrid at 64^3 and 128^3 cells per block, and Table 1
    from GPU solves (35 V(3,3)-cycles, the paper's stopping rule) for constant, linear and
    quadratic C2F at 16^3 ... 128^3 cells per block (--table1-max 256 adds the paper's largest
    size), with kappa (Eq. 3) and the paper's values beside them.  --no-blocks skips it.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-fv] [--n 513]

HBM traffic of the fine-level smoother (two counter runs, then a summary):
  rocprofv3 --pmc FETCH_SIZE --output-format csv -d out/pmc_fetch -o pmc -- python bench.py --pmc-sample
  rocprofv3 --pmc WRITE_SIZE --output-format csv -d out/pmc_write -o pmc -- python bench.py --pmc-sample
  python bench.py --summarize-pmc out/pmc_fetch out/pmc_write
--pmc-sample runs a plain device copy of 1 GiB (the calibration: its counters must read
1 GiB fetched and 1 GiB written) and 10 launches of the fused FP64 smoother at 513^3.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
SMOOTHER_KERNEL = "k_rbgs_tiled"
SMOOTHER_SOURCE = os.path.join(ROOT, "paper_2403_08063_amd", "csrc", "mg_smooth_tiled.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rbgs_tiled_f64_513_traffic.json")


def light_speed_glups(bandwidth_gbs: float, bytes_per_lup: float) -> float:
    """The paper's light-speed model (Sect. 6): maximum lattice updates per second =
    bandwidth / bytes per update."""
    return bandwidth_gbs / bytes_per_lup


def source_hash(path: str) -> str:
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def measured_traffic(interior_nodes: int):
    """HBM bytes per launch of the FP64 fused smoother from committed rocprofv3 counters,
    if they were taken on the current kernel source."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256_16") != source_hash(SMOOTHER_SOURCE) or rec.get("n") is None:
        return None
    if (rec["n"] - 2) ** 3 != interior_nodes:
        return None
    return rec.get("bytes_per_launch")


CALIB_BYTES = 1 << 30


def pmc_sample(n: int):
    """Workload profiled by the counter runs: a calibration copy, then the smoother."""
    import torch

    from paper_2403_08063_amd import Multigrid, inputs

    dev = torch.device("cuda:0")
    a = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    levels = (n - 1).bit_length() - 1
    f = torch.from_numpy(inputs.uniform_interior(3, n, seed=3)).to(dev)
    u = torch.zeros_like(f)
    mg = Multigrid(3, n, levels, precision="f64", device=dev)
    mg.smooth(0, f, u, 20)
    torch.cuda.synchronize()
    print("pmc sample done", file=sys.stderr)


def pmc_ir_sample(n: int):
    """Counter-run workload for the kernels of the FP32-refined solve: the calibration copy,
    then two FP32-refined solves of the benchmark workload."""
    import torch

    from paper_2403_08063_amd import Multigrid, inputs

    dev = torch.device("cuda:0")
    a = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    levels = (n - 1).bit_length() - 1
    f = torch.from_numpy(inputs.uniform_interior(3, n, seed=3)).to(dev)
    mg = Multigrid(3, n, levels, precision="f32_ir", device=dev)
    for _ in range(2):
        mg.solve(f, tol=1e-10)
    torch.cuda.synchronize()
    print("pmc ir sample done", file=sys.stderr)


# Algorithmic bytes per interior node of the fine-level kernels of the FP32-refined solve,
# by kernel-name pattern (a regular expression on the short name: value type, variable
# coefficient, sweeps, then any tile shape, then input mode and fused restriction):
# (pattern, what it is, bytes per node)
IR_KERNELS = [
    (r"k_rbgs_tiled<float, false, 2, \d+, \d+, \d+, 1, 1", "FP32 pre-smoothing from 0 + residual restriction",
     4 + 4 + 0.5),
    (r"k_rbgs_tiled<float, false, 2, \d+, \d+, \d+, 2, 0", "FP32 post-smoothing with the prolongation",
     4 + 4 + 4 + 0.5),
    (r"k_pass<false, 2,", "refinement pass (u += s e, r = f - A u, norm, r32)", 8 + 8 + 4 + 8 + 4),
    (r"k_pass<false, 6,", "first refinement pass (+ right-hand-side norm)", 8 + 8 + 8 + 4),
]


def summarize_pmc_kernels(fetch_dir: str, write_dir: str, n: int):
    """Per-dispatch HBM bytes of the fine-level launches (the largest dispatches of each
    kernel) of the FP32-refined solve, from the two counter runs of pmc_ir_sample, each
    counter scaled so that the calibration copy reads exactly its known size; a markdown
    table on stdout."""
    import csv
    import glob
    import re

    meas = {}
    for key, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = []
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(path)):
                if r.get("Counter_Name") == counter:
                    rows.append((_short_kernel_name(r["Kernel_Name"]), float(r["Counter_Value"])))
        copy = [v for name, v in rows if "copy" in name.lower() and "fill" not in name.lower()]
        if not copy:
            raise SystemExit(f"{counter}: no calibration copy in {d}")
        factor = (CALIB_BYTES / 1024.0) / copy[0]
        for pat, _, _ in IR_KERNELS:
            vals = [v for name, v in rows if re.match(pat, name)]
            if not vals:
                continue
            top = max(vals)
            fine = [v for v in vals if v >= 0.5 * top]  # the fine-level dispatches
            meas.setdefault(pat, {})[key] = (sum(fine) / len(fine) * 1024.0 * factor, len(fine), factor)
    m = (n - 2) ** 3
    print("| kernel (name pattern) | what | fine-level dispatches | FETCH bytes | WRITE bytes | measured / algorithmic |")
    print("|---|---|---:|---:|---:|---:|")
    for pat, what, bpn in IR_KERNELS:
        if pat not in meas or len(meas[pat]) < 2:
            continue
        fb, cnt, _ = meas[pat]["fetch"]
        wb, _, _ = meas[pat]["write"]
        print(f"| `{pat}` | {what} | {cnt} | {fb:.3e} | {wb:.3e} | "
              f"{(fb + wb) / (bpn * m):.3f} ({bpn:g} B per node) |")


def pmc_fv_sample(N: int = 512):
    """Counter-run workload for the paper's FV sweep: the calibration copy, then 10 damped
    Jacobi sweeps on the 512^3-cell level (the exact-partition pass)."""
    import torch

    from paper_2403_08063_amd import FVMultigrid, inputs

    dev = torch.device("cuda:0")
    a = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    u0, _ = inputs.fv_harmonic(N)
    mg = FVMultigrid(N, device=dev)
    u = torch.from_numpy(u0).to(dev)
    mg.jacobi(0, torch.zeros_like(u), u, 10)
    torch.cuda.synchronize()
    print("pmc fv sample done", file=sys.stderr)


def summarize_pmc_fv(fetch_dir: str, write_dir: str, N: int = 512):
    """Per-launch HBM bytes of the FV Jacobi pass from the two counter runs of
    pmc_fv_sample, calibrated as summarize_pmc does; printed, not stored."""
    import csv
    import glob

    out = {}
    for key, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = []
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(path)):
                if r.get("Counter_Name") == counter:
                    rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
        copy = [v for name, v in rows if "copy" in name.lower() and "fill" not in name.lower()]
        sweep = [v for name, v in rows if "k_pass<false, 4," in name]
        if not copy or not sweep:
            raise SystemExit(f"{counter}: no calibration copy or FV sweep dispatch in {d}")
        factor = (CALIB_BYTES / 1024.0) / copy[0]
        out[key] = {"counter_kib_per_launch": sum(sweep) / len(sweep), "calibration_kib": copy[0],
                    "scale": factor, "bytes_per_launch": sum(sweep) / len(sweep) * 1024.0 * factor,
                    "launches": len(sweep)}
    total = out["fetch"]["bytes_per_launch"] + out["write"]["bytes_per_launch"]
    alg = 24 * N ** 3
    print(json.dumps({"kernel": "k_pass<false, 4, ..> (FV damped Jacobi sweep)", "N": N,
                      "fetch": out["fetch"], "write": out["write"], "bytes_per_launch": total,
                      "algorithmic_bytes_per_launch": alg, "traffic_over_algorithmic": total / alg},
                     indent=1))


def summarize_pmc(fetch_dir: str, write_dir: str, n: int):
    """Per-launch HBM bytes of the fused FP64 smoother from the two counter runs, each
    counter scaled so that the calibration copy reads exactly its known size."""
    import csv
    import glob

    def per_kernel(d, counter):
        rows = []
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(path)):
                if r.get("Counter_Name") == counter:
                    rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
        return rows

    out = {}
    for key, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = per_kernel(d, counter)
        copy = [v for name, v in rows if "copy" in name.lower() and "fill" not in name.lower()]
        smooth = [v for name, v in rows if SMOOTHER_KERNEL in name and "double" in name]
        if not copy or not smooth:
            raise SystemExit(f"{counter}: no calibration copy or smoother dispatch in {d}")
        calib = copy[0]  # KiB the counter reads for the 1 GiB calibration copy
        factor = (CALIB_BYTES / 1024.0) / calib
        out[key] = {"counter_kib_per_launch": sum(smooth) / len(smooth),
                    "calibration_kib": calib, "scale": factor,
                    "bytes_per_launch": sum(smooth) / len(smooth) * 1024.0 * factor,
                    "launches": len(smooth)}
    rec = {
        "kernel": f"{SMOOTHER_KERNEL}<double, 2 sweeps>", "n": n,
        "source_sha256_16": source_hash(SMOOTHER_SOURCE),
        "fetch": out["fetch"], "write": out["write"],
        "bytes_per_launch": out["fetch"]["bytes_per_launch"] + out["write"]["bytes_per_launch"],
        "algorithmic_bytes_per_launch": 24 * (n - 2) ** 3,
    }
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    json.dump(rec, open(TRAFFIC_FILE, "w"), indent=1)
    print(json.dumps(rec, indent=1))


def _short_kernel_name(name: str) -> str:
    name = name.replace("void ", "").replace("mgk::", "").replace("(anonymous namespace)::", "")
    depth, out = 0, []
    for ch in name:  # drop the argument list, keep template arguments
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def summarize_trace(trace_dir: str, bench_log: str = None, top: int = 24, by_grid: bool = False):
    """Markdown summary of a `rocprofv3 --kernel-trace --stats` run of this script: the
    per-kernel table and the mean duration of the fine-level FP64 smoother launches (the
    largest grid of the plain k_rbgs_tiled<double, ...> pass), beside bench.py's own
    HIP-event figure;
    by_grid adds a table per kernel and launch grid (the levels of a multigrid run)."""
    import csv
    import glob

    stats = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    trace = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not stats or not trace:
        raise SystemExit(f"no kernel_stats / kernel_trace csv under {trace_dir}")
    rows = list(csv.DictReader(open(stats[0])))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = ["| kernel | calls | total ms | avg us | share |", "|---|---:|---:|---:|---:|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:top]:
        t = float(r["TotalDurationNs"])
        lines.append(f"| `{_short_kernel_name(r['Name'])}` | {r['Calls']} | {t / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {100 * t / total:.1f}% |")
    launches = []
    # the plain smoother (2 sweeps, input read, no fused transfer: template arguments
    # <double, false, 2, waves, rows, prefetch, 0, 0, lanes>), the kernel bench.py times
    plain = re.compile(r"<double, false, 2, \d+, \d+, \d+, 0, 0, \d+>$")
    for r in csv.DictReader(open(trace[0])):
        short = _short_kernel_name(r["Kernel_Name"])
        if short.startswith(SMOOTHER_KERNEL + "<double") and plain.search(short):
            grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            launches.append((grid, short,
                             (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3))
    head = []
    if launches:
        gmax = max(g for g, _, _ in launches)
        fine = [(k, d) for g, k, d in launches if g == gmax]
        names = sorted({k for k, _ in fine})
        mean = sum(d for _, d in fine) / len(fine)
        head.append(f"Fine-level launches (largest grid) of `{'`, `'.join(names)}` in the trace: "
                    f"{len(fine)}, mean duration {mean:.1f} us")
        if bench_log:
            for line in open(bench_log):
                if line.startswith("{"):
                    rec = json.loads(line)
                    head[-1] += (f" (bench.py's HIP-event average per launch in the same run: "
                                 f"{rec['roofline']['launch_ms'] * 1e3:.1f} us)")
        head[-1] += "."
    if by_grid:
        agg = {}
        for r in csv.DictReader(open(trace[0])):
            key = (_short_kernel_name(r["Kernel_Name"]),
                   f"{r['Grid_Size_X']}x{r['Grid_Size_Y']}x{r['Grid_Size_Z']}")
            d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            n, t = agg.get(key, (0, 0.0))
            agg[key] = (n + 1, t + d)
        lines += ["", "| kernel | grid (threads) | calls | total ms | avg us |", "|---|---|---:|---:|---:|"]
        for (k, g), (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
            lines.append(f"| `{k}` | {g} | {n} | {t / 1e3:.2f} | {t / n:.1f} |")
    print("\n".join(head + [""] + lines))


def gradient_benchmark(dev, workloads=((4, "f64"), (5, "f32_ir"))):
    """The differentiable variable-coefficient solve on its workloads (k = exp(GRF), f = 1,
    L = 0.5 ||u - u_obs||^2 with u_obs the solution for the perturbed coefficient k_obs):
    forward solve, adjoint solve and the fused gradient pass timed one by one (best of 3
    after one), and one whole torch.autograd step (forward, loss, backward with the forward
    recomputed) through solve()."""
    import numpy as np
    import torch

    from paper_2403_08063_amd import Multigrid, inputs, solve

    out = {}
    for idx, prec in workloads:
        w = inputs.config(idx)
        n, levels = w["n"], w["levels"]
        k = torch.from_numpy(w["k"]).to(dev)
        kobs = torch.from_numpy(w["k_obs"]).to(dev)
        f = torch.from_numpy(w["f"]).to(dev)
        mg = Multigrid(3, n, levels, precision=prec, variable=True, device=dev)
        mg.set_coefficients(kobs)
        uobs, _ = mg.solve(f, mg.zeros(), tol=1e-10)
        mg.set_coefficients(k)

        def best(fn, reps=3):
            fn()
            ts = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = fn()
                torch.cuda.synchronize()
                ts.append((time.perf_counter() - t0) * 1e3)
            return float(np.min(ts)), r

        t_fwd, (u, info) = best(lambda: mg.solve(f, mg.zeros(), tol=1e-10))
        g = (u - uobs).contiguous()
        t_adj, (lam, info_a) = best(lambda: mg.solve_adjoint(g, mg.zeros(), tol=1e-10))
        t_grad, _ = best(lambda: mg.grad(u, lam), reps=5)

        def step():
            kk = k.clone().requires_grad_(True)
            uu = solve(kk, f, mg=mg, tol=1e-10, precision=prec)
            loss = 0.5 * ((uu - uobs) ** 2).sum()
            loss.backward()
            return kk.grad

        t_step, _ = best(step)
        out[str(idx)] = {
            "n": n, "precision": prec,
            "forward_ms": round(t_fwd, 2), "forward_cycles": info.cycles,
            "adjoint_ms": round(t_adj, 2), "adjoint_cycles": info_a.cycles,
            "grad_pass_ms": round(t_grad, 3),
            "grad_pass_gbs": round(32 * n ** 3 / (t_grad * 1e-3) / 1e9, 1),
            "autograd_step_ms": round(t_step, 1),
        }
        print(f"bench: gradient workload {idx} ({n}^3, {prec}): forward {t_fwd:.1f} ms "
              f"({info.cycles} cycles), adjoint {t_adj:.1f} ms, gradient pass {t_grad:.3f} ms, "
              f"autograd step {t_step:.1f} ms", file=sys.stderr, flush=True)
        mg.close()
        del k, kobs, f, uobs, u, g, lam
        torch.cuda.empty_cache()
    return {"workload": "3D -div(k grad u) = 1, k = exp(GRF, corr 0.1, sigma 1), zero Dirichlet data; "
                        "L = 0.5 ||u - u_obs||^2; solves to 1e-10; gradient pass 32 B per node "
                        "(read u, lambda; write dk, df)", "workloads": out}


def galerkin_benchmark(dev, sizes=((257, 8, 4), (513, 9, 5))):
    """Galerkin against rediscretised coarse operators on the lognormal-coefficient workloads
    (f = 1, k = exp(Gaussian random field)): setup (coefficient hierarchy / Galerkin
    products), cycles and time of an FP64 solve to 1e-10 from u = 0, best of 3 after one."""
    import numpy as np
    import torch

    from paper_2403_08063_amd import GalerkinMultigrid, Multigrid, inputs

    out = {}
    for n, levels, seed in sizes:
        k = torch.from_numpy(inputs.lognormal_k(3, n, seed=seed)).to(dev)
        f = torch.from_numpy(inputs.constant_interior(3, n)).to(dev)
        rec = {}
        for name in ("galerkin", "galerkin_f32_stencils", "rediscretised"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name.startswith("galerkin"):
                mg = GalerkinMultigrid(k, levels, coarse_f32=name.endswith("f32_stencils"))
            else:
                mg = Multigrid(3, n, levels, variable=True, device=dev)
                mg.set_coefficients(k)
            torch.cuda.synchronize()
            t_setup = (time.perf_counter() - t0) * 1e3
            ms = []
            for rep in range(4):
                u = torch.zeros_like(f)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                u, info = mg.solve(f, u, tol=1e-10)
                torch.cuda.synchronize()
                if rep:
                    ms.append((time.perf_counter() - t0) * 1e3)
            rec[name] = {"setup_ms": round(t_setup, 2), "cycles": info.cycles,
                         "relres": info.relres, "solve_ms": round(float(np.min(ms)), 2)}
            if name == "galerkin":
                ug = u.clone()
            elif name == "rediscretised":
                rec["solution_rel_diff"] = float((ug - u).abs().max() / u.abs().max())
            mg.close()
            del mg, u
        out[str(n)] = rec
        print(f"bench: galerkin n={n}: {rec['galerkin']['cycles']} cycles {rec['galerkin']['solve_ms']} ms "
              f"(setup {rec['galerkin']['setup_ms']} ms); with FP32 coarse stencils "
              f"{rec['galerkin_f32_stencils']['cycles']} cycles {rec['galerkin_f32_stencils']['solve_ms']} ms; "
              f"rediscretised {rec['rediscretised']['cycles']} cycles "
              f"{rec['rediscretised']['solve_ms']} ms", file=sys.stderr, flush=True)
        del k, f, ug
        torch.cuda.empty_cache()
    return {"workload": "3D -div(k grad u) = 1, k = exp(GRF, corr 0.1, sigma 1), zero Dirichlet data, "
                        "V(2,2), FP64 to 1e-10 relative residual; Galerkin R A P coarse operators "
                        "(27-point, 8-colour Gauss-Seidel) vs rediscretised (7-point, geometric "
                        "coefficient coarsening)", "sizes": out}


def fv_benchmark(dev, copy_gbs: float, N: int = 512, cycles: int = 100):
    """The paper's benchmark solver on N^3 cells (see the module docstring)."""
    import numpy as np
    import torch

    from paper_2403_08063_amd import FVMultigrid, inputs

    levels = max(1, N.bit_length() - 2)  # coarsest 4^3 cells
    mg = FVMultigrid(N, levels, device=dev)
    stream = mg.stream
    f = torch.from_numpy(inputs.fv_uniform(N, 11)).to(dev)
    u = torch.zeros_like(f)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # fine-level Jacobi sweeps alone (20 sweeps, out of place between u and the workspace)
    sweeps = 20
    mg.jacobi(0, f, u, sweeps)
    ms = []
    for _ in range(3):
        ev0.record(stream)
        mg.jacobi(0, f, u, sweeps)
        ev1.record(stream)
        ev1.synchronize()
        ms.append(ev0.elapsed_time(ev1))
    t_sweep = float(np.median(ms)) / sweeps
    cells = N ** 3
    glups = cells / (t_sweep * 1e-3) / 1e9
    gbs = 24 * cells / (t_sweep * 1e-3) / 1e9
    # V(3,3) cycles with 256 coarsest iterations (Sect. 6)
    mg.vcycle(f, u)
    ev0.record(stream)
    for _ in range(cycles):
        mg.vcycle(f, u)
    ev1.record(stream)
    ev1.synchronize()
    t_cycle = ev0.elapsed_time(ev1) / cycles
    del f, u
    # the harmonic problem (Eq. 1-2): 35 cycles, error against the exact solution
    errs = {}
    for n_cells in (N // 2, N):
        u0, exact = inputs.fv_harmonic(n_cells)
        m2 = FVMultigrid(n_cells, max(1, n_cells.bit_length() - 2), device=dev)
        fz = torch.zeros(u0.shape, dtype=torch.float64, device=dev)
        ug, info = m2.solve(fz, torch.from_numpy(u0).to(dev), tol=1e-16)
        e = ug[1:-1, 1:-1, 1:-1] - torch.from_numpy(exact[1:-1, 1:-1, 1:-1]).to(dev)
        errs[n_cells] = (float(torch.sqrt(torch.sum(e * e) / n_cells ** 3)), info.cycles,
                         info.relres)
        m2.close()
        del fz, ug, e
    mg.close()
    return {
        "workload": f"cell-centred FV Poisson on {N}^3 cells of [0,1]^3, V(3,3) damped Jacobi "
                    f"(omega 0.8), {levels} levels down to 4^3 cells, 256 coarsest iterations",
        "jacobi_ms_per_sweep": round(t_sweep, 4),
        "jacobi_glups": round(glups, 1),
        "jacobi_algorithmic_gbs": round(gbs, 1),
        "jacobi_frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
        "jacobi_frac_of_copy": round(gbs / copy_gbs, 4),
        "light_speed_glups_peak_24B": round(light_speed_glups(HBM_PEAK_GBS, 24), 1),
        "light_speed_glups_copy_24B": round(light_speed_glups(copy_gbs, 24), 1),
        "vcycle_ms": round(t_cycle, 3),
        "vcycles_timed": cycles,
        "harmonic_l2_error": {str(k): v[0] for k, v in errs.items()},
        "harmonic_cycles": {str(k): v[1] for k, v in errs.items()},
        "harmonic_residual_norm": {str(k): v[2] for k, v in errs.items()},
        "harmonic_kappa": round(errs[N][0] / errs[N // 2][0], 4),
    }


# Sect. 5, Table 1: L2 error norm per block size for the constant, first- and second-order
# C2F schemes (the paper's printed values, for comparison only)
PAPER_TABLE1 = {
    0: {16: 0.235, 32: 0.227, 64: 0.224, 128: 0.222, 256: 0.221},
    1: {16: 1.067e-2, 32: 5.255e-3, 64: 2.611e-3, 128: 1.302e-3, 256: 6.499e-4},
    2: {16: 3.017e-3, 32: 7.215e-4, 64: 1.764e-4, 128: 4.361e-5, 256: 1.084e-5},
}


def _block_l2_error(u, B):
    """Table 1's L2 error norm of a refined-layout solution tensor against Eq. 2's exact
    solution at the inner cell centres: the root mean square over all cells (on u's device)."""
    import math

    import torch

    from paper_2403_08063_amd import inputs

    i = torch.arange(B, dtype=torch.float64, device=u.device) + 0.5
    total, count = 0.0, 0
    for b, (_, idx, w) in enumerate(inputs.block_list()):
        h = w / B
        x, y, z = (idx[a] * w + i * h for a in range(3))
        ex = (torch.sin(math.pi * x)[None, None, :] * torch.sin(math.pi * y)[None, :, None]
              * torch.sinh(math.sqrt(2.0) * math.pi * z)[:, None, None])
        d = u[b, 1:-1, 1:-1, 1:-1] - ex
        total += float(torch.sum(d * d))
        count += B ** 3
    return math.sqrt(total / count)


def refined_benchmark(dev, B: int = 64, table_sizes=(16, 32, 64, 128)):
    """The refined block layout (see the module docstring)."""
    import numpy as np
    import torch

    from paper_2403_08063_amd import RefinedBlocks, inputs

    rb = RefinedBlocks(B, 2, device=dev)
    stream = rb.stream
    u = inputs.block_harmonic_device(B, dev)
    f = torch.zeros_like(u)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 50
    rb.fill(u)
    ev0.record(stream)
    for _ in range(reps):
        rb.fill(u)
    ev1.record(stream)
    ev1.synchronize()
    t_fill = ev0.elapsed_time(ev1) / reps
    rb.jacobi(f, u, 20)
    ms = []
    for _ in range(3):
        ev0.record(stream)
        rb.jacobi(f, u, 20)
        ev1.record(stream)
        ev1.synchronize()
        ms.append(ev0.elapsed_time(ev1))
    t_sweep = float(np.median(ms)) / 20  # fill + sweep
    cells = 120 * B ** 3
    rb.close()
    del u, f
    # one V(3,3)-cycle (256 coarsest iterations), 5 cycles timed after one
    t_cycle = {}
    for Bv in (64, 128):
        rv = RefinedBlocks(Bv, 2, device=dev)
        uv = inputs.block_harmonic_device(Bv, dev)
        fv = torch.zeros_like(uv)
        rv.vcycle(fv, uv)
        ev0.record(rv.stream)
        for _ in range(5):
            rv.vcycle(fv, uv)
        ev1.record(rv.stream)
        ev1.synchronize()
        t_cycle[Bv] = ev0.elapsed_time(ev1) / 5
        rv.close()
        del uv, fv
    # Table 1: 35 cycles (L2 residual 1e-16 is below rounding), L2 error per block size
    errs, t_solve, cyc = {0: {}, 1: {}, 2: {}}, {0: {}, 1: {}, 2: {}}, {0: {}, 1: {}, 2: {}}
    for order in (0, 1, 2):
        for Bs in table_sizes:
            r2 = RefinedBlocks(Bs, order, device=dev)
            ug = inputs.block_harmonic_device(Bs, dev)
            fz = torch.zeros_like(ug)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ug, info = r2.mg_solve(fz, ug, tol=1e-16)
            torch.cuda.synchronize()
            t_solve[order][Bs] = (time.perf_counter() - t0) * 1e3
            cyc[order][Bs] = info.cycles
            errs[order][Bs] = _block_l2_error(ug, Bs)
            r2.close()
            del ug, fz
            print(f"bench: refined blocks order {order} B={Bs}: L2 error {errs[order][Bs]:.4e} "
                  f"({info.cycles} cycles, {t_solve[order][Bs]:.0f} ms)", file=sys.stderr, flush=True)
    kappa = {o: {f"{a}->{b}": round(errs[o][b] / errs[o][a], 4)
                 for a, b in zip(table_sizes[:-1], table_sizes[1:])} for o in (0, 1, 2)}
    return {
        "workload": f"2:1 refined layout of [0,1]^3 (56 level-2 + 64 level-3 blocks), {B}^3 cells "
                    "per block, quadratic C2F / linear F2C ghost exchange, damped Jacobi; "
                    "V(3,3) multigrid down to 4^3 cells per block",
        "cells": cells,
        "ghost_fill_ms": round(t_fill, 4),
        "ghost_cells_per_fill": 120 * 6 * B * B,
        "jacobi_sweep_with_fill_ms": round(t_sweep, 4),
        "jacobi_glups": round(cells / (t_sweep * 1e-3) / 1e9, 1),
        "jacobi_algorithmic_gbs": round(24 * cells / (t_sweep * 1e-3) / 1e9, 1),
        "vcycle_ms": {str(k): round(v, 3) for k, v in t_cycle.items()},
        "table1_l2_error": {str(o): {str(b): v for b, v in errs[o].items()} for o in errs},
        "table1_kappa": {str(o): kappa[o] for o in kappa},
        "table1_cycles": {str(o): {str(b): v for b, v in cyc[o].items()} for o in cyc},
        "table1_solve_ms": {str(o): {str(b): round(v, 1) for b, v in t_solve[o].items()} for o in t_solve},
        "paper_table1_l2_error": {str(o): {str(b): PAPER_TABLE1[o][b] for b in table_sizes if b in PAPER_TABLE1[o]}
                                  for o in PAPER_TABLE1},
        "table1_error_over_paper": {str(o): {str(b): round(errs[o][b] / PAPER_TABLE1[o][b], 4)
                                             for b in table_sizes if b in PAPER_TABLE1[o]}
                                    for o in errs},
    }


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(f_np, levels, fp64_cycles):
    """The oracle (OpenMP inside each colour) on the host cores: full FP64 solves of the
    workload to the same 1e-10 relative residual, at all available threads, median of 3
    after one warm-up solve, each timed from its first norm to its last cycle (the oracle's
    own clock: allocating and releasing its level hierarchy is outside).  The one-thread
    figure is sampled (one V-cycle plus one residual norm, scaled by the cycle count): a
    full solve takes about half a minute at one thread."""
    import ctypes
    import statistics

    import numpy as np

    import oracle

    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", threads))
    oracle.build()
    gomp = ctypes.CDLL("libgomp.so.1")  # the oracle's OpenMP runtime
    gomp.omp_set_num_threads(threads)

    def full_solve():
        u = np.zeros_like(f_np)
        cycles, rel, _, _ = oracle.solve(f_np, u, levels, tol=1e-10)
        return oracle.last_solve_seconds(), cycles, rel

    full_solve()  # warm-up
    runs = [full_solve() for _ in range(3)]
    t = statistics.median(r[0] for r in runs)
    cycles, rel = runs[0][1], runs[0][2]

    gomp.omp_set_num_threads(1)
    u = np.zeros_like(f_np)
    t0 = time.perf_counter()
    oracle.vcycle(f_np, u, levels)
    oracle.interior_norm2(oracle.residual(f_np, u))
    t1 = time.perf_counter() - t0
    gomp.omp_set_num_threads(threads)
    return {
        "value": round(t * 1e3, 1),
        "unit": "ms",
        "cores": threads,
        "kind": "oracle",
        "sample": f"full FP64 solve of the {f_np.shape[0]}^3 workload to 1e-10 ({cycles} cycles, "
                  f"relres {rel:.2e}) at {threads} threads, median of 3 after a warm-up "
                  f"({', '.join(f'{r[0]:.2f}' for r in runs)} s); the oracle's hierarchy "
                  f"allocation is outside the timing",
        "value_1_thread": round(t1 * cycles * 1e3, 1),
        "value_1_thread_kind": f"sampled: one FP64 V-cycle + one residual norm at 1 thread "
                               f"({t1:.2f} s), scaled by the cycle count",
        "cpu_model": _cpu_model(),
        "next_rows": next_rows_baseline(threads),
    }


def next_rows_baseline(threads):
    """The oracles of the components beyond the hot path, each timed once on a bounded sample
    beside the GPU leg that measures the same operation: the FV V(3,3)-cycle (C oracle, all
    threads), the refined-layout V(3,3)-cycle (numpy oracle) and the Galerkin solve (scipy
    oracle), with the time per million cells for comparison with the GPU figures."""
    import numpy as np

    import oracle
    from oracle import blocks as oblocks
    from oracle import galerkin as ogal
    from paper_2403_08063_amd import inputs

    out = {}
    N = 256
    u, _ = inputs.fv_harmonic(N)
    t0 = time.perf_counter()
    oracle.fv_vcycle(np.zeros_like(u), u, N.bit_length() - 2)
    t = time.perf_counter() - t0
    out["fv_vcycle"] = {"ms": round(t * 1e3, 1), "ms_per_mcell": round(t * 1e3 / (N ** 3 / 1e6), 2),
                        "sample": f"one V(3,3) cycle, {N}^3 cells, C oracle at {threads} threads"}
    B = 16
    u0, _ = inputs.block_harmonic(B)
    t0 = time.perf_counter()
    oblocks.vcycle(u0.reshape(-1).copy(), np.zeros(u0.size), oblocks.mg_block_sizes(B), 2)
    t = time.perf_counter() - t0
    out["blocks_vcycle"] = {"ms": round(t * 1e3, 1), "ms_per_mcell": round(t * 1e3 / (120 * B ** 3 / 1e6), 2),
                            "sample": f"one V(3,3) cycle, 120 blocks of {B}^3 cells, quadratic C2F, numpy oracle"}
    n = 65
    k, f = inputs.lognormal_k(3, n, seed=4), inputs.constant_interior(3, n)
    t0 = time.perf_counter()
    _, cycles, _ = ogal.solve(k, f, 6)
    t = time.perf_counter() - t0
    out["galerkin_solve"] = {"ms": round(t * 1e3, 1), "cycles": cycles,
                             "ms_per_mcell": round(t * 1e3 / (n ** 3 / 1e6), 2),
                             "sample": f"setup + FP64 solve to 1e-10, {n}^3 nodes, lognormal k, scipy oracle"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=513)
    ap.add_argument("--levels", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fv", action="store_true")
    ap.add_argument("--no-blocks", action="store_true")
    ap.add_argument("--no-galerkin", action="store_true")
    ap.add_argument("--no-gradient", action="store_true")
    ap.add_argument("--gradient-only", action="store_true",
                    help="run only the differentiable-solve leg, print its record")
    ap.add_argument("--galerkin-only", action="store_true",
                    help="run only the Galerkin-coarsening leg, print its record")
    ap.add_argument("--blocks-only", action="store_true",
                    help="run only the refined-block leg, print its record")
    ap.add_argument("--table1-max", type=int, default=128, choices=(64, 128, 256),
                    help="largest block size of the refined-layout Table 1 run")
    ap.add_argument("--blocks-vcycle-sample", type=int, default=0, metavar="B",
                    help="run 5 V(3,3)-cycles of the refined-layout multigrid with B^3 cells per "
                         "block after one warm-up cycle (a kernel-trace target), then exit")
    ap.add_argument("--fv-only", action="store_true",
                    help="run only the paper-benchmark (cell-centred FV) leg, print its record")
    ap.add_argument("--pmc-sample", action="store_true")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--pmc-ir-sample", action="store_true",
                    help="counter-run workload: calibration copy + 2 FP32-refined solves at n")
    ap.add_argument("--summarize-pmc-kernels", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="per-kernel HBM traffic of the FP32-refined solve's fine level")
    ap.add_argument("--pmc-fv-sample", action="store_true",
                    help="counter-run workload: calibration copy + 10 FV Jacobi sweeps at 512^3")
    ap.add_argument("--summarize-pmc-fv", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--summarize-trace", nargs="+", metavar=("TRACE_DIR", "BENCH_LOG"))
    ap.add_argument("--by-grid", action="store_true",
                    help="with --summarize-trace: add a table per kernel and launch grid")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace[:2], by_grid=args.by_grid)
        return
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.n)
        return
    if args.pmc_sample:
        pmc_sample(args.n)
        return
    if args.pmc_fv_sample:
        pmc_fv_sample()
        return
    if args.pmc_ir_sample:
        pmc_ir_sample(args.n)
        return
    if args.summarize_pmc_kernels:
        summarize_pmc_kernels(*args.summarize_pmc_kernels, args.n)
        return
    if args.summarize_pmc_fv:
        summarize_pmc_fv(*args.summarize_pmc_fv)
        return
    table_sizes = tuple(b for b in (16, 32, 64, 128, 256) if b <= args.table1_max)
    if args.blocks_vcycle_sample:
        import torch

        from paper_2403_08063_amd import RefinedBlocks, inputs

        dev = torch.device("cuda:0")
        Bv = args.blocks_vcycle_sample
        rv = RefinedBlocks(Bv, 2, device=dev)
        uv = inputs.block_harmonic_device(Bv, dev)
        fv = torch.zeros_like(uv)
        for _ in range(6):
            rv.vcycle(fv, uv)
        torch.cuda.synchronize()
        print(f"bench: 6 block V-cycles at B={Bv} done", flush=True)
        return
    if args.gradient_only:
        import torch

        print(json.dumps(gradient_benchmark(torch.device("cuda:0"))), flush=True)
        return
    if args.galerkin_only:
        import torch

        print(json.dumps(galerkin_benchmark(torch.device("cuda:0"))), flush=True)
        return
    if args.blocks_only:
        import torch

        print(json.dumps(refined_benchmark(torch.device("cuda:0"), table_sizes=table_sizes)), flush=True)
        return
    if args.fv_only:
        import torch

        dev = torch.device("cuda:0")
        a = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        mc = []
        for _ in range(4):
            e0.record()
            b.copy_(a)
            e1.record()
            e1.synchronize()
            mc.append(e0.elapsed_time(e1))
        del a, b
        copy_gbs = 2 * CALIB_BYTES / (min(mc[1:]) * 1e-3) / 1e9
        print(json.dumps({"copy_gbs": round(copy_gbs, 1), **fv_benchmark(dev, copy_gbs)}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the solver has no "
              "multi-GPU path (it would split the grid into z-slabs with a halo exchange per "
              "half-sweep)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2403_08063_amd import Multigrid, inputs

    n = args.n
    levels = args.levels or (n - 1).bit_length() - 1  # coarsest level 3^3
    dev = torch.device("cuda:0")
    f_np = inputs.uniform_interior(3, n, seed=3)
    f = torch.from_numpy(f_np).to(dev)
    print(f"bench: n={n} levels={levels} inputs on GPU", file=sys.stderr, flush=True)

    mg64 = Multigrid(3, n, levels, precision="f64", device=dev)
    mg32 = Multigrid(3, n, levels, precision="f32_ir", device=dev)
    u64 = torch.zeros_like(f)
    u32 = torch.zeros_like(f)

    def solve(mg, u):
        u.zero_()
        _, info = mg.solve(f, u, tol=1e-10)
        return info

    for _ in range(args.warmup):
        solve(mg32, u32)
        solve(mg64, u64)
    torch.cuda.synchronize()

    def timed(mg, u, steps):
        times, info = [], None
        for _ in range(steps):
            u.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = mg.solve(f, u, tol=1e-10)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        return times, info

    t32, info32 = timed(mg32, u32, args.steps)
    print(f"bench: fp32-ir solve {np.median(t32):.2f} ms cycles={info32.cycles}",
          file=sys.stderr, flush=True)
    t64, info64 = timed(mg64, u64, args.steps)
    print(f"bench: fp64 solve {np.median(t64):.2f} ms cycles={info64.cycles}",
          file=sys.stderr, flush=True)
    err = float((u32 - u64).abs().max() / u64.abs().max())

    # fine-level smoother alone: 20 sweeps = 10 fused launches (FP64), on the same stream
    interior = (n - 2) ** 3
    us = u64.clone()
    stream = mg64.stream
    sweeps = 20
    mg64.smooth(0, f, us, sweeps)  # warm
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3
    ms = []
    for _ in range(reps):
        ev0.record(stream)
        mg64.smooth(0, f, us, sweeps)
        ev1.record(stream)
        ev1.synchronize()
        ms.append(ev0.elapsed_time(ev1))
    t_sweeps = float(np.median(ms))
    glups64 = sweeps * interior / (t_sweeps * 1e-3) / 1e9
    launches = sweeps // 2
    t_launch = t_sweeps / launches
    bytes_launch = 24 * interior
    achieved = bytes_launch / (t_launch * 1e-3) / 1e9
    # FP32 smoother (inside the refinement cycles)
    f32 = f.float()
    u32s = torch.zeros_like(f32)
    mg32.smooth(0, f32, u32s, sweeps)
    ms32 = []
    for _ in range(reps):
        ev0.record(stream)
        mg32.smooth(0, f32, u32s, sweeps)
        ev1.record(stream)
        ev1.synchronize()
        ms32.append(ev0.elapsed_time(ev1))
    t_launch32 = float(np.median(ms32)) / launches
    glups32 = sweeps * interior / (float(np.median(ms32)) * 1e-3) / 1e9
    achieved32 = 12 * interior / (t_launch32 * 1e-3) / 1e9  # read u, f; write u (float)

    # achievable streaming bandwidth on this device: a plain 1 GiB device-to-device copy
    # (read + write bytes), the practical ceiling beside the 8 TB/s peak
    ca = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device=dev)
    cb = torch.empty_like(ca)
    cs = torch.cuda.current_stream()
    mc = []
    for _ in range(4):
        ev0.record(cs)
        cb.copy_(ca)
        ev1.record(cs)
        ev1.synchronize()
        mc.append(ev0.elapsed_time(ev1))
    copy_gbs = 2 * CALIB_BYTES / (min(mc[1:]) * 1e-3) / 1e9
    del ca, cb

    traffic = measured_traffic(interior)
    value = float(np.median(t32))
    rec = {
        "metric": "MG solve time to 1e-10 rel. residual at 513^3 (FP32 V(2,2) cycles in FP64 "
                  "iterative refinement); smoother GLUPS vs HBM roofline",
        "value": round(value, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(value, 3),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"3D Poisson 7-point FD, {n}^3 nodes, zero Dirichlet BC, f = U[-1,1] "
                        f"(seed 3), V(2,2) red-black GS, {levels} levels, FP32 cycles in FP64 "
                        "iterative refinement vs plain FP64, tol 1e-10",
            "n": n, "levels": levels, "tol": 1e-10,
        },
        "fp32ir_solve_ms": round(value, 3),
        "fp64_solve_ms": round(float(np.median(t64)), 3),
        "speedup_fp32ir_vs_fp64": round(float(np.median(t64)) / value, 3),
        "cycles_fp32ir": info32.cycles,
        "cycles_fp64": info64.cycles,
        "relres_fp32ir": info32.relres,
        "relres_fp64": info64.relres,
        "err_fp32ir_vs_fp64": err,
        "smoother_glups_fp64": round(glups64, 1),
        "smoother_glups_fp32": round(glups32, 1),
        "smoother_light_speed_glups_fp64_24B": round(light_speed_glups(HBM_PEAK_GBS, 24), 1),
        "roofline": {
            "kernel": f"{SMOOTHER_KERNEL}<double, 2 sweeps> (fine level)",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_gbs": round(traffic / (t_launch * 1e-3) / 1e9, 1) if traffic else None,
            "bytes_per_launch": bytes_launch,
            "launch_ms": round(t_launch, 4),
            "copy_gbs": round(copy_gbs, 1),
            "frac_of_copy": round(achieved / copy_gbs, 4),
        },
        "roofline_fp32_smoother": {
            "kernel": f"{SMOOTHER_KERNEL}<float, 2 sweeps> (fine level)",
            "bound": "hbm",
            "achieved": round(achieved32, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved32 / HBM_PEAK_GBS, 4),
            "bytes_per_launch": 12 * interior,
            "launch_ms": round(t_launch32, 4),
        },
    }
    if not args.no_fv:
        print("bench: paper benchmark solver (cell-centred FV, 512^3 cells)", file=sys.stderr,
              flush=True)
        del mg32, u32, us, f32, u32s
        torch.cuda.empty_cache()
        rec["fv_benchmark"] = fv_benchmark(dev, copy_gbs)
        print(f"bench: fv jacobi {rec['fv_benchmark']['jacobi_glups']} GLUP/s, V(3,3) "
              f"{rec['fv_benchmark']['vcycle_ms']} ms", file=sys.stderr, flush=True)
    if not args.no_gradient:
        print("bench: differentiable solve (lognormal k)", file=sys.stderr, flush=True)
        rec["gradient"] = gradient_benchmark(dev)
    if not args.no_galerkin:
        print("bench: Galerkin coarsening (lognormal k)", file=sys.stderr, flush=True)
        rec["galerkin"] = galerkin_benchmark(dev)
    if not args.no_blocks:
        print("bench: refined block layout (Sect. 3/5)", file=sys.stderr, flush=True)
        rec["refined_blocks"] = refined_benchmark(dev, table_sizes=table_sizes)
        print(f"bench: refined blocks fill {rec['refined_blocks']['ghost_fill_ms']} ms, V(3,3) "
              f"{rec['refined_blocks']['vcycle_ms']} ms, kappa (quadratic) "
              f"{rec['refined_blocks']['table1_kappa']['2']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(f_np, levels, info64.cycles)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
