"""Benchmark: fine-grid unknowns solved per second to a relative residual of 1e-10.

One step = the whole hot path on one batch of synthetic input already resident
in HBM: charge deposition of the spheres, boundary folding of the right-hand
side and the multigrid solve from phi = 0 to ||b - A phi|| / ||b|| < 1e-10.
Workload (default): 512^3 cells, Dirichlet phi = 0 / 1 on the z faces and
zero-Neumann sides, 2000 seeded charged spheres of radius U[3, 6], plain FP64
V(2,2)-cycles (correction factor 1.95) down to an 8^3 coarsest grid; the
largest workload that fits one GPU, with arrays far beyond the caches.

Prints one JSON line.  Also reports the FP32-in-FP64 refinement solve on the
same input at equal final accuracy, the roofline of the dominant kernel (its
launches timed with HIP events on the solver's stream in a second pass of
the same steps, so the headline timing carries no instrumentation), the 256^3
workload, the variable-permittivity solve, the microchannel forward + adjoint
step, the time-step scene and the CPU oracle's rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import paper_1410_6609_amd as pkg  # noqa: E402
import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
KERNEL_NAMES = {   # finest-level passes of a V(2,2) cycle, two sweeps fused per pass (long z-marches)
    "pre": "void k_pass<double, 4, 0, 1, 2, 8, true>",
    "post": "void k_pass<double, 4, 2, 2, 2, 8, true>",
}


def kernel_sources_sha256() -> str:
    h = hashlib.sha256()
    for f in ("paper_1410_6609_amd/csrc/ccmg_kernels.hpp", "paper_1410_6609_amd/csrc/ccmg.hip"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, which: str):
    """HBM bytes per launch of the finest-level pass from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE runs, copy-calibrated), or None when the
    summary is missing or was taken from other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if "```json" not in text:
        return None
    data = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    if data.get("kernel_source_sha256") != kernel_sources_sha256():
        return None
    best = None
    for key, v in data["kernels"].items():
        name, grid = key.rsplit("|", 1)
        if name.startswith(KERNEL_NAMES[which]) and (best is None or int(grid) > best[0]):
            best = (int(grid), v["fetch_bytes"] + v["write_bytes"])
    return None if best is None else best[1]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_solver(w: W.Workload, dev, precision=pkg.FP64, fuse=2, inner=4):
    opt = pkg.Options(levels=w.levels, nu1=w.nu1, nu2=w.nu2, omega=w.omega, precision=precision,
                      fuse_sweeps=fuse, ir_inner_cycles=inner)
    return pkg.Solver(w.shape, w.h, list(zip(w.kinds, w.values)), opt, device=dev)


def run_steps(s, sph_dev, f, phi, w, n):
    stats = None
    for _ in range(n):
        s.deposit(*sph_dev, w.eps, out=f)
        # from phi = 0: phi is output only (ccmg_solve_zero)
        _, stats = s.solve(f, phi, rtol=w.rtol, max_cycles=100, zero_guess=True)
    return stats


def timed(s, sph_dev, f, phi, w, steps):
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    st = run_steps(s, sph_dev, f, phi, w, steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return ev0.elapsed_time(ev1) / 1e3, wall, st


def host_cpu() -> dict:
    """The host's CPU model and the cores this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "usable_cores": len(os.sched_getaffinity(0))}


def cpu_baseline(w: W.Workload, sph, budget_s: float = 12.0):
    import oracle
    oracle.lib()
    cores = oracle.num_threads()
    t0 = time.perf_counter()
    runs = 0
    cycles = 0
    while True:
        f, _ = oracle.deposit(w.shape, w.h, sph.centers, sph.radii, sph.charges, w.eps)
        phi, hist, st = oracle.solve_problem(f, w.h, w.kinds, w.values, w.levels, rtol=w.rtol,
                                             nu1=w.nu1, nu2=w.nu2, omega=w.omega)
        runs += 1
        cycles = len(hist) - 1
        el = time.perf_counter() - t0
        if el >= budget_s or runs >= 4:
            break
    per = el / runs
    return {"value": w.cells / per, "unit": "unknowns/s", "cores": cores, "kind": "oracle",
            "sample": f"{runs} full solve(s) of the same workload (deposit + fold + {cycles} V(2,2)-cycles "
                      f"to 1e-10), {per:.2f} s each, OpenMP threads={cores}",
            "seconds_per_solve": per, **host_cpu()}, phi


def timestep_scene(dev, steps: int):
    """The paper's per-node time-step use of the solver: 256 x 512 x 256 cells,
    3456 moving spheres deposited with sub-sampling factor 2 (volume
    normalisation), 5 warm V(3,3)-cycles at the first step and 1 per later
    step, the residual norm of every step written on the device, then the
    electrostatic force on every sphere.  One step = deposition + fold +
    cycle(s) + force; inputs (all sphere positions) resident in HBM."""
    w = W.SCENE
    sph = W.scene_spheres(w)
    warm = 3
    traj = torch.tensor(W.scene_trajectory(w, max(steps, warm)), device=dev)
    r = torch.tensor(sph.radii, device=dev)
    q = torch.tensor(sph.charges, device=dev)
    s = make_solver(w, dev)
    f = s.zeros()
    phi = s.zeros()
    rels = torch.zeros(max(steps, warm), dtype=torch.float64, device=dev)
    force = torch.zeros((sph.n, 3), dtype=torch.float64, device=dev)
    sf, first, per = w.extra["subsample"], w.extra["first_cycles"], w.extra["cycles"]

    def run(n):
        for t in range(n):
            s.deposit(traj[t], r, q, w.eps, out=f, subsample=sf, mode=pkg.VOLUME)
            s.vcycles(phi, f, first if t == 0 else per, rels[t:t + 1])
            s.coulomb_force(phi, traj[t], r, q, subsample=sf, mode=pkg.VOLUME, out=force)

    run(warm)
    torch.cuda.synchronize()
    phi.zero_()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    run(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    secs = ev0.elapsed_time(ev1) / 1e3
    cycles = first + (steps - 1) * per
    rel = rels[:steps].cpu().numpy()
    # the two sphere kernels alone, same launches
    ev0.record(stream)
    for t in range(steps):
        s.deposit(traj[t], r, q, w.eps, out=f, subsample=sf, mode=pkg.VOLUME)
    ev1.record(stream)
    torch.cuda.synchronize()
    dep_ms = ev0.elapsed_time(ev1) / steps
    ev0.record(stream)
    for t in range(steps):
        s.coulomb_force(phi, traj[t], r, q, subsample=sf, mode=pkg.VOLUME, out=force)
    ev1.record(stream)
    torch.cuda.synchronize()
    force_ms = ev0.elapsed_time(ev1) / steps
    return {"workload": w.name, "cells": list(w.shape), "spheres": sph.n, "steps": steps, "cycles": cycles,
            "cycle": f"V({w.nu1},{w.nu2})", "levels": s.levels, "coarsest": list(s.level_dims(s.levels - 1)),
            "subsample": sf, "deposition": "volume (q/V per overlapped fraction)", "precision": "fp64",
            "ms_per_step": secs / steps * 1e3, "mlups": w.cells * steps / secs / 1e6,
            "deposit_ms_per_step": dep_ms, "force_ms_per_step": force_ms,
            "cell_cycles_per_s": w.cells * cycles / secs,
            "rel_res_step0": float(rel[0]), "rel_res_last": float(rel[-1]),
            "rel_res_max_later_steps": float(rel[1:].max()) if steps > 1 else None,
            "paper_context": {"mlups_per_node": 91.8, "hardware": "1 SuperMUC node (2x 8-core Xeon E5-2680)",
                              "note": "same scene size and cycle schedule; other machine: context, not a target"}}


def dielectric_spheres(w: W.Workload, sph, inside: float = 2.5, outside: float = 78.5) -> np.ndarray:
    """Cell permittivity: `inside` for cells whose centre lies in a sphere."""
    nx, ny, nz = w.shape
    eps = np.full((nz, ny, nx), outside)
    ax = [np.arange(n) + 0.5 for n in (nx, ny, nz)]
    for c, r in zip(sph.centers / w.h, sph.radii / w.h):
        lo = np.maximum(np.floor(c - r - 1).astype(int), 0)
        hi = np.minimum(np.ceil(c + r + 1).astype(int), [nx, ny, nz])
        Z, Y, X = np.meshgrid(ax[2][lo[2]:hi[2]], ax[1][lo[1]:hi[1]], ax[0][lo[0]:hi[0]], indexing="ij")
        inb = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2 <= r * r
        eps[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]][inb] = inside
    return eps


def variable_eps_solve(w: W.Workload, sph, sph_dev, dev, steps: int, warmup: int):
    """The same step (deposition, fold, solve to 1e-10 from zero) with the
    spheres as dielectric particles (eps 2.5 in a fluid of eps 78.5): stored
    Galerkin stencils instead of the closed-form operator."""
    eps = torch.tensor(dielectric_spheres(w, sph), device=dev)
    opt = pkg.Options(levels=w.levels, nu1=w.nu1, nu2=w.nu2, omega=w.omega, variable_eps=1)
    s = pkg.Solver(w.shape, w.h, list(zip(w.kinds, w.values)), opt, device=dev)
    s.set_permittivity(eps)
    f, phi = s.zeros(), s.zeros()
    run_steps(s, sph_dev, f, phi, w, warmup)
    t, wall, st = timed(s, sph_dev, f, phi, w, steps)
    return {"ms_per_step": t / steps * 1e3, "value": w.cells * steps / t, "unit": "unknowns/s",
            "cycles": st.cycles, "final_rel_res": st.rel_res,
            "permittivity": "2.5 inside the 200 spheres, 78.5 elsewhere (jump 31x)"}


def poisson_boltzmann(dev, steps: int, warmup: int, kappa: float = 0.25, charge_scale: float = 100.0):
    """The 256^3 workload's spheres as charged particles in an electrolyte
    (Poisson-Boltzmann, the equation the paper's outlook names): Debye length
    1/kappa = 4 cells, charges scaled so that the double layers reach a few
    thermal potentials.  The linearised (Debye-Hueckel) solve to 1e-10 in FP64
    and with FP32 refinement, and the nonlinear solve (shifted chord
    iteration, two V-cycles per step) to 1e-10, each from zero, timed."""
    w = W.C2
    sph = W.workload_spheres(w)
    c, r, q = (torch.tensor(a, device=dev) for a in (sph.centers, sph.radii, sph.charges))
    res = {"workload": w.name, "cells": list(w.shape), "spheres": w.n_spheres, "kappa": kappa,
           "debye_length_cells": 1.0 / kappa, "charge_scale": charge_scale,
           "equation": "-Lap(psi) + kappa^2 sinh(psi) = f (linear: kappa^2 psi)"}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed_runs(fn):
        for _ in range(warmup):
            out = fn()
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(steps):
            out = fn()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / steps, out

    for prec, key in ((pkg.FP64, "linear_fp64"), (pkg.FP32_IR, "linear_fp32_ir"), (pkg.FP64, "nonlinear_fp64")):
        opt = pkg.Options(levels=w.levels, nu1=w.nu1, nu2=w.nu2, omega=w.omega, precision=prec, kappa2=kappa ** 2)
        s = pkg.Solver(w.shape, w.h, list(zip(w.kinds, w.values)), opt, device=dev)
        f = s.zeros()
        s.deposit(c, r, q * charge_scale, w.eps, out=f)
        psi = s.zeros()
        if key.startswith("linear"):
            ms, (_, st) = timed_runs(lambda: s.solve(f, psi, rtol=w.rtol, zero_guess=True))
            res[key] = {"ms_per_solve": ms, "unknowns_per_s": w.cells / (ms * 1e-3), "cycles": st.cycles,
                        "final_rel_res": st.rel_res}
        else:
            def nl():
                psi.zero_()
                return s.solve_pb(f, psi, rtol=w.rtol, max_outer=300, inner=2)
            ms, (_, st) = timed_runs(nl)
            res[key] = {"ms_per_solve": ms, "unknowns_per_s": w.cells / (ms * 1e-3), "outer_steps": st.cycles,
                        "v_cycles": st.inner_cycles, "final_rel_res": st.rel_res,
                        "max_abs_psi": psi.abs().max().item()}
        del s
    return res


def forward_adjoint(dev, steps: int, warmup: int, weight_seed: int = 2005):
    """The microchannel workload (1024 x 256 x 256, 10,000 spheres, 7 levels)
    as a differentiable step: deposition, the forward solve from zero, then
    the adjoint solve of the loss L = sum_c w_c phi_c (w ~ N(0,1), seeded)
    with dL/dq per sphere; FP32 refinement against the plain FP64 solver."""
    w = W.C5
    sph = W.workload_spheres(w)
    c, r, q = (torch.tensor(a, device=dev) for a in (sph.centers, sph.radii, sph.charges))
    g = torch.tensor(W.random_field(w.shape, weight_seed), device=dev)
    stream = torch.cuda.current_stream()
    res, keep = {}, {}
    for prec, key in ((pkg.FP64, "fp64"), (pkg.FP32_IR, "fp32_ir")):
        s = make_solver(w, dev, precision=prec)
        f, phi, lam = s.zeros(), s.zeros(), s.zeros()

        def step():
            s.deposit(c, r, q, w.eps, out=f)
            _, st_f = s.solve(f, phi, rtol=w.rtol, max_cycles=100, zero_guess=True)
            _, dq, _, st_b = s.adjoint(g, c, r, w.eps, rtol=w.rtol, max_cycles=100, lam=lam)
            return st_f, st_b, dq

        for _ in range(warmup):
            step()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(steps):
            st_f, st_b, dq = step()
        ev[1].record(stream)
        torch.cuda.synchronize()
        t = ev[0].elapsed_time(ev[1]) / 1e3 / steps
        _, rel_f = s.residual(phi, f, want_field=False)
        res[key] = {"ms_per_step": t * 1e3, "solves_per_step": 2, "unknowns_per_s": 2 * w.cells / t,
                    "forward_cycles": st_f.cycles, "adjoint_cycles": st_b.cycles,
                    "forward_rel_res_fp64": rel_f, "adjoint_rel_res": st_b.rel_res}
        keep[key] = (phi.clone(), lam.clone(), dq.clone())
        del s, f, phi, lam
        torch.cuda.empty_cache()
    (p64, l64, d64), (p32, l32, d32) = keep["fp64"], keep["fp32_ir"]
    res["fp32_ir"]["speedup_vs_fp64"] = res["fp64"]["ms_per_step"] / res["fp32_ir"]["ms_per_step"]
    res["fp32_ir"]["max_abs_diff_phi_vs_fp64"] = (p32 - p64).abs().max().item()
    res["fp32_ir"]["max_abs_diff_lambda_vs_fp64"] = (l32 - l64).abs().max().item()
    res["fp32_ir"]["max_rel_diff_dq_vs_fp64"] = ((d32 - d64).abs().max() / d64.abs().max()).item()
    return {"workload": w.name, "cells": list(w.shape), "spheres": w.n_spheres, "levels": w.levels,
            "loss": "sum_c w_c phi_c, w ~ N(0,1) per cell (seeded)", **res}


def cpu_baseline_all_configs(dev, reps: int = 5):
    """The CPU-baseline leg for every workload: each solved from zero to 1e-10
    on the GPU (FP64 and FP32 refinement; deposition included for the sphere
    workloads) next to the FP64 oracle on the host's cores (all threads; also
    one thread for the three smaller workloads), with the GPU's largest
    difference from the oracle."""
    import oracle
    oracle.lib()
    threads = oracle.num_threads()
    rows = []
    for w in (W.C1, W.C2, W.C3, W.C4, W.C5):
        row = {"workload": w.name, "cells": list(w.shape), "levels": w.levels, "spheres": w.n_spheres}
        if w.n_spheres:
            sph = W.workload_spheres(w)
            sph_dev = tuple(torch.tensor(a, device=dev) for a in (sph.centers, sph.radii, sph.charges))
        else:
            f_host = W.sine_rhs(w.shape, w.h)
        phis = {}
        for prec, key in ((pkg.FP64, "gpu_fp64"), (pkg.FP32_IR, "gpu_fp32_ir")):
            s = make_solver(w, dev, precision=prec)
            f = s.zeros() if w.n_spheres else torch.tensor(f_host, device=dev)
            phi = s.zeros()

            def one():
                if w.n_spheres:
                    s.deposit(*sph_dev, w.eps, out=f)
                return s.solve(f, phi, rtol=w.rtol, max_cycles=100, zero_guess=True)[1]

            for _ in range(2):
                one()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            torch.cuda.synchronize()
            ev[0].record(torch.cuda.current_stream())
            for _ in range(reps):
                st = one()
            ev[1].record(torch.cuda.current_stream())
            torch.cuda.synchronize()
            t = ev[0].elapsed_time(ev[1]) / 1e3 / reps
            _, rel = s.residual(phi, f, want_field=False)
            row[key] = {"ms": t * 1e3, "unknowns_per_s": w.cells / t, "cycles": st.cycles,
                        "rel_res_fp64": rel}
            phis[key] = phi.cpu().numpy()
            del s, f, phi
            torch.cuda.empty_cache()
        for nthr in ([threads, 1] if w.cells <= 256 ** 3 else [threads]):
            oracle.set_num_threads(nthr)
            t0 = time.perf_counter()
            if w.n_spheres:
                f_cpu, _ = oracle.deposit(w.shape, w.h, sph.centers, sph.radii, sph.charges, w.eps)
            else:
                f_cpu = f_host
            ref, hist, _ = oracle.solve_problem(f_cpu, w.h, w.kinds, w.values, w.levels, rtol=w.rtol,
                                                nu1=w.nu1, nu2=w.nu2, omega=w.omega)
            t = time.perf_counter() - t0
            row[f"oracle_{nthr}_threads"] = {"s": t, "unknowns_per_s": w.cells / t, "cycles": len(hist) - 1}
        oracle.set_num_threads(threads)
        scale = float(np.abs(ref).max())
        row["max_abs_diff_vs_oracle"] = {k: float(np.abs(v - ref).max()) for k, v in phis.items()}
        row["max_abs_oracle_phi"] = scale
        rows.append(row)
        log(json.dumps(row))
        del phis, ref
    return {"cpu_threads": threads, **host_cpu(), "configs": rows}


def small_workload(w: W.Workload, dev, steps: int, warmup: int, inner: int):
    """Another workload's step (deposition, fold, solve from zero to 1e-10) in
    FP64 and with FP32 refinement, each timed over the same steps."""
    sph = W.workload_spheres(w)
    sph_dev = tuple(torch.tensor(a, device=dev) for a in (sph.centers, sph.radii, sph.charges))
    res = {"workload": w.name, "cells": list(w.shape), "spheres": w.n_spheres}
    keep = None
    for prec, key in ((pkg.FP64, "fp64"), (pkg.FP32_IR, "fp32_ir")):
        s = make_solver(w, dev, precision=prec, inner=inner)
        f, phi = s.zeros(), s.zeros()
        run_steps(s, sph_dev, f, phi, w, warmup)
        t, _, st = timed(s, sph_dev, f, phi, w, steps)
        res[key] = {"ms_per_step": t / steps * 1e3, "value": w.cells * steps / t, "unit": "unknowns/s",
                    "cycles": st.cycles, "final_rel_res": st.rel_res}
        if keep is None:
            keep = (s, f, phi)
        else:
            _, rel64 = keep[0].residual(phi, f, want_field=False)
            res[key]["final_rel_res_fp64"] = rel64
            res[key]["inner_fp32_cycles"] = st.inner_cycles
            res[key]["speedup_vs_fp64"] = res["fp64"]["ms_per_step"] / res[key]["ms_per_step"]
            res[key]["max_abs_diff_vs_fp64_solution"] = (phi - keep[2]).abs().max().item()
    return res


def single_thread_oracle():
    """The oracle on one host thread for the three smaller workloads (sine
    32^3, 256^3 spheres, 128^3 spheres): deposition, fold and solve to 1e-10."""
    import oracle
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    rows = {}
    try:
        for w in (W.C1, W.C2, W.C4):
            t0 = time.perf_counter()
            if w.n_spheres:
                sph = W.workload_spheres(w)
                f, _ = oracle.deposit(w.shape, w.h, sph.centers, sph.radii, sph.charges, w.eps)
            else:
                f = W.sine_rhs(w.shape, w.h)
            _, hist, _ = oracle.solve_problem(f, w.h, w.kinds, w.values, w.levels, rtol=w.rtol, nu1=w.nu1,
                                              nu2=w.nu2, omega=w.omega)
            t = time.perf_counter() - t0
            rows[w.name] = {"s": t, "unknowns_per_s": w.cells / t, "cycles": len(hist) - 1}
    finally:
        oracle.set_num_threads(threads)
    return {"threads": 1, "workloads": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=W.C3.name, choices=sorted(W.ALL))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-ir", action="store_true", help="skip the FP32-IR comparison")
    ap.add_argument("--fuse", type=int, default=2)
    ap.add_argument("--inner", type=int, default=4)
    ap.add_argument("--no-scene", action="store_true", help="skip the time-step scene")
    ap.add_argument("--no-c2", action="store_true", help="skip the 256^3 workload section")
    ap.add_argument("--no-vc", action="store_true", help="skip the variable-permittivity solve")
    ap.add_argument("--no-pb", action="store_true", help="skip the Poisson-Boltzmann solves")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the microchannel forward + adjoint step (FP64 and FP32 refinement)")
    ap.add_argument("--all-configs", action="store_true",
                    help="time every workload on the GPU next to the CPU oracle and print that JSON instead")
    ap.add_argument("--only", choices=("scene", "vc", "adjoint", "pb"), default=None,
                    help="run one secondary section alone and print its JSON object (for profiling runs)")
    ap.add_argument("--scene-steps", type=int, default=240)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain device copy of 1 GiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X (use --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    dev = torch.device("cuda:0")
    w = W.ALL[args.workload]
    sph = W.workload_spheres(w)
    sph_dev = tuple(torch.tensor(a, device=dev) for a in (sph.centers, sph.radii, sph.charges))
    if args.only == "scene":
        print(json.dumps({"timestep_scene": timestep_scene(dev, args.scene_steps)}), flush=True)
        return
    if args.all_configs:
        print(json.dumps(cpu_baseline_all_configs(dev)), flush=True)
        return
    if args.only == "adjoint":
        print(json.dumps({"forward_adjoint": forward_adjoint(dev, args.steps, args.warmup)}), flush=True)
        return
    if args.only == "pb":
        print(json.dumps({"poisson_boltzmann": poisson_boltzmann(dev, args.steps, args.warmup)}), flush=True)
        return
    if args.only == "vc":
        print(json.dumps({"variable_eps": variable_eps_solve(w, sph, sph_dev, dev, args.steps, args.warmup)}),
              flush=True)
        return
    nx, ny, nz = w.shape
    s = make_solver(w, dev, fuse=args.fuse)
    f = s.zeros()
    phi = s.zeros()
    log(f"workload {w.name}: {w.shape} levels={s.levels} ws={s.workspace.numel() / 2**20:.0f} MiB")

    run_steps(s, sph_dev, f, phi, w, args.warmup)
    if args.calib_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # headline: the timed steps carry no instrumentation
    t_gpu, wall, st = timed(s, sph_dev, f, phi, w, args.steps)
    ms_step = t_gpu / args.steps * 1e3
    value = w.cells * args.steps / t_gpu
    log(f"fp64: {ms_step:.3f} ms/step, {st.cycles} cycles, rel {st.rel_res:.2e}, wall {wall:.3f}s")
    # the same steps again with every finest-level pass bracketed by HIP events
    # on the solver's stream: per-launch durations of the dominant kernel
    s.profile(True)
    s.profile_read(0)
    s.profile_read(1)
    t_prof, _, _ = timed(s, sph_dev, f, phi, w, args.steps)
    ms0, n0 = s.profile_read(0)
    ms1, n1 = s.profile_read(1)
    s.profile(False)

    # roofline of the dominant kernel: the finest-level fused pass with the
    # larger total time.  Algorithmic bytes per launch in two units: the
    # per-sweep unit (every red-black sweep reads phi and b and writes phi,
    # 24 B per cell, plus 1 B per cell for the fused grid transfer: 49 B for
    # the two sweeps of one launch) and the fused pass's own floor (phi and b
    # read once, phi written once, plus the transfer: 25 B)
    cells = w.cells
    passes = [
        ("pre", "pre-smoothing pass (2 RB-GS sweeps + residual + restriction), finest level", ms0, n0,
         8 + 8 + 8 + 1),
        ("post", "post-smoothing pass (prolongation + 2 RB-GS sweeps + residual norm), finest level", ms1, n1,
         8 + 1 + 8 + 8),
    ]
    which, name, ms_k, n_k, bpc = max(passes, key=lambda p: p[2])
    avg_s = ms_k / max(n_k, 1) / 1e3
    unit_bpc = 2 * 24 + 1
    achieved = unit_bpc * cells / avg_s / 1e9
    fused = bpc * cells / avg_s / 1e9
    hbm = measured_traffic(w.name, which)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if hbm is None else round(hbm / avg_s / 1e9, 1),
                "kernel": name, "avg_launch_us": round(avg_s * 1e6, 2), "launches": n_k,
                "units": {"frac": f"per-sweep unit: 2 sweeps x 24 B + 1 B transfer = {unit_bpc} B per cell "
                                  "per launch (exceeds 1 when the fused pass beats separate sweeps)",
                          "frac_fused_floor": f"the fused pass's own floor: {bpc} B per cell per launch "
                                              "(phi and b read once, phi written once, 1 B transfer)",
                          "traffic": "counted HBM bytes per launch (copy-calibrated FETCH_SIZE + WRITE_SIZE) "
                                     "/ average launch time"},
                "frac_fused_floor": round(fused / HBM_PEAK_GBS, 4), "achieved_fused_floor": round(fused, 1),
                "algorithmic_bytes_per_launch": unit_bpc * cells,
                "fused_floor_bytes_per_launch": bpc * cells,
                "hbm_bytes_per_launch": hbm,
                "hbm_bytes_over_fused_floor": None if hbm is None else round(hbm / (bpc * cells), 3)}
    other = [p for p in passes if p[0] != which][0]
    o_s = other[2] / max(other[3], 1) / 1e3
    hbm_o = measured_traffic(w.name, other[0])
    roofline["other_pass"] = {"kernel": other[1], "avg_launch_us": round(o_s * 1e6, 2),
                              "frac": round(unit_bpc * cells / o_s / 1e9 / HBM_PEAK_GBS, 4),
                              "frac_fused_floor": round(other[4] * cells / o_s / 1e9 / HBM_PEAK_GBS, 4),
                              "traffic": None if hbm_o is None else round(hbm_o / o_s / 1e9, 1),
                              "hbm_bytes_over_fused_floor": None if hbm_o is None
                              else round(hbm_o / (other[4] * cells), 3)}
    roofline["finest_passes_share_of_step"] = round((ms0 + ms1) / (t_prof * 1e3), 4)

    # solve-level fraction: bytes per V(2,2)-cycle over the whole hierarchy
    # (coarse levels add 1/7) x cycles / (solve time x peak), counted two ways:
    # the per-sweep floor (4 x 24 + 2 = 98 B) and the fused design's own floor
    # (two passes of 25 B)
    t_solve = t_gpu / args.steps
    solve_level = {}
    for key, per_cell in (("per_sweep_floor", 98), ("fused_passes", 50)):
        b = per_cell * 8 / 7 * cells * st.cycles
        solve_level[key] = {"bytes_per_cell_per_cycle": round(per_cell * 8 / 7, 1),
                            "effective_GBs": round(b / t_solve / 1e9, 1),
                            "frac": round(b / t_solve / 1e9 / HBM_PEAK_GBS, 4)}
    roofline["solve_level"] = solve_level

    out = {
        "metric": "fine-grid unknowns solved/s to 1e-10 rel. residual",
        "value": value,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded charged spheres)",
        "config": {"workload": w.name, "cells": [nx, ny, nz], "levels": s.levels, "cycle": "V(2,2)",
                   "omega": w.omega,
                   "coarsest": list(s.level_dims(s.levels - 1)), "rtol": w.rtol, "spheres": w.n_spheres,
                   "precision": "fp64", "fused_sweeps_per_pass": args.fuse},
        "cycles": st.cycles,
        "final_rel_res": st.rel_res,
        "roofline": roofline,
    }

    if not args.no_ir:
        s32 = make_solver(w, dev, precision=pkg.FP32_IR, fuse=args.fuse, inner=args.inner)
        phi32 = s32.zeros()
        run_steps(s32, sph_dev, f, phi32, w, args.warmup)
        t32, wall32, st32 = timed(s32, sph_dev, f, phi32, w, args.steps)
        _, rel64 = s.residual(phi32, f, want_field=False)
        diff = (phi32 - phi).abs().max().item()
        out["fp32_ir"] = {"value": w.cells * args.steps / t32, "ms_per_step": t32 / args.steps * 1e3,
                          "speedup_vs_fp64": t_gpu / t32, "outer_steps": st32.cycles,
                          "inner_fp32_cycles": st32.inner_cycles, "final_rel_res_fp64": rel64,
                          "max_abs_diff_vs_fp64_solution": diff}
        log(f"fp32-ir: {t32 / args.steps * 1e3:.3f} ms/step, {st32.cycles} outer, rel {rel64:.2e}, "
            f"max|dphi| vs fp64 {diff:.2e}")
        del s32, phi32

    # the same step with the correction factor 2 (the library default; the
    # workloads take 1.95, which saves a cycle): its cycle count and time
    w2 = dataclasses.replace(w, omega=2.0)
    s2 = make_solver(w2, dev, fuse=args.fuse, inner=args.inner)
    phi2 = s2.zeros()
    run_steps(s2, sph_dev, f, phi2, w2, 1)
    n2 = max(1, min(args.steps, 5))
    t2, _, st2 = timed(s2, sph_dev, f, phi2, w2, n2)
    out["omega_2"] = {"cycles": st2.cycles, "ms_per_step": t2 / n2 * 1e3, "value": w.cells * n2 / t2,
                      "final_rel_res": st2.rel_res}
    log(f"omega 2: {t2 / n2 * 1e3:.3f} ms/step, {st2.cycles} cycles")
    del s2, phi2

    if w.name != W.C2.name and not args.no_c2:
        del s
        torch.cuda.empty_cache()
        out["c2_spheres_256"] = c2 = small_workload(W.C2, dev, args.steps, args.warmup, args.inner)
        log(f"256^3: fp64 {c2['fp64']['ms_per_step']:.3f} ms, fp32-ir {c2['fp32_ir']['ms_per_step']:.3f} ms per step")

    if not args.no_vc:
        wv = W.C2
        sph_v = W.workload_spheres(wv)
        sph_vd = tuple(torch.tensor(a, device=dev) for a in (sph_v.centers, sph_v.radii, sph_v.charges))
        out["variable_eps"] = vc = variable_eps_solve(wv, sph_v, sph_vd, dev, max(1, args.steps // 2), 1)
        log(f"variable eps: {vc['ms_per_step']:.3f} ms/step, {vc['cycles']} cycles, rel {vc['final_rel_res']:.2e}")

    if not args.no_pb:
        out["poisson_boltzmann"] = pb = poisson_boltzmann(dev, max(1, args.steps // 4), 1)
        log(f"poisson-boltzmann 256^3: linear {pb['linear_fp64']['ms_per_solve']:.2f} ms "
            f"({pb['linear_fp64']['cycles']} cycles), fp32-ir {pb['linear_fp32_ir']['ms_per_solve']:.2f} ms, "
            f"nonlinear {pb['nonlinear_fp64']['ms_per_solve']:.2f} ms ({pb['nonlinear_fp64']['outer_steps']} steps, "
            f"max|psi| {pb['nonlinear_fp64']['max_abs_psi']:.2f})")

    if not args.no_adjoint:
        out["forward_adjoint"] = fa = forward_adjoint(dev, max(1, args.steps // 4), 1)
        log(f"forward + adjoint ({fa['workload']}): fp64 {fa['fp64']['ms_per_step']:.2f} ms, "
            f"fp32-ir {fa['fp32_ir']['ms_per_step']:.2f} ms per step")

    if not args.no_scene:
        s = None
        torch.cuda.empty_cache()
        out["timestep_scene"] = ts = timestep_scene(dev, args.scene_steps)
        log(f"time-step scene: {ts['ms_per_step']:.3f} ms/step, {ts['mlups']:.0f} MLUPS, "
            f"rel res last {ts['rel_res_last']:.2e}, max later {ts['rel_res_max_later_steps']:.2e}")

    if not args.no_cpu:
        base, phi_cpu = cpu_baseline(w, sph)
        base["max_abs_diff_gpu_vs_oracle"] = float(np.abs(phi.cpu().numpy() - phi_cpu).max())
        base["single_thread"] = single_thread_oracle()
        out["cpu_baseline"] = base
        log(f"cpu oracle: {base['seconds_per_solve']:.2f} s/solve on {base['cores']} threads")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
