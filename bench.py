"""Benchmark of the AGCA multigrid hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sinker129]

Workload (default): the vector viscous block -div(2 nu eps(u)) = f on 129^3
nodes (7 levels), 8 tanh-smoothed sinkers of radius 0.1, contrast 1e6,
f = (0, 0, -xi); synthetic inputs from the seeded generators in workloads/.

One step = one pass over the whole hot path for the resident coefficient:
  1. rebuild both hierarchies from the resident coefficients (flags, Galerkin
     blocks of flagged elements, diagonals, coarsest inverse),
  2. a batch of fine-grid operator applications v = A_L u (FP64),
  3. an FP64 solve to 1e-8 with the FP64 AGCA V-cycle (PCG),
  4. a solve to 1e-8 with the FP32 V-cycle and BF16 finest coefficient inside
     FP64 flexible CG.
Printed metric: fine-grid apply throughput in GDoF/s (free DoFs / average
duration of the FP64 apply kernel, HIP events on the library's stream), plus
the two times to 1e-8, the roofline of that kernel and the CPU oracle baseline.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GDoF/s fine-grid apply; time-to-1e-8 residual, FP32-MG vs FP64-MG"


def apply_bytes(L: int, ncomp: int, vec_bytes: int = 8, nu_bytes: int = 8) -> int:
    """Algorithmic bytes of one fine apply: read u, write v (all (n+1)^3 slots), read nu."""
    n = 2 ** (L + 1)
    return 2 * ncomp * vec_bytes * (n + 1) ** 3 + nu_bytes * 6 * n ** 3


def make_inputs(name: str):
    from paper_2511_13109_amd.grid import element_centroids
    from workloads import workload
    w = workload(name)
    field = w.make_field()
    t0 = time.perf_counter()
    nu = [np.ascontiguousarray(field.nu(element_centroids(l))) for l in range(w.L + 1)]
    f = field.force(element_centroids(w.L), w.ncomp)
    f = np.ascontiguousarray(np.asarray(f).reshape(nu[-1].size, -1).T)
    return w, nu, f, time.perf_counter() - t0


def cpu_baseline(name: str, L_sample: int = 4, seconds: float = 12.0) -> dict:
    """The oracle's FP64 CSR operator apply on a bounded sample of the same workload."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from oracle import fem, mesh
    from workloads import workload
    w = workload(name)
    field = w.make_field()          # same seeded field (same sinkers and tanh width)
    levels = mesh.hierarchy(L_sample)
    lv = levels[L_sample]
    nu = field.nu(mesh.centroids_canonical(lv))
    t0 = time.perf_counter()
    A = fem.restrict_free(fem.assemble(lv, nu, w.ncomp), fem.free_dofs(lv, w.ncomp))
    t_asm = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    u = rng.standard_normal(A.shape[0])
    reps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        A @ u
        reps += 1
    dt = (time.perf_counter() - t0) / reps
    return {"value": A.shape[0] / dt / 1e9, "unit": "GDoF/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle CSR apply (scipy, single-threaded) of the {w.ncomp}-component "
                      f"operator of the same coefficient field on {lv.n + 1}^3 nodes "
                      f"({A.shape[0]} free DoFs), {reps} applications over {seconds:.0f} s; "
                      f"assembly ({t_asm:.1f} s) excluded"}


def profile_apply(name: str, dev) -> None:
    """Driver for hardware-counter passes: 5 FP64 fine applies, then a 256 MiB copy
    (three times) whose known size calibrates the byte counters."""
    import torch
    from paper_2511_13109_amd import Hierarchy
    w, nu, _, _ = make_inputs(name)
    nus = [torch.from_numpy(v).to(dev) for v in nu]
    H = Hierarchy(w.L, w.ncomp, nus[w.L], nus[:w.L], mg_dtype="f64")
    n = 2 ** (w.L + 1)
    u = torch.randn(w.ncomp * (n + 1) ** 3, dtype=torch.float64, device=dev)
    v = torch.empty_like(u)
    for _ in range(5):
        H.apply(w.L, u, v)
    a = torch.empty(256 * 1024 * 1024 // 8, dtype=torch.float64, device=dev).normal_()
    c = torch.empty_like(a)
    for _ in range(3):
        c.copy_(a)
    torch.cuda.synchronize()
    H.close()
    print("profile-apply done", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sinker129")
    ap.add_argument("--applies", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mg-nu", default="bf16", choices=["bf16", "f32"])
    ap.add_argument("--profile-apply", action="store_true",
                    help="only run 5 FP64 fine applies and a 256 MiB copy (counter passes)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the AGCA path here is built and timed on a single "
              "MI355X (multi-GPU sharding is a design note, not an implemented path).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2511_13109_amd import Hierarchy

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.profile_apply:
        profile_apply(args.workload, dev)
        return
    w, nu, f, t_gen = make_inputs(args.workload)
    L, nc = w.L, w.ncomp
    nus = [torch.from_numpy(v).to(dev) for v in nu]
    f_dev = torch.from_numpy(f.ravel()).to(dev)
    H64 = Hierarchy(L, nc, nus[L], nus[:L], mg_dtype="f64")
    H32 = Hierarchy(L, nc, nus[L], nus[:L], mg_dtype="f32", mg_nu_dtype=args.mg_nu)
    b = H64.load_vector(f_dev)
    gen = torch.Generator(device="cpu").manual_seed(0)
    n = 2 ** (L + 1)
    N = (n + 1) ** 3
    free_dofs = nc * (n - 1) ** 3
    u = torch.randn(nc * N, generator=gen, dtype=torch.float64).to(dev)
    v = torch.empty_like(u)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    rec = {"apply_ms": [], "setup_s": [], "t64": [], "t32": [], "it64": [], "it32": [],
           "res64": [], "res32": []}

    def step(record: bool):
        t0 = time.perf_counter()
        H64.set_nu(nus[L], nus[:L])
        H32.set_nu(nus[L], nus[:L])
        t_setup = time.perf_counter() - t0
        ev[0].record()
        for _ in range(args.applies):
            H64.apply(L, u, v)
        ev[1].record()
        x64, s64 = H64.solve(b, solver="pcg", tol=w.tol, max_iter=4000, raise_on_noconv=False)
        x32, s32 = H32.solve(b, solver="fcg", tol=w.tol, max_iter=4000, raise_on_noconv=False)
        if record:
            torch.cuda.synchronize()
            rec["apply_ms"].append(ev[0].elapsed_time(ev[1]) / args.applies)
            rec["setup_s"].append(t_setup)
            rec["t64"].append(s64["seconds"])
            rec["t32"].append(s32["seconds"])
            rec["it64"].append(s64["iterations"])
            rec["it32"].append(s32["iterations"])
            rec["res64"].append(s64["rel_residual"])
            rec["res32"].append(s32["rel_residual"])
            rec.setdefault("stat64", []).append({k: s64[k] for k in ("converged", "floor_limited",
                                                 "replacements", "recursive_rel_residual")})
            rec.setdefault("stat32", []).append({k: s32[k] for k in ("converged", "floor_limited",
                                                 "replacements", "recursive_rel_residual")})
            print(f"[step] setup {t_setup*1e3:.1f} ms, apply {rec['apply_ms'][-1]*1e3:.1f} us, "
                  f"FP64-MG PCG {s64['iterations']} it {s64['seconds']*1e3:.1f} ms "
                  f"(res {s64['rel_residual']:.2e}), FP32-MG FCG {s32['iterations']} it "
                  f"{s32['seconds']*1e3:.1f} ms (res {s32['rel_residual']:.2e})",
                  file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    apply_s = float(np.mean(rec["apply_ms"])) / 1e3
    value = free_dofs / apply_s / 1e9
    bytes_launch = apply_bytes(L, nc)
    achieved = bytes_launch / apply_s / 1e9
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "GDoF/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.description}", "levels": L + 1, "nodes": N,
                   "free_dofs": free_dofs, "elements": 6 * n ** 3, "applies_per_step": args.applies},
        "time_to_1e-8_s": {"fp64_mg_pcg": round(float(np.median(rec["t64"])), 5),
                           "fp32_mg_fcg": round(float(np.median(rec["t32"])), 5),
                           "mg_nu_dtype": args.mg_nu,
                           "speedup_fp32_over_fp64": round(float(np.median(rec["t64"]) /
                                                                 np.median(rec["t32"])), 3)},
        "iterations": {"fp64_mg_pcg": int(np.median(rec["it64"])), "fp32_mg_fcg": int(np.median(rec["it32"]))},
        "final_rel_residual_fp64": {"fp64_mg": max(rec["res64"]), "fp32_mg": max(rec["res32"])},
        "solve_status": {"fp64_mg": rec["stat64"][-1], "fp32_mg": rec["stat32"][-1]},
        "setup_s": round(float(np.median(rec["setup_s"])), 5),
        "flagged_per_level": [H64.query(l)["flagged"] for l in range(L)],
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_cube<3,double,double,APPLY> (fine-grid apply)",
                     "bytes_per_launch": bytes_launch, "avg_launch_us": round(apply_s * 1e6, 2)},
        "input_generation_s": round(t_gen, 2),
    }
    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(args.workload)
        except Exception as exc:  # the baseline is a report, never a reason to lose the line
            out["cpu_baseline"] = {"error": repr(exc)}
    H64.close()
    H32.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
