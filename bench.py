"""Benchmark of the AGCA multigrid hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
    python bench.py --workload sinker129            (the earlier 129^3 benchmark line)
    python bench.py --workload stokes257|adjoint129|coarsening|roofline [--level L]
                                                            (report lines)

Workload (default, sinker513): the vector viscous block -div(2 nu eps(u)) = f on
513^3 nodes (9 levels, 400,298,493 free DoFs), 64 tanh-smoothed sinkers with radii
in [0.02, 0.06] (seed 5), contrast 1e6, f = (0, 0, -xi); inputs generated on the
device from the seeded generators in workloads/ and resident in HBM before timing.

One step = one pass over the hot path for the resident coefficient:
  1. rebuild both hierarchies (FP64 multigrid; FP32 multigrid with the BF16 finest
     coefficient) from the resident coefficients: flags, Galerkin blocks of flagged
     elements, diagonals, coarsest inverse, spectral bounds of the Chebyshev smoother,
  2. a batch of fine-grid operator applications v = A_L u (FP64), each timed with
     HIP events on the library's stream after a 512 MiB read (cold caches),
  3. one FP64 and one FP32 V(2,2)-cycle (degree-2 Chebyshev smoother of Section 4).
After the timed steps, once: FP64-MG PCG and FP32/BF16-MG FCG (FP64 outer loop) on
A_L x = b to tol 1e-8, each recording when its verified true residual first fell
below 1e-5, 1e-6 and 1e-7, with its final residual and the rounding floor rho of
its iterate; then the 129^3 sinker workload's apply and solves as extra keys.
Printed metric: fine-grid apply throughput in GDoF/s (free DoFs / average duration
of the FP64 apply kernel), plus times to tolerance, the roofline of that kernel and
the CPU oracle baseline.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GDoF/s fine-grid apply; time-to-1e-8 residual, FP32-MG vs FP64-MG"
PROFILES = {"sinker513": os.path.join(ROOT, "profiles", "fine_apply_sinker513.md"),
            "sinker129": os.path.join(ROOT, "profiles", "fine_apply_sinker129.md")}
MILESTONES = (1e-5, 1e-6, 1e-7)
# sources whose text determines the fine-apply kernel; counter traffic is only
# reported while their hash equals the one recorded next to the counters
KERNEL_SOURCES = ["paper_2511_13109_amd/csrc/k_apply.hip", "paper_2511_13109_amd/csrc/kuhn.h",
                  "paper_2511_13109_amd/csrc/cube_math.h"]
FINE_APPLY_KERNEL = "k_cube<3, double, double, 0, false>"


def apply_bytes(L: int, ncomp: int, vec_bytes: int = 8, nu_bytes: int = 8) -> int:
    """Algorithmic bytes of one fine apply: read u, write v (all (n+1)^3 slots), read nu."""
    n = 2 ** (L + 1)
    return 2 * ncomp * vec_bytes * (n + 1) ** 3 + nu_bytes * 6 * n ** 3


def kernel_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload: str):
    """HBM bytes per fine-apply launch from the committed counter summary of a workload, or
    None when there is none or the kernel sources changed after the counters were taken."""
    try:
        text = open(PROFILES[workload]).read()
    except (OSError, KeyError):
        return None
    mt = re.search(r"^traffic_bytes_per_launch: (\d+)$", text, re.M)
    mh = re.search(r"^kernel_source_sha256_16: ([0-9a-f]+)$", text, re.M)
    if not mt or not mh or mh.group(1) != kernel_hash():
        return None
    return int(mt.group(1))


def _short(name: str) -> str:
    name = name.replace("void ", "").replace("agca::(anonymous namespace)::", "")
    depth, out = 0, []
    for ch in name:                     # drop the argument list, keep template arguments
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out)


# algorithmic bytes of the solver's finest-level kernels (vector problem): bytes per node
# of the ncomp-vectors read or written, and bytes per cell of the finest coefficient
def _vec(vb: int, nvec: int, nc: int = 3) -> int:
    return nvec * nc * vb


SOLVER_KERNEL_BYTES = {
    # k_cube<ncomp, vector type, coefficient type, mode, blocks>: mode 0 apply (u in, v out),
    # 1 residual (+b), 2 Jacobi-type pass (u, b, D^-1 in, out), 3 apply + dot, 4 first two
    # passes from zero (b, D^-1 in, out), 5 Chebyshev pass (+ previous iterate)
    "k_cube<3, double, double, 0, false>": ("apply", _vec(8, 2), 48),
    "k_cube<3, double, double, 1, false>": ("residual", _vec(8, 3), 48),
    "k_cube<3, double, double, 2, false>": ("Jacobi-type pass", _vec(8, 4), 48),
    "k_cube<3, double, double, 3, false>": ("apply + p.Ap", _vec(8, 2), 48),
    "k_cube<3, double, double, 4, false>": ("first two passes", _vec(8, 3), 48),
    "k_cube<3, double, double, 5, false>": ("Chebyshev pass", _vec(8, 5), 48),
    "k_cube<3, float, unsigned short, 1, false>": ("FP32/BF16 residual", _vec(4, 3), 12),
    "k_cube<3, float, unsigned short, 2, false>": ("FP32/BF16 Jacobi-type pass", _vec(4, 4), 12),
    "k_cube<3, float, unsigned short, 4, false>": ("FP32/BF16 first two passes", _vec(4, 3), 12),
    "k_cube<3, float, unsigned short, 5, false>": ("FP32/BF16 Chebyshev pass", _vec(4, 5), 12),
    "k_cg_update": ("x += a p, r -= a q, r.r (mixed: + FP32 r)", 3 * 6 * 8, 0),
    "k_dot2<double>": ("z.r, z.q (PCG)", 3 * 24, 0),
    "k_dot2<float>": ("z.r, z.q (FCG, FP32 z)", 3 * 20, 0),
    "k_zpbp_dev<double>": ("p = z + beta p", 3 * 24, 0),
    "k_zpbp_dev<float>": ("p = z + beta p (FP32 z)", 3 * 20, 0),
    # per fine node; the coarse vector (1/8 of the nodes) is added below
    "k_restrict<3, double>": ("restriction to the next coarser level", 3 * 8, 0),
    "k_restrict<3, float>": ("restriction to the next coarser level, FP32", 3 * 4, 0),
    "k_prolong_add<3, double>": ("prolongation from the next coarser level", 3 * 16, 0),
    "k_prolong_add<3, float>": ("prolongation from the next coarser level, FP32", 3 * 8, 0),
    "k_floor_terms<3>": ("rounding floor terms (|b| + sum |A_e||x_e|)", 3 * 16, 48),
}


def summarize_trace(path: str, L: int = 6) -> str:
    """Markdown table of the finest-level solver kernels in a rocprofv3 kernel trace of one
    bench step: for every kernel its launches on the finest level (the launch grid with
    the longest average duration: every level has its own grid), their average
    duration, the algorithmic bytes per launch and the rate."""
    import csv
    import collections
    n = 2 ** (L + 1)
    nodes = (n + 1) ** 3
    groups = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        k = _short(r["Kernel_Name"])
        if k in SOLVER_KERNEL_BYTES:
            grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            groups[k].append((grid, int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    lines = ["| kernel | what | launches | avg us | MB per launch | GB/s | of 8 TB/s |",
             "|---|---|---|---|---|---|---|"]
    nc1 = (n // 2 + 1) ** 3
    for k, (what, per_node, per_cell) in SOLVER_KERNEL_BYTES.items():
        if k not in groups:
            continue
        by_grid = collections.defaultdict(list)
        for g, d in groups[k]:
            by_grid[g].append(d)
        ds = max(by_grid.values(), key=lambda v: float(np.mean(v)))
        us = float(np.mean(ds)) / 1e3
        coarse = (per_node // 2 if "prolong" in k else per_node) * nc1 if "restrict" in k or "prolong" in k else 0
        mb = (per_node * nodes + per_cell * n ** 3 + coarse) / 1e6
        gbs = mb * 1e6 / (us * 1e-6) / 1e9
        lines.append(f"| `{k}` | {what} | {len(ds)} | {us:.2f} | {mb:.1f} | {gbs:.0f} | "
                     f"{gbs / HBM_PEAK_GBS:.3f} |")
    return "\n".join(lines)


def summarize_profile(d: str, command_prefix: str) -> str:
    """Markdown summary of a profiling directory written by the three rocprofv3 runs
    named in the text (kernel statistics of the bench command, FETCH_SIZE pass,
    WRITE_SIZE pass); the workload is the one of the bench line in <dir>/bench.json."""
    import csv
    lines = []
    stats = list(csv.DictReader(open(os.path.join(d, "stats", "bench_kernel_stats.csv"))))
    total = sum(float(r["TotalDurationNs"]) for r in stats)
    bench = json.loads(open(os.path.join(d, "bench.json")).read().strip().splitlines()[-1])
    L = bench["config"]["levels"] - 1
    n = 2 ** (L + 1)
    name = bench["config"]["workload"].split(":")[0]
    bytes_launch = apply_bytes(L, 3)
    lines += [f"# Fine-grid apply and solve kernels, vector viscous block on {n + 1}^3 nodes ({name})",
              "",
              "All commands run from /tmp after `cd /tmp && export TMPDIR=/tmp`, with the repository "
              "at `$R`; this file is written by `python3 bench.py --summarize-profile <dir>`.",
              "",
              "## Kernel statistics of the bench command",
              "",
              f"    {command_prefix}rocprofv3 --kernel-trace --stats --output-format csv -d <dir>/stats "
              "-o bench -- python3 $R/bench.py --steps 2 --warmup 1 --no-cpu-baseline > <dir>/bench.json",
              "",
              f"Total kernel time {total / 1e6:.1f} ms (hierarchy rebuilds, cold FP64 applies and "
              "V-cycles of 3 steps, the FP64-MG PCG and FP32-MG FCG solves, the 129^3 extra keys).  "
              "k_cube template arguments: <components, vector type, coefficient type, mode (0 apply, "
              "1 residual, 2 Jacobi-type pass, 3 apply with dot, 4 first two passes from zero, "
              "5 Chebyshev pass), stored blocks>.",
              "",
              "| kernel | calls | avg us | total ms | % |",
              "|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:24]:
        lines.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |")

    def counter(kind):
        rows = list(csv.DictReader(open(os.path.join(d, kind, "run_counter_collection.csv"))))
        app = [float(r["Counter_Value"]) for r in rows if _short(r["Kernel_Name"]) == FINE_APPLY_KERNEL]
        cp = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]
              and int(r["Grid_Size"]) >= 65536]
        cpd = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows
               if "copyBuffer" in r["Kernel_Name"] and int(r["Grid_Size"]) >= 65536]
        return app[1:] or app, cp, cpd
    fa, fc, cpd = counter("fetch")
    wa, wc, _ = counter("write")
    copy_kib = 256 * 1024
    ff = copy_kib / float(np.median(fc))
    fw = copy_kib / float(np.median(wc))
    read_b = float(np.median(fa)) * ff * 1024
    write_b = float(np.median(wa)) * fw * 1024
    traffic = int(round(read_b + write_b))
    copy_rate = 2 * copy_kib * 1024 / (float(np.median(cpd)) * 1e-9) / 1e9
    ro = bench["roofline"]
    fine = [r for r in stats if _short(r["Name"]) == FINE_APPLY_KERNEL]
    # launches on the finest level only (the coarse element-loop levels use the same kernel)
    tr_path = os.path.join(d, "stats", "fine_apply_trace.csv")
    fine_us = None
    rows = list(csv.DictReader(open(tr_path))) if os.path.exists(tr_path) else []
    if rows:
        big = max(int(r["Grid_Size_X"]) for r in rows)
        ds = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows
              if int(r["Grid_Size_X"]) == big]
        fine_us = (len(ds), float(np.mean(ds)) / 1e3)
    if fine:
        lines += ["", f"Fine apply `{FINE_APPLY_KERNEL}`: {fine[0]['Calls']} calls on all levels, "
                      f"rocprofv3 average {float(fine[0]['AverageNs']) / 1e3:.2f} us."]
    if fine_us:
        lines += [f"On the finest level ({n + 1}^3 nodes): {fine_us[0]} launches, rocprofv3 average "
                  f"{fine_us[1]:.1f} us; HIP events in the same run's bench line: {ro['avg_launch_us']} us."]
    lines += ["",
              f"## HBM traffic of the FP64 fine-grid apply (`{FINE_APPLY_KERNEL}`), {n + 1}^3 nodes",
              "",
              "Two counter passes, each in a run of its own; the driver builds the hierarchy, runs 5 "
              "FP64 fine applies, then copies a 256 MiB tensor three times to calibrate the counters:",
              "",
              f"    {command_prefix}rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/fetch -o run "
              f"-- python3 $R/bench.py --profile-apply --workload {name}",
              f"    {command_prefix}rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/write -o run "
              f"-- python3 $R/bench.py --profile-apply --workload {name}",
              "",
              f"* calibration (256 MiB copy): FETCH_SIZE reads {np.median(fc):.0f} KiB -> factor {ff:.3f}; "
              f"WRITE_SIZE reads {np.median(wc):.0f} KiB -> factor {fw:.3f}",
              f"* copy kernel rate in the counter run: {copy_rate:.0f} GB/s (read + write)",
              f"* apply (median of the dispatches after the first): FETCH_SIZE {np.median(fa):.0f} KiB, "
              f"WRITE_SIZE {np.median(wa):.0f} KiB",
              f"* scaled traffic per launch: read {read_b / 1e6:.1f} MB + write {write_b / 1e6:.1f} MB "
              f"= {traffic / 1e6:.1f} MB",
              f"* algorithmic bytes per launch: {bytes_launch / 1e6:.1f} MB (u and v: 3 x 8 B x {n + 1}^3 "
              f"each; nu: 8 B x 6 x {n}^3) -> traffic / algorithmic = {traffic / bytes_launch:.3f}",
              "",
              "## Bench line of the profiled run",
              "",
              f"* fine apply: {ro['avg_launch_us']} us per launch (HIP events), {ro['achieved']} GB/s "
              f"= {ro['frac']:.3f} of 8000 GB/s; {bench['value']} GDoF/s",
              "",
              f"traffic_bytes_per_launch: {traffic}",
              f"kernel_source_sha256_16: {ro.get('kernel_source_sha256_16', '(not recorded)')}",
              ""]
    return "\n".join(lines)


def make_inputs(name: str):
    from workloads.lattice import element_centroids
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
    # the oracle's multigrid set-up (assembly of every level, global Galerkin products,
    # flags, Chebyshev spectral bounds) and one V(2,2)-cycle on the same sample
    from oracle import mg
    nus = [field.nu(mesh.centroids_canonical(l)) for l in levels]
    t0 = time.perf_counter()
    H = mg.build(L_sample, nus, w.ncomp, levels=levels, smoother="chebyshev")
    t_setup = time.perf_counter() - t0
    b = rng.standard_normal(A.shape[0])
    mg.vcycle(H, b)
    t0 = time.perf_counter()
    for _ in range(3):
        mg.vcycle(H, b)
    t_vc = (time.perf_counter() - t0) / 3
    return {"value": A.shape[0] / dt / 1e9, "unit": "GDoF/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle CSR apply (scipy, single-threaded) of the {w.ncomp}-component "
                      f"operator of the same coefficient field on {lv.n + 1}^3 nodes "
                      f"({A.shape[0]} free DoFs), {reps} applications over {seconds:.0f} s; "
                      f"assembly ({t_asm:.1f} s) excluded; on the same sample the oracle's "
                      f"multigrid set-up takes {t_setup:.1f} s and one V(2,2)-cycle (Chebyshev) "
                      f"{t_vc * 1e3:.1f} ms",
            "oracle_setup_s": round(t_setup, 2), "oracle_vcycle_s": round(t_vc, 4),
            "sample_free_dofs": int(A.shape[0])}


def profile_apply(name: str, dev) -> None:
    """Driver for hardware-counter passes: 5 FP64 fine applies, then a 256 MiB copy
    (three times) whose known size calibrates the byte counters."""
    import torch
    from paper_2511_13109_amd import Hierarchy
    if name == "sinker513":     # 805 million elements: generated on the device
        from workloads import workload
        from workloads.device import device_inputs
        w = workload(name)
        nus, f = device_inputs(w, dev)
        del f
    else:
        w, nu, _, _ = make_inputs(name)
        nus = [torch.from_numpy(v).to(dev) for v in nu]
    H = Hierarchy(w.L, w.ncomp, nus[w.L], nus[:w.L], mg_dtype="f64")
    n = 2 ** (w.L + 1)
    u = torch.randn(w.ncomp * (n + 1) ** 3, dtype=torch.float64, device=dev)
    v = torch.empty_like(u)
    for _ in range(5):
        H.apply(w.L, u, v)
    del nus
    a = torch.empty(256 * 1024 * 1024 // 8, dtype=torch.float64, device=dev).normal_()
    c = torch.empty_like(a)
    for _ in range(3):
        c.copy_(a)
    torch.cuda.synchronize()
    H.close()
    print("profile-apply done", flush=True)


def profile_vcycle(name: str, smoother: str, dev) -> None:
    """Driver for instruction-counter passes over the V-cycle kernels: 3 FP32/BF16 and 3
    FP64 V-cycles of the benchmark's hierarchies on a random right-hand side."""
    import torch
    from paper_2511_13109_amd import Hierarchy
    from workloads import workload
    from workloads.device import device_inputs
    w = workload(name)
    nus, f = device_inputs(w, dev)
    del f
    for dt, nud in (("f32", "bf16"), ("f64", "f64")):
        H = Hierarchy(w.L, w.ncomp, nus[w.L], nus[:w.L], mg_dtype=dt, mg_nu_dtype=nud, smoother=smoother)
        n = 2 ** (w.L + 1)
        b = torch.randn(w.ncomp * (n + 1) ** 3, dtype=torch.float64, device=dev)
        if dt == "f32":
            b = b.float()
        z = torch.empty_like(b)
        for _ in range(3):
            H.vcycle(b, z)
        torch.cuda.synchronize()
        H.close()
        del b, z
    print("profile-vcycle done", flush=True)


# counters of the instruction passes over the V-cycle kernels (two runs of at most 8 SQ
# counters each) and the quantities the summary derives from them
VCYCLE_COUNTERS = [
    ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD",
     "SQ_INSTS_VMEM_WR", "SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES"],
    ["VALUBusy", "SQ_ACTIVE_INST_ANY", "SQ_BUSY_CYCLES", "SQ_INSTS_VALU_FMA_F32",
     "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_ADD_F64"],
    ["SQ_WAIT_INST_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_VALU",
     "SQ_INST_CYCLES_VMEM_RD", "SQ_WAIT_ANY", "SQ_WAVES", "SQ_WAVE_CYCLES"],
]


def summarize_counters(d: str, L: int) -> str:
    """Markdown table of the instruction counters of the finest-level element-loop passes
    in the counter runs under <d> (one sub-directory per run, rocprofv3 csv output)."""
    import csv
    import collections
    import glob
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    grids = collections.defaultdict(int)
    for path in glob.glob(os.path.join(d, "*", "*counter_collection.csv")):
        rows = list(csv.DictReader(open(path)))
        for r in rows:
            k = _short(r["Kernel_Name"])
            if not k.startswith("k_cube<3"):
                continue
            grids[k] = max(grids[k], int(r["Grid_Size"]))
        for r in rows:
            k = _short(r["Kernel_Name"])
            if k.startswith("k_cube<3") and int(r["Grid_Size"]) == grids[k]:
                vals[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
    lines = ["| kernel | waves | VALU / wave | FP FMA+ADD / wave | SALU / wave | VMEM / wave | "
             "LDS / wave | wait / wave cycles | VALUBusy % | LDS wait / wave cycles | "
             "LDS bank conflicts / LDS active | VALU active / wave cycles |",
             "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    med = lambda v: float(np.median(v)) if v else float("nan")
    for k in sorted(vals):
        c = {name: med(v) for name, v in vals[k].items()}
        wv = c.get("SQ_WAVES", float("nan"))
        fp = sum(c.get(f"SQ_INSTS_VALU_{op}_{t}", 0.0) for op in ("FMA", "ADD") for t in ("F32", "F64"))
        vmem = c.get("SQ_INSTS_VMEM_RD", 0.0) + c.get("SQ_INSTS_VMEM_WR", 0.0)
        lines.append(f"| `{k}` | {wv:.0f} | {c.get('SQ_INSTS_VALU', 0) / wv:.0f} | {fp / wv:.0f} | "
                     f"{c.get('SQ_INSTS_SALU', 0) / wv:.0f} | {vmem / wv:.0f} | "
                     f"{c.get('SQ_INSTS_LDS', 0) / wv:.0f} | "
                     f"{c.get('SQ_WAIT_INST_ANY', 0) / max(c.get('SQ_WAVE_CYCLES', 1), 1):.2f} | "
                     f"{c.get('VALUBusy', float('nan')):.1f} | "
                     f"{c.get('SQ_WAIT_INST_LDS', float('nan')) / max(c.get('SQ_WAVE_CYCLES', 1), 1):.3f} | "
                     f"{c.get('SQ_LDS_BANK_CONFLICT', float('nan')) / max(c.get('SQ_ACTIVE_INST_LDS', 1), 1):.3f} | "
                     f"{c.get('SQ_ACTIVE_INST_VALU', float('nan')) / max(c.get('SQ_WAVE_CYCLES', 1), 1):.3f} |")
    return "\n".join(lines)


def progress(msg: str):
    print(msg, file=sys.stderr, flush=True)


def cold_apply_us(H, level, u, v, reps=10):
    """Median duration of one apply with the Infinity Cache flushed before each (HIP events)."""
    import torch
    flush = torch.ones(512 * 1024 * 1024 // 8, dtype=torch.float64, device=u.device)
    sink = torch.zeros(1, dtype=torch.float64, device=u.device)
    ts = []
    for _ in range(reps):
        sink.add_(flush.sum())
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        H.apply(level, u, v)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e3)
    return float(np.median(ts))


def solve_record(H, b, solver: str, tol: float, max_iter: int = 8000):
    """One solve to tol with the milestones; returns x and a record of its statistics."""
    x, st = H.solve(b, solver=solver, tol=tol, max_iter=max_iter, raise_on_noconv=False,
                    record_history=False, milestones=MILESTONES)
    rec = {k: st[k] for k in ("iterations", "seconds", "rel_residual", "converged", "floor_limited",
                              "floor_estimate", "replacements", "status")}
    rec["milestones"] = {f"{m:g}": (None if v is None else {"iterations": v[0], "seconds": round(v[1], 4),
                                                            "rel_residual": v[2]})
                         for m, v in st["milestones"].items()}
    return x, rec


def time_to(rec: dict, tol: float, final_tol: float):
    """Seconds until the solve's verified true residual was <= tol, None if never."""
    if tol == final_tol:
        return round(rec["seconds"], 4) if rec["converged"] else None
    m = rec["milestones"].get(f"{tol:g}")
    return None if m is None else m["seconds"]


def speedup(a, b):
    return None if (a is None or b is None) else round(a / b, 3)


def bench_large(args, dev) -> dict:
    """The benchmark line on the 513^3 sinker workload (see the module docstring)."""
    import torch
    from paper_2511_13109_amd import Hierarchy
    from workloads import workload
    from workloads.device import device_inputs
    w = workload("sinker513", L=args.level)
    L, nc = w.L, w.ncomp
    n = 2 ** (L + 1)
    N = (n + 1) ** 3
    free_dofs = nc * (n - 1) ** 3
    t0 = time.perf_counter()
    nus, f = device_inputs(w, dev)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    progress(f"[bench] {w.name}: inputs on the device in {t_gen:.1f} s")
    H64 = Hierarchy(L, nc, nus[L], nus[:L], mg_dtype="f64", smoother=args.smoother,
                    coarse_storage=args.coarse_storage)
    H32 = Hierarchy(L, nc, nus[L], nus[:L], mg_dtype="f32", mg_nu_dtype=args.mg_nu,
                    smoother=args.smoother, coarse_storage=args.coarse_storage)
    b = H64.load_vector(f)
    del f
    b32 = b.float()
    z64, z32 = torch.empty_like(b), torch.empty_like(b32)
    gen = torch.Generator(device=dev).manual_seed(0)
    u = torch.randn(nc * N, generator=gen, dtype=torch.float64, device=dev)
    v = torch.empty_like(u)
    flush = torch.ones(512 * 1024 * 1024 // 8, dtype=torch.float64, device=dev)
    sink = torch.zeros(1, dtype=torch.float64, device=dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.applies)]
    evc = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(2)]
    rec = {"apply_ms": [], "setup_s": [], "vcycle64_ms": [], "vcycle32_ms": []}

    def step(record: bool):
        t0 = time.perf_counter()
        H64.set_nu(nus[L], nus[:L])
        H32.set_nu(nus[L], nus[:L])
        t_setup = time.perf_counter() - t0
        for e0, e1 in ev:
            sink.add_(flush.sum())
            e0.record()
            H64.apply(L, u, v)
            e1.record()
        evc[0][0].record()
        H64.vcycle(b, z64)
        evc[0][1].record()
        evc[1][0].record()
        H32.vcycle(b32, z32)
        evc[1][1].record()
        if record:
            torch.cuda.synchronize()
            rec["apply_ms"].append(float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev])))
            rec["setup_s"].append(t_setup)
            rec["vcycle64_ms"].append(evc[0][0].elapsed_time(evc[0][1]))
            rec["vcycle32_ms"].append(evc[1][0].elapsed_time(evc[1][1]))
            progress(f"[step] setup {t_setup:.3f} s, apply {rec['apply_ms'][-1] * 1e3:.1f} us, "
                     f"V-cycle FP64 {rec['vcycle64_ms'][-1]:.2f} ms, FP32 {rec['vcycle32_ms'][-1]:.2f} ms")

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    apply_s = float(np.mean(rec["apply_ms"])) / 1e3
    bytes_launch = apply_bytes(L, nc)
    achieved = bytes_launch / apply_s / 1e9
    # the FP32 / BF16 fine apply of the mixed hierarchy, timed the same way
    u32, v32 = u.float(), torch.empty_like(b32)
    t32 = cold_apply_us(H32, L, u32, v32)
    del u32, v32

    # the solves, once each, outside the timed steps
    progress("[bench] FP64-MG PCG to 1e-8 ...")
    x64, r64 = solve_record(H64, b, "pcg", w.tol)
    progress(f"[bench] FP64-MG PCG: {r64['iterations']} it, {r64['seconds']:.2f} s, res "
             f"{r64['rel_residual']:.3e}, rho {r64['floor_estimate']:.3e}, status {r64['status']}")
    x32, r32 = solve_record(H32, b, "fcg", w.tol)
    progress(f"[bench] FP32-MG FCG: {r32['iterations']} it, {r32['seconds']:.2f} s, res "
             f"{r32['rel_residual']:.3e}, rho {r32['floor_estimate']:.3e}, status {r32['status']}")
    dx = x32 - x64
    err_energy = float(torch.dot(dx, H64.apply(L, dx)) / torch.dot(x64, H64.apply(L, x64))) ** 0.5
    err_max = float(dx.abs().max() / x64.abs().max())
    del dx, x32
    info = [H64.query(l) for l in range(L)]
    info32 = [H32.query(l) for l in range(L)]
    dev64, dev32 = H64.device_bytes(), H32.device_bytes()
    peak_torch = int(torch.cuda.max_memory_allocated(dev))
    times = {}
    for tol in MILESTONES + (w.tol,):
        a, c = time_to(r64, tol, w.tol), time_to(r32, tol, w.tol)
        times[f"{tol:g}"] = {"fp64_mg_pcg": a, "fp32_mg_fcg": c, "speedup_fp32_over_fp64": speedup(a, c)}
    out = {
        "metric": METRIC, "value": round(free_dofs / apply_s / 1e9, 3), "unit": "GDoF/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "sinker513: vector -div(2 nu eps(u))=f, 513^3 nodes, 64 sinkers r in "
                               "[0.02, 0.06], contrast 1e6, FP64 and FP32/BF16 multigrid",
                   "levels": L + 1, "nodes": N, "free_dofs": free_dofs, "elements": 6 * n ** 3,
                   "applies_per_step": args.applies},
        "time_to_tol_s": times,
        "time_to_1e-8_s": times[f"{w.tol:g}"],
        "solves": {"fp64_mg_pcg": r64, "fp32_mg_fcg": r32, "mg_nu_dtype": args.mg_nu,
                   "smoother": args.smoother, "coarse_storage": args.coarse_storage},
        "mixed_vs_fp64_solution": {"energy_norm_rel": err_energy, "max_rel": err_max},
        "vcycle_ms": {"fp64": round(float(np.median(rec["vcycle64_ms"])), 3),
                      "fp32_bf16": round(float(np.median(rec["vcycle32_ms"])), 3)},
        "fp32_bf16_apply": {"us": round(t32, 1), "GDoF_s": round(free_dofs / t32 / 1e3, 2),
                            "GB_s": round(apply_bytes(L, nc, 4, 2) / t32 / 1e3, 1),
                            "frac_hbm_peak": round(apply_bytes(L, nc, 4, 2) / t32 / 1e3 / HBM_PEAK_GBS, 4)},
        "setup_s": round(float(np.median(rec["setup_s"])), 4),
        "flagged_per_level": [i["flagged"] for i in info],
        "flagged_fraction_per_level": [round(i["flagged"] / i["elements"], 6) for i in info],
        "stored_block_bytes": {"fp64_hierarchy": int(sum(i["block_bytes"] for i in info)),
                               "mixed_hierarchy": int(sum(i["block_bytes"] for i in info32))},
        "device_bytes": {"fp64_hierarchy": dev64, "mixed_hierarchy": dev32, "peak_torch": peak_torch},
        "hbm_fraction_used": round((dev64 + dev32 + peak_torch) / 288e9, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": recorded_traffic("sinker513"),
                     "kernel": "k_cube<3,double,double,APPLY> (fine-grid apply, 513^3)",
                     "bytes_per_launch": bytes_launch, "avg_launch_us": round(apply_s * 1e6, 2),
                     "kernel_source_sha256_16": kernel_hash()},
        "input_generation_s": round(t_gen, 2),
    }
    H64.close()
    H32.close()
    del x64, b, b32, z64, z32, u, v, nus, flush
    torch.cuda.empty_cache()
    return out


def extra_129(args, dev) -> dict:
    """The 129^3 sinker workload (8 sinkers r = 0.1, seed 2): cold FP64 apply, and FP64-MG
    PCG / FP32-MG FCG to 1e-8 with the 1e-7 milestone (extra keys of the benchmark line)."""
    import torch
    from paper_2511_13109_amd import Hierarchy
    w, nu, f, _ = make_inputs("sinker129")
    L, nc = w.L, w.ncomp
    nus = [torch.from_numpy(v).to(dev) for v in nu]
    H64 = Hierarchy(L, nc, nus[L], nus[:L], mg_dtype="f64", smoother=args.smoother)
    H32 = Hierarchy(L, nc, nus[L], nus[:L], mg_dtype="f32", mg_nu_dtype=args.mg_nu, smoother=args.smoother)
    b = H64.load_vector(torch.from_numpy(f.ravel()).to(dev))
    n = 2 ** (L + 1)
    free_dofs = nc * (n - 1) ** 3
    u = torch.randn(nc * (n + 1) ** 3, generator=torch.Generator(device=dev).manual_seed(0),
                    dtype=torch.float64, device=dev)
    t = cold_apply_us(H64, L, u, torch.empty_like(u), reps=20)
    for _ in range(2):      # warm-up solves (the first run of each kernel pays its load)
        solve_record(H64, b, "pcg", w.tol)
        solve_record(H32, b, "fcg", w.tol)
    # one V-cycle of each hierarchy, median of 30 back-to-back (HIP events)
    vc = {}
    for key, H, rhs in (("fp64", H64, b), ("fp32_bf16", H32, b.float())):
        z = torch.empty_like(rhs)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(30)]
        for e0, e1 in ev:
            e0.record()
            H.vcycle(rhs, z)
            e1.record()
        torch.cuda.synchronize()
        vc[key] = round(float(np.median([e0.elapsed_time(e1) for e0, e1 in ev])), 4)
    _, r64 = solve_record(H64, b, "pcg", w.tol)
    _, r32 = solve_record(H32, b, "fcg", w.tol)
    times = {}
    for tol in (1e-7, w.tol):
        a, c = time_to(r64, tol, w.tol), time_to(r32, tol, w.tol)
        times[f"{tol:g}"] = {"fp64_mg_pcg": a, "fp32_mg_fcg": c, "speedup_fp32_over_fp64": speedup(a, c)}
    H64.close()
    H32.close()
    return {"workload": f"{w.name}: {w.description}", "apply_us_cold": round(t, 2),
            "apply_GDoF_s": round(free_dofs / t / 1e3, 2),
            "apply_frac_hbm_peak": round(apply_bytes(L, nc) / t / 1e3 / HBM_PEAK_GBS, 4),
            "vcycle_ms": vc, "time_to_tol_s": times, "solves": {"fp64_mg_pcg": r64, "fp32_mg_fcg": r32}}


def report_stokes(args, dev) -> dict:
    """Generalized Stokes, velocity 257^3 / pressure 129^3, 16 sinkers: FGMRES with the
    upper block-triangular preconditioner (eq. (4.1)) and the BFBT Schur approximation
    (eq. (4.2)) or the 1/nu lumped mass, and MINRES with the block-diagonal one (lumped
    mass), each with the FP32 V-cycle against the FP64 V-cycle, to 1e-8."""
    import torch
    from paper_2511_13109_amd import Hierarchy, Stokes
    from workloads import workload
    from workloads.device import device_inputs
    w = workload(args.workload, L=args.level)
    L = w.L
    nus, f = device_inputs(w, dev)
    out = {"report": w.name, "description": w.description,
           "velocity_free_dofs": 3 * (2 ** (L + 1) - 1) ** 3, "pressure_dofs": (2 ** L + 1) ** 3,
           "fgmres_restart": args.stokes_restart, "smoother": args.smoother,
           "bfbt_z_cg_steps": args.schur_iters, "bfbt_mg_z_cg_steps": args.zmg_iters,
           "tol": args.stokes_tol or w.tol, "velocity_cycles": args.velocity_cycles,
           "fgmres_basis": args.stokes_basis}
    runs = [r for r in (("bfbt_mg", "f32", "fgmres", "triangular", "bfbt_mg"),
                        ("bfbt_mg", "f64", "fgmres", "triangular", "bfbt_mg"),
                        ("bfbt", "f32", "fgmres", "triangular", "bfbt"),
                        ("bfbt", "f64", "fgmres", "triangular", "bfbt"),
                        ("fgmres", "f32", "fgmres", "triangular", "mass"),
                        ("fgmres", "f64", "fgmres", "triangular", "mass"),
                        ("minres", "f32", "minres", "diagonal", "mass"),
                        ("minres", "f64", "minres", "diagonal", "mass"))
            if r[0] in args.stokes_solvers.split(",") and r[1] in args.stokes_mg.split(",")]
    for _, mg, solver, pc, schur in runs:
        H = Hierarchy(L, 3, nus[L], nus[:L], mg_dtype=mg, mg_nu_dtype=("bf16" if mg == "f32" else "f64"),
                      smoother=args.smoother)
        S = Stokes(H)
        fu = H.load_vector(f)
        k = args.zmg_iters if schur == "bfbt_mg" else args.schur_iters
        setup = {}
        if schur == "bfbt_mg":
            # the pressure multigrid's assembly (first use after the build), then one
            # application of S^-1 with it in place
            rp = torch.randn(S.np, dtype=torch.float64, device=dev)
            for name in ("zmg_setup_s", "schur_apply_s"):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                S.schur_apply(rp, "bfbt_mg", k)
                torch.cuda.synchronize()
                setup[name] = round(time.perf_counter() - t0, 4)
        _, _, st = S.solve(fu, solver=solver, restart=args.stokes_restart, tol=args.stokes_tol or w.tol,
                           max_iter=args.stokes_max_iter, record_history=False, raise_on_noconv=False,
                           precond=pc, schur=schur, schur_iters=k, velocity_cycles=args.velocity_cycles,
                           basis=(args.stokes_basis if solver == "fgmres" else "f64"))
        key = f"{solver}_{pc}" + ("" if schur == "mass" else f"_{schur}") + f"_{mg}_mg"
        out[key] = {k: st[k] for k in ("iterations", "seconds", "rel_residual", "converged",
                                       "floor_limited")}
        out[key].update(setup)
        print(f"[stokes] {solver} {pc} {schur} {mg}-MG: {st['iterations']} it {st['seconds']:.2f} s "
              f"res {st['rel_residual']:.2e}", file=sys.stderr, flush=True)
        H.close()
        torch.cuda.empty_cache()
    return out


def report_adjoint(args, dev) -> dict:
    """129^3 adjoint workload: forward solve, adjoint solve and the gradient kernel, with
    the homogeneity identity of the gradient as a check."""
    import torch
    from paper_2511_13109_amd import Hierarchy
    from paper_2511_13109_amd.autograd import solve as dsolve
    from workloads import workload
    from workloads.lattice import element_centroids
    w = workload(args.workload, L=args.level)
    L = w.L
    g = w.make_field()
    cf = element_centroids(L)
    g.calibrate(cf)
    log_nu = torch.from_numpy(g.log_nu(cf)).to(dev)
    nu_c = [torch.from_numpy(np.exp(g.log_nu(element_centroids(l)))).to(dev) for l in range(L)]
    f = torch.from_numpy(np.ascontiguousarray(np.asarray(g.force(cf, 3)).T)).to(dev).reshape(-1)
    log_obs = log_nu + torch.from_numpy(g.noise(log_nu.numel())).to(dev)
    H = Hierarchy(L, 3, torch.exp(log_nu), nu_c, smoother=args.smoother)
    b = H.load_vector(f)
    with torch.no_grad():
        obs = dsolve(log_obs, b, H, nu_c, tol=w.tol).clone()
    lnu = log_nu.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u = dsolve(lnu, b, H, nu_c, tol=w.tol)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    J = 0.5 * torch.sum((u - obs) ** 2)
    J_value = float(J.detach())
    t0 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    gg = lnu.grad
    hom = -float(torch.dot(u.detach() - obs, u.detach()))
    out = {"report": w.name, "description": w.description, "forward_s": round(t_fwd, 4),
           "adjoint_and_gradient_s": round(t_bwd, 4), "J": J_value,
           "homogeneity_rel_err": abs(float(gg.sum()) - hom) / abs(hom), "smoother": args.smoother}
    H.close()
    return out


def report_roofline(args, dev) -> dict:
    """Apply roofline sweep: the scalar and the vector fine-grid apply at 129^3, 257^3 and
    513^3 nodes (the 513^3 workload's coefficient generator, 64 sinkers) in FP64, FP32
    with an FP32 coefficient and FP32 with a BF16 coefficient; u ~ N(0, 1) (seed 0) on
    the free DoFs.  Median of 20 HIP-event timings after 3 warm-ups, with the Infinity
    Cache flushed before each (cold) and without (warm)."""
    import torch
    from paper_2511_13109_amd import Hierarchy
    from workloads import workload
    from workloads.device import device_inputs
    levels = [int(v) for v in args.roofline_levels.split(",")]
    flush = torch.ones(512 * 1024 * 1024 // 8, dtype=torch.float64, device=dev)
    sink = torch.zeros(1, dtype=torch.float64, device=dev)

    def timed(H, L, u, v, cold):
        for _ in range(3):
            H.apply(L, u, v)
        ts = []
        for _ in range(20):
            if cold:
                sink.add_(flush.sum())
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            H.apply(L, u, v)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e3)
        return float(np.median(ts))

    rows = []
    for L in levels:
        w = workload("sinker513", L=L)
        nus, f = device_inputs(w, dev)
        del f
        n = 2 ** (L + 1)
        N = (n + 1) ** 3
        gen = torch.Generator(device=dev).manual_seed(0)
        for nc in (1, 3):
            free = nc * (n - 1) ** 3
            u = torch.randn(nc * N, generator=gen, device=dev, dtype=torch.float64)
            v = torch.empty_like(u)
            for nu_dt in ("f32", "bf16"):
                H = Hierarchy(L, nc, nus[L], nus[:L], mg_dtype="f32", mg_nu_dtype=nu_dt)
                cases = [("f64", u, v, 8, 8)] if nu_dt == "f32" else []
                u32 = u.float()
                cases.append((f"f32/{nu_dt}", u32, torch.empty_like(u32), 4, 4 if nu_dt == "f32" else 2))
                for label, uu, vv, vb, nb in cases:
                    byt = apply_bytes(L, nc, vb, nb)
                    rec = {"nodes": f"{n + 1}^3", "ncomp": nc, "precision": label,
                           "bytes_per_launch": byt}
                    for mode in ("cold", "warm"):
                        t = timed(H, L, uu, vv, mode == "cold")
                        rec[f"{mode}_us"] = round(t, 2)
                        rec[f"{mode}_GDoF_s"] = round(free / t / 1e3, 2)
                        rec[f"{mode}_frac_hbm_peak"] = round(byt / t / 1e3 / HBM_PEAK_GBS, 4)
                    rows.append(rec)
                    progress(f"[roofline] {n + 1}^3 ncomp={nc} {label}: cold {rec['cold_us']} us "
                             f"({rec['cold_frac_hbm_peak']:.3f} of peak), warm {rec['warm_us']} us")
                H.close()
                torch.cuda.empty_cache()
        del nus
        torch.cuda.empty_cache()
    return {"report": "roofline", "coefficient": "64 sinkers, radii 0.02-0.06, contrast 1e6",
            "hbm_peak_GB_s": HBM_PEAK_GBS, "rows": rows}


def report_coarsening(args, dev) -> dict:
    """Direct against adaptive against Galerkin coarsening (Sections 2.3, 4.2-4.3): PCG
    iterations to 1e-8 of the vector viscous block with the FP64 V-cycle for the
    coefficients eta_1..eta_4 and sharp multi-sinkers eta_6 at three dynamic ratios,
    with DCA on every coarse level, the per-element ratio flag (tau = 10), the
    macro-element gradient flag (eq. (2.8), nu = 10) and Galerkin coarsening on every
    level; then the tolerance sweep of Fig. 9 on the tanh-smoothed cube."""
    import torch
    from paper_2511_13109_amd import Hierarchy, macro_gradient
    from workloads import Sinkers
    from workloads.fields import ShapeField
    from workloads.lattice import element_centroids
    L = args.level or 5
    n = 2 ** (L + 1)
    p = np.arange((n + 1) ** 3)
    xyz = np.stack([p % (n + 1), (p // (n + 1)) % (n + 1), p // (n + 1) ** 2], axis=1) / n
    cents = [element_centroids(l) for l in range(L + 1)]
    max_iter = 1000

    def run(field, mode, tol_grad=10.0, nu=None, g=None):
        if nu is None:
            nu = [torch.from_numpy(field.nu(c)).to(dev) for c in cents]
        if g is None:
            g = macro_gradient(L, torch.from_numpy(field.nu(xyz)).to(dev))
        mf = g > tol_grad
        kw = {"flag_mode": mode}
        if mode == "macro":
            kw["macro_flags"] = mf
        H = Hierarchy(L, 3, nu[L], nu[:L], smoother=args.smoother, **kw)
        f = torch.from_numpy(np.ascontiguousarray(field.force(cents[L], 3).T)).to(dev).reshape(-1)
        b = H.load_vector(f)
        _, st = H.solve(b, solver="pcg", tol=1e-8, max_iter=max_iter, raise_on_noconv=False,
                        record_history=False)
        info = [H.query(l) for l in range(L)]
        rec = {"iterations": st["iterations"] if (st["converged"] or st["floor_limited"]) else None,
               "rel_residual": float("%.3g" % st["rel_residual"]),
               "flagged_fraction": round(sum(i["flagged"] for i in info) / sum(i["elements"] for i in info), 4),
               "block_bytes": int(sum(i["block_bytes"] for i in info))}
        if mode == "macro":
            rec["macros"] = int(mf.sum())
        H.close()
        return rec

    fields = [("eta1 aligned cube", lambda dr: ShapeField("cube", dr)),
              ("eta2 unaligned cube", lambda dr: ShapeField("ucube", dr)),
              ("eta3 tanh cube omega=10", lambda dr: ShapeField("tcube", dr, 10.0)),
              ("eta3 tanh cube omega=100", lambda dr: ShapeField("tcube", dr, 100.0)),
              ("eta3 tanh cube omega=1000", lambda dr: ShapeField("tcube", dr, 1000.0)),
              ("eta4 sphere", lambda dr: ShapeField("sphere", dr)),
              ("eta6 1 sharp sinker", lambda dr: Sinkers(1, 2, radius=0.1, width=1e-9, contrast=dr)),
              ("eta6 4 sharp sinkers", lambda dr: Sinkers(4, 2, radius=0.1, width=1e-9, contrast=dr)),
              ("eta6 16 sharp sinkers", lambda dr: Sinkers(16, 2, radius=0.1, width=1e-9, contrast=dr))]
    out = {"report": "coarsening", "levels": L + 1, "nodes_per_axis": n + 1, "smoother": args.smoother,
           "solver": f"FP64-MG PCG to 1e-8, at most {max_iter} iterations (null: not reached)",
           "cases": []}
    for dr in (1e2, 1e4, 1e6):
        for name, make in fields:
            field = make(dr)
            nu = [torch.from_numpy(field.nu(c)).to(dev) for c in cents]
            g = macro_gradient(L, torch.from_numpy(field.nu(xyz)).to(dev))
            rec = {"field": name, "DR": dr}
            for mode in ("dca", "ratio", "macro", "gca"):
                rec[mode] = run(field, mode, nu=nu, g=g)
            progress(f"[coarsening] {name} DR={dr:g}: " + ", ".join(
                f"{m} {rec[m]['iterations']}" for m in ("dca", "ratio", "macro", "gca")))
            out["cases"].append(rec)
    # Fig. 9: tolerance sweep of the macro gradient test on the tanh-smoothed cube
    out["tolerance_sweep"] = []
    for omega in (10.0, 100.0, 1000.0):
        field = ShapeField("tcube", 1e6, omega)
        nu = [torch.from_numpy(field.nu(c)).to(dev) for c in cents]
        g = macro_gradient(L, torch.from_numpy(field.nu(xyz)).to(dev))
        for tol in (1e-2, 1e0, 1e2, 1e4, 1e6):
            rec = run(field, "macro", tol_grad=tol, nu=nu, g=g)
            rec.update({"omega": omega, "tolerance": tol})
            out["tolerance_sweep"].append(rec)
            progress(f"[coarsening] tanh cube omega={omega:g} tol={tol:g}: {rec['macros']} macros, "
                     f"{rec['iterations']} it, {rec['block_bytes'] / 1e6:.1f} MB")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sinker513")
    ap.add_argument("--applies", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mg-nu", default="bf16", choices=["bf16", "f32"])
    ap.add_argument("--smoother", default="chebyshev", choices=["jacobi", "chebyshev"])
    ap.add_argument("--coarse-storage", default="blocks", choices=["blocks", "mean"],
                    help="flagged elements keep their Galerkin block, or the descendant mean "
                         "of the coefficient (the same operator for P1)")
    ap.add_argument("--profile-apply", action="store_true",
                    help="only run 5 FP64 fine applies and a 256 MiB copy (counter passes)")
    ap.add_argument("--profile-vcycle", action="store_true",
                    help="only run 3 FP32/BF16 and 3 FP64 V-cycles of the 513^3 hierarchies (counter passes)")
    ap.add_argument("--summarize-counters", metavar="DIR",
                    help="print the instruction-counter table of the V-cycle counter runs under DIR")
    ap.add_argument("--summarize-trace", metavar="CSV",
                    help="print the finest-level solver-kernel table of a rocprofv3 kernel trace")
    ap.add_argument("--summarize-profile", metavar="DIR",
                    help="print the markdown summary of a profiling directory and exit")
    ap.add_argument("--level", type=int, default=None, help="finest level of a report workload")
    ap.add_argument("--roofline-levels", default="6,7,8",
                    help="finest levels of the apply roofline sweep (6: 129^3, 7: 257^3, 8: 513^3)")
    ap.add_argument("--stokes-max-iter", type=int, default=8000)
    ap.add_argument("--stokes-solvers", default="fgmres,minres",
                    help="comma-separated subset of bfbt_mg (FGMRES, triangular, BFBT with the "
                         "pressure multigrid), bfbt (the same with Jacobi-CG Z solves), fgmres "
                         "(triangular, lumped mass) and minres (diagonal, lumped mass)")
    ap.add_argument("--schur-iters", type=int, default=20,
                    help="Jacobi-CG steps per Z solve of the BFBT Schur approximation")
    ap.add_argument("--zmg-iters", type=int, default=4,
                    help="multigrid-preconditioned CG steps per Z solve of BFBT with the pressure multigrid")
    ap.add_argument("--stokes-restart", type=int, default=64)
    ap.add_argument("--velocity-cycles", type=int, default=1,
                    help="V-cycles per application of the velocity block's approximate inverse (1: the paper's)")
    ap.add_argument("--stokes-tol", type=float, default=None,
                    help="relative residual of the Stokes report solves (default: the workload's 1e-8)")
    ap.add_argument("--stokes-mg", default="f32,f64",
                    help="comma-separated V-cycle precisions of the Stokes report runs")
    ap.add_argument("--stokes-basis", default="f64", choices=["f64", "f32"],
                    help="storage of the FGMRES Arnoldi basis in the Stokes report runs")
    args = ap.parse_args()
    if args.summarize_profile:
        print(summarize_profile(args.summarize_profile, ""))
        return
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace, args.level or 6))
        return
    if args.summarize_counters:
        print(summarize_counters(args.summarize_counters, args.level or 8))
        return

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
    if args.profile_vcycle:
        profile_vcycle("sinker513", args.smoother, dev)
        return
    # the benchmark line: 513^3 (default) or the earlier 129^3 line; the other workloads
    # print a report line of their own
    reports = {"stokes257": report_stokes, "adjoint129": report_adjoint,
               "coarsening": report_coarsening, "roofline": report_roofline}
    if args.workload in reports:
        print(json.dumps(reports[args.workload](args, dev)), flush=True)
        return
    if args.workload == "sinker513":
        out = bench_large(args, dev)
        out["sinker129"] = extra_129(args, dev)
    elif args.workload == "sinker129":
        out = bench_129(args, dev)
    else:
        raise SystemExit(f"unknown workload {args.workload}")
    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(args.workload)
        except Exception as exc:  # the baseline is a report, never a reason to lose the line
            out["cpu_baseline"] = {"error": repr(exc)}
    print(json.dumps(out), flush=True)


def bench_129(args, dev) -> dict:
    """The benchmark line on the 129^3 sinker workload (steps as before: rebuild, 20 cold
    applies, both solves to 1e-8 and to 1e-7)."""
    import torch
    from paper_2511_13109_amd import Hierarchy
    w, nu, f, t_gen = make_inputs(args.workload)
    L, nc = w.L, w.ncomp
    nus = [torch.from_numpy(v).to(dev) for v in nu]
    f_dev = torch.from_numpy(f.ravel()).to(dev)
    H64 = Hierarchy(L, nc, nus[L], nus[:L], mg_dtype="f64", smoother=args.smoother)
    H32 = Hierarchy(L, nc, nus[L], nus[:L], mg_dtype="f32", mg_nu_dtype=args.mg_nu,
                    smoother=args.smoother)
    b = H64.load_vector(f_dev)
    gen = torch.Generator(device="cpu").manual_seed(0)
    n = 2 ** (L + 1)
    N = (n + 1) ** 3
    free_dofs = nc * (n - 1) ** 3
    u = torch.randn(nc * N, generator=gen, dtype=torch.float64).to(dev)
    v = torch.empty_like(u)
    # each timed apply is preceded by a read of 512 MiB, which evicts the 256 MB
    # Infinity Cache, so the apply streams its operands from HBM
    flush = torch.ones(512 * 1024 * 1024 // 8, dtype=torch.float64, device=dev)
    sink = torch.zeros(1, dtype=torch.float64, device=dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.applies)]

    rec = {"apply_ms": [], "setup_s": [], "t64": [], "t32": [], "it64": [], "it32": [],
           "res64": [], "res32": [], "t64_7": [], "t32_7": [], "it64_7": [], "it32_7": []}

    def step(record: bool):
        t0 = time.perf_counter()
        H64.set_nu(nus[L], nus[:L])
        H32.set_nu(nus[L], nus[:L])
        t_setup = time.perf_counter() - t0
        for e0, e1 in ev:
            sink.add_(flush.sum())
            e0.record()
            H64.apply(L, u, v)
            e1.record()
        x64, s64 = H64.solve(b, solver="pcg", tol=w.tol, max_iter=4000, raise_on_noconv=False)
        x32, s32 = H32.solve(b, solver="fcg", tol=w.tol, max_iter=4000, raise_on_noconv=False)
        # the same solves to 1e-7, a tolerance both reach without meeting the FP64 rounding
        # floor of this contrast (about 1e-8 for an FP64 iterate)
        _, s64_7 = H64.solve(b, solver="pcg", tol=1e-7, max_iter=4000, raise_on_noconv=False,
                             record_history=False)
        _, s32_7 = H32.solve(b, solver="fcg", tol=1e-7, max_iter=4000, raise_on_noconv=False,
                             record_history=False)
        if record:
            rec["t64_7"].append(s64_7["seconds"])
            rec["t32_7"].append(s32_7["seconds"])
            rec["it64_7"].append(s64_7["iterations"])
            rec["it32_7"].append(s32_7["iterations"])
            torch.cuda.synchronize()
            rec["apply_ms"].append(float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev])))
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
                           "mg_nu_dtype": args.mg_nu, "smoother": args.smoother,
                           "speedup_fp32_over_fp64": round(float(np.median(rec["t64"]) /
                                                                 np.median(rec["t32"])), 3)},
        "iterations": {"fp64_mg_pcg": int(np.median(rec["it64"])), "fp32_mg_fcg": int(np.median(rec["it32"]))},
        "time_to_1e-7_s": {"fp64_mg_pcg": round(float(np.median(rec["t64_7"])), 5),
                           "fp32_mg_fcg": round(float(np.median(rec["t32_7"])), 5),
                           "iterations": [int(np.median(rec["it64_7"])), int(np.median(rec["it32_7"]))],
                           "speedup_fp32_over_fp64": round(float(np.median(rec["t64_7"]) /
                                                                 np.median(rec["t32_7"])), 3)},
        "final_rel_residual_fp64": {"fp64_mg": max(rec["res64"]), "fp32_mg": max(rec["res32"])},
        "solve_status": {"fp64_mg": rec["stat64"][-1], "fp32_mg": rec["stat32"][-1]},
        "setup_s": round(float(np.median(rec["setup_s"])), 5),
        "flagged_per_level": [H64.query(l)["flagged"] for l in range(L)],
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": recorded_traffic("sinker129"),
                     "kernel": "k_cube<3,double,double,APPLY> (fine-grid apply)",
                     "bytes_per_launch": bytes_launch, "avg_launch_us": round(apply_s * 1e6, 2),
                     "kernel_source_sha256_16": kernel_hash()},
        "input_generation_s": round(t_gen, 2),
    }
    H64.close()
    H32.close()
    return out


if __name__ == "__main__":
    main()
