"""Throughput of the multiple-Arnoldi Green's-function path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 2] [--nu 30]
                    [--schedule auto] [--workflow auto] [--no-cpu] [--no-plain]
                    [--no-extra]

One step is one pass of the whole hot path over the 4,096-site vacancy cell
(8x8x8 diamond cells, 5% vacancies, sigma 0.05 A, 6 A clusters, nu = 30,
kT = 0.1 eV): pass 1 (per-column Krylov growth, projection, projected
eigensolve, spectral weights), mu by bisection, energies, then the backward
pass (pass 2 -> rho, pi -> dA/dH, dA/dS) and the Slater-Koster force
contraction.  The workflow of Eq. 3 is chosen by the library (store Y d on the
pattern when it fits in HBM, else recompute the Krylov columns in pass 2); the
recompute workflow is timed too and reported beside it.  Inputs are resident on
the GPU before the timed region.  Prints one JSON line.

Reported beside the headline: the forward alone, plain per-column launches
(and whether their rho equals the persistent launch's bit for bit), the exact
gradient of the truncated method (fwd + exact bwd), central differences of the
grand potential against both kinds of forces, the population analysis, the
COCG solver, MD steps, and two more workloads in the same line: the
32,768-site void cell at nu = 20, 30 and 40 (persistent against plain
launches) and the million-site cell (forward and force backward in the
library's workflow, and with the Krylov columns recomputed in pass 2, device
memory).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Green's-fn columns/s, fwd and fwd+force-bwd, vs plain at |Δρ|≤1e-10"
HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector (= FP64 matrix), TFLOP/s
# Per-CU rate of 16-byte vector-memory lane loads that a stand-alone kernel
# with the Krylov SpMV's access pattern sustains (three per cycle per CU,
# L2-resident data; 256 CUs at 2.4 GHz): the ceiling of the streamed blocks
VMEM_PEAK_GBS = 3 * 16 * 256 * 2.4


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="2")
    ap.add_argument("--nu", type=int, default=None)
    ap.add_argument("--schedule", default="auto")
    ap.add_argument("--workflow", default="auto")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the per-column-launch baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the void-cell and million-site workloads")
    ap.add_argument("--no-exact", action="store_true",
                    help="skip the exact gradient and the differences")
    ap.add_argument("--cpu-seconds", type=float, default=30.0)
    ap.add_argument("--cocg-columns", type=int, default=2048,
                    help="columns of the COCG sample (0: none)")
    ap.add_argument("--md-steps", type=int, default=4,
                    help="MD steps timed after the solve benchmark (0: none)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="end with a 512 MiB fill and device copy (HBM counter calibration)")
    return ap.parse_args(argv)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "krylov_kernel_traffic_c4096_vac5_nu30.md")
KERNEL_SOURCES = ("paper_1210_1531_amd/csrc/krylov.hip", "paper_1210_1531_amd/csrc/wave.h",
                  "paper_1210_1531_amd/csrc/mag_internal.h")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per Krylov launch from the committed counter profile, or None
    when the profile is missing or was taken on a different kernel source."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("source sha256") != kernel_source_hash():
        return None
    try:
        return float(fields["HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(struct, target_s):
    """Oracle (plain NumPy/SciPy, mode K) on a bounded sample of the workload's columns."""
    import numpy as np

    from oracle import pool, solve
    pool.start()  # before this process touches the GPU: the workers fork from a clean server
    cores = min(16, len(os.sched_getaffinity(0)))
    sysm = solve.geometry(struct)
    M = sysm.M
    probe = np.arange(0, M, max(1, M // 16))[:16]
    t0 = time.perf_counter()
    solve.column_data(sysm, probe, workers=1)
    per_col = (time.perf_counter() - t0) / probe.size
    n = int(min(M, max(cores * 8, target_s * cores / per_col)))
    n = (n // 4) * 4
    step = max(1, (M // 4) // (n // 4))
    atoms = np.arange(0, M // 4, step)[: n // 4]
    cols = (4 * atoms[:, None] + np.arange(4)[None, :]).ravel()
    t0 = time.perf_counter()
    solve.column_data(sysm, cols, workers=cores)
    wall = time.perf_counter() - t0
    return {
        "value": cols.size / wall,
        "unit": "columns/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{cols.size} of {M} columns ({atoms.size} atoms: every {step}-th from atom 0, "
                  f"all 4 orbitals), mode-K "
                  f"Ritz data + pattern rows, {wall:.1f} s wall on {cores} processes",
    }


def build_context(Context, model, s, torch):
    """Context with H, S and clusters of structure s; returns (ctx, pos, sk
    model, set-up milliseconds of a second SK build and set_system)."""
    ctx = Context(device=0)
    pos = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    sk = model.sk_model()
    ctx.sk_build(sk, pos, s.cell)
    rowptr, colind, H, S = ctx.sk_get_csr()
    ctx.set_system(rowptr, colind, H, S, pos=pos, cell=s.cell, r_cluster=s.r_cluster)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.sk_build(sk, pos, s.cell)
    torch.cuda.synchronize()
    t_skb = (time.perf_counter() - t0) * 1e3
    rowptr, colind, H, S = ctx.sk_get_csr()
    t0 = time.perf_counter()
    ctx.set_system(rowptr, colind, H, S, pos=pos, cell=s.cell, r_cluster=s.r_cluster)
    torch.cuda.synchronize()
    t_sys = (time.perf_counter() - t0) * 1e3
    return ctx, pos, sk, {"sk_build": t_skb, "set_system": t_sys}


def krylov_roofline(ctx, s, st, t_launch_ms, launches_per_pass=1):
    """Roofline of krylov_kernel: algorithmic bytes of the streamed-cluster
    model per launch (per column nu nnz_C 20 B / 4, the cluster's H, S values
    and index read once per Krylov step and shared by the atom's four columns,
    plus the pattern outputs 2 n_pat 8 B and the spectra 2 nu 8 B) over the
    launch's duration, against HBM peak; the streamed blocks actually issued
    per launch (every step re-reads each non-cached block, 256 B, per column)
    against the vector-memory ceiling; FP64 rate."""
    nu = s.nu
    M = 4 * s.n_atoms
    bytes_pass = 20.0 * nu * st["sum_cluster_nnz"] + 16.0 * ctx.nnz + 16.0 * nu * M
    per_launch = bytes_pass / max(launches_per_pass, 1)
    achieved = per_launch / (t_launch_ms * 1e-3) / 1e9
    streamed_blocks = max(0.0, st["sum_cluster_nnz"] / 16.0
                          - s.n_atoms * float(st["krylov_cache_blocks"]))
    vmem = 4.0 * nu * streamed_blocks * 256.0 / max(launches_per_pass, 1)
    vmem_gbs = vmem / (t_launch_ms * 1e-3) / 1e9
    return {
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "kernel": "krylov_kernel",
        "launch_ms": t_launch_ms,
        "bytes_per_launch": per_launch,
        "model": "streamed-cluster bytes: every Krylov step reads the cluster's H, S values "
                 "and indices once, shared by the atom's four columns; this working set is "
                 "served from LDS, L2 and MALL, not HBM",
        "vmem": {"issued_bytes_per_launch": vmem, "achieved_GBs": vmem_gbs,
                 "ceiling_GBs": VMEM_PEAK_GBS, "frac": vmem_gbs / VMEM_PEAK_GBS,
                 "cache_blocks": int(st["krylov_cache_blocks"])},
    }


def launch_plans(st):
    """The launch plan chosen for each cluster-size bucket of the last pass."""
    out = []
    for b, tpb in enumerate(st["plan_threads"]):
        if tpb <= 0:
            continue
        out.append({"bucket": b, "threads": tpb, "rows_per_thread": st["plan_rows"][b],
                    "workgroups_per_cu": st["plan_per_cu"][b],
                    "cached_blocks": st["plan_cache"][b],
                    "candidates": st["plan_candidates"][b],
                    "columns": int(st["plan_columns"][b]),
                    "tuned_us_per_column": st["plan_us_per_col"][b]})
    return out


def grand_potential_columns(eps, w, nu_eff, mu, kT):
    """Per-column Omega_j = sum_k w_jk omega(eps_jk), omega(e) = -kT ln(1 +
    exp(-(e - mu)/kT)), from the GPU's Ritz data."""
    import numpy as np
    x = (eps - mu) / kT
    om = -kT * (np.maximum(-x, 0.0) + np.log1p(np.exp(-np.abs(x))))
    mask = np.arange(eps.shape[1])[None, :] < nu_eff[:, None]
    return np.where(mask, w * om, 0.0).sum(axis=1)


def fd_forces(ctx, s, atoms, mu, h, torch):
    """Central differences of the GPU grand potential at fixed mu.  Columns
    whose cluster lacks the displaced atom are bitwise unchanged, so only the
    columns of its cluster enter the difference (math.fsum)."""
    import numpy as np
    ptr, catoms = (x.cpu().numpy() for x in ctx.get_clusters())
    pos0 = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    out = np.zeros((len(atoms), 3))
    for a, I in enumerate(atoms):
        near = catoms[ptr[I]:ptr[I + 1]]
        cols = torch.as_tensor((4 * near[:, None] + np.arange(4)[None, :]).ravel(),
                               device="cuda")
        for c in range(3):
            om = []
            for sgn in (1.0, -1.0):
                p = pos0.clone()
                p[I, c] += sgn * h
                Hv, Sv = ctx.sk_values(p)
                ctx.update_values(Hv, Sv)
                ctx.solve(nu=s.nu, kT=s.kT, n_electrons=s.n_electrons, mu_fixed=mu)
                eps, w, nu = ctx.spectra()
                om.append(grand_potential_columns(eps[cols].cpu().numpy(), w[cols].cpu().numpy(),
                                                  nu[cols].cpu().numpy(), mu, s.kT))
            out[a, c] = -math.fsum(om[0] - om[1]) / (2 * h)
    Hv, Sv = ctx.sk_values(pos0)
    ctx.update_values(Hv, Sv)
    return out


def extra_workload(key, nu, Context, model, torch, steps, plain_sample, recompute=False):
    """Forward and fwd+bwd of another workload in the library's launch
    configuration, with its own Krylov roofline; plain per-column launches
    on a sample of columns, bitwise against the persistent launch there."""
    import numpy as np

    import gen
    s = gen.make(key, nu=nu)
    M = 4 * s.n_atoms
    t_gen = time.perf_counter()
    ctx, pos, sk, setup = build_context(Context, model, s, torch)
    opts = dict(nu=s.nu, kT=s.kT, n_electrons=s.n_electrons)
    st0 = ctx.stats()
    ctx.solve(**opts)  # first use: launch plans timed here
    st_tune = ctx.stats()
    ctx.backward(1.0)
    ctx.forces(sk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kry_ms, kry_launch = 0.0, 0
    for _ in range(steps):
        ctx.solve(**opts)
        st = ctx.stats()
        kry_ms += st["t_krylov_ms"]
        kry_launch += st["krylov_launches"]
    torch.cuda.synchronize()
    ms_fwd = (time.perf_counter() - t0) * 1e3 / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.solve(**opts)
        ctx.backward(1.0)
        ctx.forces(sk)
    torch.cuda.synchronize()
    ms_fb = (time.perf_counter() - t0) * 1e3 / steps
    st = ctx.stats()
    free, total = torch.cuda.mem_get_info()
    out = {
        "workload": f"{s.name}: {s.meta['cells'][0]}x{s.meta['cells'][1]}x{s.meta['cells'][2]} "
                    f"diamond carbon cells, {s.n_atoms} atoms, nu {s.nu}",
        "columns": M, "nu": s.nu,
        "fwd_columns_per_s": M / (ms_fwd * 1e-3), "fwd_ms": ms_fwd,
        "fwdbwd_columns_per_s": M / (ms_fb * 1e-3), "fwdbwd_ms": ms_fb,
        "workflow_used": {0: "recompute", 1: "store"}[st["workflow_used"]],
        "krylov_buckets": st["krylov_buckets"], "krylov_threads": st["krylov_tpb"],
        "autotune_ms": st_tune["autotune_ms"] - st0["autotune_ms"],
        "krylov_plans": launch_plans(st),
        "stage_ms": {"krylov": st["t_krylov_ms"], "eig": st["t_eig_ms"],
                     "mu_energy": st["t_mu_ms"], "pass2": st["t_pass2_ms"],
                     "forces": st["t_forces_ms"]},
        "setup_ms": setup,
        "device_bytes": int(st["device_bytes"]),
        "device_used_bytes": int(total - free),
        "roofline": krylov_roofline(ctx, s, st, kry_ms / max(kry_launch, 1),
                                    max(1, kry_launch // steps) if kry_launch else 1),
        "N_minus_Ne": ctx.energy()["N"] - s.n_electrons,
    }
    if recompute and st["workflow_used"] != 0:
        # the memory-saving workflow of Eq. 3 at the same size
        ropts = dict(opts, workflow="recompute")
        ctx.solve(**ropts)
        ctx.backward(1.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.solve(**ropts)
            ctx.backward(1.0)
            ctx.forces(sk)
        torch.cuda.synchronize()
        ms_rc = (time.perf_counter() - t0) * 1e3 / steps
        out["fwdbwd_recompute_columns_per_s"] = M / (ms_rc * 1e-3)
        out["fwdbwd_recompute_ms"] = ms_rc
    if plain_sample > 0:
        rng = np.random.default_rng(7)
        atoms = np.sort(rng.choice(s.n_atoms, plain_sample // 4, replace=False))
        cols = (4 * atoms[:, None] + np.arange(4)[None, :]).ravel().astype(np.int32)
        per = ctx.column_spectra(cols, **opts, schedule="persistent")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pla = ctx.column_spectra(cols, **opts, schedule="plain")
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        same = all(bool(torch.equal(a, b)) for a, b in zip(per, pla))
        out["plain_sample"] = {"columns": int(cols.size),
                               "plain_columns_per_s": cols.size / t_plain,
                               "bitwise_equal_to_persistent": same}
        out["speedup_vs_plain"] = out["fwd_columns_per_s"] / (cols.size / t_plain)
    del ctx
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    out["wall_s"] = time.perf_counter() - t_gen
    return out


def main(argv=None):
    args = parse(argv)
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (one MI355X); --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        return 2
    import numpy as np

    import gen

    key = int(args.config) if args.config.isdigit() else args.config
    s = gen.make(key, nu=args.nu)
    print(f"# workload {s.name}: {s.n_atoms} atoms, {4 * s.n_atoms} columns, nu {s.nu}",
          file=sys.stderr, flush=True)
    # the oracle's CPU leg runs first, before anything here initialises the GPU
    cpu = None if args.no_cpu else cpu_baseline(s, args.cpu_seconds)
    import torch

    from paper_1210_1531_amd import Context, model
    torch.cuda.init()
    ctx, pos, sk, setup = build_context(Context, model, s, torch)
    st0 = ctx.stats()
    opts = dict(nu=s.nu, kT=s.kT, n_electrons=s.n_electrons, workflow=args.workflow,
                schedule=args.schedule)
    M = 4 * s.n_atoms

    def step():
        ctx.solve(**opts)
        ctx.backward(1.0)
        ctx.forces(sk)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kry_ms, kry_launch = 0.0, 0
    for _ in range(args.steps):
        step()
        st = ctx.stats()
        kry_ms += st["t_krylov_ms"]
        kry_launch += st["krylov_launches"]
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    print(f"# fwd+bwd {ms_step:.3f} ms/step", file=sys.stderr, flush=True)

    # forward only
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.solve(**opts)
    torch.cuda.synchronize()
    ms_fwd = (time.perf_counter() - t0) * 1e3 / args.steps
    st = ctx.stats()
    energy = ctx.energy()
    mu0 = ctx.solve(**opts)[0]
    rho_ref = ctx.density_matrix()[0].clone()
    eps_ref = ctx.spectra()[0].clone()

    # the memory-saving workflow (Krylov columns recomputed in pass 2)
    rec = None
    if st["workflow_used"] != 0:
        ropts = dict(opts, workflow="recompute")
        ctx.solve(**ropts)
        ctx.backward(1.0)
        torch.cuda.synchronize()
        n_rec = max(1, args.steps // 2)
        t0 = time.perf_counter()
        for _ in range(n_rec):
            ctx.solve(**ropts)
            ctx.backward(1.0)
            ctx.forces(sk)
        torch.cuda.synchronize()
        rec = M / ((time.perf_counter() - t0) / n_rec)

    # the forward solve captured in a HIP graph and replayed (when not the headline)
    graph = None
    if args.schedule != "graph":
        gopts = dict(opts, schedule="graph")
        ctx.solve(**gopts)  # eager solve + capture
        ctx.solve(**gopts)
        ctx.backward(1.0)
        ctx.forces(sk)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.solve(**gopts)
            ctx.backward(1.0)
            ctx.forces(sk)
        torch.cuda.synchronize()
        graph = M / ((time.perf_counter() - t0) / args.steps)

    # plain per-column launches (forward), and their rho against the
    # persistent launch's, bit for bit
    plain, plain_same = None, None
    if not args.no_plain:
        ctx.solve(**dict(opts, schedule="plain"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mu_p = ctx.solve(**dict(opts, schedule="plain"))[0]
        torch.cuda.synchronize()
        plain = M / (time.perf_counter() - t0)
        plain_same = (mu_p == mu0 and bool(torch.equal(ctx.spectra()[0], eps_ref))
                      and bool(torch.equal(ctx.density_matrix()[0], rho_ref)))

    nu = s.nu
    t_k = kry_ms / max(kry_launch, 1)
    roof = krylov_roofline(ctx, s, st0 | {"krylov_cache_blocks": st["krylov_cache_blocks"]}, t_k,
                           max(1, kry_launch // args.steps))
    roof["traffic"] = measured_traffic()
    # FP64 work of the same kernel: SpMV 4 nu nnz_C per column, Gram-Schmidt and
    # projection 10 n_C (k+1) per step k
    ptr, _atoms = ctx.get_clusters()
    nC = 4 * np.diff(ptr.cpu().numpy() if hasattr(ptr, "cpu") else ptr)
    flops_pass = 4.0 * nu * st0["sum_cluster_nnz"] * 4 + 4 * float(np.sum(5.0 * nC * nu * (nu + 1)))
    fp64_tflops = flops_pass / (kry_ms / args.steps * 1e-3) / 1e12
    roof["fp64_tflops"] = fp64_tflops
    roof["fp64_frac"] = fp64_tflops / FP64_PEAK_TFLOPS
    if roof["traffic"]:
        roof["hbm_measured_GBs"] = roof["traffic"] / (t_k * 1e-3) / 1e9
        roof["hbm_measured_frac"] = roof["hbm_measured_GBs"] / HBM_PEAK_GBS
    roof = {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")} | {
        k: v for k, v in roof.items() if k not in ("bound", "achieved", "peak", "unit", "frac",
                                                   "traffic")}

    out = {
        "metric": METRIC,
        "value": M / (ms_step * 1e-3),
        "unit": "columns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{s.name}: {s.meta['cells'][0]}x{s.meta['cells'][1]}x{s.meta['cells'][2]} "
                        f"diamond carbon cells, {s.n_atoms} atoms, SK sp model, "
                        f"r_cluster {s.r_cluster} A, nu {nu}, kT {s.kT} eV",
            "n_atoms": s.n_atoms,
            "columns": M,
            "nu": nu,
            "schedule": args.schedule,
            "workflow": args.workflow,
            "workflow_used": {0: "recompute", 1: "store"}[st["workflow_used"]],
            "krylov_buckets": st["krylov_buckets"],
            "krylov_threads": st["krylov_tpb"],
            "autotune_ms": st["autotune_ms"],
            "step": "fwd (pass 1 + mu + energy) + bwd (pass 2 rho/pi + forces through rho)",
        },
        "krylov_plans": launch_plans(st),
        "fwd_columns_per_s": M / (ms_fwd * 1e-3),
        "fwdbwd_recompute_columns_per_s": rec,
        "fwdbwd_graph_columns_per_s": graph,
        "fwd_ms": ms_fwd,
        "plain_fwd_columns_per_s": plain,
        "plain_rho_bitwise_equal": plain_same,
        "fwd_speedup_vs_plain": (M / (ms_fwd * 1e-3)) / plain if plain else None,
        "stage_ms": {"pass1": st["t_pass1_ms"], "krylov": st["t_krylov_ms"],
                     "eig": st["t_eig_ms"], "mu_energy": st["t_mu_ms"],
                     "pass2": st["t_pass2_ms"], "forces": st["t_forces_ms"]},
        "check": {"N_minus_Ne": energy["N"] - s.n_electrons, "E_band": energy["E_band"],
                  "A_free": energy["A_free"]},
        "roofline": roof,
    }
    _, _, nu_eff = ctx.spectra()
    nu_eff = nu_eff.cpu().numpy() if hasattr(nu_eff, "cpu") else np.asarray(nu_eff)
    out["setup_ms"] = setup
    out["nu_eff"] = {"min": int(nu_eff.min()), "mean": float(nu_eff.mean()),
                     "max": int(nu_eff.max())}
    out["device_bytes"] = int(ctx.stats()["device_bytes"])

    # the exact gradient of the truncated method (fwd + exact bwd), and
    # central differences of the grand potential at fixed mu on eight atoms
    # (h = 1e-5 and 2e-5 A, Richardson) against both kinds of forces
    if not args.no_exact:
        # forward + exact backward: the solve keeps every column's pass-1 data
        # (keep_exact), so the exact gradient needs no second Krylov pass
        ctx.solve(**opts)
        ctx.forces_exact(sk)  # with its own pass: the figure without keeping
        t_own = ctx.stats()["t_forces_exact_ms"]
        ctx.solve(keep_exact=True, **opts)
        Fx = ctx.forces_exact(sk)
        torch.cuda.synchronize()
        n_ex = max(1, args.steps // 2)
        t0 = time.perf_counter()
        for _ in range(n_ex):
            mu_x = ctx.solve(keep_exact=True, **opts)[0]
            Fx = ctx.forces_exact(sk)
        torch.cuda.synchronize()
        ms_ex = (time.perf_counter() - t0) * 1e3 / n_ex
        t_kept = ctx.stats()["t_forces_exact_ms"]
        Fh = ctx.forces(sk).cpu().numpy()
        Fx = Fx.cpu().numpy()
        out["fwd_exact_bwd"] = {"columns_per_s": M / (ms_ex * 1e-3), "ms_per_step": ms_ex,
                                "exact_forces_ms": t_kept,
                                "exact_forces_with_own_pass_ms": t_own,
                                "max_F_exact_minus_F_rho": float(np.abs(Fx - Fh).max()),
                                "sum_F_exact": float(np.abs(Fx.sum(axis=0)).max())}
        atoms = np.sort(np.random.default_rng(4).choice(s.n_atoms, 8, replace=False))
        f1 = fd_forces(ctx, s, atoms, mu_x, 1e-5, torch)
        f2 = fd_forces(ctx, s, atoms, mu_x, 2e-5, torch)
        fr = (4.0 * f1 - f2) / 3.0
        out["fd"] = {"atoms": atoms.tolist(), "h": [1e-5, 2e-5], "richardson": True,
                     "max_F_exact_minus_FD": float(np.abs(Fx[atoms] - fr).max()),
                     "max_F_rho_minus_FD": float(np.abs(Fh[atoms] - fr).max()),
                     "max_F_FD": float(np.abs(fr).max())}
        ctx.solve(**opts)
    # ICOHP per block of the pattern (the next row after the hot path): one
    # thread per block, reading rho (128 B), the H block (128 B), the column
    # index and two positions, writing three values
    ctx.solve(**opts)  # the library's own workflow again (the last solve may have been another)
    ctx.icohp(sk)
    ic = []
    for _ in range(3):
        ctx.icohp(sk)
        ic.append(ctx.stats()["t_icohp_ms"])
    nblk = ctx.nnz // 16
    t_ic = sorted(ic)[1]
    out["icohp"] = {"ms": t_ic, "blocks": nblk,
                    "GB_per_s": nblk * (128 + 128 + 4 + 48 + 24) / (t_ic * 1e-3) / 1e9}
    # energy-resolved COHP on a 256-point grid (store workflow only): per
    # block 4 nu weights, then 4 nu Lorentzians per energy
    if st["workflow_used"] == 1:
        grid = np.linspace(-25.0, 25.0, 256)
        ctx.cohp(grid, 0.05)
        t_co = ctx.stats()["t_cohp_ms"]
        terms = nblk * grid.size * 4 * s.nu
        out["cohp"] = {"ms": t_co, "blocks": nblk, "energies": int(grid.size),
                       "G_terms_per_s": terms / (t_co * 1e-3) / 1e9}
    # COCG Green's-function columns (a second solver of Eq. 1) on a sample of
    # columns at four energies, to tolerance 1e-10 (one pass over the
    # cluster's blocks per step serves the four energies)
    if args.cocg_columns > 0:
        ncol = min(args.cocg_columns, M)
        ccols = np.arange(0, M, max(1, M // ncol))[:ncol].astype(np.int32)
        zc = np.array([-6.5 + 0.05j, -1.0 + 0.2j, 0.5 + 0.2j, 3.0 + 0.05j])
        _, _, its = ctx.cocg_columns(ccols, zc, tol=1e-10, max_iter=4000)
        t_cg = ctx.stats()["t_cocg_ms"]
        out["cocg"] = {"ms": t_cg, "columns": int(ncol), "energies": int(zc.size),
                       "steps_mean": float(np.mean(its)), "steps_max": int(np.max(its)),
                       "converged": bool(np.all(its > 0)),
                       "column_energies_per_s": ncol * zc.size / (t_cg * 1e-3)}
    # MD steps: velocity Verlet at 300 K, each step rebuilding H, S, pattern
    # and clusters, solving every column and taking the forces plus the pair
    # repulsion (one warm-up step first)
    if args.md_steps > 0:
        vel = torch.tensor(gen.random_velocities(s.n_atoms, model.thermal_sigma(300.0), 1),
                           dtype=torch.float64, device="cuda")
        md_kw = dict(r_cluster=s.r_cluster, **model.PAIR_REPULSION, **opts)
        kinds = [("md", False)] + ([] if args.no_exact else [("md_exact_forces", True)])
        for name, exact in kinds:
            ctx.md_run(sk, pos, vel, s.cell, 0.5, model.MASS_CARBON, 1, exact_forces=exact,
                       **md_kw)
            _, _, _, th = ctx.md_run(sk, pos, vel, s.cell, 0.5, model.MASS_CARBON, args.md_steps,
                                     exact_forces=exact, **md_kw)
            t_md = ctx.stats()["t_md_step_ms"]
            e_tot = th[:, 0] + th[:, 1]
            out[name] = {"ms_per_step": t_md, "steps": args.md_steps, "dt_fs": 0.5,
                         "columns_per_s": M / (t_md * 1e-3),
                         "E_tot_change_per_atom": float(e_tot[-1] - e_tot[0]) / s.n_atoms,
                         "E_tot_max_dev_per_atom": float(np.abs(e_tot - e_tot[0]).max())
                         / s.n_atoms,
                         "forces": "exact gradient of the truncated method" if exact
                         else "through rho and pi",
                         "step": "rebuild H, S, pattern, clusters + fwd + bwd + forces + pair "
                                 "term"}
    if args.copy_probe:
        a = torch.full((64 * 1024 * 1024,), 1.0, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    # the void cell at three Krylov dimensions and the million-site cell
    if not args.no_extra and key == 2:
        del ctx
        torch.cuda.synchronize()
        xs = max(2, min(args.steps, 5))
        out["void_cell"] = {f"nu{v}": extra_workload(3, v, Context, model, torch, xs, 1024)
                            for v in (20, 30, 40)}
        print("# void cell done", file=sys.stderr, flush=True)
        out["million_site_cell"] = extra_workload(5, None, Context, model, torch, 1, 0,
                                                  recompute=True)
        print("# million-site cell done", file=sys.stderr, flush=True)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
