"""Benchmark of the hot path on one MI355X.

Workload: a 200-chain x 1000-bead Kremer-Grest melt (200,000 monomers, rho = 0.85, L = 61.7 sigma),
kappa = 2, the softest core-softened pair potential (n = 2, FENE k_n of Eq. 9), Langevin
velocity Verlet with dt = 0.01 tau and gamma = 1/tau, seeded random-walk start.  One bench
"step" is one pass of the whole hot path: 100 MD steps followed by one double-bridging sweep of
round(1e-3 * 200000 * 100 * 0.01) = 200 attempts (the paper's attempt rate, one sweep every 100
steps).  The full 10^4-step run is 100 such steps.

The project form (FP32 forces, FP64 state/energies/Delta E) gives `value`; the plain FP64 path is
timed the same way on the same GPU and reported beside it.  The dominant kernel (the fused force
+ integrator kernel) is timed with HIP events on the library's stream over a profiled run of the
same workload; its algorithmic bytes per launch give the roofline figure.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "monomer-timesteps/s + DB moves accepted/s vs plain FP64 path, same GPU"
HBM_PEAK_GBS = 8000.0

WORKLOAD = dict(M=200, N=1000, rho=0.85, kappa=2.0, n_exp=2.0, k_fene=0.0, dt=0.01, gamma=1.0, T=1.0,
                seed=1, warmup_steps=1000)
MD_PER_STEP = 100


def step_kernel_bytes(mixed, mean_list):
    """Algorithmic bytes per monomer of one step-kernel launch (close + open).

    reads: position x (24), velocity v_half (24), own reference-relative position (16 mixed /
    32 FP64), its value at the last rebuild (16), reference cell (4), chain-table position (4),
    its chain-table entry (4), monomer id (4), list length (4) and list entries (4 each).
    writes: new x (24), new v_half (24), new relative position (16 / 32).  Neighbours' relative
    positions and bonded partners' positions are re-reads served from cache.
    """
    rel = 16 if mixed else 32
    reads = 24 + 24 + rel + 16 + 4 + 4 + 4 + 4 + 4 + 4 * mean_list
    writes = 24 + 24 + rel
    return reads + writes


def run_gpu(kg, precision, steps, warmup, stream, profile_steps):
    params = dict(WORKLOAD, precision=precision)
    t0 = time.perf_counter()
    b = kg.Batch([params], stream=stream)
    t_init = time.perf_counter() - t0
    nm, _ = b.sizes()
    K, tune_ms = b.autotune(0, reps=30)  # neighbour-list rebuild interval; state restored
    K = -1  # attempts from the rate: 1e-3 * N_mono * (100 dt)
    for _ in range(warmup):
        b.md_steps(MD_PER_STEP)
        b.db_sweep(K)
    import torch
    torch.cuda.synchronize()
    t_md = t_db = 0.0
    acc = att = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        b.md_steps(MD_PER_STEP)
        c = time.perf_counter()
        st = b.db_sweep(K)[0]
        d = time.perf_counter()
        t_md += c - a
        t_db += d - c
        acc += st["accepted"]
        att += st["attempts"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = dict(wall_s=wall, ms_per_step=1e3 * wall / steps, md_s=t_md, db_s=t_db,
               monomer_steps_per_s=nm * MD_PER_STEP * steps / wall,
               md_only_monomer_steps_per_s=nm * MD_PER_STEP * steps / t_md,
               db_accepted_per_s=acc / wall, db_attempts=att, db_accepted=acc,
               db_attempts_per_s_in_sweeps=att / t_db if t_db > 0 else None, init_s=t_init)
    # per-launch HIP-event timing of the fused force kernel (direct launches, same workload)
    if profile_steps > 0:
        b.profile(True)
        for _ in range(max(1, profile_steps // MD_PER_STEP)):
            b.md_steps(MD_PER_STEP)
            b.db_sweep(K)
        prof = b.profile_read()
        b.profile(False)
        out["force_kernel_ms"] = prof["force_ms"] / max(prof["force_n"], 1)
        out["finalize_kernel_ms"] = prof["finalize_ms"] / max(prof["force_n"], 1)  # rebuild time per step
        out["force_launches_timed"] = prof["force_n"]
    r2n, lk, mb = b.observables()
    out["nl"] = b.nl_info()
    out["tune_ms"] = {str(k_): round(v_, 5) for k_, v_ in tune_ms.items()}
    out["ell_K"] = lk
    out["mean_bond"] = mb
    out["monomers"] = nm
    b.close()
    return out


def cpu_baseline(md_steps=15, db_attempts=8):
    """The FP64 CPU oracle (single thread) on a bounded sample of the same workload."""
    from oracle import oracle as o
    m = o.Melt(**dict(WORKLOAD, warmup_steps=60))  # untimed setup: a shortened warm-up
    t0 = time.perf_counter()
    m.md_steps(md_steps)
    t1 = time.perf_counter()
    m.db_sweep(db_attempts)
    t2 = time.perf_counter()
    t_step = (t1 - t0) / md_steps
    t_att = (t2 - t1) / db_attempts
    nm = WORKLOAD["M"] * WORKLOAD["N"]
    K = round(1e-3 * nm * MD_PER_STEP * WORKLOAD["dt"])
    chunk = MD_PER_STEP * t_step + K * t_att
    return {"value": nm * MD_PER_STEP / chunk, "unit": "monomer-timesteps/s", "cores": 1, "kind": "oracle",
            "sample": f"200k-monomer workload melt: {md_steps} MD steps ({t_step:.3f} s each) and "
                      f"{db_attempts} DB attempts ({t_att:.3f} s each), scaled to one bench step of "
                      f"{MD_PER_STEP} MD steps + {K} attempts; single-threaded FP64 C oracle"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed bench steps (100 MD steps + 1 sweep each)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--profile-steps", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); melts shard across GPUs without any "
              "exchange, so the per-GPU figure is the single-GPU one", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2109_11001_amd as kg
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    print(f"[bench] mixed path: {args.warmup} warm-up + {args.steps} timed steps", file=sys.stderr, flush=True)
    mixed = run_gpu(kg, kg.PREC_MIXED, args.steps, args.warmup, stream, args.profile_steps)
    print(f"[bench] mixed done: {mixed['monomer_steps_per_s']:.3e} monomer-steps/s", file=sys.stderr, flush=True)
    fp64 = None
    if not args.no_fp64:
        fp64 = run_gpu(kg, kg.PREC_FP64, args.steps, args.warmup, stream, args.profile_steps)
        print(f"[bench] fp64 done: {fp64['monomer_steps_per_s']:.3e} monomer-steps/s", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline()

    roof = None
    if "force_kernel_ms" in mixed:
        bpm = step_kernel_bytes(True, mixed["nl"]["mean_list"])
        bytes_launch = bpm * mixed["monomers"]
        achieved = bytes_launch / (mixed["force_kernel_ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": "k_nl_step<float, close|open> (list forces + bonded + Langevin VV)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "bytes_per_monomer": round(bpm, 1), "avg_launch_ms": mixed["force_kernel_ms"],
                "launches": mixed["force_launches_timed"], "neighbour_lists": mixed["nl"],
                "autotune_ms_per_step_by_K": mixed["tune_ms"],
                "rebuild_ms_per_step": mixed.get("finalize_kernel_ms")}
    line = {
        "metric": METRIC,
        "value": mixed["monomer_steps_per_s"],
        "unit": "monomer-timesteps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 forces / f64 state",
        "data": "synthetic (seeded random-walk melt, warm-up, no dataset)",
        "config": {"workload": "KG melt 200 chains x 1000 beads, rho 0.85, kappa 2, n 2 (k_n), dt 0.01, "
                               "gamma 1; step = 100 MD steps + 1 DB sweep of 200 attempts",
                   "monomers": mixed["monomers"], "md_steps_per_step": MD_PER_STEP,
                   "db_attempts_per_step": mixed["db_attempts"] // max(args.steps, 1)},
        "db_accepted_per_s": mixed["db_accepted_per_s"],
        "md_only_monomer_steps_per_s": mixed["md_only_monomer_steps_per_s"],
        "time_split_s": {"md": round(mixed["md_s"], 4), "db": round(mixed["db_s"], 4)},
        "rebuild_ms_per_md_step": mixed.get("finalize_kernel_ms"),
    }
    if fp64:
        line["fp64_path"] = {"value": fp64["monomer_steps_per_s"], "ms_per_step": fp64["ms_per_step"],
                             "db_accepted_per_s": fp64["db_accepted_per_s"],
                             "force_kernel_ms": fp64.get("force_kernel_ms")}
        line["speedup_vs_fp64_path"] = mixed["monomer_steps_per_s"] / fp64["monomer_steps_per_s"]
    line["roofline"] = roof
    line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
