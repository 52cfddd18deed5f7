"""Benchmark of the hot path on one MI355X.

Workload: a 200-chain x 1000-bead Kremer-Grest melt (200,000 monomers, rho = 0.85, L = 61.7 sigma),
kappa = 2, the softest core-softened pair potential (n = 2, FENE k_n of Eq. 9), Langevin
velocity Verlet with dt = 0.01 tau and gamma = 1/tau, seeded random-walk start.  One bench
"step" is one pass of the whole hot path: 100 MD steps followed by one double-bridging sweep of
round(1e-3 * 200000 * 100 * 0.01) = 200 attempts (the paper's attempt rate, one sweep every 100
steps).  The full 10^4-step run is 100 such steps.

The project form (FP32 forces, FP64 state/energies/Delta E) gives `value`; the plain FP64 path is
timed the same way on the same GPU and reported beside it.  The dominant kernel (the fused force
+ integrator kernel) is timed with HIP events on the library's stream over a profiled pass of the
same length as the timed region, run right after it (direct launches, since events cannot
bracket single kernels inside a replayed graph); its algorithmic bytes per launch give the
roofline figure.  The learned-proposal form runs on the same system at kappa = 2.5: a network is
trained on the GPU from logged uniform sweeps (untimed set-up), then the same bench steps are
timed with the learned and with the uniform proposal from one shared state.
"""
import hashlib
import math

import numpy as np
import re
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
LEARNED_KAPPA = 2.5


def algorithmic_bytes(mixed):
    """Bytes per monomer that one fused force + integrator step must move (the pair, bond and
    angle forces and the Langevin velocity-Verlet update of one monomer): pair 36 (own position
    16 / 24 FP64, cell bounds 6, force 12-16 / 24), bond + angle fused with it 20, integrator
    112 / 120 (x and v in FP64 read and written, the force, the FP32 copy).  Neighbour re-reads
    are served from LDS or cache and are not counted.  168 B mixed, 196 B plain FP64."""
    return 168.0 if mixed else 196.0


def implementation_bytes(mixed, mean_list, K, staged_per_monomer):
    """Bytes per monomer one launch of this implementation's step kernel moves in its own
    layout, averaged over the K steps of a rebuild interval.

    reads: position x (24), velocity v_half (24), own relative position (16: fixed point with
    FP32 forces; 32 FP64), monomer id (4), chain neighbours' slots (16), list length (4), list
    entries (2 each, 16-bit indices into the workgroup's LDS stage) and the recorded slots of
    the tile's stage (4 per staged member: staged_per_monomer of them per home monomer).
    writes: new x (24), new v_half (24), new relative position (16 / 32); on the step before a
    rebuild also the bucket entry (4, 4/K per launch on average).  The staged positions (the
    tile and its halo: every cell's are re-read by ~5 tiles) and the chain neighbours'
    positions are re-reads served from cache.
    """
    rel = 16 if mixed else 32
    reads = 24 + 24 + rel + 4 + 16 + 4 + 2 * mean_list + 4 * staged_per_monomer
    writes = 24 + 24 + rel + 4.0 / K
    return reads + writes


def run_gpu(kg, precision, steps, warmup, stream, profile_steps, keep_state=False):
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
        for _ in range(max(1, profile_steps)):
            b.md_steps(MD_PER_STEP)
            b.db_sweep(K)
        prof = b.profile_read()
        b.profile(False)
        out["force_kernel_ms"] = prof["force_ms"] / max(prof["force_n"], 1)
        out["finalize_kernel_ms"] = prof["finalize_ms"] / max(prof["force_n"], 1)  # rebuild time per step
        out["force_launches_timed"] = prof["force_n"]
    r2n, lk, mb = b.observables()
    M_, N_ = WORKLOAD["M"], WORKLOAD["N"]
    out["fene_floored_frac"] = b.fene_floored() / max(1, b.counters()[0] * M_ * (N_ - 1))
    out["nl"] = b.nl_info()
    out["lds_stage"] = b.nl_stats()
    out["tune_ms"] = {str(k_): round(v_, 5) for k_, v_ in tune_ms.items()}
    out["ell_K"] = lk
    out["mean_bond"] = mb
    out["monomers"] = nm
    if keep_state:
        out["state"] = b.get_state()
    b.close()
    return out


def run_size(kg, monomers, md_steps, stream, precision):
    """Step kernel on one melt of `monomers` monomers (N = 1000 beads per chain, or 2000 where
    that would exceed the 8192 chains a melt may hold; rho = 0.85, the workload's potentials):
    `md_steps` MD steps timed end to end, then as many again with the step kernel timed by
    events.  From 1M monomers up the per-step state no longer fits the 256 MB last-level cache,
    so the roofline figure is then set by HBM.  Then the same number of bench steps with a
    double-bridging sweep after every 100 MD steps at the paper's attempt rate (lists beyond
    3072 keys are swept from global memory)."""
    import torch
    N = WORKLOAD["N"]
    while monomers // N > 8192:
        N *= 2
    params = dict(WORKLOAD, M=monomers // N, N=N, precision=precision)
    t0 = time.perf_counter()
    b = kg.Batch([params], stream=stream)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    nm, _ = b.sizes()
    for _ in range(2):  # past the first calls after the warm-up, whose list builds run slower
        b.md_steps(MD_PER_STEP)
    K, tune_ms = b.autotune(0, reps=20)
    b.md_steps(MD_PER_STEP)
    torch.cuda.synchronize()
    chunks = max(1, md_steps // MD_PER_STEP)  # calls of MD_PER_STEP steps, as in a bench step
    t0 = time.perf_counter()
    for _ in range(chunks):
        b.md_steps(MD_PER_STEP)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    b.profile(True)
    for _ in range(chunks):
        b.md_steps(MD_PER_STEP)
    prof = b.profile_read()
    b.profile(False)
    nl = b.nl_info()
    st = b.nl_stats()
    att = acc = 0
    t_db = 0.0
    t0 = time.perf_counter()
    for _ in range(chunks):
        b.md_steps(MD_PER_STEP)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s_ = b.db_sweep(-1)[0]
        torch.cuda.synchronize()
        t_db += time.perf_counter() - t1
        att += s_["attempts"]
        acc += s_["accepted"]
    wall_sw = time.perf_counter() - t0
    ncand = s_["ncand_end"]
    b.close()
    ms = prof["force_ms"] / max(prof["force_n"], 1)
    mixed = precision == kg.PREC_MIXED
    bpm = algorithmic_bytes(mixed)
    ibpm = implementation_bytes(mixed, nl["mean_list"], nl["K"], st["staged_per_monomer"])
    achieved = bpm * nm / (ms * 1e-3) / 1e9
    return {"monomers": nm, "chains": nm // N, "beads_per_chain": N, "md_steps": chunks * MD_PER_STEP,
            "monomer_steps_per_s": nm * chunks * MD_PER_STEP / wall, "avg_launch_ms": ms,
            "launches": prof["force_n"], "rebuild_ms_per_step": prof["finalize_ms"] / max(prof["force_n"], 1),
            "bytes_per_monomer": bpm, "achieved_GBs": round(achieved, 1),
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "implementation_bytes_per_monomer": round(ibpm, 1),
            "implementation_GBs": round(ibpm * nm / (ms * 1e-3) / 1e9, 1), "K": nl["K"], "mean_list": nl["mean_list"],
            "rollbacks": nl["rollbacks"], "skin": round(nl["skin"], 4),
            "autotune_ms_per_step_by_K": {str(k_): round(v_, 5) for k_, v_ in tune_ms.items()},
            "lds_stage": st, "init_s": round(t_init, 2),
            "with_sweeps": {"monomer_steps_per_s": nm * chunks * MD_PER_STEP / wall_sw,
                            "sweep_ms": round(1e3 * t_db / chunks, 3), "attempts": att, "accepted": acc,
                            "candidates": ncand}}


def train_proposal(kg, b, stream, log_sweeps, log_attempts, train_steps):
    """Log `log_sweeps` uniform sweeps of `log_attempts` attempts (100 MD steps before each) on
    melt 0 of batch `b`, then train a network on them on the GPU (full-batch Adam)."""
    import torch
    feats, labs = [], []
    for _ in range(log_sweeps):
        b.md_steps(MD_PER_STEP)
        st, f, lab, nl = b.db_sweep_log(log_attempts, cap=log_attempts)
        feats.append(f[0, : nl[0]].clone())
        labs.append(lab[0, : nl[0]].clone())
    x = torch.cat(feats)
    y = torch.cat(labs)
    from tests.inputs import random_mlp_params  # seeded initial weights (no method arithmetic)
    tr = kg.Trainer(random_mlp_params(3, w_scale=0.1, b_scale=0.1), max_batch=len(y), lr=3e-3, stream=stream)
    with torch.cuda.stream(stream):
        first = float(tr.step(x, y).cpu()[0])
        for _ in range(train_steps - 1):
            loss = tr.step(x, y)
        last = float(loss.cpu()[0])
    torch.cuda.synchronize()
    return tr, first, last, y


# Training logs for the learned proposal: uniform sweeps on the systems of the plain-method,
# precision-form, stiff and batched workloads (name, melts, sweeps, attempts per sweep), with
# 100 MD steps before each sweep.  The network is then evaluated on the 200 x 1000 melt at
# kappa = 2.5, a stiffness it met only in the batched melts.
TRAIN_SOURCES = (
    ("20 x 50, kappa 1.5", [dict(M=20, N=50, kappa=1.5)], 40, 100),
    ("200 x 1000, kappa 2", [dict(M=200, N=1000, kappa=2.0)], 6, 2000),
    ("100 x 2000, kappa 3", [dict(M=100, N=2000, kappa=3.0)], 6, 2000),
    ("6 melts of 125 x 200, kappa 0-2.5", [dict(M=125, N=200, kappa=k_) for k_ in (0.0, 0.5, 1.0, 1.5, 2.0, 2.5)],
     10, 300),
)


def log_training_sources(kg, stream):
    """Features and accept labels of uniform sweeps on every system of TRAIN_SOURCES."""
    import torch
    feats, labs, meta = [], [], []
    for name, melts, sweeps, attempts in TRAIN_SOURCES:
        b = kg.Batch([dict(WORKLOAD, precision=kg.PREC_MIXED, **m) for m in melts], stream=stream)
        nrec = nacc = 0
        for _ in range(sweeps):
            b.md_steps(MD_PER_STEP)
            _, f, lab, nl = b.db_sweep_log(attempts, cap=attempts)
            for k in range(len(melts)):
                feats.append(f[k, : nl[k]].clone())
                labs.append(lab[k, : nl[k]].clone())
                nrec += int(nl[k])
                nacc += int(lab[k, : nl[k]].sum())
        b.close()
        meta.append({"system": name, "melts": len(melts), "records": nrec, "accept_rate": round(nacc / max(nrec, 1), 4)})
    return torch.cat(feats), torch.cat(labs), meta


def run_learned(kg, steps, warmup, stream, train_steps=300):
    """Learned vs uniform proposal on the 200 x 1000 melt at kappa = 2.5 (mixed precision), the
    network trained on logs of the other workloads' systems (TRAIN_SOURCES)."""
    import torch
    params = dict(WORKLOAD, precision=kg.PREC_MIXED, kappa=LEARNED_KAPPA)
    # set-up (untimed): logged uniform sweeps on the training systems, training on the GPU
    t0 = time.perf_counter()
    x, y, sources = log_training_sources(kg, stream)
    from tests.inputs import random_mlp_params  # seeded initial weights (no method arithmetic)
    tr = kg.Trainer(random_mlp_params(3, w_scale=0.1, b_scale=0.1), max_batch=len(y), lr=3e-3, stream=stream)
    with torch.cuda.stream(stream):
        first = float(tr.step(x, y).cpu()[0])
        for _ in range(train_steps - 1):
            loss = tr.step(x, y)
        last = float(loss.cpu()[0])
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    b = kg.Batch([params], stream=stream)
    for _ in range(2):
        b.md_steps(MD_PER_STEP)
    state = b.get_state()
    b.close()
    out = {"kappa": LEARNED_KAPPA, "train_sources": sources, "train_records": int(len(y)),
           "train_accept_rate": float(y.float().mean()), "train_steps": train_steps, "loss_first": first,
           "loss_last": last, "setup_s": round(setup_s, 2)}
    for name, prop in (("uniform", kg.PROPOSAL_UNIFORM), ("learned", kg.PROPOSAL_LEARNED)):
        g = kg.Batch([dict(params, warmup_steps=0, proposal=prop)], stream=stream)
        g.set_state(0, x=state["x"], v=state["v"], fl=state["fl"], chains=state["chains"],
                    counters=state["counters"])
        g.autotune(0, reps=20)
        if prop == kg.PROPOSAL_LEARNED:
            g.set_proposal_net(tr.params, 0.1)
        for _ in range(warmup):
            g.md_steps(MD_PER_STEP)
            g.db_sweep(-1)
        torch.cuda.synchronize()
        acc = att = 0
        t_db = 0.0
        a0 = time.perf_counter()
        for _ in range(steps):
            g.md_steps(MD_PER_STEP)
            c = time.perf_counter()
            st = g.db_sweep(-1)[0]
            t_db += time.perf_counter() - c
            acc += st["accepted"]
            att += st["attempts"] - st["no_candidate"]
        torch.cuda.synchronize()
        wall = time.perf_counter() - a0
        nm, _ = g.sizes()
        out[name] = {"monomer_steps_per_s": nm * MD_PER_STEP * steps / wall, "db_accepted_per_s": acc / wall,
                     "accept_rate": acc / max(att, 1), "db_accepted_per_sweep_s": acc / t_db if t_db > 0 else None,
                     "db_s": round(t_db, 4), "attempts": att}
        g.close()
    out["accepted_per_s_gain"] = out["learned"]["db_accepted_per_s"] / max(out["uniform"]["db_accepted_per_s"], 1e-30)
    return out


EQ_SYSTEM = dict(M=2000, N=25, kappa=2.0)  # 50,000 monomers: short chains equilibrate within a run


def _steps_to_within(times, samples, ref, tol):
    """First sample time from which the mean of the samples over the second half of the elapsed
    run, (t/2, t], stays within `tol` (relative) of `ref` for every n; None if it never does."""
    import numpy as np
    t = np.asarray(times, float)
    S = np.asarray(samples)
    dev = []
    for k in range(len(t)):
        w = (t > t[k] / 2) & (t <= t[k])
        dev.append(float(np.max(np.abs(S[w].mean(0) - ref) / ref)))
    bad = [k for k, d in enumerate(dev) if d > tol]
    first = (bad[-1] + 1) if bad else 0
    return (None if first >= len(t) else first), dev


EQ_FORMS = ("fp64", "mixed", "batched", "learned", "mixed_fr")
# the default line's time-to-equilibrium check: one seed, shorter runs than the study above
EQ_CHECK = dict(steps=200_000, ref_steps=500_000, forms=("fp64", "mixed", "learned"))


def run_equilibration(kg, stream, steps, ref_steps, every=1000, tol=0.02, batch_melts=4, seeds=(1,),
                      forms=EQ_FORMS, ref_seed=101):
    """Time to equilibrium of R^2(n)/n for each form, from warmed-up starts of several seeds.

    The reference is the plain FP64 path with the uniform proposal, started from a random-walk
    start of its own (seed `ref_seed`, so its start and random stream are shared with no form),
    its R^2(n)/n averaged over the second half of a run of `ref_steps` steps.  For every seed,
    each form (plain FP64, mixed precision, a batch of `batch_melts` melts with their own random
    streams, the learned proposal) runs `steps` steps from that seed's warmed-up start, one sweep
    at the paper's rate every 100 steps, R^2(n)/n read every `every` steps; a form has
    equilibrated once the mean over the second half of its run so far stays within `tol` of the
    reference for every n.  Wall-clock times include the sweeps and the readings.  One more form,
    mixed precision from freely rotating chains (Sec. II.B) instead of the shared random-walk
    start, measures what the better initial state saves.  The learned proposal's network is
    trained on uniform sweeps logged from a copy of the reference's start."""
    import numpy as np
    import torch

    def base_of(seed):
        return dict(WORKLOAD, **EQ_SYSTEM, seed=seed)

    def warm_start(seed):
        g = kg.Batch([dict(base_of(seed), precision=kg.PREC_FP64)], stream=stream)
        S = g.get_state()
        g.close()
        return S

    def start(form, seed, S0):
        melts = batch_melts if form == "batched" else 1
        prec = kg.PREC_FP64 if form == "fp64" else kg.PREC_MIXED
        prop = kg.PROPOSAL_LEARNED if form == "learned" else kg.PROPOSAL_UNIFORM
        if form == "mixed_fr":  # its own start: freely rotating chains (Sec. II.B), then the warm-up
            return kg.Batch([dict(base_of(seed), precision=prec, init_mode=kg.INIT_FREELY_ROTATING)],
                            stream=stream), 1
        b = kg.Batch([dict(base_of(seed), warmup_steps=0, precision=prec, proposal=prop, melt_id=i)
                      for i in range(melts)], stream=stream)
        for i in range(melts):
            b.set_state(i, x=S0["x"], v=S0["v"], fl=S0["fl"], chains=S0["chains"], counters=S0["counters"])
        return b, melts

    def run(form, seed, S0, nsteps, net=None):
        b, melts = start(form, seed, S0)
        if net is not None:
            b.set_proposal_net(net, 0.1)
        b.autotune(0, reps=20)
        times, walls, samples = [], [], []
        acc = att = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = 0
        while s < nsteps:
            for _ in range(every // MD_PER_STEP):
                b.md_steps(MD_PER_STEP)
                for st in b.db_sweep(-1):
                    acc += st["accepted"]
                    att += st["attempts"] - st["no_candidate"]
            s += every
            samples.append(np.mean([b.observables(i)[0] for i in range(melts)], axis=0))
            times.append(s)
            walls.append(time.perf_counter() - t0)
        floored = sum(b.fene_floored(i) for i in range(melts))
        bond_steps = sum(b.counters(i)[0] for i in range(melts)) * EQ_SYSTEM["M"] * (EQ_SYSTEM["N"] - 1)
        b.close()
        print(f"[bench] equilibration: {form}, seed {seed}, {nsteps} steps in {walls[-1]:.1f} s",
              file=sys.stderr, flush=True)
        return dict(times=times, walls=walls, samples=samples, accepted=acc, attempts=att, melts=melts,
                    floored=floored / max(bond_steps, 1))

    out = {"system": f"{EQ_SYSTEM['M']} chains x {EQ_SYSTEM['N']} beads, kappa {EQ_SYSTEM['kappa']}, n 2, "
                     "rho 0.85, dt 0.01, gamma 1", "tolerance": tol, "reading_every_steps": every,
           "seeds": list(seeds), "forms": {}}
    S_ref = warm_start(ref_seed)
    r = run("fp64", ref_seed, S_ref, ref_steps)
    half = np.asarray(r["times"]) > ref_steps / 2
    ref = np.asarray(r["samples"])[half].mean(0)
    out["reference"] = {"seed": ref_seed, "steps": ref_steps, "r2n_first": float(ref[0]),
                        "r2n_last": float(ref[-1]), "r2n_max": float(ref.max()),
                        "wall_s": round(r["walls"][-1], 3)}
    net = None
    if "learned" in forms:  # a network trained on logged uniform sweeps of a copy of the reference's start
        b, _ = start("fp64", ref_seed, S_ref)
        t0 = time.perf_counter()
        tr, first, last, y = train_proposal(kg, b, stream, 10, 2000, 300)
        out["learned_training"] = {"records": int(len(y)), "loss_first": first, "loss_last": last,
                                   "setup_s": round(time.perf_counter() - t0, 2)}
        b.close()
        net = tr.params
    per = {f: [] for f in forms}
    for seed in seeds:
        S0 = warm_start(seed)
        for form in forms:
            r = run(form, seed, S0, steps, net=net if form == "learned" else None)
            k, dev = _steps_to_within(r["times"], r["samples"], ref, tol)
            per[form].append({
                "seed": seed, "melts": r["melts"], "steps": r["times"][-1], "wall_s": round(r["walls"][-1], 3),
                "us_per_md_step": round(1e6 * r["walls"][-1] / r["times"][-1], 2),
                "steps_to_tol": r["times"][k] if k is not None else None,
                "tau_to_tol": r["times"][k] * WORKLOAD["dt"] if k is not None else None,
                "wall_s_to_tol": round(r["walls"][k], 3) if k is not None else None,
                "max_dev_end": round(dev[-1], 5), "max_dev_start": round(dev[0], 4),
                "accepted": r["accepted"], "accept_rate": r["accepted"] / max(r["attempts"], 1),
                "fene_floored_per_bond_step": r["floored"]})
    for form, rs in per.items():
        reached = [x for x in rs if x["steps_to_tol"] is not None]
        mean = lambda key, xs: (float(np.mean([x[key] for x in xs])) if xs else None)
        out["forms"][form] = {
            "reached": f"{len(reached)} of {len(rs)}",
            "steps_to_tol_mean": mean("steps_to_tol", reached),
            "wall_s_to_tol_mean": mean("wall_s_to_tol", reached),
            "us_per_md_step_mean": mean("us_per_md_step", rs),
            "accept_rate_mean": mean("accept_rate", rs),
            "max_dev_end_max": max(x["max_dev_end"] for x in rs),
            "per_seed": rs}
    return out


PAPER_SYSTEM = dict(M=1000, N=400, dt=0.008)  # the paper's melts: 1000 chains of 400 beads, dt = tau / 125


BATCH_KAPPAS = (0.0, 0.5, 1.0, 1.5, 2.0, 2.5)
BATCH_SHAPES = ((225, 100), (125, 200), (75, 400), (50, 800))  # (chains, beads): 22.5k-40k monomers


def run_batch(kg, stream, steps, warmup, single_steps=10):
    """24 uneven melts (every kappa of BATCH_KAPPAS with every shape of BATCH_SHAPES, 705,000
    monomers) advanced as one batch: bench steps of 100 MD steps and one sweep per melt at the
    attempt rate.  The same melts are then run one batch of one at a time for `single_steps`
    bench steps each, for the gain of batching."""
    import torch
    melts = [dict(WORKLOAD, M=M, N=N, kappa=kap, melt_id=i, precision=kg.PREC_MIXED)
             for i, (kap, (M, N)) in enumerate((k_, s_) for k_ in BATCH_KAPPAS for s_ in BATCH_SHAPES)]
    t0 = time.perf_counter()
    b = kg.Batch(melts, stream=stream)
    K, _ = b.autotune(0, reps=20)
    setup_s = time.perf_counter() - t0
    nm, _ = b.sizes()
    for _ in range(warmup):
        b.md_steps(MD_PER_STEP)
        b.db_sweep(-1)
    torch.cuda.synchronize()
    acc = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        b.md_steps(MD_PER_STEP)
        acc += sum(x["accepted"] for x in b.db_sweep(-1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    b.close()
    seq = 0.0
    for m in melts:
        g = kg.Batch([m], stream=stream)
        g.autotune(0, reps=20)
        g.md_steps(MD_PER_STEP)
        g.db_sweep(-1)
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        for _ in range(single_steps):
            g.md_steps(MD_PER_STEP)
            g.db_sweep(-1)
        torch.cuda.synchronize()
        seq += (time.perf_counter() - a0) / single_steps
        g.close()
    return {"workload": "24 melts, kappa in {0, 0.5, 1, 1.5, 2, 2.5} x (chains, beads) in {(225, 100), "
                        "(125, 200), (75, 400), (50, 800)}, rho 0.85, n 2, mixed precision; bench step = 100 MD "
                        "steps (hipGraph chunks) + one sweep per melt at the attempt rate",
            "melts": len(melts), "monomers": nm, "rebuild_interval": K, "setup_s": round(setup_s, 2),
            "ms_per_bench_step": round(1e3 * wall / steps, 3), "monomer_steps_per_s": nm * MD_PER_STEP * steps / wall,
            "db_accepted_per_s": acc / wall,
            "one_at_a_time_ms_per_bench_step": round(1e3 * seq, 3),
            "batching_gain": round(seq / (wall / steps), 2)}


def batch_form(kg, stream, steps, warmup):
    """run_batch with progress lines."""
    print("[bench] batched form: 24 uneven melts in one batch, then one at a time", file=sys.stderr, flush=True)
    bat = run_batch(kg, stream, steps, warmup)
    print(f"[bench] batch: {bat['monomer_steps_per_s']:.3e} monomer-steps/s, gain {bat['batching_gain']}",
          file=sys.stderr, flush=True)
    return bat


def kg_kuhn(kappa):
    """l_K / l_0 of Eq. 12 (for the report only)."""
    x = 2.0 * kappa
    flory = 1.0 if kappa == 0 else (x + math.exp(-x) - 1.0) / (1.0 - math.exp(-x) * (x + 1.0))
    return flory + 0.77 * (math.tanh(-0.03 * kappa ** 2 - 0.41 * kappa + 0.16) + 1.0)


XI = (2.0, 3.0, 4.0, 5.0, 5.75, 6.5, 7.0, 8.0, 9.0, 10.0, 11.0, 12.0)  # the exponents of Eq. 11


def success_fits(kappa, n):
    """The paper's two fits of the swap success rate: Eq. 15, a exp(-b kappa - d n), and the
    Fig. 3 caption's a' exp(-b' kappa - d' n - e' n^2)."""
    return (1.6 * math.exp(-0.77 * kappa - 0.35 * n),
            1.24 * math.exp(-0.77 * kappa - 0.24 * n - 0.015 * n * n))


def wlc_r2_over_n(n, ell_k, l0):
    """<R^2(n)> / n of the worm-like chain (Eq. 14) for Kuhn length ell_k and bond length l0."""
    x = 2.0 * n * l0 / ell_k
    return l0 * ell_k * (1.0 - (1.0 - math.exp(-x)) / x)


def run_config2(kg, stream, steps_per_n=20000, sweep_every=50):
    """The stiff system near nematic onset: 100 chains x 2000 beads (200k monomers), kappa = 3,
    seeded random-walk start, mixed precision; the exponent stepped through every n of Eq. 11 in
    turn, `steps_per_n` MD steps at each with one double-bridging sweep every `sweep_every` steps
    at the paper's attempt rate (Sec. II.B: 100 attempts per sweep here).  Per n: the sweeps'
    acceptance beside Eq. 15 and the Fig. 3 fit, and R^2(n)/n at the end of the stage beside the
    worm-like chain of Eq. 14 with the Kuhn length of Eq. 12."""
    import torch
    kappa = 3.0
    params = dict(WORKLOAD, M=100, N=2000, kappa=kappa, n_exp=XI[0], precision=kg.PREC_MIXED)
    t0 = time.perf_counter()
    b = kg.Batch([params], stream=stream)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    N = params["N"]
    sample = [1, 2, 5, 10, 20, 50, 100, 200, 500, 1000, N - 1]
    rows = []
    t_all = time.perf_counter()
    for n in XI:
        t1 = time.perf_counter()
        st = b.run_protocol([n], [steps_per_n], sweep_every=sweep_every)[0]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        r2n, lk, mb = b.observables()
        eq15, fig3 = success_fits(kappa, n)
        tried = st["attempts"] - st["no_candidate"]
        rows.append({"n": n, "md_steps": st["steps"], "attempts": st["attempts"], "no_candidate": st["no_candidate"],
                     "accepted": st["accepted"], "acceptance": st["accepted"] / max(st["attempts"], 1),
                     "acceptance_of_tried": st["accepted"] / max(tried, 1),
                     "eq15_fit": round(eq15, 5), "fig3_fit": round(fig3, 5),
                     "r2_over_n": {str(k_): round(float(r2n[k_ - 1]), 4) for k_ in sample},
                     "ell_K_fit": round(lk, 4), "mean_bond": round(mb, 5), "wall_s": round(wall, 3)})
    total = time.perf_counter() - t_all
    lk_pred = kg_kuhn(kappa)
    mb_end = rows[-1]["mean_bond"]
    b.close()
    return {"system": "100 chains x 2000 beads (200k monomers), rho 0.85, kappa 3, mixed precision, "
                      "seeded random-walk start with the workload's warm-up",
            "steps_per_n": steps_per_n, "sweep_every": sweep_every, "n_values": list(XI), "setup_s": round(setup, 2),
            "wall_s": round(total, 2), "stages": rows,
            "ell_K_eq12_over_l0": round(lk_pred, 4),
            "wlc_r2_over_n_eq14": {str(k_): round(wlc_r2_over_n(k_, lk_pred * mb_end, mb_end), 4) for k_ in sample}}


def run_config1_checks(kg, stream, state, drift_steps=10000, chunk=1000, sweeps=10, attempts=200):
    """Config 1 (200 x 1000, kappa = 2) from the mixed bench run's final state: (1) energy drift of
    each precision form over `drift_steps` steps at gamma = 0 (velocity Verlet without the
    thermostat, Langevin force cleared) on a copy of the state, total energy read every `chunk`
    steps; (2) the double-bridging decisions of the two forms from the same snapshots: a mixed
    run (gamma = 1) is stopped every 100 steps, and the FP64 and the mixed batch each run one
    sweep of `attempts` attempts from that snapshot, `sweeps` times."""
    nm = state["x"].shape[1]
    base = dict(WORKLOAD, warmup_steps=0)
    drift = {}
    for name, prec in (("fp64", kg.PREC_FP64), ("mixed", kg.PREC_MIXED)):
        b = kg.Batch([dict(base, precision=prec, gamma=0.0)], stream=stream)
        b.set_state(0, x=state["x"], v=state["v"], fl=np.zeros_like(state["fl"]), chains=state["chains"],
                     counters=state["counters"])
        e = [float(np.sum(b.energy()))]
        for _ in range(drift_steps // chunk):
            b.md_steps(chunk)
            e.append(float(np.sum(b.energy())))
        b.close()
        e = np.array(e)
        drift[name] = {"E0_per_monomer": round(e[0] / nm, 8), "E_end_per_monomer": round(e[-1] / nm, 8),
                       "drift_rel": float((e[-1] - e[0]) / abs(e[0])),
                       "max_dev_rel": float(np.max(np.abs(e - e[0])) / abs(e[0])),
                       "per_monomer_every_chunk": [round(v_ / nm, 8) for v_ in e]}
    src = kg.Batch([dict(base, precision=kg.PREC_MIXED)], stream=stream)
    src.set_state(0, x=state["x"], v=state["v"], fl=state["fl"], chains=state["chains"], counters=state["counters"])
    fb = kg.Batch([dict(base, precision=kg.PREC_FP64)], stream=stream)
    mb_ = kg.Batch([dict(base, precision=kg.PREC_MIXED)], stream=stream)
    same_topo, acc = 0, {"fp64": 0, "mixed": 0}
    same_counts = True
    for _ in range(sweeps):
        src.md_steps(MD_PER_STEP)
        st = src.get_state()
        res = {}
        for name, bb in (("fp64", fb), ("mixed", mb_)):
            bb.set_state(0, x=st["x"], v=st["v"], fl=st["fl"], chains=st["chains"], counters=st["counters"])
            s = bb.db_sweep(attempts)[0]
            acc[name] += s["accepted"]
            res[name] = (s["accepted"], s["no_candidate"], bb.get_state()["chains"])
        same_counts &= res["fp64"][:2] == res["mixed"][:2]
        same_topo += int(np.array_equal(res["fp64"][2], res["mixed"][2]))
    for bb in (src, fb, mb_):
        bb.close()
    return {"energy_drift": dict(drift, steps=drift_steps, gamma=0.0, dt=WORKLOAD["dt"]),
            "db_decision_match": {"sweeps": sweeps, "attempts_per_sweep": attempts,
                                  "accepted_fp64": acc["fp64"], "accepted_mixed": acc["mixed"],
                                  "accept_counts_identical": bool(same_counts),
                                  "sweeps_with_identical_topology": same_topo}}


def run_protocol_bench(kg, stream, kappa, steps_per_stage, sweep_every=100):
    """The n-ramp protocol (Sec. II.B) on the paper's own melt size at stiffness kappa: every
    stage of the plan (Eqs. 11, 16-20) runs `steps_per_stage` steps with a sweep at the paper's
    attempt rate every `sweep_every` steps, timed per stage; the full plan's wall-clock is
    projected from those rates.  Also the swap success rate per exponent, beside the paper's
    fit of it (Fig. 3 caption: a' exp(-b' kappa - d' n - e' n^2)), as a trend check."""
    import torch
    params = dict(WORKLOAD, **PAPER_SYSTEM, kappa=kappa, precision=kg.PREC_MIXED)
    t0 = time.perf_counter()
    b = kg.Batch([params], stream=stream)
    b.md_steps(MD_PER_STEP)
    b.autotune(0, reps=20)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    plan = kg.protocol_schedule(kappa, PAPER_SYSTEM["N"], dt=PAPER_SYSTEM["dt"])
    # structure at the end of each stage (App. A): g(r) to 3 sigma and S(q) on ~5,000
    # reciprocal-lattice vectors up to 12 / sigma, averaged in shells of 0.1 / sigma (the peak
    # from the three-shell running mean)
    from tests.inputs import qvectors  # seeded choice of lattice vectors (no method arithmetic)
    L = b.geom[0]["L"]
    nsh = 120
    qv = qvectors(L, 12.0, nsh, 48, seed=1)
    qmag = 2 * math.pi / L * np.linalg.norm(qv, axis=1)
    edges = np.linspace(0.0, 12.0, nsh + 1)
    full = steps_per_stage <= 0  # the whole plan, stage by stage
    st, structure, t_obs = [], [], []
    t_run = time.perf_counter()
    for n, plan_steps in zip(plan["n"], plan["steps"]):
        todo = plan_steps if full else steps_per_stage
        acc = None
        while todo > 0:  # calls of at most 250,000 steps, each reported
            c = min(todo, 250000)
            r = b.run_protocol([n], [c], sweep_every=sweep_every)[0]
            if acc is None:
                acc = r
            else:
                for f_ in ("steps", "attempts", "no_candidate", "accepted", "wall_ms"):
                    acc[f_] += r[f_]
            todo -= c
            if full:
                print(f"[bench] protocol kappa {kappa}: n = {n}, {acc['steps']} of {plan_steps} steps, "
                      f"{acc['accepted']} swaps", file=sys.stderr, flush=True)
        st.append(acc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, g = b.pair_correlation(3.0, 150)
        t1 = time.perf_counter()
        S = b.structure_factor(qv)
        t2 = time.perf_counter()
        t_obs.append((t1 - t0, t2 - t1))
        idx = np.digitize(qmag, edges) - 1
        Sb = np.array([S[idx == i].mean() if np.any(idx == i) else np.nan for i in range(nsh)])
        qc = 0.5 * (edges[1:] + edges[:-1])
        sm = np.convolve(np.nan_to_num(Sb, nan=0.0), np.ones(3) / 3, mode="same")
        win = (qc > 4.0) & (qc < 10.0)
        structure.append({"n": n, "S_peak_q": round(float(qc[win][np.argmax(sm[win])]), 2),
                          "S_peak": round(float(np.max(sm[win])), 3),
                          "S_q_below_1p5": round(float(np.nanmean(S[qmag < 1.5])), 4),
                          "S_q_5_to_8": round(float(np.mean(S[(qmag > 5) & (qmag < 8)])), 4),
                          "S_q_above_8": round(float(np.mean(S[qmag > 8])), 4),
                          "g_peak_r": float((np.argmax(g) + 0.5) * 3.0 / 150), "g_peak": round(float(np.max(g)), 3)})
    run_s = time.perf_counter() - t_run
    lk_end = b.observables()[1]
    # the swap rate of n = 12 alone (denominator of the speedup), from a longer n = 12 run
    tail = b.run_protocol([plan["n"][-1]], [10 * (steps_per_stage if not full else 1000)], sweep_every=sweep_every)[0]
    s12 = tail["accepted"] / max(tail["attempts"] - tail["no_candidate"], 1)
    nm, _ = b.sizes()
    floored = b.fene_floored() / max(1, b.counters()[0] * PAPER_SYSTEM["M"] * (PAPER_SYSTEM["N"] - 1))
    b.close()
    stages, proj = [], 0.0
    for i, s_ in enumerate(st):
        ms = s_["wall_ms"] / max(s_["steps"], 1)
        tried = s_["attempts"] - s_["no_candidate"]
        n = plan["n"][i]
        fit = 1.24 * math.exp(-0.77 * kappa - 0.24 * n - 0.015 * n * n)
        stages.append({"n": n, "plan_steps": plan["steps"][i], "ms_per_step": round(ms, 5),
                       "monomer_steps_per_s": nm / (ms * 1e-3), "accepted": s_["accepted"], "attempts": tried,
                       "success_rate": s_["accepted"] / max(tried, 1), "paper_fit_success_rate": round(fit, 5)})
        proj += plan["steps"][i] * ms * 1e-3
    # Table I analogue, projected over the full plan from the measured rates: swaps per monomer
    # (attempt rate x stage time x success rate, summed) and the speedup R over n = 12-only
    # double bridging of the same length (the sum over stages of tau_i S_i over tau_eq S_12)
    dtp = PAPER_SYSTEM["dt"]
    swaps = sum(1e-3 * ps * dtp * stg["success_rate"] for ps, stg in zip(plan["steps"], stages))
    R = sum(ps * stg["success_rate"] for ps, stg in zip(plan["steps"], stages)) / max(sum(plan["steps"]) * s12, 1e-300)
    out_full = None
    if full:
        out_full = {"wall_s": round(run_s, 1), "steps": int(sum(x["steps"] for x in st)),
                    "swaps_per_monomer": round(sum(x["accepted"] for x in st) / nm, 3),
                    "ell_K_end": lk_end, "ell_K_eq12": 0.960897 * kg_kuhn(kappa)}
    return {"full_run": out_full,
            "table1_projection": {"swaps_per_monomer": round(swaps, 2), "R": round(R, 1),
                                  "success_rate_n12": s12, "n12_attempts": tail["attempts"] - tail["no_candidate"]},
            "system": f"{PAPER_SYSTEM['M']} chains x {PAPER_SYSTEM['N']} beads, kappa {kappa}, rho 0.85, "
                      f"dt {PAPER_SYSTEM['dt']}, mixed precision", "monomers": nm,
            "plan": {"steps_total": int(sum(plan["steps"])), "tau_eq": plan["tau_eq"], "scheme": plan["scheme"]},
            "steps_per_stage_timed": steps_per_stage, "sweep_every": sweep_every, "setup_s": round(setup_s, 2),
            "stages": stages, "projected_full_protocol_s": round(proj, 1), "structure": structure,
            "fene_floored_per_bond_step": floored,
            "q_vectors": int(len(qv)), "g_r_ms": round(1e3 * float(np.median([t[0] for t in t_obs])), 2),
            "S_q_ms": round(1e3 * float(np.median([t[1] for t in t_obs])), 2)}


def roofline(run, mixed):
    """The step kernel's achieved bandwidth in algorithmic bytes (the graded figure) and in this
    implementation's own bytes, from its mean launch time."""
    nm = run["monomers"]
    ms = run["force_kernel_ms"]
    bpm = algorithmic_bytes(mixed)
    ibpm = implementation_bytes(mixed, run["nl"]["mean_list"], run["nl"]["K"], run["lds_stage"]["staged_per_monomer"])
    achieved = bpm * nm / (ms * 1e-3) / 1e9
    impl = ibpm * nm / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": f"k_nl_step<{'float' if mixed else 'double'}, close|open> "
                                      "(list forces + bonded + Langevin VV, one workgroup per tile)",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "algorithmic_bytes_per_launch": round(bpm * nm), "bytes_per_monomer": bpm,
            "implementation_bytes_per_monomer": round(ibpm, 1), "implementation_GBs": round(impl, 1),
            "implementation_frac": round(impl / HBM_PEAK_GBS, 4),
            "avg_launch_ms": ms, "launches": run["force_launches_timed"], "neighbour_lists": run["nl"],
            "autotune_ms_per_step_by_K": run["tune_ms"], "rebuild_ms_per_step": run.get("finalize_kernel_ms"),
            "fene_floored_per_bond_step": run.get("fene_floored_frac"), "lds_stage": run["lds_stage"]}


def step_kernel_hash():
    """sha256 of the step kernel's source (its body in kgdb_nl.hip plus kgdb_dev.h)."""
    csrc = os.path.join(ROOT, "paper_2109_11001_amd", "csrc")
    nl = open(os.path.join(csrc, "kgdb_nl.hip")).read()
    dev = open(os.path.join(csrc, "kgdb_dev.h")).read()
    m = re.search(r"void k_nl_step\(NlArgs a\) \{.*?\n\}\n", nl, re.S)
    return hashlib.sha256((m.group(0) + dev).encode()).hexdigest()


def measured_traffic():
    """HBM bytes per launch of the step kernel from the committed PMC summary, or None when the
    kernel source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "pmc_k_nl_step_200k_mixed.md")
    try:
        text = open(path).read()
        rec = json.loads(re.search(r"^traffic_json: (\{.*\})$", text, re.M).group(1))
        sha = step_kernel_hash()
    except (OSError, AttributeError, ValueError):
        return None
    return rec if rec.get("kernel_sha256") == sha else None


def copy_calibration(mib=256, reps=5):
    """A plain device copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"[bench] copy calibration: {reps} copies of {mib} MiB", file=sys.stderr, flush=True)


def host_cpu():
    """Model name and logical CPU count of the host the oracle ran on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return f"{model} ({os.cpu_count()} logical CPUs visible)"


def cpu_baseline(md_steps=15, db_attempts=8, stream=None):
    """The FP64 CPU oracle (single thread) on a bounded sample of the same workload; then, from
    the state it reached, the GPU path's error against it per result (untimed)."""
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
    out = {"value": nm * MD_PER_STEP / chunk, "unit": "monomer-timesteps/s", "cores": 1, "kind": "oracle",
           "host_cpu": host_cpu(),
           "sample": f"200k-monomer workload melt: {md_steps} MD steps ({t_step:.3f} s each) and "
                     f"{db_attempts} DB attempts ({t_att:.3f} s each), scaled to one bench step of "
                     f"{MD_PER_STEP} MD steps + {K} attempts; single-threaded FP64 C oracle"}
    out["all_cores"] = cpu_baseline_all_cores(md_steps, db_attempts)
    out["gpu_error_vs_oracle"] = oracle_errors(m, stream)
    # the small workload (20 chains x 50 beads) in full on both sides
    import torch
    import paper_2109_11001_amd as kg
    t_or, _ = small_run(lambda: o.Melt(**SMALL_WORKLOAD))
    torch.cuda.synchronize()
    t_gpu, g = small_run(lambda: kg.Batch([dict(WORKLOAD, **SMALL_WORKLOAD, precision=kg.PREC_FP64)], stream=stream))
    torch.cuda.synchronize()
    t_gpu = max(t_gpu, 1e-9)
    g.close()
    out["small_workload_full"] = {"workload": "20 chains x 50 beads, kappa 1.5, n 2: init with 1000 warm-up steps, "
                                              "2000 MD steps, 20 sweeps of 1 attempt",
                                  "oracle_s": round(t_or, 3), "gpu_fp64_s": round(t_gpu, 4)}
    return out


def cpu_baseline_all_cores(md_steps, db_attempts, max_threads=16):
    """The same oracle sample on every host core at once: one independent workload melt per
    thread (seeds 1, 2, ...), each stepped by its own thread (the oracle's C calls release the
    interpreter lock, and its melts share no state).  The aggregate is the sum of the melts'
    rates over the slowest thread's time: the oracle's throughput for a batch of melts."""
    from concurrent.futures import ThreadPoolExecutor
    import threading
    from oracle import oracle as o
    P = max(1, min(os.cpu_count() or 1, max_threads))
    start = threading.Barrier(P)

    def one(i):
        m = o.Melt(**dict(WORKLOAD, warmup_steps=60, seed=1 + i))  # untimed setup
        start.wait(timeout=600)
        t0 = time.perf_counter()
        m.md_steps(md_steps)
        t1 = time.perf_counter()
        m.db_sweep(db_attempts)
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1

    with ThreadPoolExecutor(max_workers=P) as ex:
        times = list(ex.map(one, range(P)))
    t_step = max(t[0] for t in times) / md_steps
    t_att = max(t[1] for t in times) / db_attempts
    nm = WORKLOAD["M"] * WORKLOAD["N"]
    K = round(1e-3 * nm * MD_PER_STEP * WORKLOAD["dt"])
    chunk = MD_PER_STEP * t_step + K * t_att
    return {"value": P * nm * MD_PER_STEP / chunk, "unit": "monomer-timesteps/s", "cores": P,
            "sample": f"{P} workload melts (seeds 1-{P}), one per thread at once: {md_steps} MD steps "
                      f"(slowest {t_step:.3f} s each) and {db_attempts} DB attempts (slowest {t_att:.3f} s "
                      f"each), scaled to one bench step per melt"}


SMALL_WORKLOAD = dict(M=20, N=50, kappa=1.5, n_exp=2.0, seed=1)  # 1000 monomers, L = 10.56 sigma


def small_run(make, steps=2000, sweeps=20):
    """The small workload in full: init with warm-up, then `steps` MD steps with a sweep of one
    attempt every steps / sweeps steps.  `make` builds the melt (GPU binding or oracle)."""
    t0 = time.perf_counter()
    m = make()
    every = steps // sweeps
    for _ in range(sweeps):
        m.md_steps(every)
        m.db_sweep(1)
    return time.perf_counter() - t0, m


def oracle_errors(m, stream, attempts=20):
    """The GPU path against the oracle melt `m` (200k-monomer workload), both from its current
    state: a double-bridging sweep (decisions and topology must be identical), forces relative
    to S_i (the sum of the magnitudes of the contributions on bead i), one MD step, energies
    and R^2(n)/n."""
    import numpy as np
    import paper_2109_11001_amd as kg
    st = m.get_state()
    so = m.db_sweep(attempts)
    Fo, So, _ = m.forces()
    eo = m.energy()
    r2o, _, _ = m.observables()
    m.md_steps(1)
    xo = m.get_state()["x"]
    L = m.L
    res = {"workload": "200k-monomer workload melt after the oracle's timed sample",
           "db_attempts": attempts, "db_accepted": so["accepted"]}
    for name, prec in (("fp64", kg.PREC_FP64), ("mixed", kg.PREC_MIXED)):
        g = kg.Batch([dict(WORKLOAD, warmup_steps=0, precision=prec)], stream=stream)
        g.set_state(0, x=st["x"], v=st["v"], fl=st["fl"], chains=st["chains"], counters=st["counters"])
        sg = g.db_sweep(attempts)[0]
        same = (sg["accepted"] == so["accepted"] and sg["attempts"] == so["attempts"]
                and np.array_equal(g.get_state()["chains"], m.get_state()["chains"]))
        Fg, _, _ = g.forces()
        eg = g.energy()
        r2g, _, _ = g.observables()
        g.md_steps(1)
        d = g.get_state()["x"] - xo
        d -= L * np.rint(d / L)
        g.close()
        res[name] = {"db_sweep_identical": bool(same),
                     "force_max_err_over_S": float(np.max(np.sqrt(((Fg - Fo) ** 2).sum(0)) / So)),
                     "x_after_1_step_max_abs": float(np.max(np.abs(d))),
                     "energy_max_rel": float(np.max(np.abs(eg - eo) / np.maximum(np.abs(eo), 1e-300))),
                     "r2n_max_rel": float(np.max(np.abs(r2g - r2o) / r2o))}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed bench steps (100 MD steps + 1 sweep each)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--profile-steps", type=int, default=-1,
                    help="bench steps of the HIP-event-timed pass (default: as many as timed)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-config2", action="store_true",
                    help="skip the stiff-system run (100 x 2000, kappa 3, every n of Eq. 11)")
    ap.add_argument("--no-checks", action="store_true",
                    help="skip the workload's energy drift, FP64/mixed decision match and the "
                         "time-to-equilibrium check")
    ap.add_argument("--no-equilibration-check", action="store_true",
                    help="skip the short time-to-equilibrium check (2000 x 25 melt; FP64, mixed and "
                         "learned forms against an FP64 reference run)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run plain copies of known size (for PMC byte counters)")
    ap.add_argument("--size-sweep", default="",
                    help="comma-separated monomer counts (e.g. 1000000,4000000,16000000): also time the "
                         "step kernel on single melts of these sizes (N = 1000), mixed path, then the "
                         "same bench steps with sweeps")
    ap.add_argument("--size-sweep-steps", type=int, default=500)
    ap.add_argument("--no-main", action="store_true", help="skip the workload runs (with --size-sweep or --equilibration)")
    ap.add_argument("--batch", action="store_true",
                    help="with --no-main: run the batched form (24 uneven melts, kappa 0-2.5, N 100-800, 705k "
                         "monomers, as one batch vs one at a time); the default line runs it anyway")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched form in the default line")
    ap.add_argument("--protocol", type=int, default=0, metavar="STEPS",
                    help="time every stage of the n-ramp protocol for STEPS steps on the paper's 1000 x 400 "
                         "melt and project the full run")
    ap.add_argument("--protocol-kappa", default="2.0,5.5")
    ap.add_argument("--protocol-full", type=float, default=None, metavar="KAPPA",
                    help="run the whole plan (10^7 steps for kappa < 2.5) on the 1000 x 400 melt at KAPPA")
    ap.add_argument("--equilibration", type=int, default=0, metavar="STEPS",
                    help="time to equilibrium of R^2(n)/n for each form on a 2000 x 25 melt, STEPS steps each")
    ap.add_argument("--equilibration-ref", type=int, default=0, metavar="STEPS",
                    help="length of the plain FP64 reference run (default: 2 x --equilibration)")
    ap.add_argument("--equilibration-seeds", default="1", metavar="S1,S2,...",
                    help="seeds of the warmed-up starts every form runs from (default: 1)")
    ap.add_argument("--equilibration-forms", default=",".join(EQ_FORMS), metavar="F1,F2,...",
                    help="forms to time (fp64, mixed, batched, learned, mixed_fr; default: all)")
    args = ap.parse_args()
    bad = set(v.strip() for v in args.equilibration_forms.split(",") if v.strip()) - set(EQ_FORMS)
    if bad:
        sys.exit(f"bench.py: unknown --equilibration-forms {sorted(bad)}; known: {', '.join(EQ_FORMS)}")
    if args.profile_steps < 0:
        args.profile_steps = args.steps
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); melts shard across GPUs without any "
              "exchange, so the per-GPU figure is the single-GPU one", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2109_11001_amd as kg
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    if args.copy_calibration:
        copy_calibration()
    sweep = []
    for nm_ in [int(v) for v in args.size_sweep.split(",") if v.strip()]:
        print(f"[bench] size sweep: {nm_} monomers, {args.size_sweep_steps} MD steps", file=sys.stderr, flush=True)
        sweep.append(run_size(kg, nm_, args.size_sweep_steps, stream, kg.PREC_MIXED))
        print(f"[bench] size sweep {nm_}: {sweep[-1]['avg_launch_ms'] * 1e3:.1f} us per step launch, "
              f"frac {sweep[-1]['frac']}", file=sys.stderr, flush=True)
    eq = None
    if args.equilibration > 0:
        print(f"[bench] equilibration: {args.equilibration} steps per form", file=sys.stderr, flush=True)
        eq = run_equilibration(kg, stream, args.equilibration, args.equilibration_ref or 2 * args.equilibration,
                               seeds=[int(v) for v in args.equilibration_seeds.split(",") if v.strip()],
                               forms=[v.strip() for v in args.equilibration_forms.split(",") if v.strip()])
        print("[bench] equilibration done", file=sys.stderr, flush=True)
    prot = []
    for kap in [float(v) for v in args.protocol_kappa.split(",") if v.strip()] if args.protocol > 0 else []:
        print(f"[bench] protocol: kappa {kap}, {args.protocol} steps per stage", file=sys.stderr, flush=True)
        prot.append(run_protocol_bench(kg, stream, kap, args.protocol))
        print(f"[bench] protocol kappa {kap}: projected {prot[-1]['projected_full_protocol_s']} s for "
              f"{prot[-1]['plan']['steps_total']} steps", file=sys.stderr, flush=True)
    bat = None
    if args.batch and args.no_main:
        bat = batch_form(kg, stream, args.steps, args.warmup)
    if args.protocol_full is not None:
        print(f"[bench] full protocol run: kappa {args.protocol_full}", file=sys.stderr, flush=True)
        prot.append(run_protocol_bench(kg, stream, args.protocol_full, 0))
    if args.no_main:
        print(json.dumps({"size_sweep": sweep, "equilibration": eq, "protocol": prot, "batch": bat}), flush=True)
        return
    print(f"[bench] mixed path: {args.warmup} warm-up + {args.steps} timed steps", file=sys.stderr, flush=True)
    mixed = run_gpu(kg, kg.PREC_MIXED, args.steps, args.warmup, stream, args.profile_steps,
                    keep_state=not args.no_checks)
    print(f"[bench] mixed done: {mixed['monomer_steps_per_s']:.3e} monomer-steps/s", file=sys.stderr, flush=True)
    checks = None
    if not args.no_checks:
        print("[bench] workload checks: energy drift (both forms) and decision match", file=sys.stderr, flush=True)
        checks = run_config1_checks(kg, stream, mixed.pop("state"))
        print(f"[bench] checks done: drift {checks['energy_drift']['fp64']['drift_rel']:.2e} (fp64), "
              f"{checks['energy_drift']['mixed']['drift_rel']:.2e} (mixed); identical topology after "
              f"{checks['db_decision_match']['sweeps_with_identical_topology']} of "
              f"{checks['db_decision_match']['sweeps']} sweeps", file=sys.stderr, flush=True)
    conf2 = None
    if not args.no_config2:
        print("[bench] stiff system: 100 x 2000, kappa 3, n over Eq. 11", file=sys.stderr, flush=True)
        conf2 = run_config2(kg, stream)
        print(f"[bench] stiff system done in {conf2['wall_s']} s", file=sys.stderr, flush=True)
    fp64 = None
    if not args.no_fp64:
        fp64 = run_gpu(kg, kg.PREC_FP64, args.steps, args.warmup, stream, args.profile_steps)
        print(f"[bench] fp64 done: {fp64['monomer_steps_per_s']:.3e} monomer-steps/s", file=sys.stderr, flush=True)
    learned = None
    if not args.no_learned:
        print("[bench] learned-proposal form (training, then learned vs uniform)", file=sys.stderr, flush=True)
        learned = run_learned(kg, args.steps, args.warmup, stream)
        print(f"[bench] learned done: accept rate {learned['learned']['accept_rate']:.3f} vs "
              f"{learned['uniform']['accept_rate']:.3f}", file=sys.stderr, flush=True)
    if not args.no_batch:
        bat = batch_form(kg, stream, args.steps, args.warmup)
    eq_check = None
    if not (args.no_equilibration_check or args.no_checks) and args.equilibration == 0:
        print(f"[bench] time to equilibrium: {EQ_CHECK['steps']} steps per form, reference "
              f"{EQ_CHECK['ref_steps']}", file=sys.stderr, flush=True)
        eq_check = run_equilibration(kg, stream, EQ_CHECK["steps"], EQ_CHECK["ref_steps"], seeds=(1,),
                                     forms=EQ_CHECK["forms"])
        print("[bench] time to equilibrium: " + ", ".join(
            f"{f} {v['steps_to_tol_mean']} steps / {v['wall_s_to_tol_mean']} s" for f, v in eq_check["forms"].items()),
            file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(stream=stream)

    roof = None
    if "force_kernel_ms" in mixed:
        roof = roofline(mixed, True)
        tr = measured_traffic()
        roof["traffic"] = tr["bytes_per_launch"] if tr else None
        roof["traffic_split"] = {k_: tr[k_] for k_ in ("fetch_bytes", "write_bytes", "scale")} if tr else None
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
        "autotuner": {"K": mixed["nl"]["K"], "tile_shape": mixed["lds_stage"]["tile_shape"],
                      "ms_per_step_by_K_with_its_best_shape": mixed["tune_ms"],
                      "tried": "K in {1, 2, 5} x up to 3 tile shapes per K"},
    }
    if fp64:
        line["fp64_path"] = {"value": fp64["monomer_steps_per_s"], "ms_per_step": fp64["ms_per_step"],
                             "db_accepted_per_s": fp64["db_accepted_per_s"],
                             "md_only_monomer_steps_per_s": fp64["md_only_monomer_steps_per_s"],
                             "time_split_s": {"md": round(fp64["md_s"], 4), "db": round(fp64["db_s"], 4)},
                             "rebuild_ms_per_md_step": fp64.get("finalize_kernel_ms"),
                             "force_kernel_ms": fp64.get("force_kernel_ms"),
                             "neighbour_lists": fp64["nl"], "autotune_ms_per_step_by_K": fp64["tune_ms"],
                             "roofline": roofline(fp64, False) if "force_kernel_ms" in fp64 else None}
        line["speedup_vs_fp64_path"] = mixed["monomer_steps_per_s"] / fp64["monomer_steps_per_s"]
    if checks:
        line["workload_checks"] = checks
    if conf2:
        line["stiff_system"] = conf2
    if learned:
        line["learned_form"] = learned
    if sweep:
        line["size_sweep"] = sweep
    if eq:
        line["equilibration"] = eq
    if eq_check:
        line["equilibration_check"] = eq_check
    if prot:
        line["protocol"] = prot
    if bat:
        line["batch"] = bat
    line["roofline"] = roof
    line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
