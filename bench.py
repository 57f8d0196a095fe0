"""Benchmark: leapfrog steps of the soft (long-range) part on one MI355X.

A step is one shared-timestep kick-drift-kick of the soft Hamiltonian
(Section 2.1 splitting; the hard Hermite part is not part of this path):
  v += dt/2 a;  x += dt v;  rebuild tree + groups + lists;  long-range force and
  potential;  neighbour lists within h;  v += dt/2 a.
Default workload: King W0 = 9, N = 2^20 equal-mass stars (seeded synthetic
sample of the model), theta = 0.5, n_crit = 256, r_out = 0.002, r_in = 0.1 r_out,
h = 1.1 r_out, eps = 4/N, dt = 1/256, mixed precision.

Prints ONE JSON line.  ``value`` is long-range interactions per second over
whole steps (interactions counted from the walk's lists: sum over groups of
n_g (|P_g| + |C_g|)).  The same steps are also run with the FP64 interaction
kernel; the roofline object describes the dominant kernel (the interaction
kernel), timed with HIP events on the stream it runs on.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "long-range interactions/s & ms per leapfrog step at N=1M, FP32 vs FP64, RMS err"
PEAK_TFLOPS = {"mixed": 157.3, "fp64": 78.6}     # MI355X vector FP32 (packed) / FP64
# Without packed FP32 instructions (not generated: the library is built without
# them) one FP32 FMA per lane per cycle is the ceiling: 256 CUs x 4 SIMDs x
# 16 lanes x 2 flops x 2.4 GHz.
PEAK_UNPACKED_FP32 = 78.6
# Algorithmic flops per interaction of the common path (FMA = 2, add/sub/mul = 1,
# rsqrt = 4):
#   particle: 3 differences, r^2 (3 FMA), rsqrt, m/s, 1/s^2, m/s^3, 3 FMA into a,
#             1 into phi                                                 = 23
#   cell (quadrupole): 3 differences, r^2, rsqrt, 1/s^2, 1/s^3, Q r (3 mul +
#             6 FMA), r.Q.r (1 mul + 2 FMA), 1/s^4, B, phi factor (FMA + mul),
#             radial factor (FMA + mul), 1/s^5, 6 FMA into a, 1 into phi = 57
#   cell (monopole): 3 differences, r^2, rsqrt, 1/s^2, 1/s^3, 2 mul, 3 FMA
#             into a, 1 into phi                                         = 24
F_PP = 23
F_PC_QUAD = 57
F_PC_MONO = 24
# The convention fixed before the kernels were written counts the changeover
# polynomial K(y) on every particle term and the full multipole formula with K
# and W on every cell term, whether or not the kernel evaluates them (outside
# r_out it does not): 37 flops per particle-particle and 75 per quadrupole
# particle-cell interaction.  Reported beside the count above as frac_survey.
F_PP_SURVEY = 37
F_PC_SURVEY = 75
HBM_PEAK_GBPS = 8000.0
# Algorithmic flops of one adjoint term of the VJP (common path K = W = 1, same
# convention), both sides accumulated:
#   particle-particle: d (3), s^2 (6), rsqrt (4), 1/s^2, 1/s^3 (2), g' (2),
#     w.d (5), t (4), dl/dd (12), dl/dm_j (3), accumulation (3 + 4)       = 48
#   particle-cell (quadrupole): r (3), s^2, rsqrt and the powers to 1/s^9 (15),
#     Q r, Q w, r.Q.r (35), r.w, (Q r).w (10), Hessian coefficients (17),
#     A (15), H w (21), Phi (4), w.A (5), dl/dr (6), dl/dM (3), dl/dQ (43),
#     accumulation (3 + 10)                                               = 190
F_VJP_PP = 48
F_VJP_PC = 190

# Algorithmic HBM bytes of the tree build before the walk (bounding cube to
# groups): every array read or written once per pass that needs it.
BUILD_BYTES_PER_PARTICLE = {
    "bbox": 24,                      # read positions
    "keys": 24 + 12,                 # read positions; write key + index
    "sort": 8 * (8 + 12 + 12),       # 8 passes: histogram reads the key, scatter
                                     # reads and writes key + index
    "gather": 4 + 32 + 32,           # read index, position + mass; write x y z m
    "topology": 16,                  # sorted keys read by the neighbour comparisons
    "moments": 64,                   # leaves read x y z m twice
    "groups": 12,                    # flag, scan, compaction
}
BUILD_BYTES_PER_NODE = {
    "topology": 32,                  # level first count child n_child parent prefix
    "moments": 400,                  # write S, walk and multipole records (200 B);
                                     # the parent reads them back once
}


# HBM bytes per launch of the interaction kernel come from two rocprofv3 --pmc
# passes (FETCH_SIZE, WRITE_SIZE) on the headline workload, scaled by what the
# same counters read for a plain device copy of known size; the summary holds a
# digest of the kernel sources it was taken on, and the figure is reported only
# while those sources are unchanged.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_force_king9_1m_hbm_traffic.md")
KERNEL_SOURCES = ["force.hip", "internal.h", "device_util.h"]


def kernel_sources_digest():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1506_04553_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(workload, precision):
    """HBM bytes per launch recorded for the current kernel sources, else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if line.startswith("traffic: "):
                    rec = json.loads(line[len("traffic: "):])
                    if (rec["sources_sha256"] == kernel_sources_digest()
                            and rec["workload"] == workload and rec["precision"] == precision):
                        return rec
    except (OSError, ValueError, KeyError):
        pass
    return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_steps(ctx, pos0, vel0, mass, params, dt, steps, warmup, collect_first=False):
    import torch
    pos = pos0.clone()
    vel = vel0.clone()
    acc = torch.empty_like(pos)
    pot = torch.empty_like(mass)
    ctx.build_tree(pos, mass, **params)
    ctx.long_force(acc, pot)
    first = None
    if collect_first:
        first = (acc.clone(), pot.clone(), ctx.stats())
    rec = []

    def step():
        ctx.kick_drift(pos, vel, acc, 0.5 * dt, dt)
        ctx.build_tree(pos, mass, **params)
        ctx.long_force(acc, pot)
        ctx.neighbors()
        ctx.kick_drift(pos, vel, acc, 0.5 * dt, 0.0)
        return ctx.stats()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        rec.append(step())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0), rec, first


def isolated_force(ctx, pos, mass, params, quad, reps=10):
    """The interaction kernel alone (no neighbour search beside it): reps launches
    back to back on one build, between two events on the context's stream; in
    the leapfrog steps the search shares the GPU with it."""
    import torch
    ctx.build_tree(pos, mass, **params)
    acc, pot = ctx.long_force()
    s = ctx.stats()
    flops = s["n_pp"] * F_PP + s["n_pc"] * (F_PC_QUAD if quad else F_PC_MONO)
    flops_s = s["n_pp"] * F_PP_SURVEY + s["n_pc"] * F_PC_SURVEY
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(ctx.stream)
    for _ in range(reps):
        ctx.long_force(acc, pot)
    t1.record(ctx.stream)
    t1.synchronize()
    t = t0.elapsed_time(t1) / reps
    return {"avg_launch_ms": t, "launches": reps,
            "achieved": flops / (t * 1e-3) / 1e12, "achieved_survey": flops_s / (t * 1e-3) / 1e12}


def summarize(rec, seconds, steps, quad):
    inter = sum(s["n_pp"] + s["n_pc"] for s in rec)
    force_ms = [s["ms_force"] for s in rec]
    flops = [s["n_pp"] * F_PP + s["n_pc"] * (F_PC_QUAD if quad else F_PC_MONO) for s in rec]
    flops_survey = [s["n_pp"] * F_PP_SURVEY + s["n_pc"] * F_PC_SURVEY for s in rec]
    avg_force_ms = float(np.mean(force_ms))
    avg_flops = float(np.mean(flops))
    return dict(
        ms_per_step=1e3 * seconds / steps,
        interactions_per_step=inter / steps,
        interactions_per_s=inter / seconds,
        force_ms=avg_force_ms,
        build_ms=float(np.mean([s["ms_build"] for s in rec])),
        walk_ms=float(np.mean([s["ms_walk"] for s in rec])),
        n_nodes=float(np.mean([s["n_nodes"] for s in rec])),
        neighbors_ms=float(np.mean([s["ms_neighbors"] for s in rec])),
        force_tflops=avg_flops / (avg_force_ms * 1e-3) / 1e12,
        force_tflops_survey=float(np.mean(flops_survey)) / (avg_force_ms * 1e-3) / 1e12,
        flops_per_launch=avg_flops,
        n_pp=float(np.mean([s["n_pp"] for s in rec])),
        n_pp_near=float(np.mean([s["n_pp_near"] for s in rec])),
        list_entries={k: float(np.mean([s[f"n_{k}_entries"] for s in rec]))
                      for k in ("cell", "part", "near")},
        walk_fixed_stride=float(np.mean([s["walk_fixed_stride"] for s in rec])),
        n_pc=float(np.mean([s["n_pc"] for s in rec])),
        n_groups=float(np.mean([s["n_groups"] for s in rec])),
        nnz=float(np.mean([s["nnz"] for s in rec])),
    )


def build_roofline(head, n):
    """Algorithmic HBM rate of the tree build before the walk (the walk itself is
    bound by dependent node reads, not bandwidth)."""
    tree_ms = head["build_ms"] - head["walk_ms"]
    byts = n * sum(BUILD_BYTES_PER_PARTICLE.values()) + \
        head["n_nodes"] * sum(BUILD_BYTES_PER_NODE.values())
    gbps = byts / (tree_ms * 1e-3) / 1e9
    return {"ms": head["build_ms"], "walk_ms": head["walk_ms"], "tree_ms": tree_ms,
            "algorithmic_bytes": byts, "achieved_GBps": gbps, "peak_GBps": HBM_PEAK_GBPS,
            "frac": gbps / HBM_PEAK_GBPS,
            "bytes_per_particle": BUILD_BYTES_PER_PARTICLE,
            "bytes_per_node": BUILD_BYTES_PER_NODE}


def walk_rates(head):
    """The group walk: groups per second and the bytes of lists it writes (one
    int32 per list entry plus a (begin, end) int64 segment per group and list);
    the walk's time goes to dependent node reads, so this is a rate, not a roofline."""
    ent = sum(head["list_entries"].values())
    byts = 4 * ent + 3 * 16 * head["n_groups"]
    s = head["walk_ms"] * 1e-3
    return {"ms": head["walk_ms"], "groups": head["n_groups"],
            "groups_per_s": head["n_groups"] / s, "list_entries": ent,
            "list_bytes": byts, "list_write_GBps": byts / s / 1e9}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pos, mass, params, gpu_first, target_s=12.0, seed=3):
    """The oracle on sampled groups of the step-0 tree: force rate on host cores,
    plus the RMS error of the GPU forces on those groups."""
    import oracle
    t0 = time.perf_counter()
    tree = oracle.Tree(pos, mass, params)
    t_build = time.perf_counter() - t0
    L = tree.lists()
    nd = tree.nodes()
    g = tree.groups()
    G = len(g)
    work = (nd["count"][g] * (np.diff(L["p_off"]) + np.diff(L["c_off"]))).astype(np.int64)
    rng = np.random.default_rng(seed)
    order = rng.permutation(G)
    # calibrate on a small batch, then size the sample for ~target_s of CPU work
    first = order[:16]
    t0 = time.perf_counter()
    tree.force_groups(first)
    t_cal = time.perf_counter() - t0
    rate = work[first].sum() / max(t_cal, 1e-6)
    budget = rate * target_s
    cum = np.cumsum(work[order[16:]])
    take = order[16:16 + int(np.searchsorted(cum, budget)) + 1]
    t0 = time.perf_counter()
    acc, pot = tree.force_groups(take)
    t_force = time.perf_counter() - t0
    rows = np.nonzero(~np.isnan(pot))[0]
    n_int = int(work[take].sum())
    threads = oracle.num_threads()
    # one core, on a fortieth of the sample (the paper quotes one CPU core)
    one = take[:max(1, len(take) // 40)]
    oracle.set_threads(1)
    t0 = time.perf_counter()
    tree.force_groups(one)
    t_one = time.perf_counter() - t0
    oracle.set_threads(threads)
    out = dict(value=n_int / t_force, unit="interactions/s", cores=threads,
               kind="oracle",
               sample=(f"force+potential of {len(take)} random groups of {G} "
                       f"({n_int} interactions, {len(rows)} particles) of the step-0 tree; "
                       f"oracle tree build (single-threaded, excluded) took {t_build:.1f} s"),
               one_core_value=int(work[one].sum()) / t_one, cpu_model=cpu_model())
    errs = {}
    for name, (ga, gp) in gpu_first.items():
        ga, gp = ga[rows], gp[rows]
        errs[name] = dict(
            acc_rel_rms=float(np.sqrt(((ga - acc[rows]) ** 2).sum() / (acc[rows] ** 2).sum())),
            pot_rel_rms=float(np.sqrt(((gp - pot[rows]) ** 2).sum() / (pot[rows] ** 2).sum())),
            acc_max_rel=float((np.linalg.norm(ga - acc[rows], axis=1)
                               / np.linalg.norm(acc[rows], axis=1)).max()))
    return out, errs


def vjp_timing(ctx, workload="plummer256k", seed=1, reps=3):
    """Forward + VJP of sum(w.a) + sum(c.phi) on the 2^18 Plummer workload, in
    each precision mode (the VJP's pair and cell terms follow the forward's
    precision; its sums are FP64 in both)."""
    import torch
    from inputs import WORKLOADS, make_cluster
    w_ = WORKLOADS[workload]
    c = make_cluster(w_, seed=seed)
    dev = torch.device("cuda", 0)
    pos = torch.from_numpy(c.pos).to(dev)
    mass = torch.from_numpy(c.mass).to(dev)
    rng = np.random.default_rng(seed + 1)
    wv = torch.from_numpy(rng.normal(size=(w_.n, 3))).to(dev)
    cv = torch.from_numpy(rng.normal(size=w_.n)).to(dev)
    out = {"workload": workload, "n": w_.n,
           "flops_per_term": {"pp": F_VJP_PP, "pc": F_VJP_PC}}
    grads = {}
    for prec in ("mixed", "fp64"):
        ctx.build_tree(pos, mass, **w_.params(precision=prec))
        fwd = []
        for _ in range(reps):
            ctx.long_force()
            fwd.append(ctx.stats()["ms_force"])
        grads[prec] = ctx.long_force_vjp(wv, cv)
        ms = []
        for _ in range(reps):
            ctx.long_force_vjp(wv, cv)
            ms.append(ctx.stats()["ms_vjp"])
        st = ctx.stats()
        t = float(np.median(ms))
        flops = st["n_pp"] * F_VJP_PP + st["n_pc"] * F_VJP_PC
        tf = flops / (t * 1e-3) / 1e12
        f_ms = float(np.median(fwd))
        out[prec] = {"vjp_ms": t, "forward_ms": f_ms,
                     "interactions": st["n_pp"] + st["n_pc"],
                     "flops": flops, "tflops": tf, "peak_tflops": PEAK_TFLOPS[prec],
                     "frac": tf / PEAK_TFLOPS[prec],
                     "vjp_over_forward": t / f_ms}
    (g32, m32), (g64, m64) = grads["mixed"], grads["fp64"]
    out["mixed_vs_fp64_gpu"] = {
        "gpos_rel_rms": float(((g32 - g64).norm() / g64.norm()).item()),
        "gmass_rel_rms": float(((m32 - m64).norm() / m64.norm()).item())}
    return out


HERMITE = dict(eta=0.1, alpha=0.1, dt_max_per_soft=0.25)   # Section 3: eta, alpha, dt_max
F_DIRECT = 23   # flops per pair of the direct Newton sum, counted like the tree's pp term


def direct_timing(ctx, workload="plummer256k", seed=1, reps=3, cpu=True, cpu_rows=48):
    """O(N^2) FP64 direct sums on the 2^18 Plummer workload (Newton and soft):
    median HIP-event time, pairs/s and FP64 TFLOP/s at F_DIRECT per pair; the
    numpy definition on sampled rows as the CPU baseline."""
    import torch
    from inputs import WORKLOADS, make_cluster
    from oracle import direct as odirect
    w_ = WORKLOADS[workload]
    c = make_cluster(w_, seed=seed)
    dev = torch.device("cuda", 0)
    pos = torch.from_numpy(c.pos).to(dev)
    mass = torch.from_numpy(c.mass).to(dev)
    p = w_.params(precision="fp64")
    pairs = w_.n * (w_.n - 1)
    out = {"workload": workload, "n": w_.n, "pairs": pairs, "flops_per_pair": F_DIRECT}
    for mode in ("newton", "soft"):
        ctx.direct(pos, mass, mode, **p)
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ctx.direct(pos, mass, mode, **p)
            e1.record()
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        t = float(np.median(ms))
        tf = pairs * F_DIRECT / (t * 1e-3) / 1e12
        out[mode] = {"ms": t, "pairs_per_s": pairs / (t * 1e-3), "tflops": tf,
                     "frac_of_fp64_peak": tf / PEAK_TFLOPS["fp64"]}
    if cpu:
        rows = np.random.default_rng(seed + 2).choice(w_.n, cpu_rows, replace=False)
        t0 = time.perf_counter()
        for i in rows:
            d = c.pos - c.pos[i]
            s2 = (d * d).sum(1) + p["eps"] ** 2
            f = c.mass / (s2 * np.sqrt(s2))
            f[i] = 0.0
            _ = (f[:, None] * d).sum(0)
        secs = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": cpu_rows * (w_.n - 1) / secs, "unit": "pairs/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"Newton rows of {cpu_rows} random particles by the "
                                         f"numpy definition, {secs:.2f} s"}
    return out


def p3t_step_timing(ctx, w, c, dt, steps=4, warmup=1, cpu_target_s=6.0, cpu=True):
    """Whole P3T steps (kick, neighbour lists, Hermite hard part over the soft
    step, rebuild, soft force, kick) on the workload in FP64 and mixed soft
    force, with the hard part's statistics; the oracle's Hermite integration
    timed on sampled clusters of the same lists as its CPU baseline."""
    import torch
    dev = torch.device("cuda", 0)
    mass = torch.from_numpy(c.mass).to(dev)
    hk = dict(dt_soft=dt, dt_max=dt * HERMITE["dt_max_per_soft"], eta=HERMITE["eta"],
              eta_s=HERMITE["eta"] / 10, a0=HERMITE["alpha"] * float(c.mass.mean()) / w.r_out ** 2)
    out = {"workload": w.name, "n": w.n, "hermite": dict(hk, alpha=HERMITE["alpha"]),
           "steps": steps, "warmup": warmup}
    for prec in ("mixed", "fp64"):
        params = w.params(precision=prec)
        pos = torch.from_numpy(c.pos).to(dev)
        vel = torch.from_numpy(c.vel).to(dev)
        ctx.build_tree(pos, mass, **params)
        acc, _ = ctx.long_force(want_pot=False)
        for _ in range(warmup):
            ctx.step(pos, vel, mass, acc, hk, **params)
        torch.cuda.synchronize()
        wall, herm, stats = [], [], []
        for _ in range(steps):
            t0 = time.perf_counter()
            st = ctx.step(pos, vel, mass, acc, hk, **params)
            torch.cuda.synchronize()
            wall.append((time.perf_counter() - t0) * 1e3)
            herm.append(st["ms"])
            stats.append(st)
        last = stats[-1]
        out[prec] = {"ms_per_step": float(np.median(wall)), "hermite_ms": float(np.median(herm)),
                     "n_hard": last["n_hard"], "n_clusters": last["n_clusters"],
                     "max_cluster": last["max_cluster"], "hermite_steps": last["steps"],
                     "max_block_steps": last["max_block_steps"],
                     "hermite_steps_per_s": last["steps"] / (last["ms"] * 1e-3)}
        log(f"bench: p3t step {prec}: {json.dumps(out[prec])}")
    if cpu:
        out["cpu_baseline"] = hermite_cpu_baseline(ctx, w, c, hk, cpu_target_s)
    return out


def hermite_cpu_baseline(ctx, w, c, hk, target_s, seed=4):
    """The oracle's block-step Hermite integration (single-threaded, as it
    stands) on whole clusters of the step-0 neighbour lists, drawn at random
    until about target_s seconds of work; in Hermite steps per second."""
    import oracle
    import torch
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    params = w.params(precision="fp64")
    dev = torch.device("cuda", 0)
    ctx.build_tree(torch.from_numpy(c.pos).to(dev), torch.from_numpy(c.mass).to(dev), **params)
    off, idx = (t.cpu().numpy() for t in ctx.neighbors())
    n = len(off) - 1
    hard = np.diff(off) > 0
    _, lab = connected_components(csr_matrix((np.ones(len(idx)), idx, off), shape=(n, n)),
                                  directed=False)
    comps = np.unique(lab[hard])
    rng = np.random.default_rng(seed)
    rng.shuffle(comps)
    kw = {k: hk[k] for k in ("dt_soft", "dt_max", "eta", "eta_s", "a0")}
    done_steps, secs, used, parts, start = 0, 0.0, 0, 0, 0
    chunk = 64
    while secs < target_s and start < len(comps):
        pick = comps[start:start + chunk]
        start += chunk
        sel = np.nonzero(np.isin(lab, pick) & hard)[0]
        remap = -np.ones(n, np.int64)
        remap[sel] = np.arange(len(sel))
        rows = [remap[idx[off[i]:off[i + 1]]] for i in sel]
        soff = np.zeros(len(sel) + 1, np.int64)
        soff[1:] = np.cumsum([len(r) for r in rows])
        sidx = np.concatenate(rows).astype(np.int32)
        t0 = time.perf_counter()
        _, _, ns, _ = oracle.hermite(c.pos[sel], c.vel[sel], c.mass[sel], soff, sidx, params["eps"],
                                     params["r_in"], params["r_out"], **kw)
        secs += time.perf_counter() - t0
        done_steps += int(ns.sum())
        used += len(pick)
        parts += len(sel)
        chunk = min(4 * chunk, 4096)
    return {"value": done_steps / secs, "unit": "Hermite steps/s", "cores": 1, "kind": "oracle",
            "sample": f"block-step Hermite of {used} whole clusters ({parts} particles, "
                      f"{done_steps} steps) of the step-0 neighbour lists, {secs:.1f} s"}


def sweep(args):
    """theta x n_crit sweep on the 2^22 Plummer/Salpeter workload: FP32-compensated
    vs FP64 interaction kernels, throughput and RMS / max force error on sampled
    groups against the oracle.  Prints one JSON line per setting."""
    import torch
    import oracle
    from inputs import WORKLOADS, make_cluster
    from paper_1506_04553_amd import P3T
    w = WORKLOADS["plummer4m_salpeter"]
    c = make_cluster(w, seed=args.seed)
    dev = torch.device("cuda", 0)
    pos = torch.from_numpy(c.pos).to(dev)
    mass = torch.from_numpy(c.mass).to(dev)
    ctx = P3T(0)
    rng = np.random.default_rng(7)
    for theta in w.extra["thetas"]:
        for n_crit in w.extra["n_crits"]:
            base = w.params(theta=theta, n_crit=n_crit)
            t0 = time.perf_counter()
            # the oracle walks every stride-th group only (about 640 of them), and
            # 512 of those are checked
            G_est = oracle.Tree(c.pos, c.mass, base, walk_stride=1 << 30).n_groups
            stride = max(1, G_est // 640)
            tree = oracle.Tree(c.pos, c.mass, base, walk_stride=stride)
            t_or = time.perf_counter() - t0
            G = tree.n_groups
            walked = np.arange(0, G, stride)
            sample = rng.choice(walked, min(len(walked), 512), replace=False)
            ra, rp = tree.force_groups(sample)
            rows = np.nonzero(~np.isnan(rp))[0]
            line = {"workload": w.name, "n": w.n, "theta": theta, "n_crit": n_crit,
                    "groups": G, "oracle_build_s": t_or, "sample_particles": int(len(rows))}
            for prec in ("mixed", "fp64"):
                p = dict(base, precision=prec)
                ctx.build_tree(pos, mass, **p)
                acc, pot = ctx.long_force()
                fms = []
                for _ in range(3):
                    ctx.long_force(acc, pot)
                    fms.append(ctx.stats()["ms_force"])
                st = ctx.stats()
                a = acc.cpu().numpy()[rows]
                e = np.linalg.norm(a - ra[rows], axis=1) / np.linalg.norm(ra[rows], axis=1)
                inter = st["n_pp"] + st["n_pc"]
                f_ms = float(np.median(fms))
                flops = st["n_pp"] * F_PP + st["n_pc"] * F_PC_QUAD
                line[prec] = {"force_ms": f_ms, "build_ms": st["ms_build"],
                              "interactions": inter, "interactions_per_s": inter / (f_ms * 1e-3),
                              "tflops": flops / (f_ms * 1e-3) / 1e12,
                              "acc_rel_rms": float(np.sqrt(((a - ra[rows]) ** 2).sum()
                                                           / (ra[rows] ** 2).sum())),
                              "acc_max_rel": float(e.max())}
            line["speedup_mixed_vs_fp64"] = line["fp64"]["force_ms"] / line["mixed"]["force_ms"]
            print(json.dumps(line), flush=True)
    ctx.close()


def small_configs(args, reps=10):
    """The small workloads (Plummer 4096 FP64; Plummer 65536 Salpeter FP64 and
    mixed): build and interaction-kernel times (median of reps, HIP events),
    interactions/s, TFLOP/s, and the force and potential error against the
    whole oracle force.  One JSON line per (workload, precision)."""
    import torch
    import oracle
    from inputs import WORKLOADS, make_cluster
    from paper_1506_04553_amd import P3T
    ctx = P3T(0)
    dev = torch.device("cuda", 0)
    for name, precs in (("plummer4k", ("fp64",)), ("plummer64k_salpeter", ("fp64", "mixed"))):
        w = WORKLOADS[name]
        c = make_cluster(w, seed=args.seed)
        pos = torch.from_numpy(c.pos).to(dev)
        mass = torch.from_numpy(c.mass).to(dev)
        t0 = time.perf_counter()
        oa, op = oracle.Tree(c.pos, c.mass, w.params()).force()
        t_or = time.perf_counter() - t0
        for prec in precs:
            p = w.params(precision=prec)
            bms, fms = [], []
            for _ in range(reps):
                ctx.build_tree(pos, mass, **p)
                acc, pot = ctx.long_force()
                st = ctx.stats()
                bms.append(st["ms_build"])
                fms.append(st["ms_force"])
            a, ph = acc.cpu().numpy(), pot.cpu().numpy()
            e = np.linalg.norm(a - oa, axis=1) / np.linalg.norm(oa, axis=1)
            f_ms = float(np.median(fms))
            inter = st["n_pp"] + st["n_pc"]
            flops = st["n_pp"] * F_PP + st["n_pc"] * F_PC_QUAD
            peak = PEAK_TFLOPS[prec]
            print(json.dumps({
                "workload": name, "n": w.n, "precision": prec, "theta": w.theta,
                "n_crit": w.n_crit, "build_ms": float(np.median(bms)), "force_ms": f_ms,
                "interactions": inter, "interactions_per_s": inter / (f_ms * 1e-3),
                "tflops": flops / (f_ms * 1e-3) / 1e12, "peak_tflops": peak,
                "acc_rel_rms": float(np.sqrt(((a - oa) ** 2).sum() / (oa ** 2).sum())),
                "pot_rel_rms": float(np.sqrt(((ph - op) ** 2).sum() / (op ** 2).sum())),
                "acc_max_rel": float(e.max()), "oracle_force_s": t_or,
                "oracle_cores": oracle.num_threads()}), flush=True)
    ctx.close()


def hermite_probe(reps=3, seed=0):
    """Block-step latency of the Hermite hard part: isolated groups of k equal
    stars (mass 1e-6, scatter a, 0.05 apart, lists within h inside each group),
    integrated over one soft step of the King 2^20 workload's parameters; alone
    (latency) and replicated (load).  One JSON line per case, best of reps."""
    import torch
    from paper_1506_04553_amd import P3T
    prm = dict(eps=3.8e-6, r_in=2e-4, r_out=2e-3, theta=0.5, r_search=2.2e-3, n_crit=256,
               n_leaf=16, precision="fp64")
    dt = 1.0 / 256
    hk = dict(dt_soft=dt, dt_max=dt * HERMITE["dt_max_per_soft"], eta=HERMITE["eta"],
              eta_s=HERMITE["eta"] / 10, a0=HERMITE["alpha"] * 1e-6 / prm["r_out"] ** 2)
    h2 = prm["r_search"] ** 2
    ctx = P3T(0)
    dev = torch.device("cuda", 0)
    for copies, k, a in [(1, 2, 3e-5), (1, 4, 5e-5), (1, 16, 1e-4), (1, 48, 2e-4),
                         (1024, 2, 3e-5), (16384, 2, 3e-5), (4096, 8, 6e-5)]:
        rng = np.random.default_rng(seed)
        side = int(np.ceil(copies ** (1 / 3)))
        grid = np.stack(np.meshgrid(*[np.arange(side)] * 3, indexing="ij"), -1).reshape(-1, 3)
        centres = grid[:copies] * 0.05
        pos = (centres[:, None, :] + rng.normal(scale=a, size=(copies, k, 3))).reshape(-1, 3)
        vel = rng.normal(scale=np.sqrt(k * 1e-6 / a), size=(copies * k, 3))
        mass = np.full(copies * k, 1e-6)
        rows = []
        for g in range(copies):
            p = pos[g * k:(g + 1) * k]
            d = p[None, :, :] - p[:, None, :]
            r2 = d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2]
            np.fill_diagonal(r2, np.inf)
            rows += [g * k + np.nonzero(r2[i] < h2)[0] for i in range(k)]
        off = np.zeros(copies * k + 1, np.int64)
        off[1:] = np.cumsum([len(r) for r in rows])
        idx = np.concatenate(rows).astype(np.int32)
        best, st = None, None
        for _ in range(reps):
            x = torch.from_numpy(pos.copy()).to(dev)
            v = torch.from_numpy(vel.copy()).to(dev)
            _, st = ctx.hermite_hard(x, v, torch.from_numpy(mass).to(dev),
                                     torch.from_numpy(off).to(dev), torch.from_numpy(idx).to(dev),
                                     hk, **prm)
            best = st["ms"] if best is None else min(best, st["ms"])
        print(json.dumps({"copies": copies, "members": k, "scatter": a, "list_entries": len(idx),
                          "max_block_steps": st["max_block_steps"], "hermite_steps": st["steps"],
                          "ms": best,
                          "us_per_block_step": 1e3 * best / max(1, st["max_block_steps"])}),
              flush=True)
    ctx.close()


def copy_calibration(mib=512, reps=3):
    """A plain device-to-device copy of known size, for scaling HBM byte counters
    (FETCH_SIZE / WRITE_SIZE) read by a profiler in the same way as the kernels."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.arange(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "reps": reps,
                      "kib_per_copy": n * 8 // 1024}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="king9_1m")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-vjp", action="store_true", help="skip the VJP timing")
    ap.add_argument("--no-direct", action="store_true", help="skip the O(N^2) direct-sum timing")
    ap.add_argument("--no-p3t", action="store_true",
                    help="skip the whole-P3T-step timing (soft step plus Hermite hard part)")
    ap.add_argument("--sweep", action="store_true",
                    help="run the theta x n_crit sweep on the 2^22 workload instead")
    ap.add_argument("--configs", action="store_true",
                    help="time the small workloads (Plummer 4096, Plummer 65536 Salpeter) instead")
    ap.add_argument("--hermite-probe", action="store_true",
                    help="time the Hermite hard part on isolated groups (block-step latency)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 512 MiB device copy (profiler counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(one process drives one GPU; there is no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return
    if args.hermite_probe:
        hermite_probe()
        return
    if args.sweep:
        sweep(args)
        return
    if args.configs:
        small_configs(args)
        return

    import torch
    from inputs import WORKLOADS, make_cluster
    from paper_1506_04553_amd import P3T

    w = WORKLOADS[args.workload]
    dt = w.extra.get("dt", 1.0 / 256)
    log(f"bench: generating {w.name} N={w.n} seed={args.seed}")
    c = make_cluster(w, seed=args.seed)
    dev = torch.device("cuda", 0)
    pos0 = torch.from_numpy(c.pos).to(dev)
    vel0 = torch.from_numpy(c.vel).to(dev)
    mass = torch.from_numpy(c.mass).to(dev)
    ctx = P3T(0)
    quad = True
    results, firsts = {}, {}
    precs = [args.precision] + ([] if args.no_fp64 else
                                [p for p in ("mixed", "fp64") if p != args.precision])
    for prec in precs:
        params = w.params(precision=prec)
        log(f"bench: {prec}: {args.warmup} warmup + {args.steps} timed steps")
        secs, rec, first = run_steps(ctx, pos0, vel0, mass, params, dt, args.steps, args.warmup,
                                     collect_first=True)
        results[prec] = summarize(rec, secs, args.steps, quad)
        firsts[prec] = (first[0].cpu().numpy(), first[1].cpu().numpy())
        log(f"bench: {prec}: {json.dumps(results[prec])}")
        if prec == args.precision:
            # right after the timed steps, in the same clock state
            log("bench: interaction kernel alone")
            iso = isolated_force(ctx, pos0, mass, w.params(precision=prec), quad)
    head = results[args.precision]
    peak = PEAK_TFLOPS[args.precision]
    iso["frac"] = iso["achieved"] / peak
    iso["frac_survey"] = iso["achieved_survey"] / peak
    tr = recorded_traffic(w.name, args.precision)
    traffic = None if tr is None else tr["fetch_bytes"] + tr["write_bytes"]
    out = {
        "metric": METRIC,
        "value": head["interactions_per_s"],
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "distribution": "King W0=9" if w.model == "king9"
                   else "Plummer", "imf": w.imf, "theta": w.theta, "n_crit": w.n_crit,
                   "n_leaf": w.n_leaf, "r_out": w.r_out, "r_in": w.r_in, "r_search": w.r_search,
                   "eps": w.eps, "dt": dt, "precision": args.precision, "seed": args.seed},
        "roofline": {"bound": "alu", "kernel": f"k_force<{'float' if args.precision == 'mixed' else 'double'}>",
                     "achieved": head["force_tflops"], "peak": peak, "unit": "TFLOP/s",
                     "frac": head["force_tflops"] / peak, "traffic": traffic,
                     "issue_ceiling": PEAK_UNPACKED_FP32 if args.precision == "mixed" else peak,
                     "frac_of_issue_ceiling": head["force_tflops"] /
                     (PEAK_UNPACKED_FP32 if args.precision == "mixed" else peak),
                     "traffic_split": None if tr is None else
                     {"fetch_bytes": tr["fetch_bytes"], "write_bytes": tr["write_bytes"],
                      "source": os.path.relpath(TRAFFIC_FILE, ROOT)},
                     "flops_per_launch": head["flops_per_launch"],
                     "avg_launch_ms": head["force_ms"],
                     "flops_per_interaction": {"pp": F_PP, "pc": F_PC_QUAD},
                     "achieved_survey": head["force_tflops_survey"],
                     "frac_survey": head["force_tflops_survey"] / peak,
                     "flops_per_interaction_survey": {"pp": F_PP_SURVEY, "pc": F_PC_SURVEY},
                     "isolated": iso},
        # the neighbour search runs on a second stream beside the interaction
        # kernel: its span overlaps "force" and the two do not add up
        "phase_ms": {"build": head["build_ms"], "force": head["force_ms"],
                     "neighbors_concurrent": head["neighbors_ms"]},
        "build": build_roofline(head, w.n),
        "walk": walk_rates(head),
        "interactions_per_step": head["interactions_per_step"],
        "interactions_split": {"particle_cell": head["n_pc"], "particle_particle": head["n_pp"],
                               "of_which_near": head["n_pp_near"]},
        "list_entries": head["list_entries"],
        "n_groups": head["n_groups"],
        "neighbour_pairs": head["nnz"],
    }
    if "fp64" in results and args.precision != "fp64":
        f64 = results["fp64"]
        out["fp64"] = {"ms_per_step": f64["ms_per_step"], "interactions_per_s": f64["interactions_per_s"],
                       "force_ms": f64["force_ms"], "force_tflops": f64["force_tflops"],
                       "force_frac_of_fp64_peak": f64["force_tflops"] / PEAK_TFLOPS["fp64"],
                       "force_frac_of_fp64_peak_survey":
                           f64["force_tflops_survey"] / PEAK_TFLOPS["fp64"]}
        out["speedup_mixed_vs_fp64"] = {"force_kernel": f64["force_ms"] / head["force_ms"],
                                        "step": f64["ms_per_step"] / head["ms_per_step"]}
        a32, p32 = firsts["mixed"]
        a64, p64 = firsts["fp64"]
        out["mixed_vs_fp64_gpu"] = {
            "acc_rel_rms": float(np.sqrt(((a32 - a64) ** 2).sum() / (a64 ** 2).sum())),
            "pot_rel_rms": float(np.sqrt(((p32 - p64) ** 2).sum() / (p64 ** 2).sum()))}
    if not args.no_vjp:
        log("bench: VJP timing")
        out["vjp"] = vjp_timing(ctx)
    if not args.no_direct:
        log("bench: O(N^2) direct sums")
        out["direct"] = direct_timing(ctx, cpu=not args.no_cpu_baseline)
    if not args.no_p3t:
        log("bench: P3T steps with the Hermite hard part")
        out["p3t_step"] = p3t_step_timing(ctx, w, c, dt, cpu=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline on sampled groups")
        cb, errs = cpu_baseline(c.pos, c.mass, w.params(), firsts)
        out["cpu_baseline"] = cb
        out["rms_err_vs_oracle"] = errs
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
