#!/usr/bin/env python3
"""Chemistry cells/s of the BF16 ANN step and of the FP64 integrator step on
one MI355X (2^20 cells of the 30-species / 150-reaction CH4/air mechanism,
dt = 1e-5 s), at the error measured against the CPU oracle.

One timed step = one ann_step call over all cells (network, post-processing
and FP64 fallback of flagged cells), with the input state restored from a
pristine device copy first.  The FP64 integrator (chem_step) is timed the
same way for the ratio.  The network is trained first on this GPU by the
library's own kernels (labels from chem_step on perturbed states) unless
--model names a saved one.  Prints one JSON line on stdout; progress goes to
stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "chemistry cells/s per step: BF16 ANN vs FP64 stiff integrator, at stated error"
PEAK_BF16 = 2500e12   # dense MFMA, FLOP/s
PEAK_FP64 = 78.6e12   # vector FP64, FLOP/s
PEAK_FP8 = 5000e12    # dense MFMA, FLOP/s
PEAK_HBM = 8e12       # HBM3E, bytes/s
HIDDEN = (1600, 800, 400)
COPY_PROBE_DOUBLES = 1 << 25   # 256 MiB read + 256 MiB written by one plain copy kernel
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rodas3_flops_per_attempt(mech):
    """Algorithmic FP64 flops of one attempted RODAS3 step of one cell (FMA =
    2), counted from the method, not from the kernel: one analytic Jacobian
    (40 R + 3 n^2), three right-hand sides (16 K + 33 R + 6 K each), forming
    the Newton matrix (n^2), its LU ((2/3) n^3), four pairs of triangular
    solves (2 n^2 each), the stage combinations (s^2 n) and the error norm
    (4 n); the exponentials of the rate constants (2 R per right-hand side)
    are counted separately."""
    K, R = mech.K, mech.R
    n = K + 1
    s, s_f = 4, 3
    f_rhs = 16 * K + 25 * R + 8 * R + 6 * K
    f_jac = 40 * R + 3 * n * n
    return f_jac + s_f * f_rhs + n * n + (2.0 / 3.0) * n ** 3 + s * 2 * n * n + s * s * n + 4 * n


def rodas3_exp_per_attempt(mech):
    """Exponentials per attempted step: k_f and k_r of every reaction at each
    of the three right-hand sides."""
    return 2 * mech.R * 3


def mlp_flops_per_cell(K):
    dims = [K + 2, *HIDDEN, K]
    return sum(2 * a * b for a, b in zip(dims[:-1], dims[1:]))


def source_digest(paths):
    """sha256 over the named kernel sources (relative to the repository)."""
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(label):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary, or None when the kernel sources changed since the counters were
    taken (or none were taken)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get("kernels", {}).get(label)
    if not e or source_digest(e["sources"]) != e["sha256"]:
        return None
    return e["hbm_bytes_per_launch"]


def copy_probe(dev):
    """One plain device copy of known size (torch elementwise kernel), the
    calibration point for the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    src = torch.ones(COPY_PROBE_DOUBLES, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst


def _plain(o, path="out"):
    """The bench record with NumPy scalars and arrays turned into plain
    Python values (arrays are reported on stderr: they should not occur)."""
    import numpy as np
    if isinstance(o, dict):
        return {k: _plain(v, f"{path}.{k}") for k, v in o.items()}
    if isinstance(o, (list, tuple)):
        return [_plain(v, f"{path}[{i}]") for i, v in enumerate(o)]
    if isinstance(o, np.ndarray):
        log(f"[bench] array at {path} (shape {o.shape})")
        return o.tolist()
    if isinstance(o, np.generic):
        return o.item()
    return o


def make_labels(P, mech, gm, dev, args):
    """Training pairs: perturbed states integrated over dt by the FP64 GPU
    integrator (the final temperature T1 kept for the physics terms)."""
    import torch
    import chemgen
    cfg = dict(chemgen.STATE_CONFIGS["ch4_train"])
    T, p, Y0 = chemgen.make_states(mech, cfg, N=args.train_cells)
    Td, pd, Y0d = (torch.from_numpy(a).to(dev) for a in (T, p, Y0))
    T1d, Y1d = Td.clone(), Y0d.clone()
    st = torch.zeros((3, T.size), dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    tg = time.time()
    P.chem_step(gm, 1e-5, T1d, pd, Y1d, stats=st)
    torch.cuda.synchronize()
    t_label = time.time() - tg
    ok = (st[2] == 0)
    nbad = int((~ok).sum().item())
    keep = torch.nonzero(ok).flatten()
    lab = dict(T=Td[keep].contiguous(), p=pd[keep].contiguous(), Y0=Y0d[:, keep].contiguous(),
               Y1=Y1d[:, keep].contiguous(), T1=T1d[keep].contiguous())
    log(f"[train] labels for {T.size} states in {t_label:.2f} s ({nbad} failed)")
    return lab, dict(states=int(T.size), label_seconds=round(t_label, 3), failed_labels=nbad)


def train_model(P, mech, gm, dev, args, lab, w_phys, members=1):
    """Train the network (members = K: the per-species ensemble) on the
    labelled pairs (cosine lr decay), with the physics terms of the loss
    weighted by w_phys (zeros: L1 loss only)."""
    import numpy as np
    import torch
    K = mech.K
    Td, pd, Y0d, Y1d, T1d = lab["T"], lab["p"], lab["Y0"], lab["Y1"], lab["T1"]
    n = Td.shape[0]
    m = P.AnnModel(K + 2, K, HIDDEN, seed=args.seed, members=members)
    m.fit_norm(Td, pd, Y0d, Y1d, 0.1, 1e-5)
    # tilings of the step's products for this batch, by measurement
    tuning = m.autotune_train(args.batch)
    log(f"[train] autotuned products: {tuning}")
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    terms = torch.zeros(3, dtype=torch.float32, device=dev)
    phys = any(w != 0.0 for w in w_phys)
    rng = np.random.default_rng(args.seed)
    B = args.batch
    perm = None
    pos = n
    hist = []
    torch.cuda.synchronize()
    tt = time.time()
    for it in range(args.train_steps):
        if pos + B > n:
            perm = torch.from_numpy(rng.permutation(n).astype(np.int64)).to(dev)
            pos = 0
        idx = perm[pos:pos + B]
        pos += B
        frac = it / max(1, args.train_steps - 1)
        lr = 1e-5 + 0.5 * (args.lr - 1e-5) * (1 + math.cos(math.pi * frac))
        if phys:
            m.train_step(Td, pd, Y0d, Y1d, loss, index=idx, lr=lr, mech=gm, T1=T1d,
                         w_phys=w_phys, terms=terms)
        else:
            m.train_step(Td, pd, Y0d, Y1d, loss, index=idx, lr=lr)
        if it % 500 == 0 or it == args.train_steps - 1:
            hist.append((it, float(loss.item())))
            log(f"[train w={w_phys}] step {it} lr {lr:.2e} loss {hist[-1][1]:.5f}")
    torch.cuda.synchronize()
    t_train = time.time() - tt
    info = dict(steps=args.train_steps, batch=B, w_phys=list(w_phys), members=members,
                autotuned_products_ms={k: round(v, 4) for k, v in tuning.items()},
                train_seconds=round(t_train, 2),
                ms_per_train_step=round(1e3 * t_train / max(1, args.train_steps), 3),
                loss_first=hist[0][1] if hist else None, loss_last=hist[-1][1] if hist else None)
    if phys:
        info["physics_terms_last"] = [round(float(v), 6) for v in terms.cpu().numpy()]
    return m, info


def sampled_labels(P, mech, gm, dev, args):
    """Training pairs from the random-data generation of Sec. 3.1: the
    recipe's states as seeds, perturbed (or replaced by states on the line
    between the phi = 0.45 equilibrium and air), filtered by T >= 500 K and
    Table 1, then integrated over dt by the FP64 GPU integrator."""
    import numpy as np
    import torch
    import chemgen
    K = mech.K
    t0 = time.time()
    T, p, Y = chemgen.make_states(mech, "ch4", N=args.sample_seeds, seed=58)
    c, s = chemgen.hfrd_randoms(K, T.size, seed=59, mix_fraction=0.1)
    # the equilibrium end: the recipe's fully burnt phi = 0.45 state after 10 ms
    Te, pe, Ye = chemgen.burnt_state(mech, 0.45, 2300.0)
    Ted = torch.tensor([Te], dtype=torch.float64, device=dev)
    ped = torch.tensor([pe], dtype=torch.float64, device=dev)
    Yed = torch.from_numpy(Ye[:, None].copy()).to(dev)
    st = torch.zeros((3, 1), dtype=torch.int32, device=dev)
    P.chem_step(gm, 1e-2, Ted, ped, Yed, stats=st)
    Ta, pa, Ya = chemgen.air_state(mech)
    end_eq = torch.cat([Ted, ped, Yed[:, 0]])
    end_air = torch.from_numpy(np.concatenate([[Ta, pa], Ya])).to(dev)
    Td, pd, Yd = (torch.from_numpy(a).to(dev) for a in (T, p, Y))
    cd, sd = torch.from_numpy(c).to(dev), torch.from_numpy(s).to(dev)
    To, po, Yo, keep = P.sample_states(gm, mech, Td, pd, Yd, cd, sd, end_eq, end_air)
    kept = torch.nonzero(keep).flatten()
    lab = dict(T=To[kept].contiguous(), p=po[kept].contiguous(), Y0=Yo[:, kept].contiguous())
    del Td, pd, Yd, cd, sd, To, po, Yo
    T1d, Y1d = lab["T"].clone(), lab["Y0"].clone()
    stl = torch.zeros((3, T1d.shape[0]), dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    tg = time.time()
    P.chem_step(gm, 1e-5, T1d, lab["p"], Y1d, stats=stl)
    torch.cuda.synchronize()
    t_label = time.time() - tg
    ok = torch.nonzero(stl[2] == 0).flatten()
    lab = {k: (v[ok] if v.dim() == 1 else v[:, ok]).contiguous() for k, v in lab.items()}
    lab["Y1"] = Y1d[:, ok].contiguous()
    lab["T1"] = T1d[ok].contiguous()
    info = dict(seeds=int(T.size), kept=int(kept.numel()),
                kept_fraction=round(kept.numel() / T.size, 4),
                mixing_samples=int((s >= 0).sum()), equilibrium_end_T=float(Ted.item()),
                equilibrium_end_status=int(st[2, 0].item()), label_seconds=round(t_label, 3),
                failed_labels=int(kept.numel() - ok.numel()),
                seconds=round(time.time() - t0, 2))
    log(f"[sampler] {info}")
    return lab, info


def timed_loop(run, restore, steps, warmup):
    import torch
    for _ in range(warmup):
        restore()
        run()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        restore()
        run()
    torch.cuda.synchronize()
    return time.perf_counter() - t


def time_sets(P, mech, gm, dev, args, model=None):
    """Uneven batched workload (independent cell sets of very different size
    and dt): one chem_step launch per set, against all sets on one persistent
    queue (chem_step_sets) and that call replayed as a captured graph.  Each
    variant runs once from the same restored states; the three must agree bit
    for bit, and a sample of cells from every set is checked against the
    oracle."""
    import numpy as np
    import torch
    import chemgen
    import oracle
    ws = chemgen.multiset_workload(mech, seed=44, n_sets=args.sets,
                                   max_total=args.sets_max_cells or None)
    total = int(sum(w["N"] for w in ws))
    log(f"[sets] {len(ws)} sets, {total} cells")
    pristine = [(torch.from_numpy(w["T"]).to(dev), torch.from_numpy(w["p"]).to(dev),
                 torch.from_numpy(w["Y"]).to(dev)) for w in ws]
    live = [dict(dt=w["dt"], T=T0.clone(), p=p0, Y=Y0.clone(),
                 stats=torch.zeros((3, w["N"]), dtype=torch.int32, device=dev))
            for w, (T0, p0, Y0) in zip(ws, pristine)]

    def restore():
        for d, (T0, _, Y0) in zip(live, pristine):
            d["T"].copy_(T0)
            d["Y"].copy_(Y0)

    def snapshot():
        return [(d["T"].clone(), d["Y"].clone()) for d in live]

    def same(a, b):
        return all(torch.equal(x[0], y[0]) and torch.equal(x[1], y[1]) for x, y in zip(a, b))

    def per_set():
        for d in live:
            if d["T"].shape[0]:
                P.chem_step(gm, d["dt"], d["T"], d["p"], d["Y"], stats=d["stats"])

    t_naive = timed_loop(per_set, restore, 1, 0)
    ref = snapshot()
    t_queue = timed_loop(lambda: P.chem_step_sets(gm, live), restore, 1, 0)
    eq_queue = same(snapshot(), ref)
    attempts = int(sum(int(d["stats"][0].sum() + d["stats"][1].sum()) for d in live))
    g = P.chem_step_sets_graph(gm, live)
    t_graph = timed_loop(g.launch, restore, 1, 0)
    eq_graph = same(snapshot(), ref)
    del g
    # the table already on the device: offsets and count formed on the GPU
    table, nt = P.set_table_device(gm, live, device=dev)
    t_dev = timed_loop(lambda: P.chem_step_sets_device(gm, table, nt), restore, 1, 0)
    eq_dev = same(snapshot(), ref)
    # oracle on a stratified sample: every set contributes in proportion to
    # its size (at least one cell), args.sets_oracle cells in all
    om = oracle.OracleMech(mech)
    err = 0.0
    nchk = 0
    for w, d in zip(ws, live):
        if w["N"] == 0:
            continue
        k = max(1, min(w["N"], int(round(args.sets_oracle * w["N"] / total))))
        ii = np.unique(np.linspace(0, w["N"] - 1, k).astype(np.int64))
        o = oracle.chem_step(om, w["dt"], w["T"][ii], w["p"][ii], w["Y"][:, ii])
        Tg, Yg = d["T"].cpu().numpy()[ii], d["Y"].cpu().numpy()[:, ii]
        big = np.abs(o["Y"]) > 1e-10
        err = max(err, float(np.max(np.abs(Tg - o["T"]) / o["T"])),
                  float(np.max(np.abs(Yg - o["Y"])[big] / np.abs(o["Y"])[big])))
        nchk += ii.size
    # the surrogate on the same sets, at the step it was trained for (its
    # accuracy is not claimed for the sets' own dt): one ann_step per set
    ann_side = None
    if model is not None:
        restore()

        def ann_sets():
            for d in live:
                if d["T"].shape[0]:
                    model.step(gm, 1e-5, d["T"], d["p"], d["Y"])
        t_ann = timed_loop(ann_sets, restore, 1, 1)
        ann_side = {"dt": 1e-5, "s": round(t_ann, 4), "cells_per_s": round(total / t_ann, 1),
                    "calls": len([d for d in live if d["T"].shape[0]])}
    sizes = [w["N"] for w in ws]
    out = {"workload": f"{len(ws)} CH4/air cell sets, sizes floor(10^U(3,6)) "
                       f"({min(sizes)}..{max(sizes)}), dt 10^U(-7,-4) s per set, "
                       "T ~ U(300, 2500) K (seed 44)",
           "cells": total, "attempts_per_cell": round(attempts / max(total, 1), 3),
           "one_launch_per_set": {"s": round(t_naive, 3), "cells_per_s": round(total / t_naive, 1)},
           "persistent_queue": {"s": round(t_queue, 3), "cells_per_s": round(total / t_queue, 1),
                                "equal_to_per_set": eq_queue},
           "persistent_queue_graph": {"s": round(t_graph, 3),
                                      "cells_per_s": round(total / t_graph, 1),
                                      "equal_to_per_set": eq_graph},
           "persistent_queue_device_table": {"s": round(t_dev, 3),
                                             "cells_per_s": round(total / t_dev, 1),
                                             "equal_to_per_set": eq_dev},
           "max_rel_err_vs_oracle": err, "oracle_cells": nchk,
           "oracle_sample": "stratified: each set in proportion to its size",
           "ann_at_dt_model": ann_side}
    log(f"[sets] per-set {t_naive:.2f} s, queue {t_queue:.2f} s, graph {t_graph:.2f} s")
    return out


def nrmse_table(dY_model, dY_ref, Yref_mean, names, rtol=1e-6):
    """Range-normalised RMSE of Delta-Y per species.  Majors: mean Y >= 1e-3
    and a reference Delta-Y range of at least 10 rtol mean(Y), i.e. a change
    the reference integrator resolves at its own tolerance; abundant species
    whose change is below that are listed as unresolved and not gated."""
    import numpy as np
    out = {}
    for k, nm in enumerate(names):
        rng_ = float(dY_ref[k].max() - dY_ref[k].min())
        rmse = float(np.sqrt(np.mean((dY_model[k] - dY_ref[k]) ** 2)))
        abundant = bool(Yref_mean[k] >= 1e-3)
        resolved = bool(rng_ >= 10.0 * rtol * Yref_mean[k] and rng_ > 0)
        out[nm] = dict(nrmse=rmse / rng_ if rng_ > 0 else float("nan"), range=rng_,
                       major=abundant and resolved, unresolved=abundant and not resolved)
    majors = [v["nrmse"] for v in out.values() if v["major"]]
    return out, (max(majors) if majors else float("nan"))


def big_leg(P, mech, gm, dev, args, model):
    """Inference at the training-plus-FP8 configuration's size: the BF16 and
    the FP8 steps on args.big_cells cells, their error against the FP64 GPU
    integrator on every cell and against the oracle on 2^16 of them."""
    import numpy as np
    import torch
    import chemgen
    import oracle
    N = args.big_cells
    T, p, Y = chemgen.make_states(mech, "ch4", N=N, seed=57)
    T0d, pd, Y0d = (torch.from_numpy(a).to(dev) for a in (T, p, Y))
    Td, Yd = T0d.clone(), Y0d.clone()
    nfb = torch.zeros(1, dtype=torch.int64, device=dev)

    def restore():
        Td.copy_(T0d)
        Yd.copy_(Y0d)
    steps = 3
    out = {"workload": f"{N} stratified CH4/air cells (seed 57), dt=1e-5 s", "cells": N,
           "steps": steps}
    legs = {}
    for name, prec in (("bf16", 0), ("fp8", 1)):
        if prec == 1:
            try:
                model.set_precision(1)
            except P.ChemError:
                continue
        t = timed_loop(lambda: model.step(gm, 1e-5, Td, pd, Yd, n_fallback=nfb), restore, steps,
                       1)
        legs[name] = Yd.cpu().numpy()
        out[name] = {"cells_per_s": round(N * steps / t, 1),
                     "ms_per_step": round(1e3 * t / steps, 3),
                     "fallback_cells": int(nfb.item())}
        log(f"[large {name}] {N} cells: {1e3 * t / steps:.2f} ms per step")
    model.set_precision(0)
    restore()
    torch.cuda.synchronize()
    tf = time.time()
    P.chem_step(gm, 1e-5, Td, pd, Yd)
    torch.cuda.synchronize()
    tf = time.time() - tf
    fp_Y = Yd.cpu().numpy()
    out["fp64"] = {"cells_per_s": round(N / tf, 1), "s": round(tf, 3)}
    log(f"[large fp64] {tf:.2f} s")
    dY_fp = fp_Y - Y
    fm = fp_Y.mean(axis=1)
    for name, Yv in legs.items():
        _, out[name]["nrmse_major_max_vs_gpu_fp64_all_cells"] = nrmse_table(Yv - Y, dY_fp, fm,
                                                                             mech.species)
    del dY_fp
    idx = np.linspace(0, N - 1, 1 << 16).astype(np.int64)
    o = oracle.chem_step(oracle.OracleMech(mech), 1e-5, T[idx], p[idx], Y[:, idx])
    dY_ref = o["Y"] - Y[:, idx]
    for name, Yv in legs.items():
        _, out[name]["nrmse_major_max_vs_oracle"] = nrmse_table(
            Yv[:, idx] - Y[:, idx], dY_ref, o["Y"].mean(axis=1), mech.species)
    big = np.abs(o["Y"]) > 1e-10
    out["fp64"]["max_rel_err_vs_oracle"] = max(
        float(np.max(np.abs(fp_Y[:, idx] - o["Y"])[big] / np.abs(o["Y"])[big])), 0.0)
    out["oracle_sample_cells"] = int(idx.size)
    return out


def n_params(K):
    dims = [K + 2, *HIDDEN, K]
    return sum(a * b + b for a, b in zip(dims[:-1], dims[1:]))


def train_roofline(info, K):
    """One Adam step of the batch: forward, data and weight gradients (three
    times the forward's flops) against the BF16 MFMA peak; the optimiser's
    bytes (FP32 weights, gradients and two moments read, three of them
    written, the BF16 copy written: 30 B per parameter) against HBM."""
    ms = info.get("ms_per_train_step")
    if not ms:
        return None
    B = info["batch"]
    G = info.get("members", 1)
    if G > 1:
        # K single-output members, every product of the step one grouped launch
        per_cell = G * sum(2 * a * b for a, b in zip([K + 2, *HIDDEN], [*HIDDEN, 1]))
        params = G * sum((a + 1) * b for a, b in zip([K + 2, *HIDDEN], [*HIDDEN, 1]))
    else:
        per_cell = mlp_flops_per_cell(K)
        params = n_params(K)
    flops = 3.0 * per_cell * B
    ach = flops / (ms * 1e-3)
    adam_bytes = 30.0 * params
    return {"kernel": "one training step (all launches)" if G == 1 else
            f"one training step of the {G}-member ensemble (grouped launches)", "bound": "mfma",
            "achieved": round(ach / 1e12, 2), "peak": PEAK_BF16 / 1e12, "unit": "TFLOP/s",
            "frac": round(ach / PEAK_BF16, 4), "flops_per_step": flops, "batch": B,
            "ms_per_step": ms, "adam_bytes_per_step": adam_bytes,
            "adam_bytes_time_at_8TBps_ms": round(adam_bytes / 8e12 * 1e3, 4)}


def fp8_roof(prof, K, chunk):
    """Time-weighted roof of the FP8 network: its BF16 flops (first and last
    layers) at the BF16 peak plus its FP8 flops (hidden-to-hidden layers) at
    the FP8 peak, against the measured time of its network kernels."""
    f_bf16 = 2.0 * ((K + 2) * HIDDEN[0] + HIDDEN[2] * K) * chunk
    f_fp8 = 2.0 * (HIDDEN[0] * HIDDEN[1] + HIDDEN[1] * HIDDEN[2]) * chunk
    t_roof = f_bf16 / PEAK_BF16 + f_fp8 / PEAK_FP8
    labels = ("mlp_l1", "mlp_l2_fp8", "mlp_l3_l4_fp8", "mlp_l3_fp8", "mlp_l4")
    t_net = 0.0
    for lab in labels:
        c, tot = prof.get(lab, (0, 0.0))
        if c:
            t_net += tot / c * 1e-3
    if t_net <= 0.0:
        return None
    return {"bf16_flops": f_bf16, "fp8_flops": f_fp8, "roof_ms": round(t_roof * 1e3, 4),
            "network_ms": round(t_net * 1e3, 4), "frac": round(t_roof / t_net, 4),
            "kernels": [lab for lab in labels if prof.get(lab, (0, 0))[0]]}


def small_config(P, dev, oracle, nthr):
    """The 9-species H2/air configuration (4096 cells, dt = 1e-6 s): GPU chem_step
    cells/s, parity with the oracle on every cell, and the oracle's cells/s."""
    import numpy as np
    import torch
    import chemgen
    mech = chemgen.make_mechanism("h2")
    T, p, Y = chemgen.make_states(mech, "h2")
    N, dt = T.size, 1e-6
    gm = P.Mechanism(mech)
    T0d, pd, Y0d = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (T, p, Y))
    Td, Yd = T0d.clone(), Y0d.clone()

    def restore():
        Td.copy_(T0d)
        Yd.copy_(Y0d)
    steps = 20
    t = timed_loop(lambda: P.chem_step(gm, dt, Td, pd, Yd), restore, steps, 2)
    om = oracle.OracleMech(mech)
    tc = time.time()
    o = oracle.chem_step(om, dt, T, p, Y)
    tc = time.time() - tc
    gT, gY = Td.cpu().numpy(), Yd.cpu().numpy()
    big = np.abs(o["Y"]) > 1e-10
    err = max(float(np.max(np.abs(gT - o["T"]) / o["T"])),
              float(np.max(np.abs(gY - o["Y"])[big] / np.abs(o["Y"])[big])))
    return {"workload": f"H2/air, {mech.K} species / {mech.R} reactions, {N} cells, dt=1e-6 s",
            "gpu_cells_per_s": round(N * steps / t, 1), "gpu_ms_per_step": round(1e3 * t / steps, 4),
            "max_rel_err_vs_oracle": err, "oracle_cells_per_s": round(N / tc, 1),
            "oracle_cores": nthr}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cells", type=int, default=1 << 20)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--model", default=None, help="load a saved model instead of training")
    ap.add_argument("--save-model", default=None)
    ap.add_argument("--train-cells", type=int, default=1 << 22)
    ap.add_argument("--train-steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=55)
    ap.add_argument("--oracle-sample", type=int, default=1 << 16)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--fp8", type=int, default=1, help="also time FP8 hidden layers (1/0)")
    ap.add_argument("--sets", type=int, default=64,
                    help="time the uneven multi-set workload with this many sets (0: skip)")
    ap.add_argument("--sets-max-cells", type=int, default=1 << 22,
                    help="scale the set sizes down to at most this many cells in total "
                         "(0: the drawn sizes)")
    ap.add_argument("--sets-oracle", type=int, default=1 << 16,
                    help="cells of the stratified oracle sample of the sets")
    ap.add_argument("--w-phys", type=str, default="1.0,0.3,0.3",
                    help="weights of the loss's mass, energy and heat-release terms")
    ap.add_argument("--compare-phys", type=int, default=1,
                    help="also train without the physics terms and report its accuracy")
    ap.add_argument("--big-cells", type=int, default=1 << 23,
                    help="cells of the large inference leg (BF16 and FP8; 0: skip)")
    ap.add_argument("--peaks", type=int, default=1, help="measure attainable peaks (1/0)")
    ap.add_argument("--ensemble", type=int, default=1,
                    help="also train and time the per-species ensemble of Sec. 3.2 (1/0)")
    ap.add_argument("--sample-seeds", type=int, default=1 << 21,
                    help="seeds of the Sec. 3.1 sampler leg (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the chemistry step has no inter-GPU exchange "
              "and this benchmark runs on a single MI355X; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import chemgen
    import paper_2312_05800_amd as P

    dev = torch.device("cuda:0")
    mech = chemgen.make_mechanism("ch4")
    K = mech.K
    gm = P.Mechanism(mech)
    N = args.cells

    w_phys = tuple(float(x) for x in args.w_phys.split(","))
    model_plain = None
    train_plain = None
    model_sampled = None
    sample_info = None
    model_ens = None
    train_ens = None
    if args.model and os.path.exists(args.model):
        model = P.AnnModel.load(args.model)
        train_info = dict(loaded=args.model)
    else:
        t0 = time.time()
        lab, train_info = make_labels(P, mech, gm, dev, args)
        model, tinfo = train_model(P, mech, gm, dev, args, lab, w_phys)
        train_info.update(tinfo)
        if args.compare_phys and any(w != 0.0 for w in w_phys):
            model_plain, train_plain = train_model(P, mech, gm, dev, args, lab, (0.0, 0.0, 0.0))
        if args.ensemble:
            # one network per species on the same pairs; the members each see
            # one species, so the loss is the L1 loss alone
            model_ens, train_ens = train_model(P, mech, gm, dev, args, lab, (0.0, 0.0, 0.0),
                                               members=K)
        if args.sample_seeds:
            del lab
            torch.cuda.empty_cache()
            lab, sample_info = sampled_labels(P, mech, gm, dev, args)
            model_sampled, tinfo = train_model(P, mech, gm, dev, args, lab, w_phys)
            sample_info.update(training=tinfo)
        train_info["total_seconds"] = round(time.time() - t0, 2)
        if args.save_model:
            model.save(args.save_model)
        del lab
        torch.cuda.empty_cache()

    T, p, Y = chemgen.make_states(mech, "ch4", N=N)
    T0d, pd, Y0d = (torch.from_numpy(a).to(dev) for a in (T, p, Y))
    Td, Yd = T0d.clone(), Y0d.clone()
    RR = torch.zeros((K, N), dtype=torch.float64, device=dev)
    flags = torch.zeros(N, dtype=torch.uint8, device=dev)
    nfb = torch.zeros(1, dtype=torch.int64, device=dev)

    def restore():
        Td.copy_(T0d)
        Yd.copy_(Y0d)

    # ---- BF16 ANN step (with FP64 fallback) ----
    P.profile_enable(True)
    P.profile_read()
    t_ann = timed_loop(lambda: model.step(gm, 1e-5, Td, pd, Yd, RR=RR, flags=flags,
                                          n_fallback=nfb),
                       restore, args.steps, args.warmup)
    prof_ann = P.profile_read()
    ann_T, ann_Y = Td.cpu().numpy(), Yd.cpu().numpy()
    n_fallback = int(nfb.item())
    log(f"[ann] {args.steps} steps in {t_ann:.3f} s; fallback cells {n_fallback}")

    # ---- PaSR closure of the step's rates (Sec. 4.1) ----
    tT_np, tK_np = chemgen.flow_times(N, seed=76)
    tTd, tKd = (torch.from_numpy(a).to(dev) for a in (tT_np, tK_np))
    RR_ann = RR.clone()  # the network's rates of the last step
    RRw = RR_ann.clone()
    # back-to-back closures (each scales the last one's rates again: the same
    # bytes move), so the host stays ahead of the GPU and the library's
    # per-launch events time the kernel alone
    for _ in range(args.warmup):
        P.pasr_scale(gm, Td, pd, Yd, RRw, tTd, tKd, want_tau_c=False)
    torch.cuda.synchronize()
    P.profile_read()
    t_pasr = time.perf_counter()
    for _ in range(args.steps):
        P.pasr_scale(gm, Td, pd, Yd, RRw, tTd, tKd, want_tau_c=False)
    torch.cuda.synchronize()
    t_pasr = time.perf_counter() - t_pasr
    prof_pasr = P.profile_read()
    RRw.copy_(RR_ann)
    kap_ann = P.pasr_scale(gm, Td, pd, Yd, RRw, tTd, tKd)[0].cpu().numpy()
    RRpasr_ann = RRw.cpu().numpy()
    del RRw
    # the whole step with the closure: network, fallback, then the closure
    P.profile_read()
    t_ann_pasr = timed_loop(lambda: (model.step(gm, 1e-5, Td, pd, Yd, RR=RR, flags=flags,
                                                n_fallback=nfb),
                                     P.pasr_scale(gm, Td, pd, Yd, RR, tTd, tKd,
                                                  want_tau_c=False)),
                            restore, args.steps, args.warmup)
    P.profile_read()
    log(f"[pasr] {args.steps} closures in {t_pasr:.4f} s; step + closure {t_ann_pasr:.3f} s")

    # ---- the audit: the integrator judging the network inside the step ----
    aud = torch.zeros(3 + 3 * K, dtype=torch.float64, device=dev)
    aud_frac = 1.0 / 64
    t_aud = timed_loop(lambda: model.step(gm, 1e-5, Td, pd, Yd, RR=RR, flags=flags,
                                          n_fallback=nfb, audit_fraction=aud_frac, audit=aud),
                       restore, 3, 1)
    aud_np = aud.cpu().numpy()
    log(f"[audit] 3 audited steps in {t_aud:.3f} s; compared {int(aud_np[0])} cells")

    # ---- the same step captured as a HIP graph: one launch per step ----
    P.profile_enable(False)
    graph = model.step_graph(gm, 1e-5, Td, pd, Yd, RR=RR, flags=flags, n_fallback=nfb)
    t_graph = timed_loop(graph.launch, restore, args.steps, args.warmup)
    graph_equal = bool(np.array_equal(Td.cpu().numpy(), ann_T) and
                       np.array_equal(Yd.cpu().numpy(), ann_Y))
    del graph
    P.profile_enable(True)
    P.profile_read()
    log(f"[ann graph] {args.steps} steps in {t_graph:.3f} s; equal to eager: {graph_equal}")

    # ---- FP8 E4M3 hidden layers (static per-tensor scales from 2^16 states) ----
    fp8 = None
    if args.fp8:
        Tc, pc, Yc = chemgen.make_states(mech, "ch4_val")
        model.quantize_fp8(*(torch.from_numpy(a).to(dev) for a in (Tc, pc, Yc)))
        P.profile_read()
        t_fp8 = timed_loop(lambda: model.step(gm, 1e-5, Td, pd, Yd, RR=RR, flags=flags,
                                              n_fallback=nfb),
                           restore, args.steps, args.warmup)
        prof_fp8 = P.profile_read()
        fp8 = dict(T=Td.cpu().numpy(), Y=Yd.cpu().numpy(), t=t_fp8, prof=prof_fp8,
                   fallback=int(nfb.item()), scales=[v.tolist() for v in model.fp8_scales()])
        model.set_precision(0)
        log(f"[fp8] {args.steps} steps in {t_fp8:.3f} s; fallback cells {fp8['fallback']}")

    # ---- the per-species ensemble (Sec. 3.2): the same step with K networks ----
    ens = None
    if model_ens is not None:
        steps_e = max(1, min(args.steps, 3))
        P.profile_read()
        t_ens = timed_loop(lambda: model_ens.step(gm, 1e-5, Td, pd, Yd, RR=RR, flags=flags,
                                                  n_fallback=nfb),
                           restore, steps_e, 1)
        prof_ens = P.profile_read()
        ens = dict(t=t_ens, steps=steps_e, fallback=int(nfb.item()), prof=prof_ens)
        log(f"[ensemble] {steps_e} steps in {t_ens:.3f} s; fallback cells {ens['fallback']}")

    # ---- FP64 integrator step, launch shape from the autotuner ----
    tune_default = P.chem_get_tuning(gm)
    si = torch.from_numpy(np.linspace(0, N - 1, 1 << 15).astype(np.int64)).to(dev)
    tuning = P.chem_autotune(gm, 1e-5, T0d[si].contiguous(), pd[si].contiguous(),
                             Y0d[:, si].contiguous())
    P.profile_read()  # drop the tuner's launches
    log(f"[fp64] autotuned launch shape {tuning} (default {tune_default})")
    st = torch.zeros((3, N), dtype=torch.int32, device=dev)
    t_fp64 = timed_loop(lambda: P.chem_step(gm, 1e-5, Td, pd, Yd, stats=st), restore,
                        args.fp64_steps, 1)
    prof_fp64 = P.profile_read()
    P.profile_enable(False)
    fp_T, fp_Y = Td.cpu().numpy(), Yd.cpu().numpy()
    stats = st.cpu().numpy()
    attempts = int(stats[0].sum() + stats[1].sum())
    log(f"[fp64] {args.fp64_steps} steps in {t_fp64:.3f} s; attempts/cell "
        f"{attempts / N:.2f}")

    ann_cps = N * args.steps / t_ann
    fp64_cps = N * args.fp64_steps / t_fp64
    sets_out = time_sets(P, mech, gm, dev, args, model=model) if args.sets else None

    # ---- training-plus-FP8 sizes: inference on args.big_cells cells ----
    large = None
    if args.big_cells:
        large = big_leg(P, mech, gm, dev, args, model)
    peaks = P.measure_peaks() if args.peaks else None
    if peaks:
        log(f"[peaks] {peaks}")

    # ---- accuracy against the CPU oracle on an evenly spaced sample ----
    copy_probe(dev)

    import oracle
    om = oracle.OracleMech(mech)
    idx = np.linspace(0, N - 1, args.oracle_sample).astype(np.int64)
    o = oracle.chem_step(om, 1e-5, T[idx], p[idx], Y[:, idx])
    dY_ref = o["Y"] - Y[:, idx]
    table, ann_major = nrmse_table(ann_Y[:, idx] - Y[:, idx], dY_ref, o["Y"].mean(axis=1),
                                   mech.species)
    _, frozen_major = nrmse_table(np.zeros_like(dY_ref), dY_ref, o["Y"].mean(axis=1),
                                  mech.species)
    # explicit Euler from the instantaneous rates (GPU chem_rates)
    rates = P.chem_rates(gm, T0d, pd, Y0d)
    w = rates["wdot"].cpu().numpy()[:, idx]
    rho = p[idx] / (8.314462618 * T[idx] * (Y[:, idx] / mech.W[:, None]).sum(axis=0))
    _, euler_major = nrmse_table(mech.W[:, None] * w / rho * 1e-5, dY_ref, o["Y"].mean(axis=1),
                                 mech.species)
    if fp8 is not None:
        _, fp8["nrmse"] = nrmse_table(fp8["Y"][:, idx] - Y[:, idx], dY_ref, o["Y"].mean(axis=1),
                                      mech.species)
    # fallback without the element projection: the network's own state
    # Y0 + dY (clipped at 0) tested against the same 1e-6 element residual
    nmo = model.get_norm(K + 2, K)
    idx_d = torch.from_numpy(idx).to(dev)
    U = model.forward(T0d[idx_d].contiguous(), pd[idx_d].contiguous(),
                      Y0d[:, idx_d].contiguous(), K).cpu().numpy().astype(np.float64).T
    Yraw = np.maximum(Y[:, idx] + U * nmo["sd_out"][:, None] + nmo["mu_out"][:, None], 0.0)
    Mel = (mech.awt[None, :] * mech.comp / mech.W[:, None]).T  # [E][K]
    res_raw = np.abs(Mel @ (Yraw - Y[:, idx])).max(axis=0)
    unprojected_flagged = int((res_raw > 1e-6).sum())
    del U, Yraw
    # the same network trained without the physics terms of the loss
    phys_cmp = None
    data_cmp = None
    ens_cmp = None

    def sample_step(mdl):
        Ts, ps, Ys = (T0d[idx_d].contiguous(), pd[idx_d].contiguous(),
                      Y0d[:, idx_d].contiguous())
        nf = torch.zeros(1, dtype=torch.int64, device=dev)
        mdl.step(gm, 1e-5, Ts, ps, Ys, n_fallback=nf)
        Um = mdl.forward(T0d[idx_d].contiguous(), pd[idx_d].contiguous(),
                         Y0d[:, idx_d].contiguous(), K).cpu().numpy().astype(np.float64).T
        nmm = mdl.get_norm(K + 2, K)
        Yr = np.maximum(Y[:, idx] + Um * nmm["sd_out"][:, None] + nmm["mu_out"][:, None], 0.0)
        rr = np.abs(Mel @ (Yr - Y[:, idx])).max(axis=0)
        _, mj = nrmse_table(Ys.cpu().numpy() - Y[:, idx], dY_ref, o["Y"].mean(axis=1),
                            mech.species)
        return {"nrmse_major_max": mj, "fallback_cells": int(nf.item()),
                "raw_residual_max": float(rr.max()),
                "raw_residual_median": float(np.median(rr)),
                "raw_residual_flags": int((rr > 1e-6).sum())}
    if model_plain is not None:
        phys_cmp = {"sample_cells": int(idx.size),
                    "with_terms": dict(w_phys=list(w_phys), **sample_step(model)),
                    "without_terms": sample_step(model_plain),
                    "training_without_terms": train_plain}
    if model_sampled is not None:
        data_cmp = {"sample_cells": int(idx.size),
                    "perturbed_recipe_states": sample_step(model),
                    "sec31_sampler": dict(sample_step(model_sampled), data=sample_info)}
    if ens is not None:
        fl_single = mlp_flops_per_cell(K)
        fl_member = sum(2 * a * b for a, b in zip([K + 2, *HIDDEN], [*HIDDEN, 1]))
        ens_cmp = {
            "members": K,
            "sample_cells": int(idx.size),
            "ensemble": sample_step(model_ens),
            "single_network_same_loss": None if model_plain is None else
            sample_step(model_plain),
            "single_network_with_physics_terms": sample_step(model),
            "step": {"cells_per_s": round(N * ens["steps"] / ens["t"], 1),
                     "ms_per_step": round(1e3 * ens["t"] / ens["steps"], 3),
                     "steps": ens["steps"], "fallback_cells": ens["fallback"],
                     "kernels": {k: dict(launches=v[0], avg_ms=round(v[1] / max(v[0], 1), 4))
                                 for k, v in ens["prof"].items()}},
            "training": train_ens,
            "roofline_training": train_roofline(train_ens, K),
            "mlp_flops_per_cell": {"ensemble": K * fl_member, "single": fl_single,
                                   "ratio": round(K * fl_member / fl_single, 2)}}

    # the same error against the GPU FP64 integrator, on every cell
    dY_fp = fp_Y - Y
    _, ann_vs_fp64_all = nrmse_table(ann_Y - Y, dY_fp, fp_Y.mean(axis=1), mech.species)
    fp8_vs_fp64_all = None
    if fp8 is not None:
        _, fp8_vs_fp64_all = nrmse_table(fp8["Y"] - Y, dY_fp, fp_Y.mean(axis=1), mech.species)
    del dY_fp
    big = np.abs(o["Y"]) > 1e-10
    fp_err = max(float(np.max(np.abs(fp_T[idx] - o["T"]) / o["T"])),
                 float(np.max(np.abs(fp_Y[:, idx] - o["Y"])[big] / np.abs(o["Y"])[big])))
    ann_Terr = float(np.sqrt(np.mean((ann_T[idx] - o["T"]) ** 2)))

    # the closure under the surrogate: the network's rates against the
    # oracle's step, both through the oracle's closure and the same flow times
    from oracle import pasr as opasr
    k_ref, _, RRp_ref = opasr.scale(mech, o["T"], p[idx], o["Y"], o["RR"], tT_np[idx],
                                    tK_np[idx])
    majors = [mech.index(n) for n in ("O2", "H2O", "CH4", "CO", "CO2")]
    src_err = {mech.species[k]: round(float(np.linalg.norm(RRpasr_ann[k, idx] - RRp_ref[k]) /
                                            max(np.linalg.norm(RRp_ref[k]), 1e-300)), 5)
               for k in majors}

    # the in-step audit's per-species normalised RMSE (its reference is the GPU
    # integrator on every 64th cell) next to the oracle's figure on its sample
    aud_nrmse = {}
    for k, nm_ in enumerate(mech.species):
        if table[nm_]["major"] and aud_np[0] > 0:
            rng_ = aud_np[5 + 3 * k] - aud_np[4 + 3 * k]
            aud_nrmse[nm_] = round(float(np.sqrt(aud_np[3 + 3 * k] / aud_np[0]) / rng_), 5)
    audit_out = {"fraction": aud_frac, "cells_compared": int(aud_np[0]),
                 "cells_not_compared": int(aud_np[1]),
                 "ms_per_audited_step": round(1e3 * t_aud / 3, 3),
                 "T_max_abs_err_K": float(aud_np[2]),
                 "nrmse_major": aud_nrmse,
                 "nrmse_major_max": max(aud_nrmse.values()) if aud_nrmse else None,
                 "oracle_sample_nrmse_major_max": ann_major}

    # ---- roofline of the dominant kernels, from HIP events on their streams ----
    def avg(prof, label):
        c, tot = prof.get(label, (0, 0.0))
        return (tot / c * 1e-3) if c else float("nan"), c
    chunk = min(N, 1 << 21)
    l2_flops = 2.0 * HIDDEN[0] * HIDDEN[1] * chunk
    n_in = K + 2
    if "mlp_l12" in prof_ann:
        # first two layers in one kernel: useful flops of both layers (the
        # paired-halves kernel computes the first once per cell; a per-tile
        # recomputation would not be counted); X in and H2 out (BF16), W1,
        # b1, W2, b2 once
        dom = "mlp_l12"
        dom_desc = ("mlp_l12 (32->1600->800 BF16, first layer produced on chip per K-step "
                    "once per cell, bias+GELU)")
        dom_flops = 2.0 * chunk * (n_in * HIDDEN[0] + HIDDEN[0] * HIDDEN[1])
        dom_bytes = (2 * chunk * (n_in + HIDDEN[1]) + 2 * (n_in * HIDDEN[0] + HIDDEN[0] * HIDDEN[1])
                     + 4 * (HIDDEN[0] + HIDDEN[1]))
    else:
        # H1 in and H2 out (BF16), W2 and b2 once
        dom = "mlp_l2"
        dom_desc = "mlp_l2 (1600->800 BF16 GEMM, bias+GELU)"
        dom_flops = l2_flops
        dom_bytes = 2 * chunk * (HIDDEN[0] + HIDDEN[1]) + 2 * HIDDEN[0] * HIDDEN[1] + 4 * HIDDEN[1]
    t_dom, c_dom = avg(prof_ann, dom)
    ach_bf16 = dom_flops / t_dom
    t_step, c_step = avg(prof_fp64, "chem_step")
    fl_attempt = rodas3_flops_per_attempt(mech)
    step_flops = fl_attempt * attempts
    ach_fp64 = step_flops / t_step
    kernels_ann = {k: dict(launches=v[0], avg_ms=round(v[1] / max(v[0], 1), 4))
                   for k, v in prof_ann.items()}
    t_pk, c_pk = avg(prof_pasr, "pasr_scale")
    # T, p, tau_T, tau_K, Y and RR in; RR and kappa out (tau_c not asked for)
    pasr_bytes = 8 * N * (3 * K + 5)
    pasr_gbs = pasr_bytes / t_pk / 1e9
    fp8_out = None
    if fp8 is not None:
        t8, c8 = avg(fp8["prof"], "mlp_l2_fp8")
        ach8 = l2_flops / t8
        fp8_out = {"cells_per_s": round(N * args.steps / fp8["t"], 1),
                   "ms_per_step": round(1e3 * fp8["t"] / args.steps, 4),
                   "nrmse_major_max": fp8["nrmse"], "fallback_cells": fp8["fallback"],
                   "scales_act_wgt": fp8["scales"],
                   "calibration": "2^16 perturbed CH4/air states (seed 56)",
                   "roofline": {"kernel": "mlp_l2_fp8 (1600->800 E4M3 GEMM)", "bound": "mfma",
                                "achieved": round(ach8 / 1e12, 2), "peak": PEAK_FP8 / 1e12,
                                "unit": "TFLOP/s", "frac": round(ach8 / PEAK_FP8, 4),
                                "avg_ms": round(t8 * 1e3, 4), "launches": c8},
                   "kernels": {k: dict(launches=v[0], avg_ms=round(v[1] / max(v[0], 1), 4))
                               for k, v in fp8["prof"].items()},
                   "time_weighted_roof": fp8_roof(fp8["prof"], K, chunk)}

    # ---- CPU baseline: the oracle on a bounded sample of the same cells ----
    nthr = oracle.max_threads()
    # the probe keeps every thread busy (dynamic schedule, 64 cells per chunk)
    probe_n = max(256, 128 * nthr)
    pi = np.linspace(0, N - 1, probe_n).astype(np.int64)
    tp = time.time()
    oracle.chem_step(om, 1e-5, T[pi], p[pi], Y[:, pi])
    tp = time.time() - tp
    ns = int(min(N, max(probe_n, args.cpu_seconds / max(tp, 1e-6) * probe_n)))
    si = np.linspace(0, N - 1, ns).astype(np.int64)
    tc = time.time()
    oracle.chem_step(om, 1e-5, T[si], p[si], Y[:, si])
    tc = time.time() - tc
    cpu_cps = ns / tc
    # the oracle on one core (the paper's per-core convention), ~3 s of work
    s1 = pi[:32]
    t1 = time.time()
    oracle.chem_step(om, 1e-5, T[s1], p[s1], Y[:, s1], nthreads=1)
    t1 = time.time() - t1
    n1 = int(min(N, max(32, 3.0 / max(t1, 1e-6) * 32)))
    s1 = np.linspace(0, N - 1, n1).astype(np.int64)
    t1 = time.time()
    oracle.chem_step(om, 1e-5, T[s1], p[s1], Y[:, s1], nthreads=1)
    t1 = time.time() - t1
    # the network on the host: the oracle's FP64 NumPy MLP (BLAS) on 2^16 cells
    from oracle import ann as oann
    shapes = [(HIDDEN[0], K + 2), (HIDDEN[1], HIDDEN[0]), (HIDDEN[2], HIDDEN[1]), (K, HIDDEN[2])]
    params64 = [tuple(a.astype(np.float64) for a in model.get_layer(l, shapes[l]))
                for l in range(4)]
    nmz = model.get_norm(K + 2, K)
    na = int(min(N, 1 << 16))
    ai = np.linspace(0, N - 1, na).astype(np.int64)
    ta = time.time()
    feat = oann.features(T[ai], p[ai], Y[:, ai])
    Xa = ((feat - nmz["mu_in"][:, None].astype(np.float64)) /
          nmz["sd_in"][:, None].astype(np.float64)).T
    oann.forward(params64, Xa, prec="fp64")
    ta = time.time() - ta
    # one training step of the batch size on the host: the oracle's FP64
    # forward and backward (NumPy/BLAS), no optimiser
    Bt = args.batch
    bi = np.linspace(0, N - 1, Bt).astype(np.int64)
    featb = oann.features(T[bi], p[bi], Y[:, bi])
    Xb = ((featb - nmz["mu_in"][:, None].astype(np.float64)) /
          nmz["sd_in"][:, None].astype(np.float64)).T
    tgtb = np.zeros((Bt, K))
    tb = time.time()
    oann.backward(params64, Xb, tgtb, prec="fp64")
    tb = time.time() - tb
    small = small_config(P, dev, oracle, nthr)

    out = {
        "metric": METRIC,
        "value": round(ann_cps, 1),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_ann / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {
            "workload": "stratified CH4/air, 30 species / 150 reactions, 2^20 cells, dt=1e-5 s; "
                        "BF16 MLP 32-1600-800-400-30 with FP64 RODAS3 fallback",
            "cells": N, "species": K, "reactions": mech.R, "dt": 1e-5,
            "hidden": list(HIDDEN)},
        "fp64": {"cells_per_s": round(fp64_cps, 1), "steps": args.fp64_steps,
                 "launch_shape": {"lanes_per_cell": tuning["lanes_per_cell"],
                                  "waves_per_cu": tuning["waves_per_cu"],
                                  "tuned_on": "2^15 evenly spaced cells",
                                  "default": {k: tune_default[k] for k in
                                              ("lanes_per_cell", "waves_per_cu")}},
                 "ms_per_step": round(1e3 * t_fp64 / args.fp64_steps, 3),
                 "attempts_per_cell": round(attempts / N, 3),
                 "max_rel_err_vs_oracle": fp_err, "dtype": "f64"},
        "speedup_ann_vs_fp64": round(ann_cps / fp64_cps, 2),
        "accuracy": {"sample_cells": int(idx.size),
                     "ann_nrmse_major_max": ann_major,
                     "frozen_nrmse_major_max": frozen_major,
                     "euler_nrmse_major_max": euler_major,
                     "ann_T_rmse_K": ann_Terr,
                     "fallback_cells": n_fallback,
                     "element_residual_flags_without_projection": {
                         "cells": unprojected_flagged, "of": int(idx.size),
                         "max_residual": float(res_raw.max()),
                         "median_residual": float(np.median(res_raw)), "tol": 1e-6},
                     "per_species": {k: round(v["nrmse"], 5) for k, v in table.items()
                                     if v["major"]},
                     "unresolved_abundant": {k: dict(nrmse=round(v["nrmse"], 4),
                                                     dY_range=v["range"])
                                             for k, v in table.items() if v["unresolved"]}},
        "roofline": {"kernel": dom_desc, "bound": "mfma",
                     "achieved": round(ach_bf16 / 1e12, 2), "peak": PEAK_BF16 / 1e12,
                     "unit": "TFLOP/s", "frac": round(ach_bf16 / PEAK_BF16, 4),
                     "traffic": measured_traffic(dom), "avg_ms": round(t_dom * 1e3, 4),
                     "launches": c_dom, "flops_per_launch": dom_flops,
                     "algorithmic_bytes_per_launch": dom_bytes},
        "roofline_fp64": {"kernel": "k_step (RODAS3 persistent)", "bound": "alu",
                          "achieved": round(ach_fp64 / 1e12, 3), "peak": PEAK_FP64 / 1e12,
                          "unit": "TFLOP/s", "frac": round(ach_fp64 / PEAK_FP64, 4),
                          "traffic": measured_traffic("chem_step"),
                          "avg_ms": round(t_step * 1e3, 3),
                          "launches": c_step, "flops_per_attempt": fl_attempt,
                          "attempts_per_launch": attempts,
                          # T, p, Y in; T, Y, stats out (FP64 SoA, int32 stats)
                          "algorithmic_bytes_per_launch": N * (8 + 8 + 8 * K + 8 + 8 * K + 12)},
        "kernels_ann": kernels_ann,
        "audit": audit_out,
        "pasr": {"workload": "the BF16 step's rates and state on the same 2^20 cells; Taylor "
                             "times 10^U(-4,-2) s, Kolmogorov times 10^U(-5,-3) s (seed 76)",
                 "ms_per_closure": round(1e3 * t_pasr / args.steps, 4),
                 "ann_step_with_closure": {
                     "cells_per_s": round(N * args.steps / t_ann_pasr, 1),
                     "ms_per_step": round(1e3 * t_ann_pasr / args.steps, 4)},
                 "kappa_quantiles_0_1_50_99": [float(x) for x in
                                               np.quantile(kap_ann, [0.0, 0.01, 0.5, 0.99])],
                 "cells_kappa_below_0p99": int((kap_ann < 0.99).sum()),
                 "vs_oracle": {"sample_cells": int(idx.size),
                               "kappa_max_abs_err": float(np.max(np.abs(kap_ann[idx] - k_ref))),
                               "scaled_source_rel_l2_err_major": src_err},
                 "roofline": {"kernel": "k_pasr (64 cells per block, one species row of "
                                        "64 cells per wave load, FP64 SoA)",
                              "bound": "hbm", "achieved": round(pasr_gbs, 1),
                              "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                              "frac": round(pasr_gbs * 1e9 / PEAK_HBM, 4),
                              "traffic": measured_traffic("pasr_scale"),
                              "avg_ms": round(t_pk * 1e3, 4), "launches": c_pk,
                              "algorithmic_bytes_per_launch": pasr_bytes}},
        "ann_step_graph": {"ms_per_step": round(1e3 * t_graph / args.steps, 4),
                           "equal_to_eager": graph_equal},
        "fp64_sets": sets_out,
        "physics_terms_comparison": phys_cmp,
        "training_data_comparison": data_cmp,
        "ensemble_comparison": ens_cmp,
        "large": large,
        "attainable_peaks": None if peaks is None else {
            "measured_tflops": {k: round(v, 1) for k, v in peaks.items()},
            "spec_tflops": {"bf16_mfma": PEAK_BF16 / 1e12, "fp8_mfma": PEAK_FP8 / 1e12,
                            "fp64_vector": PEAK_FP64 / 1e12},
            "roofline_frac_of_measured": round(ach_bf16 / (peaks["bf16_mfma"] * 1e12), 4),
            "roofline_fp64_frac_of_measured": round(ach_fp64 / (peaks["fp64_vector"] * 1e12), 4),
            "method": "2048 blocks x 256 threads, 8 independent accumulator chains per wave: "
                      "v_mfma_f32_16x16x32_bf16, v_mfma_scale_f32_16x16x128_f8f6f4, v_fma_f64"},
        "roofline_training": train_roofline(train_info, K),
        "fp8": fp8_out,
        "cpu_baseline": {"value": round(cpu_cps, 2), "unit": "cells/s", "cores": nthr,
                         "kind": "oracle",
                         "sample": f"{ns} evenly spaced cells of the 2^20-cell workload, "
                                   f"FP64 RODAS3 oracle (plain C, OpenMP)"},
        "training": train_info,
        "cpu_baselines_more": {
            "oracle_one_core": {"value": round(n1 / t1, 2), "unit": "cells/s", "cores": 1,
                                "sample": f"{n1} evenly spaced cells of the 2^20-cell workload"},
            "training_step_numpy_fp64": {"value": round(tb * 1e3, 1), "unit": "ms per step",
                                         "batch": Bt, "threads": os.environ.get(
                                             "OMP_NUM_THREADS", "library default"),
                                         "sample": "the oracle's FP64 forward and backward "
                                                   "(NumPy/BLAS) on one batch, no optimiser"},
            "ann_numpy_fp64": {"value": round(na / ta, 1), "unit": "cells/s",
                               "threads": os.environ.get("OMP_NUM_THREADS", "library default"),
                               "sample": f"{na} evenly spaced cells: features and the FP64 "
                                         f"MLP forward (NumPy/BLAS), no post-processing"}},
        "accuracy_vs_gpu_fp64_all_cells": {"cells": N, "ann_nrmse_major_max": ann_vs_fp64_all,
                                           "fp8_nrmse_major_max": fp8_vs_fp64_all},
        "small_config": small,
        # the paper's own speed figures, for context only (another machine,
        # mechanism and workload; not a target of this measurement)
        "paper_context": {
            "reported": "chemistry time per LES step cut by 91.3 % (about 11.5x) with the "
                        "ANN on one GPU against direct integration (CVODE) on 32 CPU cores, "
                        "a 1-GPU-to-1-core ratio of 369; neither GPU nor CPU model is named; "
                        "DRM19 (20 species), 2.5 M-cell LES, network trained at dt = 1 us "
                        "(Sec. 4.2, Sec. 5)",
            "this_run_ann_vs_cpu_oracle": round(ann_cps / cpu_cps, 1),
            "this_run_ann_vs_cpu_oracle_per_core": round(ann_cps / cpu_cps * nthr, 1),
            "cpu_oracle_cores": nthr,
        },
    }
    print(json.dumps(_plain(out)), flush=True)


if __name__ == "__main__":
    main()
