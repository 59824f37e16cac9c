"""Benchmark of the KPM density-of-states step on one MI355X.

One step = the whole hot path over one synthetic structure whose coordinates
and random-phase vectors are already in HBM: neighbour list + Hamiltonian
assembly + spectral bounds (tb_build_hamiltonian), the Chebyshev recurrence
with fused moments (kpm_moments) and the Jackson DOS (kpm_dos).

Prints one JSON line.  `value` is N * M * R / (seconds per step) in
atom*moments/s.  `roofline` rates the recurrence kernel: algorithmic bytes per
launch (Hamiltonian values, columns and slice offsets once; per vector row one
gather of T_n, one read of T_{n-1} and of r, one write of T_{n+1}; onsite when
used) over its average launch time measured with HIP events on the library's
stream, against the 8 TB/s HBM3E peak.  `cpu_baseline` times the serial FP64
oracle (one core) on a bounded sample of the same workload.  `variants` reports,
each under its own label, the same moments computed with the doubling
identities and, when all stored hoppings are equal, without reading them.
"""
import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "KPM atom·moments/s & % HBM peak; DOS err vs FP64 oracle; learned vs plain H"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="graphene_pristine_100M")
    p.add_argument("--slice", type=int, default=256)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-tune", action="store_true", help="use the default launch shape")
    p.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    p.add_argument("--no-doubling", action="store_true", help="skip the doubling-identity variant")
    p.add_argument("--train-shuffle-seed", type=int, default=None,
                   help="snapshot workload: shuffle seed of the network's training (0 = stored order; "
                        "default: the workload's)")
    p.add_argument("--launch", default=None,
                   help="snapshot workload: use this named launch shape instead of timing them all "
                        "(e.g. per_step_xcd2_tpb1; for counter runs)")
    p.add_argument("--no-train", action="store_true",
                   help="snapshot workload: skip the network's training (seeded initial parameters) and the "
                        "learned-vs-plain comparison (for counter runs of the recurrence)")
    p.add_argument("--block-shape", default=None,
                   help="block (Slater-Koster) workloads: use this slice and launch shape instead of searching, "
                        "e.g. slice=32,vpt=2,tpb=1,nt=0,xr=2,atom=1 (for counter runs)")
    p.add_argument("--no-variants", action="store_true",
                   help="skip every variant form (doubling, uniform values) and the oracle comparison run")
    p.add_argument("--retune", action="store_true",
                   help="tune afresh instead of starting from the shipped MI355X tuning table")
    p.add_argument("--copy-probe-mib", type=int, default=0,
                   help="run one plain device copy of this many MiB first (counter calibration)")
    p.add_argument("--cpu-sample-cells", type=int, default=0,
                   help="oracle sample: an n x n cell sheet of the same kind, same M and R "
                        "(default: sized for about 4e9 atom*moments, 10-30 s on one core)")
    return p.parse_args()


def cheb_step_bytes(H, Rp, elem, diag, read_r=True, read_values=True, compact=False):
    """Algorithmic bytes of one recurrence launch (see module docstring); the
    doubling form reads no r, the uniform-values form no stored hoppings, the
    compact-column form 2-byte column offsets (the few entries whose offset
    escapes 16 bits also read their 4-byte column; not counted)."""
    st = H.st
    val_b = 4 if st.fmt in (2, 4, 6) else 8
    # n_orb x n_orb blocks, or the bond's displacement (3 values) in the matrix-free form
    per_value = st.n_orb * st.n_orb if st.fmt in (3, 4) else (3 if st.fmt in (5, 6) else 1)
    b = st.n_entries * ((per_value * val_b if read_values else 0) + (2 if compact else 4)) + st.n_ptr * 8
    # gather T_n once, read T_{n-1}, write T_{n+1} (+ read r in the direct form)
    b += st.n_rows * Rp * 2 * elem * (4 if read_r else 3)
    if diag and st.has_onsite:
        b += st.n_rows * val_b
    return b


KERNEL_SOURCES = ("kpm.hip", "kpm_run.hpp", "kpm.hpp", "kpm_dev.hpp")
SEG_KERNEL_SOURCES = ("kpm_batched.hip", "kpm.hpp", "kpm_dev.hpp")


def kernel_source_hash(files=KERNEL_SOURCES):
    """Hash of a recurrence kernel's sources (a stored counter profile is valid only for these)."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2509_06525_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(workload, kernel, slice_, launch, prefix="k_cheb_step", files=KERNEL_SOURCES):
    """HBM bytes per launch of `kernel` from the counter profile stored for `workload`
    (FETCH_SIZE and WRITE_SIZE runs scaled by a plain-copy calibration), or None when
    the kernel's sources or the launch shape differ from the profiled ones."""
    path = os.path.join(ROOT, "profiles", f"{prefix}_{workload}.md")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("record "):
                parts = dict(kv.split("=", 1) for kv in line.split()[1:])
                rec[parts["kernel"]] = parts
    r = rec.get(kernel)
    if r is None or r["sources"] != kernel_source_hash(files) or int(r["slice"]) != int(slice_):
        return None
    if r["launch"] != ",".join(f"{k}:{v}" for k, v in sorted(launch.items())):
        return None
    return float(r["traffic_bytes"])


def stream_probe(dev, mib=2048, reps=5):
    """Measured HBM ceilings beside the 8 TB/s peak, with the library's probe kernels
    (tbk_bandwidth_probe): a streaming copy (read + write of `mib` MiB) and a streaming
    read of `mib` MiB, each timed with HIP events on the launch stream, median of `reps`;
    GB/s of bytes moved."""
    import torch
    from paper_2509_06525_amd import tbkpm
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    folds = torch.empty(max(tbkpm.bandwidth_probe_words(), 1), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    out = {}
    for name, mode, out_t, nbytes in (("stream_copy_gbs", "copy", dst, 2 * n * 4),
                                      ("stream_read_gbs", "read", folds, n * 4)):
        tbkpm.bandwidth_probe(src, out_t, mode, stream)
        t = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            tbkpm.bandwidth_probe(src, out_t, mode, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            t.append(e0.elapsed_time(e1) * 1e-3)
        out[name] = nbytes / float(np.median(t)) / 1e9
    out["stream_probe_mib"] = mib
    del src, dst, folds
    torch.cuda.empty_cache()
    return out


def golden_moments(workload):
    """(a, b, mu [v][n]) of the oracle's stored full-size moments of `workload`
    (tests/golden, written by a script that calls only the oracle), or None."""
    path = os.path.join(ROOT, "tests", "golden", f"oracle_moments_{workload}.txt")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        lines = fh.readlines()
    hdr = {}
    for ln in lines[:4]:
        parts = ln[1:].split()
        for k in range(0, len(parts) - 1, 2):
            hdr[parts[k]] = parts[k + 1]
    return float(hdr["a"]), float(hdr["b"]), np.loadtxt(lines[4:], ndmin=2).T


def golden_snapshot_targets():
    """(table [index, atoms, sigma, a, b, err_plain], target moments [S][M]) of the
    oracle's learned-hopping targets (tests/golden), or None."""
    d = os.path.join(ROOT, "tests", "golden")
    tp, mp = os.path.join(d, "oracle_target_snapshots_256.txt"), os.path.join(d, "oracle_target_moments_snapshots_256.npy")
    if not (os.path.exists(tp) and os.path.exists(mp)):
        return None
    return np.loadtxt(tp, comments="#", ndmin=2), np.load(mp, allow_pickle=False)


def use_shipped_tuning():
    """Point the autotuner's cache at a copy of the shipped MI355X tuning table."""
    if os.environ.get("TBKPM_AUTOTUNE_CACHE"):
        return
    import shutil
    import tempfile
    src = os.path.join(ROOT, "paper_2509_06525_amd", "tuned_gfx950.txt")
    fd, dst = tempfile.mkstemp(prefix="tbkpm_tune_", suffix=".txt")
    os.close(fd)
    shutil.copyfile(src, dst)
    os.environ["TBKPM_AUTOTUNE_CACHE"] = dst


def cpu_baseline(w, cells):
    """Time the oracle (one core, FP64) on a cells x cells sheet with the workload's M and R."""
    from oracle import oracle as O
    from paper_2509_06525_amd import synth
    sample = dict(w)
    if w["kind"] == "stripes":
        s = synth.hbn_stripes(cells, cells, 50, w["sigma"], w["seed"])
    else:
        s = synth.graphene_sheet(cells, cells, w.get("sigma", 0.0), w["seed"])
    R = w["R"]
    r = synth.random_phase(s.n, R, w["seed"] + synth.VECTOR_SEED_OFFSET)
    t0 = time.perf_counter()
    csr, _ = O.hamiltonian(s.pos, s.species, s.box, s.periodic, s.onsite, s.t_pair)
    lo, hi = O.gershgorin(csr)
    a, b = 1.01 * (hi - lo) / 2, (hi + lo) / 2
    mu, _ = O.kpm_moments(csr, a, b, r, w["M"])
    E = synth.energy_grid(a, b)
    O.kpm_dos(mu.mean(0), a, b, E)
    dt = time.perf_counter() - t0
    sample = f"{cells}x{cells}-cell sheet, N={s.n}, M={w['M']}, R={R}: full path (pairs, CSR, moments, DOS)"
    return {"value": s.n * w["M"] * R / dt, "unit": "atom*moments/s", "cores": 1, "kind": "oracle",
            "sample": sample, "seconds": dt}


def bench_snapshots(args, w):
    """Learned hoppings on uneven thermal snapshots: GPU training (untimed), then
    per step: fused learned assembly of all snapshots, their moments in one
    batched recurrence, and the DOS of each snapshot."""
    import torch
    from paper_2509_06525_amd import synth, tbkpm
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    M, R = w["M"], w["R"]
    per = (1, 1, 0)
    log("generating snapshots")
    snaps = synth.snapshot_set(w["count"], w["seed"])
    tcfg = synth.LEARNED_TRAINING
    train = synth.snapshot_set(tcfg["count"], tcfg["seed"], n_min=tcfg["n_min"], n_max=tcfg["n_max"])
    pos, sp, seg, boxes = synth.stack(snaps)
    tpos, tsp, tseg, tboxes = synth.stack(train)
    N = int(seg[-1])
    # training data and GPU training (not timed)
    t0 = time.perf_counter()
    tp = torch.from_numpy(tpos).to(dev)
    tv = tbkpm.descriptor(tp, tseg, tboxes, per, synth.R_DESC, synth.N_RADIAL)
    tb = tbkpm.bonds(tp, tseg, tboxes, per, synth.R_HOP)
    mean, std = tbkpm.feature_moments(tb, tv, synth.R_DESC)
    std = [max(x, 1e-6) for x in std]
    X = tbkpm.bond_features(tb, tv, mean, std, synth.R_DESC)
    y = tbkpm.coordination_target(tb, tv, synth.COORD_KAPPA, synth.COORD_Z0)
    trainer = tbkpm.MlpTrainer(torch.from_numpy(synth.init_mlp_params(tcfg["init_seed"])).to(dev))
    hist = []
    for epochs, lr in (() if args.no_train else tcfg["schedule"]):
        hist += trainer.train(X, y, epochs=epochs, batch=tcfg["batch"], lr=lr, wd=tcfg["wd"],
                              shuffle_seed=tcfg["shuffle_seed"] if args.train_shuffle_seed is None
                              else args.train_shuffle_seed)
    hist = hist or [float("nan")]
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"trained on {X.shape[0]} bonds: loss {hist[0]:.3e} -> {hist[-1]:.3e} in {t_train:.1f} s")
    params = trainer.params
    gpos = torch.from_numpy(pos).to(dev)
    gsp = torch.from_numpy(sp).to(dev)
    r = torch.from_numpy(synth.random_phase(N, R, w["seed"] + synth.VECTOR_SEED_OFFSET, np.complex64)).to(dev)

    held = []

    def build():
        # each step overwrites the previous step's buffers (same structures: no size pass)
        H = tbkpm.build_hamiltonian_learned(gpos, gsp, seg, boxes, per, [0.0], [[synth.T_CC_EV]], params,
                                            mean, std, r_cut=synth.R_HOP, r0=synth.R0, beta=synth.BETA,
                                            r_desc=synth.R_DESC, fmt="sell_f32", slice=64, stream=stream,
                                            into=held.pop() if held else None)
        held.append(H)
        return H

    H = build()
    a, b = H.scales()
    # launch shape: one launch per step (block order plain or XCD-aware) vs one persistent
    # launch (all exact), fastest kept
    shapes = {"per_step": tbkpm.make_config(2, 2, 1, 0, 1, 0), "persistent": tbkpm.make_config(2, 1, 1, 0, 1, 1)}
    for tpb in (1, 2, 4):
        for xr in (1, 2):
            shapes[f"per_step_xcd{xr}_tpb{tpb}"] = tbkpm.make_config(2, tpb, 1, xr, 1, 0)
    timing = {}
    if args.launch is not None:
        shapes = {args.launch: shapes[args.launch]}
    for name, cfg in shapes.items():
        try:
            tbkpm.kpm_moments_batched(H, a, b, r, 32, "c32", config=cfg, stream=stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            tbkpm.kpm_moments_batched(H, a, b, r, 64, "c32", config=cfg, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            timing[name] = e0.elapsed_time(e1) / 63
        except tbkpm.TBKError as e:
            log(f"launch shape {name} unavailable: {e}")
    best = min(timing, key=timing.get)
    cfg = shapes[best]
    log(f"launch shapes (ms/step): {timing}; using {best}")
    work = torch.empty(tbkpm.workspace_size_batched(H, R, M, "c32", cfg, stream), dtype=torch.uint8, device=dev)
    mu = torch.empty((len(snaps), R, M), dtype=torch.float64, device=dev)
    u = torch.linspace(-0.99, 0.99, 2001, dtype=torch.float64, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    kpm_ms = []

    def step():
        Hs = build()
        aa, bb = Hs.scales()
        ev[0].record(stream)
        tbkpm.kpm_moments_batched(Hs, aa, bb, r, M, "c32", work=work, mu=mu, config=cfg, stream=stream)
        ev[1].record(stream)
        mbar = tbkpm.mean_moments(mu, stream=stream)
        # each snapshot's own grid [b - 0.99 a, b + 0.99 a]
        grid = (torch.tensor(bb, dtype=torch.float64, device=dev)[:, None]
                + torch.tensor(aa, dtype=torch.float64, device=dev)[:, None] * u[None, :]).contiguous()
        rhos = tbkpm.kpm_dos_batched(mbar, aa, bb, grid, stream=stream)
        return Hs, rhos

    log(f"{len(snaps)} snapshots, N={N} M={M} R={R}: warmup {args.warmup}, timed {args.steps}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    tbkpm.step_timer(True)        # events around the step launches only (per-step launch shapes)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        Hs, rhos = step()
        torch.cuda.synchronize()
        kpm_ms.append(ev[0].elapsed_time(ev[1]))
    sec = (time.perf_counter() - t0) / args.steps
    step_ms, step_launches = tbkpm.step_timer_read()
    tbkpm.step_timer(False)
    kmed = float(np.median(kpm_ms))
    st = Hs.st
    Rp = 1
    while Rp < R:
        Rp *= 2
    launch_bytes = st.n_entries * 8 + st.n_ptr * 8 + N * Rp * 8 * 4
    launch_s = step_ms * 1e-3 / step_launches if step_launches else kmed * 1e-3 / (M - 1)
    achieved = launch_bytes / launch_s / 1e9
    comparison = None if args.no_train else learned_vs_plain(dev, gpos, gsp, seg, boxes, per, params, mean, std,
                                                             r, M, stream)
    out = {
        "metric": METRIC, "value": N * M * R / sec, "unit": "atom*moments/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "snapshots": len(snaps), "n_atoms_total": N, "moments": M,
                   "vectors": R, "format": "sell_f32", "slice": 64, "precision": "c32", "hoppings": "learned",
                   "launch": cfg.as_dict(), "launch_ms_per_step": timing},
        "training": {"snapshots": tcfg["count"], "seed": tcfg["seed"], "bonds": int(X.shape[0]),
                     "epochs": len(hist), "loss_first": hist[0], "loss_last": hist[-1], "seconds": t_train},
        "learned_vs_plain": comparison,
        "kpm_ms_median": kmed,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if cfg.persistent else profiled_traffic(
                         args.workload, "seg", 64, cfg.as_dict(), "k_cheb_step_seg", SEG_KERNEL_SOURCES),
                     "traffic_source": f"profiles/k_cheb_step_seg_{args.workload}.md (stored rocprofv3 "
                                       "FETCH_SIZE, WRITE_SIZE runs, copy-calibrated; null when the kernel or "
                                       "launch shape differs)",
                     "kernel": "k_cheb_persistent" if cfg.persistent else "k_cheb_step_seg",
                     "bytes_per_launch": launch_bytes, "launch_us": launch_s * 1e6,
                     "launches_timed": step_launches, "launch_us_kpm_window": kmed * 1e3 / (M - 1)},
    }
    out["roofline"].update(stream_probe(dev))
    print(json.dumps(out), flush=True)


def learned_vs_plain(dev, gpos, gsp, seg, boxes, per, params, mean, std, r, M, stream):
    """DOS error of the learned and of the plain-formula Hamiltonian of every snapshot
    against the oracle's target DOS (tests/golden: the coordination-corrected target
    hoppings, the oracle's scale and the same vectors), relative L2 on each
    snapshot's 2001-point grid; both DOS reconstructed by the library."""
    import torch
    from paper_2509_06525_amd import synth, tbkpm
    gold = golden_snapshot_targets()
    if gold is None:
        return None
    table, mu_t = gold
    if table.shape[0] != len(seg) - 1 or not np.array_equal(table[:, 1].astype(np.int64), np.diff(seg)):
        return None
    a, b = list(table[:, 3]), list(table[:, 4])
    u = torch.linspace(-0.99, 0.99, 2001, dtype=torch.float64, device=dev)
    grid = (torch.tensor(b, dtype=torch.float64, device=dev)[:, None]
            + torch.tensor(a, dtype=torch.float64, device=dev)[:, None] * u[None, :]).contiguous()
    rho_t = tbkpm.kpm_dos_batched(torch.from_numpy(mu_t).to(dev), a, b, grid, stream=stream).cpu().numpy()
    errs = {}
    for name, H in (("learned", tbkpm.build_hamiltonian_learned(
                        gpos, gsp, seg, boxes, per, [0.0], [[synth.T_CC_EV]], params, mean, std, fmt="sell_f32",
                        slice=64, stream=stream)),
                    ("plain", tbkpm.build_hamiltonian_batched(gpos, gsp, seg, boxes, per, [0.0], [[synth.T_CC_EV]],
                                                              fmt="sell_f32", slice=64, stream=stream))):
        mu = tbkpm.mean_moments(tbkpm.kpm_moments_batched(H, a, b, r, M, "c32", stream=stream), stream=stream)
        rho = tbkpm.kpm_dos_batched(mu, a, b, grid, stream=stream).cpu().numpy()
        errs[name] = np.linalg.norm(rho - rho_t, axis=1) / np.linalg.norm(rho_t, axis=1)
        del H
    el, ep = errs["learned"], errs["plain"]
    return {"snapshots": int(len(el)), "err_learned_max": float(el.max()), "err_learned_median": float(np.median(el)),
            "err_plain_min": float(ep.min()), "err_plain_median": float(np.median(ep)),
            "err_plain_max": float(ep.max()), "learned_over_1e-2": int((el > 1e-2).sum()),
            "learned_not_below_plain": int((el >= ep).sum()),
            "source": "tests/golden/oracle_target_moments_snapshots_256.npy"}


def kpm_variant(args, label, fields, H, a, b, r, M, R, Rp, elem, diag, precision, config, mu_direct, rho_direct,
                E, stream, dev, tune=None):
    """The same moments in another form of the recurrence (doubling identities:
    two moments per step, M/2 launches, no read of r; uniform values: the stored
    hoppings are not read), timed like the direct form and compared with it.
    `tune` (slice, config) is the form's own tuned shape; H is rebuilt when its
    slice height differs."""
    import torch
    from paper_2509_06525_amd import tbkpm
    if tune is not None:
        slice_v, cfg = tune
        if slice_v != H.st.slice:
            H = args.rebuild(slice_v)
    else:
        base = config if config is not None else tbkpm.default_config(H, R, precision)
        cfg = tbkpm.with_fields(base, **fields)
    work = tbkpm.alloc_workspace(H, R, M, precision, dev, cfg)
    mu = torch.empty((R, M), dtype=torch.float64, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tbkpm.kpm_moments(H, a, b, r, M, precision, work=work, mu=mu, stream=stream, config=cfg)
    ms = []
    for _ in range(max(1, args.steps)):
        e0.record(stream)
        tbkpm.kpm_moments(H, a, b, r, M, precision, work=work, mu=mu, stream=stream, config=cfg)
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    med = float(np.median(ms))
    rho = tbkpm.kpm_dos(tbkpm.mean_moments(mu, stream=stream), a, b, E, stream=stream).cpu().numpy()
    dbl = bool(cfg.doubling)
    launches = M // 2 if dbl else M - 1
    launch_bytes = cheb_step_bytes(H, Rp, elem, diag, read_r=not dbl, read_values=not cfg.uniform_values,
                                   compact=bool(cfg.compact_columns))
    launch_s = med * 1e-3 / launches
    achieved = launch_bytes / launch_s / 1e9
    N = H.st.n_rows
    log(f"{label}: kpm {med:.1f} ms ({launches} launches)")
    return {"kpm_ms_median": med, "kpm_atom_moments_per_s": N * M * R / (med * 1e-3), "launches": launches,
            "slice": H.st.slice, "launch": cfg.as_dict(),
            "dos_relL2_vs_direct": float(np.linalg.norm(rho - rho_direct) / np.linalg.norm(rho_direct)),
            "max_abs_dmu_over_N_vs_direct": float(np.abs(mu.cpu().numpy() - mu_direct).max() / N),
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS,
                         "traffic": profiled_traffic(args.workload, label, H.st.slice, cfg.as_dict()),
                         "kernel": f"k_cheb_step ({label})",
                         "bytes_per_launch": launch_bytes, "launch_us": launch_s * 1e6}}


def block_shape_search(H, a, b, r, geom, stream):
    """Launch shape of the block recurrence on H for the vectors r, timed over 32 moments
    (the tuner builds one-orbital Hamiltonians, so the block forms are searched here: a
    thread per orbital row, a thread per atom).  Returns (shape, ms per moment, best ms
    per form)."""
    import torch
    from paper_2509_06525_amd import tbkpm
    forms = (0, 1) if H.fmt in (tbkpm.FORMATS["bsell4_f32"], tbkpm.FORMATS["bsell4_f64"]) else (0,)
    vpts = (1, 2) if r.shape[1] >= 2 else (1,)
    tpbs = (1, 2) if geom else (1, 2, 4)
    if geom:
        forms = (1,)
    shapes = [tbkpm.make_config(v, t, nt, xr, 1, atom_rows=at) for at in forms for v in vpts
              for t in tpbs for nt in (0, 1) for xr in (0, 1, 2)]
    times = []
    for c in shapes:
        tbkpm.kpm_moments(H, a, b, r, 9, "c32", config=c, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        tbkpm.kpm_moments(H, a, b, r, 33, "c32", config=c, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    best = {}
    for c, t in zip(shapes, times):
        best[c.atom_rows] = min(best.get(c.atom_rows, float("inf")), t / 32)
    return shapes[int(np.argmin(times))], min(times) / 32, best


def bench_sk(args, w):
    """DOS step on the Slater-Koster orbital Hamiltonian (s, p: 4 rows per atom; s, p, d:
    9): build + moments + DOS per step, the recurrence rated like the one-orbital
    workloads, the doubling form as a variant, the oracle on a bounded sample as the CPU
    baseline."""
    import torch
    from paper_2509_06525_amd import synth, tbkpm
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    M, R = w["M"], w["R"]
    norb = w.get("orbitals", 4)
    dint = synth.SK_D if norb == 9 else None
    log(f"generating {args.workload}")
    s = synth.make_structure(args.workload)
    N = s.n
    pos = torch.from_numpy(s.pos).to(dev)
    sp = torch.from_numpy(s.species).to(dev)
    r = torch.from_numpy(synth.random_phase(norb * N, R, w["seed"] + synth.VECTOR_SEED_OFFSET,
                                            np.complex64)).to(dev)

    r_cut = w.get("r_cut", synth.R_HOP)
    geom = w["fmt"].startswith("bgeom")

    def build(fmt=w["fmt"], slice_=64):
        return tbkpm.build_hamiltonian_sk(pos, sp, s.box, s.periodic, *synth.SK_V, synth.SK_ES, synth.SK_EP,
                                          r_cut=r_cut, r0=synth.R0, beta=synth.BETA, fmt=fmt, slice=slice_,
                                          stream=stream, d=dint, e_d=synth.SK_ED)

    def pick_shape(H, a, b):
        return block_shape_search(H, a, b, r, geom, stream)

    # atom-slice height and launch shape, searched together (a slice of 64 for the displacement
    # form, whose shape search alone takes seconds at 100 M atoms)
    best_slice, cfg, ms, form_ms = 64, None, float("inf"), {}
    fixed = None
    if args.block_shape:
        fixed = {k: int(v) for k, v in (kv.split("=") for kv in args.block_shape.split(","))}
        best_slice = fixed["slice"]
        cfg = tbkpm.make_config(fixed["vpt"], fixed["tpb"], fixed["nt"], fixed["xr"], 1, atom_rows=fixed["atom"])
    for sl in (() if fixed else (64,) if geom else (16, 32, 64, 128)):
        H = build(slice_=sl)
        a, b = H.scale()
        c_, m_, f_ = pick_shape(H, a, b)
        for k, v in f_.items():
            form_ms[k] = min(form_ms.get(k, float("inf")), v)
        if m_ < ms:
            best_slice, cfg, ms = sl, c_, m_
        del H
    H = build(slice_=best_slice)
    a, b = H.scale()
    log(f"{w['fmt']}: slice {best_slice}, launch shape {cfg.as_dict()} ({ms:.3f} ms/step)")
    work = tbkpm.alloc_workspace(H, R, M, "c32", dev, cfg)
    mu = torch.empty((R, M), dtype=torch.float64, device=dev)
    E = torch.linspace(b - 0.99 * a, b + 0.99 * a, 2001, dtype=torch.float64, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    kpm_ms = []
    del H

    def step():
        Hs = build(slice_=best_slice)
        aa, bb = Hs.scale()
        ev[0].record(stream)
        tbkpm.kpm_moments(Hs, aa, bb, r, M, "c32", work=work, mu=mu, stream=stream, config=cfg)
        ev[1].record(stream)
        rho = tbkpm.kpm_dos(tbkpm.mean_moments(mu, stream=stream), aa, bb, E, stream=stream)
        return Hs, aa, bb, rho

    log(f"N={N} atoms, {norb * N} orbitals, M={M} R={R}: warmup {args.warmup}, timed {args.steps}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        Hs, aa, bb, rho = step()
        torch.cuda.synchronize()
        kpm_ms.append(ev[0].elapsed_time(ev[1]))
    sec = (time.perf_counter() - t0) / args.steps
    Rp = 1
    while Rp < R:
        Rp *= 2
    diag = Hs.st.has_onsite or bb != 0.0
    launch_bytes = cheb_step_bytes(Hs, Rp, 4, diag)
    kmed = float(np.median(kpm_ms))
    launch_s = kmed * 1e-3 / (M - 1)
    achieved = launch_bytes / launch_s / 1e9
    mu_c, rho_c = mu.cpu().numpy().copy(), rho.cpu().numpy()
    nr = norb * N
    out = {
        "metric": "KPM orbital*moments/s", "value": nr * M * R / sec, "unit": "orbital*moments/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "n_atoms": N, "n_orbitals": nr, "moments": M, "vectors": R,
                   "orbitals_per_atom": norb, "format": w["fmt"], "slice": best_slice, "precision": "c32",
                   "a_eV": aa, "b_eV": bb,
                   "launch": cfg.as_dict()},
        "kpm_ms_median": kmed,
        "shape_search_ms_per_launch": {("atom_form" if k else "orbital_row_form"): v for k, v in form_ms.items()},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_cheb_step_geom" if geom else (
                         "k_cheb_step_atom" if cfg.atom_rows else "k_cheb_step_blk"),
                     "bytes_per_launch": launch_bytes, "launch_us": launch_s * 1e6},
    }
    if geom:
        # stored blocks of the same matrix: norb^2 floats per bond instead of a 16-byte
        # record (the displacement form also keeps the column array: 20 B per slot)
        blk_bytes = Hs.st.n_entries * (norb * norb * 4 + 4)
        out["variants"] = {"stored_blocks": {
            "bytes": blk_bytes, "displacement_form_bytes": Hs.st.n_entries * 20,
            "note": "not run: the stored-block form of this matrix does not fit next to the vectors"
            if blk_bytes > 200e9 else "not run"}}
        if not args.no_doubling:
            out["variants"]["doubling"] = kpm_variant(args, "doubling", {"doubling": 1}, Hs, aa, bb, r, M, R, Rp,
                                                      4, diag, "c32", cfg, mu_c, rho_c, E, stream, dev)
        del Hs
    else:
        sk_block_variants(args, w, out, build, pick_shape, Hs, aa, bb, r, M, R, Rp, diag, cfg, mu, mu_c, rho_c, E,
                          ev, work, nr, norb, dint, pos, sp, s, stream, dev)
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        cells = args.cpu_sample_cells or max(8, int(math.sqrt(1.5e9 / (norb * norb * M * R))))
        ss = synth.graphene_sheet(cells, cells, w["sigma"], w["seed"])
        rs = synth.random_phase(norb * ss.n, R, w["seed"] + synth.VECTOR_SEED_OFFSET)
        t0 = time.perf_counter()
        vs = synth.SK_V + (synth.SK_D if norb == 9 else ())
        csr, _ = O.sk_hamiltonian(ss.pos, ss.box, ss.periodic, vs, synth.SK_ES, synth.SK_EP, e_d=synth.SK_ED,
                                  r_cut=r_cut, r0=synth.R0, beta=synth.BETA)
        lo, hi = O.gershgorin(csr)
        sa, sb = 1.01 * (hi - lo) / 2, (hi + lo) / 2
        mo, _ = O.kpm_moments(csr, sa, sb, rs, M)
        O.kpm_dos(mo.mean(0), sa, sb, synth.energy_grid(sa, sb))
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": norb * ss.n * M * R / dt, "unit": "orbital*moments/s", "cores": 1,
                               "kind": "oracle", "seconds": dt,
                               "sample": f"{cells}x{cells}-cell sheet, {norb * ss.n} orbitals, M={M}, R={R}: "
                                         "full path"}
    print(json.dumps(out), flush=True)


def sk_block_variants(args, w, out, build, pick_shape, Hs, aa, bb, r, M, R, Rp, diag, cfg, mu, mu_c, rho_c, E, ev,
                      work, nr, norb, dint, pos, sp, s, stream, dev):
    """Stored-block workloads: the scalar SELL expansion, the doubling form and the learned
    assembly, each timed beside the block form."""
    import torch
    from paper_2509_06525_amd import synth, tbkpm
    # the same Hamiltonian as a scalar SELL matrix (3 norb columns and values per orbital row)
    Hsc = build("sell_f32", 64)
    cfg_s, _, _ = pick_shape(Hsc, aa, bb)
    ws = tbkpm.alloc_workspace(Hsc, R, M, "c32", dev, cfg_s)
    ms_s = []
    for _ in range(max(1, args.steps)):
        ev[0].record(stream)
        tbkpm.kpm_moments(Hsc, aa, bb, r, M, "c32", work=ws, mu=mu, stream=stream, config=cfg_s)
        ev[1].record(stream)
        torch.cuda.synchronize()
        ms_s.append(ev[0].elapsed_time(ev[1]))
    med_s = float(np.median(ms_s))
    sb = cheb_step_bytes(Hsc, Rp, 4, diag)
    out["variants"] = {"scalar_sell": {
        "kpm_ms_median": med_s, "launch": cfg_s.as_dict(),
        "max_abs_dmu_over_rows_vs_block": float(np.abs(mu.cpu().numpy() - mu_c).max() / nr),
        "roofline": {"bound": "hbm", "achieved": sb / (med_s * 1e-3 / (M - 1)) / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": sb / (med_s * 1e-3 / (M - 1)) / 1e9 / HBM_PEAK_GBS,
                     "bytes_per_launch": sb, "kernel": "k_cheb_step (scalar SELL)"}}}
    del Hsc, ws
    if not args.no_doubling:
        out["variants"]["doubling"] = kpm_variant(args, "doubling", {"doubling": 1}, Hs, aa, bb, r, M, R, Rp, 4,
                                                  diag, "c32", cfg, mu_c, rho_c, E, stream, dev)
    # learned form of Eq. (2): one network per two-centre integral on the bond's edge features
    # (seeded weights, shared hidden layers; the assembly cost does not depend on their values)
    K = 4 if norb == 4 else 10
    rng = np.random.default_rng(w["seed"])
    P = np.repeat(synth.init_mlp_params(w["seed"], out_scale=0.5)[None, :], K, axis=0)
    P[:, 1600:1632] = rng.uniform(-0.5, 0.5, (K, 32)) / math.sqrt(32)
    model = dict(params=torch.from_numpy(P.astype(np.float32)).to(dev), shift=np.zeros(16),
                 scale=np.concatenate([np.full(8, 0.3), np.full(8, 1.5)]), r_desc=synth.R_DESC)
    del Hs
    times = {"plain": [], "learned": []}
    for _ in range(max(2, args.steps)):
        for lab in ("plain", "learned"):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            Hx = tbkpm.build_hamiltonian_sk(pos, sp, s.box, s.periodic, *synth.SK_V, synth.SK_ES, synth.SK_EP,
                                            r_cut=synth.R_HOP, r0=synth.R0, beta=synth.BETA, fmt=w["fmt"], slice=64,
                                            stream=stream, d=dint, e_d=synth.SK_ED,
                                            model=model if lab == "learned" else None)
            torch.cuda.synchronize()
            times[lab].append((time.perf_counter() - t1) * 1e3)
            nbonds = Hx.st.n_bonds
            del Hx
    Hl = tbkpm.build_hamiltonian_sk(pos, sp, s.box, s.periodic, *synth.SK_V, synth.SK_ES, synth.SK_EP,
                                    r_cut=synth.R_HOP, r0=synth.R0, beta=synth.BETA, fmt=w["fmt"], slice=64,
                                    stream=stream, d=dint, e_d=synth.SK_ED, model=model)
    la, lb = Hl.scale()
    ev[0].record(stream)
    tbkpm.kpm_moments(Hl, la, lb, r, M, "c32", work=work, mu=mu, stream=stream, config=cfg)
    ev[1].record(stream)
    torch.cuda.synchronize()
    out["variants"]["learned_sk"] = {
        "networks": K, "bonds": int(nbonds), "build_ms_median": float(np.median(times["learned"])),
        "plain_build_ms_median": float(np.median(times["plain"])), "kpm_ms": ev[0].elapsed_time(ev[1]),
        "a_eV": la, "b_eV": lb}
    del Hl


def bench_vac(args, w):
    """Velocity-autocorrelation conductivity (Eq. (3)): per step and frame the Hamiltonian
    and velocity operator are built, the correlation moments of n_t propagation steps
    computed (M - 1 recurrence launches per time step, whose recurrences run
    B = tbkpm.vac_time_batch(R) time steps at a time as one of R * B vectors; one
    Chebyshev-Bessel propagation of phi_R and phi_L together and one velocity product per
    time step) and sigma(E, t) formed.  A multi-frame workload also computes each frame's
    DOS moments and integrated DOS and, over the frames, the averaged plateau
    conductivity, carriers and mobility (Sec. 2.4, Sec. 3)."""
    import torch
    from paper_2509_06525_amd import synth, tbkpm
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    M, R, n_t, dt = w["M"], w["R"], w["n_t"], w["dt"]
    F = w.get("frames", 1)
    log(f"generating {args.workload}")
    frames = synth.make_frames(args.workload) if F > 1 else [synth.make_structure(args.workload)]
    s = frames[0]
    sk = bool(w.get("sk"))
    norb = w.get("orbitals", 4) if sk else 1
    N = s.n
    nr = norb * N                                      # orbital rows
    pos = [torch.from_numpy(fr.pos).to(dev) for fr in frames]
    sp = torch.from_numpy(s.species).to(dev)
    r = torch.from_numpy(synth.random_phase(nr, R, w["seed"] + synth.VECTOR_SEED_OFFSET, np.complex64)).to(dev)
    held = []
    slice_, config, config_dos = args.slice, None, None
    if not args.no_tune and not sk:
        if not args.retune:
            use_shipped_tuning()
        # the recurrence runs R * B vectors at a time (B time steps)
        tune = tbkpm.autotune(pos[0], sp, s.box, s.periodic, s.onsite, s.t_pair, R * tbkpm.vac_time_batch(R), "c32",
                              r_cut=synth.R_HOP, r0=synth.R0, beta=synth.BETA, stream=stream)
        slice_, config = tune.slice, tune.config
        log(f"tuned: slice {slice_} {config.as_dict()}")
    if sk:
        slice_ = 64                                    # atom slices

    def build(f):
        if sk:
            return tbkpm.build_hamiltonian_sk(pos[f], sp, s.box, s.periodic, *synth.SK_V, synth.SK_ES, synth.SK_EP,
                                              r_cut=synth.R_HOP, r0=synth.R0, beta=synth.BETA, fmt=w["fmt"],
                                              slice=slice_, stream=stream, d=synth.SK_D if norb == 9 else None,
                                              e_d=synth.SK_ED)
        H = tbkpm.build_hamiltonian(pos[f], sp, s.box, s.periodic, s.onsite, s.t_pair, r_cut=synth.R_HOP,
                                    r0=synth.R0, beta=synth.BETA, fmt=w["fmt"], slice=slice_, stream=stream,
                                    into=held.pop() if held else None)
        held.append(H)
        return H

    if sk and args.block_shape:
        fixed = {k: int(v) for k, v in (kv.split("=") for kv in args.block_shape.split(","))}
        slice_ = fixed["slice"]
        config = tbkpm.make_config(fixed["vpt"], fixed["tpb"], fixed["nt"], fixed["xr"], 1, atom_rows=fixed["atom"])
    elif sk and not args.no_tune:
        # atom-slice height and block launch shape, searched on the recurrence of R * B
        # vectors (B time steps at a time) that dominates the step
        rt = torch.from_numpy(synth.random_phase(nr, R * tbkpm.vac_time_batch(R),
                                                 w["seed"] + 2 + synth.VECTOR_SEED_OFFSET,
                                                 np.complex64)).to(dev)
        best_ms = float("inf")
        for sl in (16, 32, 64):
            slice_ = sl
            Ht = build(0)
            c_, m_, _ = block_shape_search(Ht, *Ht.scale(), rt, False, stream)
            if m_ < best_ms:
                best_ms, best_slice, config = m_, sl, c_
            del Ht
        slice_ = best_slice
        del rt
        log(f"tuned: slice {slice_} {config.as_dict()} ({best_ms:.3f} ms per moment)")

    scales = []
    for f in range(F):
        scales.append(build(f).scale())
    a, b = scales[0]
    n_cheb = tbkpm.chebyshev_terms(max(x[0] for x in scales), dt)
    lo = max(bb - 0.99 * aa for aa, bb in scales)
    hi = min(bb + 0.99 * aa for aa, bb in scales)
    E = torch.linspace(lo, hi, 2001, dtype=torch.float64, device=dev)
    if F > 1:
        R_dos = w["R_dos"]
        r_dos = torch.from_numpy(synth.random_phase(N, R_dos, w["seed"] + 1 + synth.VECTOR_SEED_OFFSET,
                                                    np.complex64)).to(dev)
        if not args.no_tune:
            config_dos = tbkpm.autotune(pos[0], sp, s.box, s.periodic, s.onsite, s.t_pair, R_dos, "c32",
                                        r_cut=synth.R_HOP, r0=synth.R0, beta=synth.BETA, stream=stream).config
        sig_all = torch.empty((F, n_t, E.numel()), dtype=torch.float64, device=dev)
        n_all = torch.empty((F, E.numel()), dtype=torch.float64, device=dev)

    def step():
        res = None
        for f in range(F):
            Hs = build(f)
            aa, bb = Hs.scale()
            vx = tbkpm.build_velocity(Hs, pos[f], s.box, s.periodic, 0, stream=stream)
            nu = tbkpm.vac_moments(Hs, vx, aa, bb, r, M, n_t, dt, n_cheb, "c32", config=config, stream=stream)
            sig = tbkpm.vac_sigma(tbkpm.mean_moments(nu, stream=stream), aa, bb, dt, E, stream=stream)
            if F > 1:
                sig_all[f].copy_(sig)
                mu = tbkpm.kpm_moments(Hs, aa, bb, r_dos, M, "c32", stream=stream, config=config_dos)
                n_all[f].copy_(tbkpm.integrated_dos(tbkpm.mean_moments(mu, stream=stream), aa, bb, E, stream=stream))
        if F > 1:
            res = tbkpm.mobility(sig_all, n_all, 0.5 * N, stream=stream)
        return Hs, sig, res

    log(f"N={N} x {F} frames, M={M} R={R} n_t={n_t} dt={dt} fs, {n_cheb} propagator terms: "
        f"warmup {args.warmup}, timed {args.steps}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        Hs, sig, res = step()
        torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    st = Hs.st
    Rp = 1
    while Rp < R:
        Rp *= 2
    per_val = norb * norb if sk else 1
    hb = st.n_entries * (4 * per_val + 4) + st.n_ptr * 8    # values (FP32) + columns, slice offsets
    B = tbkpm.vac_time_batch(R)
    n_batches = -(-n_t // B)
    # recurrence launches read the matrix once per batch of B time steps and, per time
    # step, its vectors (pair form: gather T_n, T_{n-1}, left vector, write T_{n+1})
    rec = n_batches * (M - 1) * hb + n_t * (M - 1) * nr * Rp * 8 * 4
    # propagator term on phi_R and phi_L together: T_k gather, T_{k-1}, T_{k+1}, acc r/w
    prop = hb + nr * 2 * Rp * 8 * 5
    vel = hb + nr * Rp * 8 * 2
    total = F * (rec + n_t * ((n_cheb - 1) * prop + vel))
    achieved = total / sec / 1e9
    out = {
        "metric": "VAC atom*moments*timesteps/s" if not sk else "VAC orbital*moments*timesteps/s",
        "value": F * nr * M * R * n_t / sec,
        "unit": "atom*moments*timesteps/s" if not sk else "orbital*moments*timesteps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "n_atoms": N, "orbital_rows": nr, "frames": F, "moments": M,
                   "vectors": R,
                   "time_steps": n_t, "time_batch": B, "dt_fs": dt, "propagator_terms": n_cheb, "format": w["fmt"],
                   "slice": slice_, "precision": "c32", "a_eV": a, "b_eV": b,
                   "launch": None if config is None else config.as_dict()},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "whole VAC step (k_cheb_step_atom pair form, k_evolve_term_atom, "
                               "k_apply_velocity_blk)" if sk else
                               "whole VAC step (k_cheb_step pair form, k_evolve_term, k_apply_velocity)",
                     "bytes_per_step": total},
        "sigma_max": float(sig[-1].abs().max()),
    }
    if F > 1:
        # carriers per cm^2 (spin 2, sheet area) and the mobility at a few concentrations
        area = float(s.box[0] * s.box[1])
        ssc, car, mob = (x.cpu().numpy() for x in res)
        conc = 2.0 * car / area * 1e16
        Eh = E.cpu().numpy()
        pts = {}
        for n_cm2 in (1e12, 5e12, 1e13):
            for sign, lab in ((1.0, "electrons"), (-1.0, "holes")):
                k = int(np.argmin(np.abs(conc - sign * n_cm2)))
                pts[f"{lab}_{n_cm2:.0e}"] = {"E_eV": float(Eh[k]), "n_cm2": float(conc[k]),
                                             "mobility_cm2_Vs": float(mob[k])}
        out["mobility"] = {"n_ref_states": 0.5 * N, "area_A2": area, "points": pts,
                           "dos_vectors": w["R_dos"],
                           "dos_launch": None if config_dos is None else config_dos.as_dict()}
    print(json.dumps(out), flush=True)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; the path's multi-GPU sharding "
                                   "(halo exchange per step, one moment all-reduce) is design only",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2509_06525_amd import synth, tbkpm

    w = dict(synth.WORKLOADS[args.workload])
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")
        del src, dst
    if w["kind"] == "snapshots":
        return bench_snapshots(args, w)
    if w.get("vac"):
        return bench_vac(args, w)
    if w.get("sk"):
        return bench_sk(args, w)
    stream = torch.cuda.current_stream()

    log(f"generating {args.workload}")
    s = synth.make_structure(args.workload)
    N, M, R = s.n, w["M"], w["R"]
    cdt = np.complex64 if w["precision"] == "c32" else np.complex128
    r_host = synth.random_phase(N, R, w["seed"] + synth.VECTOR_SEED_OFFSET, cdt)
    pos = torch.from_numpy(s.pos).to(dev)
    sp = torch.from_numpy(s.species).to(dev)
    r = torch.from_numpy(r_host).to(dev)
    del r_host
    fmt = w["fmt"]
    slice_ = 1 if fmt == "csr_f64" else args.slice
    fixed_ab = ("a" in w)
    config = None
    tune = None
    if fmt != "csr_f64" and not args.no_tune:
        if not args.retune:
            use_shipped_tuning()
        log("autotuning slice height and launch shape")
        tune = tbkpm.autotune(pos, sp, s.box, s.periodic, s.onsite, s.t_pair, R, w["precision"],
                              r_cut=synth.R_HOP, r0=synth.R0, beta=synth.BETA, stream=stream)
        slice_ = tune.slice
        config = tune.config
        log(f"tuned: slice {slice_} {config.as_dict()} {tune.ms_per_step:.4f} ms/step "
            f"({tune.candidates} candidates)")

    def build(into=None):
        return tbkpm.build_hamiltonian(pos, sp, s.box, s.periodic, s.onsite, s.t_pair,
                                       r_cut=synth.R_HOP, r0=synth.R0, beta=synth.BETA,
                                       fmt=fmt, slice=slice_, stream=stream, into=into)

    H = build()
    a, b = (w["a"], w["b"]) if fixed_ab else H.scale()
    work = tbkpm.alloc_workspace(H, R, M, w["precision"], dev, config)
    mu = torch.empty((R, M), dtype=torch.float64, device=dev)
    E = torch.linspace(b - 0.99 * a, b + 0.99 * a, 2001, dtype=torch.float64, device=dev)
    if fixed_ab:
        E = torch.linspace(w["e_lo"], w["e_hi"], w["n_e"], dtype=torch.float64, device=dev)
    held = [H]          # the Hamiltonian's buffers are rebuilt in place every step
    del H

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    kpm_ms = []

    def step():
        Hs = build(into=held.pop())
        held.append(Hs)
        aa, bb = (w["a"], w["b"]) if fixed_ab else Hs.scale()
        ev[0].record(stream)
        tbkpm.kpm_moments(Hs, aa, bb, r, M, w["precision"], work=work, mu=mu, stream=stream, config=config)
        ev[1].record(stream)
        rho = tbkpm.kpm_dos(tbkpm.mean_moments(mu, stream=stream), aa, bb, E, stream=stream)
        return Hs, aa, bb, rho

    log(f"N={N} M={M} R={R}: warmup {args.warmup}, timed {args.steps}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    tbkpm.step_timer(True)        # events around the step launches only, on the same stream
    t0 = time.perf_counter()
    for _ in range(args.steps):
        Hs, aa, bb, rho = step()
        torch.cuda.synchronize()
        kpm_ms.append(ev[0].elapsed_time(ev[1]))
    t1 = time.perf_counter()
    step_ms, step_launches = tbkpm.step_timer_read()
    tbkpm.step_timer(False)
    sec_per_step = (t1 - t0) / args.steps
    value = N * M * R / sec_per_step

    # Roofline of the recurrence kernel: its average launch time from the step timer.
    Rp = 1
    while Rp < R:
        Rp *= 2
    elem = 4 if w["precision"] == "c32" else 8
    diag = Hs.st.has_onsite or bb != 0.0
    launch_cfg = config if config is not None else tbkpm.default_config(Hs, R, w["precision"])
    launch_bytes = cheb_step_bytes(Hs, Rp, elem, diag, compact=bool(launch_cfg.compact_columns))
    kpm_med = float(np.median(kpm_ms))
    launch_s = step_ms * 1e-3 / step_launches
    achieved = launch_bytes / launch_s / 1e9
    mu_c = mu.cpu().numpy().copy()
    rho_c = rho.cpu().numpy()

    out = {
        "metric": METRIC, "value": value, "unit": "atom*moments/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec_per_step * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if w["precision"] == "c32" else "f64", "data": "synthetic",
        "config": {"workload": args.workload, "n_atoms": N, "moments": M, "vectors": R,
                   "format": fmt, "slice": slice_, "precision": w["precision"],
                   "a_eV": aa, "b_eV": bb},
        "kpm_ms_median": kpm_med,
        "tuning": None if tune is None else {"slice": tune.slice, "launch": tune.config.as_dict(),
                                             "tuned_ms_per_step": tune.ms_per_step,
                                             "candidates": tune.candidates},
        "kpm_atom_moments_per_s": N * M * R / (kpm_med * 1e-3),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": profiled_traffic(args.workload, "direct", slice_, launch_cfg.as_dict()),
                     "traffic_source": f"profiles/k_cheb_step_{args.workload}.md (stored rocprofv3 FETCH_SIZE, "
                                       "WRITE_SIZE runs, copy-calibrated; null when the kernel or launch "
                                       "shape differs)",
                     "kernel": "k_cheb_step", "bytes_per_launch": launch_bytes,
                     "launch_us": launch_s * 1e6, "launches_timed": step_launches,
                     "launch_us_kpm_window": kpm_med * 1e3 / (M - 1)},
    }
    out["roofline"].update(stream_probe(dev))

    # DOS and moments against the oracle's stored full-size moments (its vector subset,
    # its (a, b) from FP64 Gershgorin bounds), same energy grid.
    gold = None if args.no_variants else golden_moments(args.workload)
    if gold is not None:
        ga, gb, gmu = gold
        nv = gmu.shape[0]
        rg = r[:, :nv].contiguous()
        mu_g = tbkpm.kpm_moments(Hs, ga, gb, rg, M, w["precision"], stream=stream)
        Eg = torch.linspace(gb - 0.99 * ga, gb + 0.99 * ga, 2001, dtype=torch.float64, device=dev)
        rho_gpu = tbkpm.kpm_dos(tbkpm.mean_moments(mu_g, stream=stream), ga, gb, Eg, stream=stream).cpu().numpy()
        rho_orc = tbkpm.kpm_dos(torch.from_numpy(gmu.mean(0)).to(dev), ga, gb, Eg, stream=stream).cpu().numpy()
        out["vs_oracle"] = {"vectors": nv, "a_eV": ga, "b_eV": gb,
                            "dos_relL2_vs_oracle": float(np.linalg.norm(rho_gpu - rho_orc) / np.linalg.norm(rho_orc)),
                            "max_abs_dmu_over_N_vs_oracle": float(np.abs(mu_g.cpu().numpy() - gmu).max() / N),
                            "source": f"tests/golden/oracle_moments_{args.workload}.txt"}
        del mu_g

    log(f"timed: {sec_per_step * 1e3:.1f} ms/step, kpm {kpm_med:.1f} ms")
    variants = []
    if args.no_variants:
        pass
    elif not args.no_doubling and M >= 2:
        variants.append(("doubling", {"doubling": 1}))
    if Hs.st.uniform_hop and not args.no_variants:
        variants.append(("uniform_values", {"uniform_values": 1}))
        if not args.no_doubling and M >= 2:
            variants.append(("doubling_uniform_values", {"doubling": 1, "uniform_values": 1}))
    if variants:
        args.rebuild = lambda sl: tbkpm.build_hamiltonian(pos, sp, s.box, s.periodic, s.onsite, s.t_pair,
                                                          r_cut=synth.R_HOP, r0=synth.R0, beta=synth.BETA,
                                                          fmt=fmt, slice=sl, stream=stream)
        out["variants"] = {}
        for label, fields in variants:
            vt = None
            if tune is not None:
                t = tbkpm.autotune(pos, sp, s.box, s.periodic, s.onsite, s.t_pair, R, w["precision"],
                                   r_cut=synth.R_HOP, r0=synth.R0, beta=synth.BETA, stream=stream, **fields)
                vt = (t.slice, t.config)
            out["variants"][label] = kpm_variant(args, label, fields, Hs, aa, bb, r, M, R, Rp, elem, diag,
                                                 w["precision"], config, mu_c, rho_c, E, stream, dev, vt)

    # FP64 GPU path on the same structure and vectors (reported beside the C32 path).
    if not args.no_fp64 and w["precision"] == "c32":
        H64 = tbkpm.build_hamiltonian(pos, sp, s.box, s.periodic, s.onsite, s.t_pair, r_cut=synth.R_HOP,
                                      r0=synth.R0, beta=synth.BETA, fmt="sell_f64", slice=slice_,
                                      stream=stream)
        del Hs
        held.clear()
        r64 = r.to(torch.complex128)
        work = None
        torch.cuda.empty_cache()
        w64 = tbkpm.alloc_workspace(H64, R, M, "f64", dev)
        mu64 = torch.empty((R, M), dtype=torch.float64, device=dev)
        ev[2].record(stream)
        tbkpm.kpm_moments(H64, aa, bb, r64, M, "f64", work=w64, mu=mu64, stream=stream)
        ev[3].record(stream)
        torch.cuda.synchronize()
        ms64 = ev[2].elapsed_time(ev[3])
        rho64 = tbkpm.kpm_dos(tbkpm.mean_moments(mu64, stream=stream), aa, bb, E, stream=stream).cpu().numpy()
        out["fp64_path"] = {"kpm_ms": ms64, "atom_moments_per_s": N * M * R / (ms64 * 1e-3),
                            "dos_relL2_c32_vs_fp64": float(np.linalg.norm(rho_c - rho64) / np.linalg.norm(rho64)),
                            "max_abs_dmu_over_N": float(np.abs(mu_c - mu64.cpu().numpy()).max() / N)}
        del H64, w64, r64

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, one core)")
        cells = args.cpu_sample_cells or max(8, int(math.sqrt(4e9 / (4.0 * M * R))))
        if "nx" in w:
            cells = min(cells, w["nx"])
        out["cpu_baseline"] = cpu_baseline(w, cells)
        out["cpu_baseline"]["host"] = platform.processor() or platform.machine()
        out["cpu_baseline"]["nproc"] = os.cpu_count()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
