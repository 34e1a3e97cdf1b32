#!/usr/bin/env python3
"""Docking throughput on one MI355X.

A step is one ad_dock_batch call over the whole workload: every run of every
ligand goes through initial population, GA generations (pose, grid
interpolation, intramolecular pairs, energy) and ADADELTA local search
(the same plus the analytic gradient) until the evaluation cap, then the
best pose per ligand is re-scored.  Inputs (grid maps and the ligand batch)
are resident in HBM before the timed region starts.

Prints one JSON line (metric, value = ligands docked / s, evals / s,
roofline of the dominant kernel, oracle CPU baseline).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ligands docked/sec + score-grad evals/sec, 1 MI355X, plain vs screened at 95% recall"
# MI355X published FP32 vector peak, and the published FP64 vector peak
# (256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz); the FMA rates this GPU
# reaches are measured beside them (ad_microbench)
PEAK_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def flops_per_eval(info, grad):
    """Algorithmic FLOP of one evaluation of a ligand, counted from the
    scoring function's formulas (add, sub, mul 1; FMA 2; each transcendental
    1).  With the gradient: per pair 62 (distance 9, smoothing 2, 12-6/12-10
    14, electrostatics 17, desolvation 5, totals 5, force 9, accumulation 1);
    per atom 129 (grid coordinates 9, corner values 32, interpolation 24, its
    gradient 27, accumulation 1, global transform 18, torque 18); per atom and
    torsion moving it 33 (rotation 18, torsion torque 15); per torsion 38
    (sin/cos and rotation matrix 22, axis and projection 16); per pose 40
    (quaternion normalisation and matrix).  Energy only: 36, 84, 18, 22, 40."""
    P, N, T, D = info["n_pairs"], info["n_atoms"], info["n_torsions"], info["depth_sum"]
    if grad:
        return 62 * P + 129 * N + 33 * D + 38 * T + 40
    return 36 * P + 84 * N + 18 * D + 22 * T + 40


def oracle_flops_per_eval(info):
    """Floating-point operations the FP64 oracle itself runs for one energy +
    gradient evaluation, from its op-counting build (oracle/opcount.hpp:
    add, sub, mul, div and each transcendental 1): 54 per pose, 227 per atom,
    58 per (atom, torsion moving it), 27 per torsion and 28 + 78 per pair (the
    pair functions' count outside the smoothing band's lower side for a
    non-H-bond pair, their smallest).  A lower bound of the oracle's count:
    a pair below the band or an H-bond pair costs one more.  The oracle
    recomputes the type-pair constants and the force products per pair and
    the torsion sin/cos per moved atom; flops_per_eval counts the same
    function with those hoisted."""
    P, N, T, D = info["n_pairs"], info["n_atoms"], info["n_torsions"], info["depth_sum"]
    return 54 + 227 * N + 58 * D + 27 * T + 106 * P


def measured_traffic(path=None, src=None):
    """HBM bytes of one generation's local search (its launches) from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None once the
    kernel source differs from the one the counters were taken on."""
    import hashlib
    path = path or os.path.join(ROOT, "profiles", "k_ls_generation_screen64.md")
    src = src or os.path.join(ROOT, "paper_2007_03678_amd", "csrc", "kernels.hip")
    try:
        fields = dict(line.split(": ", 1) for line in open(path).read().splitlines()
                      if line.startswith("traffic_"))
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if fields.get("traffic_kernel_sha256", "").strip() != h:
            return None
        return float(fields["traffic_bytes_per_generation"])
    except (OSError, KeyError, ValueError):
        return None


def workload(name, n_ligands=None):
    import synth
    c = synth.config(name, n_ligands=n_ligands)
    return c


def cpu_baseline(c, dock, seconds, log_fn):
    """The oracle docking ligand 0 of the workload with every host core, on a
    reduced evaluation cap per run; ligands/s extrapolated by evaluation
    count to the full configuration."""
    import numpy as np

    import oracle
    import synth
    orc = oracle.Oracle(synth.forcefield())
    t0 = time.time()
    G = orc.grid(c["grid"], c["receptor"])
    log_fn(f"cpu baseline: oracle maps built in {time.time() - t0:.1f}s")
    L = orc.ligand(c["ligands"][0])
    pop, nrun = dock["pop"], dock["nrun"]
    n_ls = int(round(dock["ls_rate"] * pop))
    per_gen = (pop - 1) + n_ls * dock["ls_iters"]
    # calibrate: two generations of every run
    p = oracle.make_params(nrun=nrun, pop=pop, max_gens=2, max_evals=10**12, ls_rate=dock["ls_rate"],
                           ls_iters=dock["ls_iters"])
    t0 = time.time()
    _, _, ev, _ = orc.dock(L, G, p, 1, 0)
    rate = ev.sum() / (time.time() - t0)
    gens = max(1, int((seconds * rate / nrun - pop) / per_gen))
    p = oracle.make_params(nrun=nrun, pop=pop, max_gens=gens, max_evals=10**12, ls_rate=dock["ls_rate"],
                           ls_iters=dock["ls_iters"])
    t0 = time.time()
    _, _, ev, _ = orc.dock(L, G, p, 1, 0)
    dt = time.time() - t0
    evals_s = ev.sum() / dt
    full_gens = min(dock["max_gens"], (dock["max_evals"] - pop) // per_gen)
    evals_per_ligand = nrun * (pop + full_gens * per_gen)
    # score + gradient evaluations of the same ligand on one core and on all
    cores = orc.max_threads()
    genos = synth.random_genotypes(5, 200_000, np.full(200_000, L.n_tor), c["grid"], margin=2.0)
    rates = {}
    for threads, n in ((1, 20_000), (cores, 200_000)):
        t0 = time.time()
        orc.score_batch([L], np.zeros(n, np.int32), G, genos[:n], threads=threads)
        rates[threads] = n / (time.time() - t0)
    log_fn(f"cpu baseline: score+gradient {rates[1]:.0f}/s on 1 core, {rates[cores]:.0f}/s on {cores}")
    return dict(value=evals_s / evals_per_ligand, unit="ligands/s", cores=cores, kind="oracle",
                cpu_model=cpu_model(), host_threads=os.cpu_count(), evals_per_s=evals_s,
                score_grad_evals_per_s={"1_core": round(rates[1], 1), f"{cores}_cores": round(rates[cores], 1)},
                sample=(f"ligand 0 ({L.n} atoms, {L.n_tor} torsions), {nrun} runs x pop {pop}, {gens} "
                        f"generations ({int(ev.sum())} evaluations, {dt:.1f}s); ligands/s extrapolated by "
                        f"evaluation count to {evals_per_ligand} evaluations per ligand"))


def cpu_model():
    """Host CPU model name (first processor entry of /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_single24(log_fn):
    """The oracle docking the single-ligand configuration in full (4 runs x
    pop 50 x 50 generations, ADADELTA 300 iterations on 6 % per generation),
    runs in parallel on the host cores."""
    import oracle
    import synth
    c = workload("single24")
    d = c["dock"]
    orc = oracle.Oracle(synth.forcefield())
    G = orc.grid(c["grid"], c["receptor"])
    L = orc.ligand(c["ligands"][0])
    p = oracle.make_params(nrun=d["nrun"], pop=d["pop"], max_gens=d["max_gens"], max_evals=d["max_evals"],
                           ls_rate=d["ls_rate"], ls_iters=d["ls_iters"])
    t0 = time.time()
    _, E, ev, _ = orc.dock(L, G, p, 20200707, 0)
    dt = time.time() - t0
    log_fn(f"cpu single24: oracle docked in full in {dt:.2f}s ({int(ev.sum())} evaluations)")
    return dict(value=round(1.0 / dt, 4), unit="ligands/s", seconds=round(dt, 3), evals=int(ev.sum()),
                evals_per_s=round(float(ev.sum()) / dt, 1), best_energy=round(float(E.min()), 3),
                threads=min(d["nrun"], orc.max_threads()), kind="oracle", sample="in full")


def single24_leg(log_fn, steps=10):
    """The single-ligand configuration on the GPU: one ligand of 24 atoms and
    5 torsions, 2,000-atom receptor, 40^3 grid, 4 runs x pop 50 x 50
    generations; the docking call timed `steps` times after a warm-up (maps
    and ligand resident)."""
    import torch

    import paper_2007_03678_amd as pkg
    import synth
    c = workload("single24")
    d = c["dock"]
    ctx = pkg.create(synth.forcefield(), 0)
    ctx.ad_build_grids(c["grid"], c["receptor"])
    batch = ctx.ad_load_ligands(c["ligands"])
    params = pkg.make_params(**d)
    seed = 20200707
    ctx.ad_dock_batch(batch, params, seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = ctx.ad_dock_batch(batch, params, seed)
    dt = (time.perf_counter() - t0) / steps
    info = batch.info(0)
    batch.free()
    ctx.close()
    log_fn(f"single24: {dt * 1e3:.2f} ms per docking, best energy {r['best_energy'][0]:.3f}")
    return {"workload": (f"single24: 1 ligand ({info['n_atoms']} atoms, {info['n_torsions']} torsions), "
                         f"{len(c['receptor'].types)}-atom receptor, {c['grid'].n[0]}^3 x "
                         f"{len(c['grid'].map_types) + 2} maps, {d['nrun']} runs x pop {d['pop']} x "
                         f"{d['max_gens']} generations"),
            "ligands_per_s": round(1.0 / dt, 3), "ms_per_ligand": round(dt * 1e3, 3),
            "evals_per_s": round(float(r["evals"][0]) / dt, 1), "evals": int(r["evals"][0]),
            "best_energy": round(float(r["best_energy"][0]), 3), "steps": steps}


def score_leg(ctx, ligands, grid, log_fn, n=1 << 20):
    """ad_score_poses with energy and gradient on n random poses per
    atom-capacity bucket: each bucket's ligands loaded as a batch of their
    own (a batch's score kernel is sized by its largest ligand), device
    arrays so the timed call makes no host copies, the kernel timed with HIP
    events."""
    import numpy as np
    import torch

    import synth

    nat = np.asarray(ligands.n_atoms_per_ligand)
    out = {}
    for name, sel in (("le64_atoms", np.flatnonzero(nat <= 64)), ("le128_atoms", np.flatnonzero(nat > 64))):
        if len(sel) == 0:
            continue
        batch = ctx.ad_load_ligands(ligands.subset(sel))
        infos = [batch.info(i) for i in range(batch.n)]
        ntor = np.array([i["n_torsions"] for i in infos])
        flop = np.array([flops_per_eval(i, True) for i in infos], dtype=np.float64)
        idx = (np.arange(n) % batch.n).astype(np.int32)
        genos = synth.random_genotypes(31, n, ntor[idx], grid, margin=2.0)
        gd, idd = torch.from_numpy(genos).cuda(), torch.from_numpy(idx).cuda()
        ctx.ad_score_poses(batch, idd[:4096], gd[:4096], grad=True)
        ctx.ad_synchronize()
        ctx.ad_get_kernel_timing(reset=True)
        ctx.ad_set_kernel_timing(True)
        t0 = time.perf_counter()
        ctx.ad_score_poses(batch, idd, gd, grad=True)
        ctx.ad_synchronize()
        wall = time.perf_counter() - t0
        kt = ctx.ad_get_kernel_timing(reset=True)
        ctx.ad_set_kernel_timing(False)
        ms = kt["score"][0]
        tf = float(flop[idx].sum()) / (ms / 1e3) / 1e12
        out[name] = {"poses": n, "ligands": int(batch.n), "kernel_ms": round(ms, 3), "wall_ms": round(wall * 1e3, 3),
                     "score_grad_evals_per_s": round(n / (ms / 1e3), 1), "tflops": round(tf, 3),
                     "frac": round(tf / PEAK_TFLOPS, 4)}
        log_fn(f"score_poses {name}: {n} poses in {ms:.2f} ms, {tf:.2f} TFLOP/s")
        del gd, idd
        batch.free()
    return out


def batch_leg(args, log_fn):
    """Batched uneven docking: 4,096 ligands of lognormal size (10-100 atoms,
    0-32 torsions) in one ad_dock_batch call, 10 runs x pop 150, 100,000
    evaluations per run; runs split into the two atom-capacity buckets.  Then
    the same set through ad_dock_stream in batches of 1,024."""
    import numpy as np
    import torch

    import paper_2007_03678_amd as pkg
    import synth

    t0 = time.time()
    c = synth.config("batch4096")
    ctx = pkg.create(synth.forcefield(), 0)
    ctx.ad_build_grids(c["grid"], c["receptor"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    batch = ctx.ad_load_ligands(c["ligands"])
    load_s = time.perf_counter() - t1
    infos = [batch.info(i) for i in range(batch.n)]
    log_fn(f"batch4096: {batch.n} ligands generated and loaded in {time.time() - t0:.1f}s")
    dock = c["dock"]
    params = pkg.make_params(**dock)
    ctx.ad_get_kernel_timing(reset=True)
    ctx.ad_set_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = ctx.ad_dock_batch(batch, params, 20200707)
    dt = time.perf_counter() - t0
    kt = ctx.ad_get_kernel_timing(reset=True)
    ctx.ad_set_kernel_timing(False)
    sched = ctx.ad_get_schedule()
    shape = ctx.ad_get_launch_shape()
    queue = ctx.ad_get_work_queue()
    n_ls = int(np.floor(dock["ls_rate"] * dock["pop"] + 0.5))
    ls_flop = dock["nrun"] * n_ls * dock["ls_iters"] * sum(flops_per_eval(i, True) for i in infos)
    ls_ms, ls_n = kt["ls"]
    big = sum(1 for i in infos if i["n_atoms"] > 64)
    out = {
        "workload": (f"batch4096: {batch.n} ligands (atoms {min(i['n_atoms'] for i in infos)}-"
                     f"{max(i['n_atoms'] for i in infos)}, lognormal median 32; torsions 0-32), 8,000-atom receptor, "
                     f"80^3 x 10 FP32 maps, {dock['nrun']} runs x pop {dock['pop']}, cap {dock['max_evals']} evals/run"),
        "ligands_per_s": round(batch.n / dt, 3),
        "ligands_per_s_with_load": round(batch.n / (dt + load_s), 3),
        "load_s": round(load_s, 3),
        "evals_per_s": round(float(r["evals"].sum()) / dt, 1),
        "step_s": round(dt, 2),
        "generations": int(r["generations"][0]),
        "buckets": {"le64_atoms": batch.n - big, "le128_atoms": big},
        "ls_stage_pairs": sched["stage_pairs"], "ls_pair_unroll": shape["unroll"], "ls_wg_per_cu": shape["wg_per_cu"],
        "work_queue": queue, "packed_runs": sched["packed_runs"],
        # local-search busy time per generation: the union of the launch
        # intervals of both buckets' chains (they overlap)
        "ls_phase_avg_ms": round(kt["busy_ms"]["ls"] / max(int(r["generations"][0]), 1), 3),
        "ls_phase_tflops": (round(ls_flop / (kt["busy_ms"]["ls"] / 1e3 / int(r["generations"][0])) / 1e12, 3)
                            if ls_n else None),
        "chains": ctx.ad_get_chains(),
    }
    log_fn(f"batch4096: docked in {dt:.1f}s")
    batch.free()
    out["score_poses"] = score_leg(ctx, c["ligands"], c["grid"], log_fn)
    # the same ligands streamed in batches of 1,024: host preparation and
    # upload of the next batch overlap the docking of the current one
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs = ctx.ad_dock_stream(c["ligands"], 1024, params, 20200707)
    ts = time.perf_counter() - t0
    st = rs["stats"]
    out["stream"] = {"batch_size": 1024, "ligands_per_s": round(len(c["ligands"]) / ts, 3),
                     "host_prep_s": round(st["prep_s"], 3), "dock_s": round(st["dock_s"], 3),
                     "wall_s": round(st["wall_s"], 3),
                     "prep_hidden_frac": round(max(0.0, st["prep_s"] + st["dock_s"] - st["wall_s"]) / st["prep_s"], 3),
                     "same_results_as_one_batch": bool(np.array_equal(rs["best_energy"], r["best_energy"]))}
    log_fn(f"batch4096: streamed in batches of 1024 in {ts:.1f}s")
    ctx.close()
    return out


def screened_campaign(args, log_fn):
    """Plain against screened docking (the screening setting: many ligands,
    one receptor).  The pre-screen is trained on the GPU on labels that plain
    docking produces (5 runs x population 100 on the 8,000-atom receptor's
    64^3 grid), then ranks the campaign set (126^3 grid over the same
    receptor); the top fraction is docked with the campaign's parameters.  A
    random holdout docked in full is the judge of recall and gives the plain
    rate; recall and the share of the ranking needed for 95 % recall are
    also pooled over several disjoint holdouts.  The ranking adds to the
    network's rank a size prior whose weight is fitted on a validation tenth
    of the labelled set."""
    import numpy as np
    import torch

    import paper_2007_03678_amd as pkg
    import synth
    from paper_2007_03678_amd import screen

    seed = 20200707
    ff = synth.forcefield()
    ctx = pkg.create(ff, 0)
    rec = synth.receptor(seed, 8000)
    out = {}
    # -- labels and training ------------------------------------------------
    t0 = time.time()
    ctx.ad_build_grids(synth.make_grid(64, 0.375, map_types=synth.ALL_TYPES), rec)
    train = synth.ligand_set_fast(seed + 11, args.train_ligands, atoms=(10, 100), torsions=(0, 32),
                                  dist="lognormal", packed=True)
    tb = ctx.ad_load_ligands(train)
    log_fn(f"campaign: {len(train)} training ligands generated and loaded in {time.time() - t0:.1f}s")
    p_lab = pkg.make_params(nrun=5, pop=100, max_gens=args.label_gens, ls_rate=0.06, ls_iters=300)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lab = ctx.ad_dock_batch(tb, p_lab, seed)
    t_label = time.perf_counter() - t0
    y = lab["best_energy"].astype(np.float64)
    log_fn(f"campaign: labels by plain docking in {t_label:.1f}s")
    # a validation split of the labelled set fits the size prior of the ranking
    split = np.random.default_rng(seed + 3).permutation(len(train))
    n_val = len(train) // 10
    val, trn = np.sort(split[:n_val]).astype(np.int32), np.sort(split[n_val:]).astype(np.int32)
    # labels clipped at the quantile of the fraction to be docked: the network
    # ranks the best labels among themselves and the rest count as equal
    label_max = float(np.percentile(y[trn], 100.0 * args.screen_frac))
    ps = pkg.Prescreen(ctx, seed=1, label_max=label_max)
    t0 = time.perf_counter()
    curve = ps.ad_prescreen_train(tb, trn, y[trn], epochs=args.epochs, seed=2)
    t_train = time.perf_counter() - t0
    log_fn(f"campaign: pre-screen trained in {t_train:.1f}s, loss {curve[0]:.3f} -> {curve[-1]:.3f}")
    prior_w, prior_f = screen.choose_prior_weight(ps.ad_prescreen_predict(tb, val), y[val],
                                                  train.n_atoms_per_ligand[val], 0.95, 0.01)
    # the docked fraction, chosen on the validation labels alone: the share of
    # the ranked validation list that holds `val_recall` of its labels' top 1 %
    # (above the 95 % target: labels come from shorter docking than the judge)
    val_rank = screen.prior_score(ps.ad_prescreen_predict(tb, val), train.n_atoms_per_ligand[val], prior_w)
    f_dock = screen.fraction_for_recall(val_rank, y[val], args.val_recall, 0.01)
    log_fn(f"campaign: size prior weight {prior_w} (validation share for 95% recall {prior_f:.3f}); "
           f"docked fraction {f_dock:.4f} ({args.val_recall:.3f} recall on validation)")
    tb.free()
    # -- campaign set --------------------------------------------------------
    t0 = time.time()
    grid = synth.make_grid(126, 0.375, map_types=synth.ALL_TYPES)
    ctx.ad_build_grids(grid, rec)
    camp = synth.ligand_set_fast(seed + 12, args.campaign_ligands, atoms=(10, 100), torsions=(0, 32),
                                 dist="lognormal", packed=True)
    cb = ctx.ad_load_ligands(camp)
    torch.cuda.synchronize()
    log_fn(f"campaign: {len(camp)} ligands generated and loaded, 126^3 maps built in {time.time() - t0:.1f}s")
    n = len(camp)
    p_full = pkg.make_params(nrun=20, pop=150, max_gens=10**9, max_evals=args.campaign_evals, ls_rate=0.06,
                             ls_iters=300)
    # screened step: rank every ligand, dock the chosen top fraction
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred = ps.ad_prescreen_predict(cb)
    rank = screen.prior_score(pred, camp.n_atoms_per_ligand, prior_w)
    t_pred = time.perf_counter() - t0
    sel = screen.top_fraction(rank, f_dock).astype(np.int32)
    r_sel = ctx.ad_dock_select(cb, sel, p_full, seed)
    t_screened = time.perf_counter() - t0
    log_fn(f"campaign: screened step (rank {n}, dock {len(sel)}) {t_screened:.1f}s")
    # judge: random holdouts docked in full (the plain rate and recall).  The
    # first is the configuration's holdout; recall is also pooled over
    # `holdout_seeds` disjoint holdouts of the same size (one docking call)
    k_h = max(1, args.holdout_seeds)
    size = min(args.holdout, n // (k_h + 1))
    draw = np.random.default_rng(seed).choice(n, size=size * (k_h + 1), replace=False)
    holds = [np.sort(draw[i * size:(i + 1) * size]).astype(np.int32) for i in range(k_h)]
    all_h = np.concatenate(holds)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r_hold = ctx.ad_dock_select(cb, all_h, p_full, seed)
    t_hold = time.perf_counter() - t0
    log_fn(f"campaign: {k_h} holdouts of {size} docked in {t_hold:.1f}s")
    judge_all = r_hold["best_energy"].astype(np.float64)
    judge, hold = judge_all[:size], holds[0]

    def sub_rank(idx):   # the screen's ranking of a subset: the prior ranks within the subset
        return screen.prior_score(pred[idx], camp.n_atoms_per_ligand[idx], prior_w)

    def pooled(score_of, frac):
        hp = [screen.recall(judge_all[i * size:(i + 1) * size], screen.top_fraction(score_of(holds[i]), frac),
                            top_frac=0.01) for i in range(k_h)]
        return sum(h for h, _ in hp), sum(q for _, q in hp)

    plain_rate = len(all_h) / t_hold
    hits, pos = screen.recall(judge, screen.top_fraction(sub_rank(hold), f_dock), top_frac=0.01)
    lo, hi = screen.clopper_pearson(hits, pos)
    p_hits, p_pos = pooled(sub_rank, f_dock)
    p_lo, p_hi = screen.clopper_pearson(p_hits, p_pos)
    h10, _ = pooled(sub_rank, args.screen_frac)
    n10, _ = pooled(lambda idx: pred[idx], args.screen_frac)
    f95_pool = screen.fraction_for_recall(sub_rank(all_h), judge_all, 0.95, 0.01)
    f95_net = screen.fraction_for_recall(pred[all_h], judge_all, 0.95, 0.01)
    from scipy.stats import spearmanr
    rho = float(spearmanr(pred[hold], judge)[0])
    nat = camp.n_atoms_per_ligand[hold].astype(np.float64)
    size_hits, _ = screen.recall(judge, screen.top_fraction(-nat, f_dock), top_frac=0.01)
    # a stronger judge on one more holdout: the same docking with a 5x higher cap
    extra = np.sort(draw[k_h * size:(k_h + 1) * size]).astype(np.int32)
    p_strong = pkg.make_params(nrun=20, pop=150, max_gens=10**9, max_evals=args.judge_evals, ls_rate=0.06,
                               ls_iters=300)
    t0 = time.perf_counter()
    r_weak = ctx.ad_dock_select(cb, extra, p_full, seed)
    r_strong = ctx.ad_dock_select(cb, extra, p_strong, seed)
    t_strong = time.perf_counter() - t0
    jw, js = r_weak["best_energy"].astype(np.float64), r_strong["best_energy"].astype(np.float64)
    pick = screen.top_fraction(sub_rank(extra), f_dock)
    sw_hits, sw_pos = screen.recall(jw, pick, top_frac=0.01)
    ss_hits, ss_pos = screen.recall(js, pick, top_frac=0.01)
    ss_lo, ss_hi = screen.clopper_pearson(ss_hits, ss_pos)
    log_fn(f"campaign: holdout with a {args.judge_evals}-evaluation judge in {t_strong:.1f}s: recall "
           f"{ss_hits}/{ss_pos} (against {sw_hits}/{sw_pos} with the campaign judge)")
    evals_sel = int(r_sel["evals"].sum())
    out = {
        "workload": (f"campaign: {n} ligands (atoms lognormal median 32 in 10-100, torsions 0-32), 8,000-atom "
                     f"receptor, 126^3 x 10 FP32 maps, 20 runs x pop 150, cap {args.campaign_evals} evals/run; "
                     f"pre-screen trained on {len(trn)} of {len(train)} ligands labelled by plain docking (5 runs x pop 100, "
                     f"{args.label_gens} generations, 64^3 grid)"),
        "plain_ligands_per_s": round(plain_rate, 3),
        "screened_ligands_per_s": round(n / t_screened, 3),
        "speedup": round(n / t_screened / plain_rate, 2),
        "frac_docked": round(f_dock, 4),
        "frac_docked_rule": f"share of the validation ranking holding {args.val_recall} of the validation labels' top 1%",
        "n_docked": int(len(sel)),
        "screened_step_s": round(t_screened, 2),
        "docked_set_ligands_per_s": round(len(sel) / (t_screened - t_pred), 3),
        "predict_ligands_per_s": round(n / t_pred, 1),
        "recall_top1pct": round(hits / pos, 4),
        "recall_hits": [int(hits), int(pos)],
        "recall_ci95": [round(lo, 4), round(hi, 4)],
        "size_heuristic_recall": round(size_hits / pos, 4),
        "holdout_spearman": round(rho, 4),
        "pooled": {"holdouts": k_h, "ligands": int(len(all_h)), "recall_hits": [int(p_hits), int(p_pos)],
                   "recall_top1pct": round(p_hits / p_pos, 4), "recall_ci95": [round(p_lo, 4), round(p_hi, 4)],
                   "frac_for_95pct_recall": round(f95_pool, 4),
                   "recall_at_10pct": [int(h10), int(p_pos)],
                   "network_alone": {"recall_at_10pct": [int(n10), int(p_pos)],
                                     "frac_for_95pct_recall": round(f95_net, 4)}},
        "strong_judge": {"max_evals_per_run": args.judge_evals, "ligands": int(len(extra)),
                         "recall_hits": [int(ss_hits), int(ss_pos)], "recall_ci95": [round(ss_lo, 4), round(ss_hi, 4)],
                         "campaign_judge_recall_hits": [int(sw_hits), int(sw_pos)],
                         "spearman_weak_vs_strong": round(float(spearmanr(jw, js)[0]), 4),
                         "mean_best_energy": [round(float(jw.mean()), 3), round(float(js.mean()), 3)]},
        "ranking": {"size_prior_weight": prior_w, "validation_frac_for_95pct_recall": round(prior_f, 4),
                    "validation_ligands": int(n_val)},
        "screened_evals_per_s": round(evals_sel / (t_screened - t_pred), 1),
        "train": {"ligands": int(len(trn)), "labelled": len(train), "epochs": args.epochs,
                  "label_dock_s": round(t_label, 2), "label_max": round(label_max, 3),
                  "train_s": round(t_train, 2), "graphs_per_s": round(len(trn) * args.epochs / t_train, 1),
                  "loss_first_epoch": round(float(curve[0]), 4), "loss_last_epoch": round(float(curve[-1]), 4)},
    }
    ps.close()
    cb.free()
    ctx.close()
    return out


def search_variants(ctx, batch, dock, infos, seed, plain, log_fn):
    """The paper's other local search (Solis-Wets) and autostop, on the main
    workload's ligands, receptor and search settings.

    Solis-Wets runs a fixed number of generations without an evaluation cap,
    so every run takes all of them and the local-search evaluations are the
    total minus the GA's; its kernel is timed with HIP events like the
    ADADELTA one (energy-only evaluations).  Autostop runs the ADADELTA
    search of the main leg with per-run stopping and is compared with that
    leg's timed step (same seed)."""
    import numpy as np
    import torch

    import paper_2007_03678_amd as pkg

    n_lig, nrun, pop = batch.n, dock["nrun"], dock["pop"]
    n_ls = int(np.floor(dock["ls_rate"] * pop + 0.5))
    G = 200
    sw = dict(dock, ls_method=1, max_gens=G, max_evals=2 ** 62)
    ctx.ad_dock_batch(batch, pkg.make_params(**dict(sw, max_gens=2)), seed)
    ctx.ad_get_kernel_timing(reset=True)
    ctx.ad_set_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = ctx.ad_dock_batch(batch, pkg.make_params(**sw), seed)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kt = ctx.ad_get_kernel_timing(reset=True)
    ctx.ad_set_kernel_timing(False)
    assert np.all(r["generations"] == G)
    ls_evals = r["evals"] - nrun * (pop + G * (pop - 1))
    flop = sum(int(e) * flops_per_eval(i, False) for e, i in zip(ls_evals, infos))
    ls_ms, ls_n = kt["ls"]
    ls_busy = kt["busy_ms"]["ls"]   # the chains' launches overlap: their union
    tf = flop / (ls_busy / 1e3) / 1e12
    log_fn(f"solis-wets: {G} generations in {el:.2f}s, local-search kernel {tf:.2f} TFLOP/s")
    out = {"solis_wets": {
        "workload": (f"the main workload's ligands and grid, {nrun} runs x pop {pop}, Solis-Wets "
                     f"(at most {dock['ls_iters']} evaluations) on {n_ls}/gen, {G} generations, no evaluation cap"),
        "ligands_per_s": round(n_lig / el, 3),
        "evals_per_s": round(float(r["evals"].sum()) / el, 1),
        "ls_evals_per_search": round(float(ls_evals.sum()) / (n_lig * nrun * G * n_ls), 1),
        "ls_kernel": "k_sw_generation (energy-only evaluations)",
        "ls_kernel_tflops": round(tf, 3),
        "frac": round(tf / PEAK_TFLOPS, 4),
        "ls_kernel_ms_per_launch": round(ls_ms / max(ls_n, 1), 3),
        "ls_busy_ms_per_generation": round(ls_busy / G, 3),
        "mean_best_energy": round(float(r["best_energy"].mean()), 3),
    }}
    # autostop on the main leg's search
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = ctx.ad_dock_batch(batch, pkg.make_params(**dict(dock, autostop=1)), seed)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    log_fn(f"autostop: {el:.2f}s")
    out["autostop"] = {
        "workload": "the main leg's docking with per-run autostop (std of the best energy over 10 generations "
                    "below 0.15 kcal/mol)",
        "ligands_per_s": round(n_lig / el, 4),
        "speedup_vs_plain": round((n_lig / el) / plain["ligands_per_s"], 3),
        "evals_frac_of_plain": round(float(r["evals"].sum()) / plain["evals"], 4),
        "mean_generations_best_run": round(float(r["generations"].mean()), 1),
        "generations_plain": plain["generations"],
        "mean_best_energy_change": round(float((r["best_energy"] - plain["best_energy"]).mean()), 3),
    }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="screen64")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-campaign", action="store_true", help="skip the plain-vs-screened campaign")
    ap.add_argument("--no-batch4096", action="store_true", help="skip the batched uneven docking leg")
    ap.add_argument("--no-variants", action="store_true", help="skip the Solis-Wets and autostop measurements")
    ap.add_argument("--campaign-ligands", type=int, default=65536)
    ap.add_argument("--train-ligands", type=int, default=200_000)
    ap.add_argument("--label-gens", type=int, default=10)
    ap.add_argument("--epochs", type=int, default=15)
    ap.add_argument("--campaign-evals", type=int, default=100_000, help="evaluation cap per run in the campaign")
    ap.add_argument("--holdout", type=int, default=2048, help="campaign ligands per holdout docked in full as the judge")
    ap.add_argument("--holdout-seeds", type=int, default=5, help="disjoint holdouts pooled for recall")
    ap.add_argument("--screen-frac", type=float, default=0.1,
                    help="label clip quantile of the pre-screen training (and a reported recall point)")
    ap.add_argument("--val-recall", type=float, default=0.975,
                    help="validation recall of the labels' top 1%% that sets the docked fraction")
    ap.add_argument("--judge-evals", type=int, default=500_000,
                    help="evaluation cap per run of the stronger judge on one extra holdout")
    ap.add_argument("--max-evals", type=int, default=None,
                    help="override the workload's evaluation cap per run (short profiled runs)")
    ap.add_argument("--ls-shape", default=None,
                    help="force the local-search launch shape UNROLL,WG_PER_CU (0 = tuned), e.g. 1,0 for counter passes")
    ap.add_argument("--chains", type=int, default=2, choices=(1, 2, 3, 4),
                    help="parts per bucket whose generation launches run on streams of their own")
    ap.add_argument("--work-queue", type=int, default=-1, choices=(-1, 0, 1),
                    help="persistent work queue of the generation launches: -1 tuned, 0 off, 1 on")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB three times (reference for HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the docking path runs on one GPU; --gpus must be 1 (across GPUs the "
                                   "workload would shard by ligand, each GPU holding its own copy of the maps)", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2007_03678_amd as pkg
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t0 = time.time()
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)   # reads and writes n * 4 bytes
        torch.cuda.synchronize()
        log(f"copy calibration: 3 x {args.calibrate_copy_mib} MiB read + written")
        del src, dst
    c = workload(args.workload)
    dock = c["dock"]
    if args.max_evals is not None:
        dock = dict(dock, max_evals=args.max_evals)
    log(f"workload {args.workload}: {len(c['ligands'])} ligands generated in {time.time() - t0:.1f}s")
    ctx = pkg.create(synth.forcefield(), 0)
    if args.ls_shape:
        u, w = (int(x) for x in args.ls_shape.split(","))
        ctx.ad_set_launch_shape(u, w)
    ctx.ad_set_work_queue(args.work_queue)
    ctx.ad_set_chains(args.chains)
    t0 = time.time()
    ctx.ad_build_grids(c["grid"], c["receptor"])
    batch = ctx.ad_load_ligands(c["ligands"])
    torch.cuda.synchronize()
    log(f"maps built and ligands loaded in {time.time() - t0:.2f}s")
    params = pkg.make_params(**dock)
    infos = [batch.info(i) for i in range(batch.n)]
    seed = 20200707

    for w in range(args.warmup):
        t0 = time.time()
        r = ctx.ad_dock_batch(batch, params, seed)
        log(f"warmup {w}: {time.time() - t0:.2f}s")

    ctx.ad_get_kernel_timing(reset=True)
    ctx.ad_set_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evals = 0
    for s in range(args.steps):
        r = ctx.ad_dock_batch(batch, params, seed)
        evals += int(r["evals"].sum())
        log(f"step {s}: {time.perf_counter() - t0:.2f}s cumulative")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = ctx.ad_get_kernel_timing(reset=True)
    ctx.ad_set_kernel_timing(False)
    schedule = ctx.ad_get_schedule()
    shape = ctx.ad_get_launch_shape()
    queue = ctx.ad_get_work_queue()
    chains = ctx.ad_get_chains()
    # the same step replayed as a graph (kernel timing off), for comparison
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.ad_dock_batch(batch, params, seed)
    graph_ms = (time.perf_counter() - t0) * 1e3
    schedule_graph = ctx.ad_get_schedule()

    n_lig = batch.n
    ligands_s = n_lig * args.steps / elapsed
    evals_s = evals / elapsed
    # dominant kernel: the local-search generation (energy + gradient)
    n_ls = int(np.floor(dock["ls_rate"] * dock["pop"] + 0.5))
    ls_flop = dock["nrun"] * n_ls * dock["ls_iters"] * sum(flops_per_eval(i, True) for i in infos)
    ls_ms, ls_n = kt["ls"]
    ga_ms, ga_n = kt["ga"]
    # The unit of the roofline is one generation's local search over every
    # run: the launches of the bucket's chains, which overlap on their
    # streams.  Its time is the local search's busy time (the union of the
    # launches' HIP-event intervals) per generation.
    n_gen = int(r["generations"][0]) * args.steps
    ls_gen_s = kt["busy_ms"]["ls"] / 1e3 / max(n_gen, 1)
    ga_gen_s = kt["busy_ms"]["ga"] / 1e3 / max(n_gen, 1)
    achieved = ls_flop / ls_gen_s / 1e12
    ls_flop_oracle = dock["nrun"] * n_ls * dock["ls_iters"] * sum(oracle_flops_per_eval(i) for i in infos)
    achieved_oracle = ls_flop_oracle / ls_gen_s / 1e12
    out = {
        "metric": METRIC,
        "value": round(ligands_s, 4),
        "unit": "ligands/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64/f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}: {n_lig} ligands (atoms {min(i['n_atoms'] for i in infos)}-"
                         f"{max(i['n_atoms'] for i in infos)}, torsions {min(i['n_torsions'] for i in infos)}-"
                         f"{max(i['n_torsions'] for i in infos)}), {len(c['receptor'].types)}-atom receptor, "
                         f"{c['grid'].n[0]}^3 x {len(c['grid'].map_types) + 2} FP32 maps, {dock['nrun']} runs "
                         f"x pop {dock['pop']}, cap {dock['max_evals']} evals/run, ADADELTA "
                         f"{dock['ls_iters']} it on {n_ls}/gen"),
            "n_ligands": n_lig, "nrun": dock["nrun"], "pop": dock["pop"], "max_evals_per_run": dock["max_evals"],
            "seeds": {"inputs": c["seed"], "docking": seed},
            "generations": int(r["generations"][0]),
        },
        "evals_per_s": round(evals_s, 1),
        "kernels_ms": {k: round(kt[k][0], 3) for k in pkg.KERNEL_KINDS},
        "kernels_busy_ms": {k: round(kt["busy_ms"][k], 3) for k in pkg.KERNEL_KINDS},
        "kernel_launches": {k: kt[k][1] for k in pkg.KERNEL_KINDS},
        "roofline": {
            "bound": "alu",
            "kernel": "k_ls_generation (ADADELTA: pose + maps + pairs + gradient)",
            "achieved": round(achieved, 3),
            "peak": PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_TFLOPS, 4),
            "frac_of_fp64_peak": round(achieved / PEAK_FP64_TFLOPS, 4),
            "flop_model": "minimal: 62P + 129N + 33D + 38T + 40 per evaluation (constants hoisted); the oracle's "
                          "own op count (op-counting build) is reported beside it",
            "flop_per_eval_mean": round(ls_flop / (dock["nrun"] * n_ls * dock["ls_iters"] * n_lig), 1),
            "oracle_count_flop_per_eval_mean": round(ls_flop_oracle / (dock["nrun"] * n_ls * dock["ls_iters"] * n_lig), 1),
            "achieved_oracle_count": round(achieved_oracle, 3),
            "frac_oracle_count": round(achieved_oracle / PEAK_TFLOPS, 4),
            "traffic": measured_traffic(),
            "traffic_note": "HBM (L2-to-fabric) bytes per generation's local search (its launches) from rocprofv3 "
                            "FETCH_SIZE/WRITE_SIZE scaled by a 1 GiB copy; null if the kernel changed since",
            "unit_of_work": "one generation's local search over every run (the launches of the chains, "
                            "overlapping on their streams); time = their busy time (union of HIP-event intervals)",
            "flop_per_generation": ls_flop,
            "ls_busy_ms_per_generation": round(ls_gen_s * 1e3, 4),
            "ls_launches_per_generation": round(ls_n / max(n_gen, 1), 3),
            "avg_launch_ms": round(ls_ms / max(ls_n, 1), 4),
            # the GA launches run beside the other chain's local search, so
            # their busy time is not theirs alone; reported, not rated
            "ga_busy_ms_per_generation": round(ga_gen_s * 1e3, 4),
        },
    }
    # the rates the roofline is set against, measured on this GPU
    mb = {k: ctx.ad_microbench(k, 0) for k in ctx.MICROBENCH_KINDS[:4]}
    mb["gather_4mib_bytes_per_s"] = ctx.ad_microbench("gather_bytes_per_s", 4 << 20)
    mb["gather_32mib_bytes_per_s"] = ctx.ad_microbench("gather_bytes_per_s", 32 << 20)
    out["roofline"]["measured_rates"] = {k: float(f"{v:.4g}") for k, v in mb.items()}
    out["roofline"]["frac_of_measured_fp32_fma"] = round(achieved * 1e12 / mb["fma_f32_flops"], 4)
    out["roofline"]["frac_of_measured_fp64_fma"] = round(achieved * 1e12 / mb["fma_f64_flops"], 4)
    # score-grad evaluations per second inside the local-search kernel
    out["schedule"] = {"timed_steps": {"graph": schedule["graph"], "ls_stage_pairs": schedule["stage_pairs"],
                                       "packed_runs": schedule["packed_runs"],
                                       "ls_pair_unroll": shape["unroll"], "ls_wg_per_cu": shape["wg_per_cu"],
                                       "work_queue": queue, "chains": chains},
                       "graph_replay_ms_per_step": round(graph_ms, 2), "graph": schedule_graph["graph"]}
    out["score_grad_evals_per_s"] = round(dock["nrun"] * n_lig * n_ls * dock["ls_iters"] / ls_gen_s, 1)
    if not args.no_variants:
        plain = {"ligands_per_s": ligands_s, "evals": evals / args.steps, "best_energy": r["best_energy"],
                 "generations": int(r["generations"][0])}
        out["search_variants"] = search_variants(ctx, batch, dock, infos, seed, plain, log)
    batch.free()
    ctx.close()
    out["single24"] = single24_leg(log)
    if not args.no_batch4096:
        out["batch4096"] = batch_leg(args, log)
    if not args.no_campaign:
        out["screened"] = screened_campaign(args, log)
    if not args.no_cpu_baseline:
        log("cpu baseline: running the oracle")
        out["cpu_baseline"] = cpu_baseline(c, dock, args.cpu_seconds, log)
        out["cpu_baseline"]["single24_full"] = cpu_single24(log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
